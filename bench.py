"""Throughput of the surfel radiosity hot path on one MI355X.

One step = the whole path over one synthetic fruit-bowl scene (100,000
surfels on 20 spheres in a hemispherical bowl, SH degree 3, 128 rays per
surfel, top-512 form factors, 8 bounces, one point light):
  build_bvh -> reflectance -> form_factors -> direct_light ->
  transport_solve (with tape) -> transport_backward -> opacity_backward.
All inputs are resident in HBM before the timed region.

Prints ONE JSON line.  `value` = complete forward+backward steps per second
(ray casting included); the JSON also carries Grays/s of the form-factor
ray cast and fwd+bwd solves/s at fixed F, per-phase HIP-event timings, the
roofline position of the dominant kernel, the error of sampled outputs
against the FP64 oracle, and the oracle's own speed on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd transport solves/s + Grays/s at 100k surfels, rel err <=1e-3 vs FP64"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3

# Algorithmic work per unit (operation counts of the traversal, hit test and compositing):
FLOP_BOX = 24      # one ray / box slab test
FLOP_HIT = 40      # one ray / surfel hit decision
FLOP_COMP = 30     # compositing one hit (two exponentials, weights)


# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (bytes,
# scaled by the counters of a plain copy kernel of known size: x1.9999 for
# FETCH_SIZE, x1.0000 for WRITE_SIZE), valid only for the kernel sources
# they were taken on (sha256 over the listed files, in order).
TRAFFIC = {
    "ff_trace": {"fetch": 159148.47e6, "write": 11312.00e6,
                 "files": ["trace.hip", "traverse.h", "gsrad_internal.h", "trace_api.h"],
                 "sha256": "fdc7be6bb7adca89ecf8c86f5069128128f4043cb4bf5720abeaf58017861ffb",
                 "summary": "profiles/fruit_bowl_100k_hbm_counters.txt"},
    "dense_grad_F": {"fetch": 236949.39e6, "write": 4294.97e6,
                     "files": ["dense.hip", "dense_api.h", "gsrad_internal.h"],
                     "sha256": "93a246c63f1835d7eec00229cce3ebf5ac38b0f1d6043b6daa9f2b79004ad563",
                     "summary": "profiles/multi_light_32k_hbm_counters.txt"},
}


def _updates(count, ms):
    """Surfel-light updates per second: one update is a surfel's K x 3
    coefficients for one light in one bounce (or adjoint step); ms is the
    step's time in those launches."""
    return count / (ms * 1e-3) if ms and ms > 0 else None


def calibration_copy(args, torch, dev):
    """A plain elementwise copy that reads and writes calib_copy_mib MiB
    each: its FETCH_SIZE / WRITE_SIZE counters calibrate the ones of the
    path's kernels in the same profiled run."""
    if args.calib_copy_mib > 0:
        a = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b


def measured_traffic(kernel):
    import hashlib
    t = TRAFFIC.get(kernel)
    if t is None:
        return None
    csrc = os.path.join(ROOT, "paper_2509_18497_amd", "csrc")
    h = hashlib.sha256()
    for f in t["files"]:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(hashlib.sha256(fh.read()).hexdigest().encode() + b"  " + f.encode() + b"\n")
    return (t["fetch"] + t["write"]) if h.hexdigest() == t["sha256"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=100_000, help="surfel count (100k is the measured workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--cpu-receivers", type=int, default=500,
                    help="receivers of the bounded oracle sample (about 15 s of host work)")
    ap.add_argument("--workload", default="fruit_bowl",
                    choices=["fruit_bowl", "multi_light", "uneven_batch", "sh_transfer", "center", "mc"],
                    help="fruit_bowl: the 100k sparse path (default); multi_light: the 32k box room with 100 "
                         "lights on the dense BF16 path; uneven_batch: 64 cluster rooms of 2k-65k surfels in one "
                         "batch; sh_transfer: the directional SH transfer with the diffuse + Phong BRDF and the "
                         "geometry and light gradients on the fruit bowl's ray-cast F; center: centre-to-centre "
                         "form factors with a learnable scale, transport and gradients on the same pattern; mc: "
                         "Monte-Carlo TD(0) rounds on the fruit bowl")
    ap.add_argument("--mc-rounds", type=int, default=32, help="mc: TD(0) rounds per step")
    ap.add_argument("--fp32-lights", type=int, default=10,
                    help="multi_light: lights timed on the plain FP32 per-light path (scaled to all lights)")
    ap.add_argument("--fp32-all", type=int, default=1,
                    help="multi_light: also time the FP32 sparse path with all lights in one launch (1) or not (0)")
    ap.add_argument("--batch-precision", default="fp32", choices=["fp32", "bf16"],
                    help="uneven_batch: precision of the batched transport's gathered rows")
    ap.add_argument("--batch-lights", type=int, nargs=2, default=[8, 100], metavar=("MIN", "MAX"),
                    help="uneven_batch: lights per room drawn from U{MIN..MAX}")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain FP32 copy kernel of this size first (HBM counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this path is not sharded over "
              "several GPUs.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2509_18497_amd as g
    import scenes

    torch.cuda.set_device(0)
    if args.workload == "multi_light":
        return multi_light(args, g, scenes, torch, np)
    if args.workload == "uneven_batch":
        return uneven_batch(args, g, scenes, torch, np, lights=tuple(args.batch_lights))
    if args.workload in ("sh_transfer", "center", "mc"):
        return paper_rows(args, g, scenes, torch, np)
    sc = scenes.make_config("fruit_bowl", n=args.n)
    N, R, K, nb, topk, Lt = sc.n, sc.R, sc.K, sc.n_bounces, sc.topk, sc.n_lights
    dev = torch.device("cuda")
    sur = {k: torch.from_numpy(v).to(dev) for k, v in sc.surfels.items()}
    alb = torch.from_numpy(sc.albedo).to(dev)
    lpos = torch.from_numpy(sc.light_pos).to(dev)
    lI = torch.from_numpy(sc.light_I).to(dev)
    gB = torch.from_numpy(scenes.seeded_array((N, Lt, K, 3), seed=99, lo=-1e-6, hi=1e-6)).to(dev)
    E = torch.empty((N, Lt, K, 3), dtype=torch.float32, device=dev)
    B = torch.empty_like(E)
    st = torch.cuda.current_stream()
    state = {"bvh": None, "ff": None, "tape": None}

    def step():
        bvh = g.build_bvh(sur, state["bvh"])
        state["bvh"] = bvh
        rho = g.reflectance(bvh, alb)
        ff = g.form_factors(bvh, R, sc.seed, t_min=sc.t_min, topk=topk, ff=state["ff"])
        state["ff"] = ff
        g.direct_light(bvh, alb, lpos, lI, K, out=E)
        _, tape = g.transport_solve(ff, rho, E, nb, tape=state["tape"], out=B)
        state["tape"] = tape
        gE, grho, gF = g.transport_backward(ff, tape, rho, gB)
        go, ga = g.opacity_backward(bvh, ff, gF, grho, alb)
        return ff, gE, grho, gF, go, ga

    calibration_copy(args, torch, dev)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    g.gsrad.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.gsrad.profile_report()
    g.gsrad.profile_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    ff = out[0]
    _, nnz = ff.info()

    def avg(name):
        return prof[name]["total_ms"] / args.steps if name in prof else 0.0

    t_trace = avg("ray_pools") + avg("ff_trace")   # ray generation and sorting, then the trace
    t_ff = t_trace + avg("ff_aggregate") + avg("ff_csr")
    t_solve_bwd = avg("bounce") + avg("transpose") + avg("adjoint") + avg("sddmm") + avg("opacity_records") + \
        avg("opacity_pass1") + avg("opacity_pass2") + avg("opacity_finish")
    rays = N * R
    grays = rays / (t_trace * 1e-3) / 1e9 if t_trace > 0 else None

    # composited hits per ray on a sample (outside the timed region) for the
    # algorithmic work of the ray cast
    rng = np.random.default_rng(7)
    samp = np.sort(rng.choice(N, size=64, replace=False)).astype(np.int64)
    hits = g.ray_hits(state["bvh"], torch.from_numpy(samp).to(dev), R, sc.seed, t_min=sc.t_min, max_hits=1)
    h_avg = float(hits["count"].float().mean().item())
    flop_ray = 2 * math.log2(N) * FLOP_BOX + h_avg * (FLOP_HIT + FLOP_COMP)

    # roofline of the dominant kernel (largest share of the step)
    phases = {k: v["total_ms"] / args.steps for k, v in prof.items()}
    dom = max(phases, key=phases.get)
    dom_avg_ms = prof[dom]["avg_ms"]
    C = Lt * K * 3
    if dom in ("ff_trace", "opacity_pass1", "opacity_pass2"):
        work = rays * flop_ray * (1.0 if dom == "ff_trace" else 1.0)
        achieved = work / (dom_avg_ms * 1e-3) / 1e12
        rec_bytes = rays * (8 * h_avg + 4)   # hit records (j, +-gamma) and counts written
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(dom),
                "work_per_launch": {"rays": rays, "flop_per_ray": flop_ray, "hits_per_ray": h_avg,
                                    "algorithmic_bytes": rec_bytes,
                                    "algorithmic_GBps": rec_bytes / (dom_avg_ms * 1e-3) / 1e9}}
    else:
        per_launch = {"bounce": nnz * 8 + 3 * N * C * 4, "adjoint": nnz * 8 + 3 * N * C * 4,
                      "sddmm": nnz * 12 + 2 * nb * N * C * 4}.get(dom, 0)
        achieved = per_launch / (dom_avg_ms * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": measured_traffic(dom), "bytes_per_launch": per_launch}

    # HBM rate of the sparse bounce (for the record)
    bounce_bytes = nnz * 8 + 3 * N * C * 4
    bounce_gbs = bounce_bytes / (prof["bounce"]["avg_ms"] * 1e-3) / 1e9 if "bounce" in prof else None

    result = {
        "metric": METRIC,
        "value": 1e3 / ms,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"fruit bowl: {N} surfels, 20 spheres in a bowl, R={R} rays/surfel, top-{topk} F, "
                               f"SH K={K}, {Lt} light, {nb} bounces, fwd+bwd (MSE-style grad_B)",
                   "surfels": N, "rays_per_surfel": R, "topk": topk, "K": K, "lights": Lt, "bounces": nb},
        "grays_per_s": grays,
        "bounce_updates_per_s": _updates(nb * N * Lt, phases.get("bounce", 0.0)),
        "adjoint_updates_per_s": _updates(nb * N * Lt, phases.get("adjoint", 0.0)),
        "fwd_bwd_solves_per_s_fixed_F": (1e3 / t_solve_bwd) if t_solve_bwd > 0 else None,
        "form_factor_ms": t_ff,
        "nnz": nnz,
        "bounce_hbm_GBps": bounce_gbs,
        "phase_ms_per_step": {k: round(v, 4) for k, v in sorted(phases.items())},
        "roofline": roof,
    }

    if not args.no_check:
        result["err_vs_fp64"] = sampled_errors(g, sc, state, samp[:8], torch, np)
        result["err_vs_fp64"]["timed_step_transport"] = step_errors(g, sc, state, out, E, B, gB, alb, torch, np)
        result["err_vs_fp64"]["grad_opacity_sampled_rows"] = opacity_errors(g, sc, state, torch, np)
        result["err_vs_fp64"]["transport_full_size"] = slice_errors(g, sc, torch, np)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(sc, args.cpu_receivers, nnz, np)
    print(json.dumps(result))


def sampled_errors(g, sc, state, recv, torch, np):
    """Relative max-norm error of sampled F rows and E rows vs the oracle."""
    import oracle
    te = oracle.default_t_eps(sc.surfels)
    rp, col, val = state["ff"].csr()
    rp, col, val = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
    rpo, co, vo, _ = oracle.ff_rows(sc.surfels, recv, sc.R, sc.seed, te, sc.t_min, sc.topk)
    # An entry kept on one side only is a swap at the top-k threshold when
    # its value does not exceed the smallest kept value of the other side
    # (within 1e-6 relative): both selections are then valid, and such
    # entries are counted, not scored.
    num = den = 0.0
    swaps = 0
    for k, i in enumerate(recv):
        a = dict(zip(col[rp[i]:rp[i + 1]].tolist(), val[rp[i]:rp[i + 1]].tolist()))
        b = dict(zip(co[rpo[k]:rpo[k + 1]].tolist(), vo[rpo[k]:rpo[k + 1]].tolist()))
        full = sc.topk > 0 and len(a) == sc.topk and len(b) == sc.topk
        tha = min(a.values()) if a else 0.0
        thb = min(b.values()) if b else 0.0
        for j in set(a) | set(b):
            if full and j not in b and a[j] <= thb * (1 + 1e-6):
                swaps += 1
                continue
            if full and j not in a and b[j] <= tha * (1 + 1e-6):
                swaps += 1
                continue
            num = max(num, abs(a.get(j, 0.0) - b.get(j, 0.0)))
        den = max(den, max(b.values()) if b else 0.0)
    Eg = g.direct_light(state["bvh"], torch.from_numpy(sc.albedo).cuda(), torch.from_numpy(sc.light_pos).cuda(),
                        torch.from_numpy(sc.light_I).cuda(), sc.K).cpu().numpy()[recv]
    Eo = oracle.direct_light(sc.surfels, sc.albedo, sc.light_pos, sc.light_I, sc.K, receivers=recv)
    e_err = float(np.max(np.abs(Eg - Eo)) / max(np.max(np.abs(Eo)), 1e-300))
    return {"F_rows": num / den if den > 0 else None, "F_topk_threshold_swaps": swaps, "E_rows": e_err,
            "rows_sampled": len(recv)}


def _rel(np, x, ref):
    return float(np.max(np.abs(np.asarray(x, np.float64) - ref)) / max(np.max(np.abs(ref)), 1e-300))


def step_errors(g, sc, state, out, E, B, gB, alb, torch, np):
    """The last timed step's own transport against the FP64 oracle on its
    own ray-cast F: E comes from point lights, so it has only the DC
    coefficient, every B^(k) is DC-only, and the oracle's FP64 bounces and
    adjoint on the 3 DC columns (with the step's grad_B restricted to them)
    give the exact B, grad_E on those columns, grad_rho and every entry of
    grad_F of the whole launch; the other columns of B must be 0."""
    import oracle
    import scipy.sparse as sp
    ff, gE, grho, gF = out[0], out[1], out[2], out[3]
    rp, col, val = (x.cpu().numpy() for x in ff.csr())
    N = rp.shape[0] - 1
    F = sp.csr_matrix((val.astype(np.float64), col, rp), shape=(N, N))
    rho = g.reflectance(state["bvh"], alb).cpu().numpy()
    Ed = E.cpu().numpy()[:, :, :1, :]
    gBd = gB.cpu().numpy()[:, :, :1, :]
    Bo, tp = oracle.bounce(F, rho, Ed, sc.n_bounces, keep_tape=True)
    gEo, gro, gFo = oracle.adjoint(F, rho, tp, gBd)
    Bg = B.cpu().numpy()
    return {"B": _rel(np, Bg[:, :, :1, :], Bo), "B_non_dc_all_zero": bool(not Bg[:, :, 1:, :].any()),
            "grad_E_dc": _rel(np, gE.cpu().numpy()[:, :, :1, :], gEo), "grad_rho": _rel(np, grho.cpu().numpy(), gro),
            "grad_F": _rel(np, gF.cpu().numpy(), gFo), "entries": int(F.nnz)}


def opacity_errors(g, sc, state, torch, np, n_rows=64):
    """grad_opacity in the step's launch configuration with dL/dF non-zero on
    n_rows sampled receiver rows: the oracle's brute-force compositing
    backward over those receivers is the exact gradient of every surfel."""
    import oracle
    rp, col, _ = (x.cpu().numpy() for x in state["ff"].csr())
    N = rp.shape[0] - 1
    recv = np.sort(np.random.default_rng(19).choice(N, size=n_rows, replace=False)).astype(np.int64)
    rng = np.random.default_rng(20)
    gF = np.zeros(rp[-1], np.float32)
    gp, gc, gv = [0], [], []
    for i in recv:
        v = rng.standard_normal(rp[i + 1] - rp[i]).astype(np.float32)
        gF[rp[i]:rp[i + 1]] = v
        gc.append(col[rp[i]:rp[i + 1]])
        gv.append(v.astype(np.float64))
        gp.append(gp[-1] + v.shape[0])
    go = g.opacity_backward(state["bvh"], state["ff"], torch.from_numpy(gF).cuda(), None, None)[0].cpu().numpy()
    te = oracle.default_t_eps(sc.surfels)
    goo, _ = oracle.opacity_backward(sc.surfels, sc.albedo, sc.R, sc.seed, te, sc.t_min,
                                     (np.asarray(gp, np.int64), np.concatenate(gc), np.concatenate(gv)),
                                     receivers=recv)
    return {"grad_opacity": _rel(np, go, goo), "rows": n_rows, "surfels_reached": int(np.count_nonzero(goo))}


def slice_errors(g, sc, torch, np, slots=(0, 15)):
    """B, grad_E and grad_rho of the full-size launch (N rows, Lt*K*3
    columns, 8 bounces) on a seeded operator with the workload's row length,
    E and grad_B non-zero on two SH coefficients only: the transport is
    separable over coefficient columns, so the oracle's FP64 run on those
    two coefficients gives the exact results of the whole launch."""
    import oracle
    import scenes
    import scipy.sparse as sp
    N, Lt, K, nb = sc.n, sc.n_lights, sc.K, sc.n_bounces
    rp, c, v = scenes.seeded_csr(N, sc.topk, seed=31)
    F = sp.csr_matrix((v.astype(np.float64), c, rp), shape=(N, N))
    rho = scenes.seeded_array((N, 3), seed=1, lo=0.1, hi=0.9)
    Es = scenes.seeded_array((N, Lt, len(slots), 3), seed=2)
    gBs = scenes.seeded_array((N, Lt, len(slots), 3), seed=3, lo=-1, hi=1)
    E = np.zeros((N, Lt, K, 3), np.float32)
    gB = np.zeros((N, Lt, K, 3), np.float32)
    E[:, :, list(slots), :] = Es
    gB[:, :, list(slots), :] = gBs
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()   # noqa: E731
    ff = g.ff_from_csr(d(rp), d(c), d(v))
    B, tape = g.transport_solve(ff, d(rho), d(E), nb)
    gE, gr, _ = g.transport_backward(ff, tape, d(rho), d(gB), want_grad_F=False)
    B, gE, gr = (x.cpu().numpy() for x in (B, gE, gr))
    Bo, tp = oracle.bounce(F, rho, Es, nb, keep_tape=True)
    gEo, gro, _ = oracle.adjoint(F, rho, tp, gBs, want_grad_F=False)

    def rel(x, ref):
        return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))

    sl = list(slots)
    return {"B": rel(B[:, :, sl, :], Bo), "grad_E": rel(gE[:, :, sl, :], gEo), "grad_rho": rel(gr, gro),
            "operator": f"seeded {N}-row CSR, {F.nnz} entries, coefficients {sl} of K={K}"}


def cpu_baseline(sc, n_recv, nnz, np):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload, scaled to one full step."""
    import oracle
    import scenes
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    te = oracle.default_t_eps(sc.surfels)
    rng = np.random.default_rng(11)
    recv = np.sort(rng.choice(sc.n, size=n_recv, replace=False)).astype(np.int64)
    t0 = time.perf_counter()
    rp, co, vo, _ = oracle.ff_rows(sc.surfels, recv, sc.R, sc.seed, te, sc.t_min, sc.topk, n_threads=threads)
    t_ff = time.perf_counter() - t0
    gv = np.ones(vo.shape[0])
    t0 = time.perf_counter()
    oracle.opacity_backward(sc.surfels, sc.albedo, sc.R, sc.seed, te, sc.t_min, (rp, co, gv), receivers=recv,
                            n_threads=threads)
    t_ob = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.direct_light(sc.surfels, sc.albedo, sc.light_pos, sc.light_I, sc.K, te, receivers=recv,
                        n_threads=threads)
    t_dl = time.perf_counter() - t0
    # bounces + adjoint on a 5,000-row synthetic operator of the same row
    # length, scaled by the number of stored entries
    m = 5000
    rpc, cc, vc = scenes.seeded_csr(m, sc.topk, seed=5)
    import scipy.sparse as sp
    F = sp.csr_matrix((vc.astype(np.float64), cc, rpc), shape=(m, m))
    C = sc.n_lights * sc.K * 3
    Em = np.random.default_rng(1).uniform(0, 1, (m, C))
    rho = np.random.default_rng(2).uniform(0.1, 0.9, (m, 3))
    t0 = time.perf_counter()
    Bm, tape = oracle.bounce(F, rho, Em, sc.n_bounces, keep_tape=True)
    oracle.adjoint(F, rho, tape, Em)
    t_lin = (time.perf_counter() - t0) * (nnz / max(F.nnz, 1))
    per_receiver = (t_ff + t_ob + t_dl) / n_recv
    t_step = per_receiver * sc.n + t_lin
    return {"value": 1.0 / t_step, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_recv} receivers of the 100k fruit bowl (form-factor rows, compositing backward and direct "
                      f"light, brute force) scaled x{sc.n / n_recv:.0f}, plus bounces+adjoint on a {m}-row operator "
                      f"with {sc.topk} entries/row scaled to nnz={nnz}",
            "seconds_measured": t_ff + t_ob + t_dl + t_lin * F.nnz / max(nnz, 1)}


PEAK_BF16_TFLOPS = 2500.0


def _timed(args, torch, g, step):
    """Warm-up, then the timed steps with the library's phase events."""
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    g.gsrad.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.gsrad.profile_report()
    g.gsrad.profile_enable(False)
    return out, prof, (t1 - t0) * 1e3 / args.steps


def paper_rows(args, g, scenes, torch, np):
    """The paper's own extensions of the path on the 100k fruit bowl, with
    its ray-cast F (R=128, top-512) made once outside the timed region:
      sh_transfer  diffuse + Phong BRDF coefficients (K=16), direct light
                   through the BRDF, 8 directional bounces with tape, their
                   adjoint (dL/dE, dL/dR, dL/dF), the BRDF backward, the
                   geometry gradients through the ray-cast F for that dL/dF
                   and the light gradients for dL/dE;
      center       centre-to-centre F with a learnable scale on the ray-cast
                   pattern, 8 bounces + adjoint, and its gradients (scale and
                   the 15 surfel fields of pair ends and occluders);
      mc           --mc-rounds TD(0) rounds of the Monte-Carlo solver (groups
                   made once) with the centre-to-centre decay at scale 0.3."""
    sc = scenes.make_config("fruit_bowl", n=args.n)
    N, R, K, nb, topk, Lt = sc.n, sc.R, sc.K, sc.n_bounces, sc.topk, sc.n_lights
    dev = torch.device("cuda")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)   # noqa: E731
    sur = {k: d(v) for k, v in sc.surfels.items()}
    alb, lpos, lI = d(sc.albedo), d(sc.light_pos), d(sc.light_I)
    bvh = g.build_bvh(sur)
    ff = g.form_factors(bvh, R, sc.seed, t_min=sc.t_min, topk=topk, compact=True)
    _, nnz = ff.info()
    gB = d(scenes.seeded_array((N, Lt, K, 3), seed=99, lo=-1e-6, hi=1e-6))
    C = Lt * K * 3
    wl = args.workload
    extra = {}
    if wl == "sh_transfer":
        mat = {k: d(v) for k, v in scenes.phong_materials(N, seed=7).items()}
        state = {"tape": None}

        def step():
            Rm = g.brdf_reflectance(bvh, mat["k"], mat["albedo_d"], mat["albedo_s"], mat["shininess"], K)
            E = g.direct_light_sh(bvh, Rm, lpos, lI)
            B, tape = g.transport_solve_sh(ff, bvh, Rm, E, nb, tape=state["tape"])
            state["tape"] = tape
            gE, gR, gF = g.transport_backward_sh(ff, bvh, tape, Rm, gB)
            gb = g.brdf_backward(bvh, mat["k"], mat["albedo_d"], mat["albedo_s"], mat["shininess"], gR)
            gg = g.geometry_backward(bvh, ff, gF)
            gl = g.direct_light_backward(bvh, alb, lpos, lI, gE)
            return B, gb, gg, gl

        unit, what = "fwd+bwd solves/s", (f"fruit bowl {N} surfels, ray-cast F (R={R}, top-{topk}, made once), diffuse "
                                          f"+ Phong BRDF, K={K}, {Lt} light, {nb} directional bounces, fwd+bwd with "
                                          "geometry and light gradients")
        samp = torch.from_numpy(np.sort(np.random.default_rng(7).choice(N, 64, replace=False))).to(dev)
        h_avg = float(g.ray_hits(bvh, samp, R, sc.seed, t_min=sc.t_min, max_hits=1)["count"].float().mean())
        recs = N * R * h_avg
        work = {"bounce_sh": ("hbm", nnz * 8 + N * 64 + 3 * N * C * 4),
                "adjoint_sh": ("hbm", nnz * 8 + N * 64 + 3 * N * C * 4),
                "sddmm_sh": ("hbm", nnz * 12 + N * 64 + 2 * nb * N * C * 4),
                # two passes over the hit records (8 B each), the surfel
                # records (64 B each) and dL/dF, 15 gradient fields written
                "geometry_backward": ("hbm", 2 * (recs * 8 + N * 64 + nnz * 4) + N * 15 * 4)}
        extra["hits_per_ray"] = h_avg
    elif wl == "center":
        lam = d(np.full(N, 0.8, np.float32))
        rho = g.reflectance(bvh, alb)
        E = g.direct_light(bvh, alb, lpos, lI, K)
        state = {"fc": None, "tape": None}

        def step():
            fc = g.ff_center(bvh, ff, lam, ff=state["fc"])
            state["fc"] = fc
            B, tape = g.transport_solve(fc, rho, E, nb, tape=state["tape"])
            state["tape"] = tape
            gE, grho, gF = g.transport_backward(fc, tape, rho, gB)
            gl, gs = g.ff_center_backward(bvh, fc, lam, gF)
            return B, gl, gs

        unit, what = "fwd+bwd solves/s", (f"fruit bowl {N} surfels, centre-to-centre F (scale 0.8) on the ray-cast "
                                          f"pattern (R={R}, top-{topk}, {nnz} pairs), K={K}, {Lt} light, {nb} "
                                          "bounces, fwd+bwd with scale and geometry gradients")
        flop_seg = 2 * math.log2(N) * FLOP_BOX
        work = {"ff_center": ("alu", nnz * flop_seg), "ff_center_backward": ("alu", 2 * nnz * flop_seg)}
        extra["segments_per_launch"] = nnz
    else:
        lam = d(np.full(N, 0.3, np.float32))
        rho = g.reflectance(bvh, alb)
        E = g.direct_light(bvh, alb, lpos, lI, K)
        mc = g.mc_create(bvh)
        T = args.mc_rounds
        state = {"seed": 0}

        def step():
            state["seed"] += 1
            return g.mc_solve(mc, lam, rho, E, T, seed=state["seed"])

        G = int(round(math.sqrt(N)))
        unit, what = "receiver updates/s", (f"fruit bowl {N} surfels, {G} K-Means groups, {T} TD(0) rounds per step "
                                            f"(one next event per receiver per round), centre-to-centre decay at "
                                            f"scale 0.3, K={K}, {Lt} light")
        # per receiver: G group weights + the drawn group's members (n/G on
        # average) at ~20 flop each, and one segment walk
        flop_recv = (G + N / G) * 20 + 2 * math.log2(N) * FLOP_BOX
        work = {"mc_solve": ("alu", T * N * flop_recv)}
        extra["rounds_per_step"] = T
    out, prof, ms = _timed(args, torch, g, step)
    phases = {k: v["total_ms"] / args.steps for k, v in prof.items()}
    dom = max((k for k in phases if k in work), key=phases.get)
    bound, amount = work[dom]
    dom_ms = prof[dom]["avg_ms"]
    if bound == "hbm":
        ach = amount / (dom_ms * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "traffic": None, "bytes_per_launch": amount}
    else:
        ach = amount / (dom_ms * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_FP32_TFLOPS, "traffic": None, "flop_per_launch": amount}
    value = (N * args.mc_rounds / (ms * 1e-3)) if wl == "mc" else 1e3 / ms
    result = {"metric": f"{wl}: {unit} at 100k surfels", "value": value, "unit": unit, "n_gpus": 1,
              "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
              "config": {"workload": what, "surfels": N, "nnz": nnz, "K": K, "lights": Lt, "bounces": nb},
              "phase_ms_per_step": {k: round(v, 4) for k, v in sorted(phases.items())}, "roofline": roof}
    result.update(extra)
    if wl == "center" and not args.no_check:
        result["err_vs_fp64"] = center_errors(g, sc, bvh, state["fc"], torch, np)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = rows_cpu_baseline(wl, sc, nnz, np, T=args.mc_rounds)
    print(json.dumps(result))


def center_errors(g, sc, bvh, fc, torch, np, n_rows=8):
    """Centre-to-centre rows of the timed launch against the oracle on the
    pairs the oracle's own ray cast records for those receivers (entries on
    both sides compared; top-k threshold swaps counted, not scored)."""
    import oracle
    from oracle import center
    te = oracle.default_t_eps(sc.surfels)
    recv = np.sort(np.random.default_rng(23).choice(sc.n, size=n_rows, replace=False)).astype(np.int64)
    rpo, co, _, _ = oracle.ff_rows(sc.surfels, recv, sc.R, sc.seed, te, sc.t_min, sc.topk)
    rows = np.repeat(recv, np.diff(rpo))
    lam = np.full(sc.n, np.float32(0.8), np.float64)
    Fo, _ = center.center_ff(sc.surfels, rows, co, lam, t_eps=te)
    rp, col, val = (x.cpu().numpy() for x in fc.csr())
    num = den = 0.0
    common = other = 0
    for k, i in enumerate(recv):
        a = dict(zip(col[rp[i]:rp[i + 1]].tolist(), val[rp[i]:rp[i + 1]].tolist()))
        for j, v in zip(co[rpo[k]:rpo[k + 1]].tolist(), Fo[rpo[k]:rpo[k + 1]].tolist()):
            den = max(den, abs(v))
            if j in a:
                num = max(num, abs(a[j] - v))
                common += 1
            else:
                other += 1
    return {"F_center_rows": num / den if den > 0 else None, "pairs_compared": common,
            "pairs_only_in_one_pattern": other, "rows_sampled": n_rows}


def rows_cpu_baseline(wl, sc, nnz, np, T=32):
    """The FP64 oracle of the same row on the host cores, on a bounded
    sample scaled to one step."""
    import scipy.sparse as sp

    import oracle
    from oracle import center
    from oracle import sh as osh
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rng = np.random.default_rng(13)
    N = sc.n
    if wl == "sh_transfer":
        # 8 directional bounces + the adjoint on the first m rows' entries of a
        # seeded operator with the workload's row length, scaled by entries
        import scenes
        m = 2000
        rp, c, v = scenes.seeded_csr(m, sc.topk, seed=5)
        F = sp.csr_matrix((v.astype(np.float64), c, rp), shape=(m, m))
        sub = {k: np.ascontiguousarray(a[:m]) for k, a in sc.surfels.items()}
        Rm = rng.uniform(0, 1, (m, sc.K, 3))
        E = rng.uniform(0, 1, (m, sc.n_lights, sc.K, 3))
        t0 = time.perf_counter()
        _, tape = osh.bounce(F, sub, Rm, E, sc.n_bounces, keep_tape=True)
        osh.adjoint(F, sub, Rm, tape, E)
        dt = time.perf_counter() - t0
        return {"value": 1.0 / (dt * nnz / F.nnz), "unit": "fwd+bwd solves/s", "cores": 1, "kind": "oracle",
                "sample": f"directional bounces + adjoint on a {m}-row seeded operator ({F.nnz} entries) scaled to "
                          f"nnz={nnz}", "seconds_measured": dt}
    te = oracle.default_t_eps(sc.surfels)
    ns = 20000 if wl == "center" else 4000
    rows = rng.integers(0, N, ns).astype(np.int64)
    cols = rng.integers(0, N, ns).astype(np.int32)
    keep = rows != cols
    rows, cols = rows[keep], cols[keep]
    lam = np.ones(N)
    t0 = time.perf_counter()
    center.center_ff(sc.surfels, rows, cols, lam, t_eps=te, n_threads=threads)
    dt = time.perf_counter() - t0
    per = dt / rows.size
    if wl == "center":
        t_step = per * nnz * 3     # forward and the two-pass backward, one segment each
        return {"value": 1.0 / t_step, "unit": "fwd+bwd solves/s", "cores": threads, "kind": "oracle",
                "sample": f"{rows.size} random pairs' centre-to-centre F (brute-force segment over all surfels), "
                          f"scaled to 3 segment passes over nnz={nnz} (the transport is not counted)",
                "seconds_measured": dt}
    return {"value": 1.0 / per, "unit": "receiver updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows.size} random pairs' centre-to-centre F (one segment each, the cost of one next event "
                      "without the weight scans), scaled per receiver update", "seconds_measured": dt}


def multi_light(args, g, scenes, torch, np):
    """The 32,768-surfel box room lit by 100 point lights: one F, 100
    right-hand sides (C = 100 * 9 * 3 = 2700 columns).  A step is the whole
    path: BVH, ray-cast F (256 rays, all entries), dense BF16 copies, direct
    light, 8 bounces on the matrix cores (7 BF16 + the correction sweep) and
    the backward with the dense dL/dF.  The plain FP32 per-light path (one
    sparse solve and backward per light) is timed on a sample of lights."""
    sc = scenes.make_config("multi_light")
    N, R, K, nb, Lt = sc.n, sc.R, sc.K, sc.n_bounces, sc.n_lights
    dev = torch.device("cuda")
    sur = {k: torch.from_numpy(v).to(dev) for k, v in sc.surfels.items()}
    alb = torch.from_numpy(sc.albedo).to(dev)
    lpos = torch.from_numpy(sc.light_pos).to(dev)
    lI = torch.from_numpy(sc.light_I).to(dev)
    gB = torch.from_numpy(scenes.seeded_array((N, Lt, K, 3), seed=99, lo=-1e-3, hi=1e-3)).to(dev)
    E = torch.empty((N, Lt, K, 3), dtype=torch.float32, device=dev)
    B = torch.empty_like(E)
    state = {"bvh": None, "ff": None, "tape": None}

    def step():
        bvh = g.build_bvh(sur, state["bvh"])
        state["bvh"] = bvh
        rho = g.reflectance(bvh, alb)
        ff = g.form_factors(bvh, R, sc.seed, t_min=sc.t_min, topk=0, ff=state["ff"], records=False)
        state["ff"] = ff
        g.ff_dense(ff)
        g.direct_light(bvh, alb, lpos, lI, K, out=E)
        _, tape = g.transport_solve(ff, rho, E, nb, tape=state["tape"], out=B, precision=g.BF16)
        state["tape"] = tape
        gE, grho, gF = g.transport_backward(ff, tape, rho, gB)
        state["rho"] = rho
        return gE, grho, gF

    calibration_copy(args, torch, dev)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    g.gsrad.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.gsrad.profile_report()
    g.gsrad.profile_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    ff = state["ff"]
    _, nnz = ff.info()

    def avg(name):
        return prof[name]["total_ms"] / args.steps if name in prof else 0.0

    t_transport = sum(avg(k) for k in ("dense_bounce", "dense_bounce_fix", "dense_adjoint", "dense_adjoint_fix",
                                       "dense_grad_F"))
    # plain FP32: one sparse solve + backward per light, on a sample of lights
    rho = state["rho"]
    nl = max(1, min(args.fp32_lights, Lt))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for l in range(nl):
        El = E[:, l:l + 1].contiguous()
        gl = gB[:, l:l + 1].contiguous()
        _, tl = g.transport_solve(ff, rho, El, nb)
        g.transport_backward(ff, tl, rho, gl)
    torch.cuda.synchronize()
    t_fp32 = (time.perf_counter() - t2) * Lt / nl
    # plain FP32 with all lights in one sparse launch (C = Lt K 3 columns):
    # the same operator and right-hand sides as the BF16 path, same passes
    if args.fp32_all:
        _, t1a = g.transport_solve(ff, rho, E, nb)
        g.transport_backward(ff, t1a, rho, gB)
        del t1a
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        _, t1a = g.transport_solve(ff, rho, E, nb)
        g.transport_backward(ff, t1a, rho, gB)
        torch.cuda.synchronize()
        t_fp32_all = time.perf_counter() - t3
        del t1a
    else:
        t_fp32_all = None
    C = Lt * K * 3
    Np = (N + 255) // 256 * 256
    Cp = (C + 255) // 256 * 256
    flop_bounce = 2.0 * N * N * C             # one product F B (algorithmic, dense)
    flop_gF = 2.0 * N * N * nb * C            # dense dL/dF
    phases = {k: v["total_ms"] / args.steps for k, v in prof.items()}
    dom = max(("dense_grad_F", "dense_bounce"), key=lambda k: phases.get(k, 0.0))
    dom_ms = prof[dom]["avg_ms"]
    work = flop_gF if dom == "dense_grad_F" else flop_bounce
    achieved = work / (dom_ms * 1e-3) / 1e12
    issued = (3.0 * 2 * Np * Np * ((nb * C + 63) // 64 * 64)) if dom == "dense_grad_F" else 2.0 * Np * Np * Cp
    roof = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_BF16_TFLOPS, "traffic": measured_traffic(dom),
            "work_per_launch": {"algorithmic_flop": work, "issued_mfma_flop": issued,
                                "issued_TFLOPs": issued / (dom_ms * 1e-3) / 1e12,
                                "note": "dL/dF runs on split hi+lo operands: three BF16 products" if
                                dom == "dense_grad_F" else "one BF16 product, padded to 256-wide tiles"}}
    if "dense_bounce" in prof:
        bt = prof["dense_bounce"]["avg_ms"]
        roof["dense_bounce"] = {"avg_ms": bt, "achieved": flop_bounce / (bt * 1e-3) / 1e12,
                                "frac": flop_bounce / (bt * 1e-3) / 1e12 / PEAK_BF16_TFLOPS}
    result = {
        "metric": "fwd+bwd transport solves/s, 100 lights as right-hand sides of one F (dense BF16 MFMA)",
        "value": 1e3 / ms,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"box room: {N} surfels, {Lt} point lights on a radius-3 sphere, R={R}, all F "
                               f"entries, SH K={K}, {nb} bounces (7 BF16 + correction sweep), fwd+bwd with dense "
                               f"dL/dF",
                   "surfels": N, "lights": Lt, "K": K, "bounces": nb, "columns": C, "nnz": nnz},
        "transport_ms": t_transport,
        "transport_solves_per_s": 1e3 / t_transport if t_transport > 0 else None,
        "bounce_updates_per_s": _updates(nb * N * Lt, phases.get("dense_bounce", 0.0) + phases.get("dense_bounce_fix", 0.0)),
        "adjoint_updates_per_s": _updates(nb * N * Lt, phases.get("dense_adjoint", 0.0) + phases.get("dense_adjoint_fix", 0.0)),
        "fp32_per_light_fwd_bwd_ms": t_fp32 * 1e3,
        "fp32_lights_timed": nl,
        "speedup_vs_fp32_per_light": (t_fp32 * 1e3) / t_transport if t_transport > 0 else None,
        "fp32_all_lights_one_launch_fwd_bwd_ms": t_fp32_all * 1e3 if t_fp32_all else None,
        "speedup_vs_fp32_one_launch": (t_fp32_all * 1e3) / t_transport if t_fp32_all and t_transport > 0 else None,
        "phase_ms_per_step": {k: round(v, 4) for k, v in sorted(phases.items())},
        "roofline": roof,
    }
    if not args.no_check:
        # the dense launch does not depend on the operator's sparsity, so the
        # check uses a shorter seeded row (256 entries) to keep the oracle fast
        result["err_vs_fp64"] = dense_slice_errors(g, torch, np, N, 256, Lt, K, nb)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = dense_cpu_baseline(np, N, int(nnz // N), Lt, K, nb)
    print(json.dumps(result))


def uneven_batch(args, g, scenes, torch, np, lights=(8, 100), topk=512):
    """64 cluster rooms with log-uniform surfel counts in [2048, 65536]
    (about 1.2 M surfels, 150 M rays at R = 128), K = 9, 8 bounces, each room
    lit by U{8..100} point lights (its right-hand sides), F truncated to 512
    entries per row.  A step is the whole path: per-scene BVH, form factors
    and direct light, then one batch solve and backward (persistent
    launches, tuned lanes per row, captured bounce and adjoint loops).  The
    same transport run scene by scene is timed beside it."""
    rooms = scenes.uneven_batch(lights=lights)
    K, R, nb = rooms[0].K, rooms[0].R, rooms[0].n_bounces
    dev = torch.device("cuda")
    surs = [{k: torch.from_numpy(v).to(dev) for k, v in sc.surfels.items()} for sc in rooms]
    albs = [torch.from_numpy(sc.albedo).to(dev) for sc in rooms]
    lps = [torch.from_numpy(sc.light_pos).to(dev) for sc in rooms]
    lIs = [torch.from_numpy(sc.light_I).to(dev) for sc in rooms]
    Lts = [sc.n_lights for sc in rooms]
    st = {"bvh": [None] * len(rooms), "ff": [None] * len(rooms)}

    def step():
        Es, rhos = [], []
        for s, sc in enumerate(rooms):
            bvh = g.build_bvh(surs[s], st["bvh"][s])
            st["bvh"][s] = bvh
            st["ff"][s] = g.form_factors(bvh, R, sc.seed, t_min=sc.t_min, topk=topk, ff=st["ff"][s], records=False,
                                         compact=True)
            Es.append(g.direct_light(bvh, albs[s], lps[s], lIs[s], K))
            rhos.append(g.reflectance(bvh, albs[s]))
        batch = g.batch_create(st["ff"], Lts, K, batch=st.get("batch"))
        g.batch_set_precision(batch, g.BF16 if args.batch_precision == "bf16" else g.FP32)
        rho = torch.cat(rhos)
        E = batch.pack(Es)
        if "gB" not in st:
            st["gB"] = torch.from_numpy(scenes.seeded_array((E.shape[0],), seed=98, lo=-1e-3, hi=1e-3)).to(dev)
        B = g.batch_transport_solve(batch, rho, E, nb)
        out = g.batch_transport_backward(batch, rho, st["gB"])
        st.update(batch=batch, rho=rho, E=E, rhos=rhos, Es=Es)
        return B, out

    calibration_copy(args, torch, dev)
    print(f"uneven batch: {len(rooms)} rooms, {sum(sc.n for sc in rooms)} surfels, {sum(Lts)} lights",
          file=sys.stderr, flush=True)
    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"warm-up step {w + 1} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    g.gsrad.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        if args.steps > 1:
            print(f"timed step {k + 1} queued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"timed steps done: {(t1 - t0) / args.steps:.2f} s per step", file=sys.stderr, flush=True)
    prof = g.gsrad.profile_report()
    g.gsrad.profile_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    batch = st["batch"]
    info = batch.info()

    def avg(name):
        return prof[name]["total_ms"] / args.steps if name in prof else 0.0

    t_batch = avg("batch_bounces") + avg("batch_adjoint") + avg("batch_sddmm") + avg("transpose")
    # the same transport, one scene at a time (unbatched launches)
    gBs = batch.unpack(st["gB"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for s in range(len(rooms)):
        _, tp = g.transport_solve(st["ff"][s], st["rhos"][s], st["Es"][s], nb)
        g.transport_backward(st["ff"][s], tp, st["rhos"][s], gBs[s].contiguous())
    torch.cuda.synchronize()
    t_scene = (time.perf_counter() - t2) * 1e3
    print(f"scene-by-scene transport done: {t_scene / 1e3:.2f} s", file=sys.stderr, flush=True)
    rays = sum(sc.n for sc in rooms) * R
    phases = {k: v["total_ms"] / args.steps for k, v in prof.items()}
    bb = prof.get("batch_bounces", {}).get("avg_ms", 0.0)
    _, nnz = batch.ff().info()
    vals = info["vals"]
    # F entries + read B (FP32, or BF16 rows), E, write B (algorithmic)
    per_bounce = nnz * 8 + vals * (8.0 + (2.0 if args.batch_precision == "bf16" else 4.0))
    achieved = per_bounce * nb / (bb * 1e-3) / 1e9 if bb > 0 else None
    result = {
        "metric": "fwd+bwd transport solves/s over a batch of 64 uneven scenes",
        "value": 1e3 / ms,
        "unit": "batch solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if args.batch_precision == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": f"64 cluster rooms, {sum(sc.n for sc in rooms)} surfels (2048-65536 each), "
                               f"U{{{lights[0]}..{lights[1]}}} lights per room, R={R}, top-{topk} F, K={K}, "
                               f"{nb} bounces, fwd+bwd, {args.batch_precision.upper()} batched transport",
                   "scenes": len(rooms), "surfels": sum(sc.n for sc in rooms), "lights": sum(Lts),
                   "rays": rays, "nnz": nnz, "values": vals},
        "batch_transport_ms": t_batch,
        "per_scene_transport_ms": t_scene,
        "speedup_vs_per_scene": t_scene / t_batch if t_batch > 0 else None,
        "lanes_per_row": {"bounce": info["lanes_bounce"], "adjoint": info["lanes_adjoint"]},
        "grays_per_s": (rays / ((avg("ray_pools") + avg("ff_trace")) * 1e-3) / 1e9
                        if avg("ff_trace") > 0 else None),
        "bounce_updates_per_s": _updates(nb * sum(sc.n * l for sc, l in zip(rooms, Lts)), phases.get("batch_bounces", 0.0)),
        "adjoint_updates_per_s": _updates(nb * sum(sc.n * l for sc, l in zip(rooms, Lts)), phases.get("batch_adjoint", 0.0)),
        "phase_ms_per_step": {k: round(v, 4) for k, v in sorted(phases.items())},
        "roofline": {"kernel": "batch_bounces", "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS if achieved else None,
                     "traffic": measured_traffic("batch_bounces"),
                     "bytes_per_launch": per_bounce, "launches_per_graph": nb},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = batch_cpu_baseline(rooms, st, nnz, vals, np)
    print(json.dumps(result))


def batch_cpu_baseline(rooms, st, nnz, vals, np, n_recv=1500):
    """The FP64 oracle on the host cores on a bounded sample of the uneven
    batch, scaled to one full step: form-factor rows and direct light of
    n_recv receivers of the largest room (brute force, so a receiver costs
    in proportion to its room's size; scaled by sum n_s^2 / n_big), plus the
    bounces and adjoint of the smallest room on its ray-cast F (scaled by
    stored entries x columns)."""
    import oracle
    import scipy.sparse as sp
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    big = max(range(len(rooms)), key=lambda s: rooms[s].n)
    sm = min(range(len(rooms)), key=lambda s: rooms[s].n)
    sc = rooms[big]
    te = oracle.default_t_eps(sc.surfels)
    recv = np.sort(np.random.default_rng(13).choice(sc.n, size=n_recv, replace=False)).astype(np.int64)
    t0 = time.perf_counter()
    oracle.ff_rows(sc.surfels, recv, sc.R, sc.seed, te, sc.t_min, 512, n_threads=threads)
    oracle.direct_light(sc.surfels, sc.albedo, sc.light_pos, sc.light_I, sc.K, te, receivers=recv,
                        n_threads=threads)
    t_rows = time.perf_counter() - t0
    scale_rows = sum(r.n * r.n for r in rooms) / sc.n / n_recv
    s = rooms[sm]
    rp, col, val = (x.cpu().numpy() for x in st["ff"][sm].csr())
    F = sp.csr_matrix((val.astype(np.float64), col, rp), shape=(s.n, s.n))
    rho = st["rhos"][sm].cpu().numpy().astype(np.float64)
    E = st["Es"][sm].cpu().numpy().astype(np.float64)
    t0 = time.perf_counter()
    _, tape = oracle.bounce(F, rho, E, s.n_bounces, keep_tape=True)
    oracle.adjoint(F, rho, tape, E)
    t_lin = time.perf_counter() - t0
    C = s.n_lights * s.K * 3
    # linear algebra in proportion to stored entries x columns (vals / rows = mean columns per row)
    t_step = t_rows * scale_rows + t_lin * (nnz * (vals / sum(r.n for r in rooms))) / max(F.nnz * C, 1)
    return {"value": 1.0 / t_step, "unit": "batch solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_recv} receivers of the largest room ({sc.n} surfels; form-factor rows and direct light, "
                      f"brute force) scaled by sum n_s^2 / n_big, plus bounces+adjoint of the smallest room "
                      f"({s.n} surfels, {F.nnz} entries x {C} columns) scaled by entries x columns",
            "seconds_measured": t_rows + t_lin}


def _slice_inputs(scenes, np, N, Lt, K, lights):
    E = np.zeros((N, Lt, K, 3), np.float32)
    gB = np.zeros((N, Lt, K, 3), np.float32)
    Es = scenes.seeded_array((N, len(lights), K, 3), seed=2)
    gBs = scenes.seeded_array((N, len(lights), K, 3), seed=3, lo=-1, hi=1)
    E[:, lights] = Es
    gB[:, lights] = gBs
    return E, gB, Es, gBs


def dense_slice_errors(g, torch, np, N, k, Lt, K, nb, lights=(0, 57)):
    """BF16 results of the full launch (N rows, Lt*K*3 columns) on a seeded
    operator with k entries per row, E and grad_B non-zero for two lights
    only: the transport is separable over columns, so the oracle's
    FP64 run on those lights' columns gives B, dL/dE, dL/drho and dL/dF at
    the stored entries of the whole launch."""
    import oracle
    import scenes
    import scipy.sparse as sp
    lights = list(lights)
    rp, c, v = scenes.seeded_csr(N, k, seed=41)
    F = sp.csr_matrix((v.astype(np.float64), c, rp), shape=(N, N))
    rho = scenes.seeded_array((N, 3), seed=1, lo=0.1, hi=0.9)
    E, gB, Es, gBs = _slice_inputs(scenes, np, N, Lt, K, lights)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()   # noqa: E731
    ff = g.ff_dense(g.ff_from_csr(d(rp), d(c), d(v)))
    B, tape = g.transport_solve(ff, d(rho), d(E), nb, precision=g.BF16)
    gE, gr, gF = g.transport_backward(ff, tape, d(rho), d(gB))
    B, gE, gr, gF = (x.cpu().numpy() for x in (B, gE, gr, gF))
    Bo, tp = oracle.bounce(F, rho, Es, nb, keep_tape=True)
    gEo, gro, gFo = oracle.adjoint(F, rho, tp, gBs)

    def rel(x, ref):
        return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))

    return {"B": rel(B[:, lights], Bo), "grad_E": rel(gE[:, lights], gEo), "grad_rho": rel(gr, gro),
            "grad_F": rel(gF, gFo),
            "operator": f"seeded {N}-row CSR, {F.nnz} entries, lights {lights} of {Lt} non-zero"}


def dense_cpu_baseline(np, N, k, Lt, K, nb):
    """The FP64 oracle's bounces + adjoint (with dL/dF at the stored entries)
    for one SH coefficient of one light (3 columns) on a seeded operator of
    the workload's shape, scaled to all Lt*K*3 columns."""
    import oracle
    import scenes
    import scipy.sparse as sp
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rp, c, v = scenes.seeded_csr(N, k, seed=41)
    F = sp.csr_matrix((v.astype(np.float64), c, rp), shape=(N, N))
    rho = scenes.seeded_array((N, 3), seed=1, lo=0.1, hi=0.9)
    Es = scenes.seeded_array((N, 1, 1, 3), seed=2)
    gBs = scenes.seeded_array((N, 1, 1, 3), seed=3, lo=-1, hi=1)
    t0 = time.perf_counter()
    Bo, tp = oracle.bounce(F, rho, Es, nb, keep_tape=True)
    oracle.adjoint(F, rho, tp, gBs)
    t = time.perf_counter() - t0
    scale = Lt * K
    return {"value": 1.0 / (t * scale), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 bounces + adjoint for 3 of {Lt * K * 3} columns on a seeded {N}-row operator with "
                      f"{F.nnz} entries (scipy sparse, one thread), scaled x{scale}",
            "seconds_measured": t}


if __name__ == "__main__":
    main()
