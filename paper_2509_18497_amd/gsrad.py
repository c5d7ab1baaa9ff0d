"""Python binding of libgsrad (argument marshalling only).

Every function here forwards to the C entry point of the same name in
``include/gsrad.h``; all arithmetic runs in the HIP kernels of libgsrad.so.
PyTorch supplies device memory and the current stream.  If the shared
library is missing this module raises on first use: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsrad.so")

OK, EINVAL, ENOMEM, EHIP, ENAN, EOVERFLOW, ESTATE = 0, -1, -2, -3, -4, -5, -6
FP32 = 0
BF16 = 1
FF_NO_RECORDS = 1
FF_COMPACT = 2
SOA = ("px", "py", "pz", "tux", "tuy", "tuz", "tvx", "tvy", "tvz", "nx", "ny", "nz", "su", "sv", "opacity")

EXPORTS = ("gsrad_version", "gsrad_last_error", "gsrad_build_bvh", "gsrad_bvh_info", "gsrad_bvh_height",
           "gsrad_effective_area", "gsrad_reflectance", "gsrad_form_factors", "gsrad_ff_info", "gsrad_ff_view",
           "gsrad_ff_copy", "gsrad_ff_from_csr", "gsrad_ff_dense", "gsrad_direct_light", "gsrad_transport_solve",
           "gsrad_transport_solve_noalloc", "gsrad_brdf_reflectance", "gsrad_brdf_backward",
           "gsrad_direct_light_sh", "gsrad_transport_solve_sh", "gsrad_transport_backward_sh",
           "gsrad_batch_set_lanes", "gsrad_batch_set_precision", "gsrad_ff_center", "gsrad_ff_center_backward",
           "gsrad_geometry_backward", "gsrad_direct_light_backward", "gsrad_mc_create", "gsrad_mc_estimate",
           "gsrad_mc_solve", "gsrad_mc_destroy",
           "gsrad_transport_backward", "gsrad_tape_grad_F_dense", "gsrad_opacity_backward", "gsrad_ray_hits",
           "gsrad_check", "gsrad_check_reciprocity", "gsrad_profile_enable", "gsrad_profile_report", "gsrad_bvh_destroy", "gsrad_ff_destroy",
           "gsrad_tape_destroy", "gsrad_batch_create", "gsrad_batch_info", "gsrad_batch_ff",
           "gsrad_batch_transport_solve", "gsrad_batch_transport_backward", "gsrad_batch_destroy")


class GsradError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


class _Surfels(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in SOA] + [("n", ctypes.c_int64)]


class _SurfelGrads(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in SOA]


class _FFParams(ctypes.Structure):
    _fields_ = [("rays_per_surfel", ctypes.c_int32), ("topk", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("t_min", ctypes.c_float), ("t_eps", ctypes.c_float), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None


def lib():
    """Load libgsrad.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2509_18497_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        pvp = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "gsrad_version": ([], ctypes.c_char_p),
            "gsrad_last_error": ([], ctypes.c_char_p),
            "gsrad_build_bvh": ([ctypes.POINTER(_Surfels), pvp, vp], i32),
            "gsrad_bvh_info": ([vp, ctypes.POINTER(i64), ctypes.POINTER(f32)], i32),
            "gsrad_bvh_height": ([vp, ctypes.POINTER(i32)], i32),
            "gsrad_effective_area": ([vp, vp, vp], i32),
            "gsrad_reflectance": ([vp, vp, vp, vp], i32),
            "gsrad_form_factors": ([vp, ctypes.POINTER(_FFParams), pvp, vp], i32),
            "gsrad_ff_info": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64)], i32),
            "gsrad_ff_view": ([vp, pvp, pvp, pvp], i32),
            "gsrad_ff_copy": ([vp, vp, vp, vp, vp], i32),
            "gsrad_ff_from_csr": ([i64, i64, vp, vp, vp, pvp, vp], i32),
            "gsrad_ff_dense": ([vp, vp], i32),
            "gsrad_check_reciprocity": ([vp, vp, vp, vp], i32),
            "gsrad_batch_create": ([vp, i32, vp, i32, pvp, vp], i32),
            "gsrad_batch_info": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32),
                                  ctypes.POINTER(i32)], i32),
            "gsrad_batch_ff": ([vp, pvp], i32),
            "gsrad_batch_transport_solve": ([vp, vp, vp, i32, vp, vp], i32),
            "gsrad_batch_transport_backward": ([vp, vp, vp, vp, vp, vp, vp], i32),
            "gsrad_batch_set_lanes": ([vp, i32, i32], i32),
            "gsrad_batch_set_precision": ([vp, i32], i32),
            "gsrad_ff_center": ([vp, vp, vp, pvp, vp], i32),
            "gsrad_ff_center_backward": ([vp, vp, vp, vp, vp, ctypes.POINTER(_SurfelGrads), vp], i32),
            "gsrad_geometry_backward": ([vp, vp, vp, ctypes.POINTER(_SurfelGrads), vp], i32),
            "gsrad_direct_light_backward": ([vp, vp, vp, vp, i32, i32, vp, vp, vp, vp, ctypes.POINTER(_SurfelGrads),
                                             vp], i32),
            "gsrad_tape_grad_F_dense": ([vp, vp, vp], i32),
            "gsrad_direct_light": ([vp, vp, vp, vp, i32, i32, vp, vp], i32),
            "gsrad_transport_solve": ([vp, vp, vp, i32, i32, i32, i32, vp, pvp, vp], i32),
            "gsrad_transport_solve_noalloc": ([vp, vp, vp, i32, i32, i32, vp, vp], i32),
            "gsrad_brdf_reflectance": ([vp, vp, vp, vp, vp, i32, vp, vp], i32),
            "gsrad_brdf_backward": ([vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp], i32),
            "gsrad_direct_light_sh": ([vp, vp, i32, vp, vp, i32, vp, vp], i32),
            "gsrad_transport_solve_sh": ([vp, vp, vp, vp, i32, i32, i32, vp, pvp, vp], i32),
            "gsrad_transport_backward_sh": ([vp, vp, vp, vp, vp, vp, vp, vp, vp], i32),
            "gsrad_transport_backward": ([vp, vp, vp, vp, vp, vp, vp, vp], i32),
            "gsrad_opacity_backward": ([vp, vp, vp, vp, vp, vp, vp, vp], i32),
            "gsrad_ray_hits": ([vp, ctypes.POINTER(_FFParams), vp, i64, i32, vp, vp, vp, vp, vp, vp, vp], i32),
            "gsrad_check": ([vp, vp, vp, vp, i32, i32, ctypes.POINTER(ctypes.c_double), vp], i32),
            "gsrad_profile_enable": ([i32], i32),
            "gsrad_profile_report": ([ctypes.c_char_p, i64], i32),
            "gsrad_bvh_destroy": ([vp], None),
            "gsrad_ff_destroy": ([vp], None),
            "gsrad_tape_destroy": ([vp], None),
            "gsrad_batch_destroy": ([vp], None),
            "gsrad_mc_create": ([vp, i32, i32, pvp, vp], i32),
            "gsrad_mc_estimate": ([vp, vp, vp, vp, vp, i32, i32, ctypes.c_uint64, i32, vp, vp], i32),
            "gsrad_mc_solve": ([vp, vp, vp, vp, i32, i32, i32, ctypes.c_uint64, vp, vp, vp], i32),
            "gsrad_mc_destroy": ([vp], None),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status: int, fn: str):
    if status != OK:
        raise GsradError(fn, status, lib().gsrad_last_error().decode())


def _stream(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor], dtype=torch.float32, name: str = "tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class _Handle:
    _destroy = None

    def __init__(self):
        self.h = ctypes.c_void_p(None)

    def __del__(self):
        if self._destroy and self.h and self.h.value and _lib is not None:
            getattr(_lib, self._destroy)(self.h)
            self.h = ctypes.c_void_p(None)


class BVH(_Handle):
    _destroy = "gsrad_bvh_destroy"
    n = 0

    def info(self):
        n, te = ctypes.c_int64(), ctypes.c_float()
        _check(lib().gsrad_bvh_info(self.h, ctypes.byref(n), ctypes.byref(te)), "gsrad_bvh_info")
        return int(n.value), float(te.value)

    def height(self) -> int:
        h = ctypes.c_int32()
        _check(lib().gsrad_bvh_height(self.h, ctypes.byref(h)), "gsrad_bvh_height")
        return int(h.value)


class FF(_Handle):
    _destroy = "gsrad_ff_destroy"

    def info(self):
        n, nnz = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().gsrad_ff_info(self.h, ctypes.byref(n), ctypes.byref(nnz)), "gsrad_ff_info")
        return int(n.value), int(nnz.value)

    def csr(self, stream=None):
        """Copies of (row_ptr int64[n+1], col int32[nnz], val float32[nnz])."""
        n, nnz = self.info()
        dev = torch.device("cuda")
        rp = torch.empty(n + 1, dtype=torch.int64, device=dev)
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        val = torch.empty(max(nnz, 1), dtype=torch.float32, device=dev)
        _check(lib().gsrad_ff_copy(self.h, _ptr(rp, torch.int64), _ptr(col, torch.int32), _ptr(val), _stream(stream)),
               "gsrad_ff_copy")
        return rp, col[:nnz], val[:nnz]


class Tape(_Handle):
    _destroy = "gsrad_tape_destroy"


def version() -> str:
    return lib().gsrad_version().decode()


def build_bvh(surfels: Dict[str, torch.Tensor], bvh: Optional[BVH] = None, stream=None) -> BVH:
    n = int(surfels["px"].shape[0])
    ptrs = []
    for f in SOA:
        t = surfels[f]
        if t.shape != (n,):
            raise ValueError(f"surfel field {f} must have shape ({n},)")
        ptrs.append(_ptr(t, name=f))
    s = _Surfels(*ptrs, n)
    out = bvh if bvh is not None else BVH()
    _check(lib().gsrad_build_bvh(ctypes.byref(s), ctypes.byref(out.h), _stream(stream)), "gsrad_build_bvh")
    out.n = n
    return out


def effective_area(bvh: BVH, stream=None) -> torch.Tensor:
    a = torch.empty(bvh.n, dtype=torch.float64, device="cuda")
    _check(lib().gsrad_effective_area(bvh.h, _ptr(a, torch.float64), _stream(stream)), "gsrad_effective_area")
    return a


def reflectance(bvh: BVH, albedo: torch.Tensor, stream=None) -> torch.Tensor:
    if albedo.shape != (bvh.n, 3):
        raise ValueError("albedo must be [n, 3]")
    rho = torch.empty_like(albedo)
    _check(lib().gsrad_reflectance(bvh.h, _ptr(albedo, name="albedo"), _ptr(rho), _stream(stream)),
           "gsrad_reflectance")
    return rho


def form_factors(bvh: BVH, rays_per_surfel: int, seed: int, t_min: float = 1e-4, t_eps: float = 0.0,
                 topk: int = 0, ff: Optional[FF] = None, records: bool = True, compact: bool = False,
                 stream=None) -> FF:
    p = _FFParams(int(rays_per_surfel), int(topk), int(seed) & 0xFFFFFFFFFFFFFFFF, float(t_min), float(t_eps),
                  (0 if records else FF_NO_RECORDS) | (FF_COMPACT if compact else 0), 0)
    out = ff if ff is not None else FF()
    _check(lib().gsrad_form_factors(bvh.h, ctypes.byref(p), ctypes.byref(out.h), _stream(stream)),
           "gsrad_form_factors")
    return out


def ff_from_csr(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, ff: Optional[FF] = None,
                stream=None) -> FF:
    n = int(row_ptr.shape[0]) - 1
    nnz = int(col.shape[0])
    out = ff if ff is not None else FF()
    _check(lib().gsrad_ff_from_csr(n, nnz, _ptr(row_ptr, torch.int64, "row_ptr"), _ptr(col, torch.int32, "col"),
                                   _ptr(val, name="val"), ctypes.byref(out.h), _stream(stream)), "gsrad_ff_from_csr")
    return out


def direct_light(bvh: BVH, albedo: torch.Tensor, light_pos: torch.Tensor, light_I: torch.Tensor, K: int,
                 out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    Lt = int(light_pos.shape[0])
    if light_pos.shape != (Lt, 3) or light_I.shape != (Lt,):
        raise ValueError("light_pos must be [Lt, 3] and light_I [Lt]")
    E = out if out is not None else torch.empty((bvh.n, Lt, K, 3), dtype=torch.float32, device="cuda")
    _check(lib().gsrad_direct_light(bvh.h, _ptr(albedo, name="albedo"), _ptr(light_pos, name="light_pos"),
                                    _ptr(light_I, name="light_I"), Lt, int(K), _ptr(E, name="E"), _stream(stream)),
           "gsrad_direct_light")
    return E


class Batch(_Handle):
    """Scenes of uneven size sharing one block-diagonal F; E, B and their
    gradients are flat arrays of the scenes' [n_s, Lt_s, K, 3] blocks in
    scene order (see pack / unpack)."""
    _destroy = "gsrad_batch_destroy"

    def info(self):
        r, v, lf, la = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().gsrad_batch_info(self.h, ctypes.byref(r), ctypes.byref(v), ctypes.byref(lf), ctypes.byref(la)),
               "gsrad_batch_info")
        return {"rows": int(r.value), "vals": int(v.value), "lanes_bounce": int(lf.value),
                "lanes_adjoint": int(la.value)}

    def ff(self) -> "FF":
        """The block-diagonal F (owned by the batch)."""
        out = _BorrowedFF()
        _check(lib().gsrad_batch_ff(self.h, ctypes.byref(out.h)), "gsrad_batch_ff")
        out.owner = self
        return out

    def pack(self, blocks) -> torch.Tensor:
        """Concatenate per-scene [n_s, Lt_s, K, 3] tensors into the flat layout."""
        return torch.cat([b.reshape(-1) for b in blocks]).contiguous()

    def unpack(self, flat: torch.Tensor):
        """Split a flat array back into per-scene [n_s, Lt_s, K, 3] views."""
        out, off = [], 0
        for n, lt in zip(self.scene_rows, self.lights):
            m = n * lt * self.K * 3
            out.append(flat[off:off + m].view(n, lt, self.K, 3))
            off += m
        return out


class _BorrowedFF(FF):
    _destroy = None


def batch_create(ffs, lights, K: int, batch: Optional[Batch] = None, stream=None) -> Batch:
    """Join the scenes' operators into one batch (scene s lit by lights[s]
    lights); an existing batch of the same layout is refilled in place."""
    S = len(ffs)
    arr = (ctypes.c_void_p * S)(*[f.h.value for f in ffs])
    lt = (ctypes.c_int32 * S)(*[int(x) for x in lights])
    b = batch if batch is not None else Batch()
    _check(lib().gsrad_batch_create(arr, S, lt, int(K), ctypes.byref(b.h), _stream(stream)), "gsrad_batch_create")
    b.scene_rows = [f.info()[0] for f in ffs]
    b.lights = [int(x) for x in lights]
    b.K = int(K)
    return b


def batch_set_lanes(batch: Batch, lanes_bounce: int, lanes_adjoint: int):
    """Force the lanes per row of the batch launches (16, 32, 64; 0 = timed)."""
    _check(lib().gsrad_batch_set_lanes(batch.h, int(lanes_bounce), int(lanes_adjoint)), "gsrad_batch_set_lanes")


def batch_set_precision(batch: Batch, precision: int):
    """FP32 (default) or BF16 gathered rows in the batch's transport."""
    _check(lib().gsrad_batch_set_precision(batch.h, int(precision)), "gsrad_batch_set_precision")


def batch_transport_solve(batch: Batch, rho: torch.Tensor, E: torch.Tensor, n_bounces: int,
                          out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """B = E + rho*(F B), n_bounces times, on every scene of the batch (flat E)."""
    B = out if out is not None else torch.empty_like(E)
    _check(lib().gsrad_batch_transport_solve(batch.h, _ptr(rho, name="rho"), _ptr(E, name="E"), int(n_bounces),
                                             _ptr(B, name="B"), _stream(stream)), "gsrad_batch_transport_solve")
    return B


def batch_transport_backward(batch: Batch, rho: torch.Tensor, grad_B: torch.Tensor, want_grad_F: bool = True,
                             out: Optional[torch.Tensor] = None, stream=None):
    """dL/dE (flat, into out if given), dL/drho, dL/dF at the block-diagonal
    F's entries."""
    grad_E = out if out is not None else torch.empty_like(grad_B)
    grad_rho = torch.empty_like(rho)
    _, nnz = batch.ff().info()
    grad_F = torch.empty(max(nnz, 1), dtype=torch.float32, device="cuda") if want_grad_F else None
    _check(lib().gsrad_batch_transport_backward(batch.h, _ptr(rho, name="rho"), _ptr(grad_B, name="grad_B"),
                                                _ptr(grad_E), _ptr(grad_rho),
                                                _ptr(grad_F) if grad_F is not None else None, _stream(stream)),
           "gsrad_batch_transport_backward")
    return grad_E, grad_rho, (grad_F[:nnz] if grad_F is not None else None)


def ff_center(bvh: BVH, pattern: FF, lam: torch.Tensor, ff: Optional[FF] = None, stream=None) -> FF:
    """Centre-to-centre form factors lambda_j A_j T_ij |n_i.w||n_j.w| / (pi r^2)
    on pattern's entries (Sec. 8)."""
    out = ff if ff is not None else FF()
    _check(lib().gsrad_ff_center(bvh.h, pattern.h, _ptr(lam, name="lambda"), ctypes.byref(out.h), _stream(stream)),
           "gsrad_ff_center")
    return out


def ff_center_backward(bvh: BVH, ff: FF, lam: torch.Tensor, grad_F: torch.Tensor, stream=None):
    """(dL/dlambda [n], {field: dL/dfield [n]} for the 15 surfel fields) of
    sum grad_F * F through ff_center."""
    n = bvh.n
    dev = torch.device("cuda")
    out = {f: torch.empty(n, dtype=torch.float32, device=dev) for f in SOA}
    gl = torch.empty(n, dtype=torch.float32, device=dev)
    sg = _SurfelGrads(*[out[f].data_ptr() for f in SOA])
    gF = grad_F if grad_F.numel() > 0 else torch.zeros(1, dtype=torch.float32, device=dev)
    _check(lib().gsrad_ff_center_backward(bvh.h, ff.h, _ptr(lam, name="lambda"), _ptr(gF, name="grad_F"), _ptr(gl),
                                          ctypes.byref(sg), _stream(stream)), "gsrad_ff_center_backward")
    return gl, out


def geometry_backward(bvh: BVH, ff: FF, grad_F: torch.Tensor, stream=None) -> Dict[str, torch.Tensor]:
    """{field: dL/dfield [n]} for the 15 surfel fields through the ray-cast F
    (from its recorded hits) for dL/dF = grad_F."""
    n = bvh.n
    out = {f: torch.empty(n, dtype=torch.float32, device="cuda") for f in SOA}
    sg = _SurfelGrads(*[out[f].data_ptr() for f in SOA])
    gF = grad_F if grad_F.numel() > 0 else torch.zeros(1, dtype=torch.float32, device="cuda")
    _check(lib().gsrad_geometry_backward(bvh.h, ff.h, _ptr(gF, name="grad_F"), ctypes.byref(sg), _stream(stream)),
           "gsrad_geometry_backward")
    return out


def direct_light_backward(bvh: BVH, albedo: torch.Tensor, light_pos: torch.Tensor, light_I: torch.Tensor,
                          grad_E: torch.Tensor, stream=None):
    """(dL/dlight_pos [Lt, 3], dL/dlight_I [Lt], dL/dalbedo [n, 3],
    {field: dL/dfield [n]}) through direct_light for dL/dE = grad_E."""
    n, Lt, K = bvh.n, int(light_pos.shape[0]), int(grad_E.shape[2])
    dev = torch.device("cuda")
    glp = torch.empty((Lt, 3), dtype=torch.float32, device=dev)
    gli = torch.empty(Lt, dtype=torch.float32, device=dev)
    gal = torch.empty((n, 3), dtype=torch.float32, device=dev)
    out = {f: torch.empty(n, dtype=torch.float32, device=dev) for f in SOA}
    sg = _SurfelGrads(*[out[f].data_ptr() for f in SOA])
    _check(lib().gsrad_direct_light_backward(bvh.h, _ptr(albedo, name="albedo"), _ptr(light_pos, name="light_pos"),
                                             _ptr(light_I, name="light_I"), Lt, K, _ptr(grad_E, name="grad_E"),
                                             _ptr(glp), _ptr(gli), _ptr(gal), ctypes.byref(sg), _stream(stream)),
           "gsrad_direct_light_backward")
    return glp, gli, gal, out


class MC(_Handle):
    """Monte-Carlo TD(0) solver state (surfel groups) of one BVH."""
    _destroy = "gsrad_mc_destroy"


def mc_create(bvh: BVH, groups: int = 0, kmeans_iters: int = 8, stream=None) -> MC:
    out = MC()
    _check(lib().gsrad_mc_create(bvh.h, int(groups), int(kmeans_iters), ctypes.byref(out.h), _stream(stream)),
           "gsrad_mc_create")
    out.n = bvh.n
    return out


def mc_estimate(mc: MC, lam: torch.Tensor, rho: torch.Tensor, E: torch.Tensor, B: torch.Tensor, seed: int,
                step: int = 0, stream=None) -> torch.Tensor:
    """One next-event estimate per receiver given the current radiance B."""
    Lt, K = int(E.shape[1]), int(E.shape[2])
    out = torch.empty_like(E)
    _check(lib().gsrad_mc_estimate(mc.h, _ptr(lam, name="lambda"), _ptr(rho, name="rho"), _ptr(E, name="E"),
                                   _ptr(B, name="B"), Lt, K, int(seed) & 0xFFFFFFFFFFFFFFFF, int(step), _ptr(out),
                                   _stream(stream)), "gsrad_mc_estimate")
    return out


def mc_solve(mc: MC, lam: torch.Tensor, rho: torch.Tensor, E: torch.Tensor, steps: int, seed: int, stream=None):
    """(B, visits) after `steps` TD(0) rounds."""
    Lt, K = int(E.shape[1]), int(E.shape[2])
    B = torch.empty_like(E)
    visits = torch.empty(mc.n, dtype=torch.int32, device="cuda")
    _check(lib().gsrad_mc_solve(mc.h, _ptr(lam, name="lambda"), _ptr(rho, name="rho"), _ptr(E, name="E"), Lt, K,
                                int(steps), int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(B), _ptr(visits, torch.int32),
                                _stream(stream)), "gsrad_mc_solve")
    return B, visits


def ff_dense(ff: FF, stream=None) -> FF:
    """Make the dense BF16 copies of F (and F^T) used by precision=BF16."""
    _check(lib().gsrad_ff_dense(ff.h, _stream(stream)), "gsrad_ff_dense")
    return ff


def tape_grad_F_dense(tape: Tape, n: int, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """The dense dL/dF [n, n] of the last backward on a BF16 tape."""
    G = out if out is not None else torch.empty((n, n), dtype=torch.float32, device="cuda")
    _check(lib().gsrad_tape_grad_F_dense(tape.h, _ptr(G, name="grad_F_dense"), _stream(stream)),
           "gsrad_tape_grad_F_dense")
    return G


def transport_solve(ff: FF, rho: torch.Tensor, E: torch.Tensor, n_bounces: int, tape: Optional[Tape] = None,
                    keep_tape: bool = True, out: Optional[torch.Tensor] = None, stream=None, precision: int = FP32):
    """B = E + rho*(F B) iterated n_bounces times from B^(0) = E.  E is
    [n, Lt, K, 3].  precision FP32 (sparse CSR products) or BF16 (dense
    matrix-core products on the copies made by ff_dense).  Returns (B, tape)."""
    if E.dim() != 4 or E.shape[3] != 3:
        raise ValueError("E must be [n, Lt, K, 3]")
    n, Lt, K = int(E.shape[0]), int(E.shape[1]), int(E.shape[2])
    B = out if out is not None else torch.empty_like(E)
    tp = tape if tape is not None else (Tape() if keep_tape else None)
    _check(lib().gsrad_transport_solve(ff.h, _ptr(rho, name="rho"), _ptr(E, name="E"), Lt, K, int(n_bounces),
                                       int(precision),
                                       _ptr(B, name="B"), ctypes.byref(tp.h) if tp is not None else None,
                                       _stream(stream)), "gsrad_transport_solve")
    return B, tp


def transport_solve_noalloc(ff: FF, rho: torch.Tensor, E: torch.Tensor, n_bounces: int, out: torch.Tensor,
                            stream=None) -> torch.Tensor:
    """The FP32 bounces of transport_solve (no tape) through the entry point
    that allocates nothing: its two ping-pong iterates live in the library's
    fixed per-GPU scratch array (at most 64 MiB, i.e. n * C <= 2^23 values);
    the caller provides B in out."""
    if E.dim() != 4 or E.shape[3] != 3:
        raise ValueError("E must be [n, Lt, K, 3]")
    Lt, K = int(E.shape[1]), int(E.shape[2])
    _check(lib().gsrad_transport_solve_noalloc(ff.h, _ptr(rho, name="rho"), _ptr(E, name="E"), Lt, K, int(n_bounces),
                                               _ptr(out, name="out"), _stream(stream)), "gsrad_transport_solve_noalloc")
    return out


def brdf_reflectance(bvh: BVH, k: torch.Tensor, albedo_d: torch.Tensor, albedo_s: torch.Tensor,
                     shininess: torch.Tensor, K: int, stream=None) -> torch.Tensor:
    """R = pi o f^c [n, K, 3] of the diffuse + Phong BRDF (App. A), in each
    surfel's tangent frame."""
    R = torch.empty((bvh.n, int(K), 3), dtype=torch.float32, device="cuda")
    _check(lib().gsrad_brdf_reflectance(bvh.h, _ptr(k, name="k"), _ptr(albedo_d, name="albedo_d"),
                                        _ptr(albedo_s, name="albedo_s"), _ptr(shininess, name="shininess"), int(K),
                                        _ptr(R), _stream(stream)), "gsrad_brdf_reflectance")
    return R


def brdf_backward(bvh: BVH, k, albedo_d, albedo_s, shininess, grad_R: torch.Tensor, stream=None):
    """Gradients of sum(grad_R * R) with respect to (opacity, k, a^d, a^s, s)."""
    n, K = bvh.n, int(grad_R.shape[1])
    dev = torch.device("cuda")
    go = torch.empty(n, dtype=torch.float32, device=dev)
    gk = torch.empty(n, dtype=torch.float32, device=dev)
    gad = torch.empty((n, 3), dtype=torch.float32, device=dev)
    gas = torch.empty((n, 3), dtype=torch.float32, device=dev)
    gs = torch.empty(n, dtype=torch.float32, device=dev)
    _check(lib().gsrad_brdf_backward(bvh.h, _ptr(k, name="k"), _ptr(albedo_d, name="albedo_d"),
                                     _ptr(albedo_s, name="albedo_s"), _ptr(shininess, name="shininess"), K,
                                     _ptr(grad_R, name="grad_R"), _ptr(go), _ptr(gk), _ptr(gad), _ptr(gas), _ptr(gs),
                                     _stream(stream)), "gsrad_brdf_backward")
    return go, gk, gad, gas, gs


def direct_light_sh(bvh: BVH, R: torch.Tensor, light_pos: torch.Tensor, light_I: torch.Tensor,
                    out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """E [n, Lt, K, 3] from point lights through the BRDF coefficients R."""
    Lt, K = int(light_pos.shape[0]), int(R.shape[1])
    if light_pos.shape != (Lt, 3) or light_I.shape != (Lt,):
        raise ValueError("light_pos must be [Lt, 3] and light_I [Lt]")
    E = out if out is not None else torch.empty((bvh.n, Lt, K, 3), dtype=torch.float32, device="cuda")
    _check(lib().gsrad_direct_light_sh(bvh.h, _ptr(R, name="R"), K, _ptr(light_pos, name="light_pos"),
                                       _ptr(light_I, name="light_I"), Lt, _ptr(E, name="E"), _stream(stream)),
           "gsrad_direct_light_sh")
    return E


def transport_solve_sh(ff: FF, bvh: BVH, R: torch.Tensor, E: torch.Tensor, n_bounces: int,
                       tape: Optional[Tape] = None, keep_tape: bool = True, out: Optional[torch.Tensor] = None,
                       stream=None):
    """B = E + R (.) (T B) iterated n_bounces times (directional transfer).
    Returns (B, tape)."""
    if E.dim() != 4 or E.shape[3] != 3:
        raise ValueError("E must be [n, Lt, K, 3]")
    Lt, K = int(E.shape[1]), int(E.shape[2])
    B = out if out is not None else torch.empty_like(E)
    tp = tape if tape is not None else (Tape() if keep_tape else None)
    _check(lib().gsrad_transport_solve_sh(ff.h, bvh.h, _ptr(R, name="R"), _ptr(E, name="E"), Lt, K, int(n_bounces),
                                          _ptr(B, name="B"), ctypes.byref(tp.h) if tp is not None else None,
                                          _stream(stream)), "gsrad_transport_solve_sh")
    return B, tp


def transport_backward_sh(ff: FF, bvh: BVH, tape: Tape, R: torch.Tensor, grad_B: torch.Tensor,
                          want_grad_F: bool = True, stream=None):
    """(grad_E, grad_R, grad_F) of the directional transfer."""
    nnz = ff.info()[1]
    grad_E = torch.empty_like(grad_B)
    grad_R = torch.empty_like(R)
    grad_F = torch.empty(max(nnz, 1), dtype=torch.float32, device="cuda") if want_grad_F else None
    _check(lib().gsrad_transport_backward_sh(ff.h, bvh.h, tape.h, _ptr(R, name="R"), _ptr(grad_B, name="grad_B"),
                                             _ptr(grad_E), _ptr(grad_R),
                                             _ptr(grad_F) if grad_F is not None else None, _stream(stream)),
           "gsrad_transport_backward_sh")
    return grad_E, grad_R, (grad_F[:nnz] if grad_F is not None else None)


def transport_backward(ff: FF, tape: Tape, rho: torch.Tensor, grad_B: torch.Tensor, want_grad_F: bool = True,
                       stream=None):
    grad_E = torch.empty_like(grad_B)
    grad_rho = torch.empty_like(rho)
    _, nnz = ff.info()
    grad_F = torch.empty(max(nnz, 1), dtype=torch.float32, device="cuda") if want_grad_F else None
    _check(lib().gsrad_transport_backward(ff.h, tape.h, _ptr(rho, name="rho"), _ptr(grad_B, name="grad_B"),
                                          _ptr(grad_E), _ptr(grad_rho), _ptr(grad_F) if grad_F is not None else None,
                                          _stream(stream)), "gsrad_transport_backward")
    return grad_E, grad_rho, (grad_F[:nnz] if grad_F is not None else None)


def opacity_backward(bvh: BVH, ff: FF, grad_F: Optional[torch.Tensor], grad_rho: Optional[torch.Tensor],
                     albedo: Optional[torch.Tensor], stream=None):
    grad_o = torch.empty(bvh.n, dtype=torch.float32, device="cuda")
    grad_a = torch.empty((bvh.n, 3), dtype=torch.float32, device="cuda")
    gF = grad_F
    if gF is not None and gF.numel() == 0:
        gF = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib().gsrad_opacity_backward(bvh.h, ff.h, _ptr(gF, name="grad_F"), _ptr(grad_rho, name="grad_rho"),
                                        _ptr(albedo, name="albedo"), _ptr(grad_o), _ptr(grad_a), _stream(stream)),
           "gsrad_opacity_backward")
    return grad_o, grad_a


def ray_hits(bvh: BVH, receivers: torch.Tensor, rays_per_surfel: int, seed: int, t_min: float = 1e-4,
             t_eps: float = 0.0, max_hits: int = 256, stream=None) -> dict:
    """Directions and composited hit lists of every ray of the listed
    receivers (same decisions as form_factors)."""
    p = _FFParams(int(rays_per_surfel), 0, int(seed) & 0xFFFFFFFFFFFFFFFF, float(t_min), float(t_eps), 0, 0)
    m = int(receivers.shape[0])
    R = int(rays_per_surfel)
    dev = torch.device("cuda")
    dirs = torch.empty((m, R, 3), dtype=torch.float32, device=dev)
    cnt = torch.empty((m, R), dtype=torch.int32, device=dev)
    hj = torch.full((m, R, max_hits), -1, dtype=torch.int32, device=dev)
    ht = torch.zeros((m, R, max_hits), dtype=torch.float32, device=dev)
    hf = torch.zeros((m, R, max_hits), dtype=torch.int8, device=dev)
    hT = torch.zeros((m, R, max_hits), dtype=torch.float32, device=dev)
    _check(lib().gsrad_ray_hits(bvh.h, ctypes.byref(p), _ptr(receivers, torch.int64, "receivers"), m, int(max_hits),
                                _ptr(dirs), _ptr(cnt, torch.int32), _ptr(hj, torch.int32), _ptr(ht),
                                _ptr(hf, torch.int8), _ptr(hT), _stream(stream)), "gsrad_ray_hits")
    return {"dirs": dirs, "count": cnt, "j": hj, "t": ht, "front": hf, "T": hT}


def check_reciprocity(bvh: BVH, ff: FF, stream=None) -> dict:
    """FP64 reciprocity of F with the App. E areas: relative L1 asymmetry
    sum|A_i F_ij - A_j F_ji| / sum A_i F_ij and the largest relative entry."""
    out = (ctypes.c_double * 2)()
    _check(lib().gsrad_check_reciprocity(bvh.h, ff.h, out, _stream(stream)), "gsrad_check_reciprocity")
    return {"asymmetry": out[0], "max_entry": out[1]}


def check(ff: FF, rho: torch.Tensor, E: torch.Tensor, B: torch.Tensor, stream=None) -> dict:
    """FP64 residual ||E + rho*(F B) - B|| / ||B||, max row sum of F, and
    whether any input is non-finite."""
    out = (ctypes.c_double * 3)()
    Lt, K = int(E.shape[1]), int(E.shape[2])
    st = lib().gsrad_check(ff.h, _ptr(rho), _ptr(E), _ptr(B), Lt, K, out, _stream(stream))
    res = {"residual": out[0], "max_row_sum": out[1], "non_finite": bool(out[2])}
    if st not in (OK, ENAN):
        _check(st, "gsrad_check")
    return res


def profile_enable(on: bool = True):
    _check(lib().gsrad_profile_enable(1 if on else 0), "gsrad_profile_enable")


def profile_report() -> Dict[str, dict]:
    """Per-phase HIP-event timings since profile_enable(True)."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib().gsrad_profile_report(buf, len(buf)), "gsrad_profile_report")
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, tot, mn, mx = line.split("\t")
        out[name] = {"count": int(cnt), "total_ms": float(tot), "min_ms": float(mn), "max_ms": float(mx),
                     "avg_ms": float(tot) / max(int(cnt), 1)}
    return out


class RadiosityFn(torch.autograd.Function):
    """B = solve(F(opacity), rho = o*a, E) with the hand-written adjoint:
    backward returns dL/dopacity (compositing backward through F plus the
    receiver term), dL/dalbedo and dL/dE.  The BVH and F handles must have
    been built from the same opacity values."""

    @staticmethod
    def forward(ctx, opacity, albedo, E, bvh: BVH, ff: FF, n_bounces: int):
        rho = reflectance(bvh, albedo.contiguous())
        B, tape = transport_solve(ff, rho, E.contiguous(), n_bounces)
        ctx.bvh, ctx.ff, ctx.tape = bvh, ff, tape
        ctx.save_for_backward(rho, albedo)
        return B

    @staticmethod
    def backward(ctx, grad_B):
        rho, albedo = ctx.saved_tensors
        grad_E, grad_rho, grad_F = transport_backward(ctx.ff, ctx.tape, rho, grad_B.contiguous())
        grad_o, grad_a = opacity_backward(ctx.bvh, ctx.ff, grad_F, grad_rho, albedo.contiguous())
        return grad_o, grad_a, grad_E, None, None, None
