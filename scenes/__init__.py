"""Seeded synthetic scene generators: Gaussian surfels, albedo and point lights.

This module only *describes* scenes (where surfels sit, how they are oriented,
their scales, opacities, albedos and the light positions).  It holds none of
the light-transport arithmetic: no rays, no visibility, no form factors, no
bounces.  The same FP32 arrays it returns are fed byte for byte to both the
FP64 CPU oracle and the GPU path.

Surfel parametrisation follows the paper's geometry field (Sec. 3.1, Eq. G):
centre p, tangents t_u, t_v, scales s_u, s_v and normal n = t_u x t_v, plus
a peak opacity o (the opacity profile of App. E evaluated at the centre).

The five workloads (furnace sphere, box room, fruit bowl, multi-light box
room, uneven batch) stand in for the paper's scenes: about 100 images each lit
by a different known point light, an enclosed box with objects inside (Sec. 9,
preliminary enclosed-box experiment) and scenes of ~89K-100K primitives
(Sec. 9 ablations).  No dataset is read.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

SOA_FIELDS = ("px", "py", "pz", "tux", "tuy", "tuz", "tvx", "tvy", "tvz",
              "nx", "ny", "nz", "su", "sv", "opacity")


@dataclass
class Scene:
    """One synthetic workload.  All float arrays are C-contiguous float32."""
    name: str
    surfels: Dict[str, np.ndarray]          # SoA fields, each [N]
    albedo: np.ndarray                      # [N, 3] diffuse albedo a_i
    light_pos: np.ndarray                   # [Lt, 3]
    light_I: np.ndarray                     # [Lt] isotropic radiant intensity
    K: int                                  # SH coefficients per channel
    R: int                                  # rays per receiver surfel
    n_bounces: int
    topk: int                               # 0 = keep every F entry
    seed: int                               # Philox key for the rays
    t_min: float = 1e-4                     # transmittance cut-off
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.surfels["px"].shape[0])

    @property
    def n_lights(self) -> int:
        return int(self.light_pos.shape[0])


# --------------------------------------------------------------------------
# frames
# --------------------------------------------------------------------------
def onb_from_normal(n: np.ndarray):
    """Branchless orthonormal basis (Duff et al., JCGT 2017) for unit normals
    n [M,3]; returns (t_u, t_v) with t_u x t_v = n."""
    n = np.asarray(n, dtype=np.float64)
    sign = np.where(n[:, 2] >= 0.0, 1.0, -1.0)
    a = -1.0 / (sign + n[:, 2])
    b = n[:, 0] * n[:, 1] * a
    b1 = np.stack([1.0 + sign * n[:, 0] ** 2 * a, sign * b, -sign * n[:, 0]], axis=1)
    b2 = np.stack([b, sign + n[:, 1] ** 2 * a, -n[:, 1]], axis=1)
    # orient so that b1 x b2 = n
    c = np.cross(b1, b2)
    flip = np.einsum("ij,ij->i", c, n) < 0
    b2[flip] *= -1.0
    return b1, b2


def _spin(tu, tv, rng):
    """Rotate the tangent pair in its plane by a random angle."""
    ang = rng.uniform(0.0, 2.0 * math.pi, size=tu.shape[0])
    ca, sa = np.cos(ang)[:, None], np.sin(ang)[:, None]
    return ca * tu + sa * tv, -sa * tu + ca * tv


def _pack(p, n, tu, tv, su, sv, op, albedo):
    p = np.asarray(p, np.float64)
    d = {
        "px": p[:, 0], "py": p[:, 1], "pz": p[:, 2],
        "tux": tu[:, 0], "tuy": tu[:, 1], "tuz": tu[:, 2],
        "tvx": tv[:, 0], "tvy": tv[:, 1], "tvz": tv[:, 2],
        "nx": n[:, 0], "ny": n[:, 1], "nz": n[:, 2],
        "su": su, "sv": sv, "opacity": op,
    }
    sur = {k: np.ascontiguousarray(np.asarray(v, dtype=np.float32)) for k, v in d.items()}
    alb = np.ascontiguousarray(np.asarray(albedo, dtype=np.float32).reshape(-1, 3))
    return sur, alb


# --------------------------------------------------------------------------
# 1. furnace sphere
# --------------------------------------------------------------------------
def furnace(seed: int = 1, n: int = 512, radius: float = 0.08, opacity: float = 0.99,
            albedo: float = 0.5, R: int = 64, n_bounces: int = 6) -> Scene:
    """512 inward-facing surfels placed uniformly on the unit sphere, one point
    light of intensity 1 at the centre."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    p = g / np.linalg.norm(g, axis=1, keepdims=True)
    nrm = -p
    tu, tv = onb_from_normal(nrm)
    tu, tv = _spin(tu, tv, rng)
    su = np.full(n, radius)
    op = np.full(n, opacity)
    alb = np.full((n, 3), albedo)
    sur, alb = _pack(p, nrm, tu, tv, su, su, op, alb)
    return Scene("furnace", sur, alb,
                 np.zeros((1, 3), np.float32), np.ones(1, np.float32),
                 K=1, R=R, n_bounces=n_bounces, topk=0, seed=seed)


# --------------------------------------------------------------------------
# planar faces on a jittered grid
# --------------------------------------------------------------------------
@dataclass
class _Face:
    origin: np.ndarray   # corner
    eu: np.ndarray       # full edge vector along u
    ev: np.ndarray       # full edge vector along v
    normal: np.ndarray   # unit normal (front face)
    tag: str


def _face_points(f: _Face, h: float, rng):
    Lu, Lv = np.linalg.norm(f.eu), np.linalg.norm(f.ev)
    nu, nv = max(1, int(round(Lu / h))), max(1, int(round(Lv / h)))
    iu, iv = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    hu, hv = Lu / nu, Lv / nv
    ju = rng.uniform(-0.25, 0.25, size=iu.shape) * hu
    jv = rng.uniform(-0.25, 0.25, size=iv.shape) * hv
    uu = ((iu + 0.5) * hu + ju).ravel() / Lu
    vv = ((iv + 0.5) * hv + jv).ravel() / Lv
    pts = f.origin[None, :] + uu[:, None] * f.eu[None, :] + vv[:, None] * f.ev[None, :]
    return pts


def _box_faces(center, half, tag, outward=True, skip_bottom=True):
    c = np.asarray(center, float)
    hx, hy, hz = half
    faces = []
    s = 1.0 if outward else -1.0
    # +x / -x
    faces.append(_Face(c + [hx, -hy, -hz], np.array([0, 2 * hy, 0.]), np.array([0, 0, 2 * hz]), s * np.array([1., 0, 0]), tag + "+x"))
    faces.append(_Face(c + [-hx, -hy, -hz], np.array([0, 2 * hy, 0.]), np.array([0, 0, 2 * hz]), s * np.array([-1., 0, 0]), tag + "-x"))
    # +y / -y
    faces.append(_Face(c + [-hx, hy, -hz], np.array([2 * hx, 0, 0.]), np.array([0, 0, 2 * hz]), s * np.array([0, 1., 0]), tag + "+y"))
    if not skip_bottom:
        faces.append(_Face(c + [-hx, -hy, -hz], np.array([2 * hx, 0, 0.]), np.array([0, 0, 2 * hz]), s * np.array([0, -1., 0]), tag + "-y"))
    # +z / -z
    faces.append(_Face(c + [-hx, -hy, hz], np.array([2 * hx, 0, 0.]), np.array([0, 2 * hy, 0]), s * np.array([0, 0, 1.]), tag + "+z"))
    faces.append(_Face(c + [-hx, -hy, -hz], np.array([2 * hx, 0, 0.]), np.array([0, 2 * hy, 0]), s * np.array([0, 0, -1.]), tag + "-z"))
    return faces


BOX_ROOM_HALF = 4.0
BOX_ROOM_BOXES = (((-1.5, -2.5, -1.0), (1.0, 1.5, 1.0)),
                  ((1.5, -3.0, 1.0), (1.0, 1.0, 1.0)))


def _room_faces():
    L = BOX_ROOM_HALF
    W = 2 * L
    faces = [
        _Face(np.array([-L, -L, -L]), np.array([W, 0, 0.]), np.array([0, 0, W]), np.array([0, 1., 0]), "floor"),
        _Face(np.array([-L, L, -L]), np.array([W, 0, 0.]), np.array([0, 0, W]), np.array([0, -1., 0]), "ceiling"),
        _Face(np.array([-L, -L, -L]), np.array([0, W, 0.]), np.array([0, 0, W]), np.array([1., 0, 0]), "left"),
        _Face(np.array([L, -L, -L]), np.array([0, W, 0.]), np.array([0, 0, W]), np.array([-1., 0, 0]), "right"),
        _Face(np.array([-L, -L, -L]), np.array([W, 0, 0.]), np.array([0, W, 0]), np.array([0, 0, 1.]), "back"),
    ]
    for bi, (c, hlf) in enumerate(BOX_ROOM_BOXES):
        faces += _box_faces(c, hlf, f"box{bi}")
    return faces


def _inside_boxes(p, margin=0.0):
    inside = np.zeros(p.shape[0], bool)
    for c, hlf in BOX_ROOM_BOXES:
        c = np.asarray(c)
        hlf = np.asarray(hlf) + margin
        inside |= np.all(np.abs(p - c[None, :]) < hlf[None, :], axis=1)
    return inside


def _box_room_geometry(n: int, rng):
    faces = _room_faces()
    area = sum(np.linalg.norm(f.eu) * np.linalg.norm(f.ev) for f in faces)
    h = math.sqrt(area / n)
    for _ in range(200):
        pts, nrm, tags = [], [], []
        for f in faces:
            q = _face_points(f, h, rng)
            if f.tag == "floor":
                # floor under a box is hidden inside it
                keep = ~_inside_boxes(q + np.array([0, 1e-3, 0]), margin=0.0)
                q = q[keep]
            pts.append(q)
            nrm.append(np.repeat(f.normal[None, :], q.shape[0], axis=0))
            tags += [f.tag] * q.shape[0]
        P = np.concatenate(pts)
        if P.shape[0] >= n:
            break
        h *= 0.995
    Nn = np.concatenate(nrm)
    tags = np.array(tags)
    if P.shape[0] > n:
        keep = np.sort(rng.choice(P.shape[0], size=n, replace=False))
        P, Nn, tags = P[keep], Nn[keep], tags[keep]
    return P, Nn, tags, h


def box_room(seed: int = 2, n: int = 16384, n_lights: int = 1, K: int = 9, R: int = 256,
             n_bounces: int = 8, light_radius: float = 3.0) -> Scene:
    """Room [-4,4]^3 with five walls (the +z side is open) and two boxes on
    the floor, surfels on a jittered grid with spacing h and scale s = h.
    One light near the ceiling, or ``n_lights`` lights on a sphere."""
    rng = np.random.default_rng(seed)
    P, Nn, tags, h = _box_room_geometry(n, rng)
    tu, tv = onb_from_normal(Nn)
    tu, tv = _spin(tu, tv, rng)
    su = np.full(n, h)
    op = rng.uniform(0.9, 1.0, size=n)
    alb = rng.uniform(0.2, 0.8, size=(n, 3))
    left, right = tags == "left", tags == "right"
    alb[left] = np.stack([rng.uniform(0.6, 0.8, left.sum()), rng.uniform(0.2, 0.3, left.sum()),
                          rng.uniform(0.2, 0.3, left.sum())], axis=1)
    alb[right] = np.stack([rng.uniform(0.2, 0.3, right.sum()), rng.uniform(0.6, 0.8, right.sum()),
                           rng.uniform(0.2, 0.3, right.sum())], axis=1)
    sur, alb = _pack(P, Nn, tu, tv, su, su, op, alb)
    if n_lights == 1:
        lp = np.array([[0.0, 3.6, 0.0]], np.float32)
        li = np.array([16.0], np.float32)
    else:
        lps = []
        while len(lps) < n_lights:
            g = rng.standard_normal(3)
            q = light_radius * g / np.linalg.norm(g)
            if _inside_boxes(q[None, :], margin=0.05)[0]:
                continue
            lps.append(q)
        lp = np.asarray(lps, np.float32)
        li = np.full(n_lights, 16.0, np.float32)
    return Scene("box_room" if n_lights == 1 else "multi_light", sur, alb, lp, li, K=K, R=R,
                 n_bounces=n_bounces, topk=0, seed=seed, meta={"h": h})


# --------------------------------------------------------------------------
# 3. fruit bowl
# --------------------------------------------------------------------------
GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))


def _fib_sphere(m, rng, jitter):
    k = np.arange(m) + 0.5
    z = 1.0 - 2.0 * k / m
    phi = np.arange(m) * GOLDEN_ANGLE + rng.uniform(0, 2 * math.pi)
    rr = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    p = np.stack([rr * np.cos(phi), z, rr * np.sin(phi)], axis=1)
    p += rng.uniform(-jitter, jitter, size=p.shape)
    return p / np.linalg.norm(p, axis=1, keepdims=True)


def _fib_lower_hemisphere(m, rng, jitter):
    k = np.arange(m) + 0.5
    y = -k / m
    phi = np.arange(m) * GOLDEN_ANGLE + rng.uniform(0, 2 * math.pi)
    rr = np.sqrt(np.maximum(0.0, 1.0 - y * y))
    p = np.stack([rr * np.cos(phi), y, rr * np.sin(phi)], axis=1)
    p += rng.uniform(-jitter, jitter, size=p.shape)
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    p[:, 1] = -np.abs(p[:, 1])
    return p


def fruit_bowl(seed: int = 3, n: int = 100_000, n_fruit: int = 20, K: int = 16, R: int = 128,
               n_bounces: int = 8, topk: int = 512) -> Scene:
    """Inner face of a hemispherical bowl of radius 1 (normals towards the
    centre) holding ``n_fruit`` non-overlapping spheres of log-uniform radius
    in [0.05, 0.2]; surfel count per object proportional to its area."""
    rng = np.random.default_rng(seed)
    centers, radii = [], []
    tries = 0
    while len(centers) < n_fruit:
        tries += 1
        if tries > 200000:
            raise RuntimeError("fruit placement failed")
        r = math.exp(rng.uniform(math.log(0.05), math.log(0.2)))
        c = rng.uniform(-1, 1, size=3)
        c[1] = -abs(c[1])
        if np.linalg.norm(c) > 1.0 - r - 0.02:
            continue
        if any(np.linalg.norm(c - c2) < r + r2 + 0.02 for c2, r2 in zip(centers, radii)):
            continue
        centers.append(c)
        radii.append(r)
    areas = np.array([2 * math.pi] + [4 * math.pi * r * r for r in radii])
    counts = np.floor(areas / areas.sum() * n).astype(int)
    counts[0] += n - counts.sum()
    h = math.sqrt(areas.sum() / n)
    P, Nn = [], []
    pb = _fib_lower_hemisphere(counts[0], rng, jitter=0.25 * h)
    P.append(pb)
    Nn.append(-pb)
    for c, r, m in zip(centers, radii, counts[1:]):
        q = _fib_sphere(m, rng, jitter=0.25 * h / r)
        P.append(c[None, :] + r * q)
        Nn.append(q)
    P, Nn = np.concatenate(P), np.concatenate(Nn)
    tu, tv = onb_from_normal(Nn)
    tu, tv = _spin(tu, tv, rng)
    su = np.full(n, h)
    op = rng.beta(8.0, 1.0, size=n)
    alb = rng.uniform(0.1, 0.9, size=(n, 3))
    sur, alb = _pack(P, Nn, tu, tv, su, su, op, alb)
    return Scene("fruit_bowl", sur, alb, np.array([[0.3, 1.5, 0.2]], np.float32),
                 np.array([4.0], np.float32), K=K, R=R, n_bounces=n_bounces, topk=topk,
                 seed=seed, meta={"h": h, "fruit_centers": np.array(centers), "fruit_radii": np.array(radii)})


# --------------------------------------------------------------------------
# 5. uneven batch
# --------------------------------------------------------------------------
def cluster_room(seed: int, n: int, n_lights: int, K: int = 9, R: int = 128, n_bounces: int = 8,
                 half: float = 2.0) -> Scene:
    """Room [-half, half]^3 with five walls (the +z side open, normals
    inward) holding a cluster of 2-6 non-overlapping spheres of radius
    U[0.2, 0.6] half; surfels per object proportional to area (jittered
    grid on the walls, Fibonacci lattices on the spheres), s = h,
    o ~ U[0.85, 1), albedo U[0.2, 0.8]^3, ``n_lights`` lights of intensity 4
    drawn uniformly in the room outside the spheres."""
    rng = np.random.default_rng(seed)
    L, W = half, 2 * half
    walls = [
        _Face(np.array([-L, -L, -L]), np.array([W, 0, 0.]), np.array([0, 0, W]), np.array([0, 1., 0]), "floor"),
        _Face(np.array([-L, L, -L]), np.array([W, 0, 0.]), np.array([0, 0, W]), np.array([0, -1., 0]), "ceiling"),
        _Face(np.array([-L, -L, -L]), np.array([0, W, 0.]), np.array([0, 0, W]), np.array([1., 0, 0]), "left"),
        _Face(np.array([L, -L, -L]), np.array([0, W, 0.]), np.array([0, 0, W]), np.array([-1., 0, 0]), "right"),
        _Face(np.array([-L, -L, -L]), np.array([W, 0, 0.]), np.array([0, W, 0]), np.array([0, 0, 1.]), "back"),
    ]
    n_sph = int(rng.integers(2, 7))
    centers, radii = [], []
    while len(centers) < n_sph:
        r = rng.uniform(0.2, 0.6) * half
        c = rng.uniform(-L + r + 0.05, L - r - 0.05, size=3)
        if any(np.linalg.norm(c - c2) < r + r2 + 0.05 for c2, r2 in zip(centers, radii)):
            continue
        centers.append(c)
        radii.append(r)
    a_walls = 5 * W * W
    a_sph = np.array([4 * math.pi * r * r for r in radii])
    h = math.sqrt((a_walls + a_sph.sum()) / n)
    pts = np.concatenate([_face_points(f, h, rng) for f in walls])
    nrm = np.concatenate([np.repeat(f.normal[None, :], _face_points(f, h, np.random.default_rng(0)).shape[0], axis=0)
                          for f in walls])
    n_w = min(pts.shape[0], int(round(n * a_walls / (a_walls + a_sph.sum()))))
    keep = np.sort(rng.choice(pts.shape[0], size=n_w, replace=False))
    P, Nn = [pts[keep]], [nrm[keep]]
    counts = np.floor(a_sph / a_sph.sum() * (n - n_w)).astype(int)
    counts[0] += (n - n_w) - counts.sum()
    for c, r, m in zip(centers, radii, counts):
        q = _fib_sphere(int(m), rng, jitter=0.25 * h / r)
        P.append(c[None, :] + r * q)
        Nn.append(q)
    P, Nn = np.concatenate(P), np.concatenate(Nn)
    tu, tv = onb_from_normal(Nn)
    tu, tv = _spin(tu, tv, rng)
    su = np.full(n, h)
    op = rng.uniform(0.85, 1.0, size=n)
    alb = rng.uniform(0.2, 0.8, size=(n, 3))
    sur, alb = _pack(P, Nn, tu, tv, su, su, op, alb)
    lps = []
    while len(lps) < n_lights:
        q = rng.uniform(-0.9 * L, 0.9 * L, size=3)
        if any(np.linalg.norm(q - c) < r + 0.05 for c, r in zip(centers, radii)):
            continue
        lps.append(q)
    return Scene("cluster_room", sur, alb, np.asarray(lps, np.float32), np.full(n_lights, 4.0, np.float32), K=K,
                 R=R, n_bounces=n_bounces, topk=0, seed=seed, meta={"h": h})


def uneven_batch(seed: int = 5, n_scenes: int = 64, n_range=(2048, 65536), lights=(8, 100), K: int = 9,
                 R: int = 128, n_bounces: int = 8) -> List[Scene]:
    """Scenes of log-uniform surfel counts in n_range, each a cluster room
    lit by U{lights} point lights."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_scenes):
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        lt = int(rng.integers(lights[0], lights[1] + 1))
        out.append(cluster_room(seed=1000 * seed + s, n=n, n_lights=lt, K=K, R=R, n_bounces=n_bounces))
    return out


# --------------------------------------------------------------------------
# registry
# --------------------------------------------------------------------------
CONFIGS = {
    1: "furnace", 2: "box_room", 3: "fruit_bowl", 4: "multi_light", 5: "uneven_batch",
}


def make_config(which, seed: Optional[int] = None, n: Optional[int] = None, **kw) -> Scene:
    """Build one of the named workloads; ``n`` shrinks it for tests."""
    name = CONFIGS.get(which, which)
    if name == "furnace":
        return furnace(seed=1 if seed is None else seed, **({} if n is None else {"n": n}), **kw)
    if name == "box_room":
        return box_room(seed=2 if seed is None else seed, **({} if n is None else {"n": n}), **kw)
    if name == "fruit_bowl":
        return fruit_bowl(seed=3 if seed is None else seed, **({} if n is None else {"n": n}), **kw)
    if name == "multi_light":
        kw.setdefault("n_lights", 100)
        return box_room(seed=4 if seed is None else seed, n=32768 if n is None else n, **kw)
    raise KeyError(f"unknown config {which!r}")


def random_frame_surfels(n: int, seed: int, extent: float = 1.0, scale=(0.05, 0.15),
                         opacity=(0.5, 0.99)) -> Dict[str, np.ndarray]:
    """Tiny random scenes for brute-force tests: random centres in a cube,
    random orientations, random scales and opacities."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(-extent, extent, size=(n, 3))
    g = rng.standard_normal((n, 3))
    nrm = g / np.linalg.norm(g, axis=1, keepdims=True)
    tu, tv = onb_from_normal(nrm)
    tu, tv = _spin(tu, tv, rng)
    su = rng.uniform(*scale, size=n)
    sv = rng.uniform(*scale, size=n)
    op = rng.uniform(*opacity, size=n)
    sur, _ = _pack(p, nrm, tu, tv, su, sv, op, np.zeros((n, 3)))
    return sur


def layer_stack(n_layers: int = 160, per_layer: int = 3, spacing: float = 0.01, scale: float = 0.2,
                opacity: float = 0.02, seed: int = 0) -> Dict[str, np.ndarray]:
    """Receivers on the plane z = 0 below a stack of nearly transparent,
    slightly jittered horizontal layers: upward rays composite well over a
    hundred hits each (transmittance never reaches the cut-off)."""
    rng = np.random.default_rng(seed)
    m = n_layers * per_layer
    p = np.zeros((m + 4, 3))
    p[:4, :2] = rng.uniform(-0.05, 0.05, (4, 2))
    k = np.arange(m)
    p[4:, 0] = rng.uniform(-0.05, 0.05, m)
    p[4:, 1] = rng.uniform(-0.05, 0.05, m)
    p[4:, 2] = spacing * (1 + k // per_layer) + rng.uniform(0, 0.2 * spacing, m)
    nrm = np.tile([0.0, 0.0, 1.0], (m + 4, 1))
    nrm[4:] = -nrm[4:]
    nrm[4:, :2] += rng.uniform(-0.05, 0.05, (m, 2))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    tu, tv = onb_from_normal(nrm)
    su = np.full(m + 4, scale)
    op = np.full(m + 4, opacity)
    op[:4] = 0.9
    sur, _ = _pack(p, nrm, tu, tv, su, su, op, np.zeros((m + 4, 3)))
    return sur


def deep_chain(copies: int = 16, scale: float = 3.0, opacity: float = 0.3, seed: int = 0) -> Dict[str, np.ndarray]:
    """Centres whose 30-bit Morton codes are 0, every single bit and all
    ones: with the scene box [0, 4]^3 the quantised coordinates of the axis
    points are powers of two, so an LBVH over the sorted codes peels one code
    per level (a chain of 31 internal nodes) and the `copies` surfels sharing
    each centre add a balanced subtree below.  Surfels far larger than the
    scene make every box cover every ray origin, so a depth-first traversal
    keeps a far child pending at every level of the chain."""
    rng = np.random.default_rng(seed)
    cen = [np.zeros(3), np.full(3, 4.0)]
    for k in range(10):
        for a in range(3):
            c = np.zeros(3)
            c[a] = (2.0 ** k + 0.25) / 256.0
            cen.append(c)
    p = np.repeat(np.asarray(cen), copies, axis=0)
    m = p.shape[0]
    g = rng.standard_normal((m, 3))
    nrm = g / np.linalg.norm(g, axis=1, keepdims=True)
    tu, tv = onb_from_normal(nrm)
    tu, tv = _spin(tu, tv, rng)
    su = np.full(m, scale)
    op = np.full(m, opacity)
    sur, _ = _pack(p, nrm, tu, tv, su, su, op, np.zeros((m, 3)))
    return sur


def surfels_from_arrays(p, nrm, tu, tv, su, sv, op) -> Dict[str, np.ndarray]:
    """Pack explicit geometry (used by analytic two-surfel set-ups)."""
    sur, _ = _pack(np.asarray(p, float), np.asarray(nrm, float), np.asarray(tu, float),
                   np.asarray(tv, float), np.asarray(su, float), np.asarray(sv, float),
                   np.asarray(op, float), np.zeros((len(su), 3)))
    return sur


def seeded_array(shape, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Uniform FP32 array for operator-level tests (E, rho, grad_B, F values)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(lo, hi, size=shape).astype(np.float32))


def seeded_csr(n: int, nnz_per_row: int, seed: int, row_sum: float = 0.6, n_cols: Optional[int] = None):
    """A synthetic sparse transport matrix (CSR: int64 row_ptr, int32 columns
    strictly ascending per row, FP32 values) whose rows sum to about
    ``row_sum`` and whose columns cluster near the row index, the shape of
    ray-cast rows.  Row lengths vary in [k/2, k]; the first rows are empty."""
    rng = np.random.default_rng(seed)
    n_cols = n if n_cols is None else n_cols
    k = int(max(0, min(nnz_per_row, n_cols - 1)))
    if n == 0:
        return np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32)
    lens = rng.integers(k // 2, k + 1, size=n) if k > 0 else np.zeros(n, np.int64)
    lens[: min(2, n)] = 0
    gaps = rng.integers(1, 4, size=(n, max(k, 1)))
    offs = np.cumsum(gaps, axis=1)                       # strictly increasing, >= 1
    start = np.arange(n)[:, None] - offs[:, -1:] // 2     # centred on the row
    cols = start + offs
    cols = np.clip(cols, 0, n_cols - 1)
    keep = np.arange(max(k, 1))[None, :] < lens[:, None]
    keep &= cols != np.arange(n)[:, None]
    keep[:, 1:] &= cols[:, 1:] != cols[:, :-1]          # clipping can repeat
    lens = keep.sum(axis=1)
    row_ptr = np.zeros(n + 1, np.int64)
    row_ptr[1:] = np.cumsum(lens)
    c = cols[keep].astype(np.int32)
    v = rng.uniform(0.0, 1.0, size=c.size)
    rs = np.add.reduceat(v, row_ptr[:-1][lens > 0]) if c.size else np.zeros(0)
    scale = np.zeros(n)
    scale[lens > 0] = row_sum / np.maximum(rs, 1e-30)
    v = v * np.repeat(scale, lens)
    return row_ptr, np.ascontiguousarray(c), np.ascontiguousarray(v.astype(np.float32))


def phong_materials(n: int, seed: int, shininess=(1.0, 20.0)) -> Dict[str, np.ndarray]:
    """Seeded diffuse + Phong materials per surfel (Eq. brdf parameters):
    blend k ~ U[0, 1], diffuse and specular albedo ~ U[0.1, 0.9]^3 and
    shininess ~ U[shininess], FP32."""
    rng = np.random.default_rng(seed)
    f32 = lambda a: np.ascontiguousarray(a.astype(np.float32))  # noqa: E731
    return {"k": f32(rng.uniform(0.0, 1.0, n)), "albedo_d": f32(rng.uniform(0.1, 0.9, (n, 3))),
            "albedo_s": f32(rng.uniform(0.1, 0.9, (n, 3))), "shininess": f32(rng.uniform(*shininess, n))}
