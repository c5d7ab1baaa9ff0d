"""FP64 oracle of the directional transfer: per-surfel spherical-harmonic
radiance moved between surfels through the diffuse + Phong BRDF.

TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module.  It shares no code with
the GPU path and never imports it.

Paper passages followed:
* Sec. 3.2: real SH basis Y(w) = [Y00, Y1-1, Y10, Y11, ...], Ybar(w) = Y(-w);
  a BRDF that is a lobe about one axis expands as
  f(w_I, w_O) = sum_lm c_lm Ybar_lm(w_I) Y_lm(w_O), i.e.
  f(w_I) = f^c x Ybar(w_I) (element-wise), with c_lm = (-1)^m c_l0.
* Sec. 5.1, Eq. brdf: f = k a^d / pi + (1 - k) a^s (s + 1) / (2 pi) |w_r . w_I|^s,
  and App. A for its coefficient vector f^c (the Phong lobe clamped to the
  visible hemisphere).
* Eq. final-radiosity (Sec. 5.3): B_i = E_i + sum_j int int f_i(w_I)
  (Y(w_I)^T B_j) V_ji, with the receiver opacity absorbed into f_i; direct
  light (Sec. 5.2) from point lights of isotropic intensity.
* Eq. final_dL_dE, final-dl-dbrdf, dl-dgeo-0 (Sec. 6): the adjoint, here the
  exact adjoint of the truncated n-bounce map.

Readings (where the paper leaves a choice):
* Frames.  The coefficient vectors of surfel i (E_i, B_i, f^c_i) are taken in
  the surfel's own tangent frame, (t_u, t_v, n) as (x, y, z).  App. A's
  c_lm = (-1)^m c_l0 is the Phong lobe about the mirror direction only in a
  frame whose z axis is the normal: the reflection about the normal is the
  rotation by pi about z, which multiplies Y_lm by (-1)^m.
* Directions.  Per pair (i, j) the directional factors use the direction
  between the centres, d_ij = (p_j - p_i)/|p_j - p_i| (from the receiver to the
  sender): Sec. 8 takes the BRDF and radiance factors as constant over a
  pair.  The decay of the pair is the ray-cast form factor F_ij (or any
  other operator F given).  With w_I = -d_ij (the direction light travels),
  Ybar(w_I) = Y(d_ij) in i's frame and Y(w_I) = Y(-d_ij) in j's frame.
  Coincident centres (no direction) take the receiver's normal as d_ij.
* Normalisation.  With cosine-weighted rays the hemisphere integral of
  g(w)|n.w| is pi times the mean over rays, so the transfer is
  (T X)_i = sum_j F_ij Y(d_ij^(i)) (Y(-d_ij^(j))^T X_j) and the receiver
  factor is R_i = pi o_i f^c_i (per colour): B = E + R (.) (T B).  For a
  Lambertian surfel (k = 1, f^c = (4 a, 0, ...)) and radiance with only a DC
  coefficient this is exactly the scalar B = E + o a F B.
* Point lights (isotropic intensity I at x_l, Eq. direct illumination):
  E_i = (R_i / pi) (.) Y(d_il^(i)) I max(0, n_i . d_il) / r^2 T_il with d_il
  the unit direction to the light and T_il the shadow transmittance.

Layouts: R and f^c are [N, K, 3]; E, B and their gradients [N, Lt, K, 3].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.special

from .oracle import clamp_opacity


# ---------------------------------------------------------------------------
# real spherical harmonics (Sec. 3.2)
# ---------------------------------------------------------------------------
def sh_degree(K: int) -> int:
    L = int(round(np.sqrt(K))) - 1
    if (L + 1) ** 2 != K or L < 0:
        raise ValueError("K must be a square (1, 4, 9, 16, ...)")
    return L


def sh_basis(dirs, K: int) -> np.ndarray:
    """Real SH [..., K] of unit vectors dirs [..., 3], order Y00, Y1-1, Y10,
    Y11, Y2-2, ...: from scipy's complex Y_l^m (Condon-Shortley phase) as
    Y_lm = sqrt(2) (-1)^m Re Y_l^m (m > 0), sqrt(2) (-1)^m Im Y_l^|m| (m < 0)."""
    d = np.asarray(dirs, np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    theta = np.arccos(np.clip(z / np.sqrt(x * x + y * y + z * z), -1.0, 1.0))
    phi = np.arctan2(y, x)
    L = sh_degree(K)
    out = np.zeros(d.shape[:-1] + (K,))
    for l in range(L + 1):
        for m in range(-l, l + 1):
            c = scipy.special.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                v = np.sqrt(2.0) * (-1.0) ** m * c.real
            elif m < 0:
                v = np.sqrt(2.0) * (-1.0) ** m * c.imag
            else:
                v = c.real
            out[..., l * l + l + m] = v
    return out


def sh_l_of(K: int) -> np.ndarray:
    return np.concatenate([[l] * (2 * l + 1) for l in range(sh_degree(K) + 1)]).astype(np.int64)


def sh_m_of(K: int) -> np.ndarray:
    return np.concatenate([np.arange(-l, l + 1) for l in range(sh_degree(K) + 1)]).astype(np.int64)


# ---------------------------------------------------------------------------
# BRDF coefficients (Eq. brdf, App. A)
# ---------------------------------------------------------------------------
def _lobe_factors(l: int):
    """Numerator offsets t (factors s + t) and denominator offsets (factors
    s + u) of App. A's ratio for degree l >= 1."""
    if l % 2 == 1:
        num = [1 - 2 * q for q in range((l + 1) // 2)]          # s+1, s-1, ..., s-l+2
        den = [2 + 2 * q for q in range((l + 1) // 2)]          # s+2, s+4, ..., s+l+1
    else:
        num = [-2 * q for q in range(l // 2)]                   # s, s-2, ..., s-l+2
        den = [3 + 2 * q for q in range(l // 2)]                # s+3, s+5, ..., s+l+1
    return num, den


def phong_lobe(s, l: int):
    """g_l(s), the ratio of App. A for degree l (g_0 = 1): the coefficient of
    the clamped normalised lobe (s+1)/(2 pi) max(0, cos)^s on
    sqrt(4 pi/(2l+1)) Y_l0 about its axis."""
    s = np.asarray(s, np.float64)
    if l == 0:
        return np.ones_like(s)
    num, den = _lobe_factors(l)
    out = np.ones_like(s)
    for t in num:
        out = out * (s + t)
    for u in den:
        out = out / (s + u)
    return out


def phong_lobe_ds(s, l: int):
    """d g_l / d s by the product rule."""
    s = np.asarray(s, np.float64)
    if l == 0:
        return np.zeros_like(s)
    num, den = _lobe_factors(l)
    N = np.ones_like(s)
    dN = np.zeros_like(s)
    for t in num:
        dN = dN * (s + t) + N
        N = N * (s + t)
    D = np.ones_like(s)
    dD = np.zeros_like(s)
    for u in den:
        dD = dD * (s + u) + D
        D = D * (s + u)
    return (dN * D - N * dD) / (D * D)


def brdf_coefficients(k, ad, as_, shin, K: int) -> np.ndarray:
    """f^c [N, K, 3] (App. A): c_00 = 4 k a^d + (1 - k) a^s,
    c_lm = (-1)^m (1 - k) g_l(s) a^s for l >= 1."""
    k = np.asarray(k, np.float64)[:, None]
    ad = np.asarray(ad, np.float64)
    as_ = np.asarray(as_, np.float64)
    shin = np.asarray(shin, np.float64)
    N = ad.shape[0]
    fc = np.zeros((N, K, 3))
    ls, ms = sh_l_of(K), sh_m_of(K)
    for a in range(K):
        if a == 0:
            fc[:, 0, :] = 4.0 * k * ad + (1.0 - k) * as_
        else:
            fc[:, a, :] = (-1.0) ** ms[a] * (1.0 - k) * phong_lobe(shin, ls[a])[:, None] * as_
    return fc


def reflectance_sh(opacity, k, ad, as_, shin, K: int) -> np.ndarray:
    """R = pi o f^c [N, K, 3]: the receiver factor of the transfer (receiver
    opacity absorbed into the BRDF, Sec. 5.3; pi from the cosine-weighted
    hemisphere estimator)."""
    o = clamp_opacity(opacity).astype(np.float64)
    return np.pi * o[:, None, None] * brdf_coefficients(k, ad, as_, shin, K)


def brdf_backward(opacity, k, ad, as_, shin, K: int, grad_R):
    """Gradients of sum(grad_R * R) with respect to o (zero where the clamp
    is active), k, a^d, a^s and s."""
    o_raw = np.asarray(opacity, np.float32)
    o = clamp_opacity(o_raw).astype(np.float64)
    inside = (o_raw > 0) & (o_raw < np.float32(0.9999))
    G = np.asarray(grad_R, np.float64)
    fc = brdf_coefficients(k, ad, as_, shin, K)
    g_o = np.where(inside, np.pi * np.sum(G * fc, axis=(1, 2)), 0.0)
    Gp = np.pi * o[:, None, None] * G          # gradient on f^c
    k = np.asarray(k, np.float64)
    ad = np.asarray(ad, np.float64)
    as_ = np.asarray(as_, np.float64)
    shin = np.asarray(shin, np.float64)
    ls, ms = sh_l_of(K), sh_m_of(K)
    g_k = np.sum(Gp[:, 0, :] * (4.0 * ad - as_), axis=1)
    g_ad = Gp[:, 0, :] * 4.0 * k[:, None]
    g_as = Gp[:, 0, :] * (1.0 - k[:, None])
    g_s = np.zeros_like(shin)
    for a in range(1, K):
        sgn = (-1.0) ** ms[a]
        gl = phong_lobe(shin, ls[a])
        g_k -= np.sum(Gp[:, a, :] * sgn * gl[:, None] * as_, axis=1)
        g_as += Gp[:, a, :] * sgn * (1.0 - k[:, None]) * gl[:, None]
        g_s += np.sum(Gp[:, a, :] * sgn * as_, axis=1) * (1.0 - k) * phong_lobe_ds(shin, ls[a])
    return g_o, g_k, g_ad, g_as, g_s


# ---------------------------------------------------------------------------
# per-pair bases and the transfer (Eq. final-radiosity, directional)
# ---------------------------------------------------------------------------
def frames(surfels):
    """Centres [N, 3] and tangent frames [N, 3, 3] (rows t_u, t_v, n), FP64
    of the FP32 inputs."""
    P = np.stack([surfels["px"], surfels["py"], surfels["pz"]], 1).astype(np.float64)
    Fr = np.stack([np.stack([surfels["tux"], surfels["tuy"], surfels["tuz"]], 1),
                   np.stack([surfels["tvx"], surfels["tvy"], surfels["tvz"]], 1),
                   np.stack([surfels["nx"], surfels["ny"], surfels["nz"]], 1)], 1).astype(np.float64)
    return P, Fr


def pair_bases(F, surfels, K: int):
    """For every stored entry e = (i, j) of F (CSR order): Yd[e] = Y of the
    unit direction from p_i to p_j in i's frame, Ye[e] = Y of the opposite
    direction in j's frame."""
    F = sp.csr_matrix(F)
    P, Fr = frames(surfels)
    rows = np.repeat(np.arange(F.shape[0]), np.diff(F.indptr))
    cols = F.indices
    d = P[cols] - P[rows]
    ln = np.linalg.norm(d, axis=1)
    d = np.where(ln[:, None] > 0, d / np.where(ln > 0, ln, 1.0)[:, None], Fr[rows, 2])   # coincident: normal of i
    di = np.einsum("eab,eb->ea", Fr[rows], d)
    ej = np.einsum("eab,eb->ea", Fr[cols], -d)
    return rows, cols, sh_basis(di, K), sh_basis(ej, K)


def _as_rows(X, K):
    X = np.asarray(X, np.float64)
    return X.reshape(X.shape[0], -1, K, 3)


def _sum_by(index, n, contrib):
    """out[r] = sum of contrib[e] over the entries e with index[e] = r."""
    S = sp.csr_matrix((np.ones(index.size), (index, np.arange(index.size))), shape=(n, index.size))
    width = int(np.prod(contrib.shape[1:]))
    return (S @ contrib.reshape(index.size, width)).reshape((n,) + contrib.shape[1:])


def transfer(F, bases, X, K: int) -> np.ndarray:
    """(T X)_i[l, a, c] = sum_j F_ij Yd_ij[a] sum_b Ye_ij[b] X_j[l, b, c]."""
    F = sp.csr_matrix(F)
    rows, cols, Yd, Ye = bases
    X4 = _as_rows(X, K)
    s = np.einsum("eb,elbc->elc", Ye, X4[cols])                  # radiance of j towards i
    contrib = F.data[:, None, None, None] * Yd[:, None, :, None] * s[:, :, None, :]
    return _sum_by(rows, F.shape[0], contrib).reshape(np.shape(X))


def transfer_T(F, bases, U, K: int) -> np.ndarray:
    """The adjoint of ``transfer``:
    (T^T U)_j[l, b, c] = sum_i F_ij Ye_ij[b] sum_a Yd_ij[a] U_i[l, a, c]."""
    F = sp.csr_matrix(F)
    rows, cols, Yd, Ye = bases
    U4 = _as_rows(U, K)
    s = np.einsum("ea,elac->elc", Yd, U4[rows])
    contrib = F.data[:, None, None, None] * Ye[:, None, :, None] * s[:, :, None, :]
    return _sum_by(cols, F.shape[1], contrib).reshape(np.shape(U))


def _times_R(R, X, K):
    X4 = _as_rows(X, K)
    return (np.asarray(R, np.float64)[:, None, :, :] * X4).reshape(np.shape(X))


def bounce(F, surfels, R, E, n_bounces: int, keep_tape: bool = False):
    """B^(0) = E, B^(k+1) = E + R (.) (T B^(k)); returns B^(n) and, if asked,
    the tape ([B^(k)], [Q^(k) = T B^(k)])."""
    K = np.asarray(R).shape[1]
    bases = pair_bases(F, surfels, K)
    E = np.asarray(E, np.float64)
    B = E.copy()
    tB, tQ = [], []
    for _ in range(n_bounces):
        Q = transfer(F, bases, B, K)
        if keep_tape:
            tB.append(B)
            tQ.append(Q)
        B = E + _times_R(R, Q, K)
    return (B, (tB, tQ)) if keep_tape else B


def adjoint(F, surfels, R, tape, g):
    """Exact adjoint of ``bounce`` for dL/dB^(n) = g:
      lambda^(n) = g,  lambda^(k) = T^T (R (.) lambda^(k+1))
      grad_E = sum_k lambda^(k)
      grad_R[i, a, c] = sum_{k<n} sum_l lambda^(k+1)_i[l, a, c] Q^(k)_i[l, a, c]
      grad_F[e] = sum_{k<n} sum_{l, c} (Yd_e . (R (.) lambda^(k+1))_i[l, :, c])
                                       (Ye_e . B^(k)_j[l, :, c])
    (Eq. final_dL_dE in division-free form, Eq. final-dl-dbrdf and the decay
    term of Eq. dl-dgeo-0 before their fixed-point limits)."""
    K = np.asarray(R).shape[1]
    F = sp.csr_matrix(F)
    bases = pair_bases(F, surfels, K)
    rows, cols, Yd, Ye = bases
    tB, tQ = tape
    lam = np.asarray(g, np.float64).copy()
    grad_E = lam.copy()
    grad_R = np.zeros(np.shape(R))
    grad_F = np.zeros(F.nnz)
    for k in range(len(tB) - 1, -1, -1):
        grad_R += np.sum(_as_rows(lam, K) * _as_rows(tQ[k], K), axis=1)
        u = _times_R(R, lam, K)
        U4 = _as_rows(u, K)
        B4 = _as_rows(tB[k], K)
        grad_F += np.einsum("elc,elc->e", np.einsum("ea,elac->elc", Yd, U4[rows]),
                            np.einsum("eb,elbc->elc", Ye, B4[cols]))
        lam = transfer_T(F, bases, u, K)
        grad_E += lam
    return grad_E, grad_R, grad_F


def direct_light(surfels, R, light_pos, light_I, T):
    """E [N, Lt, K, 3] from point lights: E_i = (R_i/pi) (.) Y(d_il^(i))
    I_l max(0, n_i . d_il) / r_il^2 T_il, with T [N, Lt] the shadow
    transmittances (oracle.direct_light(..., return_T=True))."""
    R = np.asarray(R, np.float64)
    K = R.shape[1]
    P, Fr = frames(surfels)
    lp = np.asarray(light_pos, np.float64).reshape(-1, 3)
    lI = np.asarray(light_I, np.float64).reshape(-1)
    N, Lt = P.shape[0], lp.shape[0]
    E = np.zeros((N, Lt, K, 3))
    for l in range(Lt):
        v = lp[l][None, :] - P
        r2 = np.sum(v * v, axis=1)
        d = v / np.sqrt(r2)[:, None]
        loc = np.einsum("nab,nb->na", Fr, d)
        cosv = loc[:, 2]
        w = np.where(cosv > 0, lI[l] * cosv / r2 * np.asarray(T, np.float64)[:, l], 0.0)
        E[:, l] = (R / np.pi) * sh_basis(loc, K)[:, :, None] * w[:, None, None]
    return E


def dense_operator(F, surfels, R, K: int) -> np.ndarray:
    """The whole map X -> R (.) (T X) for one light as an explicit
    (N K 3) x (N K 3) matrix, assembled entry by entry from the definition
    (small N only; used to check transfer and transfer_T)."""
    F = sp.csr_matrix(F)
    rows, cols, Yd, Ye = pair_bases(F, surfels, K)
    N = F.shape[0]
    M = np.zeros((N * K * 3, N * K * 3))
    R = np.asarray(R, np.float64)
    for e in range(F.nnz):
        i, j = rows[e], cols[e]
        for a in range(K):
            for b in range(K):
                for c in range(3):
                    M[(i * K + a) * 3 + c, (j * K + b) * 3 + c] += R[i, a, c] * F.data[e] * Yd[e, a] * Ye[e, b]
    return M
