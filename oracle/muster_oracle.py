"""FP64 CPU oracle for the MUSTER per-iteration optimisation path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: it exists so that tests, the smoke check and the CPU
baseline of the benchmark can compare the HIP implementation against a plain,
slow, obviously correct statement of what the method computes.  It shares no
code with the HIP path and imports nothing from it.

Every function follows a passage of the MUSTER paper (Multi-Session Temporal
Registration, arXiv 2412.14671).  Section numbers below are the paper's:
Sec. 2.1 (deformation conventions), Sec. 2.2 (loss, Eq. cum_deformation),
Sec. 2.3 (scaling and squaring, Alg. 1), Sec. 2.4 (regularisers, Eq. reg_ss,
reg_sum), Sec. 2.6 (LNCC Eq. LNCC / sum_lncc; SiLNCC Eq. sim_loss),
Sec. 2.7 (Adam, warm-up + cosine schedule, three-stage pyramid),
Sec. 2.8 (Euclidean-distance metric).

Conventions (readings where the paper is silent; each is listed in the design
notes of the repository):
  * A volume is a C-order array (D, H, W); a vector field is (3, D, H, W) with
    components (z, y, x).  Grid point p has coordinate p (voxel indices), and
    fields hold displacements u = Phi - Omega in voxels of their own grid.
  * Trilinear sampling clamps the sample position to the grid (border
    padding), uses the cell whose lower corner is floor(q) (the last cell at the
    upper border) and has zero derivative along an axis whose coordinate was
    outside the grid.
  * Exp takes exactly K squarings of u_0 = phi / 2^K, in the displacement form
    of Alg. 1.
  * Pair fields are built by composing outward from the target session.
  * Window statistics use the maximum-likelihood (1/n) moments over w^3
    windows whose centres lie at least r = (w-1)/2 from every border.
  * All arithmetic is float64; inputs are float32 arrays promoted on entry.

Parity status: every function here is pinned by tests against closed forms,
exact identities, brute force, finite differences or library routines.  The
end-to-end optimisation (register) is pinned by the same loop driven by
torch's Adam over the pinned loss and gradient, stage by stage.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

EPS_LNCC = 1e-10   # guard on vF*vM in LNCC (silent in the paper; never active on test data)
EPS_SILNCC = 1e-6  # guard on vF in SiLNCC (silent in the paper; never active on test data)

LNCC = 0
SILNCC = 1


# ---------------------------------------------------------------------------
# Grid and trilinear sampling (Sec. 2.2)
# ---------------------------------------------------------------------------

def identity_grid(shape) -> np.ndarray:
    """Omega_I: the coordinates of every grid point, shape (3, D, H, W)."""
    return np.stack(np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape],
                                indexing="ij"))


def _axis(q: np.ndarray, n: int):
    """Cell index, fraction and derivative mask along one axis for positions q."""
    live = (q >= 0.0) & (q <= n - 1.0)
    qc = np.clip(q, 0.0, n - 1.0)
    i0 = np.minimum(np.floor(qc), n - 2).astype(np.int64)
    t = qc - i0
    return i0, t, live


def sample(f: np.ndarray, q: np.ndarray, jac: bool = False):
    """Trilinear sample of the field f (C, D, H, W) at positions q (3, ...).

    Returns the sampled values (C, ...) and, when jac is set, the derivative of
    each sampled component with respect to each coordinate of q, (C, 3, ...),
    ordered (z, y, x).
    """
    D, H, W = f.shape[1:]
    z0, tz, lz = _axis(q[0], D)
    y0, ty, ly = _axis(q[1], H)
    x0, tx, lx = _axis(q[2], W)
    flat = f.reshape(f.shape[0], -1)
    base = (z0 * H + y0) * W + x0
    v = {}
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                v[a, b, c] = np.take(flat, base + (a * H + b) * W + c, axis=1)
    c00 = v[0, 0, 0] + tx * (v[0, 0, 1] - v[0, 0, 0])
    c01 = v[0, 1, 0] + tx * (v[0, 1, 1] - v[0, 1, 0])
    c10 = v[1, 0, 0] + tx * (v[1, 0, 1] - v[1, 0, 0])
    c11 = v[1, 1, 0] + tx * (v[1, 1, 1] - v[1, 1, 0])
    c0 = c00 + ty * (c01 - c00)
    c1 = c10 + ty * (c11 - c10)
    val = c0 + tz * (c1 - c0)
    if not jac:
        return val
    dz = (c1 - c0) * lz
    dy0 = c01 - c00
    dy1 = c11 - c10
    dy = (dy0 + tz * (dy1 - dy0)) * ly
    e00 = v[0, 0, 1] - v[0, 0, 0]
    e01 = v[0, 1, 1] - v[0, 1, 0]
    e10 = v[1, 0, 1] - v[1, 0, 0]
    e11 = v[1, 1, 1] - v[1, 1, 0]
    e0 = e00 + ty * (e01 - e00)
    e1 = e10 + ty * (e11 - e10)
    dx = (e0 + tz * (e1 - e0)) * lx
    return val, np.stack([dz, dy, dx], axis=1)


def sample_adjoint(g: np.ndarray, q: np.ndarray, shape) -> np.ndarray:
    """Adjoint of sample() with respect to the sampled field's values.

    Each position q(p) hands g(p) to the 8 corners of its cell with the
    trilinear weights; the result is a field of the given grid shape.
    """
    D, H, W = shape
    C = g.shape[0]
    z0, tz, _ = _axis(q[0], D)
    y0, ty, _ = _axis(q[1], H)
    x0, tx, _ = _axis(q[2], W)
    out = np.zeros((C, D * H * W), dtype=np.float64)
    for a in (0, 1):
        wz = tz if a else 1.0 - tz
        for b in (0, 1):
            wy = ty if b else 1.0 - ty
            for c in (0, 1):
                wx = tx if c else 1.0 - tx
                w = (wz * wy * wx).ravel()
                flat = (((z0 + a) * H + (y0 + b)) * W + (x0 + c)).ravel()
                for k in range(C):
                    out[k] += np.bincount(flat, weights=w * g[k].ravel(), minlength=D * H * W)
    return out.reshape(C, D, H, W)


def jac_transpose_apply(J: np.ndarray, g: np.ndarray) -> np.ndarray:
    """(J^T g)_b = sum_a J[a, b] g[a] for J of shape (3, 3, ...)."""
    return np.einsum("ab...,a...->b...", J, g)


# ---------------------------------------------------------------------------
# Exp by scaling and squaring (Sec. 2.3, Alg. 1) and its adjoint
# ---------------------------------------------------------------------------

def exp_fwd(phi: np.ndarray, K: int) -> List[np.ndarray]:
    """Displacements u_0..u_K of Exp(phi): u_0 = phi/2^K, then K squarings
    u_{s+1} = u_s + u_s o (Omega + u_s) (the displacement form of Alg. 1)."""
    phi = np.asarray(phi, dtype=np.float64)
    g = identity_grid(phi.shape[1:])
    us = [phi * (2.0 ** -K)]
    for _ in range(K):
        u = us[-1]
        us.append(u + sample(u, g + u))
    return us


def exp_step_bwd(u: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Adjoint of one squaring u' = u + S(u, Omega + u): returns dL/du given
    G = dL/du'.  Three terms: identity, the Jacobian of the sampled field at the
    sample position, and the scatter of G to the corners that were sampled."""
    g = identity_grid(u.shape[1:])
    q = g + u
    _, J = sample(u, q, jac=True)
    return G + jac_transpose_apply(J, G) + sample_adjoint(G, q, u.shape[1:])


def exp_bwd(us: List[np.ndarray], G_K: np.ndarray) -> np.ndarray:
    """Given dL/du_K, return dL/du_0 by running the squarings backwards."""
    G = np.asarray(G_K, dtype=np.float64)
    for s in range(len(us) - 2, -1, -1):
        G = exp_step_bwd(us[s], G)
    return G


# ---------------------------------------------------------------------------
# Consecutive and pairwise deformations (Sec. 2.2 Eq. cum_deformation, Sec. 2.3)
# ---------------------------------------------------------------------------

def pair_index(i: int, j: int, N: int) -> int:
    """Slot of pair (target i, source j), i != j, in an N(N-1) array."""
    return i * (N - 1) + (j if j < i else j - 1)


def compose(U_prev: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Eq. cum_deformation in displacement form: U_prev + C o (Omega + U_prev)."""
    g = identity_grid(U_prev.shape[1:])
    return U_prev + sample(C, g + U_prev)


def compose_bwd(U_prev: np.ndarray, C: np.ndarray, G: np.ndarray):
    """Adjoint of compose(): (dL/dU_prev, dL/dC) given G = dL/dU_new."""
    g = identity_grid(U_prev.shape[1:])
    q = g + U_prev
    _, J = sample(C, q, jac=True)
    return G + jac_transpose_apply(J, G), sample_adjoint(G, q, C.shape[1:])


def chain_parent(i: int, j: int):
    """For a pair (i, j) with |i-j| >= 2: the previous pair of its chain and
    which consecutive field is sampled, as ((i, j_prev), kind, index) with kind
    'f' (forward Exp(phi_index)) or 'b' (backward Exp(-phi_index))."""
    if j > i + 1:
        return (i, j - 1), "f", j - 1
    if j < i - 1:
        return (i, j + 1), "b", j
    raise ValueError("consecutive pair has no parent")


def all_pairs(f: List[np.ndarray], b: List[np.ndarray]) -> Dict[Tuple[int, int], np.ndarray]:
    """Every U[j->i] = Phi_ji^i - Omega for i != j.

    f[i] = Exp(phi_i) lives on grid i and pulls session i+1 to session i;
    b[i] = Exp(-phi_i) lives on grid i+1 and pulls session i to session i+1.
    Longer pairs are composed outward from the target: U[j->i] samples f[j-1]
    (j > i+1) or b[j] (j < i-1) at Omega + U[j-1->i] (resp. U[j+1->i]).
    """
    N = len(f) + 1
    U: Dict[Tuple[int, int], np.ndarray] = {}
    for i in range(N):
        if i + 1 < N:
            U[(i, i + 1)] = f[i]
        if i - 1 >= 0:
            U[(i, i - 1)] = b[i - 1]
    for d in range(2, N):
        for i in range(N):
            for j in (i + d, i - d):
                if 0 <= j < N:
                    prev, kind, k = chain_parent(i, j)
                    U[(i, j)] = compose(U[prev], f[k] if kind == "f" else b[k])
    return U


# ---------------------------------------------------------------------------
# Warp and windowed similarity (Sec. 2.1, Sec. 2.6)
# ---------------------------------------------------------------------------

def warp(I: np.ndarray, U: np.ndarray) -> np.ndarray:
    """I o (Omega + U): the image I resampled on the deformed grid."""
    g = identity_grid(I.shape)
    return sample(np.asarray(I, np.float64)[None], g + U)[0]


def warp_grad(I: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Derivative of warp(I, U)(p) with respect to U(p), shape (3, D, H, W)."""
    g = identity_grid(I.shape)
    _, J = sample(np.asarray(I, np.float64)[None], g + U, jac=True)
    return J[0]


def box_sum(X: np.ndarray, r: int) -> np.ndarray:
    """Sum of X over the w^3 window (w = 2r+1) around every valid centre.

    Valid centres are r <= c_d <= n_d-1-r, so the result has shape n_d - 2r.
    The sum runs over every offset of the window, as in the definition."""
    D, H, W = X.shape
    out = np.zeros((D - 2 * r, H - 2 * r, W - 2 * r), dtype=np.float64)
    w = 2 * r + 1
    for a in range(w):
        for b in range(w):
            for c in range(w):
                out += X[a:a + D - 2 * r, b:b + H - 2 * r, c:c + W - 2 * r]
    return out


def box_adjoint(A: np.ndarray, r: int, shape) -> np.ndarray:
    """Adjoint of box_sum: every voxel y receives the sum of A over the valid
    centres whose window contains y."""
    D, H, W = shape
    out = np.zeros(shape, dtype=np.float64)
    w = 2 * r + 1
    for a in range(w):
        for b in range(w):
            for c in range(w):
                out[a:a + D - 2 * r, b:b + H - 2 * r, c:c + W - 2 * r] += A
    return out


def window_moments(F: np.ndarray, M: np.ndarray, w: int):
    """Means, ML variances and covariance of (F, M) over every valid window."""
    r = (w - 1) // 2
    n = float(w ** 3)
    F = np.asarray(F, np.float64)
    M = np.asarray(M, np.float64)
    SF, SM = box_sum(F, r), box_sum(M, r)
    SFF, SMM, SFM = box_sum(F * F, r), box_sum(M * M, r), box_sum(F * M, r)
    mF, mM = SF / n, SM / n
    vF_raw = SFF / n - mF * mF
    vM_raw = SMM / n - mM * mM
    c = SFM / n - mF * mM
    return dict(n=n, r=r, mF=mF, mM=mM, vF_raw=vF_raw, vM_raw=vM_raw,
                vF=np.maximum(vF_raw, 0.0), vM=np.maximum(vM_raw, 0.0), c=c)


def window_loss(mo, metric: int):
    """Per-window loss l_R and its derivatives a_v = dl/dvM, a_c = dl/dc.

    LNCC (Eq. LNCC): l = 1 - c / sqrt(vF vM), guarded by EPS_LNCC.
    SiLNCC (Eq. sim_loss): l = vM - c^2 / vF, i.e. the residual variance of the
    least-squares fit of the warped image on the fixed image, guarded by
    EPS_SILNCC.  The fixed image (first argument of Sim) is the regressor.
    """
    vF, vM, c = mo["vF"], mo["vM"], mo["c"]
    vm_live = mo["vM_raw"] > 0.0
    if metric == LNCC:
        den = vF * vM
        active = den > EPS_LNCC
        sd = np.sqrt(np.where(active, den, EPS_LNCC))
        l = 1.0 - c / sd
        a_c = -1.0 / sd
        a_v = np.where(active, c / (2.0 * np.where(vM > 0, vM, 1.0) * sd), 0.0)
    elif metric == SILNCC:
        d = np.maximum(vF, EPS_SILNCC)
        l = vM - c * c / d
        a_c = -2.0 * c / d
        a_v = np.ones_like(l)
    else:
        raise ValueError("unknown metric")
    a_v = np.where(vm_live, a_v, 0.0)
    return l, a_v, a_c


def similarity(F: np.ndarray, M: np.ndarray, w: int, metric: int) -> float:
    """Eq. sum_lncc / sim_loss: the mean of the per-window loss over windows."""
    mo = window_moments(F, M, w)
    l, _, _ = window_loss(mo, metric)
    return float(l.mean())


def similarity_grad_M(F: np.ndarray, M: np.ndarray, w: int, metric: int):
    """Return (Sim, dSim/dM) for the fixed image F and the warped image M."""
    mo = window_moments(F, M, w)
    l, a_v, a_c = window_loss(mo, metric)
    n = mo["n"]
    NR = l.size
    alpha = -(2.0 * mo["mM"] * a_v + mo["mF"] * a_c) / n   # dl/dS_M
    beta = a_v / n                                         # dl/dS_MM
    gamma = a_c / n                                        # dl/dS_FM
    r = mo["r"]
    shp = F.shape
    Ba = box_adjoint(alpha, r, shp)
    Bb = box_adjoint(beta, r, shp)
    Bg = box_adjoint(gamma, r, shp)
    M = np.asarray(M, np.float64)
    F = np.asarray(F, np.float64)
    dM = (Ba + 2.0 * M * Bb + F * Bg) / NR
    return float(l.mean()), dM


# ---------------------------------------------------------------------------
# Regulariser (Sec. 2.4, Eq. reg_ss; only the spatial-smoothness term is on
# the path, with alpha_L2 = alpha_ts = 0 in Eq. reg_sum)
# ---------------------------------------------------------------------------

def reg_ss(phi: np.ndarray) -> float:
    """||grad phi||_F^2 by forward differences on the flow grid: for every
    component c and axis d, the mean over valid grid points of the squared
    difference, summed over the nine (c, d) entries."""
    phi = np.asarray(phi, np.float64)
    tot = 0.0
    for d in range(3):
        diff = np.diff(phi, axis=d + 1)
        for c in range(3):
            tot += float(np.mean(diff[c] ** 2))
    return tot


def reg_ss_grad(phi: np.ndarray) -> np.ndarray:
    """Gradient of reg_ss with respect to phi."""
    phi = np.asarray(phi, np.float64)
    g = np.zeros_like(phi)
    for d in range(3):
        diff = np.diff(phi, axis=d + 1)
        m = diff[0].size
        hi = [slice(None)] * 4
        lo = [slice(None)] * 4
        hi[d + 1] = slice(1, None)
        lo[d + 1] = slice(None, -1)
        g[tuple(hi)] += 2.0 * diff / m
        g[tuple(lo)] -= 2.0 * diff / m
    return g


# ---------------------------------------------------------------------------
# Gaussian smoothing of the flow (Sec. 2.4 and Appendix A).  Appendix A
# defines the filter in the Fourier domain: the spectrum of the field is
# multiplied by exp(-(omega / omega_s)^2 / 2) and transformed back.  With the
# discrete Fourier transform of the grid, omega is the angular frequency in
# radians per voxel, omega_k = 2 pi k / n along an axis of n voxels (k taken
# in -n/2..n/2), and omega_s = 1 / sigma for a width sigma in voxels, so the
# transfer is exp(-sigma^2 |omega|^2 / 2).  The filter is therefore periodic
# (the FFT's boundary), real, and even in omega: it maps real fields to real
# fields and is its own adjoint.
# ---------------------------------------------------------------------------

def gaussian_transfer(shape, sigma: float) -> np.ndarray:
    """exp(-sigma^2 |omega|^2 / 2) on the DFT frequencies of a grid of the
    given (D, H, W) shape, omega in radians per voxel."""
    om = [2.0 * np.pi * np.fft.fftfreq(n) for n in shape]
    w2 = om[0][:, None, None] ** 2 + om[1][None, :, None] ** 2 + om[2][None, None, :] ** 2
    return np.exp(-0.5 * sigma ** 2 * w2)


def smooth(phi: np.ndarray, sigma: float) -> np.ndarray:
    """Appendix A's Fourier-domain Gaussian, applied to every component of a
    (3, D, H, W) field: forward FFT over the three spatial axes, multiply by
    the transfer function, inverse FFT, real part."""
    phi = np.asarray(phi, np.float64)
    if sigma <= 0.0:
        return phi.copy()
    tf = gaussian_transfer(phi.shape[1:], sigma)
    spec = np.fft.fftn(phi, axes=(1, 2, 3))
    return np.real(np.fft.ifftn(spec * tf[None], axes=(1, 2, 3)))


# ---------------------------------------------------------------------------
# Loss and gradient (Sec. 2.2 loss, Sec. 2.4 Eq. reg_sum)
# ---------------------------------------------------------------------------

def reg_l2(phi: np.ndarray) -> float:
    """Squared L2 norm of one flow (the second form of Eq. reg_ss): the mean
    over voxels of the squared vector norm, so that its weight does not
    depend on the grid size (the same reading as L_ss)."""
    phi = np.asarray(phi, np.float64)
    return float((phi ** 2).sum(axis=0).mean())


def reg_l2_grad(phi: np.ndarray) -> np.ndarray:
    phi = np.asarray(phi, np.float64)
    return 2.0 * phi / phi[0].size


def reg_ts(phis: List[np.ndarray], times: Sequence[float]) -> float:
    """Temporal smoothness (Eq. reg_ts): for each inner session k the flow of
    the interval before it and the flow of the interval after it, each divided
    by its interval length, should agree; the mean over voxels of the squared
    vector norm of their difference, averaged over the N-2 inner sessions.
    The earlier interval's flow is read as phi_{k-1,k} (the flow forward in
    time), under which a flow proportional to the interval length costs
    nothing.  Zero for N = 2."""
    N = len(phis) + 1
    if N < 3:
        return 0.0
    dt = np.diff(np.asarray(times, np.float64))
    tot = 0.0
    for k in range(1, N - 1):
        a = np.asarray(phis[k - 1], np.float64) / dt[k - 1] - np.asarray(phis[k], np.float64) / dt[k]
        tot += float((a ** 2).sum(axis=0).mean())
    return tot / (N - 2)


def reg_ts_grad(phis: List[np.ndarray], times: Sequence[float]) -> List[np.ndarray]:
    """d reg_ts / d phi_i for every interval i."""
    N = len(phis) + 1
    g = [np.zeros_like(np.asarray(x, np.float64)) for x in phis]
    if N < 3:
        return g
    dt = np.diff(np.asarray(times, np.float64))
    V = np.asarray(phis[0])[0].size
    for k in range(1, N - 1):
        a = np.asarray(phis[k - 1], np.float64) / dt[k - 1] - np.asarray(phis[k], np.float64) / dt[k]
        g[k - 1] += 2.0 * a / (dt[k - 1] * V * (N - 2))
        g[k] -= 2.0 * a / (dt[k] * V * (N - 2))
    return g


# ---------------------------------------------------------------------------
# Rigid adjustment (Sec. 2.5): Euler angles and a translation per session
# ---------------------------------------------------------------------------

def _rot(axis_a: int, axis_b: int, t: float, deriv: bool = False) -> np.ndarray:
    """Rotation by t in the plane of components (axis_a, axis_b), turning a
    towards b (or its derivative with respect to t)."""
    R = np.zeros((3, 3)) if deriv else np.eye(3)
    c, s_ = math.cos(t), math.sin(t)
    if deriv:
        c, s_ = -s_, c
    R[axis_a, axis_a] = c
    R[axis_b, axis_b] = c
    R[axis_a, axis_b] = -s_
    R[axis_b, axis_a] = s_
    return R


def rigid_matrix(theta, deriv: Optional[int] = None) -> np.ndarray:
    """R = Rz Ry Rx in (z, y, x) components: Rz turns y towards x, Ry turns x
    towards z, Rx turns z towards y.  With deriv = k, dR/dtheta_k."""
    tz, ty, tx = (float(v) for v in theta)
    f = [_rot(1, 2, tz, deriv == 0), _rot(2, 0, ty, deriv == 1), _rot(0, 1, tx, deriv == 2)]
    return f[0] @ f[1] @ f[2]


def rigid_displacement(params, shape) -> np.ndarray:
    """L(p) - p for the linear map L(p) = R (p - c) + c + t of one session;
    params = (theta_z, theta_y, theta_x, t_z, t_y, t_x), c the centre of the
    grid, all in voxels of that grid."""
    R = rigid_matrix(params[:3])
    g = identity_grid(shape)
    c = np.array([(n - 1) / 2.0 for n in shape])[:, None, None, None]
    q = np.einsum("cd,d...->c...", R, g - c) + c + np.asarray(params[3:], np.float64)[:, None, None, None]
    return q - g


def rigid_grad(G: np.ndarray, params) -> np.ndarray:
    """d/d params of sum_p G(p) . (L(p) - p) for a field G on the grid."""
    G = np.asarray(G, np.float64)
    shape = G.shape[1:]
    g = identity_grid(shape)
    c = np.array([(n - 1) / 2.0 for n in shape])[:, None, None, None]
    M = G.reshape(3, -1) @ (g - c).reshape(3, -1).T   # sum_p G(p) (p - c)^T
    out = np.zeros(6)
    for k in range(3):
        out[k] = float(np.sum(rigid_matrix(params[:3], deriv=k) * M))
    out[3:] = G.reshape(3, -1).sum(axis=1)
    return out


@dataclass
class Params:
    K: int = 7                 # squarings in Exp
    window: int = 5            # w, the window edge
    metric: int = LNCC         # LNCC or SILNCC
    alpha_ss: float = 1.0      # weight of L_ss
    alpha_l2: float = 0.0      # weight of L_L2
    alpha_ts: float = 0.0      # weight of L_ts (needs times)
    times: Optional[Tuple[float, ...]] = None  # acquisition times t_1..t_N
    flow_factor: int = 1       # 1: flows on the image grid; 2: on a grid twice as coarse
    rigid: bool = False        # rigid adjustment of every session but the first
    smooth_sigma: float = 0.0  # Gaussian smoothing of the flow (voxels of the level); 0 = none
    lr: float = 0.1            # peak learning rate (voxels per step)
    warmup: float = 0.2        # warm-up fraction of each stage
    betas: Tuple[float, float] = (0.9, 0.999)
    eps: float = 1e-8
    iters: Tuple[int, ...] = (50,)   # iterations per pyramid level, coarse to fine


def forward(phis: List[np.ndarray], images: List[np.ndarray], p: Params, keep: bool = False,
            rigid: Optional[List[np.ndarray]] = None):
    """Evaluate L(phi) = sum_i sum_{j != i} Sim(I_i, I_j o Phi_ji^i) + alpha_ss L_ss
    + alpha_L2 L_L2 + alpha_ts L_ts (Eq. reg_sum).

    The flow is first smoothed (smooth_sigma > 0); Exp and L_ss act on the
    smoothed flow.  Returns the loss and, with keep=True, every intermediate
    the backward pass needs (Exp steps, pair fields, warped images)."""
    N = len(images)
    imgs = [np.asarray(I, np.float64) for I in images]
    phis = [smooth(ph, p.smooth_sigma) for ph in phis]
    fwd = [exp_fwd(ph, p.K) for ph in phis]
    bwd = [exp_fwd(-ph, p.K) for ph in phis]
    f = [us[-1] for us in fwd]
    b = [us[-1] for us in bwd]
    U = all_pairs(f, b)
    # the pair fields act on the image grid: with a coarser flow grid they are
    # carried up by the same map as between pyramid levels (Sec. 2.7)
    Ui = U if p.flow_factor == 1 else {k: upsample2(v) for k, v in U.items()}
    if p.rigid and rigid is not None:
        # Sec. 2.5: the pair field that samples session j >= 1 gains the
        # displacement of that session's linear map
        Lj = [None] + [rigid_displacement(r, imgs[0].shape) for r in rigid]
        Ui = {(i, j): (v + Lj[j] if j >= 1 else v) for (i, j), v in Ui.items()}
    sims = {}
    for (i, j), Uij in Ui.items():
        M = warp(imgs[j], Uij)
        sims[(i, j)] = similarity(imgs[i], M, p.window, p.metric)
    Lsim = float(sum(sims.values()))
    Lreg = p.alpha_ss * sum(reg_ss(ph) for ph in phis) / (N - 1)
    if p.alpha_l2:
        Lreg += p.alpha_l2 * sum(reg_l2(ph) for ph in phis) / (N - 1)
    if p.alpha_ts:
        Lreg += p.alpha_ts * reg_ts(phis, p.times)
    L = Lsim + Lreg
    if not keep:
        return L
    return L, dict(fwd=fwd, bwd=bwd, f=f, b=b, U=U, U_img=Ui, sims=sims, Lsim=Lsim, Lreg=Lreg,
                   phis_s=phis)


def pair_sim_grad(images, U, i, j, p: Params):
    """(Sim, dSim/dU[j->i]) for one pair: the similarity adjoint followed by the
    warp derivative."""
    M = warp(images[j], U)
    s, dM = similarity_grad_M(images[i], M, p.window, p.metric)
    return s, dM[None] * warp_grad(images[j], U)


def loss_and_grad(phis: List[np.ndarray], images: List[np.ndarray], p: Params,
                  rigid: Optional[List[np.ndarray]] = None):
    """Return (L, [dL/dphi_i], aux) by hand-written adjoints of every step;
    with a rigid adjustment, aux["rigid_grad"] holds dL/d(params of session j)
    for j = 1..N-1."""
    N = len(images)
    imgs = [np.asarray(I, np.float64) for I in images]
    L, aux = forward(phis, imgs, p, keep=True, rigid=rigid)
    U = aux["U"]
    f, b = aux["f"], aux["b"]
    G = {}
    rg = [np.zeros(6) for _ in range(N - 1)]
    for (i, j), Uij in aux["U_img"].items():
        _, G[(i, j)] = pair_sim_grad(imgs, Uij, i, j, p)
        if p.rigid and rigid is not None and j >= 1:
            rg[j - 1] += rigid_grad(G[(i, j)], rigid[j - 1])
        if p.flow_factor != 1:
            G[(i, j)] = upsample2_adjoint(G[(i, j)], U[(i, j)].shape[1:])
    aux["G_pair_sim"] = {k: v.copy() for k, v in G.items()}
    Gf = [np.zeros_like(x) for x in f]
    Gb = [np.zeros_like(x) for x in b]
    # composition chains, deepest first
    for d in range(N - 1, 1, -1):
        for i in range(N):
            for j in (i + d, i - d):
                if 0 <= j < N:
                    prev, kind, k = chain_parent(i, j)
                    C = f[k] if kind == "f" else b[k]
                    gp, gc = compose_bwd(U[prev], C, G[(i, j)])
                    G[prev] = G[prev] + gp
                    if kind == "f":
                        Gf[k] += gc
                    else:
                        Gb[k] += gc
    for i in range(N - 1):
        Gf[i] += G[(i, i + 1)]
        Gb[i] += G[(i + 1, i)]
    aux["Gf"], aux["Gb"] = Gf, Gb
    aux["rigid_grad"] = rg
    grads = []
    scale = 2.0 ** -p.K
    gts = reg_ts_grad(aux["phis_s"], p.times) if p.alpha_ts else None
    for i in range(len(phis)):
        g0f = exp_bwd(aux["fwd"][i], Gf[i])
        g0b = exp_bwd(aux["bwd"][i], Gb[i])
        g = scale * (g0f - g0b)
        g = g + p.alpha_ss / (N - 1) * reg_ss_grad(aux["phis_s"][i])
        if p.alpha_l2:
            g = g + p.alpha_l2 / (N - 1) * reg_l2_grad(aux["phis_s"][i])
        if p.alpha_ts:
            g = g + p.alpha_ts * gts[i]
        # the smoothing is self-adjoint
        grads.append(smooth(g, p.smooth_sigma))
    return L, grads, aux


# ---------------------------------------------------------------------------
# Optimiser (Sec. 2.7: Adam, linear warm-up over the first 20 %, cosine decay)
# ---------------------------------------------------------------------------

def lr_schedule(t: int, T: int, lr0: float, warmup: float = 0.2) -> float:
    """Learning rate at Adam step t = 1..T of a stage of T steps: linear from
    0 to lr0 over the first W = ceil(warmup*T) steps, then a half cosine from
    lr0 down to 0 at t = T."""
    W = max(1, int(math.ceil(warmup * T)))
    if t <= W:
        return lr0 * t / W
    if T == W:
        return lr0
    return lr0 * 0.5 * (1.0 + math.cos(math.pi * (t - W) / (T - W)))


def adam_step(x, g, m, v, t, lr, betas=(0.9, 0.999), eps=1e-8):
    """One Adam update with bias correction and no weight decay; returns the
    new (x, m, v)."""
    b1, b2 = betas
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    x = x - lr * mhat / (np.sqrt(vhat) + eps)
    return x, m, v


# ---------------------------------------------------------------------------
# Pyramid (Sec. 2.7: three stages, each initialised from the previous one)
# ---------------------------------------------------------------------------

def pool2(I: np.ndarray) -> np.ndarray:
    """2x2x2 mean: one level down the image pyramid."""
    I = np.asarray(I, np.float64)
    D, H, W = I.shape
    return I.reshape(D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(1, 3, 5))


def upsample2(phi: np.ndarray) -> np.ndarray:
    """A displacement field on a grid twice as fine: fine voxel x sits at
    coarse coordinate (x - 0.5)/2, and voxel units halve, so values double."""
    phi = np.asarray(phi, np.float64)
    D, H, W = phi.shape[1:]
    g = identity_grid((2 * D, 2 * H, 2 * W))
    return 2.0 * sample(phi, (g - 0.5) / 2.0)


def upsample2_adjoint(g: np.ndarray, shape) -> np.ndarray:
    """Adjoint of upsample2 for a coarse grid of the given shape: each fine
    voxel hands twice its value back to the corners of the coarse cell it
    sampled, with the same trilinear weights."""
    g = np.asarray(g, np.float64)
    fine = identity_grid(g.shape[1:])
    return 2.0 * sample_adjoint(g, (fine - 0.5) / 2.0, shape)


def level_sigma(p: Params, level: int) -> float:
    """Smoothing width at a pyramid level: smooth_sigma is given in voxels of
    the finest level's flow grid and halves with every coarser level."""
    return p.smooth_sigma / 2.0 ** (len(p.iters) - 1 - level)


def rigid_lr(lr: float, shape) -> np.ndarray:
    """Step sizes of the rigid parameters: lr voxels for the translations and
    lr / r for the angles, r the largest half-extent of the grid, so that a
    step of either moves the farthest voxel by about lr."""
    r = max((n - 1) / 2.0 for n in shape)
    return np.array([lr / r] * 3 + [lr] * 3)


def register(images: List[np.ndarray], p: Params, phis0: Optional[List[np.ndarray]] = None,
             record: bool = False):
    """The whole optimisation: pyramid levels coarse to fine, each running
    Adam on L(phi) (and on the rigid parameters when p.rigid) for
    p.iters[level] steps from a schedule that restarts per level.  Returns
    (the smoothed flows that parameterise the final deformations, on the
    finest flow grid; pair fields on that grid; loss history); with p.rigid
    the rigid parameters of sessions 1..N-1 (finest grid) follow as a fourth
    item."""
    L_lv = len(p.iters)
    imgs_lv = [[np.asarray(I, np.float64) for I in images]]
    for _ in range(L_lv - 1):
        imgs_lv.insert(0, [pool2(I) for I in imgs_lv[0]])
    N = len(images)
    phis = None
    rig = [np.zeros(6) for _ in range(N - 1)]
    hist = []
    for lv in range(L_lv):
        imgs = imgs_lv[lv]
        shape = tuple(n // p.flow_factor for n in imgs[0].shape)
        if phis is None:
            phis = phis0 if phis0 is not None else [np.zeros((3,) + shape) for _ in range(N - 1)]
            phis = [np.asarray(x, np.float64) for x in phis]
        else:
            phis = [upsample2(x) for x in phis]
            # translations are in voxels of the level: twice as many one level up
            rig = [np.concatenate([r[:3], 2.0 * r[3:]]) for r in rig]
        m = [np.zeros_like(x) for x in phis]
        v = [np.zeros_like(x) for x in phis]
        rm = [np.zeros(6) for _ in range(N - 1)]
        rv = [np.zeros(6) for _ in range(N - 1)]
        rlr = rigid_lr(1.0, imgs[0].shape)
        T = p.iters[lv]
        pl = Params(**{**p.__dict__, "smooth_sigma": level_sigma(p, lv)})
        for t in range(1, T + 1):
            L, grads, aux = loss_and_grad(phis, imgs, pl, rigid=rig if p.rigid else None)
            hist.append(L)
            lr = lr_schedule(t, T, p.lr, p.warmup)
            for k in range(N - 1):
                phis[k], m[k], v[k] = adam_step(phis[k], grads[k], m[k], v[k], t, lr,
                                                p.betas, p.eps)
            if p.rigid:
                for k in range(N - 1):
                    # Adam per parameter with its own step size
                    b1, b2 = p.betas
                    g = aux["rigid_grad"][k]
                    rm[k] = b1 * rm[k] + (1 - b1) * g
                    rv[k] = b2 * rv[k] + (1 - b2) * g * g
                    mh = rm[k] / (1 - b1 ** t)
                    vh = rv[k] / (1 - b2 ** t)
                    rig[k] = rig[k] - lr * rlr * mh / (np.sqrt(vh) + p.eps)
    sm = [smooth(ph, level_sigma(p, L_lv - 1)) for ph in phis]
    fwd = [exp_fwd(ph, p.K)[-1] for ph in sm]
    bwd = [exp_fwd(-ph, p.K)[-1] for ph in sm]
    U = all_pairs(fwd, bwd)
    if p.rigid:
        return sm, U, hist, rig
    return sm, U, hist


# ---------------------------------------------------------------------------
# Evaluation (Sec. 2.8)
# ---------------------------------------------------------------------------

def jacobian_det(U: np.ndarray) -> np.ndarray:
    """det(d(Omega + U)/dx) per voxel for a displacement field U (3, D, H, W):
    the determinant of I + grad U, with the derivatives by central
    differences inside the grid and one-sided differences at its faces."""
    U = np.asarray(U, np.float64)
    J = np.empty((3, 3) + U.shape[1:])
    for c in range(3):
        g = np.gradient(U[c], axis=(0, 1, 2))
        for d in range(3):
            J[c, d] = g[d] + (1.0 if c == d else 0.0)
    return (J[0, 0] * (J[1, 1] * J[2, 2] - J[1, 2] * J[2, 1])
            - J[0, 1] * (J[1, 0] * J[2, 2] - J[1, 2] * J[2, 0])
            + J[0, 2] * (J[1, 0] * J[2, 1] - J[1, 1] * J[2, 0]))


def _roi_vectors(phi: np.ndarray, roi: Optional[np.ndarray]) -> np.ndarray:
    phi = np.asarray(phi, np.float64)
    v = phi.reshape(3, -1)
    if roi is not None:
        v = v[:, np.asarray(roi, bool).ravel()]
    return v


def pcc(phi_true: np.ndarray, phi: np.ndarray, roi: Optional[np.ndarray] = None) -> float:
    """Pearson correlation of two vector fields over the region of interest
    (Sec. 2.8): centre each field by its mean vector, then the sum of the
    per-voxel dot products over the product of the two root sums of squares."""
    a = _roi_vectors(phi_true, roi)
    b = _roi_vectors(phi, roi)
    a = a - a.mean(axis=1, keepdims=True)
    b = b - b.mean(axis=1, keepdims=True)
    return float((a * b).sum() / np.sqrt((a * a).sum() * (b * b).sum()))


def slope(phi_true: np.ndarray, phi: np.ndarray, roi: Optional[np.ndarray] = None) -> float:
    """Bias B (Sec. 2.8): fit phi = A phi_true + b by least squares over the
    region of interest (A 3x3, b a vector) and return trace(A) / 3."""
    a = _roi_vectors(phi_true, roi)
    b = _roi_vectors(phi, roi)
    X = np.vstack([a, np.ones((1, a.shape[1]))]).T        # regressors with intercept
    coef, *_ = np.linalg.lstsq(X, b.T, rcond=None)        # (4, 3): rows of A^T, then b
    A = coef[:3].T
    return float(np.trace(A) / 3.0)


def euclidean_error(phi_true: np.ndarray, phi: np.ndarray, roi: Optional[np.ndarray] = None) -> float:
    """Eu: mean over the region of interest of the point-wise vector distance."""
    d = np.sqrt(((np.asarray(phi_true, np.float64) - np.asarray(phi, np.float64)) ** 2).sum(0))
    if roi is None:
        return float(d.mean())
    return float(d[roi].mean())
