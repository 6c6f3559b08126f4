"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names the passage it rests on.  None of them re-types the oracle's
formula: they check exact identities of the method (scaling and squaring of
constant and affine fields, composition of affine maps, invariances of the
similarity metrics), closed forms (matrix powers and exponentials, the OLS
residual variance, the paper's E[LNCC] approximation), brute force on tiny
inputs, finite differences of the loss, and library routines (torch's Adam,
scipy's expm).
"""
import math

import numpy as np
import pytest
import scipy.linalg
import torch

from oracle import muster_oracle as O


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def smooth_field(shape, amp, seed, sigma=2.0):
    """A smooth random displacement field via scipy's Gaussian filter."""
    import scipy.ndimage as ndi
    r = rng(seed)
    f = np.stack([ndi.gaussian_filter(r.standard_normal(shape), sigma, mode="nearest")
                  for _ in range(3)])
    return f * (amp / np.abs(f).max())


def affine_field(shape, A, b):
    """u(x) = A x + b on the grid."""
    g = O.identity_grid(shape)
    return np.einsum("ab,b...->a...", A, g) + b[:, None, None, None]


# --------------------------------------------------------------------------
# Trilinear sampling (Sec. 2.2) -- the primitive every step uses
# --------------------------------------------------------------------------

def test_sample_reproduces_grid_values_and_affine_functions():
    r = rng(0)
    f = r.standard_normal((2, 5, 6, 7))
    g = O.identity_grid((5, 6, 7))
    got = O.sample(f, g)
    # exact away from the upper border; the last plane is reached with t = 1
    assert np.array_equal(got[:, :-1, :-1, :-1], f[:, :-1, :-1, :-1])
    assert np.allclose(got, f, rtol=0, atol=1e-14)
    # trilinear interpolation is exact on affine functions inside the grid
    A = r.standard_normal((3, 3))
    b = r.standard_normal(3)
    af = affine_field((5, 6, 7), A, b)
    q = r.uniform(0, 1, (3, 40)) * np.array([4, 5, 6])[:, None]
    want = A @ q + b[:, None]
    assert np.allclose(O.sample(af, q), want, atol=1e-12)
    _, J = O.sample(af, q, jac=True)
    assert np.allclose(J, np.broadcast_to(A[:, :, None], J.shape), atol=1e-12)


def test_sample_clamps_to_border_and_zeroes_outside_derivative():
    r = rng(1)
    f = r.standard_normal((1, 4, 4, 4))
    q = np.array([[-3.0, 10.0], [1.5, 1.5], [2.0, 2.0]])
    val, J = O.sample(f, q, jac=True)
    assert np.allclose(val[0, 0], 0.5 * (f[0, 0, 1, 2] + f[0, 0, 2, 2]))
    assert np.allclose(val[0, 1], 0.5 * (f[0, 3, 1, 2] + f[0, 3, 2, 2]))
    assert np.all(J[0, 0] == 0.0)


def test_sample_jacobian_matches_finite_differences():
    r = rng(2)
    f = r.standard_normal((3, 6, 6, 6))
    q = r.uniform(0.2, 4.8, (3, 50))
    _, J = O.sample(f, q, jac=True)
    h = 1e-6
    for d in range(3):
        e = np.zeros((3, 1))
        e[d] = h
        fd = (O.sample(f, q + e) - O.sample(f, q - e)) / (2 * h)
        assert np.allclose(J[:, d], fd, atol=1e-7)


def test_sample_adjoint_is_the_transpose():
    """<S(f, q), g> == <f, S^T(g, q)> for random f, g, q (dot-product test)."""
    r = rng(3)
    shape = (5, 7, 6)
    f = r.standard_normal((3,) + shape)
    q = r.uniform(-1.5, 8.5, (3, 4, 5, 6))
    g = r.standard_normal((3, 4, 5, 6))
    lhs = np.sum(O.sample(f, q) * g)
    rhs = np.sum(f * O.sample_adjoint(g, q, shape))
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))


# --------------------------------------------------------------------------
# Exp (Sec. 2.3, Alg. 1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("K", [0, 3, 7])
def test_T1_zero_svf_gives_identity(K):
    us = O.exp_fwd(np.zeros((3, 6, 7, 8)), K)
    assert len(us) == K + 1
    assert np.all(us[-1] == 0.0)


@pytest.mark.parametrize("K", [1, 4, 7])
def test_T2_constant_svf_gives_exact_translation(K):
    c = np.array([0.7, -1.3, 2.25])
    phi = np.broadcast_to(c[:, None, None, None], (3, 9, 8, 7)).copy()
    uK = O.exp_fwd(phi, K)[-1]
    assert np.array_equal(uK, phi)


@pytest.mark.parametrize("K", [3, 6, 8])
def test_T3_affine_svf_is_a_matrix_power(K):
    shape = (26, 26, 26)
    r = rng(10 + K)
    A = 0.01 * r.standard_normal((3, 3))
    c = np.full(3, 12.5)
    b = 0.05 * r.standard_normal(3)
    phi = affine_field(shape, A, b - A @ c)      # phi(x) = A (x - c) + b
    uK = O.exp_fwd(phi, K)[-1]
    # Phi_0 = x + phi/2^K is affine; Phi_K = Phi_0 composed 2^K times
    M0 = np.eye(4)
    M0[:3, :3] += A / 2 ** K
    M0[:3, 3] = (b - A @ c) / 2 ** K
    MK = np.linalg.matrix_power(M0, 2 ** K)
    g = O.identity_grid(shape)
    want = np.einsum("ab,b...->a...", MK[:3, :3] - np.eye(3), g) + MK[:3, 3][:, None, None, None]
    s = slice(K + 2, -(K + 2))
    assert np.max(np.abs(uK[:, s, s, s] - want[:, s, s, s])) < 1e-11
    # and it approaches the matrix exponential of the generator at O(2^-K)
    Gen = np.zeros((4, 4))
    Gen[:3, :3] = A
    Gen[:3, 3] = b - A @ c
    E = scipy.linalg.expm(Gen)
    want_e = np.einsum("ab,b...->a...", E[:3, :3] - np.eye(3), g) + E[:3, 3][:, None, None, None]
    err = np.max(np.abs(uK[:, s, s, s] - want_e[:, s, s, s]))
    assert err < 0.2 * 2.0 ** -K


def test_T4_composition_of_affine_fields_is_the_matrix_product():
    shape = (20, 20, 20)
    r = rng(4)
    A1, A2 = 0.02 * r.standard_normal((3, 3)), 0.02 * r.standard_normal((3, 3))
    b1, b2 = 0.3 * r.standard_normal(3), 0.3 * r.standard_normal(3)
    U1, C = affine_field(shape, A1, b1), affine_field(shape, A2, b2)
    out = O.compose(U1, C)
    # (x + C(x)) o (x + U1(x)) = (I + A2)((I + A1) x + b1) + b2
    Mtot = (np.eye(3) + A2) @ (np.eye(3) + A1)
    btot = (np.eye(3) + A2) @ b1 + b2
    want = affine_field(shape, Mtot - np.eye(3), btot)
    s = slice(2, -2)
    assert np.max(np.abs(out[:, s, s, s] - want[:, s, s, s])) < 1e-12


@pytest.mark.parametrize("shape", [(20, 18, 14), (24, 21, 30)])
def test_adjoints_of_a_contraction_have_closed_forms(shape):
    """With u(p) = -r (p - c) towards the grid centre every sample position
    stays inside, and the adjoints of the squaring step and the composition
    (Alg. 1, Eq. cum_deformation) reduce to closed forms:
    * composition of -r_U (p - c) and -r_C (p - c) under a constant gradient
      g: G_prev = (1 - r_C) g; with r_U = 1/2 the sample positions form a
      lattice of spacing 1/2, on which the linear hat functions sum to 2 per
      axis, so G_C = 8 g wherever each hat's support is covered and 0 farther
      than one voxel from the positions;
    * Exp adjoint: one squaring of u_s = -a_s (p - c) multiplies the sum of
      the gradient by 2 - a_s (own term 1, Jacobian term -a_s, scatter
      weights summing to 1)."""
    g = O.identity_grid(shape)
    c = np.array([(n - 1) / 2.0 for n in shape])[:, None, None, None]
    gv = np.array([1.0, -2.0, 0.5])[:, None, None, None] * np.ones((3,) + shape)
    rU, rC = 0.5, 0.25
    wp, wc = O.compose_bwd(-rU * (g - c), -rC * (g - c), gv)
    assert np.abs(wp - (1 - rC) * gv).max() < 1e-14
    inner, outer = [], []
    for n in shape:
        lo, hi = (n - 1) / 4.0, 3.0 * (n - 1) / 4.0
        inner.append(slice(int(np.ceil(lo + 1.0)), int(np.floor(hi - 1.0)) + 1))
        outer.append((int(np.floor(lo - 1.0)), int(np.ceil(hi + 1.0))))
    for a in range(3):
        assert np.abs(wc[a][tuple(inner)] - 8 * gv[a, 0, 0, 0]).max() < 1e-12
        for ax in range(3):
            lo_end, hi_start = outer[ax]
            for sl in (slice(0, lo_end + 1), slice(hi_start, shape[ax])):
                idx = [slice(None)] * 3
                idx[ax] = sl
                assert np.all(wc[a][tuple(idx)] == 0.0)
    # the mass is conserved: every weight lands somewhere
    assert np.allclose(wc.sum(axis=(1, 2, 3)), gv.sum(axis=(1, 2, 3)), rtol=1e-12)
    r, K = 0.5, 2
    us = O.exp_fwd(-r * (g - c), K)
    G0 = O.exp_bwd(us, gv)
    factor = 1.0
    for s in range(K):
        factor *= 2.0 - (1.0 - (1.0 - r / 2 ** K) ** (2 ** s))
    assert np.allclose(G0.sum(axis=(1, 2, 3)), factor * gv.sum(axis=(1, 2, 3)), rtol=1e-12)


@pytest.mark.parametrize("K", [4, 7])
def test_T5_self_composition_equals_one_more_squaring(K):
    v = smooth_field((12, 13, 14), 1.2, seed=K)
    f = O.exp_fwd(v, K)[-1]
    b = O.exp_fwd(-v, K)[-1]
    # a 3-session series whose two intervals share the same field
    U = O.all_pairs([f, f], [b, b])
    want = O.exp_fwd(2 * v, K + 1)[-1]
    assert np.array_equal(U[(0, 2)], want)
    want_b = O.exp_fwd(-2 * v, K + 1)[-1]
    assert np.array_equal(U[(2, 0)], want_b)


def test_T6_exp_of_minus_v_inverts_exp_of_v_at_second_order():
    """Exp(v) o Exp(-v) ~ identity (Sec. 2.3: the inverse is Exp(-phi)).  The
    residual, in physical units, falls at close to second order when the same
    continuous field is sampled on finer grids: clearly faster than first
    order (ratio 2 per halving), about 16x over two halvings."""
    def residual(n):
        L = 1.0
        h = L / (n - 1)
        x = np.linspace(0, L, n)
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        vphys = 0.04 * np.stack([np.sin(2 * np.pi * Y) * np.cos(np.pi * X),
                                 np.cos(2 * np.pi * Z) * np.sin(np.pi * X),
                                 np.sin(np.pi * Z) * np.sin(np.pi * Y)])
        v = vphys / h
        f = O.exp_fwd(v, 8)[-1]
        b = O.exp_fwd(-v, 8)[-1]
        res = O.compose(f, b)           # (Omega + b) o (Omega + f) - Omega
        m = n // 4
        return h * np.sqrt(np.mean(res[:, m:-m, m:-m, m:-m] ** 2))
    r1, r2, r3 = residual(17), residual(33), residual(65)
    assert r1 / r2 > 2.5 and r2 / r3 > 2.5
    assert r1 / r3 > 9.0
    assert r3 < 3e-5


# --------------------------------------------------------------------------
# Warp (Sec. 2.1) and similarity (Sec. 2.6)
# --------------------------------------------------------------------------

def test_T7_warp_of_affine_image_is_exact():
    shape = (10, 11, 12)
    g = O.identity_grid(shape)
    cvec, d = np.array([0.3, -0.2, 0.5]), 0.7
    I = np.einsum("a,a...->...", cvec, g) + d
    U = smooth_field(shape, 0.8, seed=5)
    s = slice(2, -2)
    M = O.warp(I, U)
    want = np.einsum("a,a...->...", cvec, g + U) + d
    assert np.allclose(M[s, s, s], want[s, s, s], atol=1e-12)
    G = O.warp_grad(I, U)
    assert np.allclose(G[:, s, s, s], np.broadcast_to(cvec[:, None, None, None], G[:, s, s, s].shape),
                       atol=1e-12)


@pytest.mark.parametrize("w", [3, 5, 7])
def test_T8_lncc_identities(w):
    r = rng(w)
    F = r.uniform(0, 1, (12, 12, 12))
    assert abs(O.similarity(F, F, w, O.LNCC)) < 1e-12
    assert abs(O.similarity(F, 2.5 * F - 0.4, w, O.LNCC)) < 1e-12
    assert abs(O.similarity(F, -1.5 * F + 3.0, w, O.LNCC) - 2.0) < 1e-12
    M = r.uniform(0, 1, (12, 12, 12))
    base = O.similarity(F, M, w, O.LNCC)
    assert abs(O.similarity(3 * F + 1, M, w, O.LNCC) - base) < 1e-12
    assert abs(O.similarity(F, 0.2 * M + 7, w, O.LNCC) - base) < 1e-10


@pytest.mark.parametrize("w", [3, 5, 7])
def test_T8_silncc_identities(w):
    r = rng(10 + w)
    F = r.uniform(0, 1, (12, 12, 12))
    assert abs(O.similarity(F, F, w, O.SILNCC)) < 1e-14
    assert abs(O.similarity(F, 2.5 * F - 0.4, w, O.SILNCC)) < 1e-13
    M = r.uniform(0, 1, (12, 12, 12))
    base = O.similarity(F, M, w, O.SILNCC)
    assert abs(O.similarity(3 * F + 1, M, w, O.SILNCC) - base) < 1e-12
    # not invariant in M: scales by c^2 under M -> cM + d
    assert abs(O.similarity(F, 3 * M + 5, w, O.SILNCC) - 9 * base) < 1e-11


@pytest.mark.parametrize("w", [3, 5])
def test_T9_silncc_is_the_ols_residual_variance(w):
    """M = aF + b + eps with eps ~ N(0, s^2) gives E[SiLNCC_R] = s^2 (n-2)/n,
    the residual variance of a least-squares line through n points."""
    r = rng(20 + w)
    shape = (40, 40, 40)
    F = r.uniform(0, 1, shape)
    s = 0.1
    M = 1.7 * F - 0.3 + s * r.standard_normal(shape)
    n = w ** 3
    want = s * s * (n - 2) / n
    got = O.similarity(F, M, w, O.SILNCC)
    n_indep = (40 // w) ** 3
    tol = 4 * want * math.sqrt(2.0 / (n - 2)) / math.sqrt(n_indep)
    assert abs(got - want) < tol


@pytest.mark.parametrize("w,a,sig", [(3, 1.0, 0.5), (5, 0.7, 0.3), (3, 2.0, 1.5)])
def test_T10_expected_lncc_matches_the_papers_closed_form(w, a, sig):
    """Eq. E_lncc: E[LNCC_R] ~ 1 - 1/sqrt(1 + s^2/(a^2 S^2)); the paper bounds
    the bias of this approximation by about 0.02 at 9 voxels and less at 27."""
    r = rng(30 + w)
    shape = (36, 36, 36)
    F = r.standard_normal(shape)
    M = a * F + 0.5 + sig * r.standard_normal(shape)
    mo = O.window_moments(F, F, w)
    S2 = mo["vF"].mean()
    want = 1.0 - 1.0 / math.sqrt(1.0 + sig * sig / (a * a * S2))
    got = O.similarity(F, M, w, O.LNCC)
    assert abs(got - want) < 0.02


@pytest.mark.parametrize("r_", [1, 2])
def test_T11_box_sums_match_brute_force(r_):
    r = rng(40 + r_)
    X = r.standard_normal((7, 8, 9))
    got = O.box_sum(X, r_)
    D, H, W = X.shape
    assert got.shape == (D - 2 * r_, H - 2 * r_, W - 2 * r_)
    for z in range(r_, D - r_):
        for y in range(r_, H - r_):
            for x in range(r_, W - r_):
                s = 0.0
                for dz in range(-r_, r_ + 1):
                    for dy in range(-r_, r_ + 1):
                        for dx in range(-r_, r_ + 1):
                            s += X[z + dz, y + dy, x + dx]
                assert abs(got[z - r_, y - r_, x - r_] - s) < 1e-12
    # box_adjoint is the transpose of box_sum
    A = r.standard_normal(got.shape)
    assert abs(np.sum(got * A) - np.sum(X * O.box_adjoint(A, r_, X.shape))) < 1e-10


def test_window_moments_match_numpy_statistics():
    r = rng(50)
    F = r.standard_normal((9, 9, 9))
    M = r.standard_normal((9, 9, 9))
    mo = O.window_moments(F, M, 5)
    z, y, x = 3, 4, 2
    wf = F[z:z + 5, y:y + 5, x:x + 5].ravel()
    wm = M[z:z + 5, y:y + 5, x:x + 5].ravel()
    assert abs(mo["vF"][z, y, x] - np.var(wf)) < 1e-12
    assert abs(mo["vM"][z, y, x] - np.var(wm)) < 1e-12
    assert abs(mo["c"][z, y, x] - np.cov(wf, wm, bias=True)[0, 1]) < 1e-12


# --------------------------------------------------------------------------
# Regulariser (Sec. 2.4)
# --------------------------------------------------------------------------

def test_T12_regulariser_of_affine_field_is_frobenius_norm():
    r = rng(60)
    A = r.standard_normal((3, 3))
    phi = affine_field((6, 7, 8), A, r.standard_normal(3))
    assert abs(O.reg_ss(phi) - np.sum(A * A)) < 1e-10
    assert O.reg_ss(np.full((3, 5, 5, 5), 3.3)) == 0.0


def test_T12_regulariser_gradient_matches_finite_differences():
    r = rng(61)
    phi = r.standard_normal((3, 4, 5, 6))
    g = O.reg_ss_grad(phi)
    h = 1e-6
    for _ in range(40):
        idx = tuple(int(r.integers(0, n)) for n in phi.shape)
        e = np.zeros_like(phi)
        e[idx] = h
        fd = (O.reg_ss(phi + e) - O.reg_ss(phi - e)) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7


# --------------------------------------------------------------------------
# Whole-loss gradient (Sec. 2.2 loss; adjoints of every step)
# --------------------------------------------------------------------------

def _tiny_problem(seed, shape=(8, 8, 8), N=3, amp=0.9):
    r = rng(seed)
    import scipy.ndimage as ndi
    imgs = [ndi.gaussian_filter(r.uniform(0, 1, shape), 1.0) + 0.01 * r.standard_normal(shape)
            for _ in range(N)]
    phis = [smooth_field(shape, amp, seed=seed * 10 + k, sigma=1.5) for k in range(N - 1)]
    return imgs, phis


@pytest.mark.slow
@pytest.mark.parametrize("w,K,metric,seed", [(3, 3, O.LNCC, 1), (5, 4, O.SILNCC, 2)])
def test_T13_gradient_matches_finite_differences_every_parameter(w, K, metric, seed):
    imgs, phis = _tiny_problem(seed)
    p = O.Params(K=K, window=w, metric=metric, alpha_ss=0.5)
    L, grads, _ = O.loss_and_grad(phis, imgs, p)
    gmax = max(np.abs(g).max() for g in grads)

    def fd(k, idx, h):
        pp = [x.copy() for x in phis]
        pm = [x.copy() for x in phis]
        pp[k][idx] += h
        pm[k][idx] -= h
        return (O.forward(pp, imgs, p) - O.forward(pm, imgs, p)) / (2 * h)

    bad = []
    for k in range(len(phis)):
        for idx in np.ndindex(phis[k].shape):
            g = grads[k][idx]
            ok = abs(fd(k, idx, 1e-5) - g) <= 1e-6 * gmax + 1e-5 * abs(g)
            if not ok:
                # the loss is piecewise smooth (trilinear cells, border clamp):
                # a cell face within 1e-5 of the point spoils the wide
                # difference, so look again at a narrower one
                ok = abs(fd(k, idx, 1e-6) - g) <= 1e-6 * gmax + 1e-5 * abs(g)
            if not ok:
                bad.append((k, idx))
    assert bad == []


@pytest.mark.parametrize("w,K,metric,N,seed", [(3, 5, O.SILNCC, 4, 3), (5, 6, O.LNCC, 3, 4),
                                               (3, 3, O.LNCC, 5, 5)])
def test_T13_gradient_matches_finite_differences_sampled(w, K, metric, N, seed):
    imgs, phis = _tiny_problem(seed, shape=(8, 9, 10), N=N)
    p = O.Params(K=K, window=w, metric=metric, alpha_ss=1.0)
    L, grads, _ = O.loss_and_grad(phis, imgs, p)
    r = rng(seed)
    h = 1e-5
    gmax = max(np.abs(g).max() for g in grads)
    for _ in range(60):
        k = int(r.integers(0, N - 1))
        idx = tuple(int(r.integers(0, n)) for n in phis[k].shape)
        pp = [x.copy() for x in phis]
        pm = [x.copy() for x in phis]
        pp[k][idx] += h
        pm[k][idx] -= h
        fd = (O.forward(pp, imgs, p) - O.forward(pm, imgs, p)) / (2 * h)
        assert abs(fd - grads[k][idx]) < 1e-6 * gmax + 1e-5 * abs(fd)
    # and along a random direction through every parameter at once
    dirs = [r.standard_normal(x.shape) for x in phis]
    hh = 1e-6
    Lp = O.forward([x + hh * d for x, d in zip(phis, dirs)], imgs, p)
    Lm = O.forward([x - hh * d for x, d in zip(phis, dirs)], imgs, p)
    dd = sum(np.sum(g * d) for g, d in zip(grads, dirs))
    assert abs((Lp - Lm) / (2 * hh) - dd) < 1e-5 * abs(dd) + 1e-8


# Central differences of the FP64 loss on the 64^3 series, 256 triples per
# metric.  A difference whose interval [-h, h] crosses a cell face of the
# trilinear interpolant (a kink of the loss) is off by up to about 0.6 % of
# max |g| at h = 1e-3 (5 LNCC and 11 SiLNCC triples beyond 1e-4).  At
# h = 1e-4 such crossings are rare (one triple per metric), and at h = 1e-6
# there are none: every triple of both metrics agrees with the adjoint to
# 5.2e-6 of max |g|.  Bounds: at h = 1e-6, every triple within FD6_TOL
# max |g|; at h = 1e-4, every triple within FD4_TOL max |g| but at most 2 %
# (at least one); at h = 1e-3, max |g - fd| below 2 % of max |g| and the
# relative L2 error below 4 %.
FD6_TOL = 2e-5
FD4_TOL = 1e-4
FD3_MAX, FD3_REL = 2e-2, 4e-2
FD_STEPS = {"0.001", "0.0001", "1e-06"}


def fd_check(an, fds, gmax, extra=0.0):
    """Bounds of the 64^3 differences (fds: step -> differences, keys as in
    the stored file); extra widens them by a parity tolerance (fractions of
    max |g|)."""
    f3, f4, f6 = (np.asarray(fds[h]) for h in ("0.001", "0.0001", "1e-06"))
    crossings = int((np.abs(an - f4) >= (FD4_TOL + extra) * gmax).sum())
    return bool(np.all(np.abs(an - f6) < (FD6_TOL + extra) * gmax) and
                crossings <= max(1, len(an) // 50) and
                np.abs(an - f3).max() < (FD3_MAX + extra) * gmax and
                np.linalg.norm(an - f3) < (FD3_REL + extra) * np.linalg.norm(f3))


@pytest.mark.parametrize("metric", ["lncc", "silncc"])
def test_T13_gradient_at_64cubed_matches_stored_finite_differences(metric):
    """The oracle's adjoint on the 64^3 gradient-check series (four phantom
    sessions, K 6, window 7) against central differences of its own FP64 loss
    at random triples away from the border, stored by
    tests/golden/make_phantoms_4x64_fd.py."""
    import json
    import os
    from paper_2412_14671_amd import synth
    with open(os.path.join(os.path.dirname(__file__), "golden", "phantoms_4x64_fd.json")) as f:
        gold = json.load(f)
    s = synth.phantoms_4x64()
    imgs = [x.numpy().astype(np.float64) for x in s.images]
    phis = [x.astype(np.float64) for x in (0.5 * s.svf_true).numpy().astype(np.float32)]
    p = O.Params(K=gold["K"], window=gold["window"], alpha_ss=gold["alpha_ss"],
                 metric=O.LNCC if metric == "lncc" else O.SILNCC)
    L, grads, _ = O.loss_and_grad(phis, imgs, p)
    g = np.stack(grads)
    assert abs(L - gold[metric]["loss"]) <= 1e-12 * abs(L)
    tr = [tuple(t) for t in gold[metric]["triples"]]
    an = np.array([g[t] for t in tr])
    gmax = np.abs(g).max()
    assert set(gold[metric]["fd"]) == FD_STEPS
    assert len(tr) == 256
    assert fd_check(an, gold[metric]["fd"], gmax)


# --------------------------------------------------------------------------
# Optimiser (Sec. 2.7)
# --------------------------------------------------------------------------

def test_T14_adam_matches_torch():
    r = rng(70)
    x0 = r.standard_normal((3, 4, 5, 6))
    grads = [r.standard_normal(x0.shape) * 10 ** r.uniform(-6, 0) for _ in range(12)]
    lrs = [O.lr_schedule(t, 12, 0.1) for t in range(1, 13)]
    xt = torch.tensor(x0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([xt], lr=0.1, betas=(0.9, 0.999), eps=1e-8)
    x, m, v = x0.copy(), np.zeros_like(x0), np.zeros_like(x0)
    for t, (g, lr) in enumerate(zip(grads, lrs), start=1):
        for pg in opt.param_groups:
            pg["lr"] = lr
        xt.grad = torch.tensor(g)
        opt.step()
        x, m, v = O.adam_step(x, g, m, v, t, lr)
    assert np.allclose(x, xt.detach().numpy(), rtol=0, atol=1e-12)


def test_T14_learning_rate_schedule_shape():
    T, lr0 = 50, 0.2
    W = 10
    assert O.lr_schedule(1, T, lr0) == pytest.approx(lr0 / W)
    assert O.lr_schedule(W, T, lr0) == pytest.approx(lr0)
    assert O.lr_schedule(T, T, lr0) == pytest.approx(0.0, abs=1e-15)
    assert O.lr_schedule(30, T, lr0) == pytest.approx(lr0 / 2)
    ws = [O.lr_schedule(t, T, lr0) for t in range(1, W + 1)]
    assert np.allclose(np.diff(ws), lr0 / W)
    cs = [O.lr_schedule(t, T, lr0) for t in range(W, T + 1)]
    assert all(a > b for a, b in zip(cs, cs[1:]))


# --------------------------------------------------------------------------
# Pyramid (Sec. 2.7)
# --------------------------------------------------------------------------

def test_T15_pool2_of_affine_image_is_affine_at_cell_centres():
    shape = (8, 10, 12)
    g = O.identity_grid(shape)
    c, d = np.array([0.3, -0.7, 1.1]), 2.0
    I = np.einsum("a,a...->...", c, g) + d
    P = O.pool2(I)
    gc = O.identity_grid(P.shape)
    want = np.einsum("a,a...->...", c, 2 * gc + 0.5) + d
    assert np.allclose(P, want, atol=1e-12)
    r = rng(80)
    X = r.standard_normal(shape)
    assert abs(O.pool2(X)[1, 2, 3] - X[2:4, 4:6, 6:8].mean()) < 1e-14


def test_T15_upsample2_of_affine_field_is_exact_in_the_interior():
    r = rng(81)
    A = 0.05 * r.standard_normal((3, 3))
    b = r.standard_normal(3)
    coarse = affine_field((6, 7, 8), A, b)
    fine = O.upsample2(coarse)
    assert fine.shape == (3, 12, 14, 16)
    g = O.identity_grid((12, 14, 16))
    # physical displacement 2*phi_c at coarse position (x - 0.5)/2
    want = np.einsum("ab,b...->a...", A, g - 0.5) + 2 * b[:, None, None, None]
    s = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.allclose(fine[s], want[s], atol=1e-12)


# --------------------------------------------------------------------------
# Loss assembly (Sec. 2.2 loss and Eq. cum_deformation; Sec. 2.4 Eq. reg_sum)
# --------------------------------------------------------------------------

def test_pair_fields_of_an_integer_translation_series_are_exact():
    """Sessions I_k(x) = B(x + k c) with an integer shift c are related by
    constant pair fields U[j->i] = (i - j) c; with phi_i = -c every pair field
    is reproduced exactly and every warped session equals its target away
    from the border."""
    r = rng(90)
    N = 4
    c = np.array([1, -1, 2])
    big = r.standard_normal((30, 30, 30))
    shape = (14, 15, 16)
    o = np.array([8, 8, 8])
    imgs = []
    for k in range(N):
        s = o + k * c
        imgs.append(big[s[0]:s[0] + shape[0], s[1]:s[1] + shape[1], s[2]:s[2] + shape[2]])
    phis = [np.broadcast_to(-c[:, None, None, None].astype(float), (3,) + shape).copy()
            for _ in range(N - 1)]
    _, aux = O.forward(phis, imgs, O.Params(K=5, window=3), keep=True)
    U = aux["U"]
    assert len(U) == N * (N - 1)
    m = 2 * (N - 1) + 1
    for (i, j), Uij in U.items():
        want = (i - j) * c.astype(float)
        assert np.array_equal(Uij, np.broadcast_to(want[:, None, None, None], Uij.shape))
        M = O.warp(imgs[j], Uij)
        assert np.array_equal(M[m:-m, m:-m, m:-m], imgs[i][m:-m, m:-m, m:-m])


def test_loss_sums_similarity_over_ordered_pairs():
    """N copies of one image up to a positive affine intensity change score 0;
    flipping the sign of one session turns NCC to -1 (LNCC_R = 2) in each of
    the 2(N-1) ordered pairs that involve it, so L = 4(N-1)."""
    r = rng(91)
    N = 4
    B = r.uniform(0, 1, (10, 10, 10))
    imgs = [2.0 * B + 1, 0.5 * B - 3, 1.5 * B, 3.0 * B + 0.2]
    phis = [np.zeros((3, 10, 10, 10)) for _ in range(N - 1)]
    p = O.Params(K=4, window=3, metric=O.LNCC)
    assert abs(O.forward(phis, imgs, p)) < 1e-12
    imgs[2] = -imgs[2]
    assert abs(O.forward(phis, imgs, p) - 4 * (N - 1)) < 1e-10


def test_loss_weights_the_regulariser_by_alpha_over_intervals():
    """Constant images have zero SiLNCC under any deformation, so the loss is
    alpha_ss/(N-1) sum_i ||A_i||_F^2 for affine fields phi_i = A_i x + b_i."""
    r = rng(92)
    N = 4
    shape = (9, 9, 9)
    imgs = [np.full(shape, 0.3 + 0.1 * k) for k in range(N)]
    As = [0.02 * r.standard_normal((3, 3)) for _ in range(N - 1)]
    phis = [affine_field(shape, A, 0.1 * r.standard_normal(3)) for A in As]
    p = O.Params(K=4, window=3, metric=O.SILNCC, alpha_ss=0.7)
    want = 0.7 / (N - 1) * sum(np.sum(A * A) for A in As)
    assert abs(O.forward(phis, imgs, p) - want) < 1e-12


# --------------------------------------------------------------------------
# Gaussian smoothing of the flow (Sec. 2.4, Appendix A)
# --------------------------------------------------------------------------

SMOOTH_SIGMAS = [0.375, 0.5, 0.75, 1.0, 1.5, 3.0]


@pytest.mark.parametrize("sigma", SMOOTH_SIGMAS)
def test_smoothing_scales_every_fourier_mode_by_the_transfer_of_appendix_a(sigma):
    """Appendix A: the spectrum is multiplied by exp(-(omega/omega_s)^2 / 2),
    omega_s = 1/sigma.  A sampled plane wave cos(omega . p + phase) with
    omega_d = 2 pi k_d / n_d is an eigenfunction of that filter on the
    periodic grid, with eigenvalue exp(-sigma^2 |omega|^2 / 2).  Waves along
    each axis alone (Nyquist included) and along all three at once, on a grid
    with odd and even, unequal sides: a frequency in cycles instead of
    radians, a missing 1/2, sigma in place of 1/sigma, an axis mix-up or a
    dropped axis each fail it."""
    shape = (10, 12, 15)
    g = O.identity_grid(shape)
    r = rng(103)
    cases = [(k, 0, 0) for k in (1, 2, 5)] + [(0, k, 0) for k in (1, 3, 6)] \
        + [(0, 0, k) for k in (1, 4, 7)] + [(1, 2, 3), (3, 5, 2), (5, 6, 7)]
    for kz, ky, kx in cases:
        om = [2 * np.pi * kz / shape[0], 2 * np.pi * ky / shape[1], 2 * np.pi * kx / shape[2]]
        phase = r.uniform(0, 2 * np.pi)
        wave = np.cos(om[0] * g[0] + om[1] * g[1] + om[2] * g[2] + phase)
        x = np.zeros((3,) + shape)
        c = int(r.integers(0, 3))
        x[c] = wave
        gain = math.exp(-0.5 * sigma ** 2 * (om[0] ** 2 + om[1] ** 2 + om[2] ** 2))
        y = O.smooth(x, sigma)
        assert np.abs(y[c] - gain * wave).max() < 1e-12, (kz, ky, kx)
        assert np.abs(np.delete(y, c, axis=0)).max() < 1e-12


@pytest.mark.parametrize("s1,s2", [(0.375, 0.5), (0.5, 0.75), (0.75, 1.0), (1.0, 3.0)])
def test_smoothing_composes_as_a_gaussian_semigroup(s1, s2):
    """Two Gaussian filters in a row are one of width sqrt(s1^2 + s2^2): the
    transfer functions multiply.  A sampled, truncated spatial Gaussian does
    not have this property at these widths."""
    x = rng(104).standard_normal((3, 9, 12, 14))
    want = O.smooth(x, math.hypot(s1, s2))
    assert np.abs(O.smooth(O.smooth(x, s1), s2) - want).max() < 1e-12


@pytest.mark.parametrize("sigma", [1.5, 2.0, 3.0])
def test_wide_smoothing_matches_the_continuous_gaussian_convolution(sigma):
    """For a kernel several voxels wide, the Fourier-domain filter and the
    circular convolution with the sampled continuous Gaussian (scipy, wrap
    mode, truncated far out) differ only by the aliasing of the sampled
    Gaussian's spectrum, whose size is exp(-pi^2 sigma^2 / 2) at Nyquist."""
    import scipy.ndimage as ndi
    x = rng(100).standard_normal((3, 16, 20, 24))
    want = np.stack([ndi.gaussian_filter(c, sigma, mode="wrap", truncate=10.0) for c in x])
    bound = 3.0 * math.exp(-0.5 * math.pi ** 2 * sigma ** 2) * np.abs(x).max() + 1e-12
    assert np.abs(O.smooth(x, sigma) - want).max() < bound


def test_narrow_smoothing_rings_like_the_band_limited_gaussian():
    """At sigma = 0.375 the transfer is still 0.5 at Nyquist, so the impulse
    response is not a sampled Gaussian: along one line it is the inverse DFT
    (1/n) sum_k exp(-sigma^2 omega_k^2 / 2) cos(omega_k m) with the
    frequencies of the DFT taken in -pi..pi (omega_k = 2 pi min(k, n-k) / n),
    summed here term by term, and it takes negative values (a sampled
    Gaussian never does)."""
    n, sigma = 16, 0.375
    x = np.zeros((3, 1, 1, n))
    x[0, 0, 0, 0] = 1.0
    h = O.smooth(x, sigma)[0, 0, 0]
    for m in range(n):
        want = sum(math.exp(-0.5 * sigma ** 2 * (2 * math.pi * min(k, n - k) / n) ** 2)
                   * math.cos(2 * math.pi * k * m / n) for k in range(n)) / n
        assert abs(h[m] - want) < 1e-14
    assert h.min() < -1e-3
    assert abs(h.sum() - 1.0) < 1e-14


def test_smoothing_is_self_adjoint_and_keeps_constants():
    r = rng(101)
    a = r.standard_normal((3, 8, 9, 10))
    b = r.standard_normal((3, 8, 9, 10))
    assert abs(np.sum(O.smooth(a, 1.3) * b) - np.sum(a * O.smooth(b, 1.3))) < 1e-10
    c = np.full((3, 6, 7, 8), 2.5)
    assert np.allclose(O.smooth(c, 2.0), c, atol=1e-14)
    assert np.allclose(O.smooth(a, 1.3).mean(axis=(1, 2, 3)), a.mean(axis=(1, 2, 3)), atol=1e-13)
    assert np.array_equal(O.smooth(a, 0.0), a)


def test_T13_gradient_with_smoothing_matches_finite_differences():
    imgs, phis = _tiny_problem(7, shape=(8, 9, 10), N=3)
    p = O.Params(K=4, window=3, metric=O.SILNCC, alpha_ss=1.0, smooth_sigma=0.8)
    L, grads, _ = O.loss_and_grad(phis, imgs, p)
    r = rng(7)
    gmax = max(np.abs(g).max() for g in grads)
    h = 1e-5
    for _ in range(40):
        k = int(r.integers(0, 2))
        idx = tuple(int(r.integers(0, n)) for n in phis[k].shape)
        pp = [x.copy() for x in phis]
        pm = [x.copy() for x in phis]
        pp[k][idx] += h
        pm[k][idx] -= h
        fd = (O.forward(pp, imgs, p) - O.forward(pm, imgs, p)) / (2 * h)
        assert abs(fd - grads[k][idx]) < 1e-6 * gmax + 1e-5 * abs(fd)


# --------------------------------------------------------------------------
# L_L2 and L_ts (Sec. 2.4, the second form of Eq. reg_ss, Eq. reg_ts, Eq. reg_sum)
# --------------------------------------------------------------------------

def test_l2_and_ts_of_constant_fields_have_closed_forms():
    shape = (5, 6, 7)
    a = np.array([0.3, -1.2, 0.5])
    b = np.array([1.0, 0.25, -0.75])
    fa = np.broadcast_to(a[:, None, None, None], (3,) + shape).copy()
    fb = np.broadcast_to(b[:, None, None, None], (3,) + shape).copy()
    assert abs(O.reg_l2(fa) - (a ** 2).sum()) < 1e-14
    # N = 3, intervals 0.5 and 2: the single inner session compares a/0.5 with b/2
    times = (1.0, 1.5, 3.5)
    assert abs(O.reg_ts([fa, fb], times) - ((a / 0.5 - b / 2.0) ** 2).sum()) < 1e-13
    assert O.reg_ts([fa], (0.0, 1.0)) == 0.0


def test_ts_is_zero_for_flow_proportional_to_the_interval_and_not_for_the_sign_flip():
    """The premise of Eq. reg_ts: a deformation flow proportional to time costs
    nothing.  Under the literal phi_{i,i-1} = -phi_{i-1,i} reading it would
    cost 4 |v|^2 instead; this pins the reading."""
    v = smooth_field((6, 7, 8), 1.0, seed=3)
    times = (0.0, 0.7, 2.2, 2.9, 4.0)
    dt = np.diff(times)
    phis = [v * d for d in dt]
    assert O.reg_ts(phis, times) < 1e-28
    literal = np.mean([(((-phis[k - 1]) / dt[k - 1] - phis[k] / dt[k]) ** 2).sum(axis=0).mean()
                       for k in range(1, 4)])
    assert abs(literal - 4 * (v ** 2).sum(axis=0).mean()) < 1e-12


def test_l2_and_ts_gradients_match_finite_differences():
    r = rng(7)
    phis = [0.5 * r.standard_normal((3, 4, 5, 6)) for _ in range(3)]
    times = (0.0, 1.3, 1.9, 3.4)
    h = 1e-6
    g_ts = O.reg_ts_grad(phis, times)
    for trial in range(12):
        i = int(r.integers(0, 3))
        idx = tuple(int(r.integers(0, n)) for n in phis[i].shape)
        up = [x.copy() for x in phis]
        dn = [x.copy() for x in phis]
        up[i][idx] += h
        dn[i][idx] -= h
        fd = (O.reg_ts(up, times) - O.reg_ts(dn, times)) / (2 * h)
        assert abs(fd - g_ts[i][idx]) < 1e-7 * max(1.0, abs(fd))
        fd2 = (O.reg_l2(up[i]) - O.reg_l2(dn[i])) / (2 * h)
        assert abs(fd2 - O.reg_l2_grad(phis[i])[idx]) < 1e-8


def test_total_loss_gradient_with_l2_and_ts_matches_finite_differences():
    """Whole loss (similarity + all three regularisers + smoothing) against
    central differences on sampled parameters."""
    shape = (8, 9, 10)
    r = rng(11)
    import scipy.ndimage as ndi
    imgs = [ndi.gaussian_filter(rng(40 + k).uniform(0, 1, shape), 1.0) for k in range(4)]
    phis = [smooth_field(shape, 0.8, seed=50 + k, sigma=1.5) for k in range(3)]
    p = O.Params(K=4, window=3, metric=O.SILNCC, alpha_ss=0.5, alpha_l2=0.3, alpha_ts=0.7,
                 times=(0.0, 0.6, 2.0, 2.5), smooth_sigma=0.7)
    L, grads, _ = O.loss_and_grad(phis, imgs, p)
    assert abs(L - O.forward(phis, imgs, p)) < 1e-12 * abs(L)
    h = 1e-5
    for trial in range(10):
        i = int(r.integers(0, 3))
        idx = tuple(int(r.integers(1, n - 1)) for n in phis[i].shape)
        up = [x.copy() for x in phis]
        dn = [x.copy() for x in phis]
        up[i][idx] += h
        dn[i][idx] -= h
        fd = (O.forward(up, imgs, p) - O.forward(dn, imgs, p)) / (2 * h)
        assert abs(fd - grads[i][idx]) < 2e-5 * max(1.0, np.abs(grads[i]).max())


# --------------------------------------------------------------------------
# Flow grid twice as coarse as the images (Sec. 2.7 stage geometry)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(2, 3, 4), (5, 6, 7), (8, 8, 8)])
def test_upsample2_adjoint_is_the_transpose_of_upsample2(shape):
    r = rng(200 + sum(shape))
    a = r.standard_normal((3,) + shape)
    b = r.standard_normal((3,) + tuple(2 * n for n in shape))
    lhs = float(np.sum(O.upsample2(a) * b))
    rhs = float(np.sum(a * O.upsample2_adjoint(b, shape)))
    assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs))


def test_coarse_flow_of_a_constant_svf_translates_the_images_by_twice_it():
    """A constant SVF c on the flow grid is a translation by c flow voxels,
    i.e. 2c image voxels: the warped image of the pair is the image sampled
    2c away, exactly."""
    shape = (12, 14, 16)
    c = np.array([0.25, -0.5, 0.375])
    phi = np.broadcast_to(c[:, None, None, None], (3, 6, 7, 8)).copy()
    p = O.Params(K=5, window=3, metric=O.SILNCC, alpha_ss=0.0, flow_factor=2)
    z, y, x = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    imgs = [np.sin(0.3 * z) + np.cos(0.2 * y) + 0.1 * x, np.sin(0.25 * x + 0.1 * y)]
    _, aux = O.forward([phi], imgs, p, keep=True)
    U = aux["U_img"][(0, 1)]
    assert np.allclose(U, 2 * c[:, None, None, None], atol=1e-12)


def test_loss_gradient_with_a_coarse_flow_grid_matches_finite_differences():
    r = rng(12)
    fshape = (5, 6, 7)
    shape = tuple(2 * n for n in fshape)
    import scipy.ndimage as ndi
    imgs = [ndi.gaussian_filter(rng(60 + k).uniform(0, 1, shape), 1.0) for k in range(3)]
    phis = [smooth_field(fshape, 0.6, seed=70 + k, sigma=1.2) for k in range(2)]
    p = O.Params(K=4, window=3, metric=O.LNCC, alpha_ss=0.5, flow_factor=2, smooth_sigma=0.6)
    L, grads, _ = O.loss_and_grad(phis, imgs, p)
    assert abs(L - O.forward(phis, imgs, p)) < 1e-12 * abs(L)
    h = 1e-5
    for trial in range(10):
        i = int(r.integers(0, 2))
        idx = tuple(int(r.integers(0, n)) for n in phis[i].shape)
        up = [x.copy() for x in phis]
        dn = [x.copy() for x in phis]
        up[i][idx] += h
        dn[i][idx] -= h
        fd = (O.forward(up, imgs, p) - O.forward(dn, imgs, p)) / (2 * h)
        assert abs(fd - grads[i][idx]) < 2e-5 * max(1.0, np.abs(grads[i]).max())


# --------------------------------------------------------------------------
# Outputs and evaluation: Jacobian determinants, Eu, PCC, slope (Sec. 2.8)
# --------------------------------------------------------------------------

def test_jacobian_det_of_affine_and_translation_fields_is_exact():
    shape = (6, 7, 8)
    g = np.stack(np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij"))
    M = np.array([[0.1, -0.05, 0.02], [0.03, -0.2, 0.04], [0.0, 0.06, 0.15]])
    U = np.einsum("cd,d...->c...", M, g) + np.array([1.0, -2.0, 0.5])[:, None, None, None]
    # finite differences (central and one-sided) are exact on linear fields
    assert np.allclose(O.jacobian_det(U), np.linalg.det(np.eye(3) + M), atol=1e-13)
    T = np.broadcast_to(np.array([0.3, 0.1, -0.7])[:, None, None, None], (3,) + shape)
    assert np.allclose(O.jacobian_det(T), 1.0, atol=1e-15)


def test_pcc_and_slope_closed_forms():
    r = rng(300)
    shape = (5, 6, 7)
    a = r.standard_normal((3,) + shape)
    roi = r.uniform(size=shape) > 0.3
    assert abs(O.pcc(a, a, roi) - 1.0) < 1e-12
    assert abs(O.pcc(a, 2.5 * a + np.array([1.0, 2.0, -3.0])[:, None, None, None], roi) - 1.0) < 1e-12
    assert abs(O.pcc(a, -a, roi) + 1.0) < 1e-12
    assert abs(O.slope(a, 0.7 * a + 0.2, roi) - 0.7) < 1e-12
    # a general linear map: the slope is the mean diagonal of the map
    M = np.array([[0.9, 0.1, 0.0], [0.2, 1.3, -0.1], [0.0, 0.05, 0.5]])
    b = np.einsum("cd,d...->c...", M, a) + np.array([0.1, 0.0, -0.2])[:, None, None, None]
    assert abs(O.slope(a, b, roi) - np.trace(M) / 3) < 1e-12
    # independent noise decorrelates
    n = r.standard_normal((3,) + shape)
    assert abs(O.pcc(a, n)) < 0.15


# --------------------------------------------------------------------------
# Rigid adjustment (Sec. 2.5)
# --------------------------------------------------------------------------

def test_euclidean_error_closed_forms():
    """Eu (Sec. 2.8) is the mean over the region of interest of the length of
    the difference vector: a constant offset c gives |c|; offsets of +c on
    half the region and -c on the other half still give |c| (a mean of
    lengths, not the length of a mean); differences outside the region do not
    count, and inside it they count by their share of the region."""
    shape = (6, 7, 8)
    r = rng(130)
    ref = r.standard_normal((3,) + shape)
    c = np.array([0.3, -1.2, 0.4])                       # |c| = 1.3
    assert abs(O.euclidean_error(ref, ref + c[:, None, None, None]) - 1.3) < 1e-12
    sign = np.where(r.uniform(size=shape) < 0.5, 1.0, -1.0)
    assert abs(O.euclidean_error(ref, ref + sign * c[:, None, None, None]) - 1.3) < 1e-12
    roi = np.zeros(shape, bool)
    roi[1:5, 2:6, 1:7] = True
    est = ref.copy()
    est[:, ~roi] += 7.0                                  # outside the region: ignored
    assert O.euclidean_error(ref, est, roi) == 0.0
    inside = np.argwhere(roi)
    hit = inside[r.choice(len(inside), size=10, replace=False)]
    for z, y, x in hit:
        est[:, z, y, x] += np.array([0.0, 3.0, 4.0])      # length 5 at 10 voxels
    assert abs(O.euclidean_error(ref, est, roi) - 5.0 * 10 / roi.sum()) < 1e-12
    assert O.euclidean_error(ref, est) > O.euclidean_error(ref, est, roi)


def test_level_sigma_halves_per_coarser_level_and_keeps_the_physical_width():
    """The smoothing width is given in voxels of the finest grid; a level
    2^m times coarser holds the same physical width in 2^m times fewer of its
    voxels.  So the widths of a three-level pyramid with sigma 3 are 0.75,
    1.5 and 3; and a wave of k periods over the grid is damped alike on every
    level when each level smooths with its own width."""
    p = O.Params(smooth_sigma=3.0, iters=(200, 100, 50))
    assert [O.level_sigma(p, lv) for lv in range(3)] == [0.75, 1.5, 3.0]
    assert O.level_sigma(O.Params(smooth_sigma=1.25, iters=(10,)), 0) == 1.25
    assert O.level_sigma(O.Params(smooth_sigma=2.0, iters=(5, 5, 5, 5)), 0) == 0.25
    fine = (32, 24, 16)
    gains = []
    for lv in range(3):
        shape = tuple(n >> (2 - lv) for n in fine)
        g = O.identity_grid(shape)
        wave = np.cos(2 * np.pi * 2 * g[2] / shape[2])   # two periods across x
        x = np.stack([wave, 0 * wave, 0 * wave])
        gains.append(O.smooth(x, O.level_sigma(p, lv))[0].max() / wave.max())
    assert max(gains) - min(gains) < 0.02 * max(gains)
    assert gains[0] < 0.9


def test_rigid_matrix_is_a_rotation_and_its_derivatives_are_exact():
    th = np.array([0.3, -0.2, 0.45])
    R = O.rigid_matrix(th)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-14) and abs(np.linalg.det(R) - 1) < 1e-14
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1e-6
        fd = (O.rigid_matrix(th + e) - O.rigid_matrix(th - e)) / 2e-6
        assert np.abs(fd - O.rigid_matrix(th, deriv=k)).max() < 1e-9
    # each factor fixes its own axis: a rotation about z leaves the z component
    Rz = O.rigid_matrix([0.7, 0.0, 0.0])
    assert np.allclose(Rz[0], [1, 0, 0]) and np.allclose(Rz[:, 0], [1, 0, 0])


def test_rigid_translation_of_a_translated_series_is_exact_and_zero_params_change_nothing():
    """Session 1 is session 0 read 2 voxels further along x: with phi = 0 and
    a rigid translation of 2 voxels for session 1, pair (0, 1) warps session
    1 exactly onto session 0, so that pair's SiLNCC is zero."""
    shape = (10, 12, 24)
    z, y, x = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    base = lambda xx: np.sin(0.3 * z) * np.cos(0.2 * y) + np.sin(0.15 * xx)
    imgs = [base(x), base(x - 2.0)]
    phi = [np.zeros((3,) + shape)]
    p = O.Params(K=4, window=3, metric=O.SILNCC, alpha_ss=0.0, rigid=True)
    _, aux = O.forward(phi, imgs, p, keep=True, rigid=[np.array([0, 0, 0, 0, 0, 2.0])])
    # interior windows see exact copies; the clamped border strip does not
    U = aux["U_img"][(0, 1)]
    assert np.allclose(U[2], 2.0) and np.allclose(U[:2], 0.0)
    M = O.warp(imgs[1], U)
    assert np.abs(M[:, :, :20] - imgs[0][:, :, :20]).max() < 1e-12
    p0 = O.Params(K=4, window=3, metric=O.SILNCC, alpha_ss=0.0)
    assert O.forward(phi, imgs, p0) == O.forward(phi, imgs, p, rigid=[np.zeros(6)])


def test_rigid_gradient_matches_finite_differences():
    shape = (8, 9, 10)
    import scipy.ndimage as ndi
    imgs = [ndi.gaussian_filter(rng(80 + k).uniform(0, 1, shape), 1.2) for k in range(3)]
    phis = [smooth_field(shape, 0.5, seed=90 + k, sigma=1.5) for k in range(2)]
    rig = [np.array([0.05, -0.03, 0.02, 0.3, -0.2, 0.1]), np.array([-0.02, 0.04, 0.01, -0.1, 0.25, 0.2])]
    p = O.Params(K=4, window=3, metric=O.LNCC, alpha_ss=0.3, rigid=True)
    L, grads, aux = O.loss_and_grad(phis, imgs, p, rigid=rig)
    h = 1e-6
    for j in range(2):
        for k in range(6):
            up = [r.copy() for r in rig]
            dn = [r.copy() for r in rig]
            up[j][k] += h
            dn[j][k] -= h
            fd = (O.forward(phis, imgs, p, rigid=up) - O.forward(phis, imgs, p, rigid=dn)) / (2 * h)
            assert abs(fd - aux["rigid_grad"][j][k]) < 1e-5 * max(1.0, abs(fd))


# --------------------------------------------------------------------------
# The optimisation loop (Sec. 2.7): Adam per pyramid stage, from a schedule
# that restarts per stage, each stage started from the previous one's flows
# --------------------------------------------------------------------------

def _torch_adam_registration(images, p):
    """The registration loop with torch's Adam as the optimiser: one
    optimiser per pyramid stage (so its moments and step count restart), the
    rigid angles and translations in parameter groups of their own with step
    sizes lr / r and lr, the oracle's pinned loss, gradient, pool, upsampling
    and schedule as the steps."""
    n_lv, N = len(p.iters), len(images)
    pyr = [[np.asarray(I, np.float64) for I in images]]
    for _ in range(n_lv - 1):
        pyr.insert(0, [O.pool2(I) for I in pyr[0]])
    phis, ang, tra, hist = None, [np.zeros(3)] * (N - 1), [np.zeros(3)] * (N - 1), []
    for lv, T in enumerate(p.iters):
        imgs = pyr[lv]
        if phis is None:
            phis = [np.zeros((3,) + tuple(n // p.flow_factor for n in imgs[0].shape))
                    for _ in range(N - 1)]
        else:
            phis = [O.upsample2(x) for x in phis]
            tra = [2.0 * t for t in tra]
        xs = [torch.tensor(x, requires_grad=True) for x in phis]
        at = [torch.tensor(a, requires_grad=True) for a in ang]
        tt = [torch.tensor(t, requires_grad=True) for t in tra]
        r = max((n - 1) / 2.0 for n in imgs[0].shape)
        groups = [{"params": xs, "scale": 1.0}]
        if p.rigid:
            groups += [{"params": at, "scale": 1.0 / r}, {"params": tt, "scale": 1.0}]
        opt = torch.optim.Adam(groups, lr=p.lr, betas=p.betas, eps=p.eps)
        # the smoothing width is given on the finest grid: a level that is
        # 2^m times coarser sees it as 2^m times fewer of its voxels
        pl = O.Params(**{**p.__dict__, "smooth_sigma": p.smooth_sigma / 2 ** (n_lv - 1 - lv)})
        for t in range(1, T + 1):
            rig = [np.concatenate([a.detach().numpy(), b.detach().numpy()]) for a, b in zip(at, tt)]
            L, grads, aux = O.loss_and_grad([x.detach().numpy() for x in xs], imgs, pl,
                                            rigid=rig if p.rigid else None)
            hist.append(L)
            for x, g in zip(xs, grads):
                x.grad = torch.tensor(g)
            if p.rigid:
                for a, b, g in zip(at, tt, aux["rigid_grad"]):
                    a.grad = torch.tensor(g[:3])
                    b.grad = torch.tensor(g[3:])
            for pg in opt.param_groups:
                pg["lr"] = O.lr_schedule(t, T, p.lr, p.warmup) * pg["scale"]
            opt.step()
        phis = [x.detach().numpy().copy() for x in xs]
        ang = [a.detach().numpy().copy() for a in at]
        tra = [b.detach().numpy().copy() for b in tt]
    sm = [O.smooth(x, p.smooth_sigma) for x in phis]
    return sm, hist, [np.concatenate([a, b]) for a, b in zip(ang, tra)]


@pytest.mark.parametrize("case", [
    dict(shape=(8, 8, 8), iters=(3, 2), K=3, window=3, metric=O.SILNCC, alpha_ss=0.5,
         smooth_sigma=1.0, rigid=True, flow_factor=1),
    dict(shape=(16, 12, 16), iters=(2, 3), K=4, window=3, metric=O.LNCC, alpha_ss=0.2,
         alpha_l2=0.1, alpha_ts=0.3, times=(0.0, 1.0, 2.5), smooth_sigma=0.0, rigid=False,
         flow_factor=2),
])
def test_T16_registration_loop_matches_a_torch_adam_driver(case):
    """register() against the same loop driven by torch.optim.Adam: the flows,
    the rigid parameters, the loss at every step and the pair fields agree to
    rounding.  A moment or step count carried across stages, a schedule
    indexed from 0, swapped rigid step sizes or translations not rescaled
    between stages fail it."""
    shape = case.pop("shape")
    r = rng(91)
    import scipy.ndimage as ndi
    imgs = [ndi.gaussian_filter(r.uniform(0, 1, shape), 1.0) for _ in range(3)]
    p = O.Params(lr=0.3, **case)
    out = O.register(imgs, p)
    sm, U, hist = out[0], out[1], out[2]
    sm_t, hist_t, rig_t = _torch_adam_registration(imgs, p)
    assert len(hist) == sum(p.iters)
    assert np.allclose(hist, hist_t, rtol=1e-10, atol=0)
    scale = max(np.abs(x).max() for x in sm_t)
    assert scale > 1e-3  # the flows moved
    for a, b in zip(sm, sm_t):
        assert np.abs(a - b).max() < 1e-9 * scale
    if p.rigid:
        assert max(np.abs(x).max() for x in rig_t) > 1e-4
        for a, b in zip(out[3], rig_t):
            assert np.allclose(a, b, rtol=0, atol=1e-10)
    fwd = [O.exp_fwd(x, p.K)[-1] for x in sm_t]
    bwd = [O.exp_fwd(-x, p.K)[-1] for x in sm_t]
    for key, Uk in O.all_pairs(fwd, bwd).items():
        assert np.abs(U[key] - Uk).max() < 1e-8
