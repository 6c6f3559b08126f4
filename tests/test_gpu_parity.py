"""Parity of every HIP kernel with the FP64 oracle, element by element, through
the C ABI.  Tolerances (FP32 kernels against an FP64 reference): 1e-4 voxel
maximum displacement error per integration and composition, 1e-3 relative on
losses and gradients (relative L2, and maximum error within 1e-3 of the largest
magnitude).  Shapes span several tiles and ragged tails (tiles are 8x8x16
voxels for the gather kernels and 8x32 columns for the window statistics)."""
import math
import sys

import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

from oracle import muster_oracle as O

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2412_14671_amd import Context
    c = Context(0)
    yield c
    c.close()


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def smooth_field(shape, amp, seed, sigma=3.0):
    r = rng(seed)
    f = np.stack([ndi.gaussian_filter(r.standard_normal(shape), sigma, mode="wrap") for _ in range(3)])
    return (f * (amp / np.abs(f).max())).astype(np.float32)


def smooth_image(shape, seed, sigma=2.0, noise=0.02):
    r = rng(seed)
    x = ndi.gaussian_filter(r.uniform(0, 1, shape), sigma, mode="wrap")
    x = (x - x.min()) / (x.max() - x.min())
    return (x + noise * r.standard_normal(shape)).astype(np.float32)


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def assert_grad_close(got, want, tol=1e-3):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    scale = np.abs(want).max()
    rel = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)
    mx = np.abs(got - want).max() / max(scale, 1e-300)
    assert rel < tol and mx < tol, f"rel L2 {rel:.2e}, max {mx:.2e}"


SHAPES = [(32, 32, 32), (20, 27, 35), (45, 37, 70)]


# ---------------------------------------------------------------------------
# Exp (Alg. 1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("K,sign", [(7, 1), (6, -1)])
def test_exp_matches_oracle(ctx, shape, K, sign):
    log(f"exp {shape} K={K} sign={sign}")
    phi = smooth_field(shape, 2.5, seed=sum(shape) + K)
    disp, steps = ctx.exp(gpu(phi), K, sign, steps=True)
    us = O.exp_fwd(sign * phi.astype(np.float64), K)
    st = host(steps)
    for s in range(1, K + 1):
        err = np.abs(st[s - 1] - us[s]).max()
        assert err < 1e-4, f"step {s}: {err}"
    assert np.array_equal(host(disp), st[K - 1])


def test_exp_of_constant_field_is_exact(ctx):
    shape = (19, 24, 33)
    c = np.array([0.75, -1.5, 2.25], np.float32)
    phi = np.broadcast_to(c[:, None, None, None], (3,) + shape).copy()
    out = host(ctx.exp(gpu(phi), 7, 1))
    assert np.array_equal(out, phi.astype(np.float64))
    out = host(ctx.exp(gpu(phi), 5, -1))
    assert np.array_equal(out, -phi.astype(np.float64))


def test_exp_of_zero_field_is_identity(ctx):
    out = host(ctx.exp(torch.zeros((3, 17, 18, 19), device=DEV), 7, 1))
    assert np.all(out == 0.0)


@pytest.mark.parametrize("shape,K", [((32, 32, 32), 7), ((20, 27, 35), 4), ((24, 40, 52), 6),
                                     ((21, 26, 45), 1)])
@pytest.mark.parametrize("mode", ["store", "recompute"])
@pytest.mark.parametrize("flat", [False, True])
def test_exp_bwd_matches_oracle(ctx, shape, K, mode, flat):
    """The adjoint of the integration, through the staged exchange of scatter
    boxes between squaring steps (the registration's path) and through the
    flat path, in both modes of keeping the steps."""
    log(f"exp_bwd {shape} K={K} {mode} flat={flat}")
    phi = smooth_field(shape, 2.0, seed=K + 100)
    G = smooth_field(shape, 1.0, seed=K + 200, sigma=1.0)
    for sign in (1, -1):
        got = host(ctx.exp_bwd(gpu(phi), gpu(G), K, sign, mode, flat=flat))
        us = O.exp_fwd(sign * phi.astype(np.float64), K)
        want = sign * 2.0 ** -K * O.exp_bwd(us, G.astype(np.float64))
        assert_grad_close(got, want)


def test_exp_bwd_store_and_recompute_agree(ctx):
    shape = (28, 30, 33)
    phi = smooth_field(shape, 2.0, seed=7)
    G = smooth_field(shape, 1.0, seed=8, sigma=1.0)
    a = host(ctx.exp_bwd(gpu(phi), gpu(G), 7, 1, "store"))
    b = host(ctx.exp_bwd(gpu(phi), gpu(G), 7, 1, "recompute"))
    # identical arithmetic; only the order of float atomics differs
    assert np.abs(a - b).max() <= 1e-5 * np.abs(a).max()


# ---------------------------------------------------------------------------
# Composition (Eq. cum_deformation)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", SHAPES)
def test_compose_matches_oracle(ctx, shape):
    log(f"compose {shape}")
    U = smooth_field(shape, 4.0, seed=1)
    C = smooth_field(shape, 2.0, seed=2)
    got = host(ctx.compose(gpu(U), gpu(C)))
    want = O.compose(U.astype(np.float64), C.astype(np.float64))
    assert np.abs(got - want).max() < 1e-4


@pytest.mark.parametrize("shape", SHAPES)
def test_compose_bwd_matches_oracle(ctx, shape):
    log(f"compose_bwd {shape}")
    U = smooth_field(shape, 4.0, seed=3)
    C = smooth_field(shape, 2.0, seed=4)
    G = smooth_field(shape, 1.0, seed=5, sigma=1.0)
    gp = torch.zeros((3,) + shape, device=DEV)
    gc = torch.zeros((3,) + shape, device=DEV)
    ctx.compose_bwd(gpu(U), gpu(C), gpu(G), gp, gc)
    wp, wc = O.compose_bwd(U.astype(np.float64), C.astype(np.float64), G.astype(np.float64))
    assert_grad_close(host(gp), wp)
    assert_grad_close(host(gc), wc)


def contracting_field(shape, rate):
    """u(p) = -rate (p - c), c the grid centre: Omega + u pulls every voxel
    towards c by the factor 1 - rate (affine, so trilinear sampling is exact)."""
    g = O.identity_grid(shape)
    c = np.array([(n - 1) / 2.0 for n in shape])[:, None, None, None]
    return (-rate * (g - c)).astype(np.float32)


def test_compose_bwd_survives_strong_contraction(ctx):
    """The adjoint scatter with every sample position crowded into the few
    cells around the grid centre (1/20 of the distances, and the centre on a
    grid point): a block pours about a thousand voxel-weights into one bin,
    four times what the fixed-point bins held before their scale was bounded
    by the block's summed magnitudes."""
    shape = (33, 29, 41)
    U = contracting_field(shape, 0.95)
    C = smooth_field(shape, 2.0, seed=41)
    G = (1.0 + 0.2 * smooth_field(shape, 1.0, seed=42, sigma=1.0)).astype(np.float32)
    gp = torch.zeros((3,) + shape, device=DEV)
    gc = torch.zeros((3,) + shape, device=DEV)
    ctx.compose_bwd(gpu(U), gpu(C), gpu(G), gp, gc)
    wp, wc = O.compose_bwd(U.astype(np.float64), C.astype(np.float64), G.astype(np.float64))
    assert np.abs(wc).max() > 1000 * np.abs(G).max()   # the crowding is real
    assert_grad_close(host(gp), wp)
    assert_grad_close(host(gc), wc)


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("flat", [False, True])
def test_exp_bwd_survives_strong_contraction(ctx, sign, flat):
    """Exp of -6 (p - c) contracts by e^-3 per axis at the last squaring; of
    +6 (p - c) it expands, and the border clamp then crowds every position
    beyond the grid into the border cells.  Both pour hundreds of voxel
    weights into single bins of the scatter."""
    shape = (33, 29, 41)
    K = 7
    phi = contracting_field(shape, 6.0)
    G = (1.0 + 0.2 * smooth_field(shape, 1.0, seed=43, sigma=1.0)).astype(np.float32)
    got = host(ctx.exp_bwd(gpu(phi), gpu(G), K, sign, "store", flat=flat))
    us = O.exp_fwd(sign * phi.astype(np.float64), K)
    want = sign * 2.0 ** -K * O.exp_bwd(us, G.astype(np.float64))
    assert_grad_close(got, want)


# ---------------------------------------------------------------------------
# Warp + windowed similarity (Sec. 2.6)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(32, 32, 32), (21, 26, 45), (40, 17, 66)])
@pytest.mark.parametrize("w", [3, 5, 7])
@pytest.mark.parametrize("metric", ["lncc", "silncc"])
def test_sim_matches_oracle(ctx, shape, w, metric):
    log(f"sim {shape} w={w} {metric}")
    F = smooth_image(shape, seed=w)
    I = smooth_image(shape, seed=w + 1)
    U = smooth_field(shape, 2.0, seed=w + 2)
    val, g = ctx.sim(gpu(F), gpu(I), gpu(U), w, metric, grad=True)
    m = O.LNCC if metric == "lncc" else O.SILNCC
    p = O.Params(window=w, metric=m)
    s_ref, g_ref = O.pair_sim_grad([F.astype(np.float64), I.astype(np.float64)],
                                   U.astype(np.float64), 0, 1, p)
    assert abs(val - s_ref) < 1e-3 * abs(s_ref)
    assert_grad_close(host(g), g_ref)


def test_sim_of_identical_images_is_zero(ctx):
    shape = (30, 34, 38)
    F = smooth_image(shape, seed=3)
    zero = torch.zeros((3,) + shape, device=DEV)
    v = ctx.sim(gpu(F), gpu(F), zero, 5, "lncc")
    assert abs(v) < 1e-5
    v = ctx.sim(gpu(F), gpu(2 * F + 1), zero, 5, "silncc")
    assert abs(v) < 1e-6


# ---------------------------------------------------------------------------
# Degenerate grids: the smallest edges the entry points accept (2 for the
# fields, the window for the similarity), grids smaller than one tile, and
# one-cell-thick slabs across several tiles
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(2, 2, 2), (2, 3, 70), (3, 5, 7), (9, 2, 17)])
def test_field_kernels_on_minimal_grids_match_oracle(ctx, shape):
    """Exp, its adjoint (staged and flat), the composition and its adjoint
    where every sample position is within a cell of the border and most are
    clamped."""
    log(f"minimal grid fields {shape}")
    K = 3
    phi = smooth_field(shape, 1.5, seed=sum(shape))
    G = smooth_field(shape, 1.0, seed=sum(shape) + 1, sigma=1.0)
    for sign in (1, -1):
        _, steps = ctx.exp(gpu(phi), K, sign, steps=True)
        us = O.exp_fwd(sign * phi.astype(np.float64), K)
        st = host(steps)
        for s in range(1, K + 1):
            assert np.abs(st[s - 1] - us[s]).max() < 1e-4, f"sign {sign} step {s}"
        want = sign * 2.0 ** -K * O.exp_bwd(us, G.astype(np.float64))
        for flat in (False, True):
            got = host(ctx.exp_bwd(gpu(phi), gpu(G), K, sign, "store", flat=flat))
            assert_grad_close(got, want)
    U = smooth_field(shape, 2.0, seed=sum(shape) + 2)
    C = smooth_field(shape, 1.5, seed=sum(shape) + 3)
    got = host(ctx.compose(gpu(U), gpu(C)))
    assert np.abs(got - O.compose(U.astype(np.float64), C.astype(np.float64))).max() < 1e-4
    gp = torch.zeros((3,) + shape, device=DEV)
    gc = torch.zeros((3,) + shape, device=DEV)
    ctx.compose_bwd(gpu(U), gpu(C), gpu(G), gp, gc)
    wp, wc = O.compose_bwd(U.astype(np.float64), C.astype(np.float64), G.astype(np.float64))
    assert_grad_close(host(gp), wp)
    assert_grad_close(host(gc), wc)


@pytest.mark.parametrize("shape,w", [((7, 7, 7), 7), ((5, 9, 12), 5), ((3, 3, 50), 3),
                                     ((7, 40, 9), 7)])
@pytest.mark.parametrize("metric", ["lncc", "silncc"])
def test_sim_on_minimal_grids_matches_oracle(ctx, shape, w, metric):
    """The similarity and its gradient on grids of one window edge: (7, 7, 7)
    has a single window centre, the others one row or one plane of them."""
    log(f"minimal grid sim {shape} w={w} {metric}")
    F = smooth_image(shape, seed=w + 11)
    I = smooth_image(shape, seed=w + 12)
    U = smooth_field(shape, 1.0, seed=w + 13)
    val, g = ctx.sim(gpu(F), gpu(I), gpu(U), w, metric, grad=True)
    m = O.LNCC if metric == "lncc" else O.SILNCC
    s_ref, g_ref = O.pair_sim_grad([F.astype(np.float64), I.astype(np.float64)],
                                   U.astype(np.float64), 0, 1, O.Params(window=w, metric=m))
    assert abs(val - s_ref) < 1e-3 * abs(s_ref)
    assert_grad_close(host(g), g_ref)


# ---------------------------------------------------------------------------
# Regulariser, Adam, pyramid
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(16, 16, 16), (21, 30, 47)])
def test_reg_matches_oracle(ctx, shape):
    phi = smooth_field(shape, 1.5, seed=9, sigma=1.5)
    val, g = ctx.reg(gpu(phi), grad=True)
    assert abs(val - O.reg_ss(phi.astype(np.float64))) < 1e-5 * O.reg_ss(phi.astype(np.float64))
    assert_grad_close(host(g), O.reg_ss_grad(phi.astype(np.float64)))


def test_adam_matches_oracle(ctx):
    r = rng(3)
    n = 10_001
    x0 = r.standard_normal(n).astype(np.float32)
    x, m, v = gpu(x0), torch.zeros(n, device=DEV), torch.zeros(n, device=DEV)
    xr, mr, vr = x0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 8):
        g = (r.standard_normal(n) * 1e-3).astype(np.float32)
        lr = O.lr_schedule(t, 7, 0.1)
        ctx.adam(x, gpu(g), m, v, t, lr)
        xr, mr, vr = O.adam_step(xr, g.astype(np.float64), mr, vr, t, lr)
    assert np.abs(host(x) - xr).max() < 1e-5


def test_pool2_and_upsample2_match_oracle(ctx):
    img = smooth_image((34, 40, 22), seed=4)
    got = host(ctx.pool2(gpu(img)))
    assert np.abs(got - O.pool2(img.astype(np.float64))).max() < 1e-6
    phi = smooth_field((9, 14, 11), 1.0, seed=5, sigma=1.5)
    got = host(ctx.upsample2(gpu(phi)))
    assert np.abs(got - O.upsample2(phi.astype(np.float64))).max() < 1e-5


# ---------------------------------------------------------------------------
# The whole loss and its gradient (Sec. 2.2 loss with Eq. reg_sum)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", [
    dict(shape=(32, 32, 32), N=3, K=7, w=5, metric="lncc"),
    dict(shape=(24, 30, 36), N=4, K=5, w=3, metric="silncc"),
    dict(shape=(20, 22, 40), N=5, K=4, w=7, metric="lncc"),
    dict(shape=(18, 18, 18), N=2, K=6, w=5, metric="silncc"),
])
@pytest.mark.parametrize("mode", ["store", "recompute"])
def test_loss_and_gradient_match_oracle(ctx, case, mode):
    from paper_2412_14671_amd import MusterLoss, MusterParams
    log(f"loss {case} {mode}")
    shape, N = case["shape"], case["N"]
    imgs = np.stack([smooth_image(shape, seed=10 + k) for k in range(N)])
    phis = np.stack([smooth_field(shape, 1.5, seed=20 + k) for k in range(N - 1)])
    svf = gpu(phis).requires_grad_(True)
    params = MusterParams(K=case["K"], window=case["w"], metric=case["metric"], alpha_ss=0.8,
                          exp_mode=mode)
    loss = MusterLoss.apply(svf, gpu(imgs), params, ctx)
    loss.backward()
    p = O.Params(K=case["K"], window=case["w"],
                 metric=O.LNCC if case["metric"] == "lncc" else O.SILNCC, alpha_ss=0.8)
    L_ref, g_ref, _ = O.loss_and_grad(list(phis.astype(np.float64)), list(imgs), p)
    assert abs(float(loss.detach()) - L_ref) < 1e-3 * abs(L_ref)
    assert_grad_close(host(svf.grad), np.stack(g_ref))


# ---------------------------------------------------------------------------
# Gaussian smoothing of the flow (Sec. 2.4, Appendix A)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,sigma", [((20, 27, 35), 0.375), ((20, 24, 20), 0.375),
                                         ((40, 48, 40), 0.5), ((40, 48, 40), 0.75),
                                         ((45, 37, 70), 1.0), ((32, 32, 32), 1.5),
                                         ((80, 96, 80), 1.5), ((9, 40, 23), 3.0),
                                         ((6, 7, 5), 2.0), ((33, 70, 129), 3.0)])
def test_smooth_matches_oracle(ctx, shape, sigma):
    """The smoothing kernel against Appendix A's Fourier-domain filter (the
    oracle's FFT), at every width a pyramid of the timed workloads uses (0.75,
    1.5 and 3; 0.375 with flows on a twice coarser grid) and below, on grids
    whose lines are odd and even, shorter and longer than the taps."""
    log(f"smooth {shape} sigma={sigma}")
    f = smooth_field(shape, 1.0, seed=int(10 * sigma) + shape[0], sigma=1.0)
    got = host(ctx.smooth(gpu(f), sigma))
    assert np.abs(got - O.smooth(f.astype(np.float64), sigma)).max() < 1e-6


@pytest.mark.parametrize("case", [
    dict(shape=(32, 32, 32), N=3, K=7, w=5, metric="lncc", sigma=1.0),
    dict(shape=(24, 30, 36), N=4, K=5, w=3, metric="silncc", sigma=2.0),
])
def test_loss_and_gradient_with_smoothing_match_oracle(ctx, case):
    from paper_2412_14671_amd import MusterLoss, MusterParams
    log(f"loss+smooth {case}")
    shape, N = case["shape"], case["N"]
    imgs = np.stack([smooth_image(shape, seed=30 + k) for k in range(N)])
    phis = np.stack([smooth_field(shape, 1.5, seed=40 + k, sigma=1.0) for k in range(N - 1)])
    svf = gpu(phis).requires_grad_(True)
    params = MusterParams(K=case["K"], window=case["w"], metric=case["metric"], alpha_ss=0.8,
                          smooth_sigma=case["sigma"])
    loss = MusterLoss.apply(svf, gpu(imgs), params, ctx)
    loss.backward()
    p = O.Params(K=case["K"], window=case["w"],
                 metric=O.LNCC if case["metric"] == "lncc" else O.SILNCC, alpha_ss=0.8,
                 smooth_sigma=case["sigma"])
    L_ref, g_ref, _ = O.loss_and_grad(list(phis.astype(np.float64)), list(imgs), p)
    assert abs(float(loss.detach()) - L_ref) < 1e-3 * abs(L_ref)
    assert_grad_close(host(svf.grad), np.stack(g_ref))


# ---------------------------------------------------------------------------
# Every tile shape and z chunk of the window statistics (the autotuner's
# candidates, plus chunks that leave ragged tails) against the oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape_id,zc", [(1, 32), (2, 16), (0, 5), (1, 7), (2, 64)])
@pytest.mark.parametrize("w,metric", [(3, "lncc"), (5, "silncc"), (7, "silncc")])
def test_sim_every_tiling_matches_oracle(ctx, shape_id, zc, w, metric):
    log(f"sim tiling shape={shape_id} zc={zc} w={w} {metric}")
    shape = (21, 26, 45) if shape_id != 2 else (40, 17, 70)
    F = smooth_image(shape, seed=w + 10)
    I = smooth_image(shape, seed=w + 11)
    U = smooth_field(shape, 2.0, seed=w + 12)
    ctx.set_tiling("fixed", shape_id, zc)
    try:
        val, g = ctx.sim(gpu(F), gpu(I), gpu(U), w, metric, grad=True)
    finally:
        ctx.set_tiling("autotune")
    p = O.Params(window=w, metric=O.LNCC if metric == "lncc" else O.SILNCC)
    s_ref, g_ref = O.pair_sim_grad([F.astype(np.float64), I.astype(np.float64)],
                                   U.astype(np.float64), 0, 1, p)
    assert abs(val - s_ref) < 1e-3 * abs(s_ref)
    assert_grad_close(host(g), g_ref)


# ---------------------------------------------------------------------------
# L_L2 and L_ts (Sec. 2.4, Eq. reg_ts, reg_sum) in the whole loss and gradient
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", [
    dict(shape=(24, 28, 20), N=4, K=6, w=5, metric="silncc", sigma=0.0, l2=0.4, ts=0.8,
         times=(0.0, 0.7, 2.1, 2.6)),
    dict(shape=(20, 22, 26), N=5, K=5, w=3, metric="lncc", sigma=1.2, l2=0.0, ts=1.5,
         times=(0.0, 1.0, 1.4, 3.0, 3.5)),
    dict(shape=(16, 18, 20), N=2, K=6, w=3, metric="silncc", sigma=0.0, l2=2.0, ts=1.0,
         times=(0.0, 1.3)),
])
def test_loss_and_gradient_with_l2_and_ts_match_oracle(ctx, case):
    from paper_2412_14671_amd import MusterLoss, MusterParams
    log(f"loss+l2/ts {case}")
    shape, N = case["shape"], case["N"]
    imgs = np.stack([smooth_image(shape, seed=60 + k) for k in range(N)])
    phis = np.stack([smooth_field(shape, 1.2, seed=70 + k, sigma=1.5) for k in range(N - 1)])
    svf = gpu(phis).requires_grad_(True)
    params = MusterParams(K=case["K"], window=case["w"], metric=case["metric"], alpha_ss=0.3,
                          smooth_sigma=case["sigma"], alpha_l2=case["l2"], alpha_ts=case["ts"])
    loss = MusterLoss.apply(svf, gpu(imgs), params, ctx, case["times"])
    loss.backward()
    p = O.Params(K=case["K"], window=case["w"],
                 metric=O.LNCC if case["metric"] == "lncc" else O.SILNCC, alpha_ss=0.3,
                 smooth_sigma=case["sigma"], alpha_l2=case["l2"], alpha_ts=case["ts"],
                 times=case["times"])
    L_ref, g_ref, aux = O.loss_and_grad(list(phis.astype(np.float64)), list(imgs), p)
    log(f"  loss {float(loss.detach()):.6f} oracle {L_ref:.6f} (reg part {aux['Lreg']:.6f})")
    assert abs(float(loss.detach()) - L_ref) < 1e-3 * abs(L_ref)
    assert_grad_close(host(svf.grad), np.stack(g_ref))


def test_loss_forward_needs_times_for_ts(ctx):
    from paper_2412_14671_amd import MusterLoss, MusterParams, MusterError
    shape = (12, 12, 12)
    imgs = gpu(np.stack([smooth_image(shape, seed=k) for k in range(3)]))
    svf = gpu(np.zeros((2, 3) + shape))
    with pytest.raises(MusterError):
        MusterLoss.apply(svf, imgs, MusterParams(K=4, window=3, alpha_ts=1.0), ctx)


def test_large_displacements_take_the_overflow_path_and_match_oracle(ctx):
    """Exp-backward blocks whose box of bins does not fit a staging slot fall
    back to atomics on the flat field and flag it; the next step adds it.  A
    rough field of amplitude 5 voxels makes many blocks do so."""
    from paper_2412_14671_amd import MusterLoss, MusterParams
    shape = (24, 32, 48)
    N = 3
    imgs = np.stack([smooth_image(shape, seed=90 + k) for k in range(N)])
    phis = np.stack([smooth_field(shape, 5.0, seed=95 + k, sigma=1.2) for k in range(N - 1)])
    for mode in ("store", "recompute"):
        svf = gpu(phis).requires_grad_(True)
        params = MusterParams(K=6, window=5, metric="silncc", alpha_ss=0.2, exp_mode=mode)
        loss = MusterLoss.apply(svf, gpu(imgs), params, ctx)
        loss.backward()
        p = O.Params(K=6, window=5, metric=O.SILNCC, alpha_ss=0.2)
        L_ref, g_ref, _ = O.loss_and_grad(list(phis.astype(np.float64)), list(imgs), p)
        assert abs(float(loss.detach()) - L_ref) < 1e-3 * abs(L_ref)
        assert_grad_close(host(svf.grad), np.stack(g_ref))


# ---------------------------------------------------------------------------
# Flow grid twice as coarse as the images (Sec. 2.7 stage geometry)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(5, 6, 7), (16, 12, 20), (2, 9, 33), (21, 26, 40)])
def test_upsample2_and_adjoint_match_oracle(ctx, shape):
    f = smooth_field(shape, 1.5, seed=sum(shape), sigma=1.0)
    g = smooth_field(tuple(2 * n for n in shape), 1.0, seed=sum(shape) + 1, sigma=1.0)
    up = host(ctx.upsample2(gpu(f)))
    assert np.abs(up - O.upsample2(f.astype(np.float64))).max() < 1e-5
    adj = host(ctx.upsample2_adjoint(gpu(g)))
    want = O.upsample2_adjoint(g.astype(np.float64), shape)
    assert np.abs(adj - want).max() < 1e-5 * max(1.0, np.abs(want).max())


@pytest.mark.parametrize("case", [
    dict(fshape=(12, 14, 16), N=3, K=6, w=5, metric="silncc", sigma=0.0),
    dict(fshape=(10, 12, 9), N=4, K=5, w=3, metric="lncc", sigma=1.0),
])
def test_loss_and_gradient_on_a_coarse_flow_grid_match_oracle(ctx, case):
    from paper_2412_14671_amd import MusterLoss, MusterParams
    log(f"loss coarse flow {case}")
    fshape, N = case["fshape"], case["N"]
    shape = tuple(2 * n for n in fshape)
    imgs = np.stack([smooth_image(shape, seed=110 + k) for k in range(N)])
    phis = np.stack([smooth_field(fshape, 1.0, seed=120 + k, sigma=1.2) for k in range(N - 1)])
    svf = gpu(phis).requires_grad_(True)
    params = MusterParams(K=case["K"], window=case["w"], metric=case["metric"], alpha_ss=0.5,
                          smooth_sigma=case["sigma"], flow_factor=2)
    loss = MusterLoss.apply(svf, gpu(imgs), params, ctx)
    loss.backward()
    p = O.Params(K=case["K"], window=case["w"],
                 metric=O.LNCC if case["metric"] == "lncc" else O.SILNCC, alpha_ss=0.5,
                 smooth_sigma=case["sigma"], flow_factor=2)
    L_ref, g_ref, _ = O.loss_and_grad(list(phis.astype(np.float64)), list(imgs), p)
    assert abs(float(loss.detach()) - L_ref) < 1e-3 * abs(L_ref)
    assert_grad_close(host(svf.grad), np.stack(g_ref))


# ---------------------------------------------------------------------------
# Outputs and evaluation (Sec. 2.8)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(17, 20, 23), (2, 5, 40)])
def test_jacobian_det_matches_oracle(ctx, shape):
    U = smooth_field(shape, 1.5, seed=400 + shape[0], sigma=1.5)
    got = host(ctx.jacobian_det(gpu(U)))
    assert np.abs(got - O.jacobian_det(U.astype(np.float64))).max() < 1e-5


@pytest.mark.parametrize("with_roi", [False, True])
def test_field_metrics_match_oracle(ctx, with_roi):
    shape = (24, 30, 36)
    a = smooth_field(shape, 1.0, seed=410, sigma=2.0)
    b = (0.8 * a + 0.3 * smooth_field(shape, 1.0, seed=411, sigma=2.0)).astype(np.float32)
    roi = (rng(412).uniform(size=shape) > 0.4) if with_roi else None
    eu_, pcc_, sl_ = ctx.field_metrics(gpu(a), gpu(b), None if roi is None else torch.from_numpy(roi))
    A, B = a.astype(np.float64), b.astype(np.float64)
    assert abs(eu_ - O.euclidean_error(A, B, roi)) < 1e-9
    assert abs(pcc_ - O.pcc(A, B, roi)) < 1e-9
    assert abs(sl_ - O.slope(A, B, roi)) < 1e-8


# ---------------------------------------------------------------------------
# Ownership of the autograd Function's saved state
# ---------------------------------------------------------------------------

def test_loss_state_is_freed(ctx):
    """loss_value keeps no state; an autograd forward whose input needs no
    gradient frees its saved state at once; a backward frees it after use.
    The context's arena returns to its size every time."""
    from paper_2412_14671_amd import MusterLoss, MusterParams, loss_value
    log("loss state ownership")
    shape, N = (20, 22, 24), 3
    imgs = gpu(np.stack([smooth_image(shape, seed=60 + k) for k in range(N)]))
    phis = gpu(np.stack([smooth_field(shape, 1.0, seed=70 + k) for k in range(N - 1)]))
    params = MusterParams(K=5, window=5, metric="lncc")
    # warm-up: tiling and the context's own item buffers
    svf = phis.clone().requires_grad_(True)
    MusterLoss.apply(svf, imgs, params, ctx).backward()
    torch.cuda.synchronize()
    base = ctx.memory()["in_use"]
    vals = [loss_value(phis, imgs, params, ctx) for _ in range(4)]
    assert ctx.memory()["in_use"] == base
    assert max(vals) - min(vals) <= 1e-12 * abs(vals[0])
    L = MusterLoss.apply(phis, imgs, params, ctx)  # no gradient needed
    assert ctx.memory()["in_use"] == base
    assert abs(float(L) - vals[0]) <= 1e-12 * abs(vals[0])
    svf = phis.clone().requires_grad_(True)
    L = MusterLoss.apply(svf, imgs, params, ctx)
    assert ctx.memory()["in_use"] > base  # the state the backward pass needs
    L.backward()
    assert ctx.memory()["in_use"] == base
    assert ctx.memory()["peak"] >= base
