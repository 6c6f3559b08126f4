"""Parity at the size the benchmark registers, 160x192x160 voxels, element by
element against the FP64 oracle: the integration (K 7) with every squaring
step, its adjoint, a composition and its adjoint, and one pair's warp, window
statistics and similarity gradient (SiLNCC, w 7).  Inputs are made like the
benchmark's: two phantom sessions and their interval's velocity field
(Gaussian-smoothed, sigma 6 voxels, up to 1.5 voxels), the pair field from
integrating it, and an upstream gradient smoothed at sigma 3.  The kernels run
in the configuration the benchmark times: 8x8x16-voxel tiles, the autotuned
window-statistics tiling of this shape, and for the Exp adjoint the staged
exchange of scatter boxes between squaring steps (flat in / staged out, then
staged in / staged out, then the staged G_0 unstaged), as well as the flat
path.  The oracle takes 2-40 s per step at this size.  Tolerances as in the
smaller parity tests: 1e-4 voxel per integration and composition, 1e-3
relative on values and gradients."""
import sys

import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

from oracle import muster_oracle as O

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
SHAPE = (160, 192, 160)
K = 7


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def assert_grad_close(got, want, tol=1e-3):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    rel = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)
    mx = np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)
    log(f"  rel L2 {rel:.2e}, max {mx:.2e}")
    assert rel < tol and mx < tol, f"rel L2 {rel:.2e}, max {mx:.2e}"


@pytest.fixture(scope="module")
def ctx():
    from paper_2412_14671_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def data():
    from paper_2412_14671_amd import synth
    log("full size: phantom sessions and velocity field")
    s = synth.phantom_series(SHAPE, 2, seed=61, device=DEV)
    imgs = s.images.cpu().numpy()
    phi = s.svf_true[0].cpu().numpy().astype(np.float32)
    r = np.random.Generator(np.random.PCG64(62))
    G = np.stack([ndi.gaussian_filter(r.standard_normal(SHAPE), 3.0, mode="wrap") for _ in range(3)])
    G = (G / np.abs(G).max()).astype(np.float32)
    log("full size: oracle integration")
    us = O.exp_fwd(phi.astype(np.float64), K)
    return {"imgs": imgs, "phi": phi, "G": G, "us": us}


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def test_exp_full_size(ctx, data):
    log("full size: exp K=7, every step")
    disp, steps = ctx.exp(gpu(data["phi"]), K, 1, steps=True)
    st = host(steps)
    for s in range(1, K + 1):
        err = np.abs(st[s - 1] - data["us"][s]).max()
        assert err < 1e-4, f"step {s}: {err}"
    assert np.array_equal(host(disp), st[K - 1])


def test_exp_bwd_full_size(ctx, data):
    log("full size: exp adjoint K=7, staged (store, recompute) and flat")
    want = 2.0 ** -K * O.exp_bwd(data["us"], data["G"].astype(np.float64))
    for mode, flat in (("store", False), ("recompute", False), ("store", True)):
        got = host(ctx.exp_bwd(gpu(data["phi"]), gpu(data["G"]), K, 1, mode, flat=flat))
        assert_grad_close(got, want)


def test_compose_and_adjoint_full_size(ctx, data):
    log("full size: composition and its adjoint")
    U = data["us"][K].astype(np.float32)
    C = (-1.5 * data["us"][K]).astype(np.float32)
    got = host(ctx.compose(gpu(U), gpu(C)))
    want = O.compose(U.astype(np.float64), C.astype(np.float64))
    assert np.abs(got - want).max() < 1e-4
    gp = torch.zeros((3,) + SHAPE, device=DEV)
    gc = torch.zeros((3,) + SHAPE, device=DEV)
    ctx.compose_bwd(gpu(U), gpu(C), gpu(data["G"]), gp, gc)
    wp, wc = O.compose_bwd(U.astype(np.float64), C.astype(np.float64), data["G"].astype(np.float64))
    assert_grad_close(host(gp), wp)
    assert_grad_close(host(gc), wc)


def test_similarity_and_gradient_full_size(ctx, data):
    log("full size: warp, window statistics and SiLNCC gradient of one pair, w 7")
    F, I = data["imgs"][0], data["imgs"][1]
    U = data["us"][K].astype(np.float32)
    val, g = ctx.sim(gpu(F), gpu(I), gpu(U), 7, "silncc", grad=True)
    p = O.Params(window=7, metric=O.SILNCC)
    s_ref, g_ref = O.pair_sim_grad([F.astype(np.float64), I.astype(np.float64)],
                                   U.astype(np.float64), 0, 1, p)
    log(f"  value {val:.9g} against {s_ref:.9g}")
    assert abs(val - s_ref) < 1e-3 * abs(s_ref)
    assert_grad_close(host(g), g_ref)
