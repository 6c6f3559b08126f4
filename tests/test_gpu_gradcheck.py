"""Differentiation check on the 64^3 gradient-check workload: four phantom
sessions made as the 160x192x160 phantoms are (nested ellipsoids, per-session
bias, Rician noise, uneven intervals), K = 6 squarings, window 7, LNCC and
SiLNCC, evaluated at half the ground-truth SVFs.  The hand-written adjoints of
the warp, the compositions, scaling and squaring and the window statistics
(behind the autograd Function) are checked

* against central finite differences of the FP64 oracle's loss at 256
  random (interval, component, voxel) triples away from the border per
  metric, stored in tests/golden/phantoms_4x64_fd.json by
  tests/golden/make_phantoms_4x64_fd.py, with h = 1e-3, 1e-4 and 1e-6, under
  the bounds of the oracle's own pin (a difference that crosses a cell face
  of the trilinear interpolant, a kink of the loss, is off by up to about
  0.6 % of the largest entry at h = 1e-3; at h = 1e-4 such crossings are rare
  and h = 1e-6 resolves them), widened by the 1e-3 parity bar;
* against the FP64 oracle's gradient at every voxel (1e-3 relative);
* in both modes of the squaring steps: stored steps and steps recomputed from
  the SVF must give the same gradient, and recomputing must need less device
  memory.

The differences are those of the FP64 loss, not of the library's FP32 loss:
at h = 1e-3 the FP32 window moments (about 1e-5 absolute error per window
value, from the cancellation in S_FF/n - mean^2) leave differences of the
FP32 loss with errors of the size of the gradient entries themselves.
"""
import json
import os
import sys
import time

import numpy as np
import pytest
import torch

from oracle import muster_oracle as O
from test_oracle_pins import fd_check

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
K, W = 6, 7
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "phantoms_4x64_fd.json")) as _f:
    GOLDEN = json.load(_f)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2412_14671_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def series():
    from paper_2412_14671_amd import synth
    s = synth.phantoms_4x64()
    imgs = s.images.numpy()
    phis = (0.5 * s.svf_true).numpy().astype(np.float32)
    return imgs, phis


def params(metric, mode):
    from paper_2412_14671_amd import MusterParams
    return MusterParams(K=K, window=W, metric=metric, alpha_ss=1.0, exp_mode=mode)


def gpu_grad(ctx, imgs, phis, metric, mode):
    from paper_2412_14671_amd import MusterLoss
    svf = torch.from_numpy(phis).to(DEV).requires_grad_(True)
    img = torch.from_numpy(imgs).to(DEV)
    torch.cuda.synchronize()
    ctx.memory(reset_peak=True)
    base = ctx.memory()["in_use"]
    t0 = time.perf_counter()
    loss = MusterLoss.apply(svf, img, params(metric, mode), ctx)
    loss.backward()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    peak = ctx.memory()["peak"] - base
    return float(loss.detach()), svf.grad.detach().cpu().numpy().astype(np.float64), peak, dt


@pytest.mark.parametrize("metric", ["lncc", "silncc"])
def test_gradient_matches_oracle_finite_differences_and_both_step_modes(ctx, series, metric):
    imgs, phis = series
    N = imgs.shape[0]
    log(f"gradcheck 64^3 N={N} K={K} w={W} {metric}")

    gpu_grad(ctx, imgs, phis, metric, "store")  # warm-up (tiling, first launches)
    L_s, g_s, peak_s, t_s = gpu_grad(ctx, imgs, phis, metric, "store")
    L_r, g_r, peak_r, t_r = gpu_grad(ctx, imgs, phis, metric, "recompute")
    log(f"  store: loss {L_s:.9g}, peak workspace {peak_s / 2**20:.1f} MiB, {1e3 * t_s:.1f} ms")
    log(f"  recompute: loss {L_r:.9g}, peak workspace {peak_r / 2**20:.1f} MiB, {1e3 * t_r:.1f} ms")
    gmax = np.abs(g_s).max()
    assert abs(L_s - L_r) <= 1e-12 * abs(L_s)
    # same steps, same adjoint; only the order of float atomics may differ
    assert np.abs(g_s - g_r).max() <= 1e-5 * gmax
    assert peak_r < peak_s

    # against the FP64 oracle at every voxel
    p = O.Params(K=K, window=W, metric=O.LNCC if metric == "lncc" else O.SILNCC, alpha_ss=1.0)
    L_ref, g_ref, _ = O.loss_and_grad(list(phis.astype(np.float64)),
                                      list(imgs.astype(np.float64)), p)
    g_ref = np.stack(g_ref)
    log(f"  oracle: loss {L_ref:.9g}")
    assert abs(L_s - L_ref) < 1e-3 * abs(L_ref)
    scale = np.abs(g_ref).max()
    rel = np.linalg.norm(g_s - g_ref) / np.linalg.norm(g_ref)
    mx = np.abs(g_s - g_ref).max() / scale
    log(f"  gradient vs oracle: rel L2 {rel:.2e}, max {mx:.2e}")
    assert rel < 1e-3 and mx < 1e-3

    # central differences of the FP64 loss at the stored triples
    fdj = GOLDEN[metric]
    tr = [tuple(t) for t in fdj["triples"]]
    an = np.array([g_s[t] for t in tr])
    orc = np.array([g_ref[t] for t in tr])
    for h in ("0.001", "0.0001", "1e-06"):
        fd = np.array(fdj["fd"][h])
        err = np.abs(an - fd)
        rel_fd = np.linalg.norm(an - fd) / np.linalg.norm(fd)
        log(f"  central differences, h = {h}, at {len(tr)} triples: max |g - fd| "
            f"{err.max() / gmax:.2e} of max|g|, rel L2 {rel_fd:.2e}; oracle gradient: "
            f"{np.abs(orc - fd).max() / gmax:.2e}, {np.linalg.norm(orc - fd) / np.linalg.norm(fd):.2e}")
    assert fd_check(an, fdj["fd"], gmax, extra=1e-3)
