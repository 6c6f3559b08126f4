"""The allocation-free entry point muster_sim_noalloc, called through the C
ABI, against muster_sim on the same inputs: the similarity value within
1e-3 relative and the gradient within 1e-3 (relative L2, and maximum error
within 1e-3 of the largest magnitude), on two calls in a row, the second on
a smaller grid (the scratch keeps the first call's contents, which the
second must not see).  A grid beyond the scratch's limit is refused with
E_INVALID before any launch."""
import sys
from ctypes import byref, c_double, c_void_p

import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _inputs(shape, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    imgs = []
    for _ in range(2):
        x = ndi.gaussian_filter(r.uniform(0, 1, shape), 2.0, mode="wrap")
        x = (x - x.min()) / (x.max() - x.min()) + 0.02 * r.standard_normal(shape)
        imgs.append(torch.from_numpy(x.astype(np.float32)).to(DEV))
    U = np.stack([ndi.gaussian_filter(r.standard_normal(shape), 3.0, mode="wrap") for _ in range(3)])
    U = torch.from_numpy((1.5 * U / np.abs(U).max()).astype(np.float32)).to(DEV)
    return imgs[0], imgs[1], U


def _close(got, want, tol=1e-3):
    got = got.double().cpu().numpy()
    want = want.double().cpu().numpy()
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    mx = np.abs(got - want).max() / np.abs(want).max()
    log(f"  gradient: rel L2 {rel:.2e}, max {mx:.2e}")
    assert rel < tol and mx < tol


def test_sim_noalloc_matches_sim_on_two_calls_in_a_row():
    from paper_2412_14671_amd import Context
    from paper_2412_14671_amd import _lib as L
    ctx = Context(0)
    try:
        for shape, w, metric, seed in [((48, 56, 40), 7, "silncc", 1), ((20, 26, 33), 5, "lncc", 2)]:
            log(f"sim_noalloc {shape} w{w} {metric}")
            F, I, U = _inputs(shape, seed)
            v_ref, g_ref = ctx.sim(F, I, U, w, metric, grad=True)
            v, g = ctx.sim_noalloc(F, I, U, w, metric, grad=True)
            log(f"  value {v:.9g} against {v_ref:.9g}")
            assert abs(v - v_ref) < 1e-3 * abs(v_ref)
            _close(g, g_ref)
            v2 = ctx.sim_noalloc(F, I, U, w, metric, grad=False)
            assert abs(v2 - v_ref) < 1e-3 * abs(v_ref)
        # beyond the scratch: refused before any launch
        F, I, U = _inputs((8, 8, 8), 3)
        m = L.METRIC_LNCC
        val = c_double()
        st = ctx.lib.muster_sim_noalloc(ctx.h, c_void_p(torch.cuda.current_stream().cuda_stream),
                                        L.DIMS(256, 256, 128), 5, m, c_void_p(F.data_ptr()),
                                        c_void_p(I.data_ptr()), c_void_p(U.data_ptr()),
                                        byref(val), None)
        assert st == L.E_INVALID
        assert b"exceed" in ctx.lib.muster_last_error()
    finally:
        ctx.close()
