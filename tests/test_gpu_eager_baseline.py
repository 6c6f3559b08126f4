"""The PyTorch-eager plain loop that bench.py times as a baseline computes the
same loss and gradient as the FP64 oracle (so the speed-up over it compares
like with like)."""
import numpy as np
import pytest
import torch

from oracle import muster_oracle as O

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("metric,sigma", [("silncc", 0.0), ("lncc", 1.0)])
def test_eager_loss_and_gradient_match_oracle(metric, sigma):
    import bench
    from paper_2412_14671_amd import synth
    s = synth.phantom_series((20, 24, 28), 3, seed=17)
    r = np.random.Generator(np.random.PCG64(5))
    phis = [0.5 * r.standard_normal((3, 20, 24, 28)) for _ in range(2)]
    phis = [O.smooth(p, 2.0).astype(np.float32) for p in phis]
    dev = torch.device("cuda:0")
    tp = [torch.from_numpy(p).to(dev).requires_grad_(True) for p in phis]
    L = bench.torch_loss(torch, tp, s.images.to(dev), K=6, window=5, metric=metric, alpha_ss=0.7,
                         smooth_sigma=sigma)
    L.backward()
    p = O.Params(K=6, window=5, metric=O.LNCC if metric == "lncc" else O.SILNCC, alpha_ss=0.7,
                 smooth_sigma=sigma)
    L_ref, g_ref, _ = O.loss_and_grad([x.astype(np.float64) for x in phis],
                                      list(s.images.numpy().astype(np.float64)), p)
    assert abs(float(L.detach()) - L_ref) < 1e-3 * abs(L_ref)
    g = np.stack([t.grad.cpu().numpy() for t in tp]).astype(np.float64)
    gr = np.stack(g_ref)
    assert np.linalg.norm(g - gr) / np.linalg.norm(gr) < 1e-2
