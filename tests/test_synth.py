"""Sanity of the seeded generators: shapes, ranges, determinism, and that the
generator's ground truth is the deformation the oracle's loss prefers."""
import numpy as np
import pytest
import torch

from oracle import muster_oracle as O
from paper_2412_14671_amd import synth


def test_generators_are_deterministic_and_shaped():
    a = synth.blobs_3x32()
    b = synth.blobs_3x32()
    assert torch.equal(a.images, b.images)
    assert a.images.shape == (3, 32, 32, 32) and a.images.dtype == torch.float32
    assert a.svf_true.shape == (2, 3, 32, 32, 32)
    mx = torch.sqrt((a.svf_true ** 2).sum(1)).amax()
    assert abs(float(mx) - 1.0) < 1e-5
    p = synth.phantom_series((32, 32, 32), 4, seed=7)
    assert p.images.shape == (4, 32, 32, 32)
    assert np.all(np.diff(p.times) >= 0.5) and np.all(np.diff(p.times) <= 2.0)
    assert 0.0 <= float(p.images.min()) and float(p.images.max()) < 1.3
    assert p.roi.any()


@pytest.mark.parametrize("maker,metric,w", [(synth.blobs_3x32, O.LNCC, 5),
                                            (lambda: synth.phantom_series((32, 32, 32), 3, seed=5),
                                             O.SILNCC, 5)])
def test_ground_truth_lowers_the_similarity(maker, metric, w):
    s = maker()
    imgs = [x.double().numpy() for x in s.images]
    p = O.Params(K=7, window=w, metric=metric, alpha_ss=0.0)
    zero = [np.zeros_like(x.double().numpy()) for x in s.svf_true]
    true = [x.double().numpy() for x in s.svf_true]
    assert O.forward(true, imgs, p) < O.forward(zero, imgs, p)
    flipped = [-x for x in true]
    assert O.forward(true, imgs, p) < O.forward(flipped, imgs, p)
