"""Writes tests/golden/blobs_3x32_oracle.json: the FP64 oracle's end-to-end
registration of the 3-session 32^3 blob series (50 Adam steps, K 7, LNCC w5,
alpha_ss 1, lr 0.1, one level) -- its loss trajectory and final Euclidean
error against the generator's ground truth.  Calls only the oracle and the
seeded input generator."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import muster_oracle as O  # noqa: E402
from paper_2412_14671_amd import synth  # noqa: E402


def main():
    s = synth.blobs_3x32()
    imgs = [x.numpy() for x in s.images]
    p = O.Params(K=7, window=5, metric=O.LNCC, alpha_ss=1.0, lr=0.1, iters=(50,))
    phis, U, hist = O.register(imgs, p)
    roi = s.roi.numpy()
    true = s.svf_true.numpy().astype(np.float64)
    eu = float(np.mean([O.euclidean_error(true[k], phis[k], roi) for k in range(2)]))
    eu0 = float(np.mean([O.euclidean_error(true[k], np.zeros_like(phis[k]), roi) for k in range(2)]))
    out = {"workload": "3 sessions of 32^3 blobs, 50 steps, K7, LNCC w5, alpha_ss 1, lr 0.1",
           "loss": hist, "eu_final": eu, "eu_zero": eu0}
    with open(os.path.join(HERE, "blobs_3x32_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({"eu_final": eu, "eu_zero": eu0, "loss0": hist[0], "lossT": hist[-1]}))


if __name__ == "__main__":
    main()
