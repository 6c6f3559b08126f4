"""Writes tests/golden/phantoms_4x64_fd.json: central finite differences of the
FP64 oracle's loss on the 64^3 gradient-check series (four phantom sessions,
K 6, window 7, alpha_ss 1), evaluated at half the ground-truth SVFs, at random
(interval, component, voxel) triples at least r + 2 voxels from the border:
256 triples per metric.  Steps h = 1e-3, 1e-4 and 1e-6 (the last resolves
the rare triples whose interval at 1e-4 crosses a cell face of the
trilinear interpolant, a kink of the loss); a run adds the differences of
one step to the file, for both metrics or the ones named.  Each difference
takes two whole-volume oracle evaluations, so the triples are spread over a
process pool.  Calls only the oracle and the seeded input generator.

    python tests/golden/make_phantoms_4x64_fd.py [h] [workers] [lncc] [silncc]
"""
import json
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import multiprocessing as mp  # noqa: E402

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import muster_oracle as O  # noqa: E402
from paper_2412_14671_amd import synth  # noqa: E402

K, W = 6, 7
H = 1e-3
COUNTS = {"lncc": 256, "silncc": 256}
SEEDS = {"lncc": 3, "silncc": 4}

_imgs = _phis = None


def problem():
    s = synth.phantoms_4x64()
    imgs = [x.numpy().astype(np.float64) for x in s.images]
    phis = [x.astype(np.float64) for x in (0.5 * s.svf_true).numpy().astype(np.float32)]
    return imgs, phis


def params(metric):
    return O.Params(K=K, window=W, metric=O.LNCC if metric == "lncc" else O.SILNCC, alpha_ss=1.0)


def triples(metric, shape, n_int):
    r = np.random.Generator(np.random.PCG64(SEEDS[metric]))
    lo = (W - 1) // 2 + 2
    out = []
    for _ in range(COUNTS[metric]):
        k = int(r.integers(0, n_int))
        c = int(r.integers(0, 3))
        z, y, x = (int(r.integers(lo, n - lo)) for n in shape)
        out.append((k, c, z, y, x))
    return out


def _fd(job):
    metric, h, (k, c, z, y, x) = job
    p = params(metric)
    vals = []
    for sgn in (1.0, -1.0):
        ph = [f.copy() for f in _phis]
        ph[k][c, z, y, x] += sgn * h
        vals.append(O.forward(ph, _imgs, p))
    return (vals[0] - vals[1]) / (2 * h)


def main():
    global _imgs, _phis
    h = float(sys.argv[1]) if len(sys.argv) > 1 else H
    workers = int(sys.argv[2]) if len(sys.argv) > 2 else 8
    metrics = sys.argv[3:] or ["lncc", "silncc"]
    _imgs, _phis = problem()
    shape = _imgs[0].shape
    path = os.path.join(HERE, "phantoms_4x64_fd.json")
    out = {"workload": "four 64^3 phantom sessions (seed 3), K 6, window 7, alpha_ss 1, "
                       "at half the ground-truth SVFs",
           "K": K, "window": W, "alpha_ss": 1.0}
    if os.path.exists(path):
        with open(path) as f:
            out.update(json.load(f))
    t0 = time.time()
    with mp.get_context("fork").Pool(workers) as pool:
        for metric in metrics:
            tr = triples(metric, shape, len(_phis))
            fd = pool.map(_fd, [(metric, h, t) for t in tr], chunksize=1)
            e = out.setdefault(metric, {})
            e["loss"] = O.forward(_phis, _imgs, params(metric))
            if e.get("triples") != [list(t) for t in tr]:
                e["fd"] = {}  # differences at other triples no longer apply
            e["triples"] = [list(t) for t in tr]
            e.setdefault("fd", {})[repr(h)] = fd
            print(f"{metric} h={h}: {len(tr)} differences, {time.time() - t0:.0f} s", flush=True)
            with open(path, "w") as f:
                json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
