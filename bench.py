"""Benchmark of the MUSTER registration path on one MI355X.

Default workload: one subject of six 160x192x160 phantom sessions registered
over a three-level pyramid (40x48x40, 80x96x80, 160x192x160; 200/100/50 Adam
steps), SiLNCC with a 7^3 window, K = 7 squarings, alpha_ss = 0.1 and a
Gaussian smoothing of the flow with sigma 3 finest-level voxels.  A step is
one complete registration (every step of the path at every level).  The metric counts
session-voxel-iterations: sum over levels of N * V_level * steps_level,
divided by the wall time of a step, with the input series already resident in
device memory.

Other workloads (--workload): "batch" (16 subjects of uneven size and session
count, 100 steps at the finest level, batched graph-replayed loop against the
per-subject plain loop) and "serve" (Poisson arrivals into the
continuous-batching server; p50/p99 latency).

The JSON line carries the roofline of the dominant kernel (algorithmic bytes
over its HIP-event-timed duration inside the timed region) and the FP64 oracle
timed on host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="register", choices=["register", "batch", "serve"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="replay captured graphs in the timed region (no per-kernel timing)")
    ap.add_argument("--traffic", default=None,
                    help="JSON with HBM traffic per launch of the dominant kernel from rocprofv3 counters")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (for counter calibration)")
    ap.add_argument("--shape", default="160,192,160")
    ap.add_argument("--sessions", type=int, default=6)
    ap.add_argument("--iters", default="200,100,50")
    ap.add_argument("--alpha", type=float, default=0.1, help="alpha_ss")
    ap.add_argument("--smooth", type=float, default=3.0,
                    help="Gaussian smoothing width of the flow, finest-level voxels")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=2.0)
    ap.add_argument("--batch-subjects", type=int, default=16)
    ap.add_argument("--batch-iters", type=int, default=100)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def eu(svf_true, svf, roi):
    d = np.sqrt(((svf_true.astype(np.float64) - svf.astype(np.float64)) ** 2).sum(1))
    return float(d[:, roi].mean())


def cpu_baseline_register(series, params_np, level_shape):
    """The FP64 oracle, as it stands, on a bounded sample: one Adam step
    (loss, hand-written gradient, update) of the same subject at the coarsest
    pyramid level."""
    from oracle import muster_oracle as O
    imgs = [x.astype(np.float64) for x in series]
    f = series.shape[1] // level_shape[0]
    while f > 1:
        imgs = [O.pool2(x) for x in imgs]
        f //= 2
    N = len(imgs)
    phis = [np.zeros((3,) + imgs[0].shape) for _ in range(N - 1)]
    m = [np.zeros_like(x) for x in phis]
    v = [np.zeros_like(x) for x in phis]
    t0 = time.perf_counter()
    _, grads, _ = O.loss_and_grad(phis, imgs, params_np)
    for k in range(N - 1):
        phis[k], m[k], v[k] = O.adam_step(phis[k], grads[k], m[k], v[k], 1, params_np.lr)
    dt = time.perf_counter() - t0
    V = int(np.prod(imgs[0].shape))
    return {"value": N * V / dt, "unit": "session-voxel-iterations/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"one Adam step of the same {N}-session subject at the coarsest level "
                       f"{tuple(imgs[0].shape)} (NumPy float64, single-threaded), {dt:.1f} s")}


def roofline_from_stats(stats, traffic=None):
    best = max(stats.items(), key=lambda kv: kv[1]["ms"])
    name, st = best
    if st["launches"] == 0 or st["ms"] <= 0:
        return name, None
    achieved = st["bytes"] / (st["ms"] * 1e-3) / 1e9
    tr = None
    if traffic and traffic.get("kernel") == name:
        tr = traffic.get("bytes_per_launch")
    return name, {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
                  "kernel": name, "launches": st["launches"],
                  "avg_ms": round(st["ms"] / st["launches"], 4),
                  "bytes_per_launch": round(st["bytes"] / st["launches"])}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2412_14671_amd import Context, MusterParams, synth
    from paper_2412_14671_amd import _lib
    _lib.load()  # fail loudly if the HIP library is missing
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    ctx = Context(0)
    if args.workload == "register":
        out = bench_register(args, ctx, dev, torch, synth, MusterParams)
    elif args.workload == "batch":
        out = bench_batch(args, ctx, dev, torch, synth, MusterParams)
    else:
        out = bench_serve(args, ctx, dev, torch, synth, MusterParams)
    if args.copy_calibration:
        a = torch.empty(64 * 1024 * 1024, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_register(args, ctx, dev, torch, synth, MusterParams):
    shape = tuple(int(x) for x in args.shape.split(","))
    iters = [int(x) for x in args.iters.split(",")]
    N = args.sessions
    log(f"generating {N} sessions of {shape}")
    s = synth.phantom_series(shape, N, seed=2, device=dev)
    images = s.images.contiguous()
    params = MusterParams(iters=iters, K=7, window=7, metric="silncc", alpha_ss=args.alpha, lr=0.1,
                          smooth_sigma=args.smooth, use_graph=args.graph)
    L = len(iters)
    vox_iters = sum(N * np.prod([d // 2 ** (L - 1 - l) for d in shape]) * iters[l]
                    for l in range(L))
    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        svf, _, rep = ctx.register(images, s.times, params)
    torch.cuda.synchronize()
    ctx.set_kernel_timing(not args.graph)
    ctx.kernel_stats_reset()
    log(f"timed {args.steps}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        svf, _, rep = ctx.register(images, s.times, params)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.set_kernel_timing(False)
    stats = ctx.kernel_stats()
    ms = dt / args.steps * 1e3
    value = vox_iters / (dt / args.steps)
    roi = s.roi.cpu().numpy()
    svf_np = svf.cpu().numpy()
    true_np = s.svf_true.cpu().numpy()
    traffic = json.load(open(args.traffic)) if args.traffic else None
    kname, roof = roofline_from_stats(stats, traffic)
    out = {
        "metric": "voxel-iterations/sec (fwd+bwd)",
        "value": round(float(value), 1),
        "unit": "session-voxel-iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"one subject, {N} phantom sessions {shape[0]}x{shape[1]}x{shape[2]}, "
                                f"{L}-level pyramid {'/'.join(map(str, iters))} steps, "
                                f"SiLNCC w7, K7, alpha_ss {args.alpha:g}, smoothing sigma {args.smooth:g}"),
                   "sessions": N, "dims": list(shape), "levels": L, "iters": iters,
                   "graphs": bool(args.graph)},
        "roofline": roof,
        "cpu_baseline": None,
        "eu_voxels": round(eu(true_np, svf_np, roi), 4),
        "eu_at_zero": round(eu(true_np, np.zeros_like(svf_np), roi), 4),
        "loss_first": rep["loss_first"], "loss_last": rep["loss_last"],
        "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                        "GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None}
                    for k, v in stats.items() if v["launches"]},
    }
    if not args.no_cpu_baseline:
        from oracle import muster_oracle as O
        log("cpu baseline (oracle)")
        coarse = tuple(d // 2 ** (L - 1) for d in shape)
        p = O.Params(K=7, window=7, metric=O.SILNCC, alpha_ss=args.alpha, lr=0.1,
                     smooth_sigma=args.smooth / 2 ** (L - 1))
        out["cpu_baseline"] = cpu_baseline_register(s.images.cpu().numpy(), p, coarse)
    return out


def bench_batch(args, ctx, dev, torch, synth, MusterParams):
    subjects = []
    for k in range(args.batch_subjects):
        N, shape = synth.subject_draw(100 + k)
        log(f"subject {k}: N={N} {shape}")
        subjects.append(synth.batch_subject(100 + k, device=dev))
    params_b = MusterParams(iters=[args.batch_iters], K=7, window=7, metric="silncc", lr=0.1,
                            alpha_ss=args.alpha, smooth_sigma=args.smooth, use_graph=True)
    params_p = MusterParams(iters=[args.batch_iters], K=7, window=7, metric="silncc", lr=0.1,
                            alpha_ss=args.alpha, smooth_sigma=args.smooth, use_graph=False)
    vox = sum(s.images.shape[0] * s.images[0].numel() for s in subjects) * args.batch_iters
    imgs = [s.images for s in subjects]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs, reps = ctx.register_batch(imgs, [s.times for s in subjects], params_b)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    plain = []
    for s in subjects:
        svf, _, _ = ctx.register(s.images, s.times, params_p)
        plain.append(svf)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    eu_b = [eu(s.svf_true.cpu().numpy(), o.cpu().numpy(), s.roi.cpu().numpy()) for s, o in zip(subjects, outs)]
    eu_p = [eu(s.svf_true.cpu().numpy(), o.cpu().numpy(), s.roi.cpu().numpy()) for s, o in zip(subjects, plain)]
    return {"metric": "voxel-iterations/sec (fwd+bwd) batched vs plain loop",
            "value": round(vox / tb, 1), "unit": "session-voxel-iterations/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": round(tb * 1e3, 1), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{len(subjects)} subjects, N in 3..10, sizes from 96^3/128^3/160x192x160, "
                                   f"{args.batch_iters} steps at the finest level, SiLNCC w7, K7"},
            "plain_loop_value": round(vox / tp, 1), "batched_over_plain": round(tp / tb, 3),
            "eu_batched": [round(x, 4) for x in eu_b], "eu_plain": [round(x, 4) for x in eu_p]}


def bench_serve(args, ctx, dev, torch, synth, MusterParams):
    from paper_2412_14671_amd import Server
    rng = np.random.Generator(np.random.PCG64(5))
    pool = []
    for k in range(12):
        N, shape = synth.subject_draw(500 + k)
        pool.append(synth.batch_subject(500 + k, device=dev))
    params = MusterParams(iters=[200, 100, 50], K=7, window=7, metric="silncc", lr=0.1,
                          alpha_ss=args.alpha, smooth_sigma=args.smooth)
    srv = Server(ctx)
    arrivals = []
    t = 0.0
    while t < args.serve_seconds:
        t += rng.exponential(1.0 / args.serve_rate)
        arrivals.append((t, int(rng.integers(0, len(pool)))))
    t0 = time.perf_counter()
    tickets = []
    for at, k in arrivals:
        now = time.perf_counter() - t0
        if at > now:
            time.sleep(at - now)
        s = pool[k]
        tk, out = srv.submit(s.images, s.times, params)
        tickets.append((tk, k, out))
    reps = [srv.wait(tk) for tk, _, _ in tickets]
    wall = time.perf_counter() - t0
    lat = np.array([r["seconds"] for r in reps])
    vox = sum(pool[k].images.shape[0] * sum(pool[k].images[0].numel() // 8 ** (2 - l) * it
                                            for l, it in enumerate([200, 100, 50]))
              for _, k, _ in tickets)
    return {"metric": "voxel-iterations/sec (fwd+bwd); p50/p99 job latency",
            "value": round(vox / wall, 1), "unit": "session-voxel-iterations/s", "n_gpus": 1,
            "steps": len(tickets), "warmup": 0, "ms_per_step": round(wall / len(tickets) * 1e3, 1),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"Poisson arrivals {args.serve_rate}/s for {args.serve_seconds}s, "
                                   "N in 3..10, sizes from 96^3/128^3/160x192x160, pyramid 200/100/50"},
            "jobs_per_s": round(len(tickets) / wall, 3), "p50_s": round(float(np.percentile(lat, 50)), 3),
            "p99_s": round(float(np.percentile(lat, 99)), 3),
            "failed": int(sum(r["status"] != 0 for r in reps))}


if __name__ == "__main__":
    main()
