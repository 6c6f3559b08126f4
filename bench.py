"""Benchmark of the MUSTER registration path on one MI355X.

Default workload ("headline"): the batched form of the path against a plain
per-subject loop, and the serving form's latency.
  * Sixteen subjects (seeds 100..115), each with a session count drawn from
    3..10 and a volume size from 96^3 / 128^3 / 160x192x160 (brain-like
    phantoms with per-session bias, Rician noise and per-interval velocity
    fields), registered at the finest level from phi = 0: SiLNCC w7, K = 7,
    alpha_ss = 1, no smoothing, lr 0.1.
  * A step is one iteration of every subject (forward, adjoint and Adam step
    of all sixteen, as one batched launch sequence).  W untimed steps, then K
    timed ones; value = session-voxel-iterations per second over the timed
    steps (sum of N_s * V_s per step).  The K steps are timed by the library
    between the stream synchronisations it places around them (the call that
    runs them also creates the jobs and writes their outputs: timed_call_s).
    The timed steps launch eagerly with HIP events on the dominant kernel's
    launches (for the roofline).
  * Then the whole 100-step schedule: batched (one launch sequence for all
    subjects, each step replayed from a captured hipGraph, autotuned tiles)
    against the plain loop (the same subjects one after another, the same
    kernels launched eagerly, default tiles); batched_over_plain and the
    final registration error Eu of every subject under both.
  * Serving: Poisson arrivals at 2 requests/s for 30 s into the continuous
    batching server, each request one of the sixteen subjects on the
    three-level pyramid 200/100/50; jobs/s and p50/p99 latency.
  * Extra keys: the single-subject registration of six 160x192x160 sessions
    (three levels, 200/100/50 steps).

The inputs are resident in device memory before any timed region starts.
The JSON line carries the roofline of the dominant kernel (algorithmic bytes
over its HIP-event-timed duration inside the timed region) and the FP64
oracle timed on host cores on a bounded sample of the same workload.

Other workloads (--workload): "register" (the single subject alone, a step
being one whole registration), "batch", "serve" and "blobs" (three 32^3
sessions; launch-bound).
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
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "register", "batch", "serve", "blobs"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="replay captured graphs in the timed region (no per-kernel timing)")
    ap.add_argument("--no-kernel-table", dest="kernel_table", action="store_false",
                    help="skip the extra registration that times every kernel class")
    ap.add_argument("--graph-steps", type=int, default=1,
                    help="registrations replayed from captured graphs after the timed region")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "batch16_traffic.txt"),
                    help="JSON summary of rocprofv3 FETCH_SIZE/WRITE_SIZE passes (per kernel class "
                         "and grid size); used only if it matches the current kernels")
    ap.add_argument("--l2hit", default=os.path.join(ROOT, "profiles", "batch16_l2_hit.txt"),
                    help="committed L2 hit-rate summary (TCC_HIT / TCC_MISS per kernel and grid)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a kernel that reads and writes 256 MiB once (counter calibration)")
    ap.add_argument("--shape", default="160,192,160")
    ap.add_argument("--sessions", type=int, default=6)
    ap.add_argument("--iters", default="200,100,50")
    ap.add_argument("--alpha", type=float, default=0.1,
                    help="alpha_ss of the single-subject registration (the headline uses 1)")
    ap.add_argument("--window", type=int, default=7, help="window edge w (3, 5 or 7)")
    ap.add_argument("--metric", default="silncc", choices=["silncc", "lncc"])
    ap.add_argument("--smooth", type=float, default=3.0,
                    help="Gaussian smoothing width of the flow, finest-level flow-grid voxels")
    ap.add_argument("--flow-factor", type=int, default=1,
                    help="2: flows on a grid twice as coarse as the images")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-rate", type=float, default=2.0)
    ap.add_argument("--batch-subjects", type=int, default=16)
    ap.add_argument("--batch-iters", type=int, default=100)
    ap.add_argument("--no-serve", action="store_true", help="headline: skip the serving run")
    ap.add_argument("--no-register", action="store_true",
                    help="headline: skip the single-subject registration (extra keys)")
    ap.add_argument("--no-full", action="store_true",
                    help="headline: skip the 100-step batched and plain runs")
    ap.add_argument("--batch-sizes", default="",
                    help="edge lengths of cubic subjects to draw from (e.g. 32,48,64) instead of "
                         "96^3/128^3/160x192x160")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def eu(svf_true, svf, roi):
    d = np.sqrt(((svf_true.astype(np.float64) - svf.astype(np.float64)) ** 2).sum(1))
    return float(d[:, roi].mean())


def cpu_baseline_register(series, params_np, level_shape):
    """The FP64 oracle, as it stands, on a bounded sample: Adam steps (loss,
    hand-written gradient, update) of the same subject at the coarsest
    pyramid level, as many as start within the first 10 s (at most 8)."""
    from oracle import muster_oracle as O
    imgs = [x.astype(np.float64) for x in series]
    f = series.shape[1] // level_shape[0]
    while f > 1:
        imgs = [O.pool2(x) for x in imgs]
        f //= 2
    N = len(imgs)
    ff = getattr(params_np, "flow_factor", 1)
    phis = [np.zeros((3,) + tuple(n // ff for n in imgs[0].shape)) for _ in range(N - 1)]
    m = [np.zeros_like(x) for x in phis]
    v = [np.zeros_like(x) for x in phis]
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):  # one core, BLAS included
        t0 = time.perf_counter()
        steps = 0
        while steps < 8 and (steps == 0 or time.perf_counter() - t0 < 10.0):
            steps += 1
            _, grads, _ = O.loss_and_grad(phis, imgs, params_np)
            for k in range(N - 1):
                phis[k], m[k], v[k] = O.adam_step(phis[k], grads[k], m[k], v[k], steps,
                                                  params_np.lr)
        dt = time.perf_counter() - t0
    V = int(np.prod(imgs[0].shape))
    return {"value": N * V * steps / dt, "unit": "session-voxel-iterations/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"{steps} Adam step{'s' if steps > 1 else ''} of the same {N}-session subject at the coarsest "
                       f"level {tuple(imgs[0].shape)} (NumPy float64, single-threaded), "
                       f"{dt:.1f} s")}


# ---------------------------------------------------------------------------
# Plain per-subject loop in PyTorch eager ops with autograd: the same loss
# (border-clamped trilinear sampling, scaling and squaring, outward
# composition, valid-window ML moments, SiLNCC/LNCC, diffusion regulariser,
# circular Gaussian smoothing) and the same Adam schedule, one op at a time,
# as the method is written in a tensor framework.  A baseline for the batched
# path only; nothing in the library uses it.
# ---------------------------------------------------------------------------

def _torch_sample(torch, f, q):
    """Border-clamped trilinear sample of f (C, D, H, W) at voxel positions
    q (3, D', H', W') through grid_sample (align_corners, border padding)."""
    C, D, H, W = f.shape
    g = torch.stack([2 * q[2] / (W - 1) - 1, 2 * q[1] / (H - 1) - 1, 2 * q[0] / (D - 1) - 1], -1)
    return torch.nn.functional.grid_sample(f[None], g[None], mode="bilinear",
                                           padding_mode="border", align_corners=True)[0]


def _torch_smooth(torch, phi, sigma):
    """Appendix A's filter through torch's FFT: the spectrum of each component
    times exp(-sigma^2 |omega|^2 / 2), omega in radians per voxel."""
    if sigma <= 0:
        return phi
    D, H, W = phi.shape[1:]
    dev = phi.device
    om = [2 * math.pi * torch.fft.fftfreq(n, device=dev, dtype=torch.float64) for n in (D, H)]
    omx = 2 * math.pi * torch.fft.rfftfreq(W, device=dev, dtype=torch.float64)
    w2 = om[0][:, None, None] ** 2 + om[1][None, :, None] ** 2 + omx[None, None, :] ** 2
    tf = torch.exp(-0.5 * sigma ** 2 * w2).to(phi.dtype)
    spec = torch.fft.rfftn(phi, dim=(1, 2, 3))
    return torch.fft.irfftn(spec * tf, s=(D, H, W), dim=(1, 2, 3))


def torch_loss(torch, phis, images, K=7, window=7, metric="silncc", alpha_ss=1.0,
               smooth_sigma=0.0):
    """L(phi) for the list of (3, D, H, W) flows and (N, D, H, W) images."""
    N = images.shape[0]
    D, H, W = images.shape[1:]
    dev = images.device
    grid = torch.stack(torch.meshgrid(*[torch.arange(n, device=dev, dtype=torch.float32)
                                        for n in (D, H, W)], indexing="ij"))
    flows = [_torch_smooth(torch, ph, smooth_sigma) for ph in phis]

    def expo(v):
        u = v / 2.0 ** K
        for _ in range(K):
            u = u + _torch_sample(torch, u, grid + u)
        return u

    f = [expo(v) for v in flows]
    b = [expo(-v) for v in flows]
    pool = torch.nn.functional.avg_pool3d
    loss = 0.0
    for i in range(N):
        U = None
        for j in range(i + 1, N):
            U = f[j - 1] if U is None else U + _torch_sample(torch, f[j - 1], grid + U)
            loss = loss + _torch_sim(torch, pool, images[i], images[j], U, grid, window, metric)
        U = None
        for j in range(i - 1, -1, -1):
            U = b[j] if U is None else U + _torch_sample(torch, b[j], grid + U)
            loss = loss + _torch_sim(torch, pool, images[i], images[j], U, grid, window, metric)
    reg = 0.0
    for ph in flows:
        for d in range(3):
            reg = reg + (torch.diff(ph, dim=1 + d) ** 2).mean(dim=(1, 2, 3)).sum()
    return loss + alpha_ss * reg / (N - 1)


def _torch_sim(torch, pool, Fi, Ij, U, grid, w, metric):
    M = _torch_sample(torch, Ij[None], grid + U)[0]
    F = Fi
    st = [pool(x[None, None], w, stride=1)[0, 0] for x in (F, M, F * F, M * M, F * M)]
    mF, mM = st[0], st[1]
    vF = torch.clamp(st[2] - mF * mF, min=0.0)
    vM = torch.clamp(st[3] - mM * mM, min=0.0)
    c = st[4] - mF * mM
    if metric == "lncc":
        ell = 1.0 - c / torch.sqrt(torch.clamp(vF * vM, min=1e-10))
    else:
        ell = vM - c * c / torch.clamp(vF, min=1e-6)
    return ell.mean()


def torch_register(torch, images, iters, lr=0.1, warmup=0.2, timed_iters=None, **kw):
    """Single-level Adam loop on torch_loss; returns (phis, seconds per iteration)."""
    N = images.shape[0]
    phis = [torch.zeros((3,) + tuple(images.shape[1:]), device=images.device, requires_grad=True)
            for _ in range(N - 1)]
    opt = torch.optim.Adam(phis, lr=lr, betas=(0.9, 0.999), eps=1e-8)
    T = iters
    Wu = max(1, math.ceil(warmup * T))
    n = T if timed_iters is None else min(T, timed_iters)
    t0 = None
    for t in range(1, n + 1):
        if t == 2:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        lr_t = lr * t / Wu if t <= Wu else lr * 0.5 * (1 + math.cos(math.pi * (t - Wu) / (T - Wu)))
        for g in opt.param_groups:
            g["lr"] = lr_t
        opt.zero_grad(set_to_none=True)
        L = torch_loss(torch, phis, images, **kw)
        L.backward()
        opt.step()
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / max(1, n - 1) if t0 is not None else float("nan")
    return [p.detach() for p in phis], per


def kernels_sha256():
    """SHA-256 of the kernel source and the header of its tile and bin
    constants: the counter summaries hold only while both are unchanged."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "muster_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2412_14671_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def traffic_per_launch(path, kernel, launch_grids):
    """HBM bytes per launch of `kernel` (e.g. "k_exp_bwd") from the committed
    counter summary, weighted like the timed launches ({grid in blocks:
    launches}); None if the summary is absent, lacks that kernel or grid, has
    no calibration, or predates the current kernels."""
    if not path or not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("kernels_sha256") != kernels_sha256() or not t.get("calibration"):
        return None
    per = t.get("kernels", {}).get(kernel, {}).get("per_grid", {})
    ff, wf = t["calibration"]["fetch_factor"], t["calibration"]["write_factor"]
    tot = n = 0
    for grid, launches in launch_grids.items():
        e = per.get(str(grid))
        if e is None:
            return None
        tot += launches * (e["fetch_kib"] * ff + e["write_kib"] * wf) * 1024.0
        n += launches
    return round(tot / n) if n else None


def l2_hit_per_launch(path, kernel, launch_grids):
    """L2 hit rate of `kernel` from the committed TCC_HIT / TCC_MISS summary,
    over the timed launch mix ({grid in blocks: launches}); None if the
    summary is absent or predates the current kernels."""
    if not path or not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("kernels_sha256") != kernels_sha256():
        return None
    per = t.get("kernels", {}).get(kernel, {}).get("per_grid", {})
    hit = miss = 0.0
    for grid, launches in launch_grids.items():
        e = per.get(str(grid))
        if e is None:
            return None
        hit += launches * e["hit"]
        miss += launches * e["miss"]
    return round(hit / (hit + miss), 4) if hit + miss > 0 else None


def roofline_from_stats(stats, traffic=None, timed=None):
    """Roofline of the kernel with the most time in stats, from its launches
    in timed (the timed region) when they were timed there."""
    name, st = max(stats.items(), key=lambda kv: kv[1]["ms"])
    if timed and timed.get(name, {}).get("launches"):
        st = timed[name]
    if st["launches"] == 0 or st["ms"] <= 0:
        return name, None
    achieved = st["bytes"] / (st["ms"] * 1e-3) / 1e9
    tr = traffic.get(name) if traffic else None
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
    if args.workload == "headline":
        out = bench_headline(args, ctx, dev, torch, synth, MusterParams)
    elif args.workload == "register":
        out = bench_register(args, ctx, dev, torch, synth, MusterParams)
    elif args.workload == "batch":
        out = bench_batch(args, ctx, dev, torch, synth, MusterParams)
    elif args.workload == "blobs":
        out = bench_blobs(args, ctx, dev, torch, synth, MusterParams)
    else:
        out = bench_serve(args, ctx, dev, torch, synth, MusterParams)
    if args.copy_calibration:
        # a kernel of known traffic for the counters: 64 Mi int32 read and
        # written once (256 MiB each way), under a name nothing else launches
        a = torch.zeros(64 * 1024 * 1024, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        torch.bitwise_not(a)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)
    ctx.close()


def host_info():
    """The host the CPU baseline ran on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"cpu_model": model, "cpu_count": os.cpu_count(), "cpus_allowed": aff}


def cpu_baseline_steps(images, params_np, pool_times, budget_s=10.0, max_steps=8):
    """The FP64 oracle, as it stands, on one core (BLAS held to one thread):
    Adam steps (loss, hand-written gradient, update) of the given sessions
    pooled pool_times times (2x2x2 means), as many as start within budget_s.
    Returns (session-voxel-iterations per second, steps, seconds, grid, the
    seconds of each step)."""
    from oracle import muster_oracle as O
    from threadpoolctl import threadpool_limits
    imgs = [np.asarray(x, np.float64) for x in images]
    for _ in range(pool_times):
        imgs = [O.pool2(x) for x in imgs]
    N = len(imgs)
    ff = getattr(params_np, "flow_factor", 1)
    phis = [np.zeros((3,) + tuple(n // ff for n in imgs[0].shape)) for _ in range(N - 1)]
    m = [np.zeros_like(x) for x in phis]
    v = [np.zeros_like(x) for x in phis]
    per = []
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        steps = 0
        while steps < max_steps and (steps == 0 or time.perf_counter() - t0 < budget_s):
            ts = time.perf_counter()
            steps += 1
            _, grads, _ = O.loss_and_grad(phis, imgs, params_np)
            for k in range(N - 1):
                phis[k], m[k], v[k] = O.adam_step(phis[k], grads[k], m[k], v[k], steps,
                                                  params_np.lr)
            per.append(round(time.perf_counter() - ts, 3))
        dt = time.perf_counter() - t0
    V = int(np.prod(imgs[0].shape))
    return N * V * steps / dt, steps, dt, tuple(imgs[0].shape), per


def bench_headline(args, ctx, dev, torch, synth, MusterParams):
    from paper_2412_14671_amd import Server
    W, K, T = args.warmup, args.steps, args.batch_iters
    subjects = []
    for k in range(args.batch_subjects):
        N, shape = synth.subject_draw(100 + k)
        log(f"subject {k} (seed {100 + k}): N={N} {shape}")
        subjects.append(synth.batch_subject(100 + k, device=dev))
    imgs = [s.images.contiguous() for s in subjects]
    times = [s.times for s in subjects]
    per_step = sum(int(x.shape[0]) * x[0].numel() for x in imgs)   # sum_s N_s V_s

    def params(iters, graph):
        return MusterParams(iters=[iters], K=7, window=7, metric="silncc", alpha_ss=1.0, lr=0.1,
                            use_graph=graph)

    torch.cuda.synchronize()
    if W > 0:
        log(f"warmup: {W} batched steps")
        ctx.register_batch(imgs, times, params(W, False))
        torch.cuda.synchronize()
    # timed: K batched steps, eager, events on the dominant kernel's launches
    ctx.set_kernel_timing_only(["exp_bwd"])
    ctx.kernel_stats_reset()
    log(f"timed: {K} batched steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, treps = ctx.register_batch(imgs, times, params(K, False))
    torch.cuda.synchronize()
    dt_call = time.perf_counter() - t0
    # the K steps alone, between the stream synchronisations the library
    # places around them (the call also creates the jobs, moves them to the
    # level and writes their outputs)
    dt = treps[0]["step_seconds"]
    ctx.set_kernel_timing(False)
    stats_timed = ctx.kernel_stats()
    value = per_step * K / dt
    # exp_bwd launches of one batched step: one per squaring (K = 7), each over
    # every direction of every subject
    grid = sum(2 * (s.images.shape[0] - 1) * (-(-s.images.shape[1] // 8)) * (-(-s.images.shape[2] // 8))
               * (-(-s.images.shape[3] // 16)) for s in subjects)
    traffic = {"exp_bwd": traffic_per_launch(args.traffic, "k_exp_bwd", {grid: 7 * K})}
    _, roof = roofline_from_stats(stats_timed, traffic, stats_timed)
    if roof is not None:
        roof["l2_hit_rate"] = l2_hit_per_launch(args.l2hit, "k_exp_bwd", {grid: 7 * K})
    out = {
        "metric": "voxel-iterations/sec (fwd+bwd) batched vs plain loop; p50/p99 job latency",
        "value": round(float(value), 1),
        "unit": "session-voxel-iterations/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(dt / K * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"{len(subjects)} phantom subjects (seeds 100-{99 + len(subjects)}), "
                                "N in 3..10, sizes 96^3/128^3/160x192x160, one batched step of all "
                                "subjects at the finest level, SiLNCC w7, K7, alpha_ss 1, lr 0.1"),
                   "subjects": [[int(s.images.shape[0])] + list(s.images.shape[1:]) for s in subjects],
                   "session_voxels_per_step": per_step},
        "roofline": roof,
        "cpu_baseline": None,
        "timed_call_s": round(dt_call, 3),
    }
    if not args.no_full:
        # the whole schedule, batched (graph-replayed) against the plain loop
        log(f"batched: {T} steps, graph-replayed")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs, breps = ctx.register_batch(imgs, times, params(T, True))
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        tb_steps = breps[0]["step_seconds"]
        log(f"plain loop: {T} steps per subject, eager, default tiles")
        ctx.set_tiling("default")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain = []
        tp_steps = 0.0
        for im, tm in zip(imgs, times):
            svf, _, prep = ctx.register(im, tm, params(T, False))
            plain.append(svf)
            tp_steps += prep["step_seconds"]
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        ctx.set_tiling("autotune")
        eu_b = [eu(s.svf_true.cpu().numpy(), o.cpu().numpy(), s.roi.cpu().numpy())
                for s, o in zip(subjects, outs)]
        eu_p = [eu(s.svf_true.cpu().numpy(), o.cpu().numpy(), s.roi.cpu().numpy())
                for s, o in zip(subjects, plain)]
        eu_0 = [eu(s.svf_true.cpu().numpy(), np.zeros(tuple(o.shape)), s.roi.cpu().numpy())
                for s, o in zip(subjects, outs)]
        del outs, plain
        out.update({
            "batched_value": round(per_step * T / tb, 1),
            "batched_s": round(tb, 3),
            "plain_loop_value": round(per_step * T / tp, 1),
            "plain_loop_s": round(tp, 3),
            "batched_over_plain": round(tp / tb, 3),
            "batched_steps_s": round(tb_steps, 3),
            "plain_loop_steps_s": round(tp_steps, 3),
            "batched_over_plain_steps_only": round(tp_steps / tb_steps, 3),
            "eu_batched": [round(x, 4) for x in eu_b],
            "eu_plain": [round(x, 4) for x in eu_p],
            "eu_at_zero": [round(x, 4) for x in eu_0],
            "eu_max_abs_diff": round(max(abs(a - b) for a, b in zip(eu_b, eu_p)), 5),
        })
    if not args.no_serve:
        # continuous batching: Poisson arrivals of the same subjects on the
        # three-level pyramid
        rng = np.random.Generator(np.random.PCG64(5))
        sparams = MusterParams(iters=[200, 100, 50], K=7, window=7, metric="silncc",
                               alpha_ss=1.0, lr=0.1)
        from paper_2412_14671_amd import Context
        ctx.trim()  # the batched workspaces go back before the server's context takes its budget
        sctx = Context(0)
        srv = Server(sctx)
        arrivals, t = [], 0.0
        while True:
            t += rng.exponential(1.0 / args.serve_rate)
            if t >= args.serve_seconds:
                break
            arrivals.append((t, int(rng.integers(0, len(subjects)))))
        log(f"serving: {len(arrivals)} arrivals over {args.serve_seconds:g} s")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets = []
        for at, k in arrivals:
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            tickets.append((srv.submit(imgs[k], times[k], sparams), k))
        reps = []
        for n, ((tk, _), k) in enumerate(tickets):
            reps.append(srv.wait(tk))
            if (n + 1) % 10 == 0:
                log(f"serving: {n + 1} of {len(tickets)} done")
        wall = time.perf_counter() - t0
        lat = np.array([r["seconds"] for r in reps])
        eus = [eu(subjects[k].svf_true.cpu().numpy(), o.cpu().numpy(), subjects[k].roi.cpu().numpy())
               for ((_, o), k), r in zip(tickets, reps) if r["status"] == 0]
        vox = sum(imgs[k].shape[0] * sum(imgs[k][0].numel() // 8 ** (2 - l) * it
                                         for l, it in enumerate([200, 100, 50]))
                  for _, k in tickets)
        out["serving"] = {
            "workload": (f"Poisson arrivals at {args.serve_rate:g}/s for {args.serve_seconds:g} s, "
                         "each one of the sixteen subjects, pyramid 200/100/50"),
            "jobs": len(tickets), "wall_s": round(wall, 2),
            "jobs_per_s": round(len(tickets) / wall, 3),
            "value": round(vox / wall, 1),
            "p50_s": round(float(np.percentile(lat, 50)), 3),
            "p99_s": round(float(np.percentile(lat, 99)), 3),
            "queue_p50_s": round(float(np.percentile([r["queue_seconds"] for r in reps], 50)), 3),
            "failed": int(sum(r["status"] != 0 for r in reps)),
            "eu_mean": round(float(np.mean(eus)), 4) if eus else None,
        }
        del tickets
        sctx.close()
    if not args.no_register:
        log("single subject: six 160x192x160 sessions, 3 levels")
        reg = bench_register_once(args, ctx, dev, torch, synth, MusterParams)
        out["single_subject"] = reg
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        kc = min(range(len(subjects)), key=lambda k: imgs[k].numel())
        from oracle import muster_oracle as O
        p = O.Params(K=7, window=7, metric=O.SILNCC, alpha_ss=1.0, lr=0.1)
        rate, n, dt_c, grid_c, per = cpu_baseline_steps(imgs[kc].cpu().numpy(), p, 1)
        out["cpu_baseline"] = {
            "value": rate, "unit": "session-voxel-iterations/s", "cores": 1, "kind": "oracle",
            "sample": (f"{n} Adam step{'s' if n > 1 else ''} (loss, adjoint gradient, update) of "
                       f"subject {kc} ({imgs[kc].shape[0]} sessions) with its images pooled once "
                       f"to {grid_c[0]}x{grid_c[1]}x{grid_c[2]}, NumPy float64 on one core, "
                       f"{dt_c:.1f} s"),
            "step_seconds": per, **host_info()}
    return out


def bench_register_once(args, ctx, dev, torch, synth, MusterParams):
    """One warm-up and one timed registration of the single six-session
    160x192x160 subject (three levels, 200/100/50 steps, SiLNCC w7, K7,
    alpha_ss and smoothing as set), graph-replayed; Eu against the ground
    truth."""
    shape = tuple(int(x) for x in args.shape.split(","))
    iters = [int(x) for x in args.iters.split(",")]
    N = args.sessions
    s = synth.phantom_series(shape, N, seed=2, device=dev)
    params = MusterParams(iters=iters, K=7, window=args.window, metric=args.metric,
                          alpha_ss=args.alpha, lr=0.1, smooth_sigma=args.smooth,
                          flow_factor=args.flow_factor)
    L = len(iters)
    vox = sum(N * np.prod([d // 2 ** (L - 1 - l) for d in shape]) * iters[l] for l in range(L))
    ctx.register(s.images, s.times, params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    svf, _, rep = ctx.register(s.images, s.times, params)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    roi = s.roi.cpu().numpy()
    return {"workload": (f"one subject, {N} phantom sessions {shape[0]}x{shape[1]}x{shape[2]}, "
                         f"{L}-level pyramid {'/'.join(map(str, iters))} steps, SiLNCC w{args.window}, "
                         f"K7, alpha_ss {args.alpha:g}, smoothing sigma {args.smooth:g}"),
            "seconds": round(dt, 3), "value": round(float(vox / dt), 1),
            "eu_voxels": round(eu(s.svf_true.cpu().numpy(), svf.cpu().numpy(), roi), 4),
            "eu_at_zero": round(eu(s.svf_true.cpu().numpy(), np.zeros(tuple(svf.shape)), roi), 4),
            "loss_first": rep["loss_first"], "loss_last": rep["loss_last"]}


def bench_register(args, ctx, dev, torch, synth, MusterParams):
    shape = tuple(int(x) for x in args.shape.split(","))
    iters = [int(x) for x in args.iters.split(",")]
    N = args.sessions
    log(f"generating {N} sessions of {shape}")
    s = synth.phantom_series(shape, N, seed=2, device=dev)
    images = s.images.contiguous()
    params = MusterParams(iters=iters, K=7, window=args.window, metric=args.metric, alpha_ss=args.alpha, lr=0.1,
                          smooth_sigma=args.smooth, use_graph=args.graph,
                          flow_factor=args.flow_factor)
    L = len(iters)
    vox_iters = sum(N * np.prod([d // 2 ** (L - 1 - l) for d in shape]) * iters[l]
                    for l in range(L))
    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        svf, _, rep = ctx.register(images, s.times, params)
    torch.cuda.synchronize()
    # only the dominant kernel's launches carry events in the timed region
    # (events on every launch add about 4 % to a registration); the other
    # kernels are timed in one more registration after it
    ctx.set_kernel_timing_only([] if args.graph else ["exp_bwd"])
    ctx.kernel_stats_reset()
    log(f"timed {args.steps}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        svf, _, rep = ctx.register(images, s.times, params)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.set_kernel_timing(False)
    stats_timed = ctx.kernel_stats()
    stats = stats_timed
    if not args.graph and args.kernel_table:
        log("per-kernel timing, one more registration")
        ctx.set_kernel_timing(True)
        ctx.kernel_stats_reset()
        ctx.register(images, s.times, params)
        torch.cuda.synchronize()
        ctx.set_kernel_timing(False)
        stats = ctx.kernel_stats()
    ms = dt / args.steps * 1e3
    value = vox_iters / (dt / args.steps)
    graph_replay = None
    if not args.graph and args.graph_steps > 0:
        # the same registration with each level's iteration captured once and
        # replayed (capture included in the time); per-kernel timing is off
        gparams = MusterParams(iters=iters, K=7, window=args.window, metric=args.metric, alpha_ss=args.alpha,
                               lr=0.1, smooth_sigma=args.smooth, use_graph=True,
                               flow_factor=args.flow_factor)
        log(f"graph replay {args.graph_steps}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.graph_steps):
            ctx.register(images, s.times, gparams)
        torch.cuda.synchronize()
        dg = (time.perf_counter() - t0) / args.graph_steps
        graph_replay = {"ms_per_step": round(dg * 1e3, 2), "value": round(float(vox_iters / dg), 1)}
    roi = s.roi.cpu().numpy()
    svf_np = svf.cpu().numpy()
    true_np = s.svf_true.cpu().numpy()
    # exp_bwd launches per level: K per iteration, tiles 2(N-1) x point tiles (8x8x16)
    grids = {}
    for l in range(L):
        d = [x // 2 ** (L - 1 - l) for x in shape]
        g = 2 * (N - 1) * (-(-d[0] // 8)) * (-(-d[1] // 8)) * (-(-d[2] // 16))
        grids[g] = grids.get(g, 0) + 7 * iters[l] * args.steps
    traffic = {"exp_bwd": traffic_per_launch(args.traffic, "k_exp_bwd", grids)}
    kname, roof = roofline_from_stats(stats, traffic, stats_timed)
    if roof is not None:
        roof["l2_hit_rate"] = l2_hit_per_launch(args.l2hit, "k_" + kname, grids)
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
                                f"{'SiLNCC' if args.metric == 'silncc' else 'LNCC'} w{args.window}, K7, "
                                f"alpha_ss {args.alpha:g}, smoothing sigma {args.smooth:g}"
                                + (f", flows on a grid {args.flow_factor}x coarser"
                                   if args.flow_factor > 1 else "")),
                   "sessions": N, "dims": list(shape), "levels": L, "iters": iters,
                   "graphs": bool(args.graph)},
        "roofline": roof,
        "cpu_baseline": None,
        "graph_replay": graph_replay,
        "eu_voxels": round(eu(true_np, svf_np, roi), 4),
        "eu_at_zero": round(eu(true_np, np.zeros_like(svf_np), roi), 4),
        # Sec. 2.8 metrics per interval, by the library's evaluation kernel
        "pcc_per_interval": [round(ctx.field_metrics(s.svf_true[k].contiguous(), svf[k].contiguous(),
                                                     s.roi)[1], 4) for k in range(N - 1)],
        "slope_per_interval": [round(ctx.field_metrics(s.svf_true[k].contiguous(), svf[k].contiguous(),
                                                       s.roi)[2], 4) for k in range(N - 1)],
        "loss_first": rep["loss_first"], "loss_last": rep["loss_last"],
        "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                        "GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None}
                    for k, v in stats.items() if v["launches"]},
    }
    if not args.no_cpu_baseline:
        from oracle import muster_oracle as O
        log("cpu baseline (oracle)")
        coarse = tuple(d // 2 ** (L - 1) for d in shape)
        p = O.Params(K=7, window=args.window, metric=O.SILNCC if args.metric == "silncc" else O.LNCC,
                     alpha_ss=args.alpha, lr=0.1, smooth_sigma=args.smooth / 2 ** (L - 1),
                     flow_factor=args.flow_factor)
        out["cpu_baseline"] = cpu_baseline_register(s.images.cpu().numpy(), p, coarse)
    return out


def bench_batch(args, ctx, dev, torch, synth, MusterParams):
    subjects = []
    sizes = synth.SIZES
    if args.batch_sizes:
        sizes = tuple((int(e),) * 3 for e in args.batch_sizes.split(","))
    for k in range(args.batch_subjects):
        N, shape = synth.subject_draw(100 + k, sizes)
        log(f"subject {k}: N={N} {shape}")
        subjects.append(synth.batch_subject(100 + k, device=dev, shape=shape, N=N))
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
    # PyTorch-eager plain loop: per-iteration time of every subject (first
    # iteration untimed), scaled to the same iteration count; one subject runs
    # the whole schedule to compare the final error
    t_eager = 0.0
    for k, s in enumerate(subjects):
        log(f"torch eager loop, subject {k}")
        _, per = torch_register(torch, s.images, args.batch_iters, lr=0.1, timed_iters=3, K=7,
                                window=7, metric="silncc", alpha_ss=args.alpha,
                                smooth_sigma=args.smooth)
        t_eager += per * args.batch_iters
        torch.cuda.empty_cache()
    kc = min(range(len(subjects)), key=lambda k: subjects[k].images.numel())
    log(f"torch eager loop, full schedule on subject {kc}")
    ph_e, _ = torch_register(torch, subjects[kc].images, args.batch_iters, lr=0.1, K=7, window=7,
                             metric="silncc", alpha_ss=args.alpha, smooth_sigma=args.smooth)
    sv_e = torch.stack([_torch_smooth(torch, p, args.smooth) for p in ph_e])
    eu_e = eu(subjects[kc].svf_true.cpu().numpy(), sv_e.cpu().numpy(), subjects[kc].roi.cpu().numpy())
    torch.cuda.empty_cache()
    eu_b = [eu(s.svf_true.cpu().numpy(), o.cpu().numpy(), s.roi.cpu().numpy()) for s, o in zip(subjects, outs)]
    eu_p = [eu(s.svf_true.cpu().numpy(), o.cpu().numpy(), s.roi.cpu().numpy()) for s, o in zip(subjects, plain)]
    return {"metric": "voxel-iterations/sec (fwd+bwd) batched vs plain loop",
            "value": round(vox / tb, 1), "unit": "session-voxel-iterations/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": round(tb * 1e3, 1), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{len(subjects)} subjects, N in 3..10, sizes from "
                                   + "/".join("x".join(map(str, z)) for z in sizes)
                                   + f", {args.batch_iters} steps at the finest level, SiLNCC w7, K7"},
            "plain_loop_value": round(vox / tp, 1), "batched_over_plain": round(tp / tb, 3),
            "torch_eager_loop_value": round(vox / t_eager, 1),
            "batched_over_torch_eager": round(t_eager / tb, 3),
            "torch_eager_eu_check": {"subject": kc, "eu_torch_eager": round(eu_e, 4),
                                     "eu_batched": round(eu_b[kc], 4)},
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
    eus = [eu(pool[k].svf_true.cpu().numpy(), out.cpu().numpy(), pool[k].roi.cpu().numpy())
           for (_, k, out), r in zip(tickets, reps) if r["status"] == 0]
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
            "eu_mean": round(float(np.mean(eus)), 4) if eus else None,
            "eu_max": round(float(np.max(eus)), 4) if eus else None,
            "queue_p50_s": round(float(np.percentile([r["queue_seconds"] for r in reps], 50)), 3),
            "service_mean_s": round(float(np.mean([r["seconds"] - r["queue_seconds"] for r in reps])), 3),
            "failed": int(sum(r["status"] != 0 for r in reps)),
            "failed_status": sorted({int(r["status"]) for r in reps if r["status"] != 0})}

def bench_blobs(args, ctx, dev, torch, synth, MusterParams):
    """Three 32^3 sessions of 20 Gaussian blobs (the later two flowed for t =
    1, 2), 50 Adam steps at one level, K 7, LNCC window 5, alpha_ss 1, lr 0.1:
    about 0.1 GB of traffic per iteration, so launch- and latency-bound.  The
    median over repetitions of the whole registration, eager with kernel
    timing (value) and graph-replayed (the library's default); the oracle's
    full 50-step run beside it."""
    s = synth.blobs_3x32(device=dev)
    images = s.images.contiguous()
    N, V, T = images.shape[0], images[0].numel(), 50

    def params(graph):
        return MusterParams(iters=[T], K=7, window=5, metric="lncc", alpha_ss=1.0, lr=0.1,
                            use_graph=graph)

    vox = N * V * T
    log("warmup")
    for g in (False, True):
        ctx.register(images, s.times, params(g))
    reps = max(args.steps, 5)

    def timed(graph):
        ts, out = [], None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = ctx.register(images, s.times, params(graph))
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), out

    log(f"timed {reps} eager")
    ctx.set_kernel_timing(True)
    ctx.kernel_stats_reset()
    te, (svf, _, rep) = timed(False)
    ctx.set_kernel_timing(False)
    stats = ctx.kernel_stats()
    log(f"timed {reps} graph")
    tg, _ = timed(True)
    _, roof = roofline_from_stats(stats)
    roi = s.roi.cpu().numpy()
    true_np = s.svf_true.cpu().numpy()
    svf_np = svf.cpu().numpy()
    gold_path = os.path.join(ROOT, "tests", "golden", "blobs_3x32_oracle.json")
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else {}
    out = {
        "metric": "voxel-iterations/sec (fwd+bwd)",
        "value": round(vox / te, 1),
        "unit": "session-voxel-iterations/s",
        "n_gpus": 1, "steps": reps, "warmup": 2,
        "ms_per_step": round(te * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "one subject, 3 sessions of 32^3 Gaussian blobs, 50 Adam steps "
                               "at one level, LNCC w5, K7, alpha_ss 1, lr 0.1 (median of repetitions)",
                   "sessions": N, "dims": list(images.shape[1:]), "levels": 1, "iters": [T]},
        "roofline": roof,
        "cpu_baseline": None,
        "graph_replay": {"ms_per_step": round(tg * 1e3, 2), "value": round(vox / tg, 1)},
        "eu_voxels": round(eu(true_np, svf_np, roi), 4),
        "eu_at_zero": round(eu(true_np, np.zeros_like(svf_np), roi), 4),
        "eu_oracle": gold.get("eu_final"),
        "loss_first": rep["loss_first"], "loss_last": rep["loss_last"],
    }
    if not args.no_cpu_baseline:
        from oracle import muster_oracle as O
        log("cpu baseline (oracle, full run)")
        imgs = [x.astype(np.float64) for x in images.cpu().numpy()]
        p = O.Params(K=7, window=5, metric=O.LNCC, alpha_ss=1.0, lr=0.1, iters=(T,))
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):  # one core, BLAS included
            t0 = time.perf_counter()
            O.register(imgs, p)
            dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": vox / dt, "unit": "session-voxel-iterations/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the whole 50-step registration (NumPy float64, "
                                         f"single-threaded), {dt:.1f} s"}
    return out


if __name__ == "__main__":
    main()
