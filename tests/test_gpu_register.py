"""End-to-end checks of the registration path on the GPU: one solver iteration
against the oracle, the whole optimisation against the oracle's final error,
graph replay against eager launches, batched against alone, the pairwise
outputs, failure isolation, and the continuous-batching server."""
import json
import os
import sys

import numpy as np
import pytest
import torch

from oracle import muster_oracle as O

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
HERE = os.path.dirname(os.path.abspath(__file__))


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2412_14671_amd import Context
    c = Context(0)
    yield c
    c.close()


def assert_same_run(a, b, what):
    """Two runs of the same deterministic job (params.deterministic): the
    flows are bit-identical, whatever else shared the launches."""
    d = (a - b).abs()
    log(f"{what}: max |diff| {float(d.max()):.2e}")
    assert torch.equal(a, b), f"{what}: not bit-identical (max |diff| {float(d.max()):.2e})"


def assert_close_up_to_adam_rounding(a, b, what):
    """Two runs of the same job in the default mode, which differ only in the
    order of float atomics (about 1e-7 relative per gradient).  Adam divides
    each voxel's step by the root of its second moment, so where a gradient is
    at rounding level the step's direction follows the rounding, and over
    many steps such voxels drift apart by a few step sizes while the rest
    agree to rounding.  So: a tiny mean, a tiny 99.9th percentile, and a
    bound on the few outliers of a few steps of lr.  Deterministic mode
    removes the difference altogether (assert_same_run)."""
    d = (a - b).abs().flatten().double()
    q = float(torch.quantile(d[torch.randperm(d.numel(), device=d.device)[:1 << 20]], 0.999))
    log(f"{what}: max |diff| {float(d.max()):.2e}, 99.9% {q:.2e}, mean {float(d.mean()):.2e}")
    assert float(d.mean()) < 1e-6
    assert q < 1e-4
    assert float(d.max()) < 1e-2


def eu(true, est, roi):
    d = np.sqrt(((np.asarray(true, np.float64) - np.asarray(est, np.float64)) ** 2).sum(1))
    return float(d[:, roi].mean())


def test_first_solver_step_matches_oracle(ctx):
    """One Adam step of the solver from phi = 0: the recorded loss is the
    oracle's L(0), and phi_1 = -lr m^/(sqrt(v^) + eps) with the oracle's
    gradient (compared where the gradient is not negligible)."""
    from paper_2412_14671_amd import MusterParams, synth
    s = synth.phantom_series((24, 28, 32), 4, seed=9)
    imgs = s.images.to(DEV)
    params = MusterParams(iters=[1], K=6, window=5, metric="silncc", alpha_ss=1.0, lr=0.05,
                          use_graph=False)
    svf, _, rep = ctx.register(imgs, s.times, params)
    p = O.Params(K=6, window=5, metric=O.SILNCC, alpha_ss=1.0)
    zero = [np.zeros((3, 24, 28, 32)) for _ in range(3)]
    L0, grads, _ = O.loss_and_grad(zero, [x.numpy() for x in s.images], p)
    assert abs(rep["loss_first"] - L0) < 1e-3 * abs(L0)
    g = np.stack(grads)
    want = np.zeros_like(g)
    want, _, _ = O.adam_step(want, g, np.zeros_like(g), np.zeros_like(g), 1,
                             O.lr_schedule(1, 1, 0.05))
    got = svf.cpu().numpy().astype(np.float64)
    big = np.abs(g) > 1e-2 * np.abs(g).max()
    assert big.mean() > 0.05
    assert np.abs(got[big] - want[big]).max() < 1e-3 * 0.05


def test_blob_series_registration_matches_oracle_error(ctx):
    """The 50-step single-level run on the 32^3 blob series reaches the
    oracle's final registration error (trajectories differ by rounding only)."""
    from paper_2412_14671_amd import MusterParams, synth
    gold = json.load(open(os.path.join(HERE, "golden", "blobs_3x32_oracle.json")))
    s = synth.blobs_3x32()
    params = MusterParams(iters=[50], K=7, window=5, metric="lncc", alpha_ss=1.0, lr=0.1)
    svf, pairs, rep = ctx.register(s.images.to(DEV), s.times, params, pairs=True)
    e = eu(s.svf_true.numpy(), svf.cpu().numpy(), s.roi.numpy())
    log(f"3x32^3 blobs: Eu {e:.4f} (oracle {gold['eu_final']:.4f}, zero {gold['eu_zero']:.4f})")
    assert e < 0.8 * gold["eu_zero"]
    assert abs(e - gold["eu_final"]) < 1e-3
    assert abs(rep["loss_first"] - gold["loss"][0]) < 1e-3 * abs(gold["loss"][0])
    # a 50-step FP32 trajectory drifts from the FP64 one by rounding compounded
    # through Adam; the per-evaluation bar (1e-3) applies to the first loss
    assert abs(rep["loss_last"] - gold["loss"][-1]) < 1e-2 * abs(gold["loss"][-1])
    # the pair fields returned are the compositions of the returned SVFs
    f0 = ctx.exp(svf[0].contiguous(), 7, 1)
    f1 = ctx.exp(svf[1].contiguous(), 7, 1)
    U02 = ctx.compose(f0, f1)
    N = 3
    idx = lambda i, j: i * (N - 1) + (j if j < i else j - 1)  # noqa: E731
    assert torch.allclose(pairs[idx(0, 1)], f0, atol=1e-6)
    assert torch.allclose(pairs[idx(0, 2)], U02, atol=1e-5)
    # and every pair field equals the oracle's (Sec. 2.2: consecutive fields
    # Exp(+-phi_i), composed outward from the target) for the returned SVFs
    phis = svf.cpu().numpy().astype(np.float64)
    f = [O.exp_fwd(phis[k], 7)[-1] for k in range(N - 1)]
    b = [O.exp_fwd(-phis[k], 7)[-1] for k in range(N - 1)]
    U = O.all_pairs(f, b)
    got = pairs.cpu().numpy().astype(np.float64)
    for (i, j), want in U.items():
        assert np.abs(got[idx(i, j)] - want).max() < 1e-4, (i, j)


@pytest.mark.parametrize("det", [True, False])
def test_graph_replay_matches_eager(ctx, det):
    from paper_2412_14671_amd import MusterParams, synth
    s = synth.phantom_series((32, 24, 40), 3, seed=4)
    imgs = s.images.to(DEV)
    a, _, ra = ctx.register(imgs, s.times, MusterParams(iters=[4, 6], K=5, window=3,
                                                         metric="silncc", use_graph=True,
                                                         deterministic=det))
    b, _, rb = ctx.register(imgs, s.times, MusterParams(iters=[4, 6], K=5, window=3,
                                                         metric="silncc", use_graph=False,
                                                         deterministic=det))
    if det:
        assert_same_run(a, b, "graph vs eager")
        assert abs(ra["loss_last"] - rb["loss_last"]) < 1e-12 * abs(rb["loss_last"])
    else:
        assert_close_up_to_adam_rounding(a, b, "graph vs eager (default mode)")
        assert abs(ra["loss_last"] - rb["loss_last"]) < 1e-5 * abs(rb["loss_last"])


@pytest.mark.parametrize("K", [5, 1])
def test_batch_matches_alone(ctx, K):
    """Deterministic jobs with uneven N and grids in one batched launch
    sequence give bit-identical flows and pair fields to each job alone (K 1:
    the flat Exp adjoint, every block's scatter through the fixed point)."""
    from paper_2412_14671_amd import MusterParams, synth
    subjects = [synth.phantom_series((24, 24, 24), 3, seed=31),
                synth.phantom_series((32, 40, 24), 5, seed=32),
                synth.phantom_series((16, 24, 32), 2, seed=33)]
    params = MusterParams(iters=[3, 5], K=K, window=5, metric="silncc", lr=0.1,
                          smooth_sigma=1.0, deterministic=True)
    outs, reps = ctx.register_batch([s.images.to(DEV) for s in subjects],
                                    [s.times for s in subjects], params)
    for s, o, r in zip(subjects, outs, reps):
        alone, _, ra = ctx.register(s.images.to(DEV), s.times, params)
        again, _, _ = ctx.register(s.images.to(DEV), s.times, params)
        assert r["status"] == 0
        assert_same_run(alone, again, "alone vs alone")
        assert_same_run(o, alone, "batched vs alone")
        assert abs(r["loss_last"] - ra["loss_last"]) < 1e-12 * abs(ra["loss_last"])


def test_released_workspaces_are_reused_and_trimmed():
    """The arena keeps the workspaces finished jobs release and hands them to
    later jobs of the same sizes.  A deterministic job run again on kept
    workspaces, which another job has used in between, gives the flow it gave
    on a fresh context; trim returns the kept bytes, after which nothing is
    kept and the bytes in use are unchanged."""
    from paper_2412_14671_amd import Context, MusterParams, synth
    s = synth.phantom_series((24, 32, 40), 4, seed=37)
    other = synth.phantom_series((24, 32, 40), 4, seed=38)
    p = MusterParams(iters=[2, 4], K=5, window=5, metric="silncc", smooth_sigma=1.0,
                     deterministic=True)
    c = Context(0)
    try:
        a, _, _ = c.register(s.images.to(DEV), s.times, p)
        mem = c.memory()
        c.register(other.images.to(DEV), other.times, p)
        b, _, _ = c.register(s.images.to(DEV), s.times, p)
        assert_same_run(a, b, "fresh vs kept workspaces")
        kept = c.trim()
        log(f"in use {mem['in_use']}, peak {mem['peak']}, kept {kept}")
        assert kept >= mem["peak"] - mem["in_use"] > 0
        assert c.trim() == 0
        assert c.memory()["in_use"] == mem["in_use"]
    finally:
        c.close()


def test_deterministic_mode_agrees_with_the_default_mode():
    """The fixed-point accumulation changes results only at rounding level.
    Both runs use the same (default) tiling, so only the accumulation
    differs.  After three Adam steps the flows agree to rounding except where
    a gradient is near Adam's eps, where the step lr g / (|g| + eps) follows
    the rounding: a tiny 99.9th percentile, and a maximum below 0.2 % of a
    step."""
    from paper_2412_14671_amd import Context, MusterParams, synth
    c = Context(0)
    try:
        c.set_tiling("default")
        s = synth.phantom_series((32, 40, 24), 4, seed=35)
        imgs = s.images.to(DEV)
        lr = 0.05
        kw = dict(iters=[3], K=6, window=5, metric="silncc", lr=lr, alpha_ss=0.5, smooth_sigma=1.0)
        a, _, ra = c.register(imgs, s.times, MusterParams(deterministic=True, **kw))
        b, _, rb = c.register(imgs, s.times, MusterParams(deterministic=False, **kw))
        d = (a - b).abs().flatten().double()
        q = float(torch.quantile(d, 0.999))
        log(f"deterministic vs default: max |diff| {float(d.max()):.2e}, 99.9% {q:.2e}")
        assert q < 1e-6
        assert float(d.max()) < 2e-3 * lr
        assert abs(ra["loss_last"] - rb["loss_last"]) < 1e-6 * abs(rb["loss_last"])
    finally:
        c.close()


def test_three_level_pyramid_runs_and_improves(ctx):
    from paper_2412_14671_amd import MusterParams, synth
    s = synth.phantom_series((48, 48, 48), 3, seed=12)
    params = MusterParams(iters=[30, 20, 10], K=7, window=5, metric="silncc", lr=0.1)
    svf, _, rep = ctx.register(s.images.to(DEV), s.times, params)
    roi = s.roi.numpy()
    e = eu(s.svf_true.numpy(), svf.cpu().numpy(), roi)
    e0 = eu(s.svf_true.numpy(), np.zeros(svf.shape), roi)
    log(f"pyramid: Eu {e:.4f} vs {e0:.4f} at zero; iterations {rep['iterations']}")
    assert rep["iterations"] == 60
    assert e < e0


def test_nonfinite_input_fails_only_that_job(ctx):
    from paper_2412_14671_amd import MusterError, MusterParams, synth
    s = synth.phantom_series((16, 16, 16), 3, seed=2)
    bad = s.images.clone()
    bad[1, 3, 4, 5] = float("nan")
    params = MusterParams(iters=[3], K=4, window=3, metric="silncc")
    with pytest.raises(MusterError) as ei:
        ctx.register(bad.to(DEV), s.times, params)
    assert "E_NONFINITE" in str(ei.value)
    svf, _, rep = ctx.register(s.images.to(DEV), s.times, params)
    assert torch.isfinite(svf).all() and rep["status"] == 0


def test_invalid_arguments_are_rejected(ctx):
    from paper_2412_14671_amd import MusterError, MusterParams
    imgs = torch.zeros((3, 16, 16, 16), device=DEV)
    with pytest.raises(MusterError, match="E_INVALID"):
        ctx.register(imgs, [0.0, 2.0, 1.0], MusterParams(iters=[1], window=3))
    with pytest.raises(MusterError, match="E_INVALID"):
        ctx.register(imgs, None, MusterParams(iters=[1, 1, 1, 1, 1], window=3))
    with pytest.raises(MusterError, match="E_INVALID"):
        ctx.register(imgs[:1], None, MusterParams(iters=[1], window=3))
    # an empty batch, and a batch whose jobs differ in their schedule
    with pytest.raises(MusterError, match="E_INVALID"):
        ctx.register_batch([], None, MusterParams(iters=[1], window=3))
    from paper_2412_14671_amd import _lib as L
    from paper_2412_14671_amd.api import _stream
    keep = []
    outs = [torch.empty((2, 3, 16, 16, 16), device=DEV) for _ in range(2)]
    jobs = (L.Job * 2)()
    for k, n in enumerate((1, 2)):
        jobs[k] = ctx._job(imgs, None, MusterParams(iters=[n], window=3), outs[k], None, keep=keep)
    reps = (L.Report * 2)()
    assert ctx.lib.muster_register_batch(ctx.h, _stream(), 2, jobs, reps) == L.E_INVALID


def test_server_results_match_alone(ctx):
    """Jobs submitted together are admitted, batched with each other (each
    tick steps every resident job, whatever its level) and retired between
    ticks; each result is bit-identical to the job run alone on another
    context (deterministic mode: fixed-point scatters, and the default tiling
    of the window sums rather than each context's autotuned one)."""
    from paper_2412_14671_amd import Context, MusterParams, Server, synth
    c2 = Context(0)
    srv = Server(c2)
    subjects = [synth.phantom_series((24, 24, 24), 3, seed=41),
                synth.phantom_series((32, 24, 16), 4, seed=42),
                synth.phantom_series((16, 16, 32), 3, seed=43),
                synth.phantom_series((24, 32, 24), 2, seed=44)]
    params = [MusterParams(iters=[4, 6], K=5, window=3, metric="silncc", deterministic=True),
              MusterParams(iters=[2, 3], K=5, window=3, metric="silncc", deterministic=True),
              MusterParams(iters=[5], K=5, window=3, metric="silncc", deterministic=True),
              MusterParams(iters=[1, 2, 3], K=5, window=3, metric="silncc", deterministic=True)]
    imgs = [s.images.to(DEV) for s in subjects]
    tickets = [srv.submit(im, s.times, p) for im, s, p in zip(imgs, subjects, params)]
    reps = [srv.wait(tk) for tk, _ in tickets]
    for (tk, out), im, s, p, r in zip(tickets, imgs, subjects, params, reps):
        assert r["status"] == 0, r
        alone, _, ra = ctx.register(im, s.times, p)
        assert_same_run(out, alone, "served vs alone")
        assert abs(r["loss_last"] - ra["loss_last"]) < 1e-12 * abs(ra["loss_last"])
        assert r["iterations"] == sum(p.iters)
    st = srv.stats()
    assert st["resident"] == 0 and st["queued"] == 0
    c2.close()


def test_server_mixes_levels_without_steps_and_other_windows(ctx):
    """A served job whose first level has no steps (iters [0, 5]) shares its
    ticks with stepping jobs but takes no step until its second level, and
    jobs with another window, metric or K are admitted behind it without
    waiting (they run in a launch group of their own in the same ticks):
    every result is bit-identical to the job alone."""
    from paper_2412_14671_amd import Context, MusterParams, Server, synth
    c2 = Context(0)
    try:
        srv = Server(c2)
        subjects = [synth.phantom_series((24, 24, 24), 3, seed=45),
                    synth.phantom_series((32, 24, 16), 3, seed=46),
                    synth.phantom_series((16, 24, 32), 4, seed=47),
                    synth.phantom_series((24, 16, 24), 2, seed=48)]
        params = [MusterParams(iters=[6, 4], K=5, window=3, metric="silncc", deterministic=True),
                  MusterParams(iters=[0, 5], K=5, window=3, metric="silncc", deterministic=True),
                  MusterParams(iters=[5], K=5, window=5, metric="lncc", deterministic=True),
                  MusterParams(iters=[2, 3], K=4, window=3, metric="silncc", deterministic=True)]
        imgs = [s.images.to(DEV) for s in subjects]
        tickets = [srv.submit(im, s.times, p) for im, s, p in zip(imgs, subjects, params)]
        reps = [srv.wait(tk) for tk, _ in tickets]
        for (tk, out), im, s, p, r in zip(tickets, imgs, subjects, params, reps):
            assert r["status"] == 0, r
            assert r["iterations"] == sum(p.iters)
            alone, _, ra = ctx.register(im, s.times, p)
            assert_same_run(out, alone, f"served vs alone, iters {list(p.iters)}")
            assert abs(r["loss_last"] - ra["loss_last"]) < 1e-12 * abs(ra["loss_last"])
    finally:
        c2.close()


def test_autotuned_tiling_is_valid_cached_and_reproducible():
    """The autotuner returns a valid tiling, caches it, and a registration
    under it equals one under the same tiling fixed by hand."""
    from paper_2412_14671_amd import Context, MusterParams, synth
    c = Context(0)
    try:
        sh, zc = c.sim_tiling((48, 40, 56), 7, "silncc")
        log(f"autotuned tiling for 48x40x56 w7: shape {sh}, zchunk {zc}")
        assert 0 <= sh < 3 and 1 <= zc <= 48
        assert c.sim_tiling((48, 40, 56), 7, "silncc") == (sh, zc)
        s = synth.phantom_series((48, 40, 56), 3, seed=21)
        imgs = s.images.to(DEV)
        params = MusterParams(iters=[15], K=7, window=7, metric="silncc", use_graph=False)
        a, _, ra = c.register(imgs, s.times, params)
        c.set_tiling("fixed", sh, zc)
        b, _, rb = c.register(imgs, s.times, params)
        assert_close_up_to_adam_rounding(a, b, "autotuned vs fixed")
        assert abs(ra["loss_last"] - rb["loss_last"]) <= 1e-6 * abs(ra["loss_last"])
    finally:
        c.close()


def test_solver_steps_with_l2_and_ts_match_oracle(ctx):
    """Three Adam steps with every regulariser on (the schedule's last rate is
    0, so the output is phi_2): the recorded losses are the oracle's L(0) and
    L(phi_2), and phi_2 follows the oracle's updates, whose second gradient
    carries the L_L2 and L_ts terms of phi_1."""
    from paper_2412_14671_amd import MusterParams, synth
    s = synth.phantom_series((20, 24, 28), 4, seed=13)
    imgs = [x.numpy() for x in s.images]
    params = MusterParams(iters=[3], K=6, window=5, metric="silncc", alpha_ss=0.5, alpha_l2=0.5,
                          alpha_ts=2.0, lr=0.05, use_graph=False)
    svf, _, rep = ctx.register(s.images.to(DEV), s.times, params)
    p = O.Params(K=6, window=5, metric=O.SILNCC, alpha_ss=0.5, alpha_l2=0.5, alpha_ts=2.0,
                 times=tuple(s.times))
    phi = [np.zeros((3, 20, 24, 28)) for _ in range(3)]
    m = [np.zeros_like(x) for x in phi]
    v = [np.zeros_like(x) for x in phi]
    losses, gs = [], []
    for t in (1, 2, 3):
        L, g, aux = O.loss_and_grad(phi, imgs, p)
        losses.append(L)
        gs.append(np.stack(g))
        lr = O.lr_schedule(t, 3, 0.05)
        for k in range(3):
            phi[k], m[k], v[k] = O.adam_step(phi[k], g[k], m[k], v[k], t, lr)
    log(f"losses gpu {rep['loss_first']:.6f} {rep['loss_last']:.6f} oracle {losses}")
    assert abs(rep["loss_first"] - losses[0]) < 1e-3 * abs(losses[0])
    assert abs(rep["loss_last"] - losses[2]) < 1e-3 * abs(losses[2])
    got = svf.cpu().numpy().astype(np.float64)
    want = np.stack(phi)
    big = (np.abs(gs[0]) > 1e-2 * np.abs(gs[0]).max()) & (np.abs(gs[1]) > 1e-2 * np.abs(gs[1]).max())
    assert big.mean() > 0.02
    assert np.abs(got[big] - want[big]).max() < 2e-3 * 0.05 * 2


def test_registration_on_a_coarse_flow_grid(ctx):
    """flow_factor 2: flows on a grid twice as coarse through a 2-level
    pyramid; the first loss is the oracle's L(0), outputs come back on the
    image grid, and the registration error improves on the identity."""
    from paper_2412_14671_amd import MusterParams, synth
    s = synth.phantom_series((32, 40, 48), 3, seed=15)
    params = MusterParams(iters=[20, 10], K=6, window=5, metric="silncc", alpha_ss=0.1, lr=0.1,
                          flow_factor=2, smooth_sigma=1.0)
    svf, pairs, rep = ctx.register(s.images.to(DEV), s.times, params, pairs=True)
    assert svf.shape == (2, 3, 32, 40, 48) and pairs.shape == (6, 3, 32, 40, 48)
    p = O.Params(K=6, window=5, metric=O.SILNCC, alpha_ss=0.1, flow_factor=2, smooth_sigma=0.5)
    imgs = [O.pool2(x.numpy().astype(np.float64)) for x in s.images]
    L0 = O.forward([np.zeros((3, 8, 10, 12)) for _ in range(2)], imgs, p)
    assert abs(rep["loss_first"] - L0) < 1e-3 * abs(L0)
    roi = s.roi.numpy()
    e = eu(s.svf_true.numpy(), svf.cpu().numpy(), roi)
    e0 = eu(s.svf_true.numpy(), np.zeros(svf.shape), roi)
    log(f"coarse flow grid: Eu {e:.4f} vs {e0:.4f} at zero")
    assert e < e0
    # the depth-1 pair field is Exp of the returned flow to first order; at
    # least its direction agrees with the flow on the image grid
    f01 = pairs[0].cpu().numpy().ravel()
    assert float(np.dot(f01, svf[0].cpu().numpy().ravel())) > 0


def test_solver_steps_with_rigid_adjustment_match_oracle(ctx):
    """Three Adam steps with the rigid adjustment on (the last rate is 0): the
    losses L(0) and L(step 2), the rigid parameters and phi_2 follow the
    oracle's updates."""
    from paper_2412_14671_amd import MusterParams, synth
    s = synth.phantom_series((20, 24, 28), 3, seed=17)
    imgs = [x.numpy() for x in s.images]
    params = MusterParams(iters=[3], K=5, window=5, metric="silncc", alpha_ss=0.5, lr=0.05,
                          rigid=True, use_graph=False)
    svf, _, rep = ctx.register(s.images.to(DEV), s.times, params)
    p = O.Params(K=5, window=5, metric=O.SILNCC, alpha_ss=0.5, rigid=True)
    phi = [np.zeros((3, 20, 24, 28)) for _ in range(2)]
    rig = [np.zeros(6) for _ in range(2)]
    m = [np.zeros_like(x) for x in phi]
    v = [np.zeros_like(x) for x in phi]
    rm = [np.zeros(6) for _ in range(2)]
    rv = [np.zeros(6) for _ in range(2)]
    rlr = O.rigid_lr(1.0, (20, 24, 28))
    losses, gs = [], []
    for t in (1, 2, 3):
        L, g, aux = O.loss_and_grad(phi, imgs, p, rigid=rig)
        losses.append(L)
        gs.append(np.stack(g))
        lr = O.lr_schedule(t, 3, 0.05)
        for k in range(2):
            phi[k], m[k], v[k] = O.adam_step(phi[k], g[k], m[k], v[k], t, lr)
            gr = aux["rigid_grad"][k]
            rm[k] = 0.9 * rm[k] + 0.1 * gr
            rv[k] = 0.999 * rv[k] + 0.001 * gr * gr
            rig[k] = rig[k] - lr * rlr * (rm[k] / (1 - 0.9 ** t)) / (np.sqrt(rv[k] / (1 - 0.999 ** t)) + 1e-8)
    log(f"rigid: gpu {rep['rigid'].cpu().numpy()} oracle {np.stack(rig)}")
    assert abs(rep["loss_first"] - losses[0]) < 1e-3 * abs(losses[0])
    assert abs(rep["loss_last"] - losses[2]) < 1e-3 * abs(losses[2])
    got = rep["rigid"].cpu().numpy().astype(np.float64)
    want = np.stack(rig)
    # Adam steps of about lr per parameter: compare against that scale
    assert np.abs(got - want).max() < 0.02 * 0.05 * np.maximum(1.0, np.abs(want) / 0.05).max()
    g0, g1 = gs[0], gs[1]
    big = (np.abs(g0) > 1e-2 * np.abs(g0).max()) & (np.abs(g1) > 1e-2 * np.abs(g1).max())
    assert np.abs(svf.cpu().numpy()[big] - np.stack(phi)[big]).max() < 2e-3 * 0.1


def test_rigid_adjustment_recovers_a_translation(ctx):
    """Session 1 is session 0 read (0.8, -0.6, 1.1) voxels away; with the flows
    held near zero by a strong L_L2 term, the rigid translation of session 1
    converges to the displacement that maps it back, minus that offset
    (sampling I_1 at p - offset gives I_0 at p)."""
    import math
    from paper_2412_14671_amd import MusterParams, synth
    shape = (40, 44, 48)
    rng_ = np.random.Generator(np.random.PCG64(23))
    P = synth.Phantom(shape, rng_)
    g = torch.stack(torch.meshgrid(*[torch.arange(n, dtype=torch.float64) for n in shape],
                                   indexing="ij"))
    off = torch.tensor([0.8, -0.6, 1.1], dtype=torch.float64)[:, None, None, None]
    imgs = torch.stack([P(g), P(g + off)]).float()
    params = MusterParams(iters=[60, 60], K=5, window=5, metric="silncc", alpha_ss=1.0,
                          alpha_l2=1e4, lr=0.2, rigid=True)
    _, pairs, rep = ctx.register(imgs.to(DEV), [0.0, 1.0], params, pairs=True)
    r = rep["rigid"].cpu().numpy()[0]
    log(f"recovered rigid {r}, loss {rep['loss_first']:.5f} -> {rep['loss_last']:.5f}")
    assert np.abs(r[3:] + np.array([0.8, -0.6, 1.1])).max() < 0.15
    assert np.abs(r[:3]).max() < 0.02
    # the returned pair field (0, 1) is the total deformation: about -offset
    tot = pairs[0].cpu().numpy().reshape(3, -1).mean(axis=1)
    assert np.abs(tot + np.array([0.8, -0.6, 1.1])).max() < 0.15


def test_kernel_timing_counts_every_launch(ctx):
    """Kernel timing (the events the bench reads its roofline from) sees every
    launch of the eager path: K Exp-backward launches and one finish per Adam
    step, positive durations, and a total below the wall time of the run."""
    import time
    from paper_2412_14671_amd import MusterParams, synth
    s = synth.phantom_series((24, 28, 32), 3, seed=5)
    imgs = s.images.to(DEV)
    params = MusterParams(iters=[4], K=5, window=3, metric="silncc", use_graph=False)
    ctx.register(imgs, s.times, params)
    torch.cuda.synchronize()
    ctx.set_kernel_timing(True)
    ctx.kernel_stats_reset()
    try:
        t0 = time.perf_counter()
        ctx.register(imgs, s.times, params)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3
    finally:
        ctx.set_kernel_timing(False)
    st = ctx.kernel_stats()
    log("timed kernels: " + ", ".join(f"{k} {v['launches']}x {v['ms']:.3f} ms"
                                      for k, v in st.items() if v["launches"]))
    assert st["exp_bwd"]["launches"] == 4 * 5
    assert st["finish"]["launches"] == 4
    assert st["sim_stats"]["launches"] == 4 and st["sim_grad"]["launches"] == 4
    assert all(v["ms"] > 0 for v in st.values() if v["launches"])
    assert 0 < sum(v["ms"] for v in st.values()) < wall_ms
    # timing one class: only its launches are counted, all of them
    ctx.set_kernel_timing_only(["exp_bwd"])
    ctx.kernel_stats_reset()
    try:
        ctx.register(imgs, s.times, params)
        torch.cuda.synchronize()
    finally:
        ctx.set_kernel_timing(False)
    only = ctx.kernel_stats()
    assert only["exp_bwd"]["launches"] == 4 * 5 and only["exp_bwd"]["ms"] > 0
    assert only["exp_bwd"]["bytes"] == st["exp_bwd"]["bytes"]
    assert all(v["launches"] == 0 for k, v in only.items() if k != "exp_bwd")
    from paper_2412_14671_amd import _lib as L
    assert ctx.lib.muster_set_kernel_timing_mask(ctx.h, 1 << len(L.KERNELS)) == L.E_INVALID


def test_server_budget_queue_and_cancellation():
    """Forced failures of the server: a job larger than the context's whole
    budget is refused (E_NOMEM); with a budget for one job, a second job
    waits in the queue and a third is refused while the queue is full
    (E_BUSY); cancelling the queued and the running job ends both with
    E_CANCELLED; the server then serves a new job normally."""
    import time
    from paper_2412_14671_amd import Context, MusterError, MusterParams, Server, synth
    from paper_2412_14671_amd import _lib as L
    small = synth.phantom_series((24, 24, 24), 3, seed=51)
    big = synth.phantom_series((48, 48, 48), 4, seed=52)
    long_p = MusterParams(iters=[20000], K=5, window=3, metric="silncc")
    short_p = MusterParams(iters=[3], K=5, window=3, metric="silncc")
    probe = Context(0)
    fp = probe.footprint(3, (24, 24, 24), long_p)
    probe.close()
    c = Context(0, budget_bytes=int(1.6 * fp))  # room for one such job, not two
    try:
        c.set_tiling("default")  # no autotuning scratch inside the small budget
        srv = Server(c, max_queue=1)
        with pytest.raises(MusterError) as ei:
            srv.submit(big.images.to(DEV), big.times, long_p)
        assert "E_NOMEM" in str(ei.value)
        img = small.images.to(DEV)
        ta, _ = srv.submit(img, small.times, long_p)
        t0 = time.time()
        while srv.poll(ta) != 1:  # admitted and running
            assert time.time() - t0 < 60, "job not admitted"
            time.sleep(0.01)
        tb, _ = srv.submit(img, small.times, long_p)
        time.sleep(0.05)
        assert srv.poll(tb) == 0  # no room for a second job: it waits
        st = srv.stats()
        assert st["resident"] == 1 and st["queued"] == 1
        with pytest.raises(MusterError) as ei:
            srv.submit(img, small.times, long_p)
        assert "E_BUSY" in str(ei.value)
        srv.cancel(tb)
        srv.cancel(ta)
        ra, rb = srv.wait(ta), srv.wait(tb)
        assert ra["status"] == L.E_CANCELLED and rb["status"] == L.E_CANCELLED
        assert ra["iterations"] < 20000
        td, out = srv.submit(img, small.times, short_p)
        rd = srv.wait(td)
        assert rd["status"] == 0 and rd["iterations"] == 3
        assert torch.isfinite(out).all()
        st = srv.stats()
        assert st["resident"] == 0 and st["queued"] == 0
    finally:
        c.close()
