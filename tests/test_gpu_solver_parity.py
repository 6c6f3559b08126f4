"""The paths the benchmark and the systems forms run, against the FP64 oracle:

* the loss and gradient at the pyramid levels of the benchmark's registration
  (six 40x48x40 phantom sessions with the flow smoothed at sigma 0.75, and
  80x96x80 at sigma 1.5; SiLNCC w7, K7): the staged Exp adjoint with the
  regulariser added where the two directions' G_0 are combined;
* the losses a registration records with smoothing on, and across a level
  change (the first loss of the finer level is L at the upsampled flows);
* the batched engine and the server on ragged subjects (different N and
  grids in one launch sequence), each subject's Adam step and losses against
  the oracle's.

Tolerances: 1e-3 relative on losses and gradients (relative L2, and maximum
error within 1e-3 of the largest magnitude).  After one Adam step from zero,
phi moves by lr * g / (|g| + eps) per voxel, so the flows are compared where
the first gradient is not negligible (elsewhere the step's size follows
rounding of a gradient near eps)."""
import sys

import numpy as np
import pytest
import torch

from oracle import muster_oracle as O

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2412_14671_amd import Context
    c = Context(0)
    yield c
    c.close()


def assert_grad_close(got, want, tol=1e-3):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    rel = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)
    mx = np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)
    log(f"  rel L2 {rel:.2e}, max {mx:.2e}")
    assert rel < tol and mx < tol, f"rel L2 {rel:.2e}, max {mx:.2e}"


def metric_id(m):
    return O.LNCC if m == "lncc" else O.SILNCC


@pytest.mark.parametrize("shape,N,sigma", [((40, 48, 40), 6, 0.75), ((80, 96, 80), 2, 1.5)])
def test_loss_and_gradient_at_the_benchmark_levels_match_oracle(ctx, shape, N, sigma):
    """MusterLoss at two levels of the benchmark's pyramid, with its settings
    (SiLNCC w7, K7, alpha_ss 0.1, the level's smoothing width) and flows of
    half the ground-truth size: the staged Exp adjoint (flat in / staged out,
    staged / staged) and the regulariser joined where the staged G_0 of both
    directions are pulled into the SVF gradient."""
    from paper_2412_14671_amd import MusterLoss, MusterParams, synth
    log(f"bench level {shape} N={N} sigma={sigma}")
    s = synth.phantom_series(shape, N, seed=71)
    phis = (0.5 * s.svf_true).float().contiguous()
    svf = phis.to(DEV).requires_grad_(True)
    params = MusterParams(K=7, window=7, metric="silncc", alpha_ss=0.1, smooth_sigma=sigma)
    loss = MusterLoss.apply(svf, s.images.to(DEV), params, ctx)
    loss.backward()
    p = O.Params(K=7, window=7, metric=O.SILNCC, alpha_ss=0.1, smooth_sigma=sigma)
    L_ref, g_ref, _ = O.loss_and_grad([x.numpy().astype(np.float64) for x in phis],
                                      [x.numpy().astype(np.float64) for x in s.images], p)
    log(f"  loss {float(loss.detach()):.8g} against {L_ref:.8g}")
    assert abs(float(loss.detach()) - L_ref) < 1e-3 * abs(L_ref)
    assert_grad_close(svf.grad.cpu().numpy(), np.stack(g_ref))


def test_smoothing_registration_records_the_oracles_losses(ctx):
    """Three Adam steps with smoothing and the diffusion regulariser on (the
    regulariser's value then comes from the kernel that combines the staged
    G_0): the recorded first and last losses are the oracle loop's L(0) and
    L(phi_2), and the returned (smoothed) flows are the oracle's."""
    from paper_2412_14671_amd import MusterParams, synth
    s = synth.phantom_series((24, 28, 32), 3, seed=73)
    params = MusterParams(iters=[3], K=6, window=5, metric="silncc", alpha_ss=0.5, lr=0.05,
                          smooth_sigma=1.0, use_graph=False)
    svf, _, rep = ctx.register(s.images.to(DEV), s.times, params)
    p = O.Params(K=6, window=5, metric=O.SILNCC, alpha_ss=0.5, lr=0.05, smooth_sigma=1.0,
                 iters=(3,))
    sm, _, hist = O.register([x.numpy() for x in s.images], p)
    log(f"  losses gpu {rep['loss_first']:.8g} {rep['loss_last']:.8g} oracle {hist}")
    assert rep["iterations"] == 3
    assert abs(rep["loss_first"] - hist[0]) < 1e-3 * abs(hist[0])
    assert abs(rep["loss_last"] - hist[-1]) < 1e-3 * abs(hist[-1])
    assert abs(hist[-1] - hist[0]) > 1e-2 * abs(hist[0])     # the flows moved
    assert_grad_close(svf.cpu().numpy(), np.stack(sm), tol=2e-2)


def test_level_change_records_the_oracles_loss_at_the_upsampled_flows(ctx):
    """Two levels of one step each: the first recorded loss is L(0) on the
    coarse images, the last is L at the upsampled coarse step on the fine
    images (the pyramid's carry-up, Sec. 2.7), both with the level's own
    smoothing width."""
    from paper_2412_14671_amd import MusterParams, synth
    s = synth.phantom_series((32, 40, 48), 3, seed=74)
    params = MusterParams(iters=[1, 1], K=6, window=5, metric="silncc", alpha_ss=0.3, lr=0.1,
                          smooth_sigma=1.5, use_graph=False)
    _, _, rep = ctx.register(s.images.to(DEV), s.times, params)
    p = O.Params(K=6, window=5, metric=O.SILNCC, alpha_ss=0.3, lr=0.1, smooth_sigma=1.5,
                 iters=(1, 1))
    _, _, hist = O.register([x.numpy() for x in s.images], p)
    log(f"  losses gpu {rep['loss_first']:.8g} {rep['loss_last']:.8g} oracle {hist}")
    assert len(hist) == 2 and rep["iterations"] == 2
    assert abs(rep["loss_first"] - hist[0]) < 1e-3 * abs(hist[0])
    assert abs(rep["loss_last"] - hist[1]) < 1e-3 * abs(hist[1])


RAGGED = [((24, 28, 32), 3, 81), ((16, 24, 20), 4, 82), ((20, 20, 24), 2, 83)]


def _subjects():
    from paper_2412_14671_amd import synth
    return [synth.phantom_series(shape, N, seed=seed) for shape, N, seed in RAGGED]


def _oracle_two_steps(s, lr, sigma):
    """The oracle loop of two Adam steps at one level (the second rate is 0,
    so the flows after it are the first step's), and the first gradient."""
    imgs = [x.numpy().astype(np.float64) for x in s.images]
    N = len(imgs)
    p = O.Params(K=6, window=5, metric=O.SILNCC, alpha_ss=0.5, lr=lr, smooth_sigma=sigma,
                 iters=(2,))
    sm, _, hist = O.register(imgs, p)
    zero = [np.zeros((3,) + imgs[0].shape) for _ in range(N - 1)]
    _, g, _ = O.loss_and_grad(zero, imgs, p)
    return np.stack(sm), hist, np.stack(g)


def _check_against_oracle(s, out, rep, lr, sigma):
    want, hist, g = _oracle_two_steps(s, lr, sigma)
    log(f"  N={s.images.shape[0]} {tuple(s.images.shape[1:])}: losses gpu "
        f"{rep['loss_first']:.8g} {rep['loss_last']:.8g} oracle {hist}")
    assert rep["status"] == 0 and rep["iterations"] == 2
    assert abs(rep["loss_first"] - hist[0]) < 1e-3 * abs(hist[0])
    assert abs(rep["loss_last"] - hist[1]) < 1e-3 * abs(hist[1])
    got = out.cpu().numpy().astype(np.float64)
    if sigma == 0.0:
        big = np.abs(g) > 1e-2 * np.abs(g).max()
        assert big.mean() > 0.05
        assert np.abs(got[big] - want[big]).max() < 1e-3 * lr
    else:
        assert_grad_close(got, want, tol=2e-2)


@pytest.mark.parametrize("sigma,det", [(0.0, False), (1.0, False), (1.0, True)])
def test_batch_of_ragged_subjects_matches_oracle_steps(ctx, sigma, det):
    """Three subjects with 3, 4 and 2 sessions on three different grids, in
    one batched launch sequence replayed from a captured graph: each subject's
    losses and Adam step equal the oracle's for that subject alone (also in
    the deterministic mode's fixed-point accumulation)."""
    from paper_2412_14671_amd import MusterParams
    subjects = _subjects()
    lr = 0.05
    params = MusterParams(iters=[2], K=6, window=5, metric="silncc", alpha_ss=0.5, lr=lr,
                          smooth_sigma=sigma, use_graph=True, deterministic=det)
    outs, reps = ctx.register_batch([s.images.to(DEV) for s in subjects],
                                    [s.times for s in subjects], params)
    for s, o, r in zip(subjects, outs, reps):
        _check_against_oracle(s, o, r, lr, sigma)


def test_served_ragged_subjects_match_oracle_steps():
    """The same subjects submitted together to the continuous-batching
    server (admitted, stepped in shared ticks, retired): each result equals
    the oracle's two steps for that subject alone."""
    from paper_2412_14671_amd import Context, MusterParams, Server
    c = Context(0)
    try:
        srv = Server(c)
        subjects = _subjects()
        lr = 0.05
        params = MusterParams(iters=[2], K=6, window=5, metric="silncc", alpha_ss=0.5, lr=lr,
                              smooth_sigma=1.0)
        imgs = [s.images.to(DEV) for s in subjects]
        tickets = [srv.submit(im, s.times, params) for im, s in zip(imgs, subjects)]
        reps = [srv.wait(tk) for tk, _ in tickets]
        for s, (tk, out), r in zip(subjects, tickets, reps):
            _check_against_oracle(s, out, r, lr, 1.0)
    finally:
        c.close()
