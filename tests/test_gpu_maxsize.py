"""The largest grid the entry points accept: 896 x 896 x 890 voxels, whose three
component planes (3 V = 2 143 518 720 values) come within 0.2 % of the 32-bit
offsets every kernel uses.  The oracle cannot run at this size, so the fields
are chosen for closed forms (Sec. 2.1-2.3, Alg. 1, Eq. cum_deformation):

* a contraction towards the grid centre c, u(p) = -r (p - c), keeps every
  sample position inside the grid, where trilinear sampling of an affine field
  is exact;
* one squaring of u_s = -a_s (p - c) gives u_{s+1} = -(1 - (1 - a_s)^2)(p - c),
  so Exp of -r (p - c) with K squarings is -(1 - (1 - r / 2^K)^(2^K))(p - c);
* the composition of -r_U (p - c) and -r_C (p - c) is
  -(r_U + r_C - r_U r_C)(p - c);
* with those fields and a constant upstream gradient g, the composition
  adjoint gives G_prev = (1 - r_C) g at every voxel, and G_C (the scatter of g
  at the positions c + (1 - r_U)(p - c)) is 8 g wherever every hat function
  around the voxel is covered (r_U = 1/2 puts the positions on a lattice of
  spacing 1/2, and linear B-splines on such a lattice sum to 2 per axis) and
  0 where no position is within one voxel;
* the Exp adjoint, for L = <g, u_K>, conserves sums step by step: each
  squaring multiplies the sum of the gradient by 2 - a_s (the own term, the
  Jacobian term -a_s, and the scatter, whose weights sum to 1).

Every voxel is compared (in z slabs on the device) except for the Exp adjoint,
which is checked through its sums.  Each part takes tens of GB of the GPU's
memory and frees it before the next."""
import math
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
SHAPE = (896, 896, 890)
SLAB = 64


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2412_14671_amd import Context
    c = Context(0)
    yield c
    c.close()


def release(ctx):
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    ctx.trim()


def contraction(r):
    """-r (p - c), c the grid centre, one component plane per axis."""
    D, H, W = SHAPE
    f = torch.empty((3, D, H, W), device=DEV)
    for a, n in enumerate(SHAPE):
        ax = (torch.arange(n, device=DEV, dtype=torch.float64) - (n - 1) / 2.0) * -r
        view = [1, 1, 1]
        view[a] = n
        f[a] = ax.to(torch.float32).view(view).expand(D, H, W)
    return f


def max_err_scaled(got, factor):
    """max over voxels of |got - factor (p - c)|, computed in float64 by slabs."""
    D, H, W = SHAPE
    worst = 0.0
    axes = [torch.arange(n, device=DEV, dtype=torch.float64) - (n - 1) / 2.0 for n in SHAPE]
    for z0 in range(0, D, SLAB):
        z1 = min(D, z0 + SLAB)
        for a in range(3):
            if a == 0:
                want = (factor * axes[0][z0:z1]).view(-1, 1, 1)
            elif a == 1:
                want = (factor * axes[1]).view(1, -1, 1)
            else:
                want = (factor * axes[2]).view(1, 1, -1)
            d = (got[a, z0:z1].to(torch.float64) - want).abs().max().item()
            worst = max(worst, d)
    return worst


def test_exp_on_the_largest_grid(ctx):
    r, K = 0.5, 3
    log(f"largest grid {SHAPE}: Exp, K={K}")
    phi = contraction(r)
    out = ctx.exp(phi, K, 1)
    del phi
    factor = -(1.0 - (1.0 - r / 2 ** K) ** (2 ** K))
    err = max_err_scaled(out, factor)
    largest = abs(factor) * (max(SHAPE) - 1) / 2.0
    log(f"  max error {err:.2e} voxel, largest displacement {largest:.1f}")
    # a few FP32 roundings of values up to 180 voxels per squaring
    assert err < 1e-6 * largest
    del out
    release(ctx)


def test_composition_and_adjoint_on_the_largest_grid(ctx):
    rU, rC = 0.5, 0.25
    log(f"largest grid {SHAPE}: composition and its adjoint")
    U = contraction(rU)
    C = contraction(rC)
    out = ctx.compose(U, C)
    # every value here is a dyadic fraction with few bits: exact in FP32
    err = max_err_scaled(out, -(rU + rC - rU * rC))
    log(f"  composition: max error {err:.2e} voxel")
    assert err <= 1e-6
    del out
    g = (1.0, -2.0, 0.5)
    D, H, W = SHAPE
    G = torch.empty((3, D, H, W), device=DEV)
    for a in range(3):
        G[a].fill_(g[a])
    Gp = torch.zeros_like(G)
    GC = torch.zeros_like(G)
    ctx.compose_bwd(U, C, G, Gp, GC)
    del U, C, G
    for a in range(3):
        dp = (Gp[a] - (1.0 - rC) * g[a]).abs().max().item()
        assert dp == 0.0, f"G_prev component {a}: {dp}"
    del Gp
    # per axis, the positions c + (p - c)/2 cover [(n-1)/4, 3(n-1)/4]: voxels
    # whose hat support [y-1, y+1] lies inside get 2 per axis, voxels farther
    # than one voxel from it get nothing
    inner, outer = [], []
    for n in SHAPE:
        lo, hi = (n - 1) / 4.0, 3.0 * (n - 1) / 4.0
        inner.append(slice(math.ceil(lo + 1.0), math.floor(hi - 1.0) + 1))  # lo <= y - 1, y + 1 <= hi
        outer.append((math.floor(lo - 1.0), math.ceil(hi + 1.0)))          # y <= lo - 1 or y >= hi + 1
    # the scatter sums in 32-bit fixed point per block: each contribution
    # loses less than one quantum, the block's summed largest magnitudes over
    # 2^30 (1024 voxels of magnitude max|g| here); an interior bin takes 4
    # lattice positions per axis, 64 contributions
    quantum = 1024 * max(abs(x) for x in g) / 2.0 ** 30
    for a in range(3):
        full = 8.0 * g[a]
        di = (GC[a][tuple(inner)].to(torch.float64) - full).abs().max().item()
        zero = 0.0
        for ax in range(3):
            lo_end, hi_start = outer[ax]
            for sl in (slice(0, lo_end + 1), slice(hi_start, SHAPE[ax])):
                idx = [slice(None)] * 3
                idx[ax] = sl
                zero = max(zero, GC[a][tuple(idx)].abs().max().item())
        log(f"  G_C component {a}: interior error {di:.2e} (of {full}; bound {64 * quantum:.2e}), "
            f"outside {zero:.1e}")
        assert di < 64 * quantum
        assert zero == 0.0
    del GC
    release(ctx)


def test_exp_adjoint_sums_on_the_largest_grid(ctx):
    r, K = 0.5, 2
    log(f"largest grid {SHAPE}: Exp adjoint (staged), K={K}")
    phi = contraction(r)
    g = (1.0, -2.0, 0.5)
    D, H, W = SHAPE
    G = torch.empty((3, D, H, W), device=DEV)
    for a in range(3):
        G[a].fill_(g[a])
    grad = ctx.exp_bwd(phi, G, K, 1, "store")
    del phi, G
    a0 = r / 2 ** K
    factor = 2.0 ** -K
    for s in range(K):
        a_s = 1.0 - (1.0 - a0) ** (2 ** s)
        factor *= 2.0 - a_s
    V = D * H * W
    for a in range(3):
        got = grad[a].sum(dtype=torch.float64).item()
        want = factor * g[a] * V
        log(f"  component {a}: sum {got:.6e}, closed form {want:.6e}")
        assert abs(got - want) < 1e-5 * abs(want)
        assert torch.isfinite(grad[a]).all()
    del grad
    release(ctx)


@pytest.mark.parametrize("metric", ["lncc", "silncc"])
def test_similarity_on_the_largest_grid(ctx, metric):
    """The warp, the window statistics and their adjoint over the whole grid
    (Sec. 2.6, Eq. LNCC): the moving image an affine function of the fixed
    one, M = 2F + 1 with F = sin 0.7z + sin 0.9y + sin 1.1x and U = 0, so every
    window's LNCC and SiLNCC residual is 0 up to rounding (each window's
    variance is of order 1, far above the guards). A window whose statistics
    mixed voxels of another place would not be."""
    D, H, W = SHAPE
    log(f"largest grid {SHAPE}: similarity {metric}, w 7")
    F = torch.empty(SHAPE, device=DEV)
    yy = torch.sin(0.9 * torch.arange(H, device=DEV, dtype=torch.float64)).view(1, -1, 1)
    xx = torch.sin(1.1 * torch.arange(W, device=DEV, dtype=torch.float64)).view(1, 1, -1)
    for z0 in range(0, D, SLAB):
        z1 = min(D, z0 + SLAB)
        zz = torch.sin(0.7 * torch.arange(z0, z1, device=DEV, dtype=torch.float64)).view(-1, 1, 1)
        F[z0:z1] = (zz + yy + xx).to(torch.float32)
    I = 2.0 * F + 1.0
    U = torch.zeros((3,) + SHAPE, device=DEV)
    val, g = ctx.sim(F, I, U, 7, metric, grad=True)
    gmax = g.abs().max().item()
    log(f"  loss {val:.3e}, largest gradient {gmax:.3e}")
    # a plane of mismatched windows would add about 1e-3 to the mean loss, and
    # a single mismatched window about 1 / (number of windows) = 1.4e-9 to
    # the gradient; rounding leaves far less
    assert abs(val) < 1e-4
    assert math.isfinite(gmax) and gmax < 1e-10
    del F, I, U, g
    release(ctx)
