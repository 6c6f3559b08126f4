"""Seeded synthetic session series for tests and benchmarks.

This module only draws inputs: random images, smooth random velocity fields
and the session series obtained by flowing an image along them.  It holds none
of the registration method's arithmetic (no scaling and squaring, no
composition of discrete deformations, no similarity, no gradients).  Velocity
fields are drawn as white noise smoothed by a Gaussian filter in the Fourier
domain (the recipe of the paper's Appendix A); sessions are produced by
integrating the flow ODE of Sec. 2.1 (Eq. ode) with classical fourth-order
Runge-Kutta, the field being read between grid points by torch's own
``grid_sample``.  Everything runs in float64 on the requested torch device and
is returned as contiguous float32.

Recipes (sizes, value ranges) follow the workloads the method is evaluated on:
  * blobs(): a sum of random Gaussian blobs plus Gaussian noise, sessions 2..N
    obtained by flowing one velocity field for times 1, 2, ...;
  * phantom(): a brain-like phantom of three nested smoothed ellipsoids
    (intensities 0.3/0.6/0.9) with a folded texture of amplitude 0.15 inside
    the outer one, a smooth multiplicative bias field of +-10 %
    per session, Rician noise, unevenly spaced acquisition times and one
    velocity field per interval.

Ground truth: with session k+1 equal to session k pulled back along the
time-1 flow of v_k, the consecutive velocity field that pulls session k+1 onto
session k is -v_k; svf_true holds those fields.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch


@dataclass
class Series:
    images: torch.Tensor        # (N, D, H, W) float32
    times: np.ndarray           # (N,) float64, strictly increasing
    svf_true: torch.Tensor      # (N-1, 3, D, H, W) float32, voxel units
    roi: torch.Tensor           # (D, H, W) bool
    name: str = ""


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_smooth(x: torch.Tensor, sigma: float) -> torch.Tensor:
    """Gaussian filter of the trailing three axes, applied in the Fourier
    domain with the transfer function exp(-sigma^2 |omega|^2 / 2)."""
    D, H, W = x.shape[-3:]
    dev = x.device
    wz = 2 * math.pi * torch.fft.fftfreq(D, device=dev, dtype=torch.float64)
    wy = 2 * math.pi * torch.fft.fftfreq(H, device=dev, dtype=torch.float64)
    wx = 2 * math.pi * torch.fft.rfftfreq(W, device=dev, dtype=torch.float64)
    tf = torch.exp(-0.5 * sigma ** 2 * (wz[:, None, None] ** 2 + wy[None, :, None] ** 2
                                         + wx[None, None, :] ** 2))
    X = torch.fft.rfftn(x, dim=(-3, -2, -1))
    return torch.fft.irfftn(X * tf, s=(D, H, W), dim=(-3, -2, -1))


def random_velocity(shape, sigma: float, vmax: float, rng: np.random.Generator,
                    device) -> torch.Tensor:
    """White noise per component and voxel, Gaussian-smoothed, rescaled so
    that the largest vector norm on the grid equals vmax.  (3, D, H, W) f64."""
    n = torch.from_numpy(rng.standard_normal((3,) + tuple(shape))).to(device)
    v = gaussian_smooth(n, sigma)
    mx = torch.sqrt((v * v).sum(0)).max()
    return v * (vmax / mx)


def _grid(shape, device) -> torch.Tensor:
    ax = [torch.arange(n, device=device, dtype=torch.float64) for n in shape]
    return torch.stack(torch.meshgrid(*ax, indexing="ij"))


def _eval_field(v: torch.Tensor, pts: torch.Tensor) -> torch.Tensor:
    """Value of the gridded field v (C, D, H, W) at positions pts (3, ...)
    through torch.nn.functional.grid_sample (border padding)."""
    C, D, H, W = v.shape
    shp = pts.shape[1:]
    p = pts.reshape(3, -1)
    # grid_sample wants (x, y, z) in [-1, 1] with align_corners=True
    g = torch.stack([2 * p[2] / (W - 1) - 1, 2 * p[1] / (H - 1) - 1, 2 * p[0] / (D - 1) - 1], -1)
    out = torch.nn.functional.grid_sample(v[None], g[None, None, None], mode="bilinear",
                                          padding_mode="border", align_corners=True)
    return out.reshape(C, *shp)


def flow(v: torch.Tensor, pts: torch.Tensor, t: float = 1.0, steps: int = 8) -> torch.Tensor:
    """Positions reached at time t by particles that start at pts and follow
    dx/dt = v(x) (Eq. ode with a stationary field), by RK4."""
    h = t / steps
    x = pts
    for _ in range(steps):
        k1 = _eval_field(v, x)
        k2 = _eval_field(v, x + 0.5 * h * k1)
        k3 = _eval_field(v, x + 0.5 * h * k2)
        k4 = _eval_field(v, x + h * k3)
        x = x + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return x


# ---------------------------------------------------------------------------
# Images evaluated analytically at arbitrary positions
# ---------------------------------------------------------------------------

class Blobs:
    """Sum of isotropic Gaussian blobs."""

    def __init__(self, shape, n_blobs, rng, sig=(2.0, 5.0)):
        self.c = rng.uniform(0, 1, (n_blobs, 3)) * np.asarray(shape, np.float64)
        self.s = rng.uniform(sig[0], sig[1], n_blobs)
        self.a = rng.uniform(0, 1, n_blobs)

    def __call__(self, pts: torch.Tensor) -> torch.Tensor:
        out = torch.zeros(pts.shape[1:], dtype=torch.float64, device=pts.device)
        for c, s, a in zip(self.c, self.s, self.a):
            d2 = ((pts[0] - c[0]) ** 2 + (pts[1] - c[1]) ** 2 + (pts[2] - c[2]) ** 2)
            out += a * torch.exp(-d2 / (2 * s * s))
        return out


class Phantom:
    """Three nested ellipsoids (outer to inner 0.3, 0.6, 0.9 over a zero
    background) whose edges are smoothed over about 1.5 voxels, plus a folded
    texture inside the outer ellipsoid: a Gaussian-smoothed random field
    (sigma 2 voxels) passed through tanh, amplitude 0.15, standing in for the
    grey/white-matter folding that gives a brain scan features everywhere.
    The texture is a gridded field read trilinearly, so it is one continuous
    function of position like the ellipsoids."""

    def __init__(self, shape, rng, edge=1.5, texture=0.15, texture_sigma=2.0, device="cpu"):
        dims = np.asarray(shape, np.float64)
        self.centre = dims / 2.0 - 0.5 + rng.uniform(-0.03, 0.03, 3) * dims
        self.axes = []
        for frac in (0.42, 0.32, 0.20):
            self.axes.append(frac * dims * rng.uniform(0.9, 1.1, 3))
        self.edge = edge
        self.texture = texture
        t = gaussian_smooth(torch.from_numpy(rng.standard_normal(tuple(shape))).to(device),
                            texture_sigma)
        self.tex = torch.tanh(t / t.std())[None].contiguous()

    def _layer(self, pts, a):
        rho = torch.sqrt(sum(((pts[k] - self.centre[k]) / a[k]) ** 2 for k in range(3)))
        d = (1.0 - rho) * float(np.exp(np.log(a).mean()))
        return 0.5 * (1.0 + torch.erf(d / (math.sqrt(2.0) * self.edge)))

    def __call__(self, pts: torch.Tensor) -> torch.Tensor:
        out = torch.zeros(pts.shape[1:], dtype=torch.float64, device=pts.device)
        for a in self.axes:
            out += 0.3 * self._layer(pts, a)
        if self.texture:
            out += self.texture * self._layer(pts, self.axes[0]) * _eval_field(self.tex, pts)[0]
        return out.clamp_min(0.0)


def _series_positions(vs: List[torch.Tensor], k: int, g: torch.Tensor, steps: int) -> torch.Tensor:
    """Positions at which the base image is read for session k: the time-1
    flows of v_{k-1}, ..., v_0 applied in that order to the grid."""
    pts = g
    for i in range(k - 1, -1, -1):
        pts = flow(vs[i], pts, 1.0, steps)
    return pts


def blobs_series(shape=(32, 32, 32), N=3, seed=1, n_blobs=20, sigma_v=4.0, vmax=1.0,
                 noise=0.01, device="cpu", steps=8) -> Series:
    """Blob image B; session k (0-based) is B pulled back along the time-k flow
    of one smoothed random field v, plus Gaussian noise."""
    rng = _rng(seed)
    B = Blobs(shape, n_blobs, rng)
    v = random_velocity(shape, sigma_v, vmax, rng, device)
    g = _grid(shape, device)
    imgs = []
    for k in range(N):
        pts = _series_positions([v] * (N - 1), k, g, steps)
        clean = B(pts)
        n = torch.from_numpy(rng.standard_normal(shape)).to(device) * noise
        imgs.append(clean + n)
    images = torch.stack(imgs).float().contiguous()
    times = np.arange(N, dtype=np.float64)
    svf = torch.stack([-v] * (N - 1)).float().contiguous()
    r = 2
    roi = torch.zeros(shape, dtype=torch.bool, device=device)
    roi[r:-r, r:-r, r:-r] = True
    return Series(images, times, svf, roi, f"blobs{shape}")


def phantom_series(shape=(64, 64, 64), N=4, seed=2, sigma_v=6.0, amp=(0.5, 1.5),
                   bias_sigma=32.0, bias_amp=0.1, noise=0.02, interval=(0.5, 2.0),
                   device="cpu", steps=8) -> Series:
    """Phantom series with per-interval velocity fields, unevenly spaced times,
    a per-session smooth multiplicative bias and Rician noise."""
    rng = _rng(seed)
    P = Phantom(shape, rng, device=device)
    gaps = rng.uniform(interval[0], interval[1], N - 1)
    times = np.concatenate([[0.0], np.cumsum(gaps)])
    amps = rng.uniform(amp[0], amp[1], N - 1)
    vs = [random_velocity(shape, sigma_v, float(a), rng, device) for a in amps]
    g = _grid(shape, device)
    imgs = []
    for k in range(N):
        pts = _series_positions(vs, k, g, steps)
        clean = P(pts)
        bn = torch.from_numpy(rng.standard_normal(shape)).to(device)
        b = gaussian_smooth(bn, bias_sigma)
        b = b / b.abs().max()
        x = clean * (1.0 + bias_amp * b)
        n1 = torch.from_numpy(rng.standard_normal(shape)).to(device) * noise
        n2 = torch.from_numpy(rng.standard_normal(shape)).to(device) * noise
        imgs.append(torch.sqrt((x + n1) ** 2 + n2 ** 2))
    images = torch.stack(imgs).float().contiguous()
    svf = torch.stack([-v for v in vs]).float().contiguous()
    roi = P._layer(g, P.axes[0]) > 0.5
    return Series(images, times, svf, roi, f"phantom{shape}")


# ---------------------------------------------------------------------------
# The evaluation workloads
# ---------------------------------------------------------------------------

SIZES = ((96, 96, 96), (128, 128, 128), (160, 192, 160))


def blobs_3x32(device="cpu") -> Series:
    """One subject, three 32^3 sessions of 20 blobs, flowed for t = 1, 2."""
    return blobs_series((32, 32, 32), 3, seed=1, device=device)


def phantoms_6x160x192x160(device="cpu", shape=(160, 192, 160)) -> Series:
    """One subject, six 160x192x160 phantom sessions."""
    return phantom_series(shape, 6, seed=2, device=device)


def phantoms_4x64(device="cpu") -> Series:
    """Four 64^3 phantom sessions (gradient check)."""
    return phantom_series((64, 64, 64), 4, seed=3, device=device)


def subject_draw(seed: int, sizes=SIZES):
    """Session count and volume size of one subject of the batched and served
    workloads: N uniform on 3..10, size uniform over `sizes`."""
    rng = _rng(seed)
    N = int(rng.integers(3, 11))
    shape = tuple(sizes[int(rng.integers(0, len(sizes)))])
    return N, shape


def batch_subject(seed: int, device="cpu", shape=None, N=None) -> Series:
    n0, s0 = subject_draw(seed)
    return phantom_series(shape or s0, N or n0, seed=seed, device=device)
