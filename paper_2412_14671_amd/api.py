"""Python surface of the MUSTER path: a thin layer over the C ABI that takes
torch CUDA tensors (PyTorch supplies device memory and the current stream) and
calls the library's HIP kernels.  Nothing here computes any step of the method.
"""
from __future__ import annotations

import ctypes
import dataclasses
from ctypes import byref, c_double, c_int, c_int64, c_uint64, c_void_p
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L


@dataclasses.dataclass
class MusterParams:
    """Optimisation parameters (paper Sec. 2.3, 2.4, 2.6, 2.7)."""
    iters: Sequence[int] = (100,)     # Adam steps per pyramid level, coarse to fine
    K: int = 7                        # squarings in Exp
    window: int = 5                   # window edge w
    metric: str = "lncc"              # "lncc" or "silncc"
    alpha_ss: float = 1.0             # weight of the diffusion regulariser
    lr: float = 0.1                   # peak learning rate, voxels per step
    warmup: float = 0.2               # warm-up fraction of each level
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    exp_mode: str = "store"           # "store" or "recompute"
    use_graph: bool = True
    smooth_sigma: float = 0.0         # Gaussian smoothing of the flow, finest-level voxels
    alpha_l2: float = 0.0             # weight of L_L2 (flow magnitude)
    alpha_ts: float = 0.0             # weight of L_ts (temporal smoothness; needs times)
    flow_factor: int = 1              # 2: flows on a grid twice as coarse as the images
    rigid: bool = False               # rigid adjustment of every session but the first
    deterministic: bool = False       # results independent of the order of atomic adds

    def to_c(self) -> L.Params:
        p = L.Params()
        it = list(self.iters)
        if not 1 <= len(it) <= L.MAX_LEVELS:
            raise ValueError(f"1..{L.MAX_LEVELS} pyramid levels required")
        p.levels = len(it)
        for i, n in enumerate(it):
            p.iters[i] = int(n)
        p.K = int(self.K)
        p.window = int(self.window)
        p.metric = {"lncc": L.METRIC_LNCC, "silncc": L.METRIC_SILNCC}[self.metric.lower()]
        p.alpha_ss = float(self.alpha_ss)
        p.lr = float(self.lr)
        p.warmup = float(self.warmup)
        p.beta1, p.beta2, p.eps = float(self.beta1), float(self.beta2), float(self.eps)
        p.exp_mode = {"store": L.EXP_STORE, "recompute": L.EXP_RECOMPUTE}[self.exp_mode]
        p.use_graph = 1 if self.use_graph else 0
        p.smooth_sigma = float(self.smooth_sigma)
        p.alpha_l2 = float(self.alpha_l2)
        p.alpha_ts = float(self.alpha_ts)
        p.flow_factor = int(self.flow_factor)
        p.rigid = 1 if self.rigid else 0
        p.deterministic = 1 if self.deterministic else 0
        return p


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("expected a contiguous float32 CUDA tensor")
    return c_void_p(t.data_ptr())


def _dims(shape) -> L.DIMS:
    return L.DIMS(*[int(s) for s in shape])


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A library context on one GPU (workspace arena, streams, graphs)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self.lib = L.load()
        self.device = device
        h = c_void_p()
        with torch.cuda.device(device):
            L.check(self.lib.muster_ctx_create(device, budget_bytes, byref(h)))
        self.h = h
        self._server = False

    def close(self):
        if self.h:
            self.lib.muster_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- single steps ---------------------------------------------------------------
    def exp(self, svf: torch.Tensor, K: int, sign: int = 1, steps: bool = False):
        """Exp(sign*svf) - Omega; with steps=True also returns u_1..u_K."""
        out = torch.empty_like(svf)
        st = torch.empty((K,) + tuple(svf.shape), device=svf.device) if steps else None
        L.check(self.lib.muster_exp(self.h, _stream(), _dims(svf.shape[1:]), K, sign, _ptr(svf),
                                    _ptr(out), _ptr(st)))
        return (out, st) if steps else out

    def exp_bwd(self, svf, grad_disp, K, sign=1, mode="store", flat=False):
        """Adjoint of exp.  flat=False (the default) runs the staged exchange
        between squaring steps that the registration runs; flat=True the
        flat path with global atomics."""
        out = torch.empty_like(svf)
        m = {"store": L.EXP_STORE, "recompute": L.EXP_RECOMPUTE}[mode]
        if flat:
            m |= L.EXP_FLAT
        L.check(self.lib.muster_exp_bwd(self.h, _stream(), _dims(svf.shape[1:]), K, sign,
                                        _ptr(svf), _ptr(grad_disp), _ptr(out), m))
        return out

    def compose(self, U_prev, C):
        out = torch.empty_like(U_prev)
        L.check(self.lib.muster_compose(self.h, _stream(), _dims(U_prev.shape[1:]), _ptr(U_prev),
                                        _ptr(C), _ptr(out)))
        return out

    def compose_bwd(self, U_prev, C, G, G_prev, G_C):
        L.check(self.lib.muster_compose_bwd(self.h, _stream(), _dims(U_prev.shape[1:]),
                                            _ptr(U_prev), _ptr(C), _ptr(G), _ptr(G_prev),
                                            _ptr(G_C)))

    # -- tiling of the window statistics ---------------------------------------------
    def set_tiling(self, mode: str = "autotune", shape: int = 0, zchunk: int = 32):
        """mode "default" (8x32 centres, 32 slices), "autotune" or "fixed"."""
        m = {"default": L.TILES_DEFAULT, "autotune": L.TILES_AUTOTUNE, "fixed": L.TILES_FIXED}[mode]
        L.check(self.lib.muster_ctx_set_tiling(self.h, m, shape, zchunk))

    def sim_tiling(self, dims, window=7, metric="silncc"):
        """(shape index, z chunk) the context uses for this problem shape."""
        m = {"lncc": L.METRIC_LNCC, "silncc": L.METRIC_SILNCC}[metric]
        sh, zc = c_int(), c_int()
        L.check(self.lib.muster_ctx_sim_tiling(self.h, _stream(), _dims(dims), window, m, byref(sh),
                                               byref(zc)))
        return sh.value, zc.value

    def sim(self, F, I, U, window, metric="lncc", grad=False):
        m = {"lncc": L.METRIC_LNCC, "silncc": L.METRIC_SILNCC}[metric]
        val = c_double()
        g = torch.empty_like(U) if grad else None
        L.check(self.lib.muster_sim(self.h, _stream(), _dims(F.shape), window, m, _ptr(F), _ptr(I),
                                    _ptr(U), byref(val), _ptr(g)))
        return (val.value, g) if grad else val.value

    def sim_noalloc(self, F, I, U, window, metric="lncc", grad=False):
        """sim() through the entry point that allocates no device memory."""
        m = {"lncc": L.METRIC_LNCC, "silncc": L.METRIC_SILNCC}[metric]
        val = c_double()
        g = torch.empty_like(U) if grad else None
        L.check(self.lib.muster_sim_noalloc(self.h, _stream(), _dims(F.shape), window, m, _ptr(F),
                                            _ptr(I), _ptr(U), byref(val), _ptr(g)))
        return (val.value, g) if grad else val.value

    def adam(self, x, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        L.check(self.lib.muster_adam(self.h, _stream(), c_int64(x.numel()), _ptr(x), _ptr(g),
                                     _ptr(m), _ptr(v), t, lr, beta1, beta2, eps))

    def reg(self, phi, grad=False):
        val = c_double()
        g = torch.empty_like(phi) if grad else None
        L.check(self.lib.muster_reg(self.h, _stream(), _dims(phi.shape[1:]), _ptr(phi), byref(val),
                                    _ptr(g)))
        return (val.value, g) if grad else val.value

    def pool2(self, img):
        D, H, W = img.shape
        out = torch.empty((D // 2, H // 2, W // 2), device=img.device)
        L.check(self.lib.muster_pool2(self.h, _stream(), _dims(img.shape), _ptr(img), _ptr(out)))
        return out

    def smooth(self, svf, sigma):
        out = torch.empty_like(svf)
        L.check(self.lib.muster_smooth(self.h, _stream(), _dims(svf.shape[1:]), float(sigma),
                                       _ptr(svf), _ptr(out)))
        return out

    def upsample2(self, svf):
        _, D, H, W = svf.shape
        out = torch.empty((3, 2 * D, 2 * H, 2 * W), device=svf.device)
        L.check(self.lib.muster_upsample2(self.h, _stream(), _dims(svf.shape[1:]), _ptr(svf),
                                          _ptr(out)))
        return out

    def upsample2_adjoint(self, g):
        """Adjoint of upsample2: g [3, 2D, 2H, 2W] -> [3, D, H, W]."""
        _, D2, H2, W2 = g.shape
        out = torch.empty((3, D2 // 2, H2 // 2, W2 // 2), device=g.device)
        L.check(self.lib.muster_upsample2_adjoint(self.h, _stream(), _dims(out.shape[1:]), _ptr(g),
                                                  _ptr(out)))
        return out

    # -- outputs and evaluation -------------------------------------------------------
    def jacobian_det(self, U):
        """det(I + grad U) per voxel for a displacement field U [3, D, H, W]."""
        out = torch.empty(tuple(U.shape[1:]), device=U.device)
        L.check(self.lib.muster_jacobian_det(self.h, _stream(), _dims(U.shape[1:]), _ptr(U),
                                             _ptr(out)))
        return out

    def field_metrics(self, ref, est, roi=None):
        """(Eu, PCC, slope) of est against ref over roi (bool [D, H, W] or None)."""
        r = None
        if roi is not None:
            r = roi.to(device=ref.device, dtype=torch.uint8).contiguous()
        eu, pcc, sl = c_double(), c_double(), c_double()
        L.check(self.lib.muster_field_metrics(self.h, _stream(), _dims(ref.shape[1:]), _ptr(ref),
                                              _ptr(est), None if r is None else c_void_p(r.data_ptr()),
                                              byref(eu), byref(pcc), byref(sl)))
        return eu.value, pcc.value, sl.value

    # -- whole registrations -----------------------------------------------------
    def footprint(self, N, dims, params: MusterParams) -> int:
        b = c_uint64()
        p = params.to_c()
        L.check(self.lib.muster_footprint(N, _dims(dims), byref(p), byref(b)))
        return b.value

    def register(self, images: torch.Tensor, times=None, params: Optional[MusterParams] = None,
                 pairs: bool = False):
        """Register a series images[N, D, H, W]; returns (svf, pairs or None,
        report dict).  With params.rigid the report also holds "rigid": the
        [N-1, 6] angles (radians) and translations (voxels) of sessions
        1..N-1, and the pairs are the total deformations."""
        params = params or MusterParams()
        if params.rigid:
            N = images.shape[0]
            svf = torch.empty((N - 1, 3) + tuple(images.shape[1:]), device=images.device)
            pr = torch.empty((N * (N - 1), 3) + tuple(images.shape[1:]), device=images.device) \
                if pairs else None
            rig = torch.empty((N - 1, 6), device=images.device)
            keep = []
            jobs = (L.Job * 1)()
            jobs[0] = self._job(images, times, params, svf, pr, keep=keep)
            jobs[0].rigid_out_dev = _ptr(rig)
            reps = (L.Report * 1)()
            L.check(self.lib.muster_register_batch(self.h, _stream(), 1, jobs, reps))
            rep = reps[0].as_dict()
            rep["rigid"] = rig
            return svf, pr, rep
        N = images.shape[0]
        svf = torch.empty((N - 1, 3) + tuple(images.shape[1:]), device=images.device)
        pr = torch.empty((N * (N - 1), 3) + tuple(images.shape[1:]), device=images.device) \
            if pairs else None
        t = np.ascontiguousarray(np.arange(N, dtype=np.float64) if times is None else times,
                                 dtype=np.float64)
        rep = L.Report()
        p = params.to_c()
        L.check(self.lib.muster_register(self.h, _stream(), N, _dims(images.shape[1:]),
                                         _ptr(images), t.ctypes.data_as(ctypes.POINTER(c_double)),
                                         byref(p), _ptr(svf), _ptr(pr), byref(rep)))
        return svf, pr, rep.as_dict()

    def _job(self, images, times, params, svf_out, pairs_out, svf_init=None, keep=None):
        N = images.shape[0]
        t = np.ascontiguousarray(np.arange(N, dtype=np.float64) if times is None else times,
                                 dtype=np.float64)
        if keep is not None:
            keep.append(t)
        j = L.Job()
        j.N = N
        j.dims = _dims(images.shape[1:])
        j.images_dev = _ptr(images)
        j.times_host = t.ctypes.data_as(ctypes.POINTER(c_double))
        j.svf_init_dev = _ptr(svf_init)
        j.svf_out_dev = _ptr(svf_out)
        j.pairs_out_dev = _ptr(pairs_out)
        j.params = params.to_c()
        return j

    def register_batch(self, series: List[torch.Tensor], times=None,
                       params: Optional[MusterParams] = None):
        """Register many subjects in one batched, graph-replayed loop; returns
        ([svf], [report])."""
        params = params or MusterParams()
        keep = []
        outs = [torch.empty((x.shape[0] - 1, 3) + tuple(x.shape[1:]), device=x.device) for x in series]
        jobs = (L.Job * len(series))()
        for k, x in enumerate(series):
            jobs[k] = self._job(x, None if times is None else times[k], params, outs[k], None,
                                keep=keep)
        reps = (L.Report * len(series))()
        L.check(self.lib.muster_register_batch(self.h, _stream(), len(series), jobs, reps))
        return outs, [r.as_dict() for r in reps]

    # -- kernel timing -------------------------------------------------------------
    def set_kernel_timing(self, on: bool):
        L.check(self.lib.muster_set_kernel_timing(self.h, 1 if on else 0))

    def set_kernel_timing_only(self, kernels):
        """Time the eager launches of the named kernel classes only (names as
        in kernel_stats); an empty list turns timing off."""
        mask = 0
        for k in kernels:
            mask |= 1 << L.KERNELS.index(k)
        L.check(self.lib.muster_set_kernel_timing_mask(self.h, mask))

    def kernel_stats(self) -> Dict[str, dict]:
        n = len(L.KERNELS)
        la = (c_int64 * n)()
        ms = (c_double * n)()
        by = (c_double * n)()
        L.check(self.lib.muster_kernel_stats(self.h, la, ms, by))
        return {L.KERNELS[k]: {"launches": la[k], "ms": ms[k], "bytes": by[k]} for k in range(n)}

    def kernel_stats_reset(self):
        L.check(self.lib.muster_kernel_stats_reset(self.h))

    # -- workspace memory ------------------------------------------------------------
    def memory(self, reset_peak: bool = False) -> Dict[str, int]:
        """Device bytes the library's arena holds now and at most since the
        mark was last reset (then resets the mark if asked)."""
        u, pk = c_uint64(), c_uint64()
        L.check(self.lib.muster_ctx_memory(self.h, byref(u), byref(pk), 1 if reset_peak else 0))
        return {"in_use": u.value, "peak": pk.value}

    def trim(self) -> int:
        """Return the workspaces the context keeps for reuse to the device;
        the bytes returned."""
        b = c_uint64()
        L.check(self.lib.muster_ctx_trim(self.h, byref(b)))
        return b.value


def register(images: torch.Tensor, times=None, pairs=False, ctx: Optional[Context] = None,
             **params):
    """muster.register(images[N, D, H, W], times, **params) -> (svf, pairs)."""
    c = ctx or Context(images.device.index or 0)
    svf, pr, _ = c.register(images, times, MusterParams(**params), pairs=pairs)
    return svf, pr


class _Saved:
    """Owner of a muster_saved handle: freed by the backward pass, or when the
    autograd graph holding it is dropped without one."""

    def __init__(self, owner: "Context", handle):
        self.owner, self.handle = owner, handle

    def free(self):
        # a context closed first has already let go of the job's memory
        if self.handle is not None and self.handle.value and self.owner.h:
            self.owner.lib.muster_saved_free(self.handle)
        self.handle = None

    def __del__(self):
        self.free()


def _loss_forward(lib_ctx: "Context", svf_c, img_c, params: MusterParams, times):
    loss = c_double()
    saved = c_void_p()
    p = params.to_c()
    tarr = None
    if times is not None:
        tarr = (c_double * img_c.shape[0])(*[float(t) for t in times])
    L.check(lib_ctx.lib.muster_loss_forward(lib_ctx.h, _stream(), img_c.shape[0],
                                            _dims(img_c.shape[1:]), _ptr(img_c), tarr,
                                            _ptr(svf_c), byref(p), byref(loss), byref(saved)))
    return loss.value, _Saved(lib_ctx, saved)


def loss_value(svf: torch.Tensor, images: torch.Tensor, params: MusterParams, lib_ctx: "Context",
               times=None) -> float:
    """L(phi) only (no state kept for a backward pass)."""
    val, saved = _loss_forward(lib_ctx, svf.detach().contiguous(), images.detach().contiguous(),
                               params, times)
    saved.free()
    return val


class MusterLoss(torch.autograd.Function):
    """L(phi) of the MUSTER objective at one grid as a differentiable function
    of the SVFs; forward and backward are the library's kernels (hand-written
    adjoints)."""

    @staticmethod
    def forward(ctx, svf, images, params: MusterParams, lib_ctx: Context, times=None):
        svf_c = svf.detach().contiguous()
        img_c = images.detach().contiguous()
        val, saved = _loss_forward(lib_ctx, svf_c, img_c, params, times)
        if not ctx.needs_input_grad[0]:
            saved.free()
        ctx.lib_ctx = lib_ctx
        ctx.saved = saved
        ctx.keep = (svf_c, img_c)
        return torch.tensor(val, dtype=torch.float64, device=svf.device)

    @staticmethod
    def backward(ctx, grad_out):
        lib = ctx.lib_ctx.lib
        svf_c, _ = ctx.keep
        g = torch.empty_like(svf_c)
        if ctx.saved.handle is None:
            raise RuntimeError("the saved state of this loss was already used or freed")
        try:
            L.check(lib.muster_loss_backward(ctx.lib_ctx.h, _stream(), ctx.saved.handle,
                                             float(grad_out), _ptr(g)))
        finally:
            ctx.saved.free()
        return g, None, None, None, None


class Server:
    """Continuous-batching registration server on a context."""

    def __init__(self, ctx: Context, max_queue: int = 4096):
        self.ctx = ctx
        L.check(ctx.lib.muster_server_start(ctx.h, max_queue))
        self._keep: Dict[int, list] = {}

    def submit(self, images, times=None, params: Optional[MusterParams] = None, svf_out=None):
        params = params or MusterParams()
        if svf_out is None:
            svf_out = torch.empty((images.shape[0] - 1, 3) + tuple(images.shape[1:]),
                                  device=images.device)
        keep = [images, svf_out]
        j = self.ctx._job(images, times, params, svf_out, None, keep=keep)
        tk = c_uint64()
        L.check(self.ctx.lib.muster_submit(self.ctx.h, byref(j), byref(tk)))
        self._keep[tk.value] = keep
        return tk.value, svf_out

    def poll(self, ticket) -> int:
        s = c_int()
        L.check(self.ctx.lib.muster_poll(self.ctx.h, ticket, byref(s)))
        return s.value

    def wait(self, ticket) -> dict:
        rep = L.Report()
        st = self.ctx.lib.muster_wait(self.ctx.h, ticket, byref(rep))
        self._keep.pop(ticket, None)
        d = rep.as_dict()
        d["status"] = st
        if st != L.OK:
            msg = self.ctx.lib.muster_last_error()
            d["error"] = msg.decode() if msg else ""
        return d

    def cancel(self, ticket):
        L.check(self.ctx.lib.muster_cancel(self.ctx.h, ticket))

    def stats(self):
        r, q, b = c_int(), c_int(), c_uint64()
        L.check(self.ctx.lib.muster_server_stats(self.ctx.h, byref(r), byref(q), byref(b)))
        return {"resident": r.value, "queued": q.value, "bytes": b.value}
