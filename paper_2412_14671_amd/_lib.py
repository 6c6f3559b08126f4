"""ctypes binding of libmuster.so (the C ABI declared in include/muster.h).

Argument marshalling only: every step of the registration path runs in the
library's HIP kernels.  Importing this module does not touch the GPU; loading
the library raises MusterLibraryMissing if it has not been built, so no code
path can silently fall back to something else.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_char_p, c_double, c_float, c_int, c_int64, c_uint32, c_uint64,
                    c_void_p)

HERE = os.path.dirname(os.path.abspath(__file__))
# MUSTER_LIB names another build of the library (the host-sanitizer build of
# the CPU-side tests); by default the in-tree libmuster.so
LIB_PATH = os.environ.get("MUSTER_LIB") or os.path.join(HERE, "libmuster.so")
MAX_LEVELS = 6

OK, E_INVALID, E_NOMEM, E_DEVICE, E_BUSY, E_NONFINITE, E_CANCELLED, E_INTERNAL = range(8)
STATUS_NAMES = ["OK", "E_INVALID", "E_NOMEM", "E_DEVICE", "E_BUSY", "E_NONFINITE",
                "E_CANCELLED", "E_INTERNAL"]
METRIC_LNCC, METRIC_SILNCC = 0, 1
TILES_DEFAULT, TILES_AUTOTUNE, TILES_FIXED = 0, 1, 2
SIM_SHAPES = [(8, 32), (16, 32), (8, 64)]
EXP_STORE, EXP_RECOMPUTE = 0, 1
EXP_FLAT = 4  # MUSTER_EXP_FLAT: or-ed into the mode of muster_exp_bwd
KERNELS = ["exp_fwd", "compose_fwd", "sim_stats", "sim_grad", "compose_bwd", "exp_bwd", "adam",
           "finish", "pool2", "upsample2", "smooth", "upsample2_adj", "rigid", "warp", "unstage"]


class MusterLibraryMissing(ImportError):
    pass


class MusterError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {message}")


class Params(Structure):
    _fields_ = [("levels", c_int), ("iters", c_int * MAX_LEVELS), ("K", c_int), ("window", c_int),
                ("metric", c_int), ("alpha_ss", c_float), ("lr", c_float), ("warmup", c_float),
                ("beta1", c_float), ("beta2", c_float), ("eps", c_float), ("exp_mode", c_int),
                ("use_graph", c_int), ("smooth_sigma", c_float), ("alpha_l2", c_float),
                ("alpha_ts", c_float), ("flow_factor", c_int), ("rigid", c_int),
                ("deterministic", c_int)]


class Report(Structure):
    _fields_ = [("status", c_int), ("iterations", c_int), ("loss_first", c_double),
                ("loss_last", c_double), ("seconds", c_double), ("queue_seconds", c_double),
                ("footprint_bytes", c_uint64), ("step_seconds", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Job(Structure):
    _fields_ = [("N", c_int), ("dims", c_int * 3), ("images_dev", c_void_p),
                ("times_host", POINTER(c_double)), ("svf_init_dev", c_void_p),
                ("svf_out_dev", c_void_p), ("pairs_out_dev", c_void_p), ("params", Params),
                ("rigid_out_dev", c_void_p)]


DIMS = c_int * 3
_P = c_void_p
_ST = c_int

# name -> (restype, argtypes)
SIGNATURES = {
    "muster_ctx_create": (_ST, [c_int, c_uint64, POINTER(_P)]),
    "muster_ctx_destroy": (_ST, [_P]),
    "muster_last_error": (c_char_p, []),
    "muster_version": (c_char_p, []),
    "muster_params_default": (_ST, [POINTER(Params)]),
    "muster_footprint": (_ST, [c_int, DIMS, POINTER(Params), POINTER(c_uint64)]),
    "muster_register": (_ST, [_P, _P, c_int, DIMS, _P, POINTER(c_double), POINTER(Params), _P, _P,
                              POINTER(Report)]),
    "muster_register_batch": (_ST, [_P, _P, c_int, POINTER(Job), POINTER(Report)]),
    "muster_server_start": (_ST, [_P, c_int]),
    "muster_submit": (_ST, [_P, POINTER(Job), POINTER(c_uint64)]),
    "muster_poll": (_ST, [_P, c_uint64, POINTER(c_int)]),
    "muster_wait": (_ST, [_P, c_uint64, POINTER(Report)]),
    "muster_cancel": (_ST, [_P, c_uint64]),
    "muster_server_stats": (_ST, [_P, POINTER(c_int), POINTER(c_int), POINTER(c_uint64)]),
    "muster_loss_forward": (_ST, [_P, _P, c_int, DIMS, _P, POINTER(c_double), _P, POINTER(Params),
                                  POINTER(c_double), POINTER(_P)]),
    "muster_loss_backward": (_ST, [_P, _P, _P, c_double, _P]),
    "muster_saved_free": (_ST, [_P]),
    "muster_exp": (_ST, [_P, _P, DIMS, c_int, c_int, _P, _P, _P]),
    "muster_exp_bwd": (_ST, [_P, _P, DIMS, c_int, c_int, _P, _P, _P, c_int]),
    "muster_compose": (_ST, [_P, _P, DIMS, _P, _P, _P]),
    "muster_compose_bwd": (_ST, [_P, _P, DIMS, _P, _P, _P, _P, _P]),
    "muster_sim": (_ST, [_P, _P, DIMS, c_int, c_int, _P, _P, _P, POINTER(c_double), _P]),
    "muster_sim_noalloc": (_ST, [_P, _P, DIMS, c_int, c_int, _P, _P, _P, POINTER(c_double), _P]),
    "muster_adam": (_ST, [_P, _P, c_int64, _P, _P, _P, _P, c_int, c_float, c_float, c_float,
                          c_float]),
    "muster_reg": (_ST, [_P, _P, DIMS, _P, POINTER(c_double), _P]),
    "muster_pool2": (_ST, [_P, _P, DIMS, _P, _P]),
    "muster_upsample2": (_ST, [_P, _P, DIMS, _P, _P]),
    "muster_upsample2_adjoint": (_ST, [_P, _P, DIMS, _P, _P]),
    "muster_jacobian_det": (_ST, [_P, _P, DIMS, _P, _P]),
    "muster_field_metrics": (_ST, [_P, _P, DIMS, _P, _P, _P, POINTER(c_double), POINTER(c_double),
                                   POINTER(c_double)]),
    "muster_smooth": (_ST, [_P, _P, DIMS, c_float, _P, _P]),
    "muster_ctx_set_tiling": (_ST, [_P, c_int, c_int, c_int]),
    "muster_ctx_memory": (_ST, [_P, POINTER(c_uint64), POINTER(c_uint64), c_int]),
    "muster_ctx_trim": (_ST, [_P, POINTER(c_uint64)]),
    "muster_ctx_sim_tiling": (_ST, [_P, _P, DIMS, c_int, c_int, POINTER(c_int), POINTER(c_int)]),
    "muster_set_kernel_timing": (_ST, [_P, c_int]),
    "muster_set_kernel_timing_mask": (_ST, [_P, c_uint32]),
    "muster_kernel_stats": (_ST, [_P, POINTER(c_int64), POINTER(c_double), POINTER(c_double)]),
    "muster_kernel_stats_reset": (_ST, [_P]),
    "muster_kernel_name": (c_char_p, [c_int]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libmuster.so and declare every entry point; raises
    MusterLibraryMissing when the library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise MusterLibraryMissing(
            f"{path} not found: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != OK:
        msg = load().muster_last_error()
        raise MusterError(status, msg.decode() if msg else "")
