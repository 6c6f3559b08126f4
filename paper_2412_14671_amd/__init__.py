"""MI355X (gfx950) implementation of the MUSTER registration hot path.

The work runs in hand-written HIP kernels behind the C ABI of
include/muster.h (libmuster.so in this package directory); this package holds
the ctypes binding (_lib), the torch-facing API (api) and the seeded input
generators (synth).
"""
from .api import Context, MusterLoss, MusterParams, Server, loss_value, register  # noqa: F401
from ._lib import MusterError, MusterLibraryMissing  # noqa: F401

__version__ = "0.1.0"
