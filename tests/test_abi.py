"""Host-side checks of the C ABI: the library loads, exports every entry point
include/muster.h declares, and validates arguments without touching a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2412_14671_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "muster.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(muster_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_library_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 25
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (muster_[a-z0-9_]+)", out))
    missing = [n for n in names if n not in exported]
    assert missing == []
    # and the binding declares a signature for each of them
    assert sorted(L.SIGNATURES) == names


def test_struct_layouts_match_the_header(lib, tmp_path):
    """The ctypes structures agree with the C compiler's view of muster.h."""
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "muster.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(muster_params), offsetof(muster_params, K),
         offsetof(muster_params, alpha_ss), offsetof(muster_params, use_graph),
         sizeof(muster_report), offsetof(muster_report, footprint_bytes),
         sizeof(muster_job), offsetof(muster_job, params));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(L.Params), L.Params.K.offset, L.Params.alpha_ss.offset,
            L.Params.use_graph.offset, ctypes.sizeof(L.Report), L.Report.footprint_bytes.offset,
            ctypes.sizeof(L.Job), L.Job.params.offset]
    assert got == want


def test_params_default(lib):
    p = L.Params()
    assert lib.muster_params_default(ctypes.byref(p)) == L.OK
    assert (p.levels, p.iters[0], p.K, p.window, p.metric) == (1, 100, 7, 5, L.METRIC_LNCC)
    assert abs(p.warmup - 0.2) < 1e-7 and abs(p.alpha_ss - 1.0) < 1e-7
    assert p.exp_mode == L.EXP_STORE and p.use_graph == 1 and p.smooth_sigma == 0.0
    assert p.alpha_l2 == 0.0 and p.alpha_ts == 0.0


def _fp(lib, N, dims, **kw):
    p = L.Params()
    lib.muster_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k == "iters":
            for i, n in enumerate(v):
                p.iters[i] = n
        else:
            setattr(p, k, v)
    b = ctypes.c_uint64()
    st = lib.muster_footprint(N, L.DIMS(*dims), ctypes.byref(p), ctypes.byref(b))
    return st, b.value


def test_footprint_counts_fields(lib):
    st, b = _fp(lib, 3, (32, 32, 32))
    assert st == L.OK
    F = 3 * 32 ** 3 * 4
    # phi, m, v (2 each) + 4 dirs x 7 steps + 2 deep + 6 pair grads + 8 ping-pong + 6 coef
    # + 2 combined SVF gradients of the staged Exp adjoint
    fields = 3 * 2 + 4 * 7 + 2 + 6 + 8 + 6 + 2
    # Exp-backward staging: 2 steps x 4 directions x 32 tiles of 8x8x16, each a
    # slot of 3 x 2048 floats and an 8-int descriptor
    staging = 2 * 4 * 32 * (3 * 2048 * 4 + 8 * 4)
    assert fields * F + staging <= b <= fields * F + staging + 200_000
    st2, b2 = _fp(lib, 3, (32, 32, 32), exp_mode=L.EXP_RECOMPUTE)
    assert st2 == L.OK and b2 == b - 4 * (7 - 3) * F
    st3, b3 = _fp(lib, 10, (160, 192, 160))
    assert st3 == L.OK and 20e9 < b3 < 40e9
    st4, b4 = _fp(lib, 3, (32, 32, 32), smooth_sigma=1.5)
    # smoothing: the smoothed flow and a second gradient buffer (t1 is there already)
    assert st4 == L.OK and b4 == b + 2 * 2 * F


@pytest.mark.parametrize("N,dims,kw", [
    (1, (32, 32, 32), {}),                       # one session
    (65, (32, 32, 32), {}),                      # more sessions than a job holds
    (3, (1024, 1024, 1024), {}),                 # 3 V beyond 32-bit offsets
    (3, (896, 896, 892), {}),                    # the first volume past that limit
    (3, (32, 32, 4), {}),                        # smaller than the window
    (3, (32, 32, 30), {"levels": 3, "iters": (1, 1, 1)}),  # not divisible by 4
    (3, (32, 32, 32), {"window": 4}),            # even window
    (3, (32, 32, 32), {"window": 9}),
    (3, (32, 32, 32), {"K": 0}),
    (3, (32, 32, 32), {"K": 21}),
    (3, (32, 32, 32), {"metric": 7}),
    (3, (32, 32, 32), {"levels": 0}),
    (3, (32, 32, 32), {"warmup": 1.5}),
    (3, (32, 32, 32), {"smooth_sigma": -1.0}),
    (3, (32, 32, 32), {"smooth_sigma": 30.0}),   # above the largest width
    (3, (16, 16, 520), {"smooth_sigma": 0.5}),   # taps span a line longer than 257
    (3, (32, 32, 32), {"alpha_l2": -0.5}),
    (3, (32, 32, 32), {"alpha_ts": float("nan")}),
])
def test_footprint_rejects_invalid_problems(lib, N, dims, kw):
    st, _ = _fp(lib, N, dims, **kw)
    assert st == L.E_INVALID
    assert lib.muster_last_error()


def test_largest_accepted_problem(lib):
    """The limits at their edge: 64 sessions, and the largest volume whose
    three component planes stay within 32-bit offsets (3 V < 2^31 - 1)."""
    st, b = _fp(lib, 64, (32, 32, 32))
    assert st == L.OK and b > 0
    assert 3 * 896 * 896 * 890 < 2 ** 31 - 1 <= 3 * 896 * 896 * 892
    st, b = _fp(lib, 2, (896, 896, 890))
    assert st == L.OK and b > 3 * 896 * 896 * 890 * 4


def test_null_arguments_are_rejected(lib):
    assert lib.muster_params_default(None) == L.E_INVALID
    assert lib.muster_ctx_create(0, 0, None) == L.E_INVALID
    assert lib.muster_ctx_destroy(None) == L.OK
    assert lib.muster_saved_free(None) == L.OK
    # entry points that need a context refuse a NULL one before touching HIP
    assert lib.muster_register(None, None, 3, L.DIMS(8, 8, 8), None, None, None, None, None,
                               None) == L.E_INVALID
    assert lib.muster_set_kernel_timing(None, 1) == L.E_INVALID
    assert lib.muster_set_kernel_timing_mask(None, 1) == L.E_INVALID


def test_kernel_names(lib):
    names = [lib.muster_kernel_name(k).decode() for k in range(len(L.KERNELS))]
    assert names == L.KERNELS
    assert lib.muster_kernel_name(99) == b""


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present")
def test_context_creation_without_a_gpu_fails_cleanly(lib):
    h = ctypes.c_void_p()
    st = lib.muster_ctx_create(0, 0, ctypes.byref(h))
    assert st in (L.E_DEVICE, L.E_INVALID)
    assert lib.muster_last_error()
