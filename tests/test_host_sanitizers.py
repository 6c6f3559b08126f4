"""The host runtime (context, validation, footprint, plans, the C ABI's error
paths) built with AddressSanitizer and UndefinedBehaviorSanitizer, g++ on the
host code only, and the C-ABI tests run against that build in a child
process (CPU only: no kernel is launched)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_14671_amd", "csrc")
LIB = os.path.join(ROOT, "_build", "libmuster_asan.so")

pytestmark = pytest.mark.slow


def _gcc_lib(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                          check=True).stdout.strip()


def test_abi_tests_pass_under_host_asan_and_ubsan():
    subprocess.run(["make", "-j", "4", "-C", CSRC, "asan"], check=True, capture_output=True)
    assert os.path.exists(LIB)
    env = dict(os.environ)
    # the sanitizer runtime first, and libstdc++ before it initialises so that
    # its exception interceptor finds the real __cxa_throw
    # (anything the environment already preloads stays, after them)
    pre = f"{_gcc_lib('libasan.so')} {_gcc_lib('libstdc++.so')}"
    env["LD_PRELOAD"] = f"{pre} {env['LD_PRELOAD']}" if env.get("LD_PRELOAD") else pre
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["MUSTER_LIB"] = LIB
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr
    assert " passed" in r.stdout
