"""The serving scheduler (admission, queue bounds, cancellation, levels of 0
steps, launch groups, failure isolation, device errors, the threaded loop and
its stop) on the CPU with a fake executor, built with g++ under AddressSanitizer
and UndefinedBehaviorSanitizer: tests/cpu/scheduler_fake_test.cpp."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_14671_amd", "csrc")


def test_scheduler_with_a_fake_executor():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "scheduler_fake_test")
        subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-I", CSRC,
                        os.path.join(CSRC, "scheduler.cpp"),
                        os.path.join(ROOT, "tests", "cpu", "scheduler_fake_test.cpp"),
                        "-lpthread", "-o", exe], check=True, capture_output=True, text=True)
        # whatever else the environment preloads stays; the sanitizer runtime
        # need not come first for a program linked with it
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
        print(r.stdout, r.stderr[-4000:])
        assert r.returncode == 0
        assert "all passed" in r.stdout
