"""The device-memory arena (reuse of released blocks by size, the device
synchronisation before a released block is reused, the budget, taking back
what other arenas keep when an allocation fails, trim, destruction,
concurrent use) on the CPU with a fake device, built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer: tests/cpu/arena_fake_test.cpp."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_14671_amd", "csrc")


def test_arena_with_a_fake_device():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "arena_fake_test")
        subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-I", CSRC,
                        os.path.join(ROOT, "tests", "cpu", "arena_fake_test.cpp"),
                        "-lpthread", "-o", exe], check=True, capture_output=True, text=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
        print(r.stdout, r.stderr[-4000:])
        assert r.returncode == 0
        assert "all passed" in r.stdout
