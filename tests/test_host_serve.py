"""Host logic without a GPU: the request server's scheduling core
(admission against the byte budget, LRU-2 eviction, slots, batching,
failures) driven by a simulated executor in virtual time, plus a threaded
run, built from the library's own serve_core.cpp with g++: plain, under
AddressSanitizer + UBSan, and under ThreadSanitizer."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2001_07938_amd", "csrc")


@pytest.mark.parametrize("san", [[], ["-fsanitize=address,undefined"],
                                 ["-fsanitize=thread"]],
                         ids=["plain", "asan", "tsan"])
def test_serve_core(tmp_path, san):
    exe = tmp_path / "serve_core_test"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", *san, f"-I{CSRC}",
           os.path.join(ROOT, "tests", "host", "serve_core_test.cpp"),
           os.path.join(CSRC, "serve_core.cpp"), "-o", str(exe), "-lpthread"]
    subprocess.check_call(cmd)
    env = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "serve core ok" in r.stdout
