"""Host logic without a GPU: the page-protection write tracker behind the
automatic marshaling mode, built from the library's own source with g++,
plain, under UndefinedBehaviorSanitizer, and under AddressSanitizer + UBSan
(AddressSanitizer's own SIGSEGV handler is switched off for that run: the
tracker's handler must see the protection faults it provokes)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2001_07938_amd", "csrc")


@pytest.mark.parametrize("san", [[], ["-fsanitize=undefined"],
                                 ["-fsanitize=address,undefined"]],
                         ids=["plain", "ubsan", "asan"])
def test_marshal_tracker(tmp_path, san):
    exe = tmp_path / "marshal_test"
    cmd = ["g++", "-std=c++17", "-O1", "-g", *san, f"-I{CSRC}",
           os.path.join(ROOT, "tests", "host", "marshal_test.cpp"),
           os.path.join(CSRC, "marshal.cpp"), "-o", str(exe)]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="handle_segv=0:detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "marshal ok" in r.stdout
