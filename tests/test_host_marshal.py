"""Host logic without a GPU: the page-protection write tracker behind the
automatic marshaling mode, built from the library's own source with g++
(also under AddressSanitizer/UBSan)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2001_07938_amd", "csrc")


@pytest.mark.parametrize("san", [[], ["-fsanitize=undefined"]])
def test_marshal_tracker(tmp_path, san):
    exe = tmp_path / "marshal_test"
    cmd = ["g++", "-std=c++17", "-O1", "-g", *san, f"-I{CSRC}",
           os.path.join(ROOT, "tests", "host", "marshal_test.cpp"),
           os.path.join(CSRC, "marshal.cpp"), "-o", str(exe)]
    subprocess.check_call(cmd)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "marshal ok" in r.stdout
