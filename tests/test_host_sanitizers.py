"""The library's host setup math (Gauss rule, knots, basis, banded 1D
matrices, banded LU) built with the address and undefined-behaviour
sanitizers and run over every degree, Gauss rule and small element count
(tests/host/host_math_check.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_math_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_math_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "host", "host_math_check.cpp"),
           os.path.join(ROOT, "paper_1911_08158_amd", "csrc", "host_math.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert "ok (0 failures)" in r.stdout
