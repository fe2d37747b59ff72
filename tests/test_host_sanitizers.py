"""Host C++ (mesh building, reference elements, operator assembly) under AddressSanitizer and
UndefinedBehaviorSanitizer, built with g++ from tests/sanitize_host.cpp.  CPU only: no GPU code is
compiled or run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not available")
    csrc = os.path.join(ROOT, "paper_2111_12411_amd", "csrc")
    exe = str(tmp_path / "sanitize_host")
    cmd = (["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
            "-static-libasan", "-I", csrc, "-I", os.path.join(ROOT, "include"),
            os.path.join(ROOT, "tests", "sanitize_host.cpp")]
           + [os.path.join(csrc, f) for f in ("mesh.cpp", "refelem.cpp", "assemble.cpp")]
           + ["-lpthread", "-o", exe])
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0 and "host checks: 0 failed" in r.stdout, (r.stdout[-2000:], r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
