"""Host C++ (mesh building, reference elements, operator assembly) under AddressSanitizer and
UndefinedBehaviorSanitizer, built with g++ from tests/sanitize_host.cpp.  CPU only: no GPU code is
compiled or run."""
import os
import shutil
import sys
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


ORACLE_STEPS = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import core, mesh as omesh
from paper_2111_12411_amd import workloads as W
for k in (1, 2):
    m = omesh.cube_mesh(3, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    run = core.OracleRun(m, dt, ops)
    pos, vel = W.particles("beam", 1500, 41, vth=0.02, drift=0.2)
    run.load(pos, vel, -W.Q_E, W.M_E, W.plasma_weight(len(pos), dt))
    run.step(6)
    assert run.counters[0] > 0 and run.counters[1] > 0, run.counters
    assert run.gauss_residuals()[0] < 1e-12
print("oracle steps ok")
"""


def test_oracle_loop_under_ubsan(tmp_path):
    """The oracle's plain-C particle loop built with UBSan (fatal on the first report) and driven
    through whole steps with crossings and wall reflections at both orders."""
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    lib = str(tmp_path / "liboracle_ubsan.so")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
           "-fsanitize=undefined", "-fno-sanitize-recover=all", "-o", lib,
           os.path.join(ROOT, "oracle", "oracle_particles.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, FEMPIC_ORACLE_LIB=lib, UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", ORACLE_STEPS, ROOT], capture_output=True, text=True, timeout=900,
                       env=env)
    assert r.returncode == 0 and "oracle steps ok" in r.stdout, (r.stdout[-2000:], r.stderr[-3000:])
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
