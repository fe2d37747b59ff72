"""CPU checks of bench.py's host logic: the byte model behind the roofline figures, the guard
that ties the profiled traffic to the kernel sources, the workloads' plasma weights, and the
one-GPU rule (no GPU needed)."""
import hashlib
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import bench
import paper_2111_12411_amd as F
from paper_2111_12411_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_per_particle_and_tet():
    # state: r, v in FP64 (48 B), three v and three a histories (18 values), tet (4 B)
    alg, state, tet = bench.algorithmic_bytes(2, F.MIXED, 1, 0)
    assert state == 48 + 18 * 4 + 4 == 124 and alg == 2 * 124
    alg, state, tet = bench.algorithmic_bytes(2, F.FP64, 1, 0)
    assert state == 48 + 18 * 8 + 4 == 196 and alg == 2 * 196
    # per tet: geometry (16 doubles), 20 W1 + 15 W2 coefficients with their int32 maps, 20 FP64 partials
    _, _, tet = bench.algorithmic_bytes(2, F.MIXED, 0, 1)
    assert tet == 128 + 35 * (4 + 4) + 20 * 8 == 568
    _, _, tet = bench.algorithmic_bytes(1, F.FP64, 0, 1)
    assert tet == 128 + 10 * (8 + 4) + 6 * 8
    # the benchmark launch: 16M particles, 384 000 tets
    alg, _, _ = bench.algorithmic_bytes(2, F.MIXED, 16_000_000, 384_000)
    assert alg == 4_186_112_000


def test_survey_byte_model():
    """The scope's model: 2 x 112 B (mixed) or 2 x 196 B (FP64) of state per particle, 836 B per tet
    at order 2 (312 B at order 1), 8 B per interior W1 DoF; the benchmark launch moves 3.924 GB,
    about 245 B per particle-step."""
    alg, state, tet = bench.survey_bytes(2, F.MIXED, 16_000_000, 384_000, 2_384_240)
    assert state == 112 and tet == 836
    assert alg == 16_000_000 * 224 + 384_000 * 836 + 2_384_240 * 8
    assert round(alg / 16e6) == 245
    alg, state, tet = bench.survey_bytes(2, F.FP64, 1, 0, 0)
    assert state == 196 and alg == 392
    _, _, tet = bench.survey_bytes(1, F.MIXED, 0, 1, 0)
    assert tet == 216 + 96


def test_oracle_thread_count_is_bounded():
    assert 1 <= bench.oracle_threads() <= 16


def _profile_copy(tmp_path, digest):
    root = tmp_path / "repo"
    (root / "profiles").mkdir(parents=True)
    (root / "paper_2111_12411_amd" / "csrc").mkdir(parents=True)
    for f in ("kernels.hip", "kernels.h"):
        shutil.copy(os.path.join(ROOT, "paper_2111_12411_amd", "csrc", f), root / "paper_2111_12411_amd" / "csrc" / f)
    (root / "profiles" / "k_particle_c3_mixed_hbm_counters.md").write_text(
        "```\ntraffic_bytes_per_launch: 7.5e+09\nkernel_source_sha256: %s\n```\n" % digest)
    return root


def test_pcg_bytes_per_iteration():
    # order 2, mixed: one 2x2 block row with one block: 16 B values + 4 B column; row pointer 8 B and
    # x, y, dot pairs 3 x 8 B; block-Jacobi 16 B; x, p, r, q read and x, r, z written (7 x 8 B);
    # z, p read and p written (3 x 8 B)
    assert bench.pcg_bytes_per_iter(2, F.MIXED, 2, 4) == 20 + 32 + 16 + 56 + 24
    # order 1, FP64, one row with one entry: 8 + 4, 8 + 3 x 8, Jacobi 8, 7 x 8, 3 x 8
    assert bench.pcg_bytes_per_iter(1, F.FP64, 1, 1) == 12 + 32 + 8 + 56 + 24
    # the benchmark system: 2 384 240 rows, 25 457 008 blocks -> 0.662 GB per iteration
    assert abs(bench.pcg_bytes_per_iter(2, F.MIXED, 2_384_240, 4 * 25_457_008) / 1e9 - 0.6617) < 1e-3
    # tet by tet, order 2 in pairs, mixed: one tet whose 20 DoFs are the 20 rows (10 pairs), 20
    # incidences: 10 pair ids and 10 product positions x 4 + 16 x 4 geometry + 20 x 4 p + 20 x 4
    # products; 11 row pointers x 8 + 20 x 4 products + 2 x 20 x 4; block-Jacobi 10 x 16; 7 x 80;
    # 3 x 80
    assert bench.pcg_bytes_per_iter(2, F.MIXED, 20, 0, 2, 1, 20) == (80 + 64 + 80 + 80) + (88 + 80 + 160) \
        + 160 + 560 + 240
    # order 1, FP64, one DoF per row (field_op 1): 6 ids x 4 + 16 x 8 + 6 x 8 + 6 x 8; 7 x 8 + 6 x 4
    # + 6 x 8 + 2 x 6 x 8; Jacobi 6 x 8; 7 x 48; 3 x 48
    assert bench.pcg_bytes_per_iter(1, F.FP64, 6, 0, 1, 1, 6) == (24 + 128 + 48 + 48) + (56 + 24 + 48 + 96) \
        + 48 + 336 + 144


def test_profiled_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h"):
        with open(os.path.join(ROOT, "paper_2111_12411_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    monkeypatch.setattr(bench, "ROOT", str(_profile_copy(tmp_path / "a", h.hexdigest())))
    assert bench.profiled_traffic() == 7.5e9
    monkeypatch.setattr(bench, "ROOT", str(_profile_copy(tmp_path / "b", "0" * 64)))
    assert bench.profiled_traffic() is None
    monkeypatch.setattr(bench, "ROOT", str(tmp_path / "missing"))
    assert bench.profiled_traffic() is None


@pytest.mark.parametrize("cfg_id,omega_dt", [(1, 0.1), (2, 0.1), (3, 0.02), (5, 0.01)])
def test_config_weight_gives_the_plasma_frequency(cfg_id, omega_dt):
    n, dt = 1000, 2.5e-10
    w = W.config_weight(cfg_id, n, dt)
    # omega_p^2 = n_e e^2 / (eps0 m_e), with n_e = n w / L^3 electrons per m^3 on the unit cube
    omega_p = np.sqrt(n * w * W.Q_E ** 2 / (W.EPS0 * W.M_E))
    assert abs(omega_p * dt - omega_dt) < 1e-12 * omega_dt


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
