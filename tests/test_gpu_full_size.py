"""GPU at the full sizes of the beam and two-stream workloads.

The oracle cannot run these whole, so each test runs the GPU path at full size
and then checks:
- Properties that hold at any size: charge continuity R_C, and the Gauss
  residual R_G while the fields come from the run itself.
- The GPU's last step on a sample of particles. The oracle pushes the sample
  one by one from the GPU's own state and fields before that step.
"""
import numpy as np
import pytest

import paper_2111_12411_amd as F
from paper_2111_12411_amd import workloads as W
from oracle import core, mesh as omesh
from parity_util import close, rel
from test_gpu_parity import tets_agree

pytestmark = pytest.mark.gpu

QE, ME = -W.Q_E, W.M_E


def cfl(N, k):
    m = omesh.cube_mesh(4, k)
    return core.cfl_dt(m, core.assemble(m)) * 4.0 / N


def sampled_last_step(run, m, dt, w, idx, steps_before, extra_checks=None):
    """Run steps_before steps, then compare one more step on particles idx
    with the oracle, started from the GPU state and fields."""
    run.step(steps_before)
    p0, v0, t0 = run.particles()
    vh0, ah0 = run.history()
    e0, b0 = run.fields()
    run.step(1)
    p1, v1, t1 = run.particles()
    orc = core.OracleRun(m, dt, particles_only=True)
    orc.load(p0[idx], v0[idx], QE, ME, w, tet=t0[idx])
    orc.vh = np.ascontiguousarray(vh0[idx], dtype=np.float64)
    orc.ah = np.ascontiguousarray(ah0[idx], dtype=np.float64)
    orc.e, orc.b = e0.copy(), b0.copy()
    orc.particle_step()
    return p1[idx], v1[idx], t1[idx], orc


def test_beam_order2_fp64_full_size_200_steps():
    """20^3 cube (48 000 tets), order 2, 1M-electron beam at 0.1c, FP64, 200 steps at 10 dt_cfl."""
    N, k = 20, 2
    dt = 10 * cfl(N, k)
    pos, vel = W.config_particles(2)
    n = len(pos)
    assert n == 1_000_000
    w = W.plasma_weight(n, dt)
    # the Gauss residual accumulates the solves' residuals over the 200 steps
    run = F.Run(F.Mesh.cube(N, k), dt, F.FP64, pcg_rtol=1e-15)
    run.load(pos, vel, QE, ME, w)
    m = omesh.cube_mesh(N, k)
    idx = np.random.default_rng(21).choice(n, 3000, replace=False)
    p1, v1, t1, orc = sampled_last_step(run, m, dt, w, idx, 199)
    RG, RC, RS = run.gauss()
    assert RG < 1e-12 and RC < 1e-12, (RG, RC, RS)
    close(p1, orc.pos, 1e-13)
    close(v1, orc.vel, 1e-12)
    tets_agree(m, p1, t1, orc.tet)
    st = run.stats()
    assert st["steps"] == 200 and st["reflections"] > 0
    run.close()


def test_two_stream_order2_mixed_full_size():
    """56^3 cube (1 053 696 tets), order 2, 64M electrons in two streams at +-0.2c, mixed precision."""
    N, k = 56, 2
    dt = 10 * cfl(N, k)
    pos, vel = W.config_particles(5)
    n = len(pos)
    assert n == 64_000_000
    w = W.plasma_weight(n, dt)
    run = F.Run(F.Mesh.cube(N, k), dt, F.MIXED, pcg_rtol=1e-13)
    run.load(pos, vel, QE, ME, w)
    del pos, vel
    m = omesh.cube_mesh(N, k)
    idx = np.random.default_rng(55).choice(n, 3000, replace=False)
    p1, v1, t1, orc = sampled_last_step(run, m, dt, w, idx, 2)
    RG, RC, RS = run.gauss()
    assert RC < 1e-12 and RG < 1e-12, (RG, RC, RS)
    # FP32 gather and force: position to ~1e-9, velocity to ~1e-5 relative
    close(p1, orc.pos, 1e-9)
    assert rel(v1, orc.vel) < 2e-5
    tets_agree(m, p1, t1, orc.tet, tol=1e-9)
    assert run.stats()["steps"] == 3
    run.close()


def test_mixed_vs_fp64_full_size():
    """40^3 cube (384 000 tets), order 2, 16M electrons with a 1% density perturbation in x and
    omega_p dt = 0.02, 100 steps at 10 dt_cfl: the mixed-precision path against the FP64 path from
    the same start.  Fields within 1e-5 relative, and the Gauss residual within 1e-12 in both.

    The two paths part slowly: now and then a particle ends a step within rounding distance of a
    face, the two runs put it on different sides, and since the normal component of the order-2 E
    field jumps across faces its force differs by O(1).  On this workload that leaves the fields
    ~1e-6 apart after 100 steps."""
    N, k = 40, 2
    dt = 10 * cfl(N, k)
    pos, vel = W.config_particles(3)
    n = len(pos)
    assert n == 16_000_000
    w = W.config_weight(3, n, dt)
    res = {}
    for prec in (F.FP64, F.MIXED):
        run = F.Run(F.Mesh.cube(N, k), dt, prec, pcg_rtol=1e-14)
        run.load(pos, vel, QE, ME, w)
        run.step(100)
        e, b = run.fields()
        res[prec] = (e, b, run.gauss())
        assert run.stats()["steps"] == 100
        run.close()
    e64, b64, g64 = res[F.FP64]
    e32, b32, g32 = res[F.MIXED]
    assert g64[0] < 1e-12 and g32[0] < 1e-12, (g64, g32)
    assert rel(e32, e64) < 1e-5 and rel(b32, b64) < 1e-5, (rel(e32, e64), rel(b32, b64))
