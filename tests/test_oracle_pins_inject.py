"""Pins of the oracle's particle injection (the beam source of Table III: a few
particles enter every step).

Charge enters through injection, not through a current, so the injected
particles' nodal charge joins the reference rho~^0.  Then:
- a beam injected on the wall z = 0 (where the interior W0 vanish) into a run
  with absorbing walls keeps R_G and R_C at rounding level step after step,
  while particles enter and leave;
- particles injected in the interior leave R_C at rounding level too (their
  charge is in the reference), and without the reference update it would be
  O(1): the check can fail."""
import numpy as np
import pytest

from oracle import core, mesh as omesh
from paper_2111_12411_amd import workloads as W

QE, ME = -W.Q_E, W.M_E


def beam_source(n, seed, vz=0.15):
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = np.empty((n, 3))
    pos[:, :2] = np.clip(rng.normal(0.5, 0.1, (n, 2)), 0.05, 0.95)
    pos[:, 2] = 0.0
    vel = rng.normal(0.0, 0.005 * W.C_LIGHT, (n, 3))
    vel[:, 2] = vz * W.C_LIGHT + np.abs(vel[:, 2])
    return pos, vel


@pytest.mark.parametrize("k", [1, 2])
def test_wall_injected_beam_keeps_gauss_law(k):
    m = omesh.cube_mesh(3, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    pos, vel = W.particles("thermal", 500, 3, vth=0.01)
    run = core.OracleRun(m, dt, ops, absorb=True)
    run.load(pos, vel, QE, ME, W.plasma_weight(2000, dt))
    for n in range(12):
        p, v = beam_source(150, 100 + n)
        rho_before = run.rho0.copy()
        run.inject(p, v)
        # on the wall the interior nodal functions vanish: the reference does not move there
        assert np.abs((run.rho0 - rho_before)[ops.int0]).max() < 1e-14 * abs(QE) * run.w
        run.step()
        RG, RC, RS = run.gauss_residuals()
        assert RG < 1e-12 and RC < 1e-12, (n, RG, RC, RS)
    alive = run.tet >= 0
    assert len(run.tet) == 500 + 12 * 150 and alive.sum() > 500 and run.counters[2] > 0


def test_interior_injection_enters_the_reference():
    m = omesh.cube_mesh(3, 2)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    pos, vel = W.particles("thermal", 800, 4, vth=0.01)
    run = core.OracleRun(m, dt, ops)
    run.load(pos, vel, QE, ME, W.plasma_weight(800, dt))
    run.step(2)
    p, v = W.particles("thermal", 300, 5, vth=0.01)
    rho0_old = run.rho0.copy()
    run.inject(p, v)
    run.step(3)
    RG, RC, RS = run.gauss_residuals()
    assert RC < 1e-12, RC
    # without the new charge in the reference the continuity residual is O(1)
    i0 = ops.int0
    drho = (run.rho() - rho0_old)[i0]
    assert np.linalg.norm((ops.G.T @ run.g)[i0] - drho) / np.linalg.norm(drho) > 1e-2
