"""Pins of the oracle's alternative pusher: the Boris leapfrog with a straight path.

The push is independent of the current mapping (Sec. III-B); with the Boris
scheme the stored velocity is v^{n-1/2} and, with E and B at r^n,
  v^{n+1/2} = half kick, rotation about B, half kick;   r^{n+1} = r^n + dt v^{n+1/2}.
Closed forms that fix it:
- uniform B, no E: each step rotates v about B by phi = -2 atan(q |B| dt / 2m)
  (the sign of v x B), exactly; |v| is conserved and the positions are the
  partial sums of the rotated velocities;
- uniform E, no B: v^{n+1/2} = v^{-1/2} + (n+1) (q/m) E dt and the positions are
  the matching sums;
- a particle in zero fields that meets a wall: the mirror image of the straight
  end point, with the mirrored velocity;
- the deposit of every step keeps charge continuity particle by particle.
A wrong rotation sign or angle, a missing half kick or kicks in the wrong order
fail the first two."""
import numpy as np
import pytest

from oracle import core, mesh as omesh
from paper_2111_12411_amd import workloads as W
from test_oracle_pins import project

QE, ME = -W.Q_E, W.M_E


def _run(N, k):
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    run = core.OracleRun(m, 5 * core.cfl_dt(m, ops), ops, pusher="boris")
    return run


def _rot(v, axis, phi):
    a = axis / np.linalg.norm(axis)
    return v * np.cos(phi) + np.cross(a, v) * np.sin(phi) + a * (a @ v) * (1 - np.cos(phi))


@pytest.mark.parametrize("k", [1, 2])
def test_uniform_B_rotates_by_the_boris_angle(k):
    run = _run(4, k)
    dt = run.dt
    B0 = np.array([0.01, -0.02, 0.03])
    run.b = project(run, lambda p: np.broadcast_to(B0, p.shape).copy(), 2)
    run.e = np.zeros(run.m.n1)
    r0 = np.array([0.5, 0.47, 0.52])
    v0 = np.array([0.031, 0.017, -0.022]) / dt  # crosses a few faces a step
    run.load(r0[None], v0[None], QE, ME, 1.0)
    w = QE / ME * np.linalg.norm(B0)
    phi = -2.0 * np.arctan(0.5 * w * dt)
    r = r0.copy()
    for n in range(1, 9):
        run.particle_step()
        vn = _rot(v0, B0, n * phi)
        r = r + dt * vn
        np.testing.assert_allclose(run.vel[0], vn, rtol=1e-12)
        np.testing.assert_allclose(run.pos[0], r, rtol=0, atol=1e-13)
    assert abs(np.linalg.norm(run.vel[0]) / np.linalg.norm(v0) - 1) < 1e-14
    assert abs(phi) > 0.05  # the rotation is large enough to tell a wrong angle


@pytest.mark.parametrize("k", [1, 2])
def test_uniform_E_kicks_by_q_E_dt(k):
    run = _run(4, k)
    dt = run.dt
    E0 = np.array([300.0, -150.0, 80.0])
    run.e = project(run, lambda p: np.broadcast_to(E0, p.shape).copy(), 1)
    run.b = np.zeros(run.m.n2)
    r0 = np.array([0.41, 0.52, 0.47])
    v0 = np.array([0.011, -0.007, 0.009]) / dt
    run.load(r0[None], v0[None], QE, ME, 1.0)
    kick = QE / ME * E0 * dt
    r = r0.copy()
    for n in range(1, 6):
        run.particle_step()
        vn = v0 + n * kick
        r = r + dt * vn
        np.testing.assert_allclose(run.vel[0], vn, rtol=1e-12)
        np.testing.assert_allclose(run.pos[0], r, rtol=0, atol=1e-13)
    assert np.abs(kick).max() > 1e-3 * np.abs(v0).max()


@pytest.mark.parametrize("k", [1, 2])
def test_wall_mirror_and_continuity(k):
    run = _run(4, k)
    dt = run.dt
    run.e = np.zeros(run.m.n1)
    run.b = np.zeros(run.m.n2)
    p0 = np.array([0.93, 0.47, 0.52])
    v0 = np.array([0.12, 0.035, -0.02]) / dt
    run.load(p0[None], v0[None], QE, ME, 1.0)
    before = run.rho().copy()
    dg = run.particle_step()
    after = run.rho()
    end = p0 + dt * v0
    mirror = end.copy()
    mirror[0] = 2.0 - end[0]
    np.testing.assert_allclose(run.pos[0], mirror, rtol=0, atol=1e-15)
    np.testing.assert_allclose(run.vel[0], v0 * np.array([-1, 1, 1]), rtol=1e-15)
    scale = abs(QE) * max(np.abs(after - before).max(), 1.0)
    np.testing.assert_allclose(run.ops.G.T @ dg, after - before, rtol=0, atol=1e-14 * scale)


def test_gauss_law_holds_for_a_boris_plasma():
    m = omesh.cube_mesh(3, 2)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    pos, vel = W.particles("beam", 1500, 8, vth=0.01, drift=0.12)
    run = core.OracleRun(m, dt, ops, pusher="boris")
    run.load(pos, vel, QE, ME, W.plasma_weight(len(pos), dt))
    for _ in range(10):
        run.step()
        RG, RC, RS = run.gauss_residuals()
        assert RG < 1e-12 and RC < 1e-12, (RG, RC, RS)
