"""Pins of the oracle's PEC-wall particle rule and of its explicit time-step bound.

Wall rule (reading of Sec. III-B for a particle at a PEC wall): the rest of the
step's path is mirrored about the wall plane from the crossing on, and at the
end of the step the velocity and every entry of the Adams-Bashforth velocity
and acceleration histories are mirrored.  With zero fields, or a uniform E and
the constant-acceleration start, the unreflected path is a straight line or a
parabola in closed form, so the reflected end state is its mirror image:
    r_end  = M(r0 + v0 dt + a dt^2 / 2),   v_end = M(v0 + a dt),
    v^{n-1..n-3} history = M(v0), M(v0 - a dt), M(v0 - 2 a dt),
    a history = M(a) three times,
with M the reflection about the wall plane.  Mirroring v before the velocity
update, a missing history flip or a wrong plane all fail these.

Explicit bound (reading of the "explicit CFL limit" of the workloads): the
leapfrog limit 2 / sqrt(lambda_max) of K^T *nu K x = lambda *eps x is bounded
with the element-by-element eigenvalue bound lambda_max <= max_T lambda_max of
the element pencil; a dense eigensolve of the global pencil checks that the
bound holds and how close it is.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import core, mesh as omesh
from paper_2111_12411_amd import workloads as W
from test_oracle_pins import project

QE, ME = -W.Q_E, W.M_E


def _run(N, k, dt_factor):
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    return core.OracleRun(m, dt_factor * core.cfl_dt(m, ops), ops)


def _mirror(x, axis, plane=None):
    """Reflection about the plane x[axis] = plane (a point) or of a vector (plane None)."""
    y = np.array(x, dtype=np.float64)
    y[..., axis] = (2.0 * plane - y[..., axis]) if plane is not None else -y[..., axis]
    return y


def _continuity(run, p):
    """Charge continuity of particle p's deposit over one step: G^T dg = rho~(end) - rho~(start)."""
    before = run.rho().copy()
    dg = run.particle_step(idx=[p])
    after = run.rho()
    scale = abs(QE) * max(np.abs(after - before).max(), 1.0)
    np.testing.assert_allclose(run.ops.G.T @ dg, after - before, rtol=0, atol=1e-14 * scale)
    return dg


@pytest.mark.parametrize("k", [1, 2])
def test_wall_reflection_field_free_is_the_mirror_image(k):
    run = _run(4, k, 10.0)
    dt = run.dt
    p0 = np.array([0.93, 0.47, 0.52])
    v0 = np.array([0.12, 0.035, -0.02]) / dt  # crosses x = 1 once within the step
    straight = p0 + v0 * dt
    assert straight[0] > 1.0 and np.all(straight[1:] > 0) and np.all(straight[1:] < 1)
    run.load(p0[None], v0[None], QE, ME, 1.0)
    run.counters[:] = 0
    _continuity(run, 0)
    assert run.counters[1] == 1
    np.testing.assert_allclose(run.pos[0], _mirror(straight, 0, 1.0), rtol=0, atol=1e-15)
    np.testing.assert_allclose(run.vel[0], _mirror(v0, 0), rtol=1e-15)
    for j in range(3):
        np.testing.assert_allclose(run.vh[0, j], _mirror(v0, 0), rtol=1e-15)
        assert np.all(run.ah[0, j] == 0.0)


@pytest.mark.parametrize("k", [1, 2])
def test_wall_reflection_uniform_E_is_the_mirrored_parabola(k):
    """A uniform E with a component towards the wall: the reflected end state is the mirror of the
    closed-form parabola, and each of the six history entries is the mirror of its value."""
    run = _run(4, k, 10.0)
    dt = run.dt
    E0 = np.array([4.0e3, -1.5e3, 2.5e3])
    run.e = project(run, lambda p: np.broadcast_to(E0, p.shape).copy(), 1)
    run.b = np.zeros(run.m.n2)
    a = QE / ME * E0
    p0 = np.array([0.06, 0.44, 0.57])
    v0 = np.array([-0.09, 0.02, 0.03]) / dt  # towards x = 0 against the force (q < 0: a_x < 0 too)
    x_par = p0 + v0 * dt + 0.5 * a * dt * dt
    assert x_par[0] < 0.0 and np.all(x_par[1:] > 0) and np.all(x_par[1:] < 1)
    run.load(p0[None], v0[None], QE, ME, 1.0)
    run.counters[:] = 0
    _continuity(run, 0)
    assert run.counters[1] == 1
    scale = np.abs(v0 * dt).max()
    np.testing.assert_allclose(run.pos[0], _mirror(x_par, 0, 0.0), rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(run.vel[0], _mirror(v0 + a * dt, 0), rtol=1e-12)
    for j in range(3):
        np.testing.assert_allclose(run.vh[0, j], _mirror(v0 - j * a * dt, 0), rtol=1e-12)
        np.testing.assert_allclose(run.ah[0, j], _mirror(a, 0), rtol=1e-12)
    # the unmirrored velocity update would differ: the check can fail
    assert np.abs(_mirror(v0, 0) + a * dt - _mirror(v0 + a * dt, 0)).max() > 1e-3 * np.abs(v0).max()


@pytest.mark.parametrize("k", [1, 2])
def test_two_wall_corner_hit_in_one_step(k):
    run = _run(4, k, 10.0)
    dt = run.dt
    p0 = np.array([0.95, 0.93, 0.41])
    v0 = np.array([0.1, 0.13, 0.04]) / dt  # crosses x = 1, then y = 1, within one step
    straight = p0 + v0 * dt
    assert straight[0] > 1.0 and straight[1] > 1.0
    run.load(p0[None], v0[None], QE, ME, 1.0)
    run.counters[:] = 0
    _continuity(run, 0)
    assert run.counters[1] == 2
    want = _mirror(_mirror(straight, 0, 1.0), 1, 1.0)
    np.testing.assert_allclose(run.pos[0], want, rtol=0, atol=2e-15)
    np.testing.assert_allclose(run.vel[0], _mirror(_mirror(v0, 0), 1), rtol=1e-15)
    for j in range(3):
        np.testing.assert_allclose(run.vh[0, j], _mirror(_mirror(v0, 0), 1), rtol=1e-15)


@pytest.mark.parametrize("N,k", [(2, 1), (3, 1), (4, 1), (2, 2), (3, 2), (4, 2)])
def test_explicit_bound_against_dense_global_eigensolve(N, k):
    """The element-by-element bound is an upper bound of the global lambda_max (so the workloads'
    time step, a multiple of 2/sqrt(bound), is a multiple of a step at most the leapfrog limit),
    and within 40% of it on these cubes."""
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    i1 = ops.int1
    Ki = ops.K[:, i1]
    S = (Ki.T @ ops.star_nu @ Ki).toarray()
    Me = ops.star_eps[i1][:, i1].toarray()
    lmax = sla.eigh(S, Me, eigvals_only=True)[-1]
    dt_global = 2.0 / np.sqrt(lmax)
    dt_elem = core.cfl_dt(m, ops)
    assert dt_elem <= dt_global * (1 + 1e-12)
    assert dt_elem >= 0.6 * dt_global
    # the bound is attained by a single-element pencil: a one-tet "mesh" problem with no walls
    # dropped (its global and element pencils coincide) gives equality
    M1 = core.EPS0 * ops.M1_el[0]
    S1 = ops.Kloc.T @ ops.M2_el[0] @ ops.Kloc / core.MU0
    one = sla.eigh(S1, M1, eigvals_only=True)[-1]
    assert one <= (2.0 / dt_elem) ** 2 * (1 + 1e-12)


# ------------------------------------------------------------ absorbing walls
@pytest.mark.parametrize("k", [1, 2])
def test_absorbed_particle_ends_at_the_wall_point_and_carries_its_charge_away(k):
    """Field-free particle into the wall x = 1 with the absorbing rule: it leaves the run (tet -1) at
    the closed-form point where its straight path meets the wall, and its deposit moves exactly its
    own charge off the interior nodes: G^T dg = -q w W0(r0) there (the interior W0 vanish on walls)."""
    m = omesh.cube_mesh(4, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    run = core.OracleRun(m, dt, ops, absorb=True)
    p0 = np.array([0.93, 0.47, 0.52])
    v0 = np.array([0.12, 0.035, -0.02]) / dt
    run.load(p0[None], v0[None], QE, ME, 1.0)
    rho0 = run.rho().copy()
    dg = run.particle_step()
    assert run.tet[0] == -1 and run.counters[2] == 1 and run.counters[1] == 0
    s = (1.0 - p0[0]) / (v0[0] * dt)
    np.testing.assert_allclose(run.pos[0], p0 + s * v0 * dt, rtol=0, atol=1e-15)
    i0 = ops.int0
    np.testing.assert_allclose((ops.G.T @ dg)[i0], -rho0[i0], rtol=0, atol=1e-14 * abs(QE))
    assert np.all(run.rho() == 0.0)  # no particle is left to measure


@pytest.mark.parametrize("k", [1, 2])
def test_absorbing_run_keeps_gauss_law_and_leaves_other_particles_alone(k):
    """A beam into the z walls: particles leave every step, R_G and R_C stay at rounding level; with
    the fields held fixed, the particles that never reach a wall move exactly as under reflection."""
    m = omesh.cube_mesh(3, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    pos, vel = W.particles("beam", 1500, 61 + k, vth=0.01, drift=0.15)
    run = core.OracleRun(m, dt, ops, absorb=True)
    run.load(pos, vel, QE, ME, W.plasma_weight(len(pos), dt))
    for n in range(12):
        run.step()
        RG, RC, RS = run.gauss_residuals()
        assert RG < 1e-12 and RC < 1e-12, (n, RG, RC, RS)
    gone = run.tet < 0
    assert gone.mean() > 0.5 and run.counters[2] == gone.sum()
    # fixed random fields, particles only: absorbing and reflecting runs agree on the particles
    # that stay inside
    e0, b0 = W.random_fields(m.n1, m.n2, 8, e_scale=1e3, b_scale=1e-5)
    runs = []
    for absorb in (True, False):
        r = core.OracleRun(m, dt, ops, absorb=absorb, particles_only=True)
        r.load(pos, vel, QE, ME, 1.0)
        r.e, r.b = e0 * m.int1, b0
        for _ in range(5):
            r.particle_step()
        runs.append(r)
    a, rf = runs
    alive = a.tet >= 0
    assert (~alive).sum() > 50 and rf.counters[1] > 50
    # reflected particles may later differ; those that never met a wall are bit-identical
    same = np.all(a.pos[alive] == rf.pos[alive], axis=1)
    assert same.mean() > 0.95
    assert np.array_equal(a.tet[alive][same], rf.tet[alive][same])
