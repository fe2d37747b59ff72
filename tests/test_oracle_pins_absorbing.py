"""Pins of the oracle's absorbing walls: the impedance condition of Sec. II with
the free-space wall admittance Y = 1/eta0 and the surface impedance matrix of
Sec. III-A,
  [*I]_ij = Y int_walls (n x W1_i) . (n x W1_j) dS,
entering Ampere's law as *eps de/dt + *I e = K^T *nu b - dg/dt.

- *I is symmetric and positive semi-definite, and only wall DoFs touch it;
- a constant field E0, which the order-k edge space holds exactly, gives
  e^T *I e = Y sum_walls A_w |n_w x E0|^2 (closed form), on a box with three
  different side lengths, so that wrong normals or areas show;
- the gradient of an interior nodal function has no tangential trace on the
  walls, so *I G = 0 on interior nodes: Gauss's law is untouched;
- the trapezoidal step conserves U = (e^T *eps e + b^T *nu b)/2 with PEC walls
  and, with absorbing walls, loses exactly dt (e^{n+1}+e^n)^T *I (e^{n+1}+e^n)/4
  per step (the discrete energy identity of the scheme);
- a plasma whose particles leave through absorbing walls keeps R_G at rounding."""
import numpy as np
import pytest
import scipy.sparse as sps

from oracle import core, mesh as omesh
from paper_2111_12411_amd import workloads as W
from test_oracle_pins import project

QE, ME = -W.Q_E, W.M_E
Y0 = np.sqrt(core.EPS0 / core.MU0)


def box_mesh(N, k, sides):
    xyz, tets = omesh.kuhn_cube(N, 1.0)
    return omesh.build(xyz * np.asarray(sides, dtype=np.float64), tets, k)


@pytest.mark.parametrize("k", [1, 2])
def test_impedance_matrix_is_symmetric_psd_on_wall_dofs(k):
    m = omesh.cube_mesh(2, k)
    Z = core.surface_impedance(m, Y0).toarray()
    assert np.allclose(Z, Z.T, rtol=0, atol=1e-15 * np.abs(Z).max())
    ev = np.linalg.eigvalsh(0.5 * (Z + Z.T))
    assert ev.min() > -1e-13 * ev.max()
    inner = np.nonzero(m.int1)[0]
    assert np.abs(Z[inner]).max() == 0 and np.abs(Z[:, inner]).max() == 0
    assert np.count_nonzero(np.abs(Z).sum(axis=1)) == m.n1 - m.N1_int  # every wall DoF is touched


@pytest.mark.parametrize("k", [1, 2])
def test_constant_field_closed_form(k):
    sides = (1.0, 2.0, 0.5)
    m = box_mesh(3, k, sides)
    run = core.OracleRun(m, 1e-12)
    E0 = np.array([0.7, -1.3, 2.1])
    e = project(run, lambda p: np.broadcast_to(E0, p.shape), 1)
    # the edge space holds constants: the projection is exact
    vol = np.prod(sides)
    assert e @ (run.ops.star_eps @ e) == pytest.approx(core.EPS0 * (E0 @ E0) * vol, rel=1e-12)
    Z = core.surface_impedance(m, Y0)
    want = 0.0
    for ax in range(3):
        area = np.prod(sides) / sides[ax]
        want += 2 * area * ((E0 @ E0) - E0[ax] ** 2)  # two walls with normal along this axis
    assert e @ (Z @ e) == pytest.approx(Y0 * want, rel=1e-12)


@pytest.mark.parametrize("k", [1, 2])
def test_impedance_leaves_interior_gradients_alone(k):
    m = omesh.cube_mesh(3, k)
    ops = core.assemble(m)
    Z = core.surface_impedance(m, Y0)
    ZG = (Z @ ops.G[:, ops.int0]).toarray()
    assert np.abs(ZG).max() <= 1e-14 * np.abs(Z).max()


def _random_fields(run, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    e = np.zeros(run.m.n1)
    e[run.i1] = rng.normal(size=len(run.i1))
    b = rng.normal(size=run.m.n2)
    return e, b


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("bc", ["pec", "absorbing"])
def test_energy_identity_of_the_step(k, bc):
    m = omesh.cube_mesh(3, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    run = core.OracleRun(m, dt, ops, field_bc=bc)
    run.e, run.b = _random_fields(run, 11 + k)
    Z = run.ZI
    for _ in range(5):
        u0, e0 = run.energy(), run.e.copy()
        run.field_step(np.zeros(m.n1))
        u1 = run.energy()
        loss = 0.0 if Z is None else dt * 0.25 * (run.e + e0) @ (Z @ (run.e + e0))
        assert u1 - u0 == pytest.approx(-loss, rel=1e-9, abs=1e-12 * u0)
        if Z is not None:
            assert loss > 1e-6 * u0  # the walls do absorb


@pytest.mark.parametrize("k", [1, 2])
def test_plasma_leaving_through_absorbing_walls_keeps_gauss_law(k):
    m = omesh.cube_mesh(3, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    pos, vel = W.particles("beam", 800, 21 + k, vth=0.02, drift=0.2)
    run = core.OracleRun(m, dt, ops, absorb=True, field_bc="absorbing")
    run.load(pos, vel, QE, ME, W.plasma_weight(len(pos), dt))
    for _ in range(10):
        run.step()
        rg, rc, rs = run.gauss_residuals()
        assert rg < 1e-12 and rc < 1e-12 and rs < 1e-12
    assert run.counters[2] > 0  # particles did leave
    assert np.abs(run.e[np.nonzero(~m.int1)[0]]).max() > 0  # the wall DoFs carry field


def test_three_level_scheme_with_absorbing_walls_is_refused():
    m = omesh.cube_mesh(2, 1)
    with pytest.raises(NotImplementedError):
        core.OracleRun(m, 1e-11, field_bc="absorbing", gamma=1.5, beta=1.0)
