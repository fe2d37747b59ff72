"""Pins of the oracle's general Newmark-beta field update (Sec. III-B, eq. (maxnmb);
the alternative schemes of Sec. IV-D: backward difference gamma = 1.5, beta = 1,
Galerkin gamma = 1.5, beta = 0.8).

- At gamma = 1/2, beta = 1/4 the three-level form is the sum of two trapezoidal
  steps, so from fields at rest it reproduces the two-level trapezoidal update.
- A cavity eigenmode stays a mode: with e = p phi and b = q K phi / omega the
  scheme acts on (p, q) exactly as on the 2x2 system dp/dt = omega q,
  dq/dt = -omega p.  That recurrence, written out here on its own, fixes every
  coefficient of the scheme (a wrong weight changes the modal amplitude or phase).
- Gauss's law: K G = 0 and the current taken with the mass-term stencil keep
  G^T(*eps e + g) at zero for any (gamma, beta) (the paper's claim for the
  alternative schemes), so R_G stays at rounding level with moving charge.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import core, mesh as omesh
from paper_2111_12411_amd import workloads as W

QE, ME = -W.Q_E, W.M_E
SCHEMES = [(0.5, 0.25), (1.5, 1.0), (1.5, 0.8)]


def test_three_level_at_half_quarter_is_the_trapezoidal_step():
    N, k = 3, 2
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    pos, vel = W.particles("beam", 600, 21, vth=0.01, drift=0.12)
    w = W.plasma_weight(len(pos), dt)
    a = core.OracleRun(m, dt, ops)
    b = core.OracleRun(m, dt, ops, three_level=True)
    for r in (a, b):
        r.load(pos, vel, QE, ME, w)
    for n in range(25):
        a.step()
        b.step()
        assert np.linalg.norm(b.e - a.e) <= 1e-10 * np.linalg.norm(a.e), n
        assert np.linalg.norm(b.b - a.b) <= 1e-10 * np.linalg.norm(a.b), n
    assert np.linalg.norm(a.e) > 0


def _modal_recurrence(gamma, beta, omega, dt, nsteps):
    """The scheme on x' = [[0, w], [-w, 0]] x written as M x' + S x = 0 (M = I), from x^{-1} = x^0 = (1, 0)."""
    S = np.array([[0.0, -omega], [omega, 0.0]])
    I2 = np.eye(2)
    c1, c0 = 0.5 - 2 * beta + gamma, 0.5 + beta - gamma
    L = gamma / dt * I2 + beta * S
    xs = [np.array([1.0, 0.0]), np.array([1.0, 0.0])]
    for _ in range(nsteps):
        rhs = -((1 - 2 * gamma) / dt * I2 + c1 * S) @ xs[-1] - ((gamma - 1) / dt * I2 + c0 * S) @ xs[-2]
        xs.append(np.linalg.solve(L, rhs))
    return np.array(xs[1:])


@pytest.mark.parametrize("gamma,beta", SCHEMES)
@pytest.mark.parametrize("k", [1, 2])
def test_cavity_mode_follows_the_scalar_recurrence(gamma, beta, k):
    N = 3
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    dt = 5 * core.cfl_dt(m, ops)
    i1 = ops.int1
    Ki = ops.K[:, i1]
    S = (Ki.T @ ops.star_nu @ Ki).toarray()
    Me = ops.star_eps[i1][:, i1].toarray()
    lam, vec = sla.eigh(S, Me)
    j = int(np.searchsorted(lam, 0.2 * lam[-1]))  # a mode well above the static null space
    omega = np.sqrt(lam[j])
    phi = vec[:, j]  # *eps-orthonormal
    psi = Ki @ phi / omega
    run = core.OracleRun(m, dt, ops, gamma=gamma, beta=beta, three_level=True)
    run.load(np.zeros((0, 3)), np.zeros((0, 3)), QE, ME, 1.0)
    run.e = np.zeros(m.n1)
    run.e[i1] = phi
    run.b = np.zeros(m.n2)
    nst = 40
    want = _modal_recurrence(gamma, beta, omega, dt, nst)
    nu_psi = ops.star_nu @ psi
    for n in range(nst):
        run.step()
        p = phi @ (Me @ run.e[i1])
        q = (nu_psi @ run.b) / (nu_psi @ psi)
        np.testing.assert_allclose([p, q], want[n + 1], rtol=0, atol=1e-10)
        # nothing leaks out of the mode
        assert np.linalg.norm(run.e[i1] - p * phi) < 1e-10 * np.linalg.norm(phi)
    amp = np.abs(want).max(axis=1)
    if gamma > 0.5:
        assert amp[-1] < 0.9 * amp[0]  # the alternative schemes damp the mode
    else:
        # both roots on the unit circle: no growth (from a start at rest at omega dt of about 3.7
        # the parasitic root -1 carries a large part of the mode)
        assert amp[20:].max() < 1.2 * amp[:20].max()


@pytest.mark.parametrize("gamma,beta", SCHEMES[1:])
@pytest.mark.parametrize("k", [1, 2])
def test_gauss_law_holds_for_alternative_schemes(gamma, beta, k):
    N = 3
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    pos, vel = W.particles("beam", 800, 33 + k, vth=0.01, drift=0.15)
    run = core.OracleRun(m, dt, ops, gamma=gamma, beta=beta)
    run.load(pos, vel, QE, ME, W.plasma_weight(len(pos), dt))
    for n in range(15):
        run.step()
        RG, RC, RS = run.gauss_residuals()
        assert RG < 1e-12 and RS < 1e-12, (n, RG, RC, RS)
    assert np.linalg.norm(run.e) > 0 and run.counters[0] > 50


def test_alternative_schemes_differ_from_the_trapezoidal_step():
    """The same run under the three schemes gives three different fields (the parameters act)."""
    N, k = 3, 1
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    pos, vel = W.particles("beam", 500, 5, vth=0.01, drift=0.15)
    es = []
    for gamma, beta in SCHEMES:
        run = core.OracleRun(m, dt, ops, gamma=gamma, beta=beta)
        run.load(pos, vel, QE, ME, W.plasma_weight(len(pos), dt))
        run.step(8)
        es.append(run.e)
    for i in range(3):
        for j in range(i):
            assert np.linalg.norm(es[i] - es[j]) > 1e-3 * np.linalg.norm(es[j])
