"""GPU: the field update's matrix applied tet by tet (the PCG iterations' operator with PEC walls)
against the oracle's assembled operators, and whole runs with it against runs on the assembled
matrix.

The matrix is A = *eps + c K^T *nu K over the unknown W1 DoFs (Sec. III-A, eq. (maxwell_semi)),
with c = dt^2 / 4 for the trapezoidal update and c = (beta/gamma)^2 dt^2 for the three-level
Newmark-beta form of Sec. III-B: eliminating b from the oracle's coupled three-level system
[[gamma/dt *nu, beta *nu K], [-beta K^T *nu, gamma/dt *eps]] leaves gamma/dt times that A."""
import os

import numpy as np
import pytest

import paper_2111_12411_amd as F
from paper_2111_12411_amd import workloads as W
from oracle import core, mesh as omesh
from parity_util import close, elementwise

pytestmark = pytest.mark.gpu

QE, ME = -W.Q_E, W.M_E

# FP32: each entry of y sums some 100 products in FP32 (unit roundoff 6e-8), so its error is a
# few 1e-6 of the largest entry at most; FP64 as the other FP64 parity checks
TOL = {F.FP64: 1e-12, F.MIXED: 1e-5}


def oracle_matrix(m, ops, dt, gamma=0.5, beta=0.25):
    i1 = ops.int1
    Ki = ops.K[:, i1].tocsr()
    c = (beta / gamma) ** 2 * dt * dt
    return (ops.star_eps[i1][:, i1] + c * (Ki.T @ ops.star_nu @ Ki)).tocsr(), i1


def make_run(N, k, dt, prec, matfree=True, **kw):
    old = os.environ.get("FEMPIC_MATFREE")
    os.environ["FEMPIC_MATFREE"] = "1" if matfree else "0"
    try:
        return F.Run(F.Mesh.cube(N, k), dt, prec, **kw)
    finally:
        if old is None:
            del os.environ["FEMPIC_MATFREE"]
        else:
            os.environ["FEMPIC_MATFREE"] = old


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("prec", [F.FP64, F.MIXED])
@pytest.mark.parametrize("scheme", [(0.5, 0.25), (1.5, 1.0)])
def test_operator_matches_the_oracle(k, prec, scheme):
    """y = A x for random x, the iterations' form (tet by tet) and the assembled FP64 matrix,
    element-wise against the oracle's operators, on a mesh whose wall DoFs x sets too (they must
    be ignored)."""
    N = 5
    gamma, beta = scheme
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    A, i1 = oracle_matrix(m, ops, dt, gamma, beta)
    run = make_run(N, k, dt, prec, gamma=gamma, beta=beta)
    # order 2 takes the two DoFs of each edge and face together
    assert run.stats()["field_op"] == (2 if k == 2 else 1)
    rng = np.random.Generator(np.random.PCG64(70 + 2 * k + prec))
    for trial in range(2):
        x = rng.normal(size=m.n1)
        y_orc = np.zeros(m.n1)
        y_orc[i1] = A @ x[i1]
        close(run.field_matvec(x, F.OP_ASSEMBLED), y_orc, 1e-12)
        y_it = run.field_matvec(x, F.OP_ITERATION)
        close(y_it, y_orc, TOL[prec])
        assert np.all(np.delete(y_it, i1) == 0.0)
    # a field of gradients only: the curl term vanishes, A x = *eps x
    phi = rng.normal(size=m.n0)
    phi[np.nonzero(~m.int0)[0]] = 0.0
    xg = ops.G @ phi
    y_orc = np.zeros(m.n1)
    y_orc[i1] = ops.star_eps[i1][:, i1] @ xg[i1]
    assert elementwise(run.field_matvec(xg, F.OP_ITERATION), y_orc) < 10 * TOL[prec]
    run.close()


@pytest.mark.parametrize("k", [1, 2])
def test_assembled_form_when_switched_off_or_absorbing(k):
    """FEMPIC_MATFREE=0, and absorbing walls (their impedance term is assembled), iterate on the
    assembled matrix: the iterations' form then equals the assembled one to FP32 rounding."""
    N = 4
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    rng = np.random.Generator(np.random.PCG64(90 + k))
    x = rng.normal(size=m.n1)
    for kw, mf in (({}, False), ({"field_bc": F.FIELD_ABSORB}, True)):
        run = make_run(N, k, dt, F.MIXED, matfree=mf, **kw)
        assert run.stats()["field_op"] == 0
        ya = run.field_matvec(x, F.OP_ASSEMBLED)
        close(run.field_matvec(x, F.OP_ITERATION), ya, 1e-6)
        run.close()


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("prec", [F.FP64, F.MIXED])
def test_runs_agree_with_the_assembled_iterations(k, prec):
    """A beam, 15 steps, with the PCG iterations on the operator applied tet by tet and on the
    assembled matrix: the solves refine to the same target (relative residual 1e-17 in exact
    arithmetic against the assembled FP64 matrix), so fields and particles agree to 1e-12; the
    Gauss-law residual stays at rounding level."""
    N = 6
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    pos, vel = W.particles("beam", 20000, 40 + k, vth=0.01, drift=0.1)
    w = W.plasma_weight(len(pos), dt)
    runs = []
    for mf in (True, False):
        r = make_run(N, k, dt, prec, matfree=mf, pcg_rtol=1e-13)
        r.load(pos, vel, QE, ME, w)
        r.step(15)
        runs.append(r)
    e0, b0 = runs[0].fields()
    e1, b1 = runs[1].fields()
    close(e0, e1, 1e-12)
    close(b0, b1, 1e-12)
    p0, p1 = runs[0].particles()[0], runs[1].particles()[0]
    assert np.max(np.abs(p0 - p1)) < 1e-12
    rg = runs[0].gauss()
    assert max(rg) < 1e-12, rg
    for r in runs:
        r.close()


def test_matvec_rejects_bad_arguments():
    """EINVAL for an unknown form, a short buffer and a non-finite x; the run stays usable."""
    N, k = 3, 2
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    run = make_run(N, k, dt, F.MIXED)
    x = np.ones(m.n1)
    for bad in (lambda: run.field_matvec(x, 7),
                lambda: F._check(F.lib().fempic_field_matvec(run.h, F._p(x), F._p(np.zeros(m.n1)), m.n1 - 1, 0)),
                lambda: run.field_matvec(np.full(m.n1, np.nan))):
        with pytest.raises(F.FempicError) as ei:
            bad()
        assert ei.value.code == -1
    A, i1 = oracle_matrix(m, ops, dt)
    y = np.zeros(m.n1)
    y[i1] = A @ x[i1]
    close(run.field_matvec(x), y, 1e-12)
    run.close()


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("prec", [F.FP64, F.MIXED])
def test_operator_on_a_jittered_relabelled_mesh(k, prec):
    """A general mesh: the 4^3 Kuhn cube with its inner vertices moved at random (tets of unequal
    shapes), its vertices relabelled and its tets and their vertex lists shuffled, so that the DoF
    numbering and the per-tet DoF pairs come out of the general mesh builder.  The iterations'
    form against the oracle's operators on the same arrays."""
    N = 4
    xyz, tets = omesh.kuhn_cube(N)
    rng = np.random.Generator(np.random.PCG64(300 + 2 * k + prec))
    inner = np.all((xyz > 1e-9) & (xyz < 1 - 1e-9), axis=1)
    xyz = xyz.copy()
    xyz[inner] += rng.uniform(-0.15, 0.15, size=(inner.sum(), 3)) / N
    relabel = rng.permutation(len(xyz))
    xyz2 = np.empty_like(xyz)
    xyz2[relabel] = xyz
    tets2 = relabel[np.asarray(tets)]
    tets2 = tets2[rng.permutation(len(tets2))]
    tets2 = np.array([rng.permutation(t) for t in tets2])
    m = omesh.build(xyz2, tets2, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    A, i1 = oracle_matrix(m, ops, dt)
    old = os.environ.get("FEMPIC_MATFREE")
    os.environ["FEMPIC_MATFREE"] = "1"
    try:
        run = F.Run(F.Mesh.from_arrays(xyz2, tets2, k), dt, prec)
    finally:
        if old is None:
            del os.environ["FEMPIC_MATFREE"]
        else:
            os.environ["FEMPIC_MATFREE"] = old
    assert run.stats()["field_op"] == (2 if k == 2 else 1)
    x = rng.normal(size=m.n1)
    y = np.zeros(m.n1)
    y[i1] = A @ x[i1]
    close(run.field_matvec(x, F.OP_ASSEMBLED), y, 1e-12)
    close(run.field_matvec(x, F.OP_ITERATION), y, TOL[prec])
    run.close()
