"""GPU parity of the general Newmark-beta field update (Sec. III-B, eq. (maxnmb); the
alternative schemes of Sec. IV-D): the library's eliminated three-level step
against the oracle's coupled block solve, through the C ABI."""
import numpy as np
import pytest

import paper_2111_12411_amd as F
from paper_2111_12411_amd import workloads as W
from oracle import core, mesh as omesh
from parity_util import close, rel

pytestmark = pytest.mark.gpu

QE, ME = -W.Q_E, W.M_E
ALTERNATIVES = [(1.5, 1.0), (1.5, 0.8)]


def _pair(N, k, gamma, beta, n, seed, precision=F.FP64, dt_factor=10.0):
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    dt = dt_factor * core.cfl_dt(m, ops)
    pos, vel = W.particles("beam", n, seed, vth=0.01, drift=0.12)
    w = W.plasma_weight(n, dt)
    orc = core.OracleRun(m, dt, ops, gamma=gamma, beta=beta)
    orc.load(pos, vel, QE, ME, w)
    run = F.Run(F.Mesh.cube(N, k), dt, precision, pcg_rtol=1e-15, gamma=gamma, beta=beta)
    run.load(pos, vel, QE, ME, w)
    return m, orc, run


@pytest.mark.parametrize("gamma,beta", ALTERNATIVES)
@pytest.mark.parametrize("k", [1, 2])
def test_alternative_scheme_matches_the_oracle(gamma, beta, k):
    m, orc, run = _pair(5, k, gamma, beta, 15000, 70 + k)
    for n in range(20):
        orc.step()
        run.step()
        close(run.deposit(), orc.last_dg * m.int1, 1e-12)
        if n % 5 == 4:
            e, b = run.fields()
            close(e, orc.e, 1e-12)
            close(b, orc.b, 1e-12)
            RG, RC, RS = run.gauss()
            assert RG < 1e-12 and RS < 1e-12, (n, RG, RC, RS)
    pos_g, vel_g, _ = run.particles()
    close(pos_g, orc.pos, 1e-13)
    close(vel_g, orc.vel, 1e-12)


def test_alternative_scheme_mixed_precision_within_1e5():
    m, orc, run = _pair(4, 2, 1.5, 1.0, 20000, 91, precision=F.MIXED)
    for n in range(60):
        orc.step()
        run.step()
    e, b = run.fields()
    assert rel(e, orc.e) < 1e-5 and rel(b, orc.b) < 1e-5, (rel(e, orc.e), rel(b, orc.b))
    assert run.gauss()[0] < 1e-12


@pytest.mark.parametrize("precision", [F.FP64, F.MIXED])
def test_alternative_scheme_resume_is_bitwise(tmp_path, precision):
    """The three-level scheme's previous fields and current travel in the checkpoint: 6 steps,
    save, 6 more equals a fresh run restored from the file and stepped 6 times, bit for bit."""
    N, k = 5, 2
    mesh = F.Mesh.cube(N, k)
    dt = 10 * mesh.info()["dt_cfl"]
    pos, vel = W.particles("beam", 20000, 12, vth=0.01, drift=0.1)
    w = W.plasma_weight(len(pos), dt)
    a = F.Run(mesh, dt, precision, pcg_rtol=1e-14, gamma=1.5, beta=0.8)
    a.load(pos, vel, QE, ME, w)
    a.step(6)
    path = str(tmp_path / "ck.bin")
    a.save(path)
    a.step(6)
    b = F.Run(mesh, dt, precision, pcg_rtol=1e-14, gamma=1.5, beta=0.8)
    b.restore(path)
    b.step(6)
    for x, y in zip(a.fields() + a.particles(), b.fields() + b.particles()):
        assert np.array_equal(x, y)
    # a run with other parameters refuses the file
    c = F.Run(mesh, dt, precision, pcg_rtol=1e-14, gamma=1.5, beta=1.0)
    with pytest.raises(F.FempicError) as ei:
        c.restore(path)
    assert ei.value.code == -1 and "Newmark" in str(ei.value)
