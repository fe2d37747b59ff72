"""GPU parity of the alternative pusher (Boris leapfrog, straight path; the push
is de-linked from the current mapping, Sec. III-B) against the oracle's, through
the C ABI: the deposit of every step, fields, particles and the Gauss residual
in FP64; fields within 1e-5 in mixed precision; the parameter travels in the
checkpoint and the AB4 history read-back refuses."""
import numpy as np
import pytest

import paper_2111_12411_amd as F
from paper_2111_12411_amd import workloads as W
from oracle import core, mesh as omesh
from parity_util import close, rel

pytestmark = pytest.mark.gpu

QE, ME = -W.Q_E, W.M_E


def _pair(N, k, n, seed, precision=F.FP64):
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    pos, vel = W.particles("beam", n, seed, vth=0.01, drift=0.12)
    w = W.plasma_weight(n, dt)
    orc = core.OracleRun(m, dt, ops, pusher="boris")
    orc.load(pos, vel, QE, ME, w)
    run = F.Run(F.Mesh.cube(N, k), dt, precision, pcg_rtol=1e-15, pusher=F.PUSH_BORIS)
    run.load(pos, vel, QE, ME, w)
    return m, orc, run


@pytest.mark.parametrize("k", [1, 2])
def test_boris_matches_the_oracle(k):
    m, orc, run = _pair(5, k, 15000, 90 + k)
    for n in range(15):
        orc.step()
        run.step()
        close(run.deposit(), orc.last_dg * m.int1, 1e-12)
    st = run.stats()
    assert st["crossings"] > 1000 and st["reflections"] > 0
    e, b = run.fields()
    close(e, orc.e, 1e-12)
    close(b, orc.b, 1e-12)
    p, v, t = run.particles()
    close(p, orc.pos, 1e-13)
    close(v, orc.vel, 1e-12)
    RG, RC, RS = run.gauss()
    assert RG < 1e-12 and RC < 1e-12, (RG, RC, RS)


def test_boris_mixed_precision_within_1e5():
    m, orc, run = _pair(4, 2, 20000, 93, precision=F.MIXED)
    for n in range(60):
        orc.step()
        run.step()
    e, b = run.fields()
    assert rel(e, orc.e) < 1e-5 and rel(b, orc.b) < 1e-5, (rel(e, orc.e), rel(b, orc.b))
    assert run.gauss()[0] < 1e-12


def test_boris_parameter_checks(tmp_path):
    mesh = F.Mesh.cube(3, 1)
    dt = 10 * mesh.info()["dt_cfl"]
    pos, vel = W.particles("thermal", 500, 5, vth=0.01)
    run = F.Run(mesh, dt, F.FP64, pusher=F.PUSH_BORIS)
    run.load(pos, vel, QE, ME, 1.0)
    run.step(2)
    with pytest.raises(F.FempicError) as ei:
        run.history()
    assert ei.value.code == -1
    path = str(tmp_path / "b.bin")
    run.save(path)
    other = F.Run(mesh, dt, F.FP64)
    with pytest.raises(F.FempicError) as ei:
        other.restore(path)
    assert ei.value.code == -1 and "pusher" in str(ei.value)
    with pytest.raises(F.FempicError):
        F.Run(mesh, dt, F.FP64, pusher=7)


def test_boris_resume_is_bitwise(tmp_path):
    mesh = F.Mesh.cube(4, 2)
    dt = 10 * mesh.info()["dt_cfl"]
    pos, vel = W.particles("beam", 10000, 6, vth=0.01, drift=0.1)
    w = W.plasma_weight(len(pos), dt)
    a = F.Run(mesh, dt, F.MIXED, pcg_rtol=1e-14, pusher=F.PUSH_BORIS)
    a.load(pos, vel, QE, ME, w)
    a.step(3)  # an odd count: the state lies in the second buffer set
    path = str(tmp_path / "bb.bin")
    a.save(path)
    a.step(4)
    b = F.Run(mesh, dt, F.MIXED, pcg_rtol=1e-14, pusher=F.PUSH_BORIS)
    b.restore(path)
    b.step(4)
    for x, y in zip(a.fields() + a.particles(), b.fields() + b.particles()):
        assert np.array_equal(x, y)
    b.save(str(tmp_path / "bb2.bin"))  # its history arrays are finite (zero), so the file loads
    c = F.Run(mesh, dt, F.MIXED, pcg_rtol=1e-14, pusher=F.PUSH_BORIS)
    c.restore(str(tmp_path / "bb2.bin"))

