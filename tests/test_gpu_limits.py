"""GPU checks of the library's limits through the C ABI: the crossing cap, a mesh
handle destroyed while its run lives, and the device footprint against what a
run really holds."""
import ctypes as C

import numpy as np
import pytest

import paper_2111_12411_amd as F
from paper_2111_12411_amd import workloads as W
from oracle import core, mesh as omesh
from parity_util import close

pytestmark = pytest.mark.gpu

QE, ME = -W.Q_E, W.M_E


def fast_particle(speed):
    """One electron that starts on an interior face (x = y inside a hex of the 6^3 cube) and leaves
    its tet through that face at once, so its whole path goes to the continuation kernel; the
    oracle counts 64 face crossings at 5.45e9 m/s and more than 64 at 5.6e9 m/s (walls reflect)."""
    p0 = np.array([[1.3 / 6, 1.3 / 6, 2.55 / 6]])
    d = np.array([0.37, 1.0, 0.21])
    return p0, (speed * d / np.linalg.norm(d))[None, :]


def test_path_with_64_crossings_is_legal_and_matches_the_oracle():
    N, k = 6, 1
    m = omesh.cube_mesh(N, k)
    dt = 5 * core.cfl_dt(m, core.assemble(m))
    pos, vel = fast_particle(5.45e9)
    orc = core.OracleRun(m, dt, particles_only=True)
    orc.load(pos, vel, QE, ME, 1.0)
    dg = orc.particle_step()
    assert orc.counters[0] == 64
    run = F.Run(F.Mesh.cube(N, k), dt, F.FP64, pcg_rtol=1e-14)
    run.load(pos, vel, QE, ME, 1.0)
    run.step()
    st = run.stats()
    assert st["crossings"] == 64 and st["reflections"] == orc.counters[1]
    close(run.deposit(), dg * m.int1, 1e-12)
    p, v, t = run.particles()
    close(p, orc.pos, 1e-13)
    close(v, orc.vel, 1e-13)
    assert t[0] == orc.tet[0]


def test_more_than_64_crossings_is_ecross_and_sticky():
    N, k = 6, 1
    m = omesh.cube_mesh(N, k)
    dt = 5 * core.cfl_dt(m, core.assemble(m))
    pos, vel = fast_particle(5.6e9)
    orc = core.OracleRun(m, dt, particles_only=True)
    orc.load(pos, vel, QE, ME, 1.0)
    with pytest.raises(RuntimeError):
        orc.particle_step()  # the oracle's status is ECROSS too
    run = F.Run(F.Mesh.cube(N, k), dt, F.FP64, pcg_rtol=1e-14)
    run.load(pos, vel, QE, ME, 1.0)
    with pytest.raises(F.FempicError) as ei:
        run.step()
    assert ei.value.code == -5  # ECROSS, not ENOMEM after growing the segment buffer
    with pytest.raises(F.FempicError) as ei:
        run.step()
    assert ei.value.code == -5


def test_mesh_handle_destroyed_while_its_run_lives():
    """fempic_mesh_destroy before any use of the run: load, step and read-back still work and
    give what a run whose mesh handle is alive gives."""
    L = F.lib()
    N, k = 4, 2
    dt = 5 * core.cfl_dt(omesh.cube_mesh(N, k), core.assemble(omesh.cube_mesh(N, k)))
    pos, vel = W.particles("thermal", 3000, 17, vth=0.02)
    outs = []
    for destroy_first in (True, False):
        mh = C.c_void_p()
        assert L.fempic_mesh_create_cube(N, 1.0, k, C.byref(mh)) == 0
        info = F.MeshInfo()
        assert L.fempic_mesh_info(mh, C.byref(info)) == 0
        rh = C.c_void_p()
        p = F.params(dt, F.FP64, 1e-14)
        assert L.fempic_run_create(mh, C.byref(p), None, C.byref(rh)) == 0
        if destroy_first:
            assert L.fempic_mesh_destroy(mh) == 0
        pp = np.ascontiguousarray(pos)
        vv = np.ascontiguousarray(vel)
        assert L.fempic_particles_load(rh, F._p(pp), F._p(vv), len(pp), QE, ME, 1e4) == 0
        assert L.fempic_step(rh, 3) == 0
        e = np.zeros(info.n1)
        b = np.zeros(info.n2)
        assert L.fempic_fields_get(rh, F._p(e), len(e), F._p(b), len(b)) == 0
        g = np.zeros(3)
        assert L.fempic_gauss_residual(rh, F._p(g)) == 0
        outs.append((e, b, g))
        assert L.fempic_run_destroy(rh) == 0
        if not destroy_first:
            assert L.fempic_mesh_destroy(mh) == 0
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("N,k,precision,n", [(6, 1, F.FP64, 50000), (6, 2, F.MIXED, 200000),
                                             (10, 2, F.FP64, 20000), (3, 1, F.MIXED, 0)])
def test_device_bytes_stay_within_the_footprint(N, k, precision, n):
    """What a run really holds (its peak, through load and steps) never exceeds fempic_footprint;
    the estimate is not loose by more than a third either."""
    mesh = F.Mesh.cube(N, k)
    dt = 10 * mesh.info()["dt_cfl"]
    pos, vel = W.particles("beam", n, 5 + N, vth=0.01, drift=0.1)
    run = F.Run(mesh, dt, precision, pcg_rtol=1e-13)
    run.load(pos, vel, QE, ME, W.plasma_weight(max(n, 1), dt))
    run.step(3)
    st = run.stats()
    est = F.footprint(k, 6 * N ** 3, n, precision)
    assert st["device_peak_bytes"] <= mesh.footprint(n, precision) <= est, (st["device_peak_bytes"], est)
    assert st["device_peak_bytes"] > 0.66 * mesh.footprint(n, precision)
    assert 0 < st["device_bytes"] <= st["device_peak_bytes"]
    run.close()


@pytest.mark.parametrize("k", [1, 2])
def test_absorbing_walls_match_the_oracle(k):
    """FEMPIC_ABSORB: a beam into the z walls of the 5^3 cube, FP64, 15 steps.  Every step's deposit
    DoF by DoF and the absorbed count against the oracle; then the surviving particles (the same
    set), fields and the Gauss residual; absorbed particles read back with tet -1 and NaN state."""
    N = 5
    m = omesh.cube_mesh(N, k)
    ops = core.assemble(m)
    dt = 10 * core.cfl_dt(m, ops)
    pos, vel = W.particles("beam", 12000, 81 + k, vth=0.01, drift=0.12)
    w = W.plasma_weight(len(pos), dt)
    orc = core.OracleRun(m, dt, ops, absorb=True)
    orc.load(pos, vel, QE, ME, w)
    run = F.Run(F.Mesh.cube(N, k), dt, F.FP64, pcg_rtol=1e-15, particle_bc=F.ABSORB)
    run.load(pos, vel, QE, ME, w)
    for n in range(15):
        c0 = orc.counters.copy()
        orc.step()
        run.step()
        close(run.deposit(), orc.last_dg * m.int1, 1e-12)
        st = run.stats()
        assert st["absorbed"] == orc.counters[2] - c0[2], n
        assert st["reflections"] == 0 and st["n_particles"] == int((orc.tet >= 0).sum())
    assert st["absorbed_total"] > 2000 and st["n_loaded"] == len(pos)
    p, v, t = run.particles()
    alive = orc.tet >= 0
    assert np.array_equal(t < 0, ~alive)
    assert np.all(np.isnan(p[~alive])) and np.all(np.isnan(v[~alive]))
    close(p[alive], orc.pos[alive], 1e-13)
    close(v[alive], orc.vel[alive], 1e-12)
    e, b = run.fields()
    close(e, orc.e, 1e-12)
    close(b, orc.b, 1e-12)
    rho, _ = run.rho()
    close(rho, orc.rho() * m.int0, 1e-12)
    RG, RC, RS = run.gauss()
    assert RG < 1e-12 and RC < 1e-12, (RG, RC, RS)


def test_absorbing_run_resumes_bitwise(tmp_path):
    N, k = 5, 2
    mesh = F.Mesh.cube(N, k)
    dt = 10 * mesh.info()["dt_cfl"]
    pos, vel = W.particles("beam", 20000, 13, vth=0.01, drift=0.1)
    w = W.plasma_weight(len(pos), dt)
    a = F.Run(mesh, dt, F.MIXED, pcg_rtol=1e-14, particle_bc=F.ABSORB)
    a.load(pos, vel, QE, ME, w)
    a.step(5)
    path = str(tmp_path / "ck.bin")
    a.save(path)
    a.step(5)
    b = F.Run(mesh, dt, F.MIXED, pcg_rtol=1e-14, particle_bc=F.ABSORB)
    b.restore(path)
    assert b.stats()["n_loaded"] == len(pos) and b.stats()["n_particles"] < len(pos)
    b.step(5)
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)
    pa, va, ta = a.particles()
    pb, vb, tb = b.particles()
    assert np.array_equal(ta, tb)
    ok = ta >= 0
    assert np.array_equal(pa[ok], pb[ok]) and np.array_equal(va[ok], vb[ok])
