"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances: FP64 mode, 1e-12 relative on fields, deposits, nodal charge and
particle states, both norm-wise and element-wise (the largest difference over
the largest entry); mixed mode, 1e-5 relative on fields after 100 steps; Gauss
residual R_G <= 1e-12 in both modes.
"""
import os

import numpy as np
import pytest

import paper_2111_12411_amd as F
from paper_2111_12411_amd import workloads as W
from oracle import core, mesh as omesh
from flux_check import relative_net_flux
from parity_util import close, elementwise, rel

pytestmark = pytest.mark.gpu

QE, ME = -W.Q_E, W.M_E
# host threads of the chunked oracle step at full size (the GPU machine gives a share of 16)
ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))


def cfl(N, k):
    """Oracle element bound at N, from the N=4 mesh (Kuhn meshes are similar: dt_cfl ~ 1/N)."""
    m = omesh.cube_mesh(4, k)
    return core.cfl_dt(m, core.assemble(m)) * 4.0 / N


def pair(N, k, dt, pos, vel, w, precision=F.FP64, particles_only=False):
    m = omesh.cube_mesh(N, k)
    orc = core.OracleRun(m, dt, particles_only=particles_only)
    orc.load(pos, vel, QE, ME, w)
    run = F.Run(F.Mesh.cube(N, k), dt, precision, pcg_rtol=1e-14)
    run.load(pos, vel, QE, ME, w)
    return m, orc, run


def test_c1_order1_fp64_100_steps():
    """Plain FP64, order-1 Whitney, 4^3 cube, 1000 thermal electrons, dt = 5 dt_cfl, 100 steps."""
    dt = 5 * cfl(4, 1)
    pos, vel = W.config_particles(1)
    w = W.plasma_weight(len(pos), dt)
    m, orc, run = pair(4, 1, dt, pos, vel, w)
    # start-up state
    vh_g, ah_g = run.history()
    assert rel(vh_g, orc.vh) < 1e-14
    r_g, r0_g = run.rho()
    close(r0_g, orc.rho0 * m.int0, 1e-13)
    for n in range(100):
        c0 = orc.counters.copy()
        orc.step()
        run.step()
        st = run.stats()
        assert st["crossings"] == orc.counters[0] - c0[0] and st["reflections"] == orc.counters[1] - c0[1], n
        if n < 5 or n % 10 == 9:
            close(run.deposit(), orc.last_dg * m.int1, 1e-12)
            RG, RC, RS = run.gauss()
            assert RG < 1e-12 and RC < 1e-12, (n, RG, RC, RS)
    e, b = run.fields()
    pos_g, vel_g, tet_g = run.particles()
    close(e, orc.e, 1e-12)
    close(b, orc.b, 1e-12)
    close(pos_g, orc.pos, 1e-13)
    close(vel_g, orc.vel, 1e-12)
    assert np.array_equal(tet_g, orc.tet)
    r_g, _ = run.rho()
    close(r_g, orc.rho() * m.int0, 1e-12)
    st = run.stats()
    assert st["steps"] == 100 and st["crossings"] > 0


@pytest.mark.parametrize("k", [1, 2])
def test_fp64_beam_parity(k):
    """FP64, order k, 6^3 cube, 20k-electron beam at 0.1c, dt = 10 dt_cfl, 20 steps (walls reflect):
    every step's deposit, then fields, particles and the Gauss residual."""
    dt = 10 * cfl(6, k)
    pos, vel = W.particles("beam", 20000, 2007, vth=0.005, drift=0.1)
    w = W.plasma_weight(len(pos), dt)
    m, orc, run = pair(6, k, dt, pos, vel, w)
    refl = 0
    for n in range(20):
        c0 = orc.counters.copy()
        orc.step()
        run.step()
        close(run.deposit(), orc.last_dg * m.int1, 1e-12)
        st = run.stats()
        # the same face crossings and wall reflections, step by step
        assert st["crossings"] == orc.counters[0] - c0[0], n
        assert st["reflections"] == orc.counters[1] - c0[1], n
        refl += st["reflections"]
    assert refl > 100
    e, b = run.fields()
    close(e, orc.e, 1e-12)
    close(b, orc.b, 1e-12)
    # magnetic Gauss law: no net flux out of any tet
    assert relative_net_flux(m, b) < 1e-13
    pos_g, vel_g, _ = run.particles()
    close(pos_g, orc.pos, 1e-13)
    close(vel_g, orc.vel, 1e-12)
    vh_g, ah_g = run.history()
    close(vh_g, orc.vh, 1e-12)
    close(ah_g, orc.ah, 1e-12)
    RG, RC, RS = run.gauss()
    assert RG < 1e-12, (RG, RC, RS)


def test_ragged_and_empty_inputs():
    """Particle counts that leave ragged tiles, a single particle, and no particles."""
    for n, N, k in [(1, 3, 1), (257, 3, 2), (0, 2, 1)]:
        dt = 5 * cfl(N, k)
        pos, vel = W.particles("thermal", n, 31 + n, vth=0.05)
        rng = np.random.default_rng(n)
        mm = omesh.cube_mesh(N, k)
        e0, b0 = rng.normal(size=mm.n1) * 1e3 * mm.int1, rng.normal(size=mm.n2) * 1e-5
        m, orc, run = pair(N, k, dt, pos, vel, 1.0)
        orc.e, orc.b = e0.copy(), b0.copy()
        run.set_fields(e0, b0)
        for _ in range(3):
            orc.step()
            run.step()
        e, b = run.fields()
        close(e, orc.e, 1e-12)
        close(b, orc.b, 1e-12)
        if n:
            pos_g, vel_g, _ = run.particles()
            close(pos_g, orc.pos, 1e-13)
            close(vel_g, orc.vel, 1e-12)


def test_random_fields_one_step_exact():
    """Nonzero E and B everywhere: one step, per-particle state and deposit (k = 1, 2)."""
    for k in (1, 2):
        N = 5
        dt = 10 * cfl(N, k)
        pos, vel = W.particles("beam", 5000, 77, vth=0.02, drift=0.15)
        m = omesh.cube_mesh(N, k)
        e0, b0 = W.random_fields(m.n1, m.n2, 5 + k, e_scale=2e4, b_scale=2e-4)
        e0 = e0 * m.int1
        m, orc, run = pair(N, k, dt, pos, vel, 1e3)
        orc.e, orc.b = e0.copy(), b0.copy()
        run.set_fields(e0, b0)
        dg_o = orc.particle_step()
        run.step()
        close(run.deposit(), dg_o * m.int1, 1e-12)
        pos_g, vel_g, tet_g = run.particles()
        close(pos_g, orc.pos, 1e-14)
        close(vel_g, orc.vel, 1e-13)
        assert np.array_equal(tet_g, orc.tet)
        vh_g, ah_g = run.history()
        close(vh_g, orc.vh, 1e-13)
        close(ah_g, orc.ah, 1e-13)


def test_bitwise_determinism():
    dt = 10 * cfl(5, 2)
    pos, vel = W.particles("beam", 30000, 99, vth=0.01, drift=0.15)
    out = []
    for rep in range(2):
        run = F.Run(F.Mesh.cube(5, 2), dt, F.FP64, pcg_rtol=1e-14)
        run.load(pos, vel, QE, ME, W.plasma_weight(len(pos), dt))
        run.step(5)
        e, b = run.fields()
        p, v, t = run.particles()
        out.append((e, b, p, v, t, run.deposit()))
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("k", [1, 2])
def test_mixed_precision_fields_within_1e5(k):
    """Mixed precision (FP32 gather/push + FP32 PCG with FP64 refinement) vs the FP64 oracle:
    4^3 cube, order k, 20k thermal electrons at 0.02c, dt = 10 dt_cfl, 100 steps."""
    dt = 10 * cfl(4, k)
    pos, vel = W.particles("thermal", 20000, 3007, vth=0.02)
    w = W.plasma_weight(len(pos), dt)
    m, orc, run = pair(4, k, dt, pos, vel, w, precision=F.MIXED)
    for n in range(100):
        orc.step()
        run.step()
    e, b = run.fields()
    assert rel(e, orc.e) < 1e-5 and rel(b, orc.b) < 1e-5, (rel(e, orc.e), rel(b, orc.b))
    # element-wise: mixed precision moves no single DoF far either
    assert elementwise(e, orc.e) < 1e-4 and elementwise(b, orc.b) < 1e-4, (elementwise(e, orc.e),
                                                                          elementwise(b, orc.b))
    assert relative_net_flux(m, b) < 1e-13
    RG, RC, RS = run.gauss()
    assert RG < 1e-12, (RG, RC, RS)


def test_full_size_benchmark_step_whole_deposit():
    """The benchmark's launch configuration (40^3 cube, order 2, 16M electrons), FP64: one step with
    random fields, every DoF of the deposit and every particle against the oracle (its chunked step
    on the host's threads), and charge continuity of the whole deposit (R_C) at full size."""
    N, k, n = 40, 2, 16_000_000
    dt = 10 * cfl(N, k)
    pos, vel = W.config_particles(3)
    assert len(pos) == n
    m = omesh.cube_mesh(N, k)
    e0, b0 = W.random_fields(m.n1, m.n2, 303, e_scale=1e3, b_scale=1e-5)
    e0 = e0 * m.int1
    w = W.config_weight(3, n, dt)
    run = F.Run(F.Mesh.cube(N, k), dt, F.FP64, pcg_rtol=1e-14)
    run.load(pos, vel, QE, ME, w)
    run.set_fields(e0, b0)
    run.step()
    dg_g = run.deposit()
    pos_g, vel_g, tet_g = run.particles()
    # the random initial e does not satisfy Gauss's law, so only the deposit's own
    # continuity residual R_C is meaningful here
    RG, RC, RS = run.gauss()
    assert RC < 1e-12, RC
    run.close()
    orc = core.OracleRun(m, dt, particles_only=True)
    orc.load(pos, vel, QE, ME, w)
    del pos, vel
    orc.e, orc.b = e0.copy(), b0.copy()
    dg_o = orc.particle_step(threads=ORACLE_THREADS)
    close(dg_g, dg_o * m.int1, 1e-12)
    close(pos_g, orc.pos, 1e-13)
    close(vel_g, orc.vel, 1e-12)
    tets_agree(m, pos_g, tet_g, orc.tet)


def test_full_size_beam_step_whole_deposit():
    """The beam workload at full size (20^3 cube, order 2, 1M electrons at 0.1c, FP64): two steps
    from random fields, every DoF of each step's deposit and the particle state against the oracle."""
    N, k = 20, 2
    dt = 10 * cfl(N, k)
    pos, vel = W.config_particles(2)
    m = omesh.cube_mesh(N, k)
    e0, b0 = W.random_fields(m.n1, m.n2, 202, e_scale=1e3, b_scale=1e-5)
    e0 = e0 * m.int1
    w = W.config_weight(2, len(pos), dt)
    run = F.Run(F.Mesh.cube(N, k), dt, F.FP64, pcg_rtol=1e-14)
    run.load(pos, vel, QE, ME, w)
    run.set_fields(e0, b0)
    orc = core.OracleRun(m, dt, particles_only=True)
    orc.load(pos, vel, QE, ME, w)
    orc.e, orc.b = e0.copy(), b0.copy()
    for n in range(2):
        run.set_fields(e0, b0)  # the same fields for both steps on both sides
        c0 = orc.counters.copy()
        run.step()
        dg_o = orc.particle_step(threads=ORACLE_THREADS)
        close(run.deposit(), dg_o * m.int1, 1e-12)
        st = run.stats()
        assert st["crossings"] == orc.counters[0] - c0[0] and st["reflections"] == orc.counters[1] - c0[1]
    pos_g, vel_g, tet_g = run.particles()
    close(pos_g, orc.pos, 1e-13)
    close(vel_g, orc.vel, 1e-12)
    tets_agree(m, pos_g, tet_g, orc.tet)


def test_full_size_mixed_sampled():
    """Mixed precision at the benchmark size: a sample of particles against the FP64 oracle one by
    one (FP32 gather and force), and the whole deposit within 1e-5."""
    N, k, n = 40, 2, 16_000_000
    dt = 10 * cfl(N, k)
    pos, vel = W.config_particles(3)
    m = omesh.cube_mesh(N, k)
    e0, b0 = W.random_fields(m.n1, m.n2, 303, e_scale=1e3, b_scale=1e-5)
    e0 = e0 * m.int1
    w = W.config_weight(3, n, dt)
    run = F.Run(F.Mesh.cube(N, k), dt, F.MIXED, pcg_rtol=1e-14)
    run.load(pos, vel, QE, ME, w)
    run.set_fields(e0, b0)
    run.step()
    pos_g, vel_g, tet_g = run.particles()
    RG, RC, RS = run.gauss()
    assert RC < 1e-12, RC
    idx = np.random.default_rng(5).choice(n, 3000, replace=False)
    orc = core.OracleRun(m, dt, particles_only=True)
    orc.load(pos[idx], vel[idx], QE, ME, w)
    orc.e, orc.b = e0.copy(), b0.copy()
    orc.particle_step()
    assert rel(pos_g[idx], orc.pos) < 1e-9
    assert rel(vel_g[idx], orc.vel) < 2e-5
    tets_agree(m, pos_g[idx], tet_g[idx], orc.tet, tol=1e-9)


def tets_agree(m, pos, tet_a, tet_b, tol=1e-12):
    """Tet ids are unique except for a particle on a face shared by two tets (either is correct):
    where the ids differ, the position must lie in both tets up to rounding."""
    diff = np.nonzero(tet_a != tet_b)[0]
    assert len(diff) <= max(3, len(tet_a) // 100000), len(diff)
    for i in diff:
        for t in (tet_a[i], tet_b[i]):
            lam = m.aff[t] + m.grad[t] @ pos[i]
            assert lam.min() > -tol, (i, t, lam)


def test_gauss_residuals_and_nodal_charge_match_the_oracle():
    """a8: the GPU's nodal charge rho~ (now and at load) equals the oracle's DoF by DoF, and its
    R_G, R_C, R_S stay at rounding level with the oracle's.  Negative control: a random e set on
    both sides breaks Gauss's law, and R_G and R_S then come out O(1) and equal to the oracle's,
    while R_C (deposit only) stays at rounding level."""
    for k in (1, 2):
        N = 4
        dt = 5 * cfl(N, k)
        pos, vel = W.particles("beam", 6000, 41 + k, vth=0.01, drift=0.1)
        w = W.plasma_weight(len(pos), dt)
        m, orc, run = pair(N, k, dt, pos, vel, w)
        for n in range(10):
            orc.step()
            run.step()
        rho_g, rho0_g = run.rho()
        close(rho0_g, orc.rho0 * m.int0, 1e-13)
        close(rho_g, orc.rho() * m.int0, 1e-12)
        g_gpu = run.gauss()
        g_orc = orc.gauss_residuals()
        assert max(g_gpu) < 1e-12 and max(g_orc) < 1e-12, (g_gpu, g_orc)
        e_bad = np.random.default_rng(9).normal(size=m.n1) * m.int1 * np.abs(orc.e).max()
        orc.e = e_bad.copy()
        run.set_fields(e_bad, orc.b)
        g_gpu = run.gauss()
        g_orc = orc.gauss_residuals()
        assert g_orc[0] > 1e-3 and g_orc[2] > 1e-3 and g_orc[1] < 1e-12, g_orc
        assert g_gpu[0] == pytest.approx(g_orc[0], rel=1e-10) and g_gpu[2] == pytest.approx(g_orc[2], rel=1e-10)
        assert g_gpu[1] < 1e-12, g_gpu


def test_failure_modes():
    m = F.Mesh.cube(3, 1)
    run = F.Run(m, 1e-10, F.FP64)
    with pytest.raises(F.FempicError) as ei:
        run.load(np.array([[2.0, 2.0, 2.0]]), np.zeros((1, 3)), QE, ME, 1.0)
    assert ei.value.code == -4  # EOUTSIDE
    bad_v = np.zeros((2, 3))
    bad_v[1, 2] = np.nan
    with pytest.raises(F.FempicError) as ei:
        run.load(np.full((2, 3), 0.5), bad_v, QE, ME, 1.0)
    assert ei.value.code == -1 and "non-finite" in str(ei.value)  # EINVAL
    e_bad, b_ok = np.zeros(m.info()["n1"]), np.zeros(m.info()["n2"])
    e_bad[3] = np.inf
    with pytest.raises(F.FempicError) as ei:
        run.set_fields(e_bad, b_ok)
    assert ei.value.code == -1 and "non-finite" in str(ei.value)
    pos, vel = W.particles("thermal", 500, 5, vth=0.05)
    run2 = F.Run(m, 5 * cfl(3, 1), F.FP64, pcg_rtol=1e-30, pcg_maxit=1)
    run2.load(pos, vel, QE, ME, 1e6)
    with pytest.raises(F.FempicError) as ei:
        run2.step()
    assert ei.value.code == -6  # ESOLVE
    with pytest.raises(F.FempicError):  # sticky
        run2.step()


def test_step_redone_when_counts_exceed_bounds():
    """The queue and spill stages run on counts that stay on the device, with launches sized by
    bounds from the previous step; a step whose counts exceed them is redone with the exact counts.
    Particles at rest for two steps (empty queue, so the bounds are at their minimum), then a strong
    field set before the second makes most of them cross faces in the third: that step must be
    redone, and it must match the oracle started from the GPU's state and fields."""
    N, k = 4, 2
    m = omesh.cube_mesh(N, k)
    dt = 5 * cfl(N, k)
    n = 12000
    pos, _ = W.particles("thermal", n, 4242)
    vel = np.zeros_like(pos)
    w = W.plasma_weight(n, dt)
    run = F.Run(F.Mesh.cube(N, k), dt, F.FP64)
    run.load(pos, vel, QE, ME, w)
    run.step(1)
    assert run.stats()["crossings"] == 0
    e0, b0 = W.random_fields(m.n1, m.n2, 77, e_scale=2e5, b_scale=1e-5)
    run.set_fields(e0 * m.int1, b0)
    run.step(1)
    assert run.stats()["crossings"] == 0
    p0, v0, t0 = run.particles()
    vh0, ah0 = run.history()
    e1, b1 = run.fields()
    run.step(1)
    p1, v1, t1 = run.particles()
    # far more queued paths than the bound taken from the previous (empty) step
    assert run.stats()["crossings"] > 3 * 4096
    orc = core.OracleRun(m, dt, particles_only=True)
    orc.load(p0, v0, QE, ME, w, tet=t0)
    orc.vh = np.ascontiguousarray(vh0, dtype=np.float64)
    orc.ah = np.ascontiguousarray(ah0, dtype=np.float64)
    orc.e, orc.b = e1.copy(), b1.copy()
    orc.particle_step()
    assert rel(p1, orc.pos) < 1e-13
    assert rel(v1, orc.vel) < 1e-12
    assert np.mean(t1 == orc.tet) > 0.999
    run.close()
