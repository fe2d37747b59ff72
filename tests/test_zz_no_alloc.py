"""fempic_gauss_residual_noalloc through the C ABI: the same residuals, bit for
bit, as fempic_gauss_residual, with nothing allocated during the call; two calls
in a row, the second on a smaller run, and a mesh too large for the scratch."""
import ctypes as C

import numpy as np
import pytest

import paper_2111_12411_amd as F
from paper_2111_12411_amd import workloads as W

pytestmark = pytest.mark.gpu

QE, ME = -W.Q_E, W.M_E


def _run(N, k, n, seed, precision):
    mesh = F.Mesh.cube(N, k)
    dt = 5 * mesh.info()["dt_cfl"]
    pos, vel = W.particles("beam", n, seed, vth=0.01, drift=0.1)
    run = F.Run(mesh, dt, precision, pcg_rtol=1e-14)
    run.load(pos, vel, QE, ME, W.plasma_weight(n, dt))
    return run


def _noalloc_counting(run):
    """fempic_gauss_residual_noalloc with an allocator installed that counts (and refuses) every
    request, so any allocation the call made would show."""
    calls = []
    keep_a = F.ALLOC_FN(lambda n, ctx: calls.append(n) or None)
    keep_f = F.FREE_FN(lambda p, ctx: calls.append(-1))
    L = F.lib()
    assert L.fempic_set_allocator(C.cast(keep_a, C.c_void_p), C.cast(keep_f, C.c_void_p), None) == 0
    try:
        out = np.zeros(3)
        code = L.fempic_gauss_residual_noalloc(run.h, F._p(out))
    finally:
        assert L.fempic_set_allocator(None, None, None) == 0
    assert calls == []
    assert code == 0, L.fempic_last_error().decode()
    return out


def test_noalloc_gauss_equals_gauss_on_two_runs_the_second_smaller():
    big = _run(8, 2, 60000, 3, F.FP64)
    big.step(4)
    want = big.gauss()
    got = _noalloc_counting(big)
    assert np.array_equal(got, want), (got, want)
    assert got[0] < 1e-12
    # a random e breaks Gauss's law: the residual is O(1) and still the same bit for bit
    info = big.info
    e_bad = np.random.default_rng(4).normal(size=info["n1"]) * 1e3
    _, b = big.fields()
    big.set_fields(e_bad, b)
    want = big.gauss()
    got = _noalloc_counting(big)
    assert np.array_equal(got, want) and got[0] > 1e-3, (got, want)
    big.close()
    # the second call, on a smaller run (fewer tets, DoFs and particles, order 1, mixed precision):
    # whatever the first call left in the scratch does not reach it
    small = _run(3, 1, 500, 5, F.MIXED)
    small.step(2)
    want = small.gauss()
    got = _noalloc_counting(small)
    assert np.array_equal(got, want), (got, want)
    got2 = small.gauss_noalloc()
    assert np.array_equal(got2, want)
    small.close()


def test_noalloc_gauss_refuses_a_mesh_beyond_the_scratch():
    """The 48^3 cube at order 2 needs about 140 MB of scratch for the check; the library holds 96 MiB."""
    run = _run(48, 2, 1000, 7, F.MIXED)
    out = np.zeros(3)
    code = F.lib().fempic_gauss_residual_noalloc(run.h, F._p(out))
    assert code == -1 and "scratch" in F.lib().fempic_last_error().decode()
    assert np.all(out == 0)
    # the run itself is untouched: the ordinary check still works
    run.gauss()
    run.close()
