"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and
its host-side mesh / DoF logic agrees with the oracle (no GPU needed)."""
import os
import re

import numpy as np
import pytest

import paper_2111_12411_amd as F
from oracle import core, mesh as omesh

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fempic.h")


@pytest.fixture(scope="module")
def L():
    return F.lib()


def test_exports_every_declared_symbol(L):
    src = open(HEADER).read()
    names = set(re.findall(r"\b(fempic_[a-z0-9_]+)\s*\(", src))
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(F.SYMBOLS) == names


@pytest.mark.parametrize("N,k", [(1, 1), (2, 2), (4, 1), (4, 2), (6, 2)])
def test_cube_counts_match_oracle(N, k):
    info = F.Mesh.cube(N, k).info()
    m = omesh.cube_mesh(N, k)
    assert (info["n_vert"], info["n_edge"], info["n_face"], info["n_tet"]) == (m.nv, m.ne, m.nf, m.nt)
    assert (info["n1"], info["n1_int"], info["n2"], info["n0"], info["n0_int"]) == (m.n1, m.N1_int, m.n2, m.n0,
                                                                                    m.N0_int)
    assert (info["n1_loc"], info["n2_loc"], info["n0_loc"]) == ((6, 4, 4) if k == 1 else (20, 15, 10))


@pytest.mark.parametrize("N,k", [(2, 1), (3, 2)])
def test_cfl_bound_matches_oracle(N, k):
    """Explicit-limit bound: product (C++ Cholesky + Jacobi) vs oracle (numpy eigvalsh)."""
    info = F.Mesh.cube(N, k).info()
    m = omesh.cube_mesh(N, k)
    assert info["dt_cfl"] == pytest.approx(core.cfl_dt(m, core.assemble(m)), rel=1e-10)


def test_generic_mesh_and_errors():
    xyz, tets = omesh.kuhn_cube(2)
    rng = np.random.default_rng(0)
    perm = rng.permutation(4)
    mg = F.Mesh.from_arrays(xyz, tets[:, perm], 2)  # vertex order inside a tet does not matter
    mc = F.Mesh.cube(2, 2)
    a, b = mg.info(), mc.info()
    for key in ("n1", "n1_int", "n2", "n0_int"):
        assert a[key] == b[key]
    assert a["dt_cfl"] == pytest.approx(b["dt_cfl"], rel=1e-12)
    with pytest.raises(F.FempicError) as ei:
        F.Mesh.cube(4, 3)
    assert ei.value.code == -1  # EINVAL
    bad = np.array([[0, 1, 2, 3]])
    flat = np.zeros((4, 3))
    flat[1, 0] = 1
    flat[2, 1] = 1
    flat[3, :2] = 1  # coplanar -> zero volume
    with pytest.raises(F.FempicError) as ei:
        F.Mesh.from_arrays(flat, bad, 1)
    assert ei.value.code == -3  # EMESH
    with pytest.raises(F.FempicError):
        F.Mesh.from_arrays(xyz, np.array([[0, 1, 2, 99999]]), 1)
    assert mc.footprint(1000) > 0


def test_run_rejects_bad_params_without_gpu():
    m = F.Mesh.cube(2, 1)
    h = F.C.c_void_p()
    # Newmark-beta outside the unconditionally stable family 2 beta >= gamma >= 1/2
    for gamma, beta in ((0.4, 0.25), (1.5, 0.7), (float("nan"), 0.25), (0.5, float("inf"))):
        p = F.params(1e-11, gamma=gamma, beta=beta)
        assert F.lib().fempic_run_create(m.h, F.C.byref(p), None, F.C.byref(h)) == -1
        assert "Newmark" in F.lib().fempic_last_error().decode()
    p = F.params(-1.0)
    assert F.lib().fempic_run_create(m.h, F.C.byref(p), None, F.C.byref(h)) == -1
    # absorbing walls only with the trapezoidal scheme; unknown wall conditions
    p = F.params(1e-11, gamma=1.5, beta=1.0, field_bc=F.FIELD_ABSORB)
    assert F.lib().fempic_run_create(m.h, F.C.byref(p), None, F.C.byref(h)) == -1
    assert "trapezoidal" in F.lib().fempic_last_error().decode()
    p = F.params(1e-11, field_bc=2)
    assert F.lib().fempic_run_create(m.h, F.C.byref(p), None, F.C.byref(h)) == -1
    assert "wall" in F.lib().fempic_last_error().decode() or "boundary" in F.lib().fempic_last_error().decode()


def test_run_rejects_negative_gauss_cadence_without_gpu():
    m = F.Mesh.cube(2, 1)
    h = F.C.c_void_p()
    p = F.params(1e-11, gauss_every=-1)
    assert F.lib().fempic_run_create(m.h, F.C.byref(p), None, F.C.byref(h)) == -1
    assert "gauss_every" in F.lib().fempic_last_error().decode()


def test_set_allocator_arguments_without_gpu():
    """One of the two functions alone is EINVAL; both NULL (hipMalloc/hipFree) is OK."""
    keep = F.ALLOC_FN(lambda n, ctx: None)
    assert F.lib().fempic_set_allocator(F.C.cast(keep, F.C.c_void_p), None, None) == -1
    assert F.lib().fempic_set_allocator(None, None, None) == 0
    with pytest.raises(ValueError):
        F.set_allocator(lambda n: 0, None)
    F.set_allocator()


def test_torch_allocator_refuses_a_second_hip_runtime_without_gpu():
    """Loaded before torch, the library has a HIP runtime of its own, and torch's memory must not
    reach it: use_torch_allocator raises (in a child process, so the import order is known)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, sys.argv[1]); import paper_2111_12411_amd as F; F.lib(); "
            "import torch\n"
            "try:\n    F.use_torch_allocator(0)\nexcept RuntimeError as e:\n    print('refused:', e)\n")
    r = subprocess.run([sys.executable, "-c", code, root], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "refused: two HIP runtimes" in r.stdout, r.stdout


def test_null_handles_are_einval_without_gpu():
    """Every run entry point refuses a null handle with EINVAL and a message (no GPU is touched)."""
    L = F.lib()
    buf = (F.C.c_double * 8)()
    calls = [
        lambda: L.fempic_step(None, 1),
        lambda: L.fempic_sync(None),
        lambda: L.fempic_gauss_residual(None, buf),
        lambda: L.fempic_gauss_residual_noalloc(None, buf),
        lambda: L.fempic_fields_get(None, buf, 1, buf, 1),
        lambda: L.fempic_fields_set(None, buf, 1, buf, 1),
        lambda: L.fempic_deposit_get(None, buf, 1),
        lambda: L.fempic_field_matvec(None, buf, buf, 1, 0),
        lambda: L.fempic_particles_get(None, buf, buf, None, 1),
        lambda: L.fempic_rho_get(None, buf, buf, 1),
        lambda: L.fempic_history_get(None, buf, buf, 1),
        lambda: L.fempic_run_save(None, b"x"),
        lambda: L.fempic_run_load(None, b"x"),
        lambda: L.fempic_run_set_log(None, b"x"),
        lambda: L.fempic_stats(None, buf),
        lambda: L.fempic_particles_load(None, buf, buf, 1, 1.0, 1.0, 1.0),
    ]
    for call in calls:
        assert call() == -1
        assert L.fempic_last_error().decode() != ""
    assert L.fempic_run_destroy(None) == 0  # destroying NULL is a no-op


@pytest.mark.parametrize("N,k", [(2, 1), (5, 2), (12, 1), (20, 2)])
def test_footprint_by_tet_count_equals_mesh_footprint_for_cubes(N, k):
    """fempic_footprint(order, n_tet, n, precision) is the estimate of the N^3 cube's own counts."""
    m = F.Mesh.cube(N, k)
    for prec in (F.FP64, F.MIXED):
        for n in (0, 1000, 3_000_000):
            a = F.footprint(k, 6 * N ** 3, n, prec)
            b = m.footprint(n, prec)
            # the by-count form takes totals for interior counts, so it may only be larger
            assert b <= a <= 1.3 * b + (1 << 20), (N, k, prec, n, a, b)
    assert F.footprint(k, 6 * N ** 3, 10 ** 6, F.FP64) > F.footprint(k, 6 * N ** 3, 10 ** 6, F.MIXED)


def test_footprint_arguments_and_cube_bound_without_gpu():
    L = F.lib()
    out = F.C.c_size_t()
    assert L.fempic_footprint(3, 100, 10, F.FP64, F.C.byref(out)) == -1
    assert L.fempic_footprint(1, 0, 10, F.FP64, F.C.byref(out)) == -1
    assert L.fempic_footprint(1, 100, -1, F.FP64, F.C.byref(out)) == -1
    assert L.fempic_footprint(1, 100, 10, 7, F.C.byref(out)) == -1
    assert L.fempic_footprint(1, 100, 10, F.FP64, None) == -1
    # (N+1)^3 must stay below 2^21 vertices: N = 126 is the largest cube, and a larger one is
    # refused before anything of its size is allocated
    with pytest.raises(F.FempicError) as ei:
        F.Mesh.cube(127, 1)
    assert ei.value.code == -1 and "126" in str(ei.value)
    with pytest.raises(F.FempicError):
        F.Mesh.cube(1024, 1)
