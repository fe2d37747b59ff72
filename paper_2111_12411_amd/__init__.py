"""Python binding of libfempic (C ABI in include/fempic.h).

Argument marshalling only: every step of the method runs in the HIP library.
The library is loaded on first use; if it has not been built the binding
raises instead of falling back to anything else.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfempic.so")

FP64, MIXED = 0, 1
REFLECT, ABSORB = 0, 1
PUSH_AB4, PUSH_BORIS = 0, 1
FIELD_PEC, FIELD_ABSORB = 0, 1
OP_ASSEMBLED, OP_ITERATION = 0, 1
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EMESH", -4: "EOUTSIDE", -5: "ECROSS", -6: "ESOLVE",
          -7: "EDEVICE", -8: "EAGAIN", -9: "EBUSY"}


class FempicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class MeshInfo(C.Structure):
    _fields_ = [("n_vert", C.c_int64), ("n_edge", C.c_int64), ("n_face", C.c_int64), ("n_tet", C.c_int64),
                ("n1", C.c_int64), ("n1_int", C.c_int64), ("n2", C.c_int64), ("n0", C.c_int64),
                ("n0_int", C.c_int64), ("order", C.c_int32), ("n1_loc", C.c_int32), ("n2_loc", C.c_int32),
                ("n0_loc", C.c_int32), ("dt_cfl", C.c_double)]


class Params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("dt", C.c_double), ("gamma", C.c_double), ("beta", C.c_double),
                ("pcg_rtol", C.c_double), ("pcg_maxit", C.c_int32), ("particle_bc", C.c_int32),
                ("spill_slots", C.c_int32), ("gauss_every", C.c_int32), ("pusher", C.c_int32),
                ("field_bc", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("n_particles", C.c_int64), ("n_loaded", C.c_int64), ("absorbed", C.c_int64),
                ("absorbed_total", C.c_int64), ("particle_ms", C.c_double),
                ("particle_kernel_ms", C.c_double), ("continue_kernel_ms", C.c_double), ("field_ms", C.c_double), ("pcg_iters", C.c_int32),
                ("pcg_relres", C.c_double), ("crossings", C.c_int64), ("reflections", C.c_int64),
                ("spills", C.c_int64), ("gauss", C.c_double * 3), ("gauss_step", C.c_int64),
                ("a_rows", C.c_int64), ("a_nnz", C.c_int64), ("device_bytes", C.c_int64),
                ("device_peak_bytes", C.c_int64), ("phase_replays", C.c_int64), ("field_op", C.c_int32),
                ("a_inc", C.c_int64)]


class ServerParams(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_slots", C.c_int32)]


class Job(C.Structure):
    _fields_ = [("N", C.c_int32), ("L", C.c_double), ("order", C.c_int32), ("params", Params),
                ("pos", C.c_void_p), ("vel", C.c_void_p), ("n", C.c_int64), ("q", C.c_double), ("m", C.c_double),
                ("w", C.c_double), ("n_steps", C.c_int32)]


class JobResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("n1", C.c_int64), ("n2", C.c_int64), ("n", C.c_int64),
                ("e", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double)), ("pos", C.POINTER(C.c_double)),
                ("vel", C.POINTER(C.c_double)), ("gauss", C.c_double * 3), ("queue_ms", C.c_double),
                ("run_ms", C.c_double), ("step_done_ms", C.POINTER(C.c_double)), ("n_steps", C.c_int32),
                ("message", C.c_char_p)]


SYMBOLS = {
    "fempic_last_error": (C.c_char_p, []),
    "fempic_mesh_create": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]),
    "fempic_mesh_create_cube": (C.c_int32, [C.c_int32, C.c_double, C.c_int32, C.c_void_p]),
    "fempic_mesh_destroy": (C.c_int32, [C.c_void_p]),
    "fempic_mesh_info": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fempic_run_create": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fempic_run_destroy": (C.c_int32, [C.c_void_p]),
    "fempic_particles_load": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                          C.c_double]),
    "fempic_step": (C.c_int32, [C.c_void_p, C.c_int32]),
    "fempic_sync": (C.c_int32, [C.c_void_p]),
    "fempic_gauss_residual": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fempic_gauss_residual_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fempic_fields_get": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64]),
    "fempic_fields_set": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64]),
    "fempic_deposit_get": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64]),
    "fempic_field_matvec": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]),
    "fempic_rho_get": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "fempic_particles_inject": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "fempic_particles_get": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "fempic_history_get": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "fempic_run_save": (C.c_int32, [C.c_void_p, C.c_char_p]),
    "fempic_run_load": (C.c_int32, [C.c_void_p, C.c_char_p]),
    "fempic_run_set_log": (C.c_int32, [C.c_void_p, C.c_char_p]),
    "fempic_set_allocator": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fempic_stats": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fempic_footprint": (C.c_int32, [C.c_int32, C.c_int64, C.c_int64, C.c_int32, C.c_void_p]),
    "fempic_footprint_mesh": (C.c_int32, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]),
    "fempic_impressed_points": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64]),
    "fempic_impressed_set": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p,
                                         C.c_int64]),
    "fempic_server_create": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fempic_server_destroy": (C.c_int32, [C.c_void_p]),
    "fempic_submit": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fempic_poll": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p]),
    "fempic_result_release": (C.c_int32, [C.c_void_p, C.c_int64]),
}

_lib = None


def lib():
    """Load libfempic.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfempic.so is not built: run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SYMBOLS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise FempicError(code, lib().fempic_last_error().decode())


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class Mesh:
    """Tetrahedral mesh with order-k DoF numbering (host side; no GPU needed)."""

    def __init__(self, handle):
        self.h = handle

    @classmethod
    def cube(cls, N, order, L=1.0):
        h = C.c_void_p()
        _check(lib().fempic_mesh_create_cube(N, L, order, C.byref(h)))
        return cls(h)

    @classmethod
    def from_arrays(cls, xyz, tets, order):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int64)
        h = C.c_void_p()
        _check(lib().fempic_mesh_create(_p(xyz), len(xyz), _p(tets), len(tets), order, C.byref(h)))
        return cls(h)

    def info(self):
        i = MeshInfo()
        _check(lib().fempic_mesh_info(self.h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in MeshInfo._fields_}

    def impressed_points(self, n1d):
        """Points (n_tet * n1d^3, 3) at which an impressed B is sampled (fempic_impressed_points)."""
        n = self.info()["n_tet"] * n1d ** 3
        xyz = np.zeros((n, 3))
        _check(lib().fempic_impressed_points(self.h, n1d, _p(xyz), n))
        return xyz

    def footprint(self, n_particles, precision=FP64):
        """Device bytes of a run on this mesh (fempic_footprint_mesh)."""
        b = C.c_size_t()
        _check(lib().fempic_footprint_mesh(self.h, n_particles, precision, C.byref(b)))
        return b.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fempic_mesh_destroy(self.h)
            self.h = None


def params(dt, precision=FP64, pcg_rtol=1e-13, pcg_maxit=20000, gauss_every=0, gamma=0.5, beta=0.25,
           particle_bc=0, pusher=0, field_bc=0):
    return Params(precision, dt, gamma, beta, pcg_rtol, pcg_maxit, particle_bc, 0, gauss_every, pusher, field_bc)


def footprint(order, n_tet, n_particles, precision=FP64):
    """Device bytes of a run on a Kuhn-cube-like mesh of n_tet tets (fempic_footprint)."""
    b = C.c_size_t()
    _check(lib().fempic_footprint(order, n_tet, n_particles, precision, C.byref(b)))
    return b.value


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
# every callback pair ever installed: buffers made through a pair keep using it
_allocators = []


def set_allocator(alloc=None, free=None):
    """Make the library's device buffers through alloc(nbytes) -> address and
    free(address) from now on (fempic_set_allocator); no arguments restores
    hipMalloc/hipFree."""
    if alloc is None and free is None:
        _check(lib().fempic_set_allocator(None, None, None))
        return
    if alloc is None or free is None:
        raise ValueError("set_allocator needs both functions, or neither")
    a = ALLOC_FN(lambda n, ctx: alloc(n) or None)
    f = FREE_FN(lambda ptr, ctx: free(ptr))
    _allocators.append((a, f))
    _check(lib().fempic_set_allocator(C.cast(a, C.c_void_p), C.cast(f, C.c_void_p), None))


def hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process."""
    with open("/proc/self/maps") as f:
        return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})


def use_torch_allocator(device=None):
    """Route the library's device buffers through torch's caching allocator.

    torch ships its own HIP runtime.  The library shares it only when torch is
    imported before the library is first loaded; otherwise the process holds two
    runtimes and torch's memory must not reach the library's kernels, so this
    raises."""
    import torch
    lib()
    if len(hip_runtimes()) != 1:
        raise RuntimeError("two HIP runtimes are loaded (%s): import torch before the library's first use"
                           % ", ".join(hip_runtimes()))
    dev = torch.cuda.current_device() if device is None else device
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n, dev), torch.cuda.caching_allocator_delete)


class Run:
    """One simulation on the current HIP device."""

    def __init__(self, mesh, dt, precision=FP64, pcg_rtol=1e-13, pcg_maxit=20000, stream=None, gauss_every=0,
                 gamma=0.5, beta=0.25, particle_bc=0, pusher=PUSH_AB4, field_bc=FIELD_PEC):
        self.mesh = mesh
        self.info = mesh.info()
        self.h = C.c_void_p()
        p = params(dt, precision, pcg_rtol, pcg_maxit, gauss_every, gamma, beta, particle_bc, pusher, field_bc)
        _check(lib().fempic_run_create(mesh.h, C.byref(p), stream, C.byref(self.h)))
        self.n = 0

    def load(self, pos, vel, q, m, w):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
        self.n = len(pos)
        _check(lib().fempic_particles_load(self.h, _p(pos), _p(vel), self.n, q, m, w))

    def step(self, n=1):
        _check(lib().fempic_step(self.h, n))

    def sync(self):
        _check(lib().fempic_sync(self.h))

    def gauss(self):
        out = np.zeros(3)
        _check(lib().fempic_gauss_residual(self.h, _p(out)))
        return out

    def gauss_noalloc(self):
        """fempic_gauss_residual_noalloc: the same check with nothing allocated."""
        out = np.zeros(3)
        _check(lib().fempic_gauss_residual_noalloc(self.h, _p(out)))
        return out

    def fields(self):
        e = np.zeros(self.info["n1"])
        b = np.zeros(self.info["n2"])
        _check(lib().fempic_fields_get(self.h, _p(e), len(e), _p(b), len(b)))
        return e, b

    def set_fields(self, e, b):
        e = np.ascontiguousarray(e, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        _check(lib().fempic_fields_set(self.h, _p(e), len(e), _p(b), len(b)))

    def deposit(self):
        d = np.zeros(self.info["n1"])
        _check(lib().fempic_deposit_get(self.h, _p(d), len(d)))
        return d

    def field_matvec(self, x, form=None):
        """y = A x with the field update's matrix (fempic_field_matvec), natural W1 numbering;
        form OP_ASSEMBLED (default) or OP_ITERATION."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.info["n1"])
        if len(x) < len(y):
            raise ValueError("x needs n1 entries")
        _check(lib().fempic_field_matvec(self.h, _p(x), _p(y), len(y), OP_ASSEMBLED if form is None else form))
        return y

    def rho(self):
        """Nodal charge now and at load (fempic_rho_get), natural W0 numbering."""
        r = np.zeros(self.info["n0"])
        r0 = np.zeros(self.info["n0"])
        _check(lib().fempic_rho_get(self.h, _p(r), _p(r0), len(r)))
        return r, r0

    def inject(self, pos, vel):
        """Append particles of the loaded species (fempic_particles_inject)."""
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
        _check(lib().fempic_particles_inject(self.h, _p(pos), _p(vel), len(pos)))
        self.n += len(pos)

    def impress(self, B, n1d, constrained=True):
        """Project B sampled at Mesh.impressed_points(n1d) and keep it as the run's impressed
        field (fempic_impressed_set); returns its face coefficients."""
        B = np.ascontiguousarray(B, dtype=np.float64).reshape(-1, 3)
        b = np.zeros(self.info["n2"])
        _check(lib().fempic_impressed_set(self.h, _p(B), len(B), n1d, 1 if constrained else 0, _p(b), len(b)))
        return b

    def particles(self):
        pos = np.zeros((self.n, 3))
        vel = np.zeros((self.n, 3))
        tet = np.zeros(self.n, dtype=np.int64)
        _check(lib().fempic_particles_get(self.h, _p(pos), _p(vel), _p(tet), self.n))
        return pos, vel, tet

    def history(self):
        vh = np.zeros((self.n, 3, 3))
        ah = np.zeros((self.n, 3, 3))
        _check(lib().fempic_history_get(self.h, _p(vh), _p(ah), self.n))
        return vh, ah

    def save(self, path):
        """Write the run's state to a checkpoint file (fempic_run_save)."""
        _check(lib().fempic_run_save(self.h, os.fsencode(path)))

    def restore(self, path):
        """Replace the run's state with a checkpoint of a run on the same mesh (fempic_run_load)."""
        _check(lib().fempic_run_load(self.h, os.fsencode(path)))
        self.n = self.stats()["n_loaded"]

    def set_log(self, path):
        """Append one JSON line per step to `path` (fempic_run_set_log); None stops."""
        _check(lib().fempic_run_set_log(self.h, os.fsencode(path) if path else None))

    def stats(self):
        s = Stats()
        _check(lib().fempic_stats(self.h, C.byref(s)))
        out = {k: getattr(s, k) for k, _ in Stats._fields_}
        out["gauss"] = list(out["gauss"])
        return out

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fempic_run_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Server:
    """Continuous-batching server of independent runs (fempic_submit / fempic_poll)."""

    def __init__(self, hbm_budget, max_slots):
        self.h = C.c_void_p()
        sp = ServerParams(hbm_budget, max_slots)
        _check(lib().fempic_server_create(C.byref(sp), C.byref(self.h)))
        self._keep = {}

    def submit(self, N, order, pos, vel, q, m, w, n_steps, dt, precision=FP64, L=1.0, pcg_rtol=1e-13):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
        job = Job(N, L, order, params(dt, precision, pcg_rtol), _p(pos), _p(vel), len(pos), q, m, w, n_steps)
        t = C.c_int64()
        _check(lib().fempic_submit(self.h, C.byref(job), C.byref(t)))
        return t.value

    def poll(self, ticket):
        """None while queued or running; then a dict of numpy copies of the result."""
        r = JobResult()
        code = lib().fempic_poll(self.h, ticket, C.byref(r))
        if code == -8:
            return None
        _check(code)
        out = dict(status=r.status, gauss=list(r.gauss), queue_ms=r.queue_ms, run_ms=r.run_ms,
                   message=(r.message or b"").decode(errors="replace"))
        if r.status == 0:
            out["e"] = np.ctypeslib.as_array(r.e, (r.n1,)).copy()
            out["b"] = np.ctypeslib.as_array(r.b, (r.n2,)).copy()
            out["pos"] = np.ctypeslib.as_array(r.pos, (r.n * 3,)).reshape(-1, 3).copy() if r.n else np.zeros((0, 3))
            out["vel"] = np.ctypeslib.as_array(r.vel, (r.n * 3,)).reshape(-1, 3).copy() if r.n else np.zeros((0, 3))
            out["step_done_ms"] = (np.ctypeslib.as_array(r.step_done_ms, (r.n_steps,)).copy()
                                   if r.n_steps else np.zeros(0))
        _check(lib().fempic_result_release(self.h, ticket))
        return out

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fempic_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
