"""ctypes bridge to the oracle's plain-C particle loop (oracle_particles.c).

TEST INFRASTRUCTURE ONLY.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle_particles.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force=True):
    """Compile the oracle loop with gcc (plain C, -O2, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-fopenmp", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class OMesh(C.Structure):
    _fields_ = [
        ("n_tet", C.c_int64),
        ("aff", C.c_void_p), ("grad", C.c_void_p), ("nbr", C.c_void_p),
        ("n1", C.c_int32), ("n2", C.c_int32), ("n0", C.c_int32),
        ("map1", C.c_void_p), ("map2", C.c_void_p), ("map0", C.c_void_p),
        ("e1", C.c_void_p), ("q1", C.c_void_p), ("f2", C.c_void_p), ("q2", C.c_void_p), ("p0", C.c_void_p),
        ("n_gl", C.c_int32), ("gl_x", C.c_void_p), ("gl_w", C.c_void_p),
    ]


_lib = None


def lib():
    """The compiled loop; FEMPIC_ORACLE_LIB names another build of the same source
    (the sanitizer test loads one built with UBSan)."""
    global _lib
    if _lib is None:
        path = os.environ.get("FEMPIC_ORACLE_LIB")
        if not path:
            if not os.path.exists(LIB):
                build()
            path = LIB
        L = C.CDLL(path)
        vp, i64, f64 = C.c_void_p, C.c_int64, C.c_double
        L.oracle_step.restype = C.c_int
        L.oracle_step.argtypes = [vp, vp, vp, i64, vp, i64, vp, vp, vp, vp, vp, f64, f64, f64, f64, vp, vp, C.c_int,
                                  C.c_int]
        L.oracle_step_chunked.restype = C.c_int
        L.oracle_step_chunked.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, f64, f64, f64, f64, vp, i64, vp,
                                          C.c_int, vp, C.c_int, C.c_int]
        L.oracle_startup.restype = None
        L.oracle_startup.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, f64, f64, f64]
        L.oracle_gather.restype = None
        L.oracle_gather.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
        L.oracle_rho.restype = None
        L.oracle_rho.argtypes = [vp, i64, vp, vp, f64, vp]
        L.oracle_path_deposit.restype = C.c_int64
        L.oracle_path_deposit.argtypes = [vp, i64, vp, f64, vp, vp, vp, vp, vp]
        L.oracle_first_negative.restype = C.c_int
        L.oracle_first_negative.argtypes = [vp, f64, f64, vp]
        _lib = L
    return _lib


def ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class CMesh:
    """Keeps the numpy arrays alive behind an OMesh struct."""

    def __init__(self, mesh, tables, gl):
        e1, q1, f2, q2, p0 = tables
        self.arrs = dict(
            aff=np.ascontiguousarray(mesh.aff, dtype=np.float64),
            grad=np.ascontiguousarray(mesh.grad, dtype=np.float64),
            nbr=np.ascontiguousarray(mesh.nbr, dtype=np.int64),
            map1=np.ascontiguousarray(mesh.map1, dtype=np.int64),
            map2=np.ascontiguousarray(mesh.map2, dtype=np.int64),
            map0=np.ascontiguousarray(mesh.map0, dtype=np.int64),
            e1=np.ascontiguousarray(e1, dtype=np.int32), q1=np.ascontiguousarray(q1, dtype=np.float64),
            f2=np.ascontiguousarray(f2, dtype=np.int32), q2=np.ascontiguousarray(q2, dtype=np.float64),
            p0=np.ascontiguousarray(p0, dtype=np.float64),
            gl_x=np.ascontiguousarray(gl[0], dtype=np.float64), gl_w=np.ascontiguousarray(gl[1], dtype=np.float64),
        )
        a = self.arrs
        self.s = OMesh(mesh.nt, ptr(a["aff"]), ptr(a["grad"]), ptr(a["nbr"]),
                       len(q1), len(q2), len(p0), ptr(a["map1"]), ptr(a["map2"]), ptr(a["map0"]),
                       ptr(a["e1"]), ptr(a["q1"]), ptr(a["f2"]), ptr(a["q2"]), ptr(a["p0"]),
                       len(gl[0]), ptr(a["gl_x"]), ptr(a["gl_w"]))

    @property
    def ref(self):
        return C.c_void_p(C.addressof(self.s))
