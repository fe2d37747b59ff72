"""Comparison helpers of the GPU parity tests.

rel: relative 2-norm error (the norm-wise measure of the tolerances).
elementwise: max_i |a_i - b_i| / max_i |b_i|, so that one DoF far off cannot
hide inside a norm over many.
"""
import numpy as np


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def elementwise(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    mb = np.max(np.abs(b)) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0)) if a.size else 0.0


def close(a, b, tol):
    """Both the norm-wise and the element-wise relative error within tol; returns them."""
    r, e = rel(a, b), elementwise(a, b)
    assert r < tol and e < tol, (r, e, tol)
    return r, e
