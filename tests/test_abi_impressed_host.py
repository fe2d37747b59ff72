"""CPU checks of the impressed-field entry points: the sample points of a Kuhn
cube (no GPU needed: the points are host work) and the argument errors."""
import ctypes as C

import numpy as np
import pytest

import paper_2111_12411_amd as F
from oracle import impressed as I, mesh as omesh


@pytest.mark.parametrize("n1d", [1, 2, 4])
def test_points_are_the_collapsed_rule_in_every_tet(n1d):
    m = omesh.cube_mesh(2, 2)
    mesh = F.Mesh.cube(2, 2)
    P = n1d ** 3
    pts = mesh.impressed_points(n1d).reshape(m.nt, P, 3)
    lam, w = I.tet_rule(n1d)
    for t in range(m.nt):
        np.testing.assert_allclose(pts[t], lam @ m.xyz[m.tets[t]], rtol=0, atol=1e-15)


def test_points_reject_bad_arguments():
    L = F.lib()
    mesh = F.Mesh.cube(2, 1)
    buf = np.zeros((6 * 8 * 27, 3))
    assert L.fempic_impressed_points(mesh.h, 0, F._p(buf), len(buf)) == -1
    assert L.fempic_impressed_points(mesh.h, 9, F._p(buf), len(buf)) == -1
    assert L.fempic_impressed_points(mesh.h, 3, F._p(buf), len(buf) - 1) == -1
    assert L.fempic_impressed_points(None, 3, F._p(buf), len(buf)) == -1
    assert L.fempic_impressed_set(None, F._p(buf), len(buf), 3, 1, None, 0) == -1
