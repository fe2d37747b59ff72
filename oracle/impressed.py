"""Oracle: projection of an impressed magnetic flux density onto the order-k face
space, without and with the constraint of Gauss's magnetic law (Sec. III-C,
eq. (conB)).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Non-constrained: [*mu^-1] b = f with f_i = <W2_i, mu^-1 B>.
Constrained:     [[*mu^-1, [div]^T], [[div], 0]] [b; lambda] = [f; 0], with the
higher-order discrete divergence [div] = [*3]^-1 [div~], [*3]_ij = <W3_i, W3_j>
and [div~]_ij = <W3_i, div W2_j>, all integrated tet by tet.

Reading of the volume functions (the Appendix formula is garbled): W3 = Q3 w,
with w = 6 grad l_1 . (grad l_2 x grad l_3) = +-1/V the oriented Whitney 3-form
of the tet (vertices in ascending global order, as for every other form) and
Q3 the product of shifted Silvester polynomials of argument (k+3) lambda over
all four vertices (|alpha| = k+3, every alpha_m >= 1): k = 1 gives w itself,
k = 2 the four functions (5 l_s - 1) w, which span the polynomials of degree
k-1 times w, the space div W2 lies in.
"""
import itertools

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from . import basis, core


def w3_q(k):
    """Q3 of the order-k volume functions as [c, c0, c1, c2, c3] (Q = c + sum c_m l_m)."""
    n = k + 3
    alphas = [al for al in itertools.product(range(1, n + 1), repeat=4) if sum(al) == n]
    out = []
    for al in sorted(alphas, reverse=True):
        Q = 1
        for m in range(4):
            Q *= basis.Rhat(al[m], n, basis.LS[m])
        out.append(basis._lin_coeffs(Q))
    return np.array(out)


def tet_rule(n):
    """Collapsed Gauss-Legendre rule on a tet: barycentric points (P,4), weights summing to 1."""
    x, w = np.polynomial.legendre.leggauss(n)
    x, w = 0.5 * (x + 1), 0.5 * w
    pts, wts = [], []
    for (u, wu), (v, wv), (t, wt) in itertools.product(zip(x, w), zip(x, w), zip(x, w)):
        X, Y, Z = u, v * (1 - u), t * (1 - u) * (1 - v)
        pts.append([1 - X - Y - Z, X, Y, Z])
        wts.append(6.0 * wu * wv * wt * (1 - u) ** 2 * (1 - v))
    return np.array(pts), np.array(wts)


def _qval(q, lam):
    return q[0] + lam @ q[1:]


def w2_values(m, t, lam):
    """W2_l and div W2_l of tet t at barycentric points lam (P,4): (n2,P,3), (n2,P).
    div(Q W~) = grad Q . W~ + Q div W~, W~_abc = 2(l_a gb x gc + l_b gc x ga + l_c ga x gb),
    div W~_abc = 6 ga . (gb x gc)."""
    _, _, f2, q2, _ = basis.c_tables(m.order)
    g = m.grad[t]
    W, D = [], []
    for (a, b, c), q in zip(f2, q2):
        Wt = 2.0 * (lam[:, a, None] * np.cross(g[b], g[c]) + lam[:, b, None] * np.cross(g[c], g[a])
                    + lam[:, c, None] * np.cross(g[a], g[b]))
        Q = _qval(q, lam)
        gradQ = q[1:] @ g
        div_t = 6.0 * g[a] @ np.cross(g[b], g[c])
        W.append(Q[:, None] * Wt)
        D.append(Wt @ gradQ + Q * div_t)
    return np.array(W), np.array(D)


def local_div(m, t, rule=None):
    """[div]_T = [*3]_T^-1 [div~]_T of tet t by quadrature (n3 x n2)."""
    lam, wq = rule if rule is not None else tet_rule(3)
    q3 = w3_q(m.order)
    g = m.grad[t]
    w = 6.0 * g[1] @ np.cross(g[2], g[3])
    W3 = np.array([_qval(q, lam) for q in q3]) * w
    _, D2 = w2_values(m, t, lam)
    wv = wq * m.vol[t]
    star3 = (W3 * wv) @ W3.T
    divt = (W3 * wv) @ D2.T
    return np.linalg.solve(star3, divt), star3


def div_matrix(m):
    """Global [div] (rows: W3 DoFs, n3 per tet, tet-major; columns: W2 DoFs) and block [*3]."""
    rule = tet_rule(3)
    n3 = len(w3_q(m.order))
    rows, cols, vals, s_r, s_c, s_v = [], [], [], [], [], []
    for t in range(m.nt):
        Dt, S3 = local_div(m, t, rule)
        for i in range(n3):
            for j in range(Dt.shape[1]):
                rows.append(t * n3 + i)
                cols.append(m.map2[t, j])
                vals.append(Dt[i, j])
            for j in range(n3):
                s_r.append(t * n3 + i)
                s_c.append(t * n3 + j)
                s_v.append(S3[i, j])
    N3 = m.nt * n3
    return (sps.csr_matrix((vals, (rows, cols)), shape=(N3, m.n2)),
            sps.csr_matrix((s_v, (s_r, s_c)), shape=(N3, N3)))


def rhs(m, field, n=6):
    """f_i = <W2_i, mu0^-1 B> by an n^3-point collapsed Gauss rule per tet; field(points (P,3)) -> (P,3)."""
    lam, wq = tet_rule(n)
    f = np.zeros(m.n2)
    for t in range(m.nt):
        pts = lam @ m.xyz[m.tets[t]]
        B = field(pts)
        W, _ = w2_values(m, t, lam)
        contrib = np.einsum("lpk,pk,p->l", W, B, wq * m.vol[t]) / core.MU0
        np.add.at(f, m.map2[t], contrib)
    return f


def project(m, ops, field, constrained):
    """Coefficients b of the impressed field in the face space (non-constrained or constrained)."""
    f = rhs(m, field)
    if not constrained:
        return spla.spsolve(ops.star_nu.tocsc(), f)
    D, _ = div_matrix(m)
    # the same system with both sides of the first row times mu0 and the constraint rows scaled
    # to the mass block's size (b is unchanged; only lambda scales), which a direct solve needs
    M2 = core.MU0 * ops.star_nu
    s = abs(M2).max() / abs(D).max()
    K = sps.bmat([[M2, s * D.T], [s * D, None]]).tocsc()
    x = spla.spsolve(K, np.concatenate([core.MU0 * f, np.zeros(D.shape[0])]))
    return x[:m.n2]


def errors(m, b, field, n=6):
    """Relative L2 error of the reconstructed field, and the L2 norm of its divergence."""
    lam, wq = tet_rule(n)
    num = den = dsq = 0.0
    for t in range(m.nt):
        pts = lam @ m.xyz[m.tets[t]]
        B = field(pts)
        W, D2 = w2_values(m, t, lam)
        Bt = np.einsum("l,lpk->pk", b[m.map2[t]], W)
        dv = b[m.map2[t]] @ D2
        wv = wq * m.vol[t]
        num += np.sum(wv * np.sum((Bt - B) ** 2, axis=1))
        den += np.sum(wv * np.sum(B ** 2, axis=1))
        dsq += np.sum(wv * dv ** 2)
    return np.sqrt(num / den), np.sqrt(dsq)


def block_mesh(n, size, order):
    """Kuhn-split box [0, size_x] x [0, size_y] x [0, size_z] with n^3 hexes."""
    from . import mesh as omesh
    xyz, tets = omesh.kuhn_cube(n)
    return omesh.build(xyz * np.asarray(size, dtype=np.float64), tets, order)
