"""Oracle: higher-order interpolatory Whitney bases, exact local exterior
derivatives and exact reference mass tensors.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

The bases follow the paper's Appendix (Silvester polynomials; nodal, edge and
face functions built as a Silvester product times the lowest-order Whitney
form).  Readings taken where the printed text is garbled or silent:
  * the Silvester argument is n*lambda with a form-specific n: n = k for W0,
    n = k+1 for W1, n = k+2 for W2 (the printed k*lambda makes the order-2 edge
    set rank deficient);
  * the lowest-order face form is 2(l_a grad l_b x grad l_c + cyclic), which has
    unit flux through its face (the printed three-term formula is not a face
    function);
  * dependent candidates are dropped by a fixed rule: on face (a<b<c) the edge
    candidate on (b,c) with alpha_a = 1; among the interior face candidates the
    one of face (1,2,3);
  * in W0 the distinguished vertex s is the one with the largest multi-index
    entry (ties: smallest local index).
Everything here is exact (sympy rationals) on the reference tet
(0,0,0),(1,0,0),(0,1,0),(0,0,1), where l0 = 1-x-y-z, l1 = x, l2 = y, l3 = z.
"""
from fractions import Fraction
from functools import lru_cache
from math import factorial
import itertools

import numpy as np
import sympy as sp

from .mesh import LOCAL_EDGES, LOCAL_FACES

X, Y, Z = sp.symbols("x y z")
LS = sp.symbols("L0 L1 L2 L3")  # formal barycentric symbols
LAM_REF = [1 - X - Y - Z, X, Y, Z]
GRAD_REF = [sp.Matrix([-1, -1, -1]), sp.Matrix([1, 0, 0]), sp.Matrix([0, 1, 0]), sp.Matrix([0, 0, 1])]


def R(i, n, lam):
    """Silvester polynomial R_i(n, lam) = (1/i!) prod_{m=0}^{i-1} (n lam - m), R_0 = 1."""
    out = sp.Integer(1)
    for mm in range(i):
        out *= (n * lam - mm)
    return sp.expand(out / factorial(i))


def Rhat(i, n, lam):
    """Shifted Silvester polynomial (1/(i-1)!) prod_{m=1}^{i-1} (n lam - m), Rhat_1 = 1."""
    assert i >= 1
    out = sp.Integer(1)
    for mm in range(1, i):
        out *= (n * lam - mm)
    return sp.expand(out / factorial(i - 1))


# ---------------------------------------------------------------- definitions
def w0_defs(k):
    """Nodal functions: list of (alpha, scalar expression in formal L)."""
    if k == 1:
        alphas = [tuple(1 if m == v else 0 for m in range(4)) for v in range(4)]
    elif k == 2:
        alphas = [tuple(2 if m == v else 0 for m in range(4)) for v in range(4)]
        alphas += [tuple(1 if m in e else 0 for m in range(4)) for e in LOCAL_EDGES]
    else:
        raise ValueError(k)
    out = []
    for al in alphas:
        s = max(range(4), key=lambda m: (al[m], -m))
        f = LS[s] * Rhat(al[s], k, LS[s])
        for m in range(4):
            if m != s:
                f *= R(al[m], k, LS[m])
        out.append((al, sp.expand(f)))
    return out


def w1_defs(k):
    """Edge functions: list of (edge (a,b), alpha, Q in formal L); W = Q (l_a grad l_b - l_b grad l_a)."""
    n = k + 1
    cands = []
    if k == 1:
        for (a, b) in LOCAL_EDGES:
            cands.append(((a, b), tuple(1 if m in (a, b) else 0 for m in range(4))))
    elif k == 2:
        for (a, b) in LOCAL_EDGES:
            for hi in (a, b):
                al = [0] * 4
                al[a] = al[b] = 1
                al[hi] = 2
                cands.append(((a, b), tuple(al)))
        for (a, b, c) in LOCAL_FACES:
            cands.append(((a, b), tuple(1 if m in (a, b, c) else 0 for m in range(4))))
            cands.append(((a, c), tuple(1 if m in (a, b, c) else 0 for m in range(4))))
    else:
        raise ValueError(k)
    out = []
    for (a, b), al in cands:
        Q = Rhat(al[a], n, LS[a]) * Rhat(al[b], n, LS[b])
        for m in range(4):
            if m not in (a, b):
                Q *= R(al[m], n, LS[m])
        out.append(((a, b), al, sp.expand(Q)))
    return out


def w2_defs(k):
    """Face functions: list of (face (a,b,c), alpha, Q); W = Q * 2(l_a gb x gc + l_b gc x ga + l_c ga x gb)."""
    n = k + 2
    cands = []
    if k == 1:
        for f in LOCAL_FACES:
            cands.append((f, tuple(1 if m in f else 0 for m in range(4))))
    elif k == 2:
        for f in LOCAL_FACES:
            for x in f:
                al = [1 if m in f else 0 for m in range(4)]
                al[x] = 2
                cands.append((f, tuple(al)))
        for f in LOCAL_FACES[:3]:
            cands.append((f, (1, 1, 1, 1)))
    else:
        raise ValueError(k)
    out = []
    for f, al in cands:
        Q = sp.Integer(1)
        for m in range(4):
            Q *= Rhat(al[m], n, LS[m]) if m in f else R(al[m], n, LS[m])
        out.append((f, al, sp.expand(Q)))
    return out


# ------------------------------------------------ reference-tet vector fields
def _ref(expr):
    return sp.expand(expr.subs(dict(zip(LS, LAM_REF)), simultaneous=True))


def w0_ref(k):
    return [_ref(f) for _, f in w0_defs(k)]


def w1_ref(k):
    out = []
    for (a, b), _, Q in w1_defs(k):
        W = LAM_REF[a] * GRAD_REF[b] - LAM_REF[b] * GRAD_REF[a]
        out.append((_ref(Q) * W).applyfunc(sp.expand))
    return out


def w2_ref(k):
    out = []
    for (a, b, c), _, Q in w2_defs(k):
        g = GRAD_REF
        W = 2 * (LAM_REF[a] * g[b].cross(g[c]) + LAM_REF[b] * g[c].cross(g[a]) + LAM_REF[c] * g[a].cross(g[b]))
        out.append((_ref(Q) * W).applyfunc(sp.expand))
    return out


def _grad(f):
    return sp.Matrix([sp.diff(f, v) for v in (X, Y, Z)])


def _curl(F):
    return sp.Matrix([
        sp.diff(F[2], Y) - sp.diff(F[1], Z),
        sp.diff(F[0], Z) - sp.diff(F[2], X),
        sp.diff(F[1], X) - sp.diff(F[0], Y),
    ])


def _coeff_rows(vecs):
    """Coefficient matrix (rows: monomial x component, cols: functions)."""
    monos = set()
    polys = []
    for v in vecs:
        pv = [sp.Poly(c, X, Y, Z) for c in v]
        polys.append(pv)
        for p in pv:
            monos.update(p.as_dict().keys())
    monos = sorted(monos)
    M = sp.zeros(3 * len(monos), len(vecs))
    for j, pv in enumerate(polys):
        for comp in range(3):
            d = pv[comp].as_dict()
            for r, mo in enumerate(monos):
                M[3 * r + comp, j] = d.get(mo, 0)
    return M, monos


def _express(targets, basis):
    """Exact coefficients C with targets[j] = sum_i C[i,j] basis[i]."""
    B, monos = _coeff_rows(basis)
    T, monos_t = _coeff_rows(targets)
    # align monomial sets
    allm = sorted(set(monos) | set(monos_t))

    def realign(M, ms):
        out = sp.zeros(3 * len(allm), M.shape[1])
        for r, mo in enumerate(ms):
            rr = allm.index(mo)
            for comp in range(3):
                out[3 * rr + comp, :] = M[3 * r + comp, :]
        return out

    B = realign(B, monos)
    T = realign(T, monos_t)
    # least squares in exact arithmetic: (B^T B) C = B^T T, then verify B C = T
    BtB = B.T * B
    C = BtB.LUsolve(B.T * T)
    assert (B * C - T).applyfunc(sp.simplify) == sp.zeros(*T.shape), "not in the span"
    return C


@lru_cache(maxsize=None)
def local_G(k):
    """Exact local gradient matrix: grad W0_j = sum_i G[i,j] W1_i  (n1 x n0), Fractions."""
    grads = [_grad(f) for f in w0_ref(k)]
    C = _express(grads, w1_ref(k))
    return [[Fraction(int(sp.fraction(C[i, j])[0]), int(sp.fraction(C[i, j])[1])) for j in range(C.shape[1])]
            for i in range(C.shape[0])]


@lru_cache(maxsize=None)
def local_K(k):
    """Exact local curl matrix: curl W1_j = sum_l K[l,j] W2_l  (n2 x n1), Fractions."""
    curls = [_curl(F) for F in w1_ref(k)]
    C = _express(curls, w2_ref(k))
    return [[Fraction(int(sp.fraction(C[i, j])[0]), int(sp.fraction(C[i, j])[1])) for j in range(C.shape[1])]
            for i in range(C.shape[0])]


def basis_rank(k):
    """Ranks (W0, W1, W2) of the function sets on the reference tet."""
    r0 = sp.Matrix([[sp.Poly(f, X, Y, Z).as_dict().get(mo, 0) for f in w0_ref(k)]
                    for mo in sorted({m for f in w0_ref(k) for m in sp.Poly(f, X, Y, Z).as_dict()})]).rank()
    r1 = _coeff_rows(w1_ref(k))[0].rank()
    r2 = _coeff_rows(w2_ref(k))[0].rank()
    return r0, r1, r2


# ------------------------------------------------------ exact mass tensors
def monomial_integral(alpha):
    """int_T l^alpha dV / (6 V) = alpha! / (|alpha| + 3)!  (textbook formula)."""
    num = 1
    for a in alpha:
        num *= factorial(a)
    return Fraction(num, factorial(sum(alpha) + 3))


def _poly_L(expr):
    """Polynomial in the formal L symbols -> {exponent tuple: Fraction}."""
    p = sp.Poly(sp.expand(expr), *LS)
    return {mo: Fraction(int(sp.fraction(c)[0]), int(sp.fraction(c)[1])) for mo, c in p.as_dict().items()}


def _pmul(p, q):
    out = {}
    for a, ca in p.items():
        for b, cb in q.items():
            m = tuple(x + y for x, y in zip(a, b))
            out[m] = out.get(m, 0) + ca * cb
    return out


def _pint(p):
    return sum((c * monomial_integral(m) for m, c in p.items()), Fraction(0))


def w1_grad_coeffs(k):
    """W1_i = sum_m phi_i^m(l) grad l_m ; returns list over i of 4 polynomials (dicts)."""
    out = []
    for (a, b), _, Q in w1_defs(k):
        phi = [{} for _ in range(4)]
        phi[b] = _poly_L(Q * LS[a])
        phi[a] = _poly_L(-Q * LS[b])
        out.append(phi)
    return out


PAIRS = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def w2_pair_coeffs(k):
    """W2_l = sum_{p=(m<n)} psi_l^p(l) grad l_m x grad l_n ; list over l of 6 polynomials."""
    out = []
    for (a, b, c), _, Q in w2_defs(k):
        psi = {p: sp.Integer(0) for p in PAIRS}

        def add(lam_i, m, n, sgn):
            if m < n:
                psi[(m, n)] += sgn * 2 * Q * LS[lam_i]
            else:
                psi[(n, m)] -= sgn * 2 * Q * LS[lam_i]

        add(a, b, c, 1)
        add(b, c, a, 1)
        add(c, a, b, 1)
        out.append([_poly_L(psi[p]) if psi[p] != 0 else {} for p in PAIRS])
    return out


@lru_cache(maxsize=None)
def mass1_tensor(k):
    """C1[i,j,m,n] with int_T W1_i . W1_j = 6V sum_{mn} C1[i,j,m,n] (grad l_m . grad l_n)."""
    phis = w1_grad_coeffs(k)
    n1 = len(phis)
    C = np.zeros((n1, n1, 4, 4))
    for i in range(n1):
        for j in range(n1):
            for m in range(4):
                for n in range(4):
                    if phis[i][m] and phis[j][n]:
                        C[i, j, m, n] = float(_pint(_pmul(phis[i][m], phis[j][n])))
    return C


def face_monomial_integral(alpha, o):
    """int_F l^alpha dS / (2 A) over the face F opposite local vertex o, where l_o = 0:
    alpha! / (|alpha| + 2)! over the three face coordinates (textbook formula), 0 if alpha_o > 0."""
    if alpha[o] > 0:
        return Fraction(0)
    num = 1
    for a in alpha:
        num *= factorial(a)
    return Fraction(num, factorial(sum(alpha) + 2))


@lru_cache(maxsize=None)
def face_mass1_tensor(k):
    """F1[o,i,j,m,n] with int_F W1_i . P W1_j dS = 2 A sum_{mn} F1[o,i,j,m,n] (grad l_m . P grad l_n)
    over the face F opposite local vertex o, for any 3x3 matrix P (the tangential projector
    I - n n^T gives the surface impedance matrix)."""
    phis = w1_grad_coeffs(k)
    n1 = len(phis)
    C = np.zeros((4, n1, n1, 4, 4))
    for o in range(4):
        for i in range(n1):
            for j in range(n1):
                for m in range(4):
                    for n in range(4):
                        if phis[i][m] and phis[j][n]:
                            p = _pmul(phis[i][m], phis[j][n])
                            C[o, i, j, m, n] = float(sum((c * face_monomial_integral(mo, o) for mo, c in p.items()),
                                                         Fraction(0)))
    return C


@lru_cache(maxsize=None)
def mass2_tensor(k):
    """C2[l,l',p,q] with int_T W2_l . W2_l' = 6V sum_{pq} C2 * (g_p . g_q), g_p = grad l_m x grad l_n."""
    psis = w2_pair_coeffs(k)
    n2 = len(psis)
    C = np.zeros((n2, n2, 6, 6))
    for i in range(n2):
        for j in range(n2):
            for p in range(6):
                for q in range(6):
                    if psis[i][p] and psis[j][q]:
                        C[i, j, p, q] = float(_pint(_pmul(psis[i][p], psis[j][q])))
    return C


# ------------------------------------------------ numeric tables for the C loop
MONO15 = [()] + [(m,) for m in range(4)] + [(m, n) for m in range(4) for n in range(m, 4)]


def _lin_coeffs(expr):
    """Degree<=1 polynomial in L -> [c, c0, c1, c2, c3]."""
    p = _poly_L(expr)
    out = [0.0] * 5
    for mo, c in p.items():
        deg = sum(mo)
        if deg == 0:
            out[0] = float(c)
        elif deg == 1:
            out[1 + mo.index(1)] = float(c)
        else:
            raise ValueError("Q of degree > 1")
    return out


def c_tables(k):
    """Arrays consumed by the C particle loop."""
    d1 = w1_defs(k)
    d2 = w2_defs(k)
    d0 = w0_defs(k)
    e1 = np.array([ab for ab, _, _ in d1], dtype=np.int32)
    q1 = np.array([_lin_coeffs(Q) for _, _, Q in d1])
    f2 = np.array([f for f, _, _ in d2], dtype=np.int32)
    q2 = np.array([_lin_coeffs(Q) for _, _, Q in d2])
    p0 = np.zeros((len(d0), 15))
    for j, (_, f) in enumerate(d0):
        for mo, c in _poly_L(f).items():
            key = tuple(sorted(itertools.chain.from_iterable([m] * e for m, e in enumerate(mo))))
            p0[j, MONO15.index(key)] += float(c)
    return e1, q1, f2, q2, p0


def gauss_legendre01(n):
    """Gauss-Legendre nodes and weights on [0, 1] (numpy's leggauss mapped)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w
