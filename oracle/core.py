"""Oracle: global operators, implicit field update and the whole PIC step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Field discretisation (Sec. III-A): E in the order-k edge space, B in the
order-k face space, on the primal mesh; Hodge matrices
  [*eps]_ij = eps0 <W1_i, W1_j>,   [*nu]_ij = (1/mu0) <W2_i, W2_j>,
and the curl of an edge function expressed in the face space,
  curl W1_j = sum_l K_lj W2_l   (K is topological: fixed rationals per tet).
Readings of the semi-discrete system and of the Newmark-beta scheme
(gamma = 1/2, beta = 1/4, Sec. III-B), taken where the printed equations are
garbled:
  Faraday holds strongly:            d b / dt = -K e
  Ampere is tested with W1:          *eps de/dt = K^T *nu b - d g / dt
where g_i = <W1_i, int_0^t J> is the time-integrated current moment.  The
average-acceleration scheme is the trapezoidal rule; eliminating b^{n+1}:
  A (e^{n+1} - e^n) = dt K^T *nu (b^n - dt/2 K e^n) - (g^{n+1} - g^n),
  A = *eps + dt^2/4 K^T *nu K,
  b^{n+1} = b^n - dt/2 K (e^n + e^{n+1}).
Only the W1 DoFs off the PEC walls are unknowns (n x E = 0 on the walls); with
absorbing walls every W1 DoF is, and the surface impedance matrix enters
Ampere's law (see OracleRun).
Gauss's law: with G the local gradient matrix (grad W0 = sum G W1) and K G = 0,
G^T (*eps e + g) is invariant, and the exact path integral gives
G^T (g^{n} - g^0) = rho~^n - rho~^0 where rho~_j = q w sum_p W0_j(r_p).
"""
import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from . import basis, mesh as omesh, cloop

C_LIGHT = 299792458.0
MU0 = 1.25663706212e-6
EPS0 = 1.0 / (MU0 * C_LIGHT ** 2)
Q_E = 1.602176634e-19
M_E = 9.1093837015e-31


class Operators:
    pass


def assemble(m):
    """Global sparse operators of mesh m (natural DoF numbering)."""
    k = m.order
    ops = Operators()
    C1 = basis.mass1_tensor(k)
    C2 = basis.mass2_tensor(k)
    g = np.einsum("tmk,tnk->tmn", m.grad, m.grad)
    six_v = 6.0 * m.vol
    M1 = six_v[:, None, None] * np.einsum("ijmn,tmn->tij", C1, g)
    gp = np.stack([np.cross(m.grad[:, a], m.grad[:, b]) for a, b in basis.PAIRS], axis=1)  # (nt,6,3)
    G2 = np.einsum("tpk,tqk->tpq", gp, gp)
    M2 = six_v[:, None, None] * np.einsum("ijpq,tpq->tij", C2, G2)
    ops.M1_el, ops.M2_el = M1, M2

    def scatter(el, rmap, cmap, n_r, n_c):
        nt, a, b = el.shape
        rows = np.repeat(rmap[:, :, None], b, axis=2).ravel()
        cols = np.repeat(cmap[:, None, :], a, axis=1).ravel()
        return sps.csr_matrix((el.ravel(), (rows, cols)), shape=(n_r, n_c))

    ops.star_eps = EPS0 * scatter(M1, m.map1, m.map1, m.n1, m.n1)
    ops.star_nu = (1.0 / MU0) * scatter(M2, m.map2, m.map2, m.n2, m.n2)

    # topological operators by assignment from the exact local matrices
    Kloc = np.array(basis.local_K(k), dtype=np.float64)
    Gloc = np.array(basis.local_G(k), dtype=np.float64)
    ops.K = _assign(Kloc, m.map2, m.map1, m.n2, m.n1)
    ops.G = _assign(Gloc, m.map1, m.map0, m.n1, m.n0)
    ops.Kloc, ops.Gloc = Kloc, Gloc
    ops.int1 = np.nonzero(m.int1)[0]
    ops.int0 = np.nonzero(m.int0)[0]
    return ops


def surface_impedance(m, Y):
    """[*I]_ij = Y int_{walls} (n x W1_i) . (n x W1_j) dS (Sec. III-A, surface impedance matrix),
    natural numbering, n1 x n1.  (n x u) . (n x v) = u . (I - n n^T) v; W1 = sum_m phi^m grad l_m
    with the face integrals of phi_i^m phi_j^n exact (face_mass1_tensor).  Y is the wall
    admittance: 1 / eta0 for the first-order absorbing condition."""
    k = m.order
    F1 = basis.face_mass1_tensor(k)
    rows, cols, vals = [], [], []
    n1l = m.map1.shape[1]
    for t in range(m.nt):
        for lf in range(4):
            if not m.bface[m.tet_face[t, lf]]:
                continue
            o = 3 - lf  # the face opposite local vertex o
            a, b, c = m.tets[t, list(omesh.LOCAL_FACES[lf])]
            xa, xb, xc = m.xyz[a], m.xyz[b], m.xyz[c]
            nrm = np.cross(xb - xa, xc - xa)
            area = 0.5 * np.linalg.norm(nrm)
            nu = nrm / np.linalg.norm(nrm)
            P = np.eye(3) - np.outer(nu, nu)
            gPg = m.grad[t] @ P @ m.grad[t].T  # (4,4): grad l_m . P grad l_n
            el = Y * 2.0 * area * np.einsum("ijmn,mn->ij", F1[o], gPg)
            rows.append(np.repeat(m.map1[t], n1l))
            cols.append(np.tile(m.map1[t], n1l))
            vals.append(el.ravel())
    if not rows:
        return sps.csr_matrix((m.n1, m.n1))
    return sps.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m.n1, m.n1))


def _assign(loc, rmap, cmap, n_r, n_c):
    """Global matrix whose (rmap[t,i], cmap[t,j]) entry is loc[i,j] for every tet t;
    every tet that touches an entry must give the same value."""
    nt = rmap.shape[0]
    rows = np.repeat(rmap[:, :, None], cmap.shape[1], axis=2).ravel()
    cols = np.repeat(cmap[:, None, :], rmap.shape[1], axis=1).ravel()
    vals = np.broadcast_to(loc, (nt,) + loc.shape).ravel()
    key = rows * n_c + cols
    order = np.argsort(key, kind="stable")
    key, vals, rows, cols = key[order], vals[order], rows[order], cols[order]
    first = np.ones(len(key), dtype=bool)
    first[1:] = key[1:] != key[:-1]
    grp = np.cumsum(first) - 1
    ref = vals[first][grp]
    assert np.all(ref == vals), "local matrices disagree between tets"
    nz = first & (vals != 0)
    return sps.csr_matrix((vals[nz], (rows[nz], cols[nz])), shape=(n_r, n_c))


def cfl_dt(m, ops):
    """Explicit (leapfrog) limit 2/sqrt(lmax) with lmax bounded per element:
    lmax(*eps^-1 K^T *nu K) <= max_T lmax(M1_T^-1 S_T), S_T = Kloc^T M2_T Kloc / mu0."""
    M1 = EPS0 * ops.M1_el
    S = np.einsum("li,tlm,mj->tij", ops.Kloc, ops.M2_el, ops.Kloc) / MU0
    Lc = np.linalg.cholesky(M1)
    Li = np.linalg.inv(Lc)
    Cm = Li @ S @ np.transpose(Li, (0, 2, 1))
    lmax = np.linalg.eigvalsh(0.5 * (Cm + np.transpose(Cm, (0, 2, 1))))[:, -1].max()
    return 2.0 / np.sqrt(lmax)


class OracleRun:
    """Whole PIC loop in FP64: C particle loop + scipy sparse direct field solve.

    gamma, beta: parameters of the Newmark-beta scheme (Sec. III-B).  At 1/2, 1/4
    the step is the two-level trapezoidal form above (unless three_level is set);
    otherwise, or with three_level, it is the three-level weighted-residual form
    of the scheme for M dX/dt + S X = F (field_step_newmark)."""

    def __init__(self, m, dt, ops=None, particles_only=False, gamma=0.5, beta=0.25, three_level=False,
                 absorb=False, pusher="ab4", field_bc="pec"):
        """particles_only: skip the field operators (particle steps with given fields).
        absorb: a particle that reaches a wall deposits its current up to the wall and leaves the
        run (tet -1); otherwise walls reflect.
        pusher: "ab4" (the paper's fourth-order Adams-Bashforth push, quartic path) or "boris"
        (Boris leapfrog, straight path; the stored velocity is then v^{n-1/2}).
        field_bc: "pec" (n x E = 0 on the walls: the wall W1 DoFs are not unknowns) or
        "absorbing": the impedance condition of Sec. II with Psi_I = 0 and the free-space wall
        admittance Y = 1/eta0 (the first-order absorbing condition); every W1 DoF is an unknown and
        the surface impedance matrix *I enters Ampere's law as  *eps de/dt + *I e = K^T *nu b - dg/dt
        (Sec. III-A), trapezoidal in time like the rest:
          (A + dt/2 *I) (e^{n+1} - e^n) = dt K^T *nu (b^n - dt/2 K e^n) - dt *I e^n - (g^{n+1} - g^n)."""
        self.m = m
        self.absorb = 1 if absorb else 0
        self.pusher = {"ab4": 0, "boris": 1}[pusher]
        self.k = m.order
        self.dt = dt
        self.lu = None
        self.gamma, self.beta = gamma, beta
        self.three_level = three_level or (gamma, beta) != (0.5, 0.25)
        self.lu3 = None
        self.prev = None  # (b^{n-1}, e^{n-1}, g^{n-1}) of the three-level scheme
        self.field_bc = field_bc
        if field_bc not in ("pec", "absorbing"):
            raise ValueError("field_bc must be 'pec' or 'absorbing'")
        if field_bc == "absorbing" and self.three_level:
            raise NotImplementedError("absorbing walls with the two-level trapezoidal scheme only")
        if not particles_only:
            self.ops = ops if ops is not None else assemble(m)
            o = self.ops
            # the unknown W1 DoFs: off the walls (PEC), or all of them (absorbing)
            self.i1 = o.int1 if field_bc == "pec" else np.arange(m.n1)
            i1 = self.i1
            self.Ki = o.K[:, i1].tocsr()
            self.A = (o.star_eps[i1][:, i1] + (dt * dt / 4.0) * (self.Ki.T @ o.star_nu @ self.Ki)).tocsc()
            self.ZI = None
            if field_bc == "absorbing":
                self.ZI = surface_impedance(m, np.sqrt(EPS0 / MU0))
                self.A = (self.A + (dt / 2.0) * self.ZI).tocsc()
        self.tables = basis.c_tables(self.k)
        self.gl = basis.gauss_legendre01(2 * self.k + 2)
        self.cm = cloop.CMesh(m, self.tables, self.gl)
        self.e = np.zeros(m.n1)
        self.b = np.zeros(m.n2)
        self.g = np.zeros(m.n1)  # accumulated current moments
        self.counters = np.zeros(3, dtype=np.int64)  # crossings, reflections, absorbed
        self.step_count = 0

    # ------------------------------------------------------------ particles
    def load(self, pos, vel, q, mass, w, tet=None):
        self.pos = np.array(pos, dtype=np.float64).reshape(-1, 3).copy()
        self.vel = np.array(vel, dtype=np.float64).reshape(-1, 3).copy()
        n = len(self.pos)
        self.tet = (omesh.locate_kuhn(self.m, self.pos) if tet is None else np.asarray(tet, dtype=np.int64)).copy()
        self.vh = np.zeros((n, 3, 3))
        self.ah = np.zeros((n, 3, 3))
        self.q, self.mass, self.w = q, mass, w
        L = cloop.lib()
        L.oracle_startup(self.cm.ref, cloop.ptr(self.e), cloop.ptr(self.b), n, cloop.ptr(self.pos),
                         cloop.ptr(self.vel), cloop.ptr(self.vh), cloop.ptr(self.ah), cloop.ptr(self.tet),
                         q, mass, self.dt)
        self.rho0 = self.rho()

    def inject(self, pos, vel):
        """Append particles of the loaded species, started like loaded ones (the AB4 history from
        the current fields).  Their charge enters here, not through a current, so it joins the
        reference rho~^0 of the Gauss check, like the charge present at load."""
        pos = np.array(pos, dtype=np.float64).reshape(-1, 3).copy()
        vel = np.array(vel, dtype=np.float64).reshape(-1, 3).copy()
        n = len(pos)
        tet = omesh.locate_kuhn(self.m, pos).copy()
        vh = np.zeros((n, 3, 3))
        ah = np.zeros((n, 3, 3))
        L = cloop.lib()
        L.oracle_startup(self.cm.ref, cloop.ptr(self.e), cloop.ptr(self.b), n, cloop.ptr(pos), cloop.ptr(vel),
                         cloop.ptr(vh), cloop.ptr(ah), cloop.ptr(tet), self.q, self.mass, self.dt)
        rho_new = np.zeros(self.m.n0)
        L.oracle_rho(self.cm.ref, n, cloop.ptr(pos), cloop.ptr(tet), self.q * self.w, cloop.ptr(rho_new))
        self.pos = np.concatenate([self.pos, pos])
        self.vel = np.concatenate([self.vel, vel])
        self.vh = np.concatenate([self.vh, vh])
        self.ah = np.concatenate([self.ah, ah])
        self.tet = np.concatenate([self.tet, tet])
        self.rho0 = self.rho0 + rho_new

    def particle_step(self, idx=None, threads=1):
        """Gather + push + track + deposit for all particles (or idx); returns dg (n1).
        threads > 1: the particles in that many contiguous chunks on as many threads, each
        chunk's deposit summed apart and the chunks added in order."""
        dg = np.zeros(self.m.n1)
        L = cloop.lib()
        n = len(self.pos)
        if threads > 1 and idx is None:
            work = np.empty(threads * self.m.n1)
            st = L.oracle_step_chunked(self.cm.ref, cloop.ptr(self.e), cloop.ptr(self.b), n, cloop.ptr(self.pos),
                                       cloop.ptr(self.vel), cloop.ptr(self.vh), cloop.ptr(self.ah),
                                       cloop.ptr(self.tet), self.q, self.mass, self.w, self.dt, cloop.ptr(dg),
                                       self.m.n1, cloop.ptr(self.counters), threads, cloop.ptr(work),
                                       self.absorb, self.pusher)
            if st != 0:
                raise RuntimeError("oracle particle step failed with status %d" % st)
            return dg
        if idx is None:
            ip, ni = None, 0
        else:
            idx = np.ascontiguousarray(idx, dtype=np.int64)
            ip, ni = cloop.ptr(idx), len(idx)
        st = L.oracle_step(self.cm.ref, cloop.ptr(self.e), cloop.ptr(self.b), n, ip, ni, cloop.ptr(self.pos),
                           cloop.ptr(self.vel), cloop.ptr(self.vh), cloop.ptr(self.ah), cloop.ptr(self.tet),
                           self.q, self.mass, self.w, self.dt, cloop.ptr(dg), cloop.ptr(self.counters), self.absorb,
                           self.pusher)
        if st != 0:
            raise RuntimeError("oracle particle step failed with status %d" % st)
        return dg

    # ---------------------------------------------------------------- fields
    def field_step(self, dg):
        o, dt, i1 = self.ops, self.dt, self.i1
        ei = self.e[i1]
        rhs = dt * (self.Ki.T @ (o.star_nu @ (self.b - 0.5 * dt * (self.Ki @ ei)))) - dg[i1]
        if self.ZI is not None:
            rhs = rhs - dt * (self.ZI @ ei)
        if self.lu is None:
            self.lu = spla.splu(self.A)
        d = self.lu.solve(rhs)
        enew = ei + d
        self.b = self.b - 0.5 * dt * (self.Ki @ (ei + enew))
        self.e = np.zeros(self.m.n1)
        self.e[i1] = enew
        self.last_solve_residual = np.linalg.norm(self.A @ d - rhs) / max(np.linalg.norm(rhs), 1e-300)

    def field_step_newmark(self, g_old):
        """Three-level Newmark-beta step (Sec. III-B, eq. (maxnmb)), read as the weighted-residual
        scheme for M dX/dt + S X = F with X = (b, e):
          M [gamma X^{n+1} + (1 - 2 gamma) X^n + (gamma - 1) X^{n-1}] / dt
            + S [beta X^{n+1} + (1/2 - 2 beta + gamma) X^n + (1/2 + beta - gamma) X^{n-1}] = F~,
        with M = diag(*nu, *eps) and S = [[0, *nu K], [-K^T *nu, 0]] (PEC walls: no impedance
        block), and the current term -dG/dt taken with the same time stencil as M:
          F~ = (0, -[gamma g^{n+1} + (1 - 2 gamma) g^n + (gamma - 1) g^{n-1}] / dt).
        The coupled system for (b^{n+1}, e^{n+1}) is solved directly.  Before the first step the
        history is at rest: X^{-1} = X^0 and g^{-1} = g^0.  self.g holds g^{n+1}; g_old is g^n."""
        o, dt, i1 = self.ops, self.dt, self.ops.int1
        gm, bt = self.gamma, self.beta
        c1, c0 = 0.5 - 2.0 * bt + gm, 0.5 + bt - gm  # weights of X^n and X^{n-1} in the S term
        Ki, nu = self.Ki, o.star_nu
        Me = o.star_eps[i1][:, i1]
        e_n, b_n = self.e[i1], self.b
        if self.prev is None:
            self.prev = (b_n.copy(), e_n.copy(), g_old.copy())
        b_m, e_m, g_m = self.prev
        if self.lu3 is None:
            top = sps.hstack([(gm / dt) * nu, bt * (nu @ Ki)])
            bot = sps.hstack([-bt * (Ki.T @ nu), (gm / dt) * Me])
            self.lu3 = spla.splu(sps.vstack([top, bot]).tocsc())
        rb = -((1 - 2 * gm) / dt) * (nu @ b_n) - c1 * (nu @ (Ki @ e_n)) \
             - ((gm - 1) / dt) * (nu @ b_m) - c0 * (nu @ (Ki @ e_m))
        gt = (gm * self.g + (1 - 2 * gm) * g_old + (gm - 1) * g_m)[i1]
        re = -((1 - 2 * gm) / dt) * (Me @ e_n) + c1 * (Ki.T @ (nu @ b_n)) \
             - ((gm - 1) / dt) * (Me @ e_m) + c0 * (Ki.T @ (nu @ b_m)) - gt / dt
        x = self.lu3.solve(np.concatenate([rb, re]))
        self.prev = (b_n.copy(), e_n.copy(), g_old.copy())
        n2 = self.m.n2
        self.b = x[:n2].copy()
        self.e = np.zeros(self.m.n1)
        self.e[i1] = x[n2:]

    def step(self, n=1):
        for _ in range(n):
            dg = self.particle_step()
            self.last_dg = dg
            g_old = self.g.copy()
            self.g += dg
            if self.three_level:
                self.field_step_newmark(g_old)
            else:
                self.field_step(dg)
            self.step_count += 1

    # ----------------------------------------------------------- diagnostics
    def rho(self):
        rho = np.zeros(self.m.n0)
        L = cloop.lib()
        L.oracle_rho(self.cm.ref, len(self.pos), cloop.ptr(self.pos), cloop.ptr(self.tet),
                     self.q * self.w, cloop.ptr(rho))
        return rho

    def gauss_residuals(self):
        """(R_G, R_C, R_S) on interior nodal DoFs, normalised by ||rho~^n - rho~^0||."""
        o = self.ops
        i0 = o.int0
        drho = (self.rho() - self.rho0)[i0]
        GtDe = (o.G.T @ (o.star_eps @ self.e))[i0]
        Gtg = (o.G.T @ self.g)[i0]
        nrm = np.linalg.norm(drho)
        if nrm == 0:
            nrm = 1.0
        RG = np.linalg.norm(GtDe + drho) / nrm
        RC = np.linalg.norm(Gtg - drho) / nrm
        RS = np.linalg.norm(GtDe + Gtg) / nrm
        return RG, RC, RS

    def energy(self):
        o = self.ops
        return 0.5 * (self.e @ (o.star_eps @ self.e) + self.b @ (o.star_nu @ self.b))

    def gather(self, pos, tet):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        tet = np.ascontiguousarray(tet, dtype=np.int64)
        E = np.zeros_like(pos)
        B = np.zeros_like(pos)
        cloop.lib().oracle_gather(self.cm.ref, cloop.ptr(self.e), cloop.ptr(self.b), len(pos), cloop.ptr(pos),
                                  cloop.ptr(tet), cloop.ptr(E), cloop.ptr(B))
        return E, B


def path_deposit(run, t0, coeffs, qw):
    """Track + deposit one given path (5x3 power-basis coefficients) from tet t0."""
    c = np.ascontiguousarray(np.array(coeffs, dtype=np.float64).reshape(5, 3))
    dg = np.zeros(run.m.n1)
    cnt = np.zeros(2, dtype=np.int64)
    tt = np.zeros(70, dtype=np.int64)
    ts = np.zeros(70)
    nt = np.zeros(1, dtype=np.int32)
    t = cloop.lib().oracle_path_deposit(run.cm.ref, t0, cloop.ptr(c), qw, cloop.ptr(dg), cloop.ptr(cnt),
                                        cloop.ptr(tt), cloop.ptr(ts), cloop.ptr(nt))
    n = int(nt[0])
    return t, dg, c, cnt, tt[:n].copy(), ts[:n].copy()


def first_negative(q, lo, hi):
    q = np.ascontiguousarray(q, dtype=np.float64)
    u = np.zeros(1)
    ok = cloop.lib().oracle_first_negative(cloop.ptr(q), lo, hi, cloop.ptr(u))
    return u[0] if ok else None
