/*
 * Oracle particle loop: plain FP64, single-threaded, written for readability.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  The product path never does.
 *
 * One step of one particle, in the paper's order (Sec. III-B and the PIC cycle
 * of Sec. III):
 *   1. gather E and B at r^n through the order-k Whitney edge / face bases
 *      (Sec. III-A; bases in the Appendix);
 *   2. non-relativistic Lorentz acceleration and a 4th-order Adams-Bashforth
 *      update of v (Sec. III-B); the position follows the quartic path
 *      r(s) = r^n + dt sum_j v^{n-j} L_j(s), s in [0,1], where L_j is the
 *      integral of the cubic Lagrange basis on the nodes 0,-1,-2,-3 (this is the
 *      "fourth order Lagrange polynomial" path), so r(1) is the AB4 position;
 *   3. the path is split into segments at tet faces: the exit of a tet is the
 *      first s where a barycentric coordinate becomes negative (Bernstein
 *      bounds, de Casteljau-style subdivision, bisection, Newton polish);
 *   4. on each segment the current moments receive q w int W1_i(r(s)).r'(s) ds,
 *      integrated with Gauss-Legendre exact for the polynomial degree (the
 *      integrand has degree 4k+3, so 2k+2 points) - the exact path integral
 *      that keeps charge conserved (Sec. III-B, eq. for G and g_i);
 *   5. a boundary (PEC) face reflects the remaining path, and the velocity and
 *      the whole AB4 history are mirrored at the end of the step; or, with the
 *      absorbing rule, the path ends there: its current is deposited up to the
 *      wall and the particle leaves the run (tet = -1, position at the wall).
 *
 * The push and the current mapping are independent (Sec. III-B: the particle
 * integrator is de-linked from the field update); with pusher = 1 the step uses
 * the Boris leapfrog instead: the stored velocity is v^{n-1/2}, the Boris
 * rotation (half electric kick, rotation about B through the angle
 * 2 atan(|q| |B| dt / 2m), half kick) gives v^{n+1/2}, and the path is the
 * straight line r(s) = r^n + s dt v^{n+1/2}; tracking, deposit and walls are the
 * same, and the AB4 histories are not used.
 */
#include <math.h>
#include <string.h>
#include <stdint.h>

#define ORACLE_MAX_CROSS 64
#define ORACLE_ECROSS (-5)
#define ORACLE_ABSORBED (-100) /* track_and_deposit: the path ended at a wall */

typedef struct {
    int64_t n_tet;
    const double *aff;    /* [n_tet][4]    lambda_m(r) = aff[m] + grad[m].r */
    const double *grad;   /* [n_tet][4][3] */
    const int64_t *nbr;   /* [n_tet][4]    tet across the face opposite vertex m, -1 = wall */
    int32_t n1, n2, n0;
    const int64_t *map1;  /* [n_tet][n1] global W1 DoF */
    const int64_t *map2;  /* [n_tet][n2] global W2 DoF */
    const int64_t *map0;  /* [n_tet][n0] global W0 DoF */
    const int32_t *e1;    /* [n1][2]  edge (a,b) of each local W1 function */
    const double *q1;     /* [n1][5]  Q = c + sum_m c_m lambda_m            */
    const int32_t *f2;    /* [n2][3]  face (a,b,c) of each local W2 function */
    const double *q2;     /* [n2][5] */
    const double *p0;     /* [n0][15] W0 as a polynomial on MONO15           */
    int32_t n_gl;
    const double *gl_x;   /* Gauss-Legendre nodes on [0,1]  */
    const double *gl_w;   /* and weights */
} OMesh;

/* integral of the cubic Lagrange basis l_j on nodes 0,-1,-2,-3: L_j(s) = sum_k LC[j][k] s^k */
static const double LC[4][5] = {
    {0.0, 1.0, 11.0 / 12.0, 1.0 / 3.0, 1.0 / 24.0},
    {0.0, 0.0, -3.0 / 2.0, -5.0 / 6.0, -1.0 / 8.0},
    {0.0, 0.0, 3.0 / 4.0, 2.0 / 3.0, 1.0 / 8.0},
    {0.0, 0.0, -1.0 / 6.0, -1.0 / 6.0, -1.0 / 24.0},
};

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static void bary(const OMesh *m, int64_t t, const double *r, double *lam)
{
    for (int k = 0; k < 4; k++)
        lam[k] = m->aff[4 * t + k] + dot3(&m->grad[12 * t + 3 * k], r);
}

static double qval(const double *q, const double *lam)
{
    return q[0] + q[1] * lam[0] + q[2] * lam[1] + q[3] * lam[2] + q[4] * lam[3];
}

/* W1_i at barycentric lam in tet t (Cartesian vector) */
static void w1_eval(const OMesh *m, int64_t t, int i, const double *lam, double *out)
{
    int a = m->e1[2 * i], b = m->e1[2 * i + 1];
    const double *ga = &m->grad[12 * t + 3 * a], *gb = &m->grad[12 * t + 3 * b];
    double Q = qval(&m->q1[5 * i], lam);
    for (int c = 0; c < 3; c++) out[c] = Q * (lam[a] * gb[c] - lam[b] * ga[c]);
}

/* W2_l at lam in tet t */
static void w2_eval(const OMesh *m, int64_t t, int l, const double *lam, double *out)
{
    int a = m->f2[3 * l], b = m->f2[3 * l + 1], c = m->f2[3 * l + 2];
    const double *ga = &m->grad[12 * t + 3 * a], *gb = &m->grad[12 * t + 3 * b], *gc = &m->grad[12 * t + 3 * c];
    double bc[3], ca[3], ab[3];
    cross3(gb, gc, bc);
    cross3(gc, ga, ca);
    cross3(ga, gb, ab);
    double Q = qval(&m->q2[5 * l], lam);
    for (int k = 0; k < 3; k++) out[k] = 2.0 * Q * (lam[a] * bc[k] + lam[b] * ca[k] + lam[c] * ab[k]);
}

static double w0_eval(const OMesh *m, int j, const double *lam)
{
    const double *p = &m->p0[15 * j];
    double v = p[0] + p[1] * lam[0] + p[2] * lam[1] + p[3] * lam[2] + p[4] * lam[3];
    int idx = 5;
    for (int a = 0; a < 4; a++)
        for (int b = a; b < 4; b++) v += p[idx++] * lam[a] * lam[b];
    return v;
}

/* E(r), B(r) in tet t from global coefficient vectors e (W1) and b (W2) */
static void gather(const OMesh *m, int64_t t, const double *r, const double *e, const double *bv, double *E, double *B)
{
    double lam[4], w[3];
    bary(m, t, r, lam);
    E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = 0.0;
    for (int i = 0; i < m->n1; i++) {
        double c = e[m->map1[(int64_t)m->n1 * t + i]];
        w1_eval(m, t, i, lam, w);
        for (int k = 0; k < 3; k++) E[k] += c * w[k];
    }
    for (int l = 0; l < m->n2; l++) {
        double c = bv[m->map2[(int64_t)m->n2 * t + l]];
        w2_eval(m, t, l, lam, w);
        for (int k = 0; k < 3; k++) B[k] += c * w[k];
    }
}

/* ------------------------------------------------------------- polynomials */
static double horner4(const double *p, double s)
{
    return (((p[4] * s + p[3]) * s + p[2]) * s + p[1]) * s + p[0];
}

/* coefficients of p(u + a) */
static void taylor_shift(const double *p, double a, double *out)
{
    double c[5];
    memcpy(c, p, sizeof c);
    for (int i = 0; i < 4; i++)
        for (int j = 3; j >= i; j--) c[j] += a * c[j + 1];
    memcpy(out, c, sizeof c);
}

/* Bernstein coefficients of q on [lo, hi] (q in power basis of u) */
static void bernstein(const double *q, double lo, double hi, double *bc)
{
    static const double binom[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0}, {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};
    double d[5], h = hi - lo, hk = 1.0;
    taylor_shift(q, lo, d);
    for (int k = 0; k < 5; k++) {
        d[k] *= hk;
        hk *= h;
    }
    for (int i = 0; i < 5; i++) {
        double s = 0.0;
        for (int k = 0; k <= i; k++) s += binom[i][k] / binom[4][k] * d[k];
        bc[i] = s;
    }
}

/* smallest u in [lo, hi] with q(u) < 0; returns 1 and *u, or 0 */
static int first_negative(const double *q, double lo, double hi, int depth, double *u)
{
    double bc[5];
    bernstein(q, lo, hi, bc);
    int first = -1;
    for (int i = 0; i < 5; i++)
        if (bc[i] != 0.0) { first = i; break; }
    if (first < 0) return 0;                 /* q == 0 on the interval */
    if (bc[first] < 0.0) { *u = lo; return 1; } /* negative right away */
    int any_neg = 0, changes = 0;
    double prev = bc[first];
    for (int i = first + 1; i < 5; i++) {
        if (bc[i] < 0.0) any_neg = 1;
        if (bc[i] != 0.0) {
            if ((bc[i] < 0.0) != (prev < 0.0)) changes++;
            prev = bc[i];
        }
    }
    if (!any_neg) return 0;                  /* q >= 0: no exit here */
    if (changes == 1 && bc[4] < 0.0) {
        /* exactly one crossing in (lo, hi): bisection, then one Newton polish */
        double a = lo, b = hi;
        while (b - a > 0x1p-60) {
            double mid = 0.5 * (a + b);
            if (mid <= a || mid >= b) break;
            if (horner4(q, mid) < 0.0) b = mid; else a = mid;
        }
        double x = 0.5 * (a + b);
        double dq = (((4.0 * q[4] * x + 3.0 * q[3]) * x + 2.0 * q[2]) * x + q[1]);
        if (dq != 0.0) {
            double xn = x - horner4(q, x) / dq;
            if (xn >= a && xn <= b) x = xn;
        }
        *u = x;
        return 1;
    }
    if (depth >= 60) return 0;               /* tangency narrower than 2^-60 */
    double mid = 0.5 * (lo + hi);
    if (first_negative(q, lo, mid, depth + 1, u)) return 1;
    return first_negative(q, mid, hi, depth + 1, u);
}

/* ------------------------------------------------------------ one particle */
typedef struct {
    double qw;      /* charge times macro weight */
    double *dg;     /* global W1 accumulator (natural numbering) */
    int64_t ncross;
    int64_t nrefl;
    int absorb;     /* 1: a wall absorbs the particle instead of reflecting it */
    int64_t nabs;   /* particles absorbed */
    double s_wall;  /* path parameter where the last absorbed path met the wall */
    int64_t *trace_t; /* optional: tet of every segment */
    double *trace_s;  /* optional: end parameter of every segment */
    int ntrace;
    int pusher;     /* 0: AB4 quartic path; 1: Boris leapfrog, straight path */
} DepCtx;

static void path_eval(const double c[5][3], double s, double *r, double *dr)
{
    for (int k = 0; k < 3; k++) {
        r[k] = (((c[4][k] * s + c[3][k]) * s + c[2][k]) * s + c[1][k]) * s + c[0][k];
        if (dr) dr[k] = ((4.0 * c[4][k] * s + 3.0 * c[3][k]) * s + 2.0 * c[2][k]) * s + c[1][k];
    }
}

/* q w int_{sa}^{sb} W1_i(r(s)) . r'(s) ds for all local i of tet t, into dg */
static void deposit_segment(const OMesh *m, int64_t t, const double c[5][3], double sa, double sb, DepCtx *ctx)
{
    double h = sb - sa;
    if (!(h > 0.0)) return;
    for (int g = 0; g < m->n_gl; g++) {
        double s = sa + h * m->gl_x[g];
        double r[3], dr[3], lam[4], w[3];
        path_eval(c, s, r, dr);
        bary(m, t, r, lam);
        for (int i = 0; i < m->n1; i++) {
            w1_eval(m, t, i, lam, w);
            ctx->dg[m->map1[(int64_t)m->n1 * t + i]] += ctx->qw * h * m->gl_w[g] * dot3(w, dr);
        }
    }
}

/* reflect a point about the plane lambda_m = 0 of tet t, or a vector (is_point = 0) */
static void reflect(const OMesh *m, int64_t t, int f, double *x, int is_point)
{
    const double *g = &m->grad[12 * t + 3 * f];
    double gg = dot3(g, g);
    double s = dot3(g, x) + (is_point ? m->aff[4 * t + f] : 0.0);
    for (int k = 0; k < 3; k++) x[k] -= 2.0 * s / gg * g[k];
}

/*
 * Track the path with coefficients c (modified in place by reflections) from
 * tet t0 over s in [0,1], depositing on every segment.  Returns the final tet,
 * or a negative status.  refl_t/refl_f record the reflections in order.
 */
static int64_t track_and_deposit(const OMesh *m, int64_t t0, double c[5][3], DepCtx *ctx,
                                 int *nrefl, int64_t *refl_t, int *refl_f)
{
    int64_t t = t0;
    double s_lo = 0.0;
    int entry = -1;
    int ncross = 0;
    *nrefl = 0;
    for (;;) {
        /* barycentric coordinates along the path, as polynomials in s */
        double L[4][5];
        for (int f = 0; f < 4; f++) {
            const double *g = &m->grad[12 * t + 3 * f];
            for (int k = 0; k < 5; k++) L[f][k] = dot3(g, c[k]);
            L[f][0] += m->aff[4 * t + f];
        }
        double s_exit = 2.0;
        int f_exit = -1;
        for (int f = 0; f < 4; f++) {
            double qf[5], u;
            taylor_shift(L[f], s_lo, qf);
            if (f == entry) qf[0] = 0.0;  /* on the entry face the coordinate is zero */
            if (first_negative(qf, 0.0, 1.0 - s_lo, 0, &u)) {
                double s = s_lo + u;
                if (s < s_exit) { s_exit = s; f_exit = f; }
            }
        }
        if (f_exit < 0) {
            deposit_segment(m, t, c, s_lo, 1.0, ctx);
            if (ctx->trace_t) { ctx->trace_t[ctx->ntrace] = t; ctx->trace_s[ctx->ntrace] = 1.0; ctx->ntrace++; }
            return t;
        }
        deposit_segment(m, t, c, s_lo, s_exit, ctx);
        if (ctx->trace_t) { ctx->trace_t[ctx->ntrace] = t; ctx->trace_s[ctx->ntrace] = s_exit; ctx->ntrace++; }
        if (++ncross > ORACLE_MAX_CROSS) return ORACLE_ECROSS;
        ctx->ncross++;
        int64_t nb = m->nbr[4 * t + f_exit];
        if (nb < 0 && ctx->absorb) {
            ctx->nabs++;
            ctx->s_wall = s_exit;
            return ORACLE_ABSORBED;
        }
        if (nb >= 0) {
            int e = -1;
            for (int f = 0; f < 4; f++)
                if (m->nbr[4 * nb + f] == t) e = f;
            t = nb;
            entry = e;
        } else {
            /* PEC wall: mirror the path about the face plane */
            reflect(m, t, f_exit, c[0], 1);
            for (int k = 1; k < 5; k++) reflect(m, t, f_exit, c[k], 0);
            refl_t[*nrefl] = t;
            refl_f[*nrefl] = f_exit;
            (*nrefl)++;
            ctx->nrefl++;
            entry = f_exit;
        }
        s_lo = s_exit;
    }
}

/*
 * One time step of particle p: gather, AB4, path, track + deposit into ctx->dg,
 * then the new state.  Returns 0 or a negative status.
 */
/* Boris: v^{n+1/2} from v^{n-1/2} with the fields E, B at r^n */
static void boris(double qm, double dt, const double *E, const double *B, const double *v, double *out)
{
    double h = 0.5 * qm * dt, t[3], s[3], vm[3], vp[3], c[3];
    for (int k = 0; k < 3; k++) {
        t[k] = h * B[k];
        vm[k] = v[k] + h * E[k];
    }
    double tt = dot3(t, t);
    for (int k = 0; k < 3; k++) s[k] = 2.0 * t[k] / (1.0 + tt);
    cross3(vm, t, c);
    for (int k = 0; k < 3; k++) vp[k] = vm[k] + c[k];
    cross3(vp, s, c);
    for (int k = 0; k < 3; k++) out[k] = vm[k] + c[k] + h * E[k];
}

static int step_one(const OMesh *m, const double *e, const double *bv, int64_t p, double *pos, double *vel,
                    double *vh, double *ah, int64_t *tet, double q, double mass, double dt, DepCtx *ctx)
{
    if (tet[p] < 0) return 0; /* absorbed at a wall in an earlier step */
    double *r = &pos[3 * p], *v = &vel[3 * p], *VH = &vh[9 * p], *AH = &ah[9 * p];
    double E[3], B[3], vxB[3], a[3];
    gather(m, tet[p], r, e, bv, E, B);
    if (ctx->pusher == 1) {
        double vn[3], c[5][3] = {{0}};
        boris(q / mass, dt, E, B, v, vn);
        for (int k = 0; k < 3; k++) {
            c[0][k] = r[k];
            c[1][k] = dt * vn[k];
        }
        int nrefl;
        int64_t refl_t[ORACLE_MAX_CROSS + 1];
        int refl_f[ORACLE_MAX_CROSS + 1];
        int64_t tn = track_and_deposit(m, tet[p], c, ctx, &nrefl, refl_t, refl_f);
        if (tn == ORACLE_ABSORBED) {
            path_eval(c, ctx->s_wall, r, NULL);
            tet[p] = -1;
            return 0;
        }
        if (tn < 0) return (int)tn;
        path_eval(c, 1.0, r, NULL);
        for (int i = 0; i < nrefl; i++) reflect(m, refl_t[i], refl_f[i], vn, 0);
        memcpy(v, vn, 3 * sizeof(double));
        tet[p] = tn;
        return 0;
    }
    cross3(v, B, vxB);
    for (int k = 0; k < 3; k++) a[k] = q / mass * (E[k] + vxB[k]);
    /* path from v^n, v^{n-1}, v^{n-2}, v^{n-3} */
    const double *vj[4] = {v, &VH[0], &VH[3], &VH[6]};
    double c[5][3];
    for (int k = 0; k < 3; k++) {
        c[0][k] = r[k];
        for (int d = 1; d < 5; d++) {
            double s = 0.0;
            for (int j = 0; j < 4; j++) s += LC[j][d] * vj[j][k];
            c[d][k] = dt * s;
        }
    }
    double vnew[3];
    for (int k = 0; k < 3; k++)
        vnew[k] = v[k] + dt / 24.0 * (55.0 * a[k] - 59.0 * AH[k] + 37.0 * AH[3 + k] - 9.0 * AH[6 + k]);
    int nrefl;
    int64_t refl_t[ORACLE_MAX_CROSS + 1];
    int refl_f[ORACLE_MAX_CROSS + 1];
    int64_t tn = track_and_deposit(m, tet[p], c, ctx, &nrefl, refl_t, refl_f);
    if (tn == ORACLE_ABSORBED) {
        /* gone: its last position is the point where it met the wall */
        path_eval(c, ctx->s_wall, r, NULL);
        tet[p] = -1;
        return 0;
    }
    if (tn < 0) return (int)tn;
    double rn[3];
    path_eval(c, 1.0, rn, NULL);
    /* shift histories: v^{n}, v^{n-1}, v^{n-2};  a^{n}, a^{n-1}, a^{n-2} */
    memmove(&VH[3], &VH[0], 6 * sizeof(double));
    memcpy(&VH[0], v, 3 * sizeof(double));
    memmove(&AH[3], &AH[0], 6 * sizeof(double));
    memcpy(&AH[0], a, 3 * sizeof(double));
    memcpy(v, vnew, 3 * sizeof(double));
    for (int i = 0; i < nrefl; i++) {
        reflect(m, refl_t[i], refl_f[i], v, 0);
        for (int j = 0; j < 3; j++) {
            reflect(m, refl_t[i], refl_f[i], &VH[3 * j], 0);
            reflect(m, refl_t[i], refl_f[i], &AH[3 * j], 0);
        }
    }
    memcpy(r, rn, 3 * sizeof(double));
    tet[p] = tn;
    return 0;
}

/*
 * One time step for particles idx[0..n_idx) (or all n_p if idx == NULL).
 * State per particle: pos[3], vel[3], vh[3][3] = v^{n-1..n-3}, ah[3][3] = a^{n-1..n-3}, tet.
 * dg (length n1 global) accumulates q w int W1 . dr.  Returns 0 or a negative status.
 */
int oracle_step(const OMesh *m, const double *e, const double *bv, int64_t n_p, const int64_t *idx, int64_t n_idx,
                double *pos, double *vel, double *vh, double *ah, int64_t *tet, double q, double mass, double w,
                double dt, double *dg, int64_t *counters, int absorb, int pusher)
{
    DepCtx ctx = {q * w, dg, 0, 0, absorb, 0, 0.0, NULL, NULL, 0, pusher};
    int64_t n = idx ? n_idx : n_p;
    for (int64_t ii = 0; ii < n; ii++) {
        int st = step_one(m, e, bv, idx ? idx[ii] : ii, pos, vel, vh, ah, tet, q, mass, dt, &ctx);
        if (st) return st;
    }
    if (counters) {
        counters[0] += ctx.ncross;
        counters[1] += ctx.nrefl;
        counters[2] += ctx.nabs;
    }
    return 0;
}

/*
 * The same step for all n_p particles on n_threads threads (OpenMP; one
 * thread without it): the particles are split into n_threads contiguous
 * chunks, chunk c deposits into its own buffer of n_dg entries, and the
 * buffers are added to dg in chunk order, so the result depends only on
 * n_threads.  work holds n_threads * n_dg doubles.  Returns the first failing
 * chunk's status, or 0.
 */
int oracle_step_chunked(const OMesh *m, const double *e, const double *bv, int64_t n_p, double *pos, double *vel,
                        double *vh, double *ah, int64_t *tet, double q, double mass, double w, double dt, double *dg,
                        int64_t n_dg, int64_t *counters, int n_threads, double *work, int absorb, int pusher)
{
    int status[256];
    int64_t ncr[256], nrf[256], nab[256];
    if (n_threads < 1 || n_threads > 256) return -1;
#ifdef _OPENMP
#pragma omp parallel for num_threads(n_threads) schedule(static, 1)
#endif
    for (int c = 0; c < n_threads; c++) {
        double *buf = &work[(int64_t)c * n_dg];
        memset(buf, 0, (size_t)n_dg * sizeof(double));
        DepCtx ctx = {q * w, buf, 0, 0, absorb, 0, 0.0, NULL, NULL, 0, pusher};
        int64_t lo = n_p * c / n_threads, hi = n_p * (c + 1) / n_threads;
        status[c] = 0;
        for (int64_t p = lo; p < hi && !status[c]; p++)
            status[c] = step_one(m, e, bv, p, pos, vel, vh, ah, tet, q, mass, dt, &ctx);
        ncr[c] = ctx.ncross;
        nrf[c] = ctx.nrefl;
        nab[c] = ctx.nabs;
    }
    for (int c = 0; c < n_threads; c++) {
        if (status[c]) return status[c];
        const double *buf = &work[(int64_t)c * n_dg];
        for (int64_t i = 0; i < n_dg; i++) dg[i] += buf[i];
        if (counters) {
            counters[0] += ncr[c];
            counters[1] += nrf[c];
            counters[2] += nab[c];
        }
    }
    return 0;
}

/* AB4 start-up: a^0 from the fields at r^0; a^{-j} = a^0, v^{-j} = v^0 - j dt a^0 */
void oracle_startup(const OMesh *m, const double *e, const double *bv, int64_t n_p, double *pos, double *vel,
                    double *vh, double *ah, const int64_t *tet, double q, double mass, double dt)
{
    for (int64_t p = 0; p < n_p; p++) {
        double E[3], B[3], vxB[3], a[3];
        gather(m, tet[p], &pos[3 * p], e, bv, E, B);
        cross3(&vel[3 * p], B, vxB);
        for (int k = 0; k < 3; k++) a[k] = q / mass * (E[k] + vxB[k]);
        for (int j = 1; j <= 3; j++)
            for (int k = 0; k < 3; k++) {
                ah[9 * p + 3 * (j - 1) + k] = a[k];
                vh[9 * p + 3 * (j - 1) + k] = vel[3 * p + k] - j * dt * a[k];
            }
    }
}

/* E and B at given points (tests) */
void oracle_gather(const OMesh *m, const double *e, const double *bv, int64_t n, const double *pos,
                   const int64_t *tet, double *Eo, double *Bo)
{
    for (int64_t p = 0; p < n; p++) gather(m, tet[p], &pos[3 * p], e, bv, &Eo[3 * p], &Bo[3 * p]);
}

/* nodal charge measurement rho_j = q w sum_p W0_j(r_p)  (global W0 numbering) */
void oracle_rho(const OMesh *m, int64_t n, const double *pos, const int64_t *tet, double qw, double *rho)
{
    for (int64_t p = 0; p < n; p++) {
        double lam[4];
        if (tet[p] < 0) continue; /* absorbed */
        bary(m, tet[p], &pos[3 * p], lam);
        for (int j = 0; j < m->n0; j++) rho[m->map0[(int64_t)m->n0 * tet[p] + j]] += qw * w0_eval(m, j, lam);
    }
}

/* track + deposit a given path (coefficients c[5][3]) from tet t0 (tests) */
int64_t oracle_path_deposit(const OMesh *m, int64_t t0, double *cflat, double qw, double *dg, int64_t *counters,
                            int64_t *trace_t, double *trace_s, int32_t *ntrace)
{
    double c[5][3];
    memcpy(c, cflat, sizeof c);
    DepCtx ctx = {qw, dg, 0, 0, 0, 0, 0.0, trace_t, trace_s, 0};
    int nrefl;
    int64_t refl_t[ORACLE_MAX_CROSS + 1];
    int refl_f[ORACLE_MAX_CROSS + 1];
    int64_t t = track_and_deposit(m, t0, c, &ctx, &nrefl, refl_t, refl_f);
    memcpy(cflat, c, sizeof c);
    if (counters) {
        counters[0] += ctx.ncross;
        counters[1] += ctx.nrefl;
    }
    if (ntrace) *ntrace = ctx.ntrace;
    return t;
}

/* exit root of one polynomial (tests of the root finder) */
int oracle_first_negative(const double *q, double lo, double hi, double *u)
{
    return first_negative(q, lo, hi, 0, u);
}
