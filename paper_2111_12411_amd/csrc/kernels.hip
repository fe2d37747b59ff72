// HIP kernels of the fempic hot path for gfx950 (CDNA4, wave64).
//
//  * k_locate_cube        point location on a Kuhn cube
//  * k_startup            first gather and AB4 history start
//  * k_rs_hist/_scatter   stable LSD radix sort of (tet, slot) pairs (the
//                         per-step sort of particles by tet)
//  * k_particle           gather E,B (order-k edge/face bases) + AB4 push +
//                         quartic-path tet tracking + exact path-integral
//                         deposit; home-tet contributions reduced in LDS in a
//                         fixed order, other segments appended to a spill pool
//  * k_spill_*            deterministic reduction of the spill pool per tet
//  * k_scatter            per-tet partials -> DoF current moments (fixed order)
//  * k_mf_elem, k_mf_sum*  the field system's matrix applied tet by tet (the
//                         PCG iterations' product)
//  * SpMV / PCG / norms   field update, deterministic reductions
//
// No floating-point atomics anywhere: every floating-point sum is taken in a
// fixed order, so a run is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "kernels.h"

namespace fempic {

namespace {

constexpr int BLK = 256;

// integral of the cubic Lagrange basis on nodes 0,-1,-2,-3 (AB4 path), s^d coefficients
__device__ __constant__ const double LCOEF[4][5] = {
    {0.0, 1.0, 11.0 / 12.0, 1.0 / 3.0, 1.0 / 24.0},
    {0.0, 0.0, -3.0 / 2.0, -5.0 / 6.0, -1.0 / 8.0},
    {0.0, 0.0, 3.0 / 4.0, 2.0 / 3.0, 1.0 / 8.0},
    {0.0, 0.0, -1.0 / 6.0, -1.0 / 6.0, -1.0 / 24.0},
};

template <int K>
struct Ord;
// threads per block of the particle kernel; a block owns up to TPW_MAX
// consecutive tets and walks their particles in chunks of PBLK
constexpr int PBLK = PARTICLE_BLOCK;
template <>
struct Ord<1> {
    static constexpr int N1 = 6, N2 = 4, N0 = 4, NG = 4, TPW_MAX = PARTICLE_TPW_MAX_1;
};
template <>
struct Ord<2> {
    static constexpr int N1 = 20, N2 = 15, N0 = 10, NG = 6, TPW_MAX = PARTICLE_TPW_MAX_2;
};

// local edges (a,b) and faces (a,b,c); face f opposite vertex 3-f
__device__ __constant__ const int EA[6] = {0, 0, 0, 1, 1, 2};
__device__ __constant__ const int EB[6] = {1, 2, 3, 2, 3, 3};
// per face: vertices, pair ids of (b,c), (a,c), (a,b)
__device__ __constant__ const int FV[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
__device__ __constant__ const int FP[4][3] = {{3, 1, 0}, {4, 2, 0}, {5, 2, 1}, {5, 4, 3}};

}  // namespace

namespace {

// l_0 from the stored l_1..l_3 (always in this order of operations)
__device__ __forceinline__ double bary0(double l1, double l2, double l3) { return 1.0 - l1 - l2 - l3; }

// global-memory views of the pointers a kernel reads from its argument block:
// accesses through them compile to global (not flat) memory instructions, so
// waits on LDS reads do not also wait for outstanding global stores
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> glb(T *p)
{
    return (gptr<T>)p;
}

struct GMesh {
    gptr<const double> geo;
    gptr<const int32_t> nbr, map1, map2;
    int32_t nt;
};
__device__ inline GMesh gview(const DevMesh &m)
{
    return GMesh{glb(m.geo), glb(m.nbr), glb(m.map1), glb(m.map2), m.nt};
}

// the fields of row s, in the packed layout of precision R
template <typename R>
struct GParticles {
    static constexpr PartLayout L = sizeof(R) == 4 ? PART_MIXED : PART_FP64;
    gptr<char> w;
    int64_t cap;
    template <typename T>
    __device__ __forceinline__ gptr<T> at(int u, int64_t s) const
    {
        return (gptr<T>)(w + part_off(u, cap, s));
    }
    __device__ __forceinline__ gptr<double> lam(int c, int64_t s) const { return at<double>(L.lam + 2 * c, s); }
    __device__ __forceinline__ gptr<double> v(int c, int64_t s) const { return at<double>(L.v + 2 * c, s); }
    __device__ __forceinline__ gptr<R> vh(int c, int64_t s) const { return at<R>(L.vh + L.hs * c, s); }
    __device__ __forceinline__ gptr<R> ah(int c, int64_t s) const { return at<R>(L.ah + L.hs * c, s); }
    __device__ __forceinline__ gptr<int32_t> tet(int64_t s) const { return at<int32_t>(L.tet, s); }
    __device__ __forceinline__ gptr<int32_t> id(int64_t s) const { return at<int32_t>(L.id, s); }
};
template <typename R>
__device__ inline GParticles<R> gview(const DevParticles &p)
{
    return GParticles<R>{glb((char *)p.w), p.cap};
}

// ---------------------------------------------------------------- locate
// (the position, the l_1..l_3 units until k_to_bary, and tet share their units in
// both layouts)
__device__ __forceinline__ double *prow_lam(const DevParticles &P, int c, int64_t p)
{
    return (double *)((char *)P.w + part_off(PART_MIXED.lam + 2 * c, P.cap, p));
}
__device__ __forceinline__ int32_t *prow_tet(const DevParticles &P, int64_t p)
{
    return (int32_t *)((char *)P.w + part_off(PART_MIXED.tet, P.cap, p));
}
static_assert(PART_MIXED.lam == PART_FP64.lam && PART_MIXED.tet == PART_FP64.tet, "shared units");

__global__ void k_locate_cube(DevMesh m, int64_t n, DevParticles P, int32_t *__restrict__ err)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int N = m.cube_N;
    const double L = m.cube_L;
    double r[3] = {*prow_lam(P, 0, p), *prow_lam(P, 1, p), *prow_lam(P, 2, p)};
    const double tol = 1e-12 * L;
    int idx[3];
    bool ok = true;
    for (int k = 0; k < 3; k++) {
        if (!(r[k] >= -tol && r[k] <= L + tol)) ok = false;
        double f = ok ? floor(r[k] * N / L) : 0.0;
        int i = (int)f;
        idx[k] = i < 0 ? 0 : (i > N - 1 ? N - 1 : i);
    }
    int64_t h = idx[0] + (int64_t)N * (idx[1] + (int64_t)N * idx[2]);
    double best = -1e300;
    int32_t bt = (int32_t)(6 * h);
    for (int q = 0; q < 6; q++) {
        int64_t t = 6 * h + q;
        const double *g = &m.geo[16 * t];
        double mn = 1e300;
        for (int f = 0; f < 4; f++) {
            double l = g[4 * f] + g[4 * f + 1] * r[0] + g[4 * f + 2] * r[1] + g[4 * f + 3] * r[2];
            mn = fmin(mn, l);
        }
        if (mn > best) {
            best = mn;
            bt = (int32_t)t;
        }
    }
    *prow_tet(P, p) = bt;
    if (!ok || !(best >= -1e-10)) atomicOr(err, (int)ERR_OUTSIDE);
}

// positions replaced in place by l_1..l_3 of their tets
__global__ void k_to_bary(DevMesh m, int64_t n, DevParticles P)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double *g = &m.geo[16 * (int64_t)*prow_tet(P, p)];
    const double r0 = *prow_lam(P, 0, p), r1 = *prow_lam(P, 1, p), r2 = *prow_lam(P, 2, p);
    double l[3];
    for (int f = 1; f < 4; f++) l[f - 1] = g[4 * f] + g[4 * f + 1] * r0 + g[4 * f + 2] * r1 + g[4 * f + 3] * r2;
    for (int c = 0; c < 3; c++) *prow_lam(P, c, p) = l[c];
}

// ------------------------------------------------------------- gather
// E = sum_m cE[m] grad l_m ; B = sum_p cB[p] (grad l_a x grad l_b)_p
template <int K, typename R>
__device__ inline void gather_coeffs(const R *ec, const R *bc, const R lam[4], R cE[4], R cB[6])
{
#pragma unroll
    for (int m = 0; m < 4; m++) cE[m] = R(0);
#pragma unroll
    for (int p = 0; p < 6; p++) cB[p] = R(0);
    if constexpr (K == 1) {
#pragma unroll
        for (int e = 0; e < 6; e++) {
            R w = ec[e];
            cE[EB[e]] += w * lam[EA[e]];
            cE[EA[e]] -= w * lam[EB[e]];
        }
#pragma unroll
        for (int f = 0; f < 4; f++) {
            R s = R(2) * bc[f];
            cB[FP[f][0]] += s * lam[FV[f][0]];
            cB[FP[f][1]] -= s * lam[FV[f][1]];
            cB[FP[f][2]] += s * lam[FV[f][2]];
        }
    } else {
#pragma unroll
        for (int e = 0; e < 6; e++) {
            const int a = EA[e], b = EB[e];
            R w = ec[2 * e] * (R(3) * lam[a] - R(1)) + ec[2 * e + 1] * (R(3) * lam[b] - R(1));
            cE[b] += w * lam[a];
            cE[a] -= w * lam[b];
        }
#pragma unroll
        for (int f = 0; f < 4; f++) {
            const int a = FV[f][0], b = FV[f][1], c = FV[f][2];
            R w1 = ec[12 + 2 * f] * (R(3) * lam[c]);  // W_ab
            cE[b] += w1 * lam[a];
            cE[a] -= w1 * lam[b];
            R w2 = ec[13 + 2 * f] * (R(3) * lam[b]);  // W_ac
            cE[c] += w2 * lam[a];
            cE[a] -= w2 * lam[c];
            R s = bc[3 * f] * (R(4) * lam[a] - R(1)) + bc[3 * f + 1] * (R(4) * lam[b] - R(1)) +
                  bc[3 * f + 2] * (R(4) * lam[c] - R(1));
            if (f < 3) s += bc[12 + f] * (R(4) * lam[3 - f]);
            s *= R(2);
            cB[FP[f][0]] += s * lam[a];
            cB[FP[f][1]] -= s * lam[b];
            cB[FP[f][2]] += s * lam[c];
        }
    }
}

template <typename R>
__device__ inline void cross3(const R *a, const R *b, R *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// ---------------------------------------------------------------- startup
template <int K, typename R>
__global__ void k_startup(DevMesh m, const R *__restrict__ e, const R *__restrict__ b, DevParticles P, int64_t n,
                          double qm, double dt)
{
    using O = Ord<K>;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const GParticles<R> Q = gview<R>(P);
    const int64_t t = *Q.tet(p);
    const double *g = &m.geo[16 * t];
    const double l1 = *Q.lam(0, p), l2 = *Q.lam(1, p), l3 = *Q.lam(2, p);
    R lam[4] = {(R)bary0(l1, l2, l3), (R)l1, (R)l2, (R)l3}, gr[4][3];
    for (int f = 0; f < 4; f++)
        for (int k = 0; k < 3; k++) gr[f][k] = (R)g[4 * f + 1 + k];
    R ec[O::N1], bc[O::N2];
    for (int i = 0; i < O::N1; i++) ec[i] = e[m.map1[t * O::N1 + i]];
    for (int l = 0; l < O::N2; l++) bc[l] = b[m.map2[t * O::N2 + l]];
    R cE[4], cB[6];
    gather_coeffs<K, R>(ec, bc, lam, cE, cB);
    R E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
    for (int f = 0; f < 4; f++)
        for (int k = 0; k < 3; k++) E[k] += cE[f] * gr[f][k];
    for (int q = 0; q < 6; q++) {
        R X[3];
        cross3(gr[EA[q]], gr[EB[q]], X);
        for (int k = 0; k < 3; k++) B[k] += cB[q] * X[k];
    }
    const double vd[3] = {*Q.v(0, p), *Q.v(1, p), *Q.v(2, p)};
    R v[3] = {(R)vd[0], (R)vd[1], (R)vd[2]}, vxB[3], a[3];
    cross3(v, B, vxB);
    for (int k = 0; k < 3; k++) a[k] = (R)qm * (E[k] + vxB[k]);
    R vh[9], ah[9];
    // velocity history as differences from the current velocity: v^{n-j} - v^n
    for (int j = 1; j <= 3; j++)
        for (int k = 0; k < 3; k++) {
            ah[3 * (j - 1) + k] = a[k];
            vh[3 * (j - 1) + k] = (R)(-j * dt * (double)a[k]);
        }
    for (int c = 0; c < 9; c++) {
        *Q.vh(c, p) = vh[c];
        *Q.ah(c, p) = ah[c];
    }
}

// ------------------------------------------------------------ root finding
__device__ inline double horner4(const double *q, double u)
{
    return fma(fma(fma(fma(q[4], u, q[3]), u, q[2]), u, q[1]), u, q[0]);
}

__device__ inline double dhorner4(const double *q, double u)
{
    return fma(fma(fma(4.0 * q[4], u, 3.0 * q[3]), u, 2.0 * q[2]), u, q[1]);
}

// coefficients of p(u + a)
__device__ inline void taylor_shift(const double *p, double a, double *o)
{
    double c0 = p[0], c1 = p[1], c2 = p[2], c3 = p[3], c4 = p[4];
    c3 = fma(a, c4, c3);
    c2 = fma(a, c3, c2);
    c1 = fma(a, c2, c1);
    c0 = fma(a, c1, c0);
    c3 = fma(a, c4, c3);
    c2 = fma(a, c3, c2);
    c1 = fma(a, c2, c1);
    c3 = fma(a, c4, c3);
    c2 = fma(a, c3, c2);
    c3 = fma(a, c4, c3);
    o[0] = c0;
    o[1] = c1;
    o[2] = c2;
    o[3] = c3;
    o[4] = c4;
}

// Bernstein coefficients on [lo, hi] of q (power basis in u)
__device__ inline void bernstein(const double *q, double lo, double hi, double *bc)
{
    double d[5];
    taylor_shift(q, lo, d);
    const double h = hi - lo;
    double d1 = d[1] * h, d2 = d[2] * h * h, d3 = d[3] * h * h * h, d4 = d[4] * (h * h) * (h * h);
    bc[0] = d[0];
    bc[1] = d[0] + 0.25 * d1;
    bc[2] = d[0] + 0.5 * d1 + d2 / 6.0;
    bc[3] = d[0] + 0.75 * d1 + 0.5 * d2 + 0.25 * d3;
    bc[4] = d[0] + d1 + d2 + d3 + d4;
}

// Newton refinement of the single crossing of q in (lo, hi): q(lo) >= 0 > q(hi)
// (values flo, fhi).  Regula-falsi start, Newton steps kept inside the
// shrinking bracket (bisection when a step leaves it).  Stops once the Newton
// correction is below tol (absolute, in u): at convergence the corrected point
// can round onto a bracket end, which must not be taken for a step that left
// the bracket.  The bracket bound ends the loop in any case (about 60 halvings
// reach tol from a bracket of length H).
__device__ inline double refine_root(const double *q, double lo, double hi, double flo, double fhi, double tol)
{
    double a = lo, b = hi;
    double x = lo + (hi - lo) * (flo / (flo - fhi));
    if (!(x > a && x < b)) x = 0.5 * (a + b);
    for (int it = 0; it < 64; it++) {
        const double fx = horner4(q, x);
        if (fx == 0.0) break;
        if (fx < 0.0) b = x; else a = x;
        const double dx = fx / dhorner4(q, x);
        if (fabs(dx) <= tol) {
            x -= dx;
            break;
        }
        double xn = x - dx;
        if (!(xn > a && xn < b)) xn = 0.5 * (a + b);
        x = xn;
        if (b - a <= tol) break;
    }
    return fmin(fmax(x, lo), hi);
}

// smallest u in [0, H] with q(u) < 0 (q in power basis of u).  Dyadic
// subdivision driven by Bernstein sign tests, then safeguarded Newton on the
// isolated crossing.  Visits a bounded number of intervals.
__device__ bool first_negative(const double *q, double H, double &uout)
{
    constexpr int MAXD = 40;
    int d = 0;
    int64_t idx = 0;
    for (int guard = 0; guard < 1024; guard++) {
        const double lo = H * ldexp((double)idx, -d);
        const double hi = H * ldexp((double)(idx + 1), -d);
        double bc[5];
        bernstein(q, lo, hi, bc);
        int first = -1;
#pragma unroll
        for (int i = 4; i >= 0; i--)
            if (bc[i] != 0.0) first = i;
        bool advance = false;
        if (first < 0) {
            advance = true;
        } else if (bc[first] < 0.0) {
            uout = lo;
            return true;
        } else {
            bool any_neg = false;
            int changes = 0;
            double prev = bc[first];
#pragma unroll
            for (int i = 0; i < 5; i++) {
                if (i <= first) continue;
                if (bc[i] < 0.0) any_neg = true;
                if (bc[i] != 0.0) {
                    if ((bc[i] < 0.0) != (prev < 0.0)) changes++;
                    prev = bc[i];
                }
            }
            if (!any_neg) {
                advance = true;
            } else if (changes == 1 && bc[4] < 0.0) {
                // one crossing in (lo, hi): q(lo) >= 0 > q(hi)
                uout = refine_root(q, lo, hi, bc[0], bc[4], 4e-16 * H);
                return true;
            } else if (d >= MAXD) {
                advance = true;  // tangency narrower than H 2^-40
            }
        }
        if (advance) {
            while (idx & 1) {
                idx >>= 1;
                d--;
            }
            if (d == 0) return false;
            idx += 1;
        } else {
            d++;
            idx <<= 1;
        }
    }
    return false;
}

// -------------------------------------------------------------- particle
// barycentric coordinate of face f (opposite vertex f) along the path, as a
// polynomial in u = s - s_lo: its value l0 at s_lo plus grad l_f . (r(s) - r(s_lo)),
// where dp holds the displacement r(s) - r(0) as powers 1..4 of s.  The value at
// s_lo is carried from segment to segment (and from step to step) rather than
// recomputed from a position, so that the W0 values at the ends of consecutive
// segments are the same numbers and the deposit telescopes exactly.
template <bool FROM_ZERO, typename GPtr>
__device__ inline void face_poly(GPtr G, int f, const double (&dp)[4][3], double s_lo, double l0, double *q)
{
    const double gx = G[4 * f + 1], gy = G[4 * f + 2], gz = G[4 * f + 3];
    q[0] = 0.0;
#pragma unroll
    for (int d = 1; d < 5; d++) q[d] = fma(gz, dp[d - 1][2], fma(gy, dp[d - 1][1], gx * dp[d - 1][0]));
    if (!FROM_ZERO) taylor_shift(q, s_lo, q);
    q[0] = l0;
}

// exit of tet G from s_lo along the path dp, whose barycentric coordinates at
// s_lo are l0: the first s > s_lo where a coordinate turns negative (the entry
// face's coordinate is zero at s_lo).  A face whose Bernstein coefficients on [s_lo, 1] are all
// non-negative cannot be crossed; this straight-line test settles most lanes.
// The flagged faces of a lane (usually one) then go through the full search,
// in increasing face order, each limited to the best crossing found so far.
template <bool FROM_ZERO, typename GPtr>
__device__ inline int find_exit(GPtr G, const double (&dp)[4][3], const double (&l0)[4], double s_lo, int entry,
                                double &s_exit)
{
    s_exit = 2.0;
    const double H = 1.0 - s_lo;
    if (!(H > 0.0)) return -1;
    const double H2 = H * H;
    unsigned negmask = 0;
#pragma unroll
    for (int f = 0; f < 4; f++) {
        double q[5];
        face_poly<FROM_ZERO>(G, f, dp, s_lo, l0[f], q);
        if (f == entry) q[0] = 0.0;
        const double d1 = q[1] * H, d2 = q[2] * H2, d3 = q[3] * H2 * H, d4 = q[4] * H2 * H2;
        const double b1 = fma(0.25, d1, q[0]);
        const double b2 = fma(1.0 / 6.0, d2, fma(0.5, d1, q[0]));
        const double b3 = fma(0.25, d3, fma(0.5, d2, fma(0.75, d1, q[0])));
        const double b4 = q[0] + d1 + d2 + d3 + d4;
        const double mn = fmin(fmin(q[0], b1), fmin(fmin(b2, b3), b4));
        negmask |= (mn < 0.0 ? 1u : 0u) << f;
    }
    if (!negmask) return -1;
    double ubest = H;
    int fbest = -1;
    while (negmask) {
        const int f = __builtin_ctz(negmask);
        negmask &= negmask - 1u;
        double q[5];
        face_poly<FROM_ZERO>(G, f, dp, s_lo, l0[f], q);
        if (f == entry) q[0] = 0.0;
        double u;
        if (first_negative(q, fbest < 0 ? H : ubest, u) && (fbest < 0 || u < ubest)) {
            ubest = u;
            fbest = f;
        }
    }
    if (fbest < 0) return -1;
    s_exit = s_lo + ubest;
    return fbest;
}

// Exit search without data-dependent loops, for the common cases.  Each face
// is classified by its Bernstein coefficients on [s_lo, 1]: all non-negative
// (never crossed), or positive at s_lo and negative at 1 with exactly one sign
// change (exactly one crossing inside).  The crossing face with the smallest
// regula-falsi estimate is refined by a fixed number of bracketed Newton steps;
// every other crossing face must then stay non-negative up to that root (its
// Bernstein coefficients on [s_lo, root] are non-negative).  Returns the exit
// face (s_exit set), -1 for no exit, or -2 when the case needs the full search
// (any other sign pattern, a start on a face, or no convergence).
template <bool FROM_ZERO, typename GPtr>
__device__ inline int fast_exit(GPtr G, const double (&dp)[4][3], const double (&l0)[4], double s_lo, int entry,
                                double &s_exit)
{
    s_exit = 2.0;
    const double H = 1.0 - s_lo;
    if (!(H > 0.0)) return -1;
    const double H2 = H * H;
    int best = -1;
    double bnum = 0.0, bden = 1.0;  // regula-falsi estimate of the best face: H bnum / bden
    bool hard = false;
    unsigned cand = 0;
#pragma unroll
    for (int f = 0; f < 4; f++) {
        double q[5];
        face_poly<FROM_ZERO>(G, f, dp, s_lo, l0[f], q);
        if (f == entry) q[0] = 0.0;
        const double d1 = q[1] * H, d2 = q[2] * H2, d3 = q[3] * H2 * H, d4 = q[4] * H2 * H2;
        const double b0 = q[0];
        const double b1 = fma(0.25, d1, b0);
        const double b2 = fma(1.0 / 6.0, d2, fma(0.5, d1, b0));
        const double b3 = fma(0.25, d3, fma(0.5, d2, fma(0.75, d1, b0)));
        const double b4 = b0 + d1 + d2 + d3 + d4;
        const double mn = fmin(fmin(b0, b1), fmin(fmin(b2, b3), b4));
        if (mn < 0.0) {
            const int ch = ((b1 < 0.0) != (b0 < 0.0)) + ((b2 < 0.0) != (b1 < 0.0)) + ((b3 < 0.0) != (b2 < 0.0)) +
                           ((b4 < 0.0) != (b3 < 0.0));
            if (b0 > 0.0 && b4 < 0.0 && ch == 1) {
                // estimates compared without dividing: b0/(b0-b4) < bnum/bden
                cand |= 1u << f;
                if (best < 0 || b0 * bden < bnum * (b0 - b4)) {
                    best = f;
                    bnum = b0;
                    bden = b0 - b4;
                }
            } else {
                hard = true;
            }
        }
    }
    if (hard) return -2;
    if (best < 0) return -1;
    double q[5];
    face_poly<FROM_ZERO>(G, best, dp, s_lo, l0[best], q);
    double a = 0.0, b = H, x = H * (bnum / bden);
    if (!(x > a && x < b)) x = 0.5 * H;
    const double tol = 4e-16 * H;
    bool conv = false;
#pragma unroll
    for (int it = 0; it < 6; it++) {
        if (__all(conv)) break;
        const double fx = horner4(q, x);
        const double dx = fx / dhorner4(q, x);
        if (!conv) {
            if (fx < 0.0) b = x; else a = x;
            if (fx == 0.0 || fabs(dx) <= tol) {
                if (fx != 0.0) x -= dx;
                conv = true;
            } else {
                double xn = x - dx;
                if (!(xn > a && xn < b)) xn = 0.5 * (a + b);
                x = xn;
            }
        }
    }
    if (!conv) return -2;
    x = fmin(fmax(x, 0.0), H);
    cand &= ~(1u << best);
    const double x2 = x * x;
#pragma unroll
    for (int f = 0; f < 4; f++) {
        if (cand & (1u << f)) {
            face_poly<FROM_ZERO>(G, f, dp, s_lo, l0[f], q);
            const double d1 = q[1] * x, d2 = q[2] * x2, d3 = q[3] * x2 * x, d4 = q[4] * x2 * x2;
            const double b1 = fma(0.25, d1, q[0]);
            const double b2 = fma(1.0 / 6.0, d2, fma(0.5, d1, q[0]));
            const double b3 = fma(0.25, d3, fma(0.5, d2, fma(0.75, d1, q[0])));
            const double b4 = q[0] + d1 + d2 + d3 + d4;
            if (fmin(fmin(b1, b2), fmin(b3, b4)) < 0.0) hard = true;
        }
    }
    if (hard) return -2;
    s_exit = s_lo + x;
    return best;
}

// current moments of a path segment inside one tet:
// dep_i = q w int Q_i(l) (l_a l_b' - l_b l_a') du over u in [0, h], where
// lq[m-1] holds l_m (m = 1..3) along the path as a quartic in u (the face
// polynomials of the exit search), l_0 = 1 - l_1 - l_2 - l_3 and
// l_0' = -(l_1' + l_2' + l_3'); Gauss-Legendre nodes on [0, h].  Only the
// local DoFs C0 <= i < C1 are accumulated (a caller short of registers takes
// the DoFs in two passes).
// LINE: the path is straight (the Boris push), so the coordinates are linear in
// u and the integrand has degree k: ceil((k+1)/2) Gauss-Legendre points are
// exact (1 at order 1, 2 at order 2) instead of the 2k+2 of the quartic path.
template <bool LINE>
struct SegRule;
template <>
struct SegRule<true> {
    // Gauss-Legendre on [0, 1]: 1 point (x = 1/2) and 2 points (x = 1/2 -+ 1/(2 sqrt 3))
    static constexpr double X2 = 0.5 / 1.7320508075688772935;
    __device__ static double x(int n, int g) { return n == 1 ? 0.5 : (g == 0 ? 0.5 - X2 : 0.5 + X2); }
    __device__ static double w(int n, int) { return n == 1 ? 1.0 : 0.5; }
};
template <int K, int C0 = 0, int C1 = Ord<K>::N1, bool LINE = false>
__device__ inline void segment_moments(const double (&lq)[3][5], double h, double qw, const GLRule &gl, double *dep)
{
    using O = Ord<K>;
    constexpr int NG = LINE ? (K + 2) / 2 : O::NG;
#pragma unroll
    for (int c = C0; c < C1; c++) dep[c] = 0.0;
    const double qwh = qw * h;
#pragma unroll
    for (int g = 0; g < NG; g++) {
        const double u = h * (LINE ? SegRule<true>::x(NG, g) : gl.x[g]);
        const double wg = qwh * (LINE ? SegRule<true>::w(NG, g) : gl.w[g]);
        double lam[4], dl[4];  // dl carries the quadrature weight
#pragma unroll
        for (int m = 1; m < 4; m++) {
            if constexpr (LINE) {
                lam[m] = fma(lq[m - 1][1], u, lq[m - 1][0]);
                dl[m] = wg * lq[m - 1][1];
            } else {
                lam[m] = horner4(lq[m - 1], u);
                dl[m] = wg * dhorner4(lq[m - 1], u);
            }
        }
        lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
        dl[0] = -(dl[1] + dl[2] + dl[3]);
        double w[6];
#pragma unroll
        for (int e = 0; e < 6; e++) w[e] = fma(lam[EA[e]], dl[EB[e]], -lam[EB[e]] * dl[EA[e]]);
        auto acc = [&](int c, double f, double x) {
            if (c >= C0 && c < C1) dep[c] = fma(f, x, dep[c]);
        };
        if constexpr (K == 1) {
#pragma unroll
            for (int e = 0; e < 6; e++) acc(e, 1.0, w[e]);
        } else {
#pragma unroll
            for (int e = 0; e < 6; e++) {
                acc(2 * e, 3.0 * lam[EA[e]] - 1.0, w[e]);
                acc(2 * e + 1, 3.0 * lam[EB[e]] - 1.0, w[e]);
            }
            // faces (a,b,c): 3 l_c W_ab and 3 l_b W_ac
            acc(12, 3.0 * lam[2], w[0]);
            acc(13, 3.0 * lam[1], w[1]);
            acc(14, 3.0 * lam[3], w[0]);
            acc(15, 3.0 * lam[1], w[2]);
            acc(16, 3.0 * lam[3], w[1]);
            acc(17, 3.0 * lam[2], w[2]);
            acc(18, 3.0 * lam[3], w[3]);
            acc(19, 3.0 * lam[2], w[4]);
        }
    }
}

struct GPool {
    gptr<double> val;
    gptr<int32_t> tet;
    gptr<int64_t> tag;
    gptr<int32_t> pid, count, rcount;
    int64_t cap;
};
__device__ inline GPool gview(const SpillPool &p)
{
    return GPool{glb(p.val), glb(p.tet), glb(p.tag), glb(p.pid), glb(p.count), glb(p.rcount), p.cap};
}

// leave tet t through face f, with lam the coordinates of tet t at the crossing
// point: move to the neighbour, whose coordinates there replace lam, or at a PEC
// wall mirror the rest of the path about the face plane together with the
// stored velocity and AB4 histories of particle i (written before tracking).
// With absorb, a wall ends the path instead: nothing is mirrored and true is
// returned.
template <typename R, typename GPtr>
__device__ inline bool cross_face(const GMesh &m, GPtr G, int f, int &t, int &entry, double (&dp)[4][3],
                                  double (&lam)[4], const GParticles<R> &out, int64_t i, unsigned long long &nrf,
                                  bool absorb, bool hist)
{
    const int nx = m.nbr[(int64_t)t * 4 + f];
    if (nx >= 0) {
        // both tets list their vertices in ascending global order, so the three
        // shared vertices come in the same order in each: they keep their
        // coordinates, and the neighbour's vertex across the face starts at 0
        const int e = nx & 3;
        const double s0 = f == 0 ? lam[1] : lam[0];
        const double s1 = f <= 1 ? lam[2] : lam[1];
        const double s2 = f <= 2 ? lam[3] : lam[2];
        lam[0] = e == 0 ? 0.0 : s0;
        lam[1] = e == 0 ? s0 : (e == 1 ? 0.0 : s1);
        lam[2] = e <= 1 ? s1 : (e == 2 ? 0.0 : s2);
        lam[3] = e <= 2 ? s2 : 0.0;
        entry = e;
        t = nx >> 2;
        return false;
    }
    if (absorb) return true;
    lam[f] = 0.0;
    const double gx = G[4 * f + 1], gy = G[4 * f + 2], gz = G[4 * f + 3];
    const double inv = 2.0 / (gx * gx + gy * gy + gz * gz);
    // the crossing point lies on the plane: mirroring the displacement from it
    // mirrors the path
#pragma unroll
    for (int d = 0; d < 4; d++) {
        const double sd = (gx * dp[d][0] + gy * dp[d][1] + gz * dp[d][2]) * inv;
        dp[d][0] -= sd * gx;
        dp[d][1] -= sd * gy;
        dp[d][2] -= sd * gz;
    }
    {
        const double x0 = *out.v(0, i), x1 = *out.v(1, i), x2 = *out.v(2, i);
        const double sd = (gx * x0 + gy * x1 + gz * x2) * inv;
        *out.v(0, i) = x0 - sd * gx;
        *out.v(1, i) = x1 - sd * gy;
        *out.v(2, i) = x2 - sd * gz;
    }
#pragma unroll 1
    for (int h = 0; h < (hist ? 6 : 0); h++) {  // no histories with the Boris push
        const int c0 = 3 * (h % 3);
        const gptr<R> h0 = h < 3 ? out.vh(c0, i) : out.ah(c0, i);
        const gptr<R> h1 = h < 3 ? out.vh(c0 + 1, i) : out.ah(c0 + 1, i);
        const gptr<R> h2 = h < 3 ? out.vh(c0 + 2, i) : out.ah(c0 + 2, i);
        const double x0 = *h0, x1 = *h1, x2 = *h2;
        const double sd = (gx * x0 + gy * x1 + gz * x2) * inv;
        *h0 = (R)(x0 - sd * gx);
        *h1 = (R)(x1 - sd * gy);
        *h2 = (R)(x2 - sd * gz);
    }
    nrf++;
    entry = f;
    return false;
}

// wave-aggregated slot in a shared append buffer
__device__ inline int64_t append_slot(gptr<int32_t> count)
{
    const unsigned long long mask = __ballot(1);
    const int lane = __lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    int basei = 0;
    if (lane == leader)
        basei = __hip_atomic_fetch_add(count, (int)__popcll(mask), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    basei = __shfl(basei, leader);
    return (int64_t)basei + rank;
}

// A path crosses at most MAX_CROSS faces in one step, so it has at most
// MAX_CROSS + 1 segments; every segment of a path handed whole to k_continue
// is a spill record.  Spill tags: (queued record << 8) | (last << 7) | segment.
constexpr int MAX_CROSS = 64;
constexpr int MAX_SEG = MAX_CROSS + 1;

// claims the spill record for segment nsp_i of queued record r (tet t): segments 0 and 1 take the fixed slots 2r and 2r+1, later ones are
// appended after the fixed region of 2 nq slots.  The record of the path's
// last segment (last) also carries the particle's sorted index i.  Returns the
// slot, or -1 (and flags ERR_POOL) when the pool is full.
__device__ inline int64_t spill_slot(const GPool &pool, int64_t r, int64_t nq, int t, bool last, int64_t i,
                                     int &nsp_i, int &errs)
{
    int64_t slot = nsp_i < 2 ? 2 * r + nsp_i : 2 * nq + append_slot(pool.count);
    if (slot < pool.cap && nsp_i < MAX_SEG) {
        pool.tet[slot] = t;
        pool.tag[slot] = (r << 8) | ((int64_t)last << 7) | nsp_i;
        if (last) pool.pid[slot] = (int32_t)i;
    } else {
        errs |= ERR_POOL;
        slot = -1;
    }
    nsp_i++;
    return slot;
}

// counters of a block (crossings, reflections, spills, error flags, absorbed),
// summed in a fixed order and written to the block's own slot of cntb
__device__ inline void block_counters(gptr<unsigned long long> cntb, unsigned long long ncr, unsigned long long nrf,
                                      unsigned long long nsp, int errs, unsigned long long nab)
{
    __shared__ unsigned long long s_c[BLK / 64][NCNT];
    for (int o = 32; o > 0; o >>= 1) {
        ncr += __shfl_xor(ncr, o);
        nrf += __shfl_xor(nrf, o);
        nsp += __shfl_xor(nsp, o);
        errs |= __shfl_xor(errs, o);
        nab += __shfl_xor(nab, o);
    }
    const int w = threadIdx.x / 64;
    if (__lane_id() == 0) {
        s_c[w][CNT_CROSS] = ncr;
        s_c[w][CNT_REFL] = nrf;
        s_c[w][CNT_SPILL] = nsp;
        s_c[w][CNT_ERR] = (unsigned long long)errs;
        s_c[w][CNT_ABSORB] = nab;
        for (int k = CNT_ABSORB + 1; k < NCNT; k++) s_c[w][k] = 0ull;
    }
    __syncthreads();
    if (threadIdx.x < NCNT) {
        unsigned long long v = 0;
        for (int k = 0; k < BLK / 64; k++)
            v = threadIdx.x == CNT_ERR ? (v | s_c[k][CNT_ERR]) : v + s_c[k][threadIdx.x];
        cntb[(int64_t)blockIdx.x * NCNT + threadIdx.x] = v;
    }
}

// lanes [lo, hi) of a wave as a bit mask (bounds clamped to [0, 64])
__device__ inline unsigned long long lane_range(int lo, int hi)
{
    lo = max(lo, 0);
    hi = min(hi, 64);
    if (lo >= hi) return 0ull;
    const unsigned long long up = hi == 64 ? ~0ull : (1ull << hi) - 1ull;
    return up & ~((1ull << lo) - 1ull);
}

// Kernel 1: per particle (sorted by tet), gather + AB4 push + the first path
// segment, which lies in the home tet; its current moments are summed per tet
// in LDS in a fixed order.  A particle whose path leaves the home tet is queued
// for k_continue.
// BORIS: the Boris leapfrog (the stored velocity is v^{n-1/2}) with a straight
// path, in place of the AB4 push and its quartic path; no histories are read or
// written.
template <int K, typename R, bool BORIS = false>
__global__ __launch_bounds__(PBLK, 3) void k_particle(const ParticleArgs *__restrict__ A)
{
    const GMesh m = gview(A->m);
    const gptr<const R> e = glb((const R *)A->e);
    const gptr<const R> b = glb((const R *)A->b);
    const gptr<const uint32_t> perm = glb(A->perm);
    const gptr<const int32_t> off = glb(A->off);
    const GParticles<R> in = gview<R>(A->in);
    const GParticles<R> out = gview<R>(A->out);
    const StepParams &sp = A->sp;
    const GLRule &gl = A->gl;
    const gptr<double> P = glb(A->P);
    const gptr<ContRec> qrec = glb(A->cq.rec);
    const gptr<uint8_t> qflag = glb(A->cq.flag);
    const gptr<uint8_t> qmoved = glb(A->cq.moved);
    using O = Ord<K>;
    constexpr int N1 = O::N1, N2 = O::N2, TM = O::TPW_MAX;
    __shared__ double s_geo[TM][16];
    __shared__ R s_X[TM][18];
    __shared__ R s_e[TM][N1];
    __shared__ R s_b[TM][N2];
    __shared__ int32_t s_off[TM + 1];
    __shared__ int32_t s_nstay[TM];  // particles of each tet that are not queued
    __shared__ int32_t s_nbr[TM][4];
    __shared__ double s_hc[N1][PBLK + 1];

    const int tid = threadIdx.x;
    const int tpw = sp.tpw;
    const int T0 = blockIdx.x * tpw;
    const int T1 = min(T0 + tpw, m.nt);
    const int ntl = T1 - T0;
    // sort slot of this thread's particle in the block's first chunk, requested
    // ahead of the staging below (each chunk requests the next chunk's slot)
    const int pbeg = off[T0], pend = off[T1];
    uint32_t nslot = pbeg + tid < pend ? perm[pbeg + tid] : 0u;
    for (int k = tid; k < ntl * 16; k += PBLK) s_geo[k / 16][k % 16] = m.geo[(int64_t)T0 * 16 + k];
    for (int k = tid; k <= ntl; k += PBLK) s_off[k] = off[T0 + k];
    for (int k = tid; k < ntl * 4; k += PBLK) s_nbr[k / 4][k % 4] = m.nbr[(int64_t)T0 * 4 + k];
    for (int k = tid; k < TM; k += PBLK) s_nstay[k] = 0;
    // the step's counters, which later kernels of the step accumulate into
    if (blockIdx.x == 0 && tid < NCNT) glb(A->cnt)[tid] = 0ull;
    if (blockIdx.x == 0 && tid == 0) {
        *glb(A->pool.count) = 0;
        *glb(A->perr) = 0ull;
    }
    for (int k = tid; k < ntl * N1; k += PBLK) {
        int t = k / N1, i = k % N1;
        s_e[t][i] = e[m.map1[(int64_t)(T0 + t) * N1 + i]];
    }
    for (int k = tid; k < ntl * N2; k += PBLK) {
        int t = k / N2, l = k % N2;
        s_b[t][l] = b[m.map2[(int64_t)(T0 + t) * N2 + l]];
    }
    __syncthreads();
    for (int k = tid; k < ntl * 6; k += PBLK) {
        int t = k / 6, q = k % 6;
        double ga[3], gb[3], X[3];
        for (int c = 0; c < 3; c++) {
            ga[c] = s_geo[t][4 * EA[q] + 1 + c];
            gb[c] = s_geo[t][4 * EB[q] + 1 + c];
        }
        cross3(ga, gb, X);
        for (int c = 0; c < 3; c++) s_X[t][3 * q + c] = (R)X[c];
    }
    __syncthreads();

    // (tet, component) pairs of the block's sums: pair tid + q PBLK for q < NP
    constexpr int NP = (TM * N1 + PBLK - 1) / PBLK;
    double acc[NP];
#pragma unroll
    for (int q = 0; q < NP; q++) acc[q] = 0.0;
    const R dtR = (R)sp.dt;
    const R qmR = (R)sp.qm;

    for (int base = pbeg; base < pend; base += PBLK) {
#pragma unroll
        for (int c = 0; c < N1; c++) s_hc[c][tid] = 0.0;
        const int i = base + tid;
        const uint32_t slot = min(nslot, (uint32_t)(in.cap - 1));  // perm holds slots < cap
        if (i + PBLK < pend) nslot = perm[i + PBLK];
        if (i < pend) {
            const int th = *in.tet(slot);
            const int lt = th - T0;
            const double l1 = *in.lam(0, slot), l2 = *in.lam(1, slot), l3 = *in.lam(2, slot);
            const double ls[4] = {bary0(l1, l2, l3), l1, l2, l3};
            double vd[3];
            R vh[9], ah[9];
#pragma unroll
            for (int c = 0; c < 3; c++) vd[c] = *in.v(c, slot);
            if constexpr (!BORIS) {
#pragma unroll
                for (int c = 0; c < 9; c++) {
                    vh[c] = *in.vh(c, slot);
                    ah[c] = *in.ah(c, slot);
                }
            }
            const R v[3] = {(R)vd[0], (R)vd[1], (R)vd[2]};
            // fields at r^n (home tet, LDS)
            const R lam[4] = {(R)ls[0], (R)ls[1], (R)ls[2], (R)ls[3]};
            R cE[4], cB[6];
            gather_coeffs<K, R>(s_e[lt], s_b[lt], lam, cE, cB);
            R E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
#pragma unroll
            for (int f = 0; f < 4; f++)
#pragma unroll
                for (int c = 0; c < 3; c++) E[c] += cE[f] * (R)s_geo[lt][4 * f + 1 + c];
#pragma unroll
            for (int q = 0; q < 6; q++)
#pragma unroll
                for (int c = 0; c < 3; c++) B[c] += cB[q] * s_X[lt][3 * q + c];
            double dv[3], vn[3];
            double dp[4][3];
            if constexpr (!BORIS) {
                // Lorentz acceleration (precision R); AB4 velocity increment in R added to the FP64 velocity
                R vxB[3], a[3];
                cross3(v, B, vxB);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    a[c] = qmR * (E[c] + vxB[c]);
                    dv[c] = (double)(dtR / R(24) * (R(55) * a[c] - R(59) * ah[c] + R(37) * ah[3 + c] - R(9) * ah[6 + c]));
                    vn[c] = vd[c] + dv[c];
                }
                // quartic path r(s) = r^n + sum_{d=1..4} dp_d s^d (FP64 in both modes);
                // the history holds v^{n-j} - v^n, so in R it is rounded relative to
                // the change of velocity, not to the velocity
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const double v0 = vd[c], v1 = vd[c] + (double)vh[c], v2 = vd[c] + (double)vh[3 + c],
                                 v3 = vd[c] + (double)vh[6 + c];
#pragma unroll
                    for (int d = 1; d < 5; d++)
                        dp[d - 1][c] =
                            sp.dt * (LCOEF[0][d] * v0 + LCOEF[1][d] * v1 + LCOEF[2][d] * v2 + LCOEF[3][d] * v3);
                }
                // new velocity and shifted histories, written now (wall reflections patch them)
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    *out.v(c, i) = vn[c];
                    *out.vh(c, i) = (R)(-dv[c]);
                    *out.vh(3 + c, i) = (R)((double)vh[c] - dv[c]);
                    *out.vh(6 + c, i) = (R)((double)vh[3 + c] - dv[c]);
                    *out.ah(c, i) = a[c];
                    *out.ah(3 + c, i) = ah[c];
                    *out.ah(6 + c, i) = ah[3 + c];
                }
            } else {
                // Boris: half kick, rotation about B through 2 atan(q |B| dt / 2m), half
                // kick (precision R); the change of velocity added to the FP64 velocity
                const R h = R(0.5) * qmR * dtR;
                R t[3], sv[3], vm[3], vp[3], cr[3];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    t[c] = h * B[c];
                    vm[c] = v[c] + h * E[c];
                }
                const R f = R(2) / (R(1) + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
#pragma unroll
                for (int c = 0; c < 3; c++) sv[c] = f * t[c];
                cross3(vm, t, cr);
#pragma unroll
                for (int c = 0; c < 3; c++) vp[c] = vm[c] + cr[c];
                cross3(vp, sv, cr);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    // v^{n+1/2} - v^{n-1/2} = 2 h E + vp x s: formed as the change itself,
                    // so that in R it is rounded relative to the change, not to v
                    dv[c] = (double)(R(2) * h * E[c] + cr[c]);
                    vn[c] = vd[c] + dv[c];
                    // straight path r(s) = r^n + s dt v^{n+1/2}
                    dp[0][c] = sp.dt * vn[c];
                    dp[1][c] = dp[2][c] = dp[3][c] = 0.0;
                    *out.v(c, i) = vn[c];
                }
            }
            *out.id(i) = *in.id(slot);
            // first segment: in the home tet from s = 0.  A path whose exit
            // needs the full search is handed whole to k_continue; a path that
            // leaves is handed over at its exit point (the crossing itself is
            // done there).
            const double *G = &s_geo[lt][0];
            double s_exit;
            const int f_exit = fast_exit<true>(G, dp, ls, 0.0, -1, s_exit);
            // queued paths of the wave go to the start of the wave's own particle
            // range (its active lanes are a prefix of the wave), in lane order
            const unsigned long long qmask = __ballot(f_exit != -1);
            const int lane = tid & 63;
            qflag[i] = lane < __popcll(qmask) ? 1 : 0;
            qmoved[i] = f_exit != -1 ? 1 : 0;
            {
                // the first lane of each tet in the wave counts the tet's staying lanes
                const unsigned long long st = __ballot(f_exit == -1);
                const int wb = i - lane;
                const int lo = max(s_off[lt] - wb, 0);
                if (lane == lo) atomicAdd(&s_nstay[lt], __popcll(st & lane_range(lo, s_off[lt + 1] - wb)));
            }
            const int64_t qi = (int64_t)(i - lane) + __popcll(qmask & ((1ull << lane) - 1ull));
            const gptr<ContRec> rec = qrec + qi;
            if (f_exit != -1) {
#pragma unroll
                for (int d = 0; d < 4; d++)
#pragma unroll
                    for (int c = 0; c < 3; c++) rec->dp[3 * d + c] = dp[d][c];
                rec->s_lo = f_exit >= 0 ? s_exit : 0.0;
                rec->i = i;
                // an exit into a neighbour is crossed here (below), one into a wall
                // is left pending to k_continue
                const int nx = f_exit >= 0 ? s_nbr[lt][f_exit] : -1;
                rec->t = nx >= 0 ? nx >> 2 : th;
                rec->entry = nx >= 0 ? nx & 3 : -1;
                rec->ncross = nx >= 0 ? 1 : 0;
                rec->pending = f_exit >= 0 && nx < 0 ? f_exit : -1;
            }
            double lq[3][5];  // l_1..l_3 along the path in the home tet
            if (f_exit != -2) {
#pragma unroll
                for (int mm = 1; mm < 4; mm++) face_poly<true>(G, mm, dp, 0.0, ls[mm], lq[mm - 1]);
            }
            if (f_exit != -1) {
                // coordinates where k_continue takes the path up: the exit point, or
                // the start for a path handed over whole
                double le[4];
#pragma unroll
                for (int c = 0; c < 3; c++) le[c + 1] = f_exit >= 0 ? horner4(lq[c], s_exit) : ls[c + 1];
                const int nx = f_exit >= 0 ? s_nbr[lt][f_exit] : -1;
                if (nx >= 0) {
                    // the crossing into the neighbour: the three shared vertices keep
                    // their coordinates, listed in the same order in both tets, and
                    // the neighbour's vertex across the face starts at 0
                    le[0] = bary0(le[1], le[2], le[3]);
                    const int e = nx & 3;
                    const double s0 = f_exit == 0 ? le[1] : le[0];
                    const double s1 = f_exit <= 1 ? le[2] : le[1];
                    const double s2 = f_exit <= 2 ? le[3] : le[2];
                    le[1] = e == 0 ? s0 : (e == 1 ? 0.0 : s1);
                    le[2] = e <= 1 ? s1 : (e == 2 ? 0.0 : s2);
                    le[3] = e <= 2 ? s2 : 0.0;
                }
#pragma unroll
                for (int c = 0; c < 3; c++) rec->lam[c] = le[c + 1];
            } else {
#pragma unroll
                for (int c = 0; c < 3; c++) *out.lam(c, i) = horner4(lq[c], 1.0);
                *out.tet(i) = th;
            }
            if (f_exit != -2) {
                const double s_hi = f_exit < 0 ? 1.0 : s_exit;
                if (s_hi > 0.0) {
                    double dep[N1];
                    segment_moments<K, 0, N1, BORIS>(lq, s_hi, sp.qw, gl, dep);
#pragma unroll
                    for (int c = 0; c < N1; c++) s_hc[c][tid] = dep[c];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NP; q++) {
            const int pr = tid + q * PBLK;
            if (pr < ntl * N1) {
                // fixed order: four interleaved partial sums, then (0+1)+(2+3)
                const int wt = pr / N1, wc = pr % N1;
                const int lo = max(s_off[wt], base) - base;
                const int hi = min(s_off[wt + 1], base + PBLK) - base;
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                int j = lo;
                for (; j + 3 < hi; j += 4) {
                    a0 += s_hc[wc][j];
                    a1 += s_hc[wc][j + 1];
                    a2 += s_hc[wc][j + 2];
                    a3 += s_hc[wc][j + 3];
                }
                if (j < hi) a0 += s_hc[wc][j];
                if (j + 1 < hi) a1 += s_hc[wc][j + 1];
                if (j + 2 < hi) a2 += s_hc[wc][j + 2];
                acc[q] += (a0 + a1) + (a2 + a3);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NP; q++) {
        const int pr = tid + q * PBLK;
        if (pr < ntl * N1) P[(int64_t)T0 * N1 + pr] = acc[q];
    }
    if (tid < ntl) glb(A->cq.nstay)[T0 + tid] = s_nstay[tid];
}

// Kernel 2: the rest of the paths of queued particles, segment by segment;
// every segment's current moments go to the spill pool tagged with
// (sorted particle, segment), so their reduction order is canonical.
template <int K, typename R, bool BORIS = false>
__global__ __launch_bounds__(BLK, 2) void k_continue(const ParticleArgs *__restrict__ A)
{
    const GMesh m = gview(A->m);
    const GParticles<R> out = gview<R>(A->out);
    const StepParams &sp = A->sp;
    const GLRule &gl = A->gl;
    const GPool pool = gview(A->pool);
    const gptr<ContRec> qrec = glb(A->cq.rec);
    const gptr<const int32_t> qidx = glb((const int32_t *)A->cq.idx);
    const gptr<unsigned long long> cntb = glb(A->cntb);
    constexpr int N1 = Ord<K>::N1;
    const int32_t nq = *glb(A->cq.count);
    const bool absorb = sp.absorb != 0;
    unsigned long long ncr = 0, nrf = 0, nsp = 0, nab = 0;
    int errs = 0;
    for (int64_t r = (int64_t)blockIdx.x * BLK + threadIdx.x; r < nq; r += (int64_t)gridDim.x * BLK) {
        const gptr<ContRec> rec = qrec + qidx[r];
        double s_lo = rec->s_lo;
        const int64_t i = rec->i;
        int t = rec->t, entry = rec->entry, ncross = rec->ncross, nsp_i = 0;
        const int pending = rec->pending;
        ncr += ncross;  // a crossing into a neighbour that k_particle made
        bool gone = false;  // absorbed at a wall
        if (pending >= 0) {
            // the exit found in the home tet: cross it now
            double dp[4][3], lam[4];
#pragma unroll
            for (int d = 0; d < 4; d++)
#pragma unroll
                for (int c = 0; c < 3; c++) dp[d][c] = rec->dp[3 * d + c];
            lam[1] = rec->lam[0];
            lam[2] = rec->lam[1];
            lam[3] = rec->lam[2];
            lam[0] = bary0(lam[1], lam[2], lam[3]);
            ncross++;
            ncr++;
            const unsigned long long nrf0 = nrf;
            gone = cross_face<R>(m, m.geo + (int64_t)t * 16, pending, t, entry, dp, lam, out, i, nrf, absorb,
                                 !BORIS);
#pragma unroll
            for (int c = 0; c < 3; c++) rec->lam[c] = lam[c + 1];
            if (nrf != nrf0) {
#pragma unroll
                for (int d = 0; d < 4; d++)
#pragma unroll
                    for (int c = 0; c < 3; c++) rec->dp[3 * d + c] = dp[d][c];
            }
            if (gone) nab++;
        }
        while (!gone) {
            // the path stays in the record between segments and is re-read here,
            // so that it is not held in registers through the deposit
            double dp[4][3], ls[4];
#pragma unroll
            for (int d = 0; d < 4; d++)
#pragma unroll
                for (int c = 0; c < 3; c++) dp[d][c] = rec->dp[3 * d + c];
            ls[1] = rec->lam[0];
            ls[2] = rec->lam[1];
            ls[3] = rec->lam[2];
            ls[0] = bary0(ls[1], ls[2], ls[3]);
            const gptr<const double> G = m.geo + (int64_t)t * 16;
            double s_exit;
            int f_exit = fast_exit<false>(G, dp, ls, s_lo, entry, s_exit);
            if (f_exit == -2) f_exit = find_exit<false>(G, dp, ls, s_lo, entry, s_exit);
            const double s_hi = f_exit < 0 ? 1.0 : s_exit;
            double lq[3][5];  // l_1..l_3 of this tet along the path from s_lo
#pragma unroll
            for (int mm = 1; mm < 4; mm++) face_poly<false>(G, mm, dp, s_lo, ls[mm], lq[mm - 1]);
            const int t_seg = t;
            const bool crossing = f_exit >= 0 && ncross < MAX_CROSS;
            bool more = false;
            {
                // coordinates at the segment's end: the exit point, handed to the
                // next tet, or the end of the path
                double le[4];
#pragma unroll
                for (int c = 0; c < 3; c++) le[c + 1] = horner4(lq[c], (crossing ? s_exit : 1.0) - s_lo);
                le[0] = bary0(le[1], le[2], le[3]);
                if (crossing) {
                    ncross++;
                    ncr++;
                    // the path again from the record (a wall mirrors it), not held
                    // in registers since the exit search
                    asm volatile("" ::: "memory");
                    double dq[4][3];
#pragma unroll
                    for (int d = 0; d < 4; d++)
#pragma unroll
                        for (int c = 0; c < 3; c++) dq[d][c] = rec->dp[3 * d + c];
                    const unsigned long long nrf0 = nrf;
                    gone = cross_face<R>(m, G, f_exit, t, entry, dq, le, out, i, nrf, absorb, !BORIS);
#pragma unroll
                    for (int c = 0; c < 3; c++) rec->lam[c] = le[c + 1];
                    if (nrf != nrf0) {  // a wall reflection changed the path
#pragma unroll
                        for (int d = 0; d < 4; d++)
#pragma unroll
                            for (int c = 0; c < 3; c++) rec->dp[3 * d + c] = dq[d][c];
                    }
                    more = !gone;
                    if (gone) nab++;
                } else {
                    if (f_exit >= 0) errs |= ERR_CROSS;
#pragma unroll
                    for (int c = 0; c < 3; c++) *out.lam(c, i) = le[c + 1];
                    if (!(le[1] == le[1] && le[2] == le[2] && le[3] == le[3])) errs |= ERR_NAN;
                    *out.tet(i) = t;
                }
            }
            asm volatile("" ::: "memory");
            // every path's last segment has a record, also of zero length: it
            // names the tet the particle ends in (an absorbed particle's segment
            // up to the wall is not a last one: the particle is not placed again)
            const bool last = !more && !gone;
            if (s_hi > s_lo || last) {
                const int64_t slot = spill_slot(pool, r, nq, t_seg, last, i, nsp_i, errs);
                if (slot >= 0) {
                    double dep[N1];
                    segment_moments<K, 0, N1, BORIS>(lq, fmax(s_hi - s_lo, 0.0), sp.qw, gl, dep);
                    const gptr<double> dst = pool.val + slot * N1;
#pragma unroll
                    for (int c = 0; c < N1; c++) dst[c] = dep[c];
                }
            }
            if (!more) break;
            s_lo = s_exit;
        }
        // fixed slots left unused are marked empty
        for (int j = nsp_i; j < 2; j++)
            if (2 * r + j < pool.cap) pool.tag[2 * r + j] = -1;
        nsp += nsp_i;
        pool.rcount[r] = nsp_i;
    }
    block_counters(cntb, ncr, nrf, nsp, errs, nab);
}

// step counters: sum (or, for the error flags) of the per-block counters
// (integer sums: exact in any order)
__global__ __launch_bounds__(BLK) void k_counters(const unsigned long long *__restrict__ cntb, int nb,
                                                  unsigned long long *__restrict__ cnt)
{
    __shared__ unsigned long long s_v[NCNT][BLK];
    unsigned long long v[NCNT] = {};
    for (int b = blockIdx.x * BLK + threadIdx.x; b < nb; b += gridDim.x * BLK)
        for (int k = 0; k < NCNT; k++)
            v[k] = k == CNT_ERR ? (v[k] | cntb[b * NCNT + k]) : v[k] + cntb[b * NCNT + k];
    for (int k = 0; k < NCNT; k++) s_v[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = BLK / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < NCNT; k++)
                s_v[k][threadIdx.x] = k == CNT_ERR ? (s_v[k][threadIdx.x] | s_v[k][threadIdx.x + h])
                                                   : s_v[k][threadIdx.x] + s_v[k][threadIdx.x + h];
        __syncthreads();
    }
    // integer sums (and the error bits' or): exact in any order, so the
    // workgroups add theirs atomically
    if (threadIdx.x < NCNT) {
        const int k = threadIdx.x;
        if (k == CNT_ERR) atomicOr(&cnt[k], s_v[k][0]);
        else atomicAdd(&cnt[k], s_v[k][0]);
    }
}

// compacted list of the queued record slots: idx[pos[i]] = i where flag[i]
// Queue compaction: the slots whose byte flag is set, in increasing order, in
// two passes over tiles of QTILE flags (16 per thread): per-tile counts, then,
// after a scan of the counts, each tile writes its slots from its offset.
constexpr int QT_ITEMS = 16;
constexpr int QTILE = BLK * QT_ITEMS;

// the 16 flags from base as bits (flags are 0 or 1; those at n and beyond read as 0)
__device__ inline uint32_t flag_bits16(const uint8_t *__restrict__ flag, int64_t base, int64_t n)
{
    uint32_t b = 0;
    if (base + QT_ITEMS <= n) {
        const uint4 u = *(const uint4 *)(flag + base);
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int k = 0; k < 4; k++) b |= ((w[q] >> (8 * k)) & 1u) << (4 * q + k);
    } else {
        for (int k = 0; k < QT_ITEMS; k++)
            if (base + k < n && flag[base + k]) b |= 1u << k;
    }
    return b;
}

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_w, uint32_t &total);

__global__ __launch_bounds__(BLK) void k_flag_count(const uint8_t *__restrict__ flag, int64_t n,
                                                    uint32_t *__restrict__ tsum)
{
    __shared__ uint32_t s_w[BLK / 64];
    const int64_t base = (int64_t)blockIdx.x * QTILE + (int64_t)threadIdx.x * QT_ITEMS;
    uint32_t tot;
    block_exclusive_scan((uint32_t)__popc(flag_bits16(flag, base, n)), s_w, tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(BLK) void k_flag_compact(const uint8_t *__restrict__ flag, int64_t n,
                                                      const uint32_t *__restrict__ tpos, int32_t *__restrict__ idx)
{
    __shared__ uint32_t s_w[BLK / 64];
    const int64_t base = (int64_t)blockIdx.x * QTILE + (int64_t)threadIdx.x * QT_ITEMS;
    uint32_t b = flag_bits16(flag, base, n), tot;
    uint32_t pos = tpos[blockIdx.x] + block_exclusive_scan((uint32_t)__popc(b), s_w, tot);
    while (b) {
        const int k = __builtin_ctz(b);
        b &= b - 1u;
        idx[pos++] = (int32_t)(base + k);
    }
}

// ------------------------------------------------------------ permute
template <int NW>
__global__ void k_permute(DevParticles in, DevParticles out, const uint32_t *__restrict__ perm, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    typedef unsigned int word __attribute__((ext_vector_type(4)));  // one 16-byte word
    const gptr<const word> a = glb((const word *)in.w);
    const gptr<word> b = glb((word *)out.w);
#pragma unroll
    for (int k = 0; k < NW; k++) b[k * out.cap + i] = a[k * in.cap + j];
}

__global__ void k_tet_keys(DevParticles p, int64_t n, uint32_t *__restrict__ keys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = (uint32_t)*(const int32_t *)((const char *)p.w + part_off(PART_MIXED.tet, p.cap, i));
}

// ----------------------------------------------------------- radix sort
// element count of a launch sized on the host for n: the count at dn when
// given (a device value the host has not read), else n
__device__ inline int64_t dev_count(int64_t n, const int32_t *dn)
{
    return dn ? min(n, (int64_t)max(*dn, 0)) : n;
}

constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = BLK * RS_ITEMS;

__global__ __launch_bounds__(BLK) void k_rs_hist(const uint32_t *__restrict__ key, int64_t n, int shift,
                                                 uint32_t *__restrict__ hist, int64_t ntiles,
                                                 const int32_t *__restrict__ dn)
{
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    n = dev_count(n, dn);
    h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
    for (int r = 0; r < RS_ITEMS; r++) {
        int64_t idx = base + r * BLK + tid;
        if (idx < n) atomicAdd(&h[(key[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
}

__global__ __launch_bounds__(BLK) void k_rs_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                    uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n,
                                                    int shift, const uint32_t *__restrict__ offs, int64_t ntiles,
                                                    int iota, const int32_t *__restrict__ dn)
{
    __shared__ uint32_t run[256];
    n = dev_count(n, dn);
    __shared__ uint32_t wcnt[BLK / 64][256];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    run[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int r = 0; r < RS_ITEMS; r++) {
#pragma unroll
        for (int q = 0; q < BLK / 64; q++) wcnt[q][tid] = 0;
        __syncthreads();
        const int64_t idx = base + r * BLK + tid;
        const bool valid = idx < n;
        const uint32_t k = valid ? kin[idx] : 0u;
        const uint32_t d = (k >> shift) & 255u;
        unsigned long long match = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; bit++) {
            const bool on = (d >> bit) & 1u;
            const unsigned long long bb = __ballot(valid && on);
            match &= on ? bb : ~bb;
        }
        const int rank = __popcll(match & lt);
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(match);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + (uint32_t)rank;
            for (int q = 0; q < w; q++) pos += wcnt[q][d];
            kout[pos] = k;
            vout[pos] = iota ? (uint32_t)idx : vin[idx];
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int q = 0; q < BLK / 64; q++) add += wcnt[q][tid];
        run[tid] += add;
        __syncthreads();
    }
}

// ----------------------------------------------------------------- scan
constexpr int SC_THREADS = 1024;
constexpr int SC_ITEMS = 4;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;
// up to this many tiles a scan adds the tile sums per tile directly (each
// workgroup reads at most this many sums) instead of scanning them first
constexpr int64_t SCAN_DIRECT_TILES = 4096;

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_w, uint32_t &total)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    if (w == 0) {
        const int nw = blockDim.x / 64;
        uint32_t t = lane < nw ? s_w[lane] : 0u;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(t, o);
            if (lane >= o) t += y;
        }
        if (lane < nw) s_w[lane] = t;
    }
    __syncthreads();
    const uint32_t wprefix = w > 0 ? s_w[w - 1] : 0u;
    total = s_w[blockDim.x / 64 - 1];
    __syncthreads();
    return wprefix + x - v;
}

__global__ __launch_bounds__(SC_THREADS) void k_scan_tile(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                          int64_t n, uint32_t *__restrict__ sums,
                                                          const int32_t *__restrict__ dn)
{
    __shared__ uint32_t s_w[SC_THREADS / 64];
    n = dev_count(n, dn);
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
    uint32_t v[SC_ITEMS], s = 0;
#pragma unroll
    for (int k = 0; k < SC_ITEMS; k++) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(s, s_w, tot);
#pragma unroll
    for (int k = 0; k < SC_ITEMS; k++) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0 && sums) sums[blockIdx.x] = tot;
}

// a single-tile scan that also writes the total
__global__ __launch_bounds__(SC_THREADS) void k_scan_tile1(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                           int64_t n, uint32_t *__restrict__ total,
                                                           const int32_t *__restrict__ dn)
{
    __shared__ uint32_t s_w[SC_THREADS / 64];
    n = dev_count(n, dn);
    const int64_t base = (int64_t)threadIdx.x * SC_ITEMS;
    uint32_t v[SC_ITEMS], s = 0;
#pragma unroll
    for (int k = 0; k < SC_ITEMS; k++) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(s, s_w, tot);
#pragma unroll
    for (int k = 0; k < SC_ITEMS; k++) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

__global__ void k_scan_add(uint32_t *__restrict__ out, int64_t n, const uint32_t *__restrict__ sums,
                           const int32_t *__restrict__ dn)
{
    n = dev_count(n, dn);
    const int64_t base = (int64_t)blockIdx.x * SC_TILE;
    const uint32_t add = sums[blockIdx.x];
    for (int k = threadIdx.x; k < SC_TILE; k += blockDim.x)
        if (base + k < n) out[base + k] += add;
}

// the same for few tiles, without a scan of the tile sums: each workgroup adds
// up the sums of the tiles before it; the last one also writes the total
__global__ __launch_bounds__(BLK) void k_scan_add_direct(uint32_t *__restrict__ out, int64_t n,
                                                         const uint32_t *__restrict__ sums,
                                                         uint32_t *__restrict__ total, const int32_t *__restrict__ dn)
{
    __shared__ uint32_t s_w[BLK / 64];
    n = dev_count(n, dn);
    uint32_t a = 0;
    for (int64_t k = threadIdx.x; k < (int64_t)blockIdx.x; k += BLK) a += sums[k];
    uint32_t add;
    (void)block_exclusive_scan(a, s_w, add);
    const int64_t base = (int64_t)blockIdx.x * SC_TILE;
    for (int k = threadIdx.x; k < SC_TILE; k += BLK)
        if (base + k < n) out[base + k] += add;
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = add + sums[blockIdx.x];
}

__global__ void k_scan_total(const uint32_t *__restrict__ in, const uint32_t *__restrict__ out, int64_t n,
                             uint32_t *__restrict__ total, const int32_t *__restrict__ dn)
{
    n = dev_count(n, dn);
    *total = n > 0 ? out[n - 1] + in[n - 1] : 0u;
}

// ------------------------------------------------------------- offsets
__global__ void k_offsets(const uint32_t *__restrict__ key, int64_t n, int32_t nt, int32_t *__restrict__ off,
                          const int32_t *__restrict__ dn)
{
    n = dev_count(n, dn);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n == 0) {
        for (int64_t t = i; t <= nt; t += (int64_t)gridDim.x * blockDim.x) off[t] = 0;
        return;
    }
    if (i >= n) return;
    // keys are tets; the clamp keeps the writes inside off whatever the keys hold
    const int64_t k = min((int64_t)key[i], (int64_t)nt);
    const int64_t kp = i == 0 ? -1 : min((int64_t)key[i - 1], (int64_t)nt);
    for (int64_t t = kp + 1; t <= k; t++) off[t] = (int32_t)i;
    if (i == n - 1)
        for (int64_t t = k + 1; t <= nt; t++) off[t] = (int32_t)n;
}

// ------------------------------------------------------------- spills
__global__ void k_spill_compact(const int32_t *__restrict__ ptet, const int64_t *__restrict__ ptag, int64_t nrec,
                                const uint32_t *__restrict__ pos, uint32_t *__restrict__ key, uint32_t *__restrict__ val,
                                const int32_t *__restrict__ nq, const int32_t *__restrict__ nappend, int64_t kcap)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // slots in use: the fixed pair of each queued record, then the appended ones
    if (nq) nrec = min(nrec, 2 * (int64_t)max(*nq, 0) + max(*nappend, 0));
    if (r >= nrec) return;
    const int64_t tag = ptag[r];
    if (tag < 0) return;  // unused fixed slot
    const int64_t q = tag >> 8;
    const int j = (int)(tag & 127);
    const uint32_t dst = pos[q] + (uint32_t)j;
    if (dst >= kcap) return;  // only when the pool overflowed (the step is redone)
    key[dst] = (uint32_t)ptet[r];
    val[dst] = (uint32_t)r | ((tag >> 7) & 1 ? SREC_LAST : 0u);
}

template <int N1>
__global__ void k_spill_reduce(int32_t nt, const int32_t *__restrict__ soff, const uint32_t *__restrict__ rec,
                               const double *__restrict__ recval, int64_t cap, double *__restrict__ P,
                               const int32_t *__restrict__ nstay, uint32_t *__restrict__ cnt)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)nt * N1) return;
    const int64_t t = g / N1;
    const int c = (int)(g % N1);
    const int32_t lo = soff[t], hi = soff[t + 1];
    // fixed order: four interleaved partial sums, then (0+1)+(2+3), added to the
    // home sum; the last-segment records are counted on the way
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int32_t narr = 0;
    // (slots are below cap in a valid step; the clamp keeps any other inside the pool)
    auto slot = [&](uint32_t v) { return min((int64_t)(v & ~SREC_LAST), cap - 1); };
    int32_t k = lo;
    for (; k + 3 < hi; k += 4) {
        const uint32_t v0 = rec[k], v1 = rec[k + 1], v2 = rec[k + 2], v3 = rec[k + 3];
        narr += (int32_t)((v0 >> 31) + (v1 >> 31) + (v2 >> 31) + (v3 >> 31));
        a0 += recval[slot(v0) * N1 + c];
        a1 += recval[slot(v1) * N1 + c];
        a2 += recval[slot(v2) * N1 + c];
        a3 += recval[slot(v3) * N1 + c];
    }
    for (int q = 0; q < 3 && k + q < hi; q++) {
        const uint32_t v = rec[k + q];
        narr += (int32_t)(v >> 31);
        const double x = recval[slot(v) * N1 + c];
        if (q == 0) a0 += x;
        else if (q == 1) a1 += x;
        else a2 += x;
    }
    // size of tet t's bucket in the next particle order
    if (cnt && c == 0) cnt[t] = (uint32_t)(nstay[t] + narr);
    if (lo == hi) return;
    P[g] += (a0 + a1) + (a2 + a3);
}

// Next step's particle order (see launch_place), one block per tet range of
// the particle kernel's partition.  Two passes place items in order within
// each tet: first the tets' particles that stayed (items: old positions, tet
// ranges off), then their arrivals (items: sorted spill records, tet ranges
// soff, the last-segment ones).  An item goes to its tet's next place: its
// rank among the tet's placed items, from earlier chunks (a per-tet carry in
// LDS), earlier waves and lower lanes of its chunk (wave ballots).
constexpr int PLACE_TPW_MAX = PARTICLE_TPW_MAX_1 > PARTICLE_TPW_MAX_2 ? PARTICLE_TPW_MAX_1 : PARTICLE_TPW_MAX_2;
__global__ __launch_bounds__(BLK) void k_place(int32_t nt, int32_t tpw, const int32_t *__restrict__ off,
                                               const int32_t *__restrict__ noff, const uint8_t *__restrict__ moved,
                                               const int32_t *__restrict__ soff, const uint32_t *__restrict__ srec,
                                               int64_t nrec, const int32_t *__restrict__ pid, int64_t pool_cap,
                                               int64_t np, uint32_t *__restrict__ perm,
                                               unsigned long long *__restrict__ err)
{
    __shared__ int32_t s_off[PLACE_TPW_MAX + 1], s_soff[PLACE_TPW_MAX + 1], s_noff[PLACE_TPW_MAX + 1];
    __shared__ int32_t s_carry[PLACE_TPW_MAX];
    __shared__ unsigned long long s_mask[2][BLK / 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int T0 = blockIdx.x * tpw, ntl = min(T0 + tpw, nt) - T0;
    for (int k = tid; k <= ntl; k += BLK) {
        s_off[k] = off[T0 + k];
        s_noff[k] = noff[T0 + k];
        s_soff[k] = nrec > 0 ? soff[T0 + k] : 0;
    }
    for (int k = tid; k < ntl; k += BLK) s_carry[k] = 0;
    __syncthreads();
    int par = 0;
    auto pass = [&](const int32_t *R, auto sel, auto value) {
        for (int base = R[0]; base < R[ntl]; base += BLK) {
            const int j = base + tid;
            const bool on = j < R[ntl] && sel(j);
            const unsigned long long mk = __ballot(on);
            if (lane == 0) s_mask[par][wv] = mk;
            __syncthreads();
            if (on) {
                // j's tet: the last one whose range starts at or before j
                int lo = 0, hi = ntl;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (R[mid] <= j) lo = mid;
                    else hi = mid;
                }
                const int tb = R[lo] - base, te = R[lo + 1] - base;
                int rk = s_carry[lo];
                for (int w2 = 0; w2 < wv; w2++) rk += __popcll(s_mask[par][w2] & lane_range(tb - 64 * w2, te - 64 * w2));
                rk += __popcll(mk & lane_range(tb - 64 * wv, lane));
                const int64_t dst = (int64_t)s_noff[lo] + rk;
                if (dst < s_noff[lo + 1] && dst < np) perm[dst] = value(j);
            }
            __syncthreads();
            if (tid < ntl) {
                const int tb = R[tid] - base, te = R[tid + 1] - base;
                int c = 0;
#pragma unroll
                for (int w2 = 0; w2 < BLK / 64; w2++) c += __popcll(s_mask[par][w2] & lane_range(tb - 64 * w2, te - 64 * w2));
                s_carry[tid] += c;
            }
            par ^= 1;
        }
    };
    pass(s_off, [&](int j) { return moved[j] == 0; }, [&](int j) { return (uint32_t)j; });
    if (nrec > 0)
        pass(s_soff, [&](int k) { return (srec[k] & SREC_LAST) != 0; },
             [&](int k) { return (uint32_t)pid[min((int64_t)(srec[k] & ~SREC_LAST), pool_cap - 1)]; });
    // every tet's bucket is full (the carries were last updated by these threads)
    if (tid < ntl && s_carry[tid] != s_noff[tid + 1] - s_noff[tid]) *err = 1;
    if (blockIdx.x == 0 && tid == 0 && noff[nt] > np) *err = 1;
}

__global__ void k_scatter(const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx, int64_t n,
                          const double *__restrict__ P, double *__restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    const int64_t e = ptr[j + 1];
    int64_t k = ptr[j];
    // four entries' loads issued together, added in the same order as one at a time
    for (; k + 3 < e; k += 4) {
        int32_t i4[4];
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) i4[u] = idx[k + u];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = P[i4[u]];
#pragma unroll
        for (int u = 0; u < 4; u++) s += v[u];
    }
    for (; k < e; k++) s += P[idx[k]];
    out[j] = s;
}

// nodal charge per tet (order-k W0 values times q w), same tiling as k_particle
template <int K>
__global__ __launch_bounds__(BLK) void k_rho_tet(DevMesh m, const uint32_t *__restrict__ perm,
                                                 const int32_t *__restrict__ off, DevParticles P, double qw, int tpw,
                                                 double *__restrict__ Pr)
{
    using O = Ord<K>;
    constexpr int N0 = O::N0;
    __shared__ double s_w[N0][BLK + 1];
    __shared__ int32_t s_off[BLK / N0 + 2];
    const int tid = threadIdx.x;
    const int T0 = blockIdx.x * tpw;
    const int T1 = min(T0 + tpw, m.nt);
    const int ntl = T1 - T0;
    for (int k = tid; k <= ntl; k += BLK) s_off[k] = off[T0 + k];
    __syncthreads();
    const int pbeg = s_off[0], pend = s_off[ntl];
    const int wt = tid / N0, wc = tid % N0;
    const bool worker = tid < ntl * N0;
    double acc = 0.0;
    for (int base = pbeg; base < pend; base += BLK) {
        const int i = base + tid;
        if (i < pend) {
            const uint32_t slot = perm[i];
            double l[4];
            l[1] = *prow_lam(P, 0, slot);
            l[2] = *prow_lam(P, 1, slot);
            l[3] = *prow_lam(P, 2, slot);
            l[0] = bary0(l[1], l[2], l[3]);
            if constexpr (K == 1) {
                for (int f = 0; f < 4; f++) s_w[f][tid] = qw * l[f];
            } else {
                for (int f = 0; f < 4; f++) s_w[f][tid] = qw * (l[f] * (2.0 * l[f] - 1.0));
                for (int q = 0; q < 6; q++) s_w[4 + q][tid] = qw * (2.0 * l[EA[q]] * l[EB[q]]);
            }
        }
        __syncthreads();
        if (worker) {
            const int lo = max(s_off[wt], base) - base;
            const int hi = min(s_off[wt + 1], base + BLK) - base;
            for (int j = lo; j < hi; j++) acc += s_w[wc][j];
        }
        __syncthreads();
    }
    if (worker) Pr[(int64_t)(T0 + wt) * N0 + wc] = acc;
}

// --------------------------------------------------------- linear algebra
// Reductions are deterministic: every block sums a fixed set of rows in a fixed
// order, and k_finish sums the (at most RED_BLOCKS) block partials in order.
constexpr int RED_BLOCKS = 2048;

// blocks (2x2 SpMV) or entries (CSR SpMV) per lane whose loads are issued together
constexpr int BSPMV_U = 2;

// y = alpha A x + beta z (CSR), LANES lanes per row; optional fused partial
// dot(dotv, y) per workgroup (fixed order).  Loads are grouped as in k_bspmv:
// each lane takes its entries k = start + lane, start + lane + LANES, ... in
// that order, BSPMV_U of them requested together.
template <int LANES, typename T>
__global__ __launch_bounds__(BLK) void k_spmv(int64_t rows, const int64_t *__restrict__ ptr,
                                              const int32_t *__restrict__ idx, const T *__restrict__ val,
                                              const T *__restrict__ x, T *__restrict__ y, double alpha, double beta,
                                              const T *__restrict__ z, const T *__restrict__ dotv,
                                              double *__restrict__ partial)
{
    __shared__ double s_red[BLK / LANES];
    constexpr int RPB = BLK / LANES;
    constexpr int U = BSPMV_U;
    const int tid = threadIdx.x;
    const int lane = tid % LANES;
    const int64_t stride = (int64_t)gridDim.x * RPB;
    double d = 0.0;
    int64_t row = (int64_t)blockIdx.x * RPB + tid / LANES;
    int64_t kb = 0, ke = 0;
    if (row < rows) {
        kb = ptr[row];
        ke = ptr[row + 1];
    }
    for (int64_t row0 = (int64_t)blockIdx.x * RPB; row0 < rows; row0 += stride, row += stride) {
        const int64_t e = ke;
        int64_t k0 = kb + lane;
        if (row + stride < rows) {
            kb = ptr[row + stride];
            ke = ptr[row + stride + 1];
        }
        const bool wr = row < rows && lane == 0;
        T z0 = 0, w0 = 0;
        if (wr && beta != 0.0) z0 = z[row];
        if (wr && dotv) w0 = dotv[row];
        double sum = 0.0;
        if (row < rows) {
            for (; k0 < e; k0 += U * LANES) {
                // lanes past the row's end load its last entry again and do not add it
                int32_t c[U];
                T v[U], xv[U];
#pragma unroll
                for (int u = 0; u < U; u++) c[u] = idx[min(k0 + u * LANES, e - 1)];
#pragma unroll
                for (int u = 0; u < U; u++) v[u] = val[min(k0 + u * LANES, e - 1)];
#pragma unroll
                for (int u = 0; u < U; u++) xv[u] = x[c[u]];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const double t = fma((double)v[u], (double)xv[u], sum);
                    sum = k0 + u * LANES < e ? t : sum;
                }
            }
        }
#pragma unroll
        for (int o = LANES / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, LANES);
        if (wr) {
            // keeps the conversions of z0 and w0 (and the wait for them) here
            asm volatile("" : "+v"(z0), "+v"(w0));
            const double yv = alpha * sum + (beta != 0.0 ? beta * (double)z0 : 0.0);
            y[row] = (T)yv;
            if (dotv) d += (double)w0 * (double)(T)yv;
        }
    }
    if (partial) {
        if (lane == 0) s_red[tid / LANES] = d;
        __syncthreads();
        for (int o = RPB / 2; o > 0; o >>= 1) {
            if (tid < o) s_red[tid] += s_red[tid + o];
            __syncthreads();
        }
        if (tid == 0) partial[blockIdx.x] = s_red[0];
    }
}

// y = alpha A x + beta z with A in 2x2 blocks: LANES lanes per block row, a
// block's four values and the two x entries it needs are loaded as vectors;
// optional fused partial dot(dotv, y) per workgroup (fixed order).  Rows go to
// the blocks in a grid stride, so at any time the GPU works on one compact
// window of rows and the x entries it references stay in every XCD's L2.
// Each lane takes its blocks k = start + lane, start + lane + LANES, ... in
// that order; BSPMV_U of them are requested together (indices, then values,
// then x entries), and the next row's bounds are read one row ahead.
template <int LANES, typename T>
__global__ __launch_bounds__(BLK) void k_bspmv(int64_t brows, const int64_t *__restrict__ bptr,
                                               const int32_t *__restrict__ bidx, const T *__restrict__ bval,
                                               const T *__restrict__ x, T *__restrict__ y, double alpha, double beta,
                                               const T *__restrict__ z, const T *__restrict__ dotv,
                                               double *__restrict__ partial)
{
    __shared__ double s_red[BLK / LANES];
    constexpr int RPB = BLK / LANES;
    constexpr int U = BSPMV_U;
    const int tid = threadIdx.x;
    const int lane = tid % LANES;
    const int64_t stride = (int64_t)gridDim.x * RPB;
    double d = 0.0;
    int64_t br = (int64_t)blockIdx.x * RPB + tid / LANES;
    int64_t kb = 0, ke = 0;
    if (br < brows) {
        kb = bptr[br];
        ke = bptr[br + 1];
    }
    for (int64_t row0 = (int64_t)blockIdx.x * RPB; row0 < brows; row0 += stride, br += stride) {
        const int64_t e = ke;
        int64_t k0 = kb + lane;
        if (br + stride < brows) {
            kb = bptr[br + stride];
            ke = bptr[br + stride + 1];
        }
        // the row's z and dotv entries, requested before its products
        const bool wr = br < brows && lane == 0;
        T z0 = 0, z1 = 0, w0 = 0, w1 = 0;
        if (wr && beta != 0.0) {
            z0 = z[2 * br];
            z1 = z[2 * br + 1];
        }
        if (wr && dotv) {
            w0 = dotv[2 * br];
            w1 = dotv[2 * br + 1];
        }
        double s0 = 0.0, s1 = 0.0;
        if (br < brows) {
            for (; k0 < e; k0 += U * LANES) {
                // lanes past the row's end load its last block again (in
                // bounds, same lines) and do not add it
                int64_t c[U];
                T v[U][4], xv[U][2];
#pragma unroll
                for (int u = 0; u < U; u++) c[u] = 2 * (int64_t)bidx[min(k0 + u * LANES, e - 1)];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int64_t k = min(k0 + u * LANES, e - 1);
#pragma unroll
                    for (int j = 0; j < 4; j++) v[u][j] = bval[4 * k + j];
                }
#pragma unroll
                for (int u = 0; u < U; u++) {
                    xv[u][0] = x[c[u]];
                    xv[u][1] = x[c[u] + 1];
                }
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const bool in = k0 + u * LANES < e;
                    const double x0 = (double)xv[u][0], x1 = (double)xv[u][1];
                    const double t0 = fma((double)v[u][0], x0, fma((double)v[u][1], x1, s0));
                    const double t1 = fma((double)v[u][2], x0, fma((double)v[u][3], x1, s1));
                    s0 = in ? t0 : s0;
                    s1 = in ? t1 : s1;
                }
            }
        }
#pragma unroll
        for (int o = LANES / 2; o > 0; o >>= 1) {
            s0 += __shfl_xor(s0, o, LANES);
            s1 += __shfl_xor(s1, o, LANES);
        }
        if (wr) {
            // an empty statement that takes the four values here, so that their
            // conversions (and the wait for their loads) are not moved up
            asm volatile("" : "+v"(z0), "+v"(z1), "+v"(w0), "+v"(w1));
            const double y0 = alpha * s0 + (beta != 0.0 ? beta * (double)z0 : 0.0);
            const double y1 = alpha * s1 + (beta != 0.0 ? beta * (double)z1 : 0.0);
            y[2 * br] = (T)y0;
            y[2 * br + 1] = (T)y1;
            if (dotv) d += (double)w0 * (double)(T)y0 + (double)w1 * (double)(T)y1;
        }
    }
    if (partial) {
        if (lane == 0) s_red[tid / LANES] = d;
        __syncthreads();
        for (int o = RPB / 2; o > 0; o >>= 1) {
            if (tid < o) s_red[tid] += s_red[tid + o];
            __syncthreads();
        }
        if (tid == 0) partial[blockIdx.x] = s_red[0];
    }
}

// ------------------------------------------------ system operator, tet by tet
// The matrix of the implicit update (Sec. III-A, eq. (maxwell_semi); Sec. III-B),
// A = eps0 M1 + c S / mu0, applied without the assembled matrix.  In a tet,
// E = sum_j x_j W1_j = sum_m P_m(l) grad l_m, with P_m a homogeneous polynomial
// of degree K in the barycentric coordinates (every W1_j is (qc + qs l_v) times
// l_a grad l_b - l_b grad l_a, and l_a = l_a (l_0 + ... + l_3)).  Then
//   int_T E.E' = sum_{m,n} (grad l_m . grad l_n) int_T P_m P'_n,
//   curl E = sum_{n<m} (dP_m/dl_n - dP_n/dl_m) grad l_n x grad l_m,
// and the monomial integrals are exact: (1/V) int_T l^a = 6 a! / (|a| + 3)!
// (a! = a_0! a_1! a_2! a_3!).  The product A x is the derivative of the
// tet's energy, so it takes the transposes of the same linear maps.

// monomials of degree 2: (a, b), a <= b, in the order 00 01 02 03 11 12 13 22 23 33
__host__ __device__ constexpr int mono2(int a, int b)
{
    return a <= b ? a * 4 - a * (a - 1) / 2 + (b - a) : b * 4 - b * (b - 1) / 2 + (a - b);
}
__host__ __device__ constexpr int mono2_a(int u) { return u < 4 ? 0 : (u < 7 ? 1 : (u < 9 ? 2 : 3)); }
__host__ __device__ constexpr int mono2_b(int u) { return u < 4 ? u : (u < 7 ? u - 3 : (u < 9 ? u - 5 : 3)); }
// local edges (a, b) and faces as compile-time functions (the same numbering as
// EA, EB and FV): face f is opposite vertex 3 - f
__host__ __device__ constexpr int ea_(int p) { return p < 3 ? 0 : (p < 5 ? 1 : 2); }
__host__ __device__ constexpr int eb_(int p) { return p < 3 ? p + 1 : (p < 5 ? p - 1 : 3); }
__host__ __device__ constexpr int fv_(int f, int i) { return i < 3 - f ? i : i + 1; }
static_assert(ea_(0) == 0 && eb_(0) == 1 && ea_(3) == 1 && eb_(3) == 2 && ea_(4) == 1 && eb_(4) == 3 &&
                  ea_(5) == 2 && eb_(5) == 3,
              "local edges");
static_assert(fv_(0, 2) == 2 && fv_(1, 2) == 3 && fv_(2, 1) == 2 && fv_(3, 0) == 1, "local faces");
static_assert(mono2(0, 3) == 3 && mono2(1, 1) == 4 && mono2(3, 2) == 8 && mono2_a(7) == 2 && mono2_b(6) == 3,
              "degree-2 monomials");
__host__ __device__ constexpr int fact(int n) { return n <= 1 ? 1 : n * fact(n - 1); }
// (1/V) int_T of l_i l_j l_k l_l (degree 4) and of l_i l_j (degree 2)
__host__ __device__ constexpr double gram4(int i, int j, int k, int l)
{
    int a[4] = {0, 0, 0, 0};
    a[i]++;
    a[j]++;
    a[k]++;
    a[l]++;
    return 6.0 * fact(a[0]) * fact(a[1]) * fact(a[2]) * fact(a[3]) / fact(7);
}
__host__ __device__ constexpr double gram2(int i, int j) { return i == j ? 0.1 : 0.05; }

template <int K>
struct MonoN;
template <>
struct MonoN<1> {
    static constexpr int NM = 4, NS = 1;
};
template <>
struct MonoN<2> {
    static constexpr int NM = 10, NS = 4;
};

// the coefficients of the P_m as linear maps of the tet's W1 coefficients:
// f(j, m, u, c) for every term "P_m contains c x_j times monomial u"
template <int K, typename F>
__device__ __forceinline__ void w1_terms(F &&f)
{
    if constexpr (K == 1) {
#pragma unroll
        for (int e = 0; e < 6; e++) {
            f(e, eb_(e), ea_(e), 1.0f);   // l_a grad l_b
            f(e, ea_(e), eb_(e), -1.0f);  // - l_b grad l_a
        }
    } else {
        // l_a as the sum over n of l_a l_n
        auto lin = [&](int j, int m, int a, float c) {
#pragma unroll
            for (int n = 0; n < 4; n++) f(j, m, mono2(a, n), c);
        };
#pragma unroll
        for (int e = 0; e < 6; e++) {
            const int a = ea_(e), b = eb_(e);
            // DoF 2e: (3 l_a - 1) W_ab ; DoF 2e+1: (3 l_b - 1) W_ab
            f(2 * e, b, mono2(a, a), 3.0f);
            lin(2 * e, b, a, -1.0f);
            f(2 * e, a, mono2(a, b), -3.0f);
            lin(2 * e, a, b, 1.0f);
            f(2 * e + 1, b, mono2(a, b), 3.0f);
            lin(2 * e + 1, b, a, -1.0f);
            f(2 * e + 1, a, mono2(b, b), -3.0f);
            lin(2 * e + 1, a, b, 1.0f);
        }
#pragma unroll
        for (int fc = 0; fc < 4; fc++) {
            const int a = fv_(fc, 0), b = fv_(fc, 1), c = fv_(fc, 2);
            // DoF 12+2f: 3 l_c W_ab ; DoF 13+2f: 3 l_b W_ac
            f(12 + 2 * fc, b, mono2(a, c), 3.0f);
            f(12 + 2 * fc, a, mono2(b, c), -3.0f);
            f(13 + 2 * fc, c, mono2(a, b), 3.0f);
            f(13 + 2 * fc, a, mono2(b, c), -3.0f);
        }
    }
}

// coefficient of monomial v (degree K-1) in dP/dl_i for the monomial u of P
// (degree K): d(l_a l_b)/dl_i over the degree-1 monomials; degree 1: d l_a / dl_i
template <int K>
__device__ __forceinline__ constexpr float dmono(int u, int i, int v)
{
    if constexpr (K == 1) {
        return u == i ? 1.0f : 0.0f;
    } else {
        const int a = mono2_a(u), b = mono2_b(u);
        if (a == b) return (a == i && v == a) ? 2.0f : 0.0f;
        return (a == i && v == b) || (b == i && v == a) ? 1.0f : 0.0f;
    }
}

// PAIRS (order 2): map1 holds per tet the N1/2 pair ids j of its DoF pairs
// (local 2i, 2i+1 are the unknowns 2j, 2j+1; -1 when they are not unknowns),
// and x is read a pair at a time
// With PAIRS the products of pair i go to position slot[t][i] of the pairs'
// incidence lists (pe then holds T pairs in incidence order; -1: not unknowns),
// so that the row sums read them contiguously.
template <int K, typename T, bool PAIRS>
__global__ __launch_bounds__(BLK) void k_mf_elem(int64_t nt, const int32_t *__restrict__ map1, int64_t n1s,
                                                 const T *__restrict__ geo, const T *__restrict__ x, T kM, T kC,
                                                 T *__restrict__ pe, const int32_t *__restrict__ slot)
{
    constexpr int N1 = Ord<K>::N1, NM = MonoN<K>::NM, NS = MonoN<K>::NS;
    // workgroups go round-robin to the 8 XCDs; each XCD takes one contiguous
    // eighth of the tets, so that neighbouring tets' parts of the same rows meet
    // in one L2 before they are written back
    // (XCD x = b % 8 holds the q + (x < r) workgroups b = x, x + 8, ..., with q, r =
    // G / 8, G % 8 for G workgroups, and takes the range starting at x q + min(x, r):
    // a bijection of [0, G))
    const int64_t ng = gridDim.x, bk = blockIdx.x, q = ng / 8, r = ng % 8, xc = bk % 8;
    const int64_t wb = xc * q + (xc < r ? xc : r) + bk / 8;
    const int64_t t = wb * BLK + threadIdx.x;
    if (t >= nt) return;
    const gptr<const T> gg = glb(geo) + t * 16;
    T gl[4][3];
#pragma unroll
    for (int m = 0; m < 4; m++)
#pragma unroll
        for (int c = 0; c < 3; c++) gl[m][c] = gg[3 * m + c];
    const T vol = gg[12];
    T xl[N1];
    if constexpr (PAIRS) {
        static_assert(N1 % 2 == 0, "pairs");
        using T2 = T __attribute__((ext_vector_type(2)));
        const gptr<const int32_t> mp = glb(map1) + t * (N1 / 2);
        int32_t d[N1 / 2];
#pragma unroll
        for (int j = 0; j < N1 / 2; j++) d[j] = mp[j];
#pragma unroll
        for (int j = 0; j < N1 / 2; j++) {
            const T2 v = d[j] >= 0 ? *(glb((const T2 *)x) + d[j]) : T2{T(0), T(0)};
            xl[2 * j] = v.x;
            xl[2 * j + 1] = v.y;
        }
    } else {
        const gptr<const int32_t> mp = glb(map1) + t * N1;
        int32_t d[N1];
#pragma unroll
        for (int j = 0; j < N1; j++) d[j] = mp[j];
#pragma unroll
        for (int j = 0; j < N1; j++) xl[j] = d[j] < n1s ? x[d[j]] : T(0);
    }
    // P_m coefficients
    T C[4][NM];
#pragma unroll
    for (int m = 0; m < 4; m++)
#pragma unroll
        for (int u = 0; u < NM; u++) C[m][u] = T(0);
    w1_terms<K>([&](int j, int m, int u, float c) { C[m][u] += T(c) * xl[j]; });
    // grad l_m . grad l_n and (grad l_a x grad l_b) . (grad l_c x grad l_d)
    T g[4][4], X[6][3], G2[6][6];
#pragma unroll
    for (int m = 0; m < 4; m++)
#pragma unroll
        for (int n = m; n < 4; n++) g[m][n] = g[n][m] = gl[m][0] * gl[n][0] + gl[m][1] * gl[n][1] + gl[m][2] * gl[n][2];
#pragma unroll
    for (int p = 0; p < 6; p++) cross3(gl[ea_(p)], gl[eb_(p)], X[p]);
#pragma unroll
    for (int p = 0; p < 6; p++)
#pragma unroll
        for (int q = p; q < 6; q++) G2[p][q] = G2[q][p] = X[p][0] * X[q][0] + X[p][1] * X[q][1] + X[p][2] * X[q][2];
    // curl: S_p = dP_m/dl_n - dP_n/dl_m for the pair p = (n, m), n < m
    T S[6][NS];
#pragma unroll
    for (int p = 0; p < 6; p++) {
        const int n = ea_(p), m = eb_(p);
#pragma unroll
        for (int v = 0; v < NS; v++) {
            T s = T(0);
#pragma unroll
            for (int u = 0; u < NM; u++) {
                const float d1 = dmono<K>(u, n, v), d2 = dmono<K>(u, m, v);
                if (d1 != 0.0f) s += T(d1) * C[m][u];
                if (d2 != 0.0f) s -= T(d2) * C[n][u];
            }
            S[p][v] = s;
        }
    }
    // mass: D[m] = kM V sum_n g[m][n] H C[n], H the degree-K Gram matrix
    T D[4][NM];
    {
        T h[4][NM];
#pragma unroll
        for (int n = 0; n < 4; n++)
#pragma unroll
            for (int u = 0; u < NM; u++) {
                T s = T(0);
#pragma unroll
                for (int w = 0; w < NM; w++) {
                    if constexpr (K == 1) s += T(gram2(u, w)) * C[n][w];
                    else s += T(gram4(mono2_a(u), mono2_b(u), mono2_a(w), mono2_b(w))) * C[n][w];
                }
                h[n][u] = s;
            }
        const T sm = kM * vol;
#pragma unroll
        for (int m = 0; m < 4; m++)
#pragma unroll
            for (int u = 0; u < NM; u++)
                D[m][u] = sm * (g[m][0] * h[0][u] + g[m][1] * h[1][u] + g[m][2] * h[2][u] + g[m][3] * h[3][u]);
    }
    // curl: dS[p] = kC V sum_q G2[p][q] H' S[q] (H' the degree-(K-1) Gram matrix), then
    // the transpose of the map C -> S into D
    {
        T hs[6][NS];
#pragma unroll
        for (int q = 0; q < 6; q++)
#pragma unroll
            for (int v = 0; v < NS; v++) {
                if constexpr (K == 1) {
                    hs[q][v] = S[q][v];
                } else {
                    T s = T(0);
#pragma unroll
                    for (int w = 0; w < NS; w++) s += T(gram2(v, w)) * S[q][w];
                    hs[q][v] = s;
                }
            }
        const T sc = kC * vol;
#pragma unroll
        for (int p = 0; p < 6; p++) {
            const int n = ea_(p), m = eb_(p);
#pragma unroll
            for (int v = 0; v < NS; v++) {
                T ds = T(0);
#pragma unroll
                for (int q = 0; q < 6; q++) ds += G2[p][q] * hs[q][v];
                ds *= sc;
#pragma unroll
                for (int u = 0; u < NM; u++) {
                    const float d1 = dmono<K>(u, n, v), d2 = dmono<K>(u, m, v);
                    if (d1 != 0.0f) D[m][u] += T(d1) * ds;
                    if (d2 != 0.0f) D[n][u] -= T(d2) * ds;
                }
            }
        }
    }
    T yl[N1];
#pragma unroll
    for (int j = 0; j < N1; j++) yl[j] = T(0);
    w1_terms<K>([&](int j, int m, int u, float c) { yl[j] += T(c) * D[m][u]; });
    if constexpr (PAIRS) {
        using T2 = T __attribute__((ext_vector_type(2)));
        const gptr<const int32_t> sl = glb(slot) + t * (N1 / 2);
        const gptr<T2> po = glb((T2 *)pe);
#pragma unroll
        for (int j = 0; j < N1 / 2; j++) {
            const int32_t s = sl[j];
            if (s >= 0) po[s] = T2{yl[2 * j], yl[2 * j + 1]};
        }
    } else {
        const gptr<T> po = glb(pe) + t * N1;
#pragma unroll
        for (int j = 0; j < N1; j++) po[j] = yl[j];
    }
}

// the same sums a pair of DoFs (2j, 2j+1) at a time: they meet the same tets, at
// adjacent local positions, and k_mf_elem has put their products at positions
// [ptr[j], ptr[j+1]) of pe, in tet order
template <typename T>
__global__ __launch_bounds__(BLK) void k_mf_sum2(int64_t npair, const int64_t *__restrict__ ptr,
                                                 const T *__restrict__ pe, T *__restrict__ y,
                                                 const T *__restrict__ dotv, double *__restrict__ partial)
{
    using T2 = T __attribute__((ext_vector_type(2)));
    __shared__ double s_red[BLK];
    constexpr int U = 8;
    const int tid = threadIdx.x;
    const gptr<const T2> pe2 = glb((const T2 *)pe);
    double d = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * BLK + tid; j < npair; j += (int64_t)gridDim.x * BLK) {
        const int64_t kb = ptr[j], ke = ptr[j + 1];
        const T2 w = dotv ? *(glb((const T2 *)dotv) + j) : T2{T(0), T(0)};
        T s0 = T(0), s1 = T(0);
        for (int64_t k = kb; k < ke; k += U) {
            // entries past the row's end load its last one again and are not added
            T2 v[U];
#pragma unroll
            for (int u = 0; u < U; u++) v[u] = pe2[min(k + u, ke - 1)];
#pragma unroll
            for (int u = 0; u < U; u++)
                if (k + u < ke) {
                    s0 += v[u].x;
                    s1 += v[u].y;
                }
        }
        *(glb((T2 *)y) + j) = T2{s0, s1};
        d += (double)w.x * (double)s0 + (double)w.y * (double)s1;
    }
    if (partial) {
        s_red[tid] = d;
        __syncthreads();
        for (int o = BLK / 2; o > 0; o >>= 1) {
            if (tid < o) s_red[tid] += s_red[tid + o];
            __syncthreads();
        }
        if (tid == 0) partial[blockIdx.x] = s_red[0];
    }
}

// y_i = sum of the tets' products over the incidences of unknown DoF i, in tet
// order; optional fused partial dot(dotv, y) per workgroup (fixed order)
template <typename T>
__global__ __launch_bounds__(BLK) void k_mf_sum(int64_t n, const int64_t *__restrict__ ptr,
                                                const int32_t *__restrict__ idx, const T *__restrict__ pe,
                                                T *__restrict__ y, const T *__restrict__ dotv,
                                                double *__restrict__ partial)
{
    __shared__ double s_red[BLK];
    constexpr int U = 8;
    const int tid = threadIdx.x;
    double d = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLK + tid; i < n; i += (int64_t)gridDim.x * BLK) {
        const int64_t kb = ptr[i], ke = ptr[i + 1];
        const T w = dotv ? dotv[i] : T(0);
        T s = T(0);
        for (int64_t k = kb; k < ke; k += U) {
            // entries past the row's end load its last one again and are not added
            int32_t ix[U];
#pragma unroll
            for (int u = 0; u < U; u++) ix[u] = idx[min(k + u, ke - 1)];
            T v[U];
#pragma unroll
            for (int u = 0; u < U; u++) v[u] = pe[ix[u]];
#pragma unroll
            for (int u = 0; u < U; u++)
                if (k + u < ke) s += v[u];
        }
        y[i] = s;
        d += (double)w * (double)s;
    }
    if (partial) {
        s_red[tid] = d;
        __syncthreads();
        for (int o = BLK / 2; o > 0; o >>= 1) {
            if (tid < o) s_red[tid] += s_red[tid + o];
            __syncthreads();
        }
        if (tid == 0) partial[blockIdx.x] = s_red[0];
    }
}

// fixed-order sum of n partials (one block of 1024 threads), k values interleaved
__global__ __launch_bounds__(1024) void k_finish(const double *__restrict__ partial, int64_t n, int k,
                                                 double *__restrict__ out)
{
    __shared__ double s[4][1024];
    const int tid = threadIdx.x;
    double acc[4] = {0, 0, 0, 0};
    for (int64_t i = tid; i < n; i += 1024)
        for (int q = 0; q < k; q++) acc[q] += partial[i * k + q];
    for (int q = 0; q < k; q++) s[q][tid] = acc[q];
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (tid < o)
            for (int q = 0; q < k; q++) s[q][tid] += s[q][tid + o];
        __syncthreads();
    }
    if (tid == 0)
        for (int q = 0; q < k; q++) out[q] = s[q][0];
}

// PCG scalars (device double block): RZ[2] ping-pong by iteration parity,
// PQ, and after k_finish: sc[8] = r.z (new), sc[9] = r.r
// x += a p ; r -= a q ; z = dinv r ; partial (r.z, r.r), with a = rz / pq
// the preconditioner: Jacobi (dinv[i] = 1 / A_ii), or with BLOCK 2x2 block
// Jacobi (dinv[4j..4j+3] = inverse of the diagonal block of rows 2j, 2j+1,
// row-major); with BLOCK a thread handles one pair of rows
// sums over i < n of v[2 i + q] (q = 0, 1; two = false: of v[i] alone) in one fixed
// order, the same in every workgroup: strided entries per thread, then a tree
// in LDS (blockDim.x == BLK)
template <bool TWO>
__device__ __forceinline__ void block_totals(const double *__restrict__ v, int64_t n, double *s0, double *s1,
                                             double &t0, double &t1)
{
    const int tid = threadIdx.x;
    double a0 = 0.0, a1 = 0.0;
    for (int64_t i = tid; i < n; i += BLK) {
        if constexpr (TWO) {
            a0 += v[2 * i];
            a1 += v[2 * i + 1];
        } else {
            a0 += v[i];
        }
    }
    s0[tid] = a0;
    if constexpr (TWO) s1[tid] = a1;
    __syncthreads();
    for (int o = BLK / 2; o > 0; o >>= 1) {
        if (tid < o) {
            s0[tid] += s0[tid + o];
            if constexpr (TWO) s1[tid] += s1[tid + o];
        }
        __syncthreads();
    }
    t0 = s0[0];
    t1 = TWO ? s1[0] : 0.0;
    __syncthreads();
}

// pq: the npq workgroup partials of p.q, summed here by every workgroup
template <typename T, bool BLOCK>
__global__ __launch_bounds__(BLK) void k_update_xr(int64_t n, T *__restrict__ x, T *__restrict__ r, T *__restrict__ z,
                                                   const T *__restrict__ p, const T *__restrict__ q,
                                                   const T *__restrict__ dinv, const double *__restrict__ sc, int par,
                                                   const double *__restrict__ pqpart, int64_t npq,
                                                   double *__restrict__ partial)
{
    __shared__ double s0[BLK], s1[BLK];
    const int tid = threadIdx.x;
    double pq, unused;
    block_totals<false>(pqpart, npq, s0, s1, pq, unused);
    const double a = pq != 0.0 ? sc[SC_RZ + 10 * par] / pq : 0.0;
    double rz = 0, rr = 0;
    if constexpr (BLOCK) {
        for (int64_t j = (int64_t)blockIdx.x * BLK + tid; 2 * j < n; j += (int64_t)gridDim.x * BLK) {
            const int64_t i = 2 * j;
            x[i] = (T)((double)x[i] + a * (double)p[i]);
            x[i + 1] = (T)((double)x[i + 1] + a * (double)p[i + 1]);
            const T r0 = (T)((double)r[i] - a * (double)q[i]);
            const T r1 = (T)((double)r[i + 1] - a * (double)q[i + 1]);
            r[i] = r0;
            r[i + 1] = r1;
            const T z0 = dinv[4 * j] * r0 + dinv[4 * j + 1] * r1;
            const T z1 = dinv[4 * j + 2] * r0 + dinv[4 * j + 3] * r1;
            z[i] = z0;
            z[i + 1] = z1;
            rz += (double)r0 * (double)z0 + (double)r1 * (double)z1;
            rr += (double)r0 * (double)r0 + (double)r1 * (double)r1;
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * BLK + tid; i < n; i += (int64_t)gridDim.x * BLK) {
            x[i] = (T)((double)x[i] + a * (double)p[i]);
            T ri = (T)((double)r[i] - a * (double)q[i]);
            r[i] = ri;
            T zi = dinv[i] * ri;
            z[i] = zi;
            rz += (double)ri * (double)zi;
            rr += (double)ri * (double)ri;
        }
    }
    s0[tid] = rz;
    s1[tid] = rr;
    __syncthreads();
    for (int o = BLK / 2; o > 0; o >>= 1) {
        if (tid < o) {
            s0[tid] += s0[tid + o];
            s1[tid] += s1[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        partial[2 * blockIdx.x] = s0[0];
        partial[2 * blockIdx.x + 1] = s1[0];
    }
}

// p = z + b p with b = rz_new / rz_old, rz_new and r.r summed by every workgroup
// from the nrz (r.z, r.r) partials; keeps r.z for the next iteration in the
// other parity slot (no other thread reads that slot in this launch) and r.r
template <typename T>
__global__ __launch_bounds__(BLK) void k_update_p(int64_t n, T *__restrict__ p, const T *__restrict__ z,
                                                  double *__restrict__ sc, int par, const double *__restrict__ rzpart,
                                                  int64_t nrz)
{
    __shared__ double s0[BLK], s1[BLK];
    double rzn, rrn;
    block_totals<true>(rzpart, nrz, s0, s1, rzn, rrn);
    const double rzo = sc[SC_RZ + 10 * par];
    const double bt = rzo != 0.0 ? rzn / rzo : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[SC_RZ + 10 * (1 - par)] = rzn;
        sc[SC_RR] = rrn;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (T)((double)z[i] + bt * (double)p[i]);
}

// r = b, x = 0, z = dinv r, p = z ; partial (r.z, r.r)
template <typename T, bool BLOCK>
__global__ __launch_bounds__(BLK) void k_pcg_init(int64_t n, const T *__restrict__ b, T *__restrict__ x,
                                                  T *__restrict__ r, T *__restrict__ z, T *__restrict__ p,
                                                  const T *__restrict__ dinv, double *__restrict__ partial)
{
    __shared__ double s0[BLK], s1[BLK];
    const int tid = threadIdx.x;
    double rz = 0, rr = 0;
    if constexpr (BLOCK) {
        for (int64_t j = (int64_t)blockIdx.x * BLK + tid; 2 * j < n; j += (int64_t)gridDim.x * BLK) {
            const int64_t i = 2 * j;
            const T r0 = b[i], r1 = b[i + 1];
            x[i] = T(0);
            x[i + 1] = T(0);
            r[i] = r0;
            r[i + 1] = r1;
            const T z0 = dinv[4 * j] * r0 + dinv[4 * j + 1] * r1;
            const T z1 = dinv[4 * j + 2] * r0 + dinv[4 * j + 3] * r1;
            z[i] = z0;
            z[i + 1] = z1;
            p[i] = z0;
            p[i + 1] = z1;
            rz += (double)r0 * (double)z0 + (double)r1 * (double)z1;
            rr += (double)r0 * (double)r0 + (double)r1 * (double)r1;
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * BLK + tid; i < n; i += (int64_t)gridDim.x * BLK) {
            T ri = b[i];
            x[i] = T(0);
            r[i] = ri;
            T zi = dinv[i] * ri;
            z[i] = zi;
            p[i] = zi;
            rz += (double)ri * (double)zi;
            rr += (double)ri * (double)ri;
        }
    }
    s0[tid] = rz;
    s1[tid] = rr;
    __syncthreads();
    for (int o = BLK / 2; o > 0; o >>= 1) {
        if (tid < o) {
            s0[tid] += s0[tid + o];
            s1[tid] += s1[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        partial[2 * blockIdx.x] = s0[0];
        partial[2 * blockIdx.x + 1] = s1[0];
    }
}

__global__ void k_init_sc(double *sc)
{
    sc[SC_RZ] = sc[8];
    sc[SC_RR] = sc[9];
    sc[SC_BB] = sc[9];
}

__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b, const double *__restrict__ y,
                        double *__restrict__ o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = a * x[i] + (b != 0.0 ? b * y[i] : 0.0);
}

__global__ void k_cast_d2f(int64_t n, const double *__restrict__ in, float *__restrict__ out, double scale)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)(in[i] * scale);
}

__global__ void k_add_f2d(int64_t n, const float *__restrict__ in, double scale, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += scale * (double)in[i];
}

// Gauss check partial sums: |GtDe + d|^2, |Gtg - d|^2, |GtDe + Gtg|^2, |d|^2 with d = rho - rho0
__global__ __launch_bounds__(BLK) void k_gauss_partial(int64_t n, const double *__restrict__ a,
                                                       const double *__restrict__ g, const double *__restrict__ rho,
                                                       const double *__restrict__ rho0, double gscale,
                                                       double *__restrict__ partial)
{
    __shared__ double s[4][BLK];
    const int tid = threadIdx.x;
    double v[4] = {0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * BLK + tid; i < n; i += (int64_t)gridDim.x * BLK) {
        const double d = rho[i] - rho0[i], ai = a[i] / gscale, gi = g[i] / gscale;
        double x1 = ai + d, x2 = gi - d, x3 = ai + gi;
        v[0] += x1 * x1;
        v[1] += x2 * x2;
        v[2] += x3 * x3;
        v[3] += d * d;
    }
    for (int q = 0; q < 4; q++) s[q][tid] = v[q];
    __syncthreads();
    for (int o = BLK / 2; o > 0; o >>= 1) {
        if (tid < o)
            for (int q = 0; q < 4; q++) s[q][tid] += s[q][tid + o];
        __syncthreads();
    }
    if (tid == 0)
        for (int q = 0; q < 4; q++) partial[4 * blockIdx.x + q] = s[q][0];
}

__global__ __launch_bounds__(BLK) void k_dot_partial(int64_t n, const double *__restrict__ a,
                                                     const double *__restrict__ b, double *__restrict__ partial)
{
    __shared__ double s[BLK];
    const int tid = threadIdx.x;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLK + tid; i < n; i += (int64_t)gridDim.x * BLK) acc += a[i] * b[i];
    s[tid] = acc;
    __syncthreads();
    for (int o = BLK / 2; o > 0; o >>= 1) {
        if (tid < o) s[tid] += s[tid + o];
        __syncthreads();
    }
    if (tid == 0) partial[blockIdx.x] = s[0];
}

inline unsigned nblk(int64_t n, int b = BLK) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// =================================================================== launchers
hipError_t launch_locate_cube(const DevMesh &m, int64_t n, DevParticles p, int32_t *err, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_locate_cube, dim3(nblk(n)), dim3(BLK), 0, s, m, n, p, err);
    return hipGetLastError();
}

hipError_t launch_to_bary(const DevMesh &m, int64_t n, DevParticles p, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_bary, dim3(nblk(n)), dim3(BLK), 0, s, m, n, p);
    return hipGetLastError();
}

hipError_t launch_startup(int order, bool mixed, const DevMesh &m, const double *e, const double *b, const float *e32,
                          const float *b32, DevParticles p, int64_t n, double qm, double dt, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (order == 1) {
        if (mixed) hipLaunchKernelGGL((k_startup<1, float>), dim3(nblk(n)), dim3(BLK), 0, s, m, e32, b32, p, n, qm, dt);
        else hipLaunchKernelGGL((k_startup<1, double>), dim3(nblk(n)), dim3(BLK), 0, s, m, e, b, p, n, qm, dt);
    } else {
        if (mixed) hipLaunchKernelGGL((k_startup<2, float>), dim3(nblk(n)), dim3(BLK), 0, s, m, e32, b32, p, n, qm, dt);
        else hipLaunchKernelGGL((k_startup<2, double>), dim3(nblk(n)), dim3(BLK), 0, s, m, e, b, p, n, qm, dt);
    }
    return hipGetLastError();
}

int64_t sort_hist_entries(int64_t n) { return 256 * std::max<int64_t>(1, (n + RS_TILE - 1) / RS_TILE); }

int64_t scan_tmp_entries(int64_t n)
{
    // level sums + their scan
    int64_t t = 0, m = n;
    while (m > SC_TILE) {
        m = (m + SC_TILE - 1) / SC_TILE;
        t += 2 * m + 2;
    }
    return t + 4;
}

hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, uint32_t *total,
                              hipStream_t s, const int32_t *dn)
{
    const int32_t *nodn = nullptr;
    if (n == 0) {
        if (total) hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, s, in, out, n, total, nodn);
        return hipGetLastError();
    }
    const int64_t nb = (n + SC_TILE - 1) / SC_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_tile1, dim3(1), dim3(SC_THREADS), 0, s, in, out, n, total, dn);
        return hipGetLastError();
    }
    if (nb <= SCAN_DIRECT_TILES) {
        // two launches: tile scans, then each tile adds the sums before it (and the total)
        uint32_t *sums = tmp;
        hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nb), dim3(SC_THREADS), 0, s, in, out, n, sums, dn);
        hipLaunchKernelGGL(k_scan_add_direct, dim3((unsigned)nb), dim3(BLK), 0, s, out, n, sums, total, dn);
        return hipGetLastError();
    }
    {
        uint32_t *sums = tmp;
        uint32_t *sums_scan = tmp + nb;
        hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nb), dim3(SC_THREADS), 0, s, in, out, n, sums, dn);
        hipError_t err = exclusive_scan_u32(sums, sums_scan, nb, tmp + 2 * nb, nullptr, s);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(BLK), 0, s, out, n, sums_scan, dn);
    }
    if (total) hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, s, in, out, n, total, dn);
    return hipGetLastError();
}

hipError_t radix_sort(SortBuffers &sb, int64_t n, int bits, bool vals_are_iota, int *result_buf, hipStream_t s,
                      const uint32_t *key_in, const int32_t *dn)
{
    int cur = 0;
    if (n == 0) {
        *result_buf = 0;
        return hipSuccess;
    }
    const int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    int passes = std::max(1, (bits + 7) / 8);
    for (int pass = 0; pass < passes; pass++) {
        const int shift = 8 * pass;
        const uint32_t *kin = (pass == 0 && key_in) ? key_in : sb.key[cur];
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntiles), dim3(BLK), 0, s, kin, n, shift, sb.hist, ntiles, dn);
        hipError_t err = exclusive_scan_u32(sb.hist, sb.hist, 256 * ntiles, sb.scan_tmp, nullptr, s);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntiles), dim3(BLK), 0, s, kin, sb.val[cur],
                           sb.key[1 - cur], sb.val[1 - cur], n, shift, sb.hist, ntiles,
                           (pass == 0 && vals_are_iota) ? 1 : 0, dn);
        cur = 1 - cur;
    }
    *result_buf = cur;
    return hipGetLastError();
}

hipError_t launch_permute(bool mixed, DevParticles in, DevParticles out, const uint32_t *perm, int64_t n,
                          hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (mixed) hipLaunchKernelGGL(k_permute<PART_MIXED.nw>, dim3(nblk(n)), dim3(BLK), 0, s, in, out, perm, n);
    else hipLaunchKernelGGL(k_permute<PART_FP64.nw>, dim3(nblk(n)), dim3(BLK), 0, s, in, out, perm, n);
    return hipGetLastError();
}

__global__ void k_merge_order(int64_t np0, int64_t n, int32_t nt, const int32_t *__restrict__ off,
                              const int32_t *__restrict__ noff_new, const uint32_t *__restrict__ perm,
                              const uint32_t *__restrict__ nkey, const uint32_t *__restrict__ nval, uint32_t slot0,
                              int32_t *__restrict__ next_off, uint32_t *__restrict__ next_perm)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < np0) {
        // the present particle's tet: the last one whose range starts at or before it
        int lo = 0, hi = nt;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (off[mid] <= g) lo = mid;
            else hi = mid;
        }
        next_perm[g + noff_new[lo]] = perm[g];
    } else if (g < np0 + n) {
        const int64_t q = g - np0;
        next_perm[off[nkey[q] + 1] + q] = slot0 + nval[q];
    } else if (g <= np0 + n + nt) {
        const int64_t t = g - np0 - n;
        next_off[t] = off[t] + noff_new[t];
    }
}

hipError_t launch_merge_order(int64_t np0, int64_t n, int32_t nt, const int32_t *off, const int32_t *noff_new,
                              const uint32_t *perm, const uint32_t *nkey, const uint32_t *nval, uint32_t slot0,
                              int32_t *next_off, uint32_t *next_perm, hipStream_t s)
{
    const int64_t w = np0 + n + nt + 1;
    hipLaunchKernelGGL(k_merge_order, dim3(nblk(w)), dim3(BLK), 0, s, np0, n, nt, off, noff_new, perm, nkey, nval,
                       slot0, next_off, next_perm);
    return hipGetLastError();
}

hipError_t launch_tet_keys(DevParticles p, int64_t n, uint32_t *keys, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tet_keys, dim3(nblk(n)), dim3(BLK), 0, s, p, n, keys);
    return hipGetLastError();
}

// the same offsets for few keys over many buckets (a host count below nt): one
// thread per bucket finds its first key by bisection, so that no thread walks a
// long run of empty buckets
__global__ void k_offsets_sparse(const uint32_t *__restrict__ key, int64_t n, int32_t nt, int32_t *__restrict__ off,
                                 const int32_t *__restrict__ dn)
{
    n = dev_count(n, dn);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > nt) return;
    int64_t lo = 0, hi = n;  // first index whose key (clamped to nt) is >= t
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (min((int64_t)key[mid], (int64_t)nt) < t) lo = mid + 1;
        else hi = mid;
    }
    off[t] = (int32_t)lo;
}

hipError_t launch_offsets(const uint32_t *key, int64_t n, int32_t nt, int32_t *off, hipStream_t s, const int32_t *dn)
{
    if (n < (int64_t)nt) {
        hipLaunchKernelGGL(k_offsets_sparse, dim3(nblk((int64_t)nt + 1)), dim3(BLK), 0, s, key, n, nt, off, dn);
        return hipGetLastError();
    }
    // with a device count, n may come out as 0: then nt + 1 threads clear off
    const int64_t w = dn ? std::max<int64_t>(n, (int64_t)nt + 1) : (n > 0 ? n : (int64_t)nt + 1);
    hipLaunchKernelGGL(k_offsets, dim3(nblk(w)), dim3(BLK), 0, s, key, n, nt, off, dn);
    return hipGetLastError();
}

hipError_t launch_particle(int order, bool mixed, bool boris, const ParticleArgs *A, int32_t nt, int32_t tpw,
                           hipStream_t s)
{
    const unsigned grid = (unsigned)((nt + tpw - 1) / tpw);
    const int v = (order == 1 ? 0 : 4) + (mixed ? 0 : 2) + (boris ? 1 : 0);
    switch (v) {
    case 0: hipLaunchKernelGGL((k_particle<1, float, false>), dim3(grid), dim3(PBLK), 0, s, A); break;
    case 1: hipLaunchKernelGGL((k_particle<1, float, true>), dim3(grid), dim3(PBLK), 0, s, A); break;
    case 2: hipLaunchKernelGGL((k_particle<1, double, false>), dim3(grid), dim3(PBLK), 0, s, A); break;
    case 3: hipLaunchKernelGGL((k_particle<1, double, true>), dim3(grid), dim3(PBLK), 0, s, A); break;
    case 4: hipLaunchKernelGGL((k_particle<2, float, false>), dim3(grid), dim3(PBLK), 0, s, A); break;
    case 5: hipLaunchKernelGGL((k_particle<2, float, true>), dim3(grid), dim3(PBLK), 0, s, A); break;
    case 6: hipLaunchKernelGGL((k_particle<2, double, false>), dim3(grid), dim3(PBLK), 0, s, A); break;
    default: hipLaunchKernelGGL((k_particle<2, double, true>), dim3(grid), dim3(PBLK), 0, s, A); break;
    }
    return hipGetLastError();
}

hipError_t launch_queue_index(const ContQueue &cq, int64_t np, uint32_t *tmp, hipStream_t s)
{
    if (np == 0) return exclusive_scan_u32(tmp, tmp, 0, tmp, (uint32_t *)cq.count, s);
    const int64_t nt = (np + QTILE - 1) / QTILE;
    uint32_t *tsum = tmp, *tpos = tmp + nt;
    hipLaunchKernelGGL(k_flag_count, dim3((unsigned)nt), dim3(BLK), 0, s, cq.flag, np, tsum);
    hipError_t err = exclusive_scan_u32(tsum, tpos, nt, tmp + 2 * nt, (uint32_t *)cq.count, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_flag_compact, dim3((unsigned)nt), dim3(BLK), 0, s, cq.flag, np, tpos, cq.idx);
    return hipGetLastError();
}

hipError_t launch_continue(int order, bool mixed, bool boris, const ParticleArgs *A, int64_t nq_hint,
                           unsigned long long *cntb, unsigned long long *cnt, hipStream_t s)
{
    // about one queued path per thread (a grid-stride loop covers a longer queue)
    const int64_t want = (nq_hint + nq_hint / 8 + BLK - 1) / BLK + 16;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(CONT_BLOCKS, want));
    if (order == 1) {
        if (boris) {
            if (mixed) hipLaunchKernelGGL((k_continue<1, float, true>), dim3(grid), dim3(BLK), 0, s, A);
            else hipLaunchKernelGGL((k_continue<1, double, true>), dim3(grid), dim3(BLK), 0, s, A);
        } else {
            if (mixed) hipLaunchKernelGGL((k_continue<1, float>), dim3(grid), dim3(BLK), 0, s, A);
            else hipLaunchKernelGGL((k_continue<1, double>), dim3(grid), dim3(BLK), 0, s, A);
        }
    } else {
        if (boris) {
            if (mixed) hipLaunchKernelGGL((k_continue<2, float, true>), dim3(grid), dim3(BLK), 0, s, A);
            else hipLaunchKernelGGL((k_continue<2, double, true>), dim3(grid), dim3(BLK), 0, s, A);
        } else {
            if (mixed) hipLaunchKernelGGL((k_continue<2, float>), dim3(grid), dim3(BLK), 0, s, A);
            else hipLaunchKernelGGL((k_continue<2, double>), dim3(grid), dim3(BLK), 0, s, A);
        }
    }
    hipLaunchKernelGGL(k_counters, dim3(std::min<unsigned>(64u, (grid + BLK - 1) / BLK)), dim3(BLK), 0, s, cntb,
                       (int)grid, cnt);
    return hipGetLastError();
}

hipError_t launch_spill_compact(const SpillPool &pool, int64_t nrec, const int32_t *nq, const uint32_t *pos,
                                uint32_t *key, uint32_t *val, int64_t kcap, hipStream_t s)
{
    if (nrec == 0) return hipSuccess;
    hipLaunchKernelGGL(k_spill_compact, dim3(nblk(nrec)), dim3(BLK), 0, s, pool.tet, pool.tag, nrec, pos, key, val, nq,
                       (const int32_t *)pool.count, kcap);
    return hipGetLastError();
}

hipError_t launch_spill_reduce(int n1l, int32_t nt, const int32_t *soff, const uint32_t *rec, const double *recval,
                               int64_t cap, double *P, const int32_t *nstay, uint32_t *cnt, hipStream_t s)
{
    const int64_t n = (int64_t)nt * n1l;
    if (n == 0 || cap < 1) return hipSuccess;
    if (n1l == 6)
        hipLaunchKernelGGL(k_spill_reduce<6>, dim3(nblk(n)), dim3(BLK), 0, s, nt, soff, rec, recval, cap, P, nstay,
                           cnt);
    else
        hipLaunchKernelGGL(k_spill_reduce<20>, dim3(nblk(n)), dim3(BLK), 0, s, nt, soff, rec, recval, cap, P, nstay,
                           cnt);
    return hipGetLastError();
}

hipError_t launch_place(int64_t np, int32_t nt, int32_t tpw, const int32_t *off, const uint8_t *moved,
                        const int32_t *soff, const uint32_t *srec, int64_t nrec, const int32_t *pid, int64_t cap,
                        const int32_t *noff, uint32_t *perm, unsigned long long *err, hipStream_t s)
{
    if (tpw < 1 || tpw > PLACE_TPW_MAX) return hipErrorInvalidValue;
    if (cap < 1) nrec = 0;
    if (nt > 0)
        hipLaunchKernelGGL(k_place, dim3((unsigned)((nt + tpw - 1) / tpw)), dim3(BLK), 0, s, nt, tpw, off, noff,
                           moved, soff, srec, nrec, pid, cap, np, perm, err);
    return hipGetLastError();
}

hipError_t launch_scatter(const int64_t *ptr, const int32_t *idx, int64_t n, const double *P, double *out,
                          hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(nblk(n)), dim3(BLK), 0, s, ptr, idx, n, P, out);
    return hipGetLastError();
}

hipError_t launch_rho_tet(int order, const DevMesh &m, const uint32_t *perm, const int32_t *off, DevParticles p,
                          double qw, double *Pr, hipStream_t s)
{
    const int tpw = order == 1 ? 64 : 25;  // BLK / n0
    const unsigned grid = (unsigned)((m.nt + tpw - 1) / tpw);
    if (order == 1)
        hipLaunchKernelGGL(k_rho_tet<1>, dim3(grid), dim3(BLK), 0, s, m, perm, off, p, qw, tpw, Pr);
    else
        hipLaunchKernelGGL(k_rho_tet<2>, dim3(grid), dim3(BLK), 0, s, m, perm, off, p, qw, tpw, Pr);
    return hipGetLastError();
}

namespace {
inline unsigned red_grid(int64_t n, int per_block) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(RED_BLOCKS, (n + per_block - 1) / per_block)); }

template <typename T>
hipError_t spmv_t(const DevCSR &A, const T *val, const T *x, T *y, double alpha, double beta, const T *z,
                  const T *dotv, double *partial, unsigned &grid, hipStream_t s)
{
    const T *bv = nullptr;
    if constexpr (sizeof(T) == 8) bv = (const T *)A.bval;
    else bv = (const T *)A.bval32;
    if (A.bptr && bv) {
        constexpr int BL = 8;
        grid = red_grid(A.brows, BLK / BL);
        hipLaunchKernelGGL((k_bspmv<BL, T>), dim3(grid), dim3(BLK), 0, s, A.brows, A.bptr, A.bidx, bv, x, y, alpha,
                           beta, z, dotv, partial);
        return hipGetLastError();
    }
    grid = red_grid(A.rows, BLK / A.lanes);
    if (A.rows == 0) return hipSuccess;
    switch (A.lanes) {
    case 4:
        hipLaunchKernelGGL((k_spmv<4, T>), dim3(grid), dim3(BLK), 0, s, A.rows, A.ptr, A.idx, val, x, y, alpha, beta, z,
                           dotv, partial);
        break;
    case 8:
        hipLaunchKernelGGL((k_spmv<8, T>), dim3(grid), dim3(BLK), 0, s, A.rows, A.ptr, A.idx, val, x, y, alpha, beta, z,
                           dotv, partial);
        break;
    case 16:
        hipLaunchKernelGGL((k_spmv<16, T>), dim3(grid), dim3(BLK), 0, s, A.rows, A.ptr, A.idx, val, x, y, alpha, beta,
                           z, dotv, partial);
        break;
    default:
        hipLaunchKernelGGL((k_spmv<32, T>), dim3(grid), dim3(BLK), 0, s, A.rows, A.ptr, A.idx, val, x, y, alpha, beta,
                           z, dotv, partial);
        break;
    }
    return hipGetLastError();
}
}  // namespace

hipError_t spmv(const DevCSR &A, const double *x, double *y, double alpha, double beta, const double *z, hipStream_t s)
{
    unsigned g;
    return spmv_t<double>(A, A.val, x, y, alpha, beta, z, nullptr, nullptr, g, s);
}

hipError_t spmv32(const DevCSR &A, const float *x, float *y, hipStream_t s)
{
    unsigned g;
    return spmv_t<float>(A, A.val32, x, y, 1.0, 0.0, nullptr, nullptr, nullptr, g, s);
}

hipError_t axpby(int64_t n, double a, const double *x, double b, const double *y, double *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(BLK), 0, s, n, a, x, b, y, out);
    return hipGetLastError();
}

namespace {
template <typename T>
hipError_t pcg_init_t(int64_t n, const T *b, T *x, T *r, T *z, T *p, const T *dinv, double *partial, double *sc,
                      bool block, hipStream_t s)
{
    const unsigned g = red_grid(block ? (n + 1) / 2 : n, BLK);
    if (block) hipLaunchKernelGGL((k_pcg_init<T, true>), dim3(g), dim3(BLK), 0, s, n, b, x, r, z, p, dinv, partial);
    else hipLaunchKernelGGL((k_pcg_init<T, false>), dim3(g), dim3(BLK), 0, s, n, b, x, r, z, p, dinv, partial);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, partial, (int64_t)g, 2, sc + 8);
    hipLaunchKernelGGL(k_init_sc, dim3(1), dim3(1), 0, s, sc);
    return hipGetLastError();
}

template <typename T>
hipError_t mf_apply_t(const DevMF &mf, const T *x, T *y, const T *dotv, double *partial, unsigned &grid,
                      hipStream_t s)
{
    // order 2 is applied in DoF pairs only (the set-up uses the assembled matrix otherwise)
    const bool pairs = mf.order == 2;
    if (pairs && !mf.map1p) return hipErrorInvalidValue;
    grid = red_grid(pairs ? mf.n1s / 2 : mf.n1s, BLK);
    if (mf.nt > 0) {
        const unsigned ge = (unsigned)((mf.nt + BLK - 1) / BLK);
        if (pairs)
            hipLaunchKernelGGL((k_mf_elem<2, T, true>), dim3(ge), dim3(BLK), 0, s, mf.nt, mf.map1p, mf.n1s,
                               (const T *)mf.geo, x, (T)mf.kM, (T)mf.kC, (T *)mf.pe, mf.slot2);
        else
            hipLaunchKernelGGL((k_mf_elem<1, T, false>), dim3(ge), dim3(BLK), 0, s, mf.nt, mf.map1, mf.n1s,
                               (const T *)mf.geo, x, (T)mf.kM, (T)mf.kC, (T *)mf.pe, (const int32_t *)nullptr);
    }
    if (mf.n1s > 0) {
        if (pairs)
            hipLaunchKernelGGL(k_mf_sum2<T>, dim3(grid), dim3(BLK), 0, s, mf.n1s / 2, mf.ptr2, (const T *)mf.pe, y,
                               dotv, partial);
        else
            hipLaunchKernelGGL(k_mf_sum<T>, dim3(grid), dim3(BLK), 0, s, mf.n1s, mf.ptr, mf.idx, (const T *)mf.pe,
                               y, dotv, partial);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t pcg_iter_t(const DevCSR &A, const T *val, const DevMF *mf, int64_t n, T *x, T *r, T *z, T *p, T *q,
                      const T *dinv, double *partial, double *sc, int par, hipStream_t s)
{
    unsigned g1;
    hipError_t err = mf && mf->order ? mf_apply_t<T>(*mf, p, q, p, partial, g1, s)
                                     : spmv_t<T>(A, val, p, q, 1.0, 0.0, (const T *)nullptr, p, partial, g1, s);
    if (err != hipSuccess) return err;
    // the product's partials of p.q at partial[0, g1), the update's (r.z, r.r) ones
    // after them; each consumer sums the partials itself
    double *part2 = partial + RED_BLOCKS;
    const bool block = A.bptr != nullptr;
    const unsigned g2 = red_grid(block ? (n + 1) / 2 : n, BLK);
    if (block)
        hipLaunchKernelGGL((k_update_xr<T, true>), dim3(g2), dim3(BLK), 0, s, n, x, r, z, p, q, dinv, sc, par,
                           partial, (int64_t)g1, part2);
    else
        hipLaunchKernelGGL((k_update_xr<T, false>), dim3(g2), dim3(BLK), 0, s, n, x, r, z, p, q, dinv, sc, par,
                           partial, (int64_t)g1, part2);
    hipLaunchKernelGGL(k_update_p<T>, dim3(g2), dim3(BLK), 0, s, n, p, z, sc, par, part2, (int64_t)g2);
    return hipGetLastError();
}
}  // namespace

hipError_t pcg_init(int64_t n, const double *b, double *x, double *r, double *z, double *p, const double *dinv,
                    double *partial, double *sc, bool block, hipStream_t s)
{
    return pcg_init_t<double>(n, b, x, r, z, p, dinv, partial, sc, block, s);
}

hipError_t pcg_iter(const DevCSR &A, const DevMF *mf, int64_t n, double *x, double *r, double *z, double *p,
                    double *q, const double *dinv, double *partial, double *sc, int par, hipStream_t s)
{
    return pcg_iter_t<double>(A, A.val, mf, n, x, r, z, p, q, dinv, partial, sc, par, s);
}

hipError_t mf_apply(const DevMF &mf, const double *x, double *y, hipStream_t s)
{
    unsigned g;
    return mf_apply_t<double>(mf, x, y, nullptr, nullptr, g, s);
}

hipError_t mf_apply32(const DevMF &mf, const float *x, float *y, hipStream_t s)
{
    unsigned g;
    return mf_apply_t<float>(mf, x, y, nullptr, nullptr, g, s);
}

hipError_t pcg32_init(int64_t n, const float *b, float *x, float *r, float *z, float *p, const float *dinv,
                      double *partial, double *sc, bool block, hipStream_t s)
{
    return pcg_init_t<float>(n, b, x, r, z, p, dinv, partial, sc, block, s);
}

hipError_t pcg32_iter(const DevCSR &A, const DevMF *mf, int64_t n, float *x, float *r, float *z, float *p, float *q,
                      const float *dinv, double *partial, double *sc, int par, hipStream_t s)
{
    return pcg_iter_t<float>(A, A.val32, mf, n, x, r, z, p, q, dinv, partial, sc, par, s);
}

hipError_t cast_d2f(int64_t n, const double *in, float *out, double scale, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cast_d2f, dim3(nblk(n)), dim3(BLK), 0, s, n, in, out, scale);
    return hipGetLastError();
}

hipError_t add_f2d(int64_t n, const float *in, double scale, double *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_f2d, dim3(nblk(n)), dim3(BLK), 0, s, n, in, scale, out);
    return hipGetLastError();
}

hipError_t gauss_norms(int64_t n, const double *GtDe, const double *Gtg, const double *rho, const double *rho0,
                       double gscale, double *partial, double *out4, hipStream_t s)
{
    const int64_t nb = red_grid(n, BLK);
    hipLaunchKernelGGL(k_gauss_partial, dim3((unsigned)nb), dim3(BLK), 0, s, n, GtDe, Gtg, rho, rho0, gscale,
                       partial);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, partial, nb, 4, out4);
    return hipGetLastError();
}

hipError_t dot_det(int64_t n, const double *a, const double *b, double *partial, double *out, hipStream_t s)
{
    const int64_t nb = red_grid(n, BLK);
    hipLaunchKernelGGL(k_dot_partial, dim3((unsigned)nb), dim3(BLK), 0, s, n, a, b, partial);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, partial, nb, 1, out);
    return hipGetLastError();
}

int64_t gauss_partial_entries() { return 4 * (int64_t)RED_BLOCKS; }

// ------------------------------------------- compensated sums, double-double SpMV
// Error-free transformations (Knuth's TwoSum, and TwoProd through the fused
// multiply-add) for the Gauss check: the running sums e and g keep their plain
// FP64 value in hi (bit for bit what hi + d gives) and the rounding error of
// every addition in lo, and the check's products are accumulated as in the
// compensated dot product of Ogita, Rump and Oishi (Dot2), i.e. as if in twice
// the working precision.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    // no contraction here or in the helpers below: once inlined, a product
    // feeding these sums must not fuse into an FMA, which would drop the
    // rounding errors the pairs carry
#pragma clang fp contract(off)
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__global__ void k_add_comp(int64_t n, double *__restrict__ hi, double *__restrict__ lo, const double *__restrict__ d)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s, e;
    two_sum(hi[i], d[i], s, e);
    hi[i] = s;
    lo[i] += e;
}

hipError_t add_comp(int64_t n, double *hi, double *lo, const double *d, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_comp, dim3(nblk(n)), dim3(BLK), 0, s, n, hi, lo, d);
    return hipGetLastError();
}


// Linear combination of sparse products and vectors in double-double:
//   out = a1 (P1 x1) + a2 (P2 (x2 + x2lo)) + c1 v1 + c2 v2
// (any operand may be null), as out_hi + out_lo (out_lo may be null: out_hi is
// then the rounded result).  L lanes per row each accumulate a compensated dot
// product (Dot2), the lanes' pairs are added with TwoSum, and the row's terms
// are scaled with TwoProd and summed compensated.  The field update takes its
// right-hand side and its refinement residuals from here, so that their
// discrete divergence is that of the exact arithmetic to about twice FP64.
struct DD {
    double s = 0.0, c = 0.0;
};
__device__ __forceinline__ void dd_add(DD &a, double x)
{
#pragma clang fp contract(off)
    double t, e;
    two_sum(a.s, x, t, e);
    a.s = t;
    a.c += e;
}
__device__ __forceinline__ void dd_fma(DD &a, double u, double v)  // a += u v
{
#pragma clang fp contract(off)
    const double p = u * v;
    const double q = fma(u, v, -p);
    dd_add(a, p);
    a.c += q;
}
__device__ __forceinline__ void dd_add_scaled(DD &a, double k, const DD &b)  // a += k b
{
#pragma clang fp contract(off)
    dd_fma(a, k, b.s);
    a.c += k * b.c;
}

template <int L>
__device__ inline DD row_dot_dd(const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                const double *__restrict__ val, const double *__restrict__ x,
                                const double *__restrict__ xlo, int64_t r, int lane)
{
#pragma clang fp contract(off)
    DD a;
    const int64_t e = ptr[r + 1];
    int64_t k = ptr[r] + lane;
    // four of the lane's entries at a time: their loads are issued together, and
    // they are added in the same order as one at a time
    constexpr int U = 4;
    for (; k + (U - 1) * L < e; k += U * L) {
        double v[U], xv[U], xl[U];
        int32_t j[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            v[u] = val[k + u * L];
            j[u] = idx[k + u * L];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            xv[u] = x[j[u]];
            xl[u] = xlo ? xlo[j[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            dd_fma(a, v[u], xv[u]);
            if (xlo) a.c += v[u] * xl[u];
        }
    }
    for (; k < e; k += L) {
        const double v = val[k];
        const int32_t j = idx[k];
        dd_fma(a, v, x[j]);
        if (xlo) a.c += v * xlo[j];
    }
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) {
        const double s2 = __shfl_xor(a.s, o, L), c2 = __shfl_xor(a.c, o, L);
        double t, e;
        two_sum(a.s, s2, t, e);
        a.s = t;
        a.c += c2 + e;
    }
    return a;
}

template <int L>
__global__ __launch_bounds__(BLK) void k_combo_dd(int64_t rows, DevCSR P1, const double *__restrict__ x1, double a1,
                                                  DevCSR P2, const double *__restrict__ x2,
                                                  const double *__restrict__ x2lo, double a2,
                                                  const double *__restrict__ v1, double c1,
                                                  const double *__restrict__ v2, double c2,
                                                  double *__restrict__ out_hi, double *__restrict__ out_lo)
{
#pragma clang fp contract(off)
    const int64_t r = ((int64_t)blockIdx.x * BLK + threadIdx.x) / L;
    const int lane = threadIdx.x % L;
    if (r >= rows) return;  // whole groups of L lanes leave together
    DD acc;
    if (P1.ptr) {
        const DD d = row_dot_dd<L>(P1.ptr, P1.idx, P1.val, x1, nullptr, r, lane);
        dd_add_scaled(acc, a1, d);
    }
    if (P2.ptr) {
        const DD d = row_dot_dd<L>(P2.ptr, P2.idx, P2.val, x2, x2lo, r, lane);
        dd_add_scaled(acc, a2, d);
    }
    if (lane != 0) return;
    if (v1) dd_fma(acc, c1, v1[r]);
    if (v2) dd_fma(acc, c2, v2[r]);
    double h, l;
    two_sum(acc.s, acc.c, h, l);
    out_hi[r] = h;
    if (out_lo) out_lo[r] = l;
}

hipError_t combo_dd(int64_t rows, const DevCSR *P1, const double *x1, double a1, const DevCSR *P2, const double *x2,
                    const double *x2lo, double a2, const double *v1, double c1, const double *v2, double c2,
                    double *out_hi, double *out_lo, hipStream_t s)
{
    if (rows == 0) return hipSuccess;
    DevCSR none{};
    constexpr int L = 8;
    const int64_t threads = rows * L;
    hipLaunchKernelGGL(k_combo_dd<L>, dim3((unsigned)((threads + BLK - 1) / BLK)), dim3(BLK), 0, s, rows,
                       P1 ? *P1 : none, x1, a1, P2 ? *P2 : none, x2, x2lo, a2, v1, c1, v2, c2, out_hi, out_lo);
    return hipGetLastError();
}

hipError_t spmv_dd(const DevCSR &A, const double *x_hi, const double *x_lo, double *y_hi, double *y_lo,
                   hipStream_t s)
{
    return combo_dd(A.rows, nullptr, nullptr, 0.0, &A, x_hi, x_lo, 1.0, nullptr, 0.0, nullptr, 0.0, y_hi, y_lo, s);
}

// x += scale f, compensated: the rounding error of each addition goes to xlo
__global__ void k_add_f2d_comp(int64_t n, const float *__restrict__ f, double scale, double *__restrict__ x,
                               double *__restrict__ xlo)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s, e;
    two_sum(x[i], scale * (double)f[i], s, e);
    x[i] = s;
    xlo[i] += e;
}

hipError_t add_f2d_comp(int64_t n, const float *f, double scale, double *x, double *xlo, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_f2d_comp, dim3(nblk(n)), dim3(BLK), 0, s, n, f, scale, x, xlo);
    return hipGetLastError();
}

// ------------------------------------------------------ impressed field
// Moments f_l = sum_q w_q vol_T scale B(x_q) . W2_l(x_q) of one tet per thread
// (collapsed Gauss rule: P points with barycentrics lamq, weights wq summing to
// 1), into Pf[t][n2l].  W2_l = phi_l(lam) W~_abc with W~_abc = 2 (l_a X_bc
// - l_b X_ac + l_c X_ab), X_pq = grad l_p x grad l_q: the face functions the
// gather evaluates.
template <int K>
__global__ void k_impressed_rhs(DevMesh m, int P, const double *__restrict__ lamq, const double *__restrict__ wq,
                                const double *__restrict__ B, double scale, double *__restrict__ Pf)
{
    using O = Ord<K>;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m.nt) return;
    const double *g = &m.geo[16 * t];
    double X[6][3];
    for (int q = 0; q < 6; q++) {
        const double *ga = &g[4 * EA[q] + 1], *gb = &g[4 * EB[q] + 1];
        X[q][0] = ga[1] * gb[2] - ga[2] * gb[1];
        X[q][1] = ga[2] * gb[0] - ga[0] * gb[2];
        X[q][2] = ga[0] * gb[1] - ga[1] * gb[0];
    }
    // grad l_1 . (grad l_2 x grad l_3) = 1 / (6 vol), up to sign
    const double det = g[5] * X[5][0] + g[6] * X[5][1] + g[7] * X[5][2];
    const double vs = scale / (6.0 * fabs(det));
    double f[O::N2];
    for (int l = 0; l < O::N2; l++) f[l] = 0.0;
    for (int q = 0; q < P; q++) {
        const double *lam = &lamq[4 * q];
        const double *b = &B[3 * (t * P + q)];
        const double w = wq[q] * vs;
        double BX[6];
        for (int p = 0; p < 6; p++) BX[p] = b[0] * X[p][0] + b[1] * X[p][1] + b[2] * X[p][2];
        for (int fi = 0; fi < 4; fi++) {
            const int a = FV[fi][0], bb = FV[fi][1], c = FV[fi][2];
            const double tf = w * 2.0 * (lam[a] * BX[FP[fi][0]] - lam[bb] * BX[FP[fi][1]] + lam[c] * BX[FP[fi][2]]);
            if constexpr (K == 1) {
                f[fi] += tf;
            } else {
                f[3 * fi] += (4.0 * lam[a] - 1.0) * tf;
                f[3 * fi + 1] += (4.0 * lam[bb] - 1.0) * tf;
                f[3 * fi + 2] += (4.0 * lam[c] - 1.0) * tf;
                if (fi < 3) f[12 + fi] += 4.0 * lam[3 - fi] * tf;
            }
        }
    }
    for (int l = 0; l < O::N2; l++) Pf[t * O::N2 + l] = f[l];
}

hipError_t launch_impressed_rhs(int order, const DevMesh &m, int P, const double *lamq, const double *wq,
                                const double *B, double scale, double *Pf, hipStream_t s)
{
    if (m.nt == 0) return hipSuccess;
    const unsigned grid = (unsigned)((m.nt + BLK - 1) / BLK);
    if (order == 1)
        hipLaunchKernelGGL(k_impressed_rhs<1>, dim3(grid), dim3(BLK), 0, s, m, P, lamq, wq, B, scale, Pf);
    else
        hipLaunchKernelGGL(k_impressed_rhs<2>, dim3(grid), dim3(BLK), 0, s, m, P, lamq, wq, B, scale, Pf);
    return hipGetLastError();
}

// out = a .* b
__global__ void k_mul(int64_t n, const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] * b[i];
}

hipError_t mul(int64_t n, const double *a, const double *b, double *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mul, dim3(nblk(n)), dim3(BLK), 0, s, n, a, b, out);
    return hipGetLastError();
}

// Jacobi weights: 1 / (diagonal of A), or of A diag(D)^-1 A^T when Dinv is given
// (with A = K^T and Dinv = 1 / diag(*nu): the diagonal of K^T *nu K without
// *nu's off-diagonal part); 1 where the diagonal is not positive
__global__ void k_jacobi(int64_t rows, const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                         const double *__restrict__ val, const double *__restrict__ Dinv, double *__restrict__ dinv)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    double d = 0.0;
    for (int64_t k = ptr[r]; k < ptr[r + 1]; k++) {
        if (Dinv) d += val[k] * val[k] / Dinv[idx[k]];
        else if (idx[k] == r) d = val[k];
    }
    dinv[r] = d > 0.0 ? 1.0 / d : 1.0;
}

hipError_t jacobi(const DevCSR &A, const double *Dinv, double *dinv, hipStream_t s)
{
    if (A.rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_jacobi, dim3(nblk(A.rows)), dim3(BLK), 0, s, A.rows, A.ptr, A.idx, A.val, Dinv, dinv);
    return hipGetLastError();
}

// --------------------------------------------------- no-allocation scratch
// Device memory of the entry point that allocates nothing: one array per
// device (every device the library runs on holds its own copy until the process
// ends).  Host code never passes the array's name to a kernel: its device
// address comes from hipGetSymbolAddress, looked up once per device with that
// device current, and kept.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void **ptr)
{
    static std::mutex mu;
    static void *addr[NOALLOC_MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace fempic
