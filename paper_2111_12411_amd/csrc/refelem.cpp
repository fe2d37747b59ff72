// Reference-element tables for the order-k interpolatory Whitney bases
// (paper Appendix): basis descriptions, the local gradient / curl matrices
// (exact small rationals, recovered here numerically by least squares on a
// reference tet and snapped to 1/48), reference mass tensors (collapsed-
// coordinate Gauss quadrature, exact for the polynomial degrees involved) and
// the Gauss-Legendre rule of the deposit.
//
// Readings of the Appendix (its printed forms are partly garbled):
//  * Silvester argument n*lambda with n = k (W0), k+1 (W1), k+2 (W2), so the
//    interpolation nodes sit at alpha/n;
//  * lowest face form 2(l_a gb x gc + l_b gc x ga + l_c ga x gb) (unit flux);
//  * dropped dependent candidates: on face (a<b<c) the one on edge (b,c); among
//    the interior face candidates the one of face (1,2,3).
#include <cmath>
#include <cstring>
#include <mutex>

#include "fempic_impl.h"

namespace fempic {

const int LOC_EDGE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
const int LOC_FACE[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};

namespace {

struct V3 { double x, y, z; };
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// reference tet (0,0,0),(1,0,0),(0,1,0),(0,0,1)
const V3 GR[4] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

double qv_of(int qv, double qs, double qc, const double *l) { return qc + (qv >= 0 ? qs * l[qv] : 0.0); }

V3 w1_val(const W1Fn &f, const double *l)
{
    double Q = qv_of(f.qv, f.qs, f.qc, l);
    return Q * (l[f.a] * GR[f.b] - l[f.b] * GR[f.a]);
}

V3 w1_curl(const W1Fn &f, const double *l)
{
    double Q = qv_of(f.qv, f.qs, f.qc, l);
    V3 W = l[f.a] * GR[f.b] - l[f.b] * GR[f.a];
    V3 c = 2.0 * Q * cross(GR[f.a], GR[f.b]);
    if (f.qv >= 0) c = c + cross(f.qs * GR[f.qv], W);
    return c;
}

V3 w2_val(const W2Fn &f, const double *l)
{
    double Q = qv_of(f.qv, f.qs, f.qc, l);
    V3 s = l[f.a] * cross(GR[f.b], GR[f.c]) + l[f.b] * cross(GR[f.c], GR[f.a]) + l[f.c] * cross(GR[f.a], GR[f.b]);
    return 2.0 * Q * s;
}

V3 w0_grad(const W0Fn &f, const double *l)
{
    if (f.b < 0) return f.c1 * (2.0 * f.cs * l[f.a] + f.cc) * GR[f.a];
    return f.c1 * (l[f.b] * GR[f.a] + l[f.a] * GR[f.b]);
}

// deterministic sample points (barycentric) inside the reference tet
void sample_points(int n, std::vector<double> &lam)
{
    lam.resize(4 * n);
    uint64_t s = 0x9E3779B97F4A7C15ull;
    auto rnd = [&]() {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return ((s >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    };
    for (int p = 0; p < n; p++) {
        double w[4], t = 0;
        for (int k = 0; k < 4; k++) { w[k] = -std::log(rnd()); t += w[k]; }
        for (int k = 0; k < 4; k++) lam[4 * p + k] = w[k] / t;
    }
}

// Solve min |A x - b| for each of ncol right-hand sides via normal equations
// (A: m x n row-major, B: m x ncol); X: n x ncol.
void least_squares(const std::vector<double> &A, int m, int n, const std::vector<double> &B, int ncol,
                   std::vector<double> &X)
{
    std::vector<double> N(n * n, 0.0), R(n * ncol, 0.0);
    for (int r = 0; r < m; r++)
        for (int i = 0; i < n; i++) {
            for (int j = 0; j < n; j++) N[i * n + j] += A[r * n + i] * A[r * n + j];
            for (int c = 0; c < ncol; c++) R[i * ncol + c] += A[r * n + i] * B[r * ncol + c];
        }
    // Cholesky
    for (int j = 0; j < n; j++) {
        double d = N[j * n + j];
        for (int k = 0; k < j; k++) d -= N[j * n + k] * N[j * n + k];
        if (!(d > 0)) throw Error(FEMPIC_EMESH, "reference basis is rank deficient");
        d = std::sqrt(d);
        N[j * n + j] = d;
        for (int i = j + 1; i < n; i++) {
            double s = N[i * n + j];
            for (int k = 0; k < j; k++) s -= N[i * n + k] * N[j * n + k];
            N[i * n + j] = s / d;
        }
    }
    X.assign(n * ncol, 0.0);
    for (int c = 0; c < ncol; c++) {
        std::vector<double> y(n);
        for (int i = 0; i < n; i++) {
            double s = R[i * ncol + c];
            for (int k = 0; k < i; k++) s -= N[i * n + k] * y[k];
            y[i] = s / N[i * n + i];
        }
        for (int i = n - 1; i >= 0; i--) {
            double s = y[i];
            for (int k = i + 1; k < n; k++) s -= N[k * n + i] * X[k * ncol + c];
            X[i * ncol + c] = s / N[i * n + i];
        }
    }
}

double snap48(double x)
{
    double r = std::nearbyint(x * 48.0) / 48.0;
    if (std::fabs(r - x) > 1e-9) throw Error(FEMPIC_EMESH, "local exterior derivative is not a small rational");
    return r;
}

// collapsed-coordinate Gauss rule on the reference tet (weights sum to 1/6)
void tet_rule(int n, std::vector<double> &lam, std::vector<double> &w);

void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; i++) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pn = (n == 1) ? z : p1;
            double pnm1 = (n == 1) ? 1.0 : p0;
            dp = n * (z * pn - pnm1) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        x[n - 1 - i] = 0.5 * (z + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2)P'^2) halved for [0,1]
    }
}

void tet_rule(int n, std::vector<double> &lam, std::vector<double> &w)
{
    std::vector<double> gx, gw;
    gauss_legendre01(n, gx, gw);
    lam.clear();
    w.clear();
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                double u = gx[i], v = gx[j], t = gx[k];
                double X = u, Y = v * (1 - u), Z = t * (1 - u) * (1 - v);
                double J = (1 - u) * (1 - u) * (1 - v);
                lam.push_back(1 - X - Y - Z);
                lam.push_back(X);
                lam.push_back(Y);
                lam.push_back(Z);
                w.push_back(gw[i] * gw[j] * gw[k] * J);
            }
}

RefElem make(int k)
{
    RefElem R;
    R.order = k;
    if (k == 1) {
        for (auto &e : LOC_EDGE) R.w1.push_back({e[0], e[1], -1, 0.0, 1.0});
        for (auto &f : LOC_FACE) R.w2.push_back({f[0], f[1], f[2], -1, 0.0, 1.0});
        for (int a = 0; a < 4; a++) R.w0.push_back({a, -1, 1.0, 0.0, 1.0});
    } else if (k == 2) {
        for (auto &e : LOC_EDGE) {
            R.w1.push_back({e[0], e[1], e[0], 3.0, -1.0});  // alpha 2 on the lower vertex
            R.w1.push_back({e[0], e[1], e[1], 3.0, -1.0});  // alpha 2 on the upper vertex
        }
        for (auto &f : LOC_FACE) {
            R.w1.push_back({f[0], f[1], f[2], 3.0, 0.0});   // 3 l_c W_ab
            R.w1.push_back({f[0], f[2], f[1], 3.0, 0.0});   // 3 l_b W_ac
        }
        for (auto &f : LOC_FACE)
            for (int x = 0; x < 3; x++) R.w2.push_back({f[0], f[1], f[2], f[x], 4.0, -1.0});
        for (int fi = 0; fi < 3; fi++) {
            const int *f = LOC_FACE[fi];
            int d = 6 - f[0] - f[1] - f[2];
            R.w2.push_back({f[0], f[1], f[2], d, 4.0, 0.0});  // 4 l_d W_f
        }
        for (int a = 0; a < 4; a++) R.w0.push_back({a, -1, 1.0, 2.0, -1.0});
        for (auto &e : LOC_EDGE) R.w0.push_back({e[0], e[1], 2.0, 0.0, 0.0});
    } else {
        throw Error(FEMPIC_EINVAL, "order must be 1 or 2");
    }
    R.n1 = (int)R.w1.size();
    R.n2 = (int)R.w2.size();
    R.n0 = (int)R.w0.size();

    // local curl and gradient matrices by least squares on sample points
    const int P = 40;
    std::vector<double> lam;
    sample_points(P, lam);
    {
        std::vector<double> A(3 * P * R.n2), B(3 * P * R.n1), X;
        for (int p = 0; p < P; p++) {
            const double *l = &lam[4 * p];
            for (int j = 0; j < R.n2; j++) {
                V3 v = w2_val(R.w2[j], l);
                A[(3 * p + 0) * R.n2 + j] = v.x;
                A[(3 * p + 1) * R.n2 + j] = v.y;
                A[(3 * p + 2) * R.n2 + j] = v.z;
            }
            for (int j = 0; j < R.n1; j++) {
                V3 v = w1_curl(R.w1[j], l);
                B[(3 * p + 0) * R.n1 + j] = v.x;
                B[(3 * p + 1) * R.n1 + j] = v.y;
                B[(3 * p + 2) * R.n1 + j] = v.z;
            }
        }
        least_squares(A, 3 * P, R.n2, B, R.n1, X);
        R.K.resize(R.n2 * R.n1);
        for (int i = 0; i < R.n2 * R.n1; i++) R.K[i] = snap48(X[i]);
    }
    {
        std::vector<double> A(3 * P * R.n1), B(3 * P * R.n0), X;
        for (int p = 0; p < P; p++) {
            const double *l = &lam[4 * p];
            for (int j = 0; j < R.n1; j++) {
                V3 v = w1_val(R.w1[j], l);
                A[(3 * p + 0) * R.n1 + j] = v.x;
                A[(3 * p + 1) * R.n1 + j] = v.y;
                A[(3 * p + 2) * R.n1 + j] = v.z;
            }
            for (int j = 0; j < R.n0; j++) {
                V3 v = w0_grad(R.w0[j], l);
                B[(3 * p + 0) * R.n0 + j] = v.x;
                B[(3 * p + 1) * R.n0 + j] = v.y;
                B[(3 * p + 2) * R.n0 + j] = v.z;
            }
        }
        least_squares(A, 3 * P, R.n1, B, R.n0, X);
        R.G.resize(R.n1 * R.n0);
        for (int i = 0; i < R.n1 * R.n0; i++) R.G[i] = snap48(X[i]);
    }
    // K G must vanish exactly (de Rham sequence)
    for (int l = 0; l < R.n2; l++)
        for (int j = 0; j < R.n0; j++) {
            double s = 0;
            for (int i = 0; i < R.n1; i++) s += R.K[l * R.n1 + i] * R.G[i * R.n0 + j];
            if (std::fabs(s) > 1e-12) throw Error(FEMPIC_EMESH, "local curl of gradient is not zero");
        }

    // reference mass tensors: int_ref phi_i^m phi_j^n (reference volume 1/6 -> equals (1/6V) int_T)
    std::vector<double> ql, qw;
    tet_rule(6, ql, qw);
    const int NQ = (int)qw.size();
    R.C1.assign((size_t)R.n1 * R.n1 * 16, 0.0);
    R.C2.assign((size_t)R.n2 * R.n2 * 36, 0.0);
    std::vector<double> phi(R.n1 * 4), psi(R.n2 * 6);
    for (int q = 0; q < NQ; q++) {
        const double *l = &ql[4 * q];
        std::fill(phi.begin(), phi.end(), 0.0);
        for (int i = 0; i < R.n1; i++) {
            const W1Fn &f = R.w1[i];
            double Q = qv_of(f.qv, f.qs, f.qc, l);
            phi[4 * i + f.b] += Q * l[f.a];
            phi[4 * i + f.a] -= Q * l[f.b];
        }
        std::fill(psi.begin(), psi.end(), 0.0);
        auto pair_id = [](int m, int n) {
            for (int p = 0; p < 6; p++)
                if (LOC_EDGE[p][0] == m && LOC_EDGE[p][1] == n) return p;
            return -1;
        };
        for (int l2 = 0; l2 < R.n2; l2++) {
            const W2Fn &f = R.w2[l2];
            double Q = 2.0 * qv_of(f.qv, f.qs, f.qc, l);
            psi[6 * l2 + pair_id(f.b, f.c)] += Q * l[f.a];
            psi[6 * l2 + pair_id(f.a, f.c)] -= Q * l[f.b];
            psi[6 * l2 + pair_id(f.a, f.b)] += Q * l[f.c];
        }
        for (int i = 0; i < R.n1; i++)
            for (int j = 0; j < R.n1; j++)
                for (int m = 0; m < 4; m++)
                    for (int n = 0; n < 4; n++)
                        R.C1[((size_t)(i * R.n1 + j) * 4 + m) * 4 + n] += qw[q] * phi[4 * i + m] * phi[4 * j + n];
        for (int i = 0; i < R.n2; i++)
            for (int j = 0; j < R.n2; j++)
                for (int p = 0; p < 6; p++)
                    for (int r = 0; r < 6; r++)
                        R.C2[((size_t)(i * R.n2 + j) * 6 + p) * 6 + r] += qw[q] * psi[6 * i + p] * psi[6 * j + r];
    }
    // face tensors: (1/A) int over the face opposite vertex o of phi_i^m phi_j^n,
    // on a collapsed Gauss rule of the triangle (exact for degree 2k)
    {
        std::vector<double> gx, gw;
        gauss_legendre01(k + 2, gx, gw);
        R.F1.assign((size_t)4 * R.n1 * R.n1 * 16, 0.0);
        std::vector<double> phi1(R.n1 * 4);
        for (int o = 0; o < 4; o++) {
            int fv[3], c = 0;
            for (int v = 0; v < 4; v++)
                if (v != o) fv[c++] = v;
            double *F = &R.F1[(size_t)o * R.n1 * R.n1 * 16];
            for (size_t a = 0; a < gx.size(); a++)
                for (size_t b = 0; b < gx.size(); b++) {
                    // (u, v) on the square onto the triangle; the average over it has weight 2 (1-u)
                    const double u = gx[a], v = gx[b], wq = 2.0 * gw[a] * gw[b] * (1.0 - u);
                    double l[4] = {0, 0, 0, 0};
                    l[fv[0]] = u;
                    l[fv[1]] = v * (1.0 - u);
                    l[fv[2]] = (1.0 - u) * (1.0 - v);
                    std::fill(phi1.begin(), phi1.end(), 0.0);
                    for (int i = 0; i < R.n1; i++) {
                        const W1Fn &f = R.w1[i];
                        const double Q = qv_of(f.qv, f.qs, f.qc, l);
                        phi1[4 * i + f.b] += Q * l[f.a];
                        phi1[4 * i + f.a] -= Q * l[f.b];
                    }
                    for (int i = 0; i < R.n1; i++)
                        for (int j = 0; j < R.n1; j++)
                            for (int m = 0; m < 4; m++)
                                for (int n = 0; n < 4; n++)
                                    F[((size_t)(i * R.n1 + j) * 4 + m) * 4 + n] += wq * phi1[4 * i + m] * phi1[4 * j + n];
                }
        }
    }
    gauss_legendre01(2 * k + 2, R.glx, R.glw);
    return R;
}

}  // namespace

void impressed_rule(int n, std::vector<double> &lam, std::vector<double> &w)
{
    tet_rule(n, lam, w);
    for (double &x : w) x *= 6.0;
}

const RefElem &ref_elem(int order)
{
    static RefElem r1, r2;
    static std::once_flag f1, f2;
    if (order == 1) {
        std::call_once(f1, [] { r1 = make(1); });
        return r1;
    }
    if (order == 2) {
        std::call_once(f2, [] { r2 = make(2); });
        return r2;
    }
    throw Error(FEMPIC_EINVAL, "order must be 1 or 2");
}

}  // namespace fempic
