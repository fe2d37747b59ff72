// Global sparse operators of the implicit field update (paper Sec. III-A,
// Sec. III-B) in CSR over the internal DoF numbering:
//   *eps  = eps0 <W1_i, W1_j>,  *nu = (1/mu0) <W2_i, W2_j>,
//   K     = local curl matrix by assignment (curl W1_j = sum_l K_lj W2_l),
//   A     = *eps + c dt^2 K^T *nu K  (assembled element by element; c = (beta/gamma)^2
//           of the Newmark-beta scheme, 1/4 for gamma = 1/2, beta = 1/4),
//   *nu and K^T apart (the field update applies K^T to *nu u in double-double,
//   so that G^T of it vanishes as in exact arithmetic), and G^T by assignment,
//   scaled to integer entries.
// Only W1 DoFs off the PEC walls are unknowns; W0 rows of the Gauss check are
// the interior nodal DoFs.  Also the explicit time-step bound and the
// DoF -> (tet, local) incidence lists that the deterministic deposit scatter uses.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <thread>
#include <tuple>

#include "fempic_impl.h"

namespace fempic {

void element_mass(const HostMesh &m, int64_t t, double *M1, double *M2)
{
    const RefElem &R = ref_elem(m.order);
    const double *geo = &m.geo[16 * t];
    double g[4][4];
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++)
            g[a][b] = geo[4 * a + 1] * geo[4 * b + 1] + geo[4 * a + 2] * geo[4 * b + 2] + geo[4 * a + 3] * geo[4 * b + 3];
    const double six_v = 6.0 * m.vol[t];
    const int n1 = R.n1, n2 = R.n2;
    for (int i = 0; i < n1; i++)
        for (int j = 0; j < n1; j++) {
            const double *c = &R.C1[(size_t)(i * n1 + j) * 16];
            double s = 0;
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) s += c[4 * a + b] * g[a][b];
            M1[i * n1 + j] = six_v * s;
        }
    double G2[6][6];
    for (int p = 0; p < 6; p++)
        for (int q = 0; q < 6; q++) {
            int a = LOC_EDGE[p][0], b = LOC_EDGE[p][1], c = LOC_EDGE[q][0], d = LOC_EDGE[q][1];
            G2[p][q] = g[a][c] * g[b][d] - g[a][d] * g[b][c];
        }
    for (int i = 0; i < n2; i++)
        for (int j = 0; j < n2; j++) {
            const double *c = &R.C2[(size_t)(i * n2 + j) * 36];
            double s = 0;
            for (int p = 0; p < 6; p++)
                for (int q = 0; q < 6; q++) s += c[6 * p + q] * G2[p][q];
            M2[i * n2 + j] = six_v * s;
        }
}

namespace {

// element curl-curl S = K^T M2 K (n1 x n1) and K^T M2 (n1 x n2)
void curl_products(const RefElem &R, const double *M2, double *S, double *KtM2)
{
    const int n1 = R.n1, n2 = R.n2;
    for (int i = 0; i < n1; i++)
        for (int l = 0; l < n2; l++) {
            double s = 0;
            for (int m = 0; m < n2; m++) s += R.K[m * n1 + i] * M2[m * n2 + l];
            KtM2[i * n2 + l] = s;
        }
    for (int i = 0; i < n1; i++)
        for (int j = 0; j < n1; j++) {
            double s = 0;
            for (int l = 0; l < n2; l++) s += KtM2[i * n2 + l] * R.K[l * n1 + j];
            S[i * n1 + j] = s;
        }
}

// Symmetric eigenvalues by cyclic Jacobi (small n); returns the largest.
double jacobi_max_eig(std::vector<double> a, int n)
{
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) (i == j ? tot : off) += a[i * n + j] * a[i * n + j];
        if (off <= 1e-30 * (tot + off)) break;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) {
                double apq = a[p * n + q];
                if (apq == 0.0) continue;
                double th = 0.5 * (a[q * n + q] - a[p * n + p]) / apq;
                double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; k++) {
                    double akp = a[k * n + p], akq = a[k * n + q];
                    a[k * n + p] = c * akp - s * akq;
                    a[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; k++) {
                    double apk = a[p * n + k], aqk = a[q * n + k];
                    a[p * n + k] = c * apk - s * aqk;
                    a[q * n + k] = s * apk + c * aqk;
                }
            }
    }
    double mx = a[0];
    for (int i = 1; i < n; i++) mx = std::max(mx, a[i * n + i]);
    return mx;
}

// Run f(lo, hi) over [0, n) split into contiguous chunks on the host's threads.
template <typename F>
void parallel_for(int64_t n, F f)
{
    int nth = (int)std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
    nth = (int)std::max<int64_t>(1, std::min<int64_t>(nth, n));
    std::vector<std::thread> th;
    for (int k = 0; k < nth; k++) {
        int64_t lo = n * k / nth, hi = n * (k + 1) / nth;
        th.emplace_back([=, &f] { f(lo, hi); });
    }
    for (auto &t : th) t.join();
}

// row -> (tet, local row) incidence, tets ascending
struct RowInc {
    std::vector<int64_t> ptr, idx;  // idx = t * nr + i
};

template <typename RMap>
RowInc row_incidence(const HostMesh &m, int64_t rows, int nr, RMap rmap)
{
    RowInc ri;
    ri.ptr.assign(rows + 1, 0);
    for (int64_t t = 0; t < m.nt; t++)
        for (int i = 0; i < nr; i++) {
            int64_t r = rmap(t, i);
            if (r >= 0) ri.ptr[r + 1]++;
        }
    for (int64_t r = 0; r < rows; r++) ri.ptr[r + 1] += ri.ptr[r];
    ri.idx.assign(ri.ptr[rows], 0);
    std::vector<int64_t> fill(ri.ptr.begin(), ri.ptr.end() - 1);
    for (int64_t t = 0; t < m.nt; t++)
        for (int i = 0; i < nr; i++) {
            int64_t r = rmap(t, i);
            if (r >= 0) ri.idx[fill[r]++] = t * nr + i;
        }
    return ri;
}

// CSR from element contributions, row-parallel.  Each row gathers the entries
// of its incident tets in ascending tet order (deterministic sums).  cmap gives
// the global column of a local column (or -1); mask (optional) drops structural
// zeros; `assign` stores the value (every tet must agree) instead of adding.
template <typename CMap, typename Val>
void build_csr(const RowInc &ri, int64_t rows, int64_t cols, int nr, int nc, CMap cmap, const double *mask, Val val,
               bool assign, CSR &A)
{
    A.rows = rows;
    A.cols = cols;
    const int nth = 64;
    std::vector<std::vector<int32_t>> cidx(nth);
    std::vector<std::vector<double>> cval(nth);
    std::vector<int64_t> rowlen(rows, 0);
    std::vector<int> bad(nth, 0);
    parallel_for(nth, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; c++) {
            const int64_t r0 = rows * c / nth, r1 = rows * (c + 1) / nth;
            std::vector<int32_t> colv;
            std::vector<double> vals;
            std::vector<uint8_t> set;
            for (int64_t r = r0; r < r1; r++) {
                colv.clear();
                for (int64_t k = ri.ptr[r]; k < ri.ptr[r + 1]; k++) {
                    const int64_t t = ri.idx[k] / nr;
                    const int i = (int)(ri.idx[k] % nr);
                    for (int j = 0; j < nc; j++) {
                        if (mask && mask[i * nc + j] == 0.0) continue;
                        const int64_t cc = cmap(t, j);
                        if (cc >= 0) colv.push_back((int32_t)cc);
                    }
                }
                std::sort(colv.begin(), colv.end());
                colv.erase(std::unique(colv.begin(), colv.end()), colv.end());
                vals.assign(colv.size(), 0.0);
                set.assign(colv.size(), 0);
                for (int64_t k = ri.ptr[r]; k < ri.ptr[r + 1]; k++) {
                    const int64_t t = ri.idx[k] / nr;
                    const int i = (int)(ri.idx[k] % nr);
                    for (int j = 0; j < nc; j++) {
                        if (mask && mask[i * nc + j] == 0.0) continue;
                        const int64_t cc = cmap(t, j);
                        if (cc < 0) continue;
                        const size_t p = std::lower_bound(colv.begin(), colv.end(), (int32_t)cc) - colv.begin();
                        const double v = val(t, i, j);
                        if (assign) {
                            if (set[p] && vals[p] != v) bad[c] = 1;
                            vals[p] = v;
                            set[p] = 1;
                        } else {
                            vals[p] += v;
                        }
                    }
                }
                rowlen[r] = (int64_t)colv.size();
                cidx[c].insert(cidx[c].end(), colv.begin(), colv.end());
                cval[c].insert(cval[c].end(), vals.begin(), vals.end());
            }
        }
    });
    for (int c = 0; c < nth; c++)
        if (bad[c]) throw Error(FEMPIC_EMESH, "local exterior derivative disagrees between tets");
    A.ptr.assign(rows + 1, 0);
    for (int64_t r = 0; r < rows; r++) A.ptr[r + 1] = A.ptr[r] + rowlen[r];
    A.idx.resize(A.ptr[rows]);
    A.val.resize(A.ptr[rows]);
    int64_t off = 0;
    for (int c = 0; c < nth; c++) {
        std::copy(cidx[c].begin(), cidx[c].end(), A.idx.begin() + off);
        std::copy(cval[c].begin(), cval[c].end(), A.val.begin() + off);
        off += (int64_t)cidx[c].size();
    }
}

void incidence(const HostMesh &m, int64_t ndof, int nloc, const std::vector<int32_t> &map, std::vector<int64_t> &ptr,
               std::vector<int32_t> &idx)
{
    ptr.assign(ndof + 1, 0);
    for (int64_t t = 0; t < m.nt; t++)
        for (int i = 0; i < nloc; i++) {
            int32_t d = map[t * nloc + i];
            if (d < ndof) ptr[d + 1]++;
        }
    for (int64_t d = 0; d < ndof; d++) ptr[d + 1] += ptr[d];
    idx.assign(ptr[ndof], 0);
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t t = 0; t < m.nt; t++)
        for (int i = 0; i < nloc; i++) {
            int32_t d = map[t * nloc + i];
            if (d < ndof) idx[fill[d]++] = (int32_t)(t * nloc + i);
        }
}

}  // namespace

double cfl_bound(const HostMesh &m)
{
    const RefElem &R = ref_elem(m.order);
    const int n1 = R.n1, n2 = R.n2;
    std::vector<double> M1(n1 * n1), M2(n2 * n2), S(n1 * n1), KtM2(n1 * n2), L(n1 * n1), C(n1 * n1), T(n1 * n1);
    // the Kuhn cube is 6 translated tet shapes: the first hex holds all of them
    const int64_t nt = m.is_cube ? std::min<int64_t>(6, m.nt) : m.nt;
    double lmax = 0;
    for (int64_t t = 0; t < nt; t++) {
        element_mass(m, t, M1.data(), M2.data());
        curl_products(R, M2.data(), S.data(), KtM2.data());
        // Cholesky of eps0 M1
        std::fill(L.begin(), L.end(), 0.0);
        for (int j = 0; j < n1; j++) {
            double d = EPS0 * M1[j * n1 + j];
            for (int k = 0; k < j; k++) d -= L[j * n1 + k] * L[j * n1 + k];
            d = std::sqrt(d);
            L[j * n1 + j] = d;
            for (int i = j + 1; i < n1; i++) {
                double s = EPS0 * M1[i * n1 + j];
                for (int k = 0; k < j; k++) s -= L[i * n1 + k] * L[j * n1 + k];
                L[i * n1 + j] = s / d;
            }
        }
        // C = L^{-1} (S/mu0) L^{-T}
        for (int c = 0; c < n1; c++)  // T = L^{-1} S (column by column)
            for (int i = 0; i < n1; i++) {
                double s = S[i * n1 + c] / MU0;
                for (int k = 0; k < i; k++) s -= L[i * n1 + k] * T[k * n1 + c];
                T[i * n1 + c] = s / L[i * n1 + i];
            }
        for (int r = 0; r < n1; r++)  // C = T L^{-T}: solve L C^T = T^T
            for (int i = 0; i < n1; i++) {
                double s = T[r * n1 + i];
                for (int k = 0; k < i; k++) s -= L[i * n1 + k] * C[r * n1 + k];
                C[r * n1 + i] = s / L[i * n1 + i];
            }
        for (int i = 0; i < n1; i++)
            for (int j = 0; j < i; j++) C[i * n1 + j] = C[j * n1 + i] = 0.5 * (C[i * n1 + j] + C[j * n1 + i]);
        lmax = std::max(lmax, jacobi_max_eig(C, n1));
    }
    return 2.0 / std::sqrt(lmax);
}

// Surface impedance matrix [*I]_ij = Y int_walls (n x W1_i) . (n x W1_j) dS
// (Sec. III-A) over the first n1s internal W1 DoFs: per wall face of a tet,
// (n x u) . (n x v) = u . (I - n n^T) v and W1 = sum_m phi^m grad l_m, so the
// face's element matrix is Y A sum_mn F1[o][i][j][m][n] (grad l_m . P grad l_n)
// with o the vertex opposite the face and A its area.
void surface_impedance(const HostMesh &m, const RefElem &R, int64_t n1s, double Y, CSR &Z)
{
    const int n1 = R.n1;
    std::vector<std::tuple<int32_t, int32_t, double>> trip;
    std::vector<double> el(n1 * n1);
    for (int64_t t = 0; t < m.nt; t++)
        for (int lf = 0; lf < 4; lf++) {
            if (!m.bface[m.tet_face[4 * t + lf]]) continue;
            const int o = 3 - lf;  // local face lf lies opposite vertex 3 - lf
            const double *g = &m.geo[16 * t];
            const double *gn = g + 4 * o + 1;
            const double gg = gn[0] * gn[0] + gn[1] * gn[1] + gn[2] * gn[2];
            double e1[3], e2[3], cr[3];
            const int32_t *tv = &m.tets[4 * t];
            const int va = tv[LOC_FACE[lf][0]], vb = tv[LOC_FACE[lf][1]], vc = tv[LOC_FACE[lf][2]];
            for (int c = 0; c < 3; c++) {
                e1[c] = m.xyz[3 * vb + c] - m.xyz[3 * va + c];
                e2[c] = m.xyz[3 * vc + c] - m.xyz[3 * va + c];
            }
            cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
            cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
            cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
            const double area = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            // grad l_m . P grad l_n with P = I - n n^T, n along grad l_o
            double gpg[4][4];
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    const double *ga = g + 4 * a + 1, *gb = g + 4 * b + 1;
                    const double d = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
                    const double na = ga[0] * gn[0] + ga[1] * gn[1] + ga[2] * gn[2];
                    const double nb = gb[0] * gn[0] + gb[1] * gn[1] + gb[2] * gn[2];
                    gpg[a][b] = d - na * nb / gg;
                }
            const double *F = &R.F1[(size_t)o * n1 * n1 * 16];
            for (int i = 0; i < n1; i++)
                for (int j = 0; j < n1; j++) {
                    double v = 0.0;
                    for (int a = 0; a < 4; a++)
                        for (int b = 0; b < 4; b++) v += F[((size_t)(i * n1 + j) * 4 + a) * 4 + b] * gpg[a][b];
                    el[i * n1 + j] = Y * area * v;
                }
            // symmetric as the exact matrix is (the two sums round in different orders)
            for (int i = 0; i < n1; i++)
                for (int j = i + 1; j < n1; j++) el[i * n1 + j] = el[j * n1 + i] = 0.5 * (el[i * n1 + j] + el[j * n1 + i]);
            for (int i = 0; i < n1; i++) {
                const int32_t r = m.map1[t * n1 + i];
                if (r >= n1s) continue;
                for (int j = 0; j < n1; j++) {
                    const int32_t c = m.map1[t * n1 + j];
                    if (c < n1s && el[i * n1 + j] != 0.0) trip.emplace_back(r, c, el[i * n1 + j]);
                }
            }
        }
    std::sort(trip.begin(), trip.end(), [](const auto &x, const auto &y) {
        return std::get<0>(x) != std::get<0>(y) ? std::get<0>(x) < std::get<0>(y) : std::get<1>(x) < std::get<1>(y);
    });
    Z.rows = Z.cols = n1s;
    Z.ptr.assign(n1s + 1, 0);
    Z.idx.clear();
    Z.val.clear();
    for (size_t k = 0; k < trip.size(); k++) {
        const auto [r, c, v] = trip[k];
        if (!Z.idx.empty() && k > 0 && std::get<0>(trip[k - 1]) == r && Z.idx.back() == c) {
            Z.val.back() += v;  // faces of a tet share DoFs on their common edge
        } else {
            Z.idx.push_back(c);
            Z.val.push_back(v);
            Z.ptr[r + 1]++;
        }
    }
    for (int64_t r = 0; r < n1s; r++) Z.ptr[r + 1] += Z.ptr[r];
}

void assemble(const HostMesh &m, double dt, Operators &ops, double c_dt2, bool absorbing)
{
    const RefElem &R = ref_elem(m.order);
    const int n1 = R.n1, n2 = R.n2, n0 = R.n0;
    // the unknown W1 DoFs (see Operators): the internal numbering puts the wall ones last
    const int64_t N1i = absorbing ? m.N1 : m.N1_int, N0i = m.N0_int, nt = m.nt;
    ops.n1s = N1i;
    auto w1int = [&](int64_t t, int i) -> int64_t {
        int32_t d = m.map1[t * n1 + i];
        return d < N1i ? d : -1;
    };
    auto w2 = [&](int64_t t, int l) -> int64_t { return m.map2[t * n2 + l]; };
    auto w0int = [&](int64_t t, int j) -> int64_t {
        int32_t d = m.map0[t * n0 + j];
        return d < N0i ? d : -1;
    };
    // element matrices of every tet: eps0 M1, curl-curl S / mu0, K^T M2 / mu0
    // (uninitialised storage: every entry is written by the parallel loop below)
    std::unique_ptr<double[]> Mel(new double[(size_t)nt * n1 * n1]), Sel(new double[(size_t)nt * n1 * n1]),
        Nel(new double[(size_t)nt * n2 * n2]);
    parallel_for(nt, [&](int64_t t0, int64_t t1) {
        std::vector<double> M1(n1 * n1), M2(n2 * n2), S(n1 * n1), KtM2(n1 * n2);
        for (int64_t t = t0; t < t1; t++) {
            element_mass(m, t, M1.data(), M2.data());
            curl_products(R, M2.data(), S.data(), KtM2.data());
            double *me = &Mel[(size_t)t * n1 * n1], *se = &Sel[(size_t)t * n1 * n1], *ne = &Nel[(size_t)t * n2 * n2];
            for (int i = 0; i < n1 * n1; i++) {
                me[i] = EPS0 * M1[i];
                se[i] = S[i] / MU0;
            }
            for (int i = 0; i < n2 * n2; i++) ne[i] = M2[i] / MU0;
        }
    });
    const double c_stiff = c_dt2 * dt * dt;
    RowInc r1 = row_incidence(m, N1i, n1, w1int);
    build_csr(r1, N1i, N1i, n1, n1, w1int, nullptr,
              [&](int64_t t, int i, int j) {
                  const size_t k = ((size_t)t * n1 + i) * n1 + j;
                  return Mel[k] + c_stiff * Sel[k];
              },
              false, ops.A);
    build_csr(r1, N1i, N1i, n1, n1, w1int, nullptr,
              [&](int64_t t, int i, int j) { return Mel[((size_t)t * n1 + i) * n1 + j]; }, false, ops.Meps);
    RowInc r2 = row_incidence(m, m.N2, n2, w2);
    build_csr(r2, m.N2, m.N2, n2, n2, w2, nullptr,
              [&](int64_t t, int l, int q) { return Nel[((size_t)t * n2 + l) * n2 + q]; }, false, ops.Mnu);
    build_csr(r2, m.N2, N1i, n2, n1, w1int, R.K.data(), [&](int64_t, int l, int i) { return R.K[l * n1 + i]; },
              true, ops.K);
    std::vector<double> KT(n1 * n2);
    for (int i = 0; i < n1; i++)
        for (int l = 0; l < n2; l++) KT[i * n2 + l] = R.K[l * n1 + i];
    build_csr(r1, N1i, m.N2, n1, n2, w2, KT.data(), [&](int64_t, int i, int l) { return KT[i * n2 + l]; }, true,
              ops.Kt);
    // G's entries are rationals (thirds at order 2); scaled to integers they make
    // the Gauss check's products exact
    ops.gscale = 0.0;
    for (int sc = 1; sc <= 12 && ops.gscale == 0.0; sc++) {
        bool ok = true;
        for (double gv : R.G) ok = ok && std::fabs(gv * sc - std::nearbyint(gv * sc)) < 1e-9;
        if (ok) ops.gscale = sc;
    }
    if (ops.gscale == 0.0) throw Error(FEMPIC_EMESH, "gradient matrix without a small integer scale");
    std::vector<double> Gt(n0 * n1);
    for (int j = 0; j < n0; j++)
        for (int i = 0; i < n1; i++) Gt[j * n1 + i] = std::nearbyint(R.G[i * n0 + j] * ops.gscale);
    RowInc r0 = row_incidence(m, N0i, n0, w0int);
    build_csr(r0, N0i, N1i, n0, n1, w1int, Gt.data(), [&](int64_t, int j, int i) { return Gt[j * n1 + i]; }, true,
              ops.Gt);
    ops.Z = CSR{};
    if (absorbing) {
        // wall admittance of free space; the step takes the impedance term at
        // the half step, as it takes the curl-curl one
        surface_impedance(m, R, N1i, std::sqrt(EPS0 / MU0), ops.Z);
        for (int64_t r = 0; r < N1i; r++)
            for (int64_t k = ops.Z.ptr[r]; k < ops.Z.ptr[r + 1]; k++) {
                const int32_t *b = ops.A.idx.data() + ops.A.ptr[r], *e = ops.A.idx.data() + ops.A.ptr[r + 1];
                const int32_t *p = std::lower_bound(b, e, ops.Z.idx[k]);
                if (p == e || *p != ops.Z.idx[k]) throw Error(FEMPIC_EMESH, "impedance entry outside the field matrix");
                ops.A.val[p - ops.A.idx.data()] += 0.5 * dt * ops.Z.val[k];
            }
    }
    ops.Adiag_inv.assign(N1i, 0.0);
    for (int64_t r = 0; r < N1i; r++) {
        const int32_t *b = ops.A.idx.data() + ops.A.ptr[r], *e = ops.A.idx.data() + ops.A.ptr[r + 1];
        const int32_t *p = std::lower_bound(b, e, (int32_t)r);
        if (p == e || *p != r) throw Error(FEMPIC_EMESH, "field matrix row without a diagonal");
        const double d = ops.A.val[p - ops.A.idx.data()];
        if (!(d > 0)) throw Error(FEMPIC_EMESH, "field matrix has a non-positive diagonal");
        ops.Adiag_inv[r] = 1.0 / d;
    }
    incidence(m, N1i, n1, m.map1, ops.inc_ptr, ops.inc_idx);
    incidence(m, N0i, n0, m.map0, ops.inc0_ptr, ops.inc0_idx);
}

void assemble_impressed(const HostMesh &m, ImpressedOps &io)
{
    const RefElem &R = ref_elem(m.order);
    const int n1 = R.n1, n2 = R.n2;
    auto w1all = [&](int64_t t, int i) -> int64_t { return m.map1[t * n1 + i]; };
    auto w2 = [&](int64_t t, int l) -> int64_t { return m.map2[t * n2 + l]; };
    RowInc r2 = row_incidence(m, m.N2, n2, w2);
    build_csr(r2, m.N2, m.N1, n2, n1, w1all, R.K.data(), [&](int64_t, int l, int i) { return R.K[l * n1 + i]; },
              true, io.K);
    std::vector<double> KT(n1 * n2);
    for (int i = 0; i < n1; i++)
        for (int l = 0; l < n2; l++) KT[i * n2 + l] = R.K[l * n1 + i];
    RowInc r1 = row_incidence(m, m.N1, n1, w1all);
    build_csr(r1, m.N1, m.N2, n1, n2, w2, KT.data(), [&](int64_t, int i, int l) { return KT[i * n2 + l]; }, true,
              io.Kt);
    incidence(m, m.N2, n2, m.map2, io.inc2_ptr, io.inc2_idx);
}

}  // namespace fempic
