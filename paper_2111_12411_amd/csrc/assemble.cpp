// Global sparse operators of the implicit field update (paper Sec. III-A,
// Sec. III-B) in CSR over the internal DoF numbering:
//   *eps  = eps0 <W1_i, W1_j>,  *nu = (1/mu0) <W2_i, W2_j>,
//   K     = local curl matrix by assignment (curl W1_j = sum_l K_lj W2_l),
//   A     = *eps + dt^2/4 K^T *nu K  (assembled element by element),
//   K^T *nu, G^T (gradient matrix by assignment).
// Only W1 DoFs off the PEC walls are unknowns; W0 rows of the Gauss check are
// the interior nodal DoFs.  Also the explicit time-step bound and the
// DoF -> (tet, local) incidence lists that the deterministic deposit scatter uses.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

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

// Generic CSR from element contributions.  rmap/cmap give the global row /
// column of a local index (or -1 to skip); mask (optional) drops structural
// zeros; `assign` stores the value (all tets must agree) instead of adding.
struct ElemSpec {
    int64_t rows, cols;
    int nr, nc;
    std::function<int64_t(int64_t, int)> rmap, cmap;
    const double *mask = nullptr;
    bool assign = false;
};

void csr_pattern(const HostMesh &m, const ElemSpec &s, CSR &A)
{
    A.rows = s.rows;
    A.cols = s.cols;
    // row -> (tet, local row) incidence, tet ascending
    std::vector<int64_t> cnt(s.rows + 1, 0);
    for (int64_t t = 0; t < m.nt; t++)
        for (int i = 0; i < s.nr; i++) {
            int64_t r = s.rmap(t, i);
            if (r >= 0) cnt[r + 1]++;
        }
    for (int64_t r = 0; r < s.rows; r++) cnt[r + 1] += cnt[r];
    std::vector<int64_t> inc(cnt[s.rows]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t t = 0; t < m.nt; t++)
        for (int i = 0; i < s.nr; i++) {
            int64_t r = s.rmap(t, i);
            if (r >= 0) inc[fill[r]++] = t * s.nr + i;
        }
    A.ptr.assign(s.rows + 1, 0);
    std::vector<int32_t> cols;
    std::vector<int32_t> all;
    all.reserve((size_t)s.rows * 16);
    for (int64_t r = 0; r < s.rows; r++) {
        cols.clear();
        for (int64_t k = cnt[r]; k < cnt[r + 1]; k++) {
            int64_t t = inc[k] / s.nr;
            int i = (int)(inc[k] % s.nr);
            for (int j = 0; j < s.nc; j++) {
                if (s.mask && s.mask[i * s.nc + j] == 0.0) continue;
                int64_t c = s.cmap(t, j);
                if (c >= 0) cols.push_back((int32_t)c);
            }
        }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        all.insert(all.end(), cols.begin(), cols.end());
        A.ptr[r + 1] = (int64_t)all.size();
    }
    A.idx.swap(all);
    A.val.assign(A.idx.size(), 0.0);
}

inline int64_t find_pos(const CSR &A, int64_t r, int32_t c)
{
    const int32_t *b = A.idx.data() + A.ptr[r], *e = A.idx.data() + A.ptr[r + 1];
    const int32_t *p = std::lower_bound(b, e, c);
    return p - A.idx.data();
}

void csr_add(const ElemSpec &s, CSR &A, int64_t t, const double *el, std::vector<uint8_t> *set)
{
    for (int i = 0; i < s.nr; i++) {
        int64_t r = s.rmap(t, i);
        if (r < 0) continue;
        for (int j = 0; j < s.nc; j++) {
            if (s.mask && s.mask[i * s.nc + j] == 0.0) continue;
            int64_t c = s.cmap(t, j);
            if (c < 0) continue;
            int64_t p = find_pos(A, r, (int32_t)c);
            if (s.assign) {
                if ((*set)[p] && A.val[p] != el[i * s.nc + j])
                    throw Error(FEMPIC_EMESH, "local exterior derivative disagrees between tets");
                A.val[p] = el[i * s.nc + j];
                (*set)[p] = 1;
            } else {
                A.val[p] += el[i * s.nc + j];
            }
        }
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

void assemble(const HostMesh &m, double dt, Operators &ops)
{
    const RefElem &R = ref_elem(m.order);
    const int n1 = R.n1, n2 = R.n2, n0 = R.n0;
    const int64_t N1i = m.N1_int, N0i = m.N0_int;
    auto w1int = [&](int64_t t, int i) -> int64_t {
        int32_t d = m.map1[t * n1 + i];
        return d < N1i ? d : -1;
    };
    auto w2 = [&](int64_t t, int l) -> int64_t { return m.map2[t * n2 + l]; };
    auto w0int = [&](int64_t t, int j) -> int64_t {
        int32_t d = m.map0[t * n0 + j];
        return d < N0i ? d : -1;
    };

    ElemSpec sA{N1i, N1i, n1, n1, w1int, w1int};
    ElemSpec sC{N1i, m.N2, n1, n2, w1int, w2};
    ElemSpec sK{m.N2, N1i, n2, n1, w2, w1int, R.K.data(), true};
    std::vector<double> Gt(n0 * n1);
    for (int j = 0; j < n0; j++)
        for (int i = 0; i < n1; i++) Gt[j * n1 + i] = R.G[i * n0 + j];
    ElemSpec sG{N0i, N1i, n0, n1, w0int, w1int, Gt.data(), true};

    csr_pattern(m, sA, ops.A);
    ops.Meps.rows = ops.A.rows;
    ops.Meps.cols = ops.A.cols;
    ops.Meps.ptr = ops.A.ptr;
    ops.Meps.idx = ops.A.idx;
    ops.Meps.val.assign(ops.A.idx.size(), 0.0);
    csr_pattern(m, sC, ops.Ct);
    csr_pattern(m, sK, ops.K);
    csr_pattern(m, sG, ops.Gt);

    std::vector<double> M1(n1 * n1), M2(n2 * n2), S(n1 * n1), KtM2(n1 * n2), Ael(n1 * n1), Mel(n1 * n1),
        Cel(n1 * n2);
    std::vector<uint8_t> setK(ops.K.idx.size(), 0), setG(ops.Gt.idx.size(), 0);
    const double c_stiff = dt * dt / 4.0 / MU0;
    for (int64_t t = 0; t < m.nt; t++) {
        element_mass(m, t, M1.data(), M2.data());
        curl_products(R, M2.data(), S.data(), KtM2.data());
        for (int i = 0; i < n1 * n1; i++) {
            Mel[i] = EPS0 * M1[i];
            Ael[i] = Mel[i] + c_stiff * S[i];
        }
        for (int i = 0; i < n1 * n2; i++) Cel[i] = KtM2[i] / MU0;
        csr_add(sA, ops.A, t, Ael.data(), nullptr);
        csr_add(sA, ops.Meps, t, Mel.data(), nullptr);
        csr_add(sC, ops.Ct, t, Cel.data(), nullptr);
        csr_add(sK, ops.K, t, R.K.data(), &setK);
        csr_add(sG, ops.Gt, t, Gt.data(), &setG);
    }
    ops.Adiag_inv.assign(N1i, 0.0);
    for (int64_t r = 0; r < N1i; r++) {
        int64_t p = find_pos(ops.A, r, (int32_t)r);
        double d = ops.A.val[p];
        if (!(d > 0)) throw Error(FEMPIC_EMESH, "field matrix has a non-positive diagonal");
        ops.Adiag_inv[r] = 1.0 / d;
    }
    incidence(m, N1i, n1, m.map1, ops.inc_ptr, ops.inc_idx);
    incidence(m, N0i, n0, m.map0, ops.inc0_ptr, ops.inc0_idx);
}

}  // namespace fempic
