// Host-side mesh building, reference elements and operator assembly, built with
// g++ under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py (no GPU code is involved).  Exits non-zero on a
// failed check; the sanitizers abort on a memory error or undefined behaviour.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <memory>
#include <numeric>
#include <vector>

#include "fempic_impl.h"

using namespace fempic;

static int fails = 0;
#define CHECK(c)                                                                \
    do {                                                                        \
        if (!(c)) {                                                             \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            fails++;                                                            \
        }                                                                       \
    } while (0)

static void check_csr(const CSR &A, int64_t rows, int64_t cols)
{
    CHECK(A.rows == rows && A.cols == cols);
    CHECK((int64_t)A.ptr.size() == A.rows + 1);
    CHECK(A.ptr[0] == 0 && A.ptr[A.rows] == A.nnz());
    CHECK(A.val.size() == A.idx.size());
    for (int64_t r = 0; r < A.rows; r++) {
        CHECK(A.ptr[r] <= A.ptr[r + 1]);
        for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; k++) {
            CHECK(A.idx[k] >= 0 && A.idx[k] < A.cols);
            CHECK(std::isfinite(A.val[k]));
        }
    }
}

int main()
{
    for (int k = 1; k <= 2; k++) {
        for (int N : {1, 2, 3}) {
            std::unique_ptr<HostMesh> m(build_cube(N, 1.0, k));
            CHECK(m->nt == 6LL * N * N * N);
            CHECK(m->nv == (int64_t)(N + 1) * (N + 1) * (N + 1));
            CHECK(m->dt_cfl > 0 && std::isfinite(m->dt_cfl));
            Operators ops;
            assemble(*m, 5 * m->dt_cfl, ops);
            check_csr(ops.A, m->N1_int, m->N1_int);
            check_csr(ops.Meps, m->N1_int, m->N1_int);
            check_csr(ops.Mnu, m->N2, m->N2);
            check_csr(ops.K, m->N2, m->N1_int);
            check_csr(ops.Kt, m->N1_int, m->N2);
            CHECK(ops.gscale == (m->order == 2 ? 3.0 : 1.0));
            for (double v : ops.Gt.val) CHECK(v == std::nearbyint(v));
            check_csr(ops.Gt, m->N0_int, m->N1_int);
            CHECK((int64_t)ops.Adiag_inv.size() >= m->N1_int);
            CHECK((int64_t)ops.inc_ptr.size() == m->N1_int + 1);
            CHECK((int64_t)ops.inc0_ptr.size() == m->N0_int + 1);
            for (int32_t s : ops.inc_idx) CHECK(s >= 0 && s < m->nt * m->n1l);
            for (int32_t s : ops.inc0_idx) CHECK(s >= 0 && s < m->nt * m->n0l);
            CHECK(ops.n1s == m->N1_int && ops.Z.nnz() == 0);
            // absorbing walls: every W1 DoF an unknown, the surface impedance matrix
            // symmetric, on the wall DoFs only, and inside A's pattern
            Operators ab;
            assemble(*m, 5 * m->dt_cfl, ab, 0.25, true);
            CHECK(ab.n1s == m->N1);
            check_csr(ab.A, m->N1, m->N1);
            check_csr(ab.Z, m->N1, m->N1);
            check_csr(ab.Gt, m->N0_int, m->N1);
            CHECK((int64_t)ab.inc_ptr.size() == m->N1 + 1);
            CHECK(ab.Z.nnz() > 0);
            double zmax = 0.0;
            for (double v : ab.Z.val) zmax = std::max(zmax, std::fabs(v));
            for (int64_t r = 0; r < ab.Z.rows; r++)
                for (int64_t q = ab.Z.ptr[r]; q < ab.Z.ptr[r + 1]; q++) {
                    const int32_t c = ab.Z.idx[q];
                    CHECK(r >= m->N1_int && c >= m->N1_int);
                    const int32_t *b = ab.Z.idx.data() + ab.Z.ptr[c], *e = ab.Z.idx.data() + ab.Z.ptr[c + 1];
                    const int32_t *f = std::lower_bound(b, e, (int32_t)r);
                    CHECK(f != e && *f == r);
                    if (f != e && *f == r) {
                        const double vt = ab.Z.val[f - ab.Z.idx.data()];
                        CHECK(std::fabs(vt - ab.Z.val[q]) <= 1e-14 * zmax);
                    }
                }
            // the generic path: the same cube with vertex ids permuted and tet corners unsorted
            const int64_t nv = m->nv, nt = m->nt;
            std::vector<int64_t> perm(nv);
            for (int64_t v = 0; v < nv; v++) perm[v] = (v * 7 + 3) % nv;
            std::vector<double> xyz(3 * nv);
            for (int64_t v = 0; v < nv; v++)
                for (int c = 0; c < 3; c++) xyz[3 * perm[v] + c] = m->xyz[3 * v + c];
            std::vector<int64_t> tets(4 * nt);
            for (int64_t t = 0; t < nt; t++)
                for (int j = 0; j < 4; j++) tets[4 * t + j] = perm[m->tets[4 * t + (j + t) % 4]];
            std::unique_ptr<HostMesh> g(build_mesh(xyz.data(), nv, tets.data(), nt, k));
            CHECK(g->ne == m->ne && g->nf == m->nf && g->N1_int == m->N1_int && g->N0_int == m->N0_int);
            CHECK(std::fabs(g->dt_cfl - m->dt_cfl) <= 1e-12 * m->dt_cfl);
        }
    }
    // a flat tet is refused
    try {
        const double xyz[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 1, 1, 0};
        const int64_t t4[4] = {0, 1, 2, 3};
        std::unique_ptr<HostMesh> m(build_mesh(xyz, 4, t4, 1, 1));
        CHECK(false);
    } catch (const Error &e) {
        CHECK(e.code == FEMPIC_EMESH);
    }
    std::printf("host checks: %d failed\n", fails);
    return fails ? 1 : 0;
}
