// Tetrahedral mesh complex {nodes, edges, faces, tets} (paper Sec. III-A):
// sorted-vertex tets, lexicographic edge / face numbering, face neighbours,
// PEC wall entities, per-tet affine barycentric maps and the order-k DoF maps.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "fempic_impl.h"

namespace fempic {

namespace {

void geometry(HostMesh &m)
{
    m.geo.assign(m.nt * 16, 0.0);
    m.vol.assign(m.nt, 0.0);
    for (int64_t t = 0; t < m.nt; t++) {
        const int32_t *v = &m.tets[4 * t];
        const double *x0 = &m.xyz[3 * v[0]];
        double J[3][3];  // columns x_m - x_0
        for (int c = 0; c < 3; c++)
            for (int r = 0; r < 3; r++) J[r][c] = m.xyz[3 * v[c + 1] + r] - x0[r];
        double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        double scale = 0;
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) scale = std::max(scale, std::fabs(J[r][c]));
        if (!(std::fabs(det) > 1e-13 * scale * scale * scale))
            throw Error(FEMPIC_EMESH, "degenerate tetrahedron " + std::to_string(t));
        // rows of J^{-1} are grad lambda_1..3
        double inv[3][3];
        inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        double *g = &m.geo[16 * t];
        double sa = 0, sg[3] = {0, 0, 0};
        for (int k = 1; k < 4; k++) {
            double a = -(inv[k - 1][0] * x0[0] + inv[k - 1][1] * x0[1] + inv[k - 1][2] * x0[2]);
            g[4 * k] = a;
            for (int c = 0; c < 3; c++) {
                g[4 * k + 1 + c] = inv[k - 1][c];
                sg[c] += inv[k - 1][c];
            }
            sa += a;
        }
        g[0] = 1.0 - sa;
        for (int c = 0; c < 3; c++) g[1 + c] = -sg[c];
        m.vol[t] = std::fabs(det) / 6.0;
    }
}

void topology(HostMesh &m)
{
    const int64_t nt = m.nt, nv = m.nv;
    // edges
    std::vector<std::pair<uint64_t, int64_t>> ek(6 * nt);
    for (int64_t t = 0; t < nt; t++)
        for (int e = 0; e < 6; e++) {
            uint64_t a = m.tets[4 * t + LOC_EDGE[e][0]], b = m.tets[4 * t + LOC_EDGE[e][1]];
            ek[6 * t + e] = {a * (uint64_t)nv + b, 6 * t + e};
        }
    std::sort(ek.begin(), ek.end());
    m.tet_edge.assign(6 * nt, -1);
    std::vector<uint64_t> edge_key;
    for (size_t i = 0; i < ek.size(); i++) {
        if (i == 0 || ek[i].first != ek[i - 1].first) edge_key.push_back(ek[i].first);
        m.tet_edge[ek[i].second] = (int32_t)(edge_key.size() - 1);
    }
    m.ne = (int64_t)edge_key.size();
    // faces
    std::vector<std::pair<uint64_t, int64_t>> fk(4 * nt);
    for (int64_t t = 0; t < nt; t++)
        for (int f = 0; f < 4; f++) {
            uint64_t a = m.tets[4 * t + LOC_FACE[f][0]], b = m.tets[4 * t + LOC_FACE[f][1]],
                     c = m.tets[4 * t + LOC_FACE[f][2]];
            fk[4 * t + f] = {(a * (uint64_t)nv + b) * (uint64_t)nv + c, 4 * t + f};
        }
    std::sort(fk.begin(), fk.end());
    m.tet_face.assign(4 * nt, -1);
    m.nbr.assign(4 * nt, -1);
    std::vector<uint64_t> face_key;
    std::vector<int32_t> face_cnt;
    for (size_t i = 0; i < fk.size(); i++) {
        if (i == 0 || fk[i].first != fk[i - 1].first) {
            face_key.push_back(fk[i].first);
            face_cnt.push_back(0);
        }
        m.tet_face[fk[i].second] = (int32_t)(face_key.size() - 1);
        face_cnt.back()++;
        if (face_cnt.back() > 2) throw Error(FEMPIC_EMESH, "a face is shared by more than two tets");
        if (face_cnt.back() == 2) {
            int64_t s0 = fk[i - 1].second, s1 = fk[i].second;
            int64_t t0 = s0 / 4, t1 = s1 / 4;
            int f0 = (int)(s0 % 4), f1 = (int)(s1 % 4);
            m.nbr[4 * t0 + (3 - f0)] = (int32_t)t1;  // face f is opposite vertex 3 - f
            m.nbr[4 * t1 + (3 - f1)] = (int32_t)t0;
        }
    }
    m.nf = (int64_t)face_key.size();
    // wall entities
    m.bface.assign(m.nf, 0);
    m.bedge.assign(m.ne, 0);
    m.bvert.assign(nv, 0);
    for (int64_t f = 0; f < m.nf; f++) m.bface[f] = face_cnt[f] == 1;
    for (int64_t t = 0; t < nt; t++)
        for (int f = 0; f < 4; f++) {
            if (!m.bface[m.tet_face[4 * t + f]]) continue;
            for (int k = 0; k < 3; k++) m.bvert[m.tets[4 * t + LOC_FACE[f][k]]] = 1;
            for (int e = 0; e < 6; e++) {
                int a = LOC_EDGE[e][0], b = LOC_EDGE[e][1];
                bool in_a = false, in_b = false;
                for (int k = 0; k < 3; k++) {
                    in_a |= LOC_FACE[f][k] == a;
                    in_b |= LOC_FACE[f][k] == b;
                }
                if (in_a && in_b) m.bedge[m.tet_edge[6 * t + e]] = 1;
            }
        }
}

void number_from_mask(const std::vector<uint8_t> &is_wall, std::vector<int64_t> &nat2int, std::vector<int64_t> &int2nat,
                      int64_t &n_int)
{
    const int64_t n = (int64_t)is_wall.size();
    nat2int.assign(n, -1);
    int2nat.assign(n, -1);
    int64_t k = 0;
    for (int64_t i = 0; i < n; i++)
        if (!is_wall[i]) { nat2int[i] = k; int2nat[k] = i; k++; }
    n_int = k;
    for (int64_t i = 0; i < n; i++)
        if (is_wall[i]) { nat2int[i] = k; int2nat[k] = i; k++; }
}

void dofs(HostMesh &m)
{
    const RefElem &R = ref_elem(m.order);
    const int64_t nt = m.nt, E = m.ne, F = m.nf, V = m.nv;
    m.n1l = R.n1;
    m.n2l = R.n2;
    m.n0l = R.n0;
    std::vector<uint8_t> wall1, wall0;
    std::vector<int64_t> nat1(nt * R.n1), nat2(nt * R.n2), nat0(nt * R.n0);
    if (m.order == 1) {
        m.N1 = E;
        m.N2 = F;
        m.N0 = V;
        wall1 = m.bedge;
        wall0 = m.bvert;
        for (int64_t t = 0; t < nt; t++) {
            for (int i = 0; i < 6; i++) nat1[6 * t + i] = m.tet_edge[6 * t + i];
            for (int l = 0; l < 4; l++) nat2[4 * t + l] = m.tet_face[4 * t + l];
            for (int j = 0; j < 4; j++) nat0[4 * t + j] = m.tets[4 * t + j];
        }
    } else {
        m.N1 = 2 * E + 2 * F;
        m.N2 = 3 * F + 3 * nt;
        m.N0 = V + E;
        wall1.assign(m.N1, 0);
        for (int64_t e = 0; e < E; e++) wall1[2 * e] = wall1[2 * e + 1] = m.bedge[e];
        for (int64_t f = 0; f < F; f++) wall1[2 * E + 2 * f] = wall1[2 * E + 2 * f + 1] = m.bface[f];
        wall0.assign(m.N0, 0);
        for (int64_t v = 0; v < V; v++) wall0[v] = m.bvert[v];
        for (int64_t e = 0; e < E; e++) wall0[V + e] = m.bedge[e];
        for (int64_t t = 0; t < nt; t++) {
            for (int le = 0; le < 6; le++) {
                nat1[20 * t + 2 * le] = 2 * (int64_t)m.tet_edge[6 * t + le];
                nat1[20 * t + 2 * le + 1] = 2 * (int64_t)m.tet_edge[6 * t + le] + 1;
            }
            for (int lf = 0; lf < 4; lf++) {
                nat1[20 * t + 12 + 2 * lf] = 2 * E + 2 * (int64_t)m.tet_face[4 * t + lf];
                nat1[20 * t + 12 + 2 * lf + 1] = 2 * E + 2 * (int64_t)m.tet_face[4 * t + lf] + 1;
                for (int x = 0; x < 3; x++) nat2[15 * t + 3 * lf + x] = 3 * (int64_t)m.tet_face[4 * t + lf] + x;
            }
            for (int x = 0; x < 3; x++) nat2[15 * t + 12 + x] = 3 * F + 3 * t + x;
            for (int j = 0; j < 4; j++) nat0[10 * t + j] = m.tets[4 * t + j];
            for (int le = 0; le < 6; le++) nat0[10 * t + 4 + le] = V + m.tet_edge[6 * t + le];
        }
    }
    number_from_mask(wall1, m.nat2int1, m.int2nat1, m.N1_int);
    number_from_mask(wall0, m.nat2int0, m.int2nat0, m.N0_int);
    if (m.N1 >= INT32_MAX || m.N2 >= INT32_MAX || m.N0 >= INT32_MAX)
        throw Error(FEMPIC_EINVAL, "mesh too large for 32-bit DoF ids");
    m.map1.resize(nt * R.n1);
    m.map2.resize(nt * R.n2);
    m.map0.resize(nt * R.n0);
    for (size_t i = 0; i < nat1.size(); i++) m.map1[i] = (int32_t)m.nat2int1[nat1[i]];
    for (size_t i = 0; i < nat2.size(); i++) m.map2[i] = (int32_t)nat2[i];
    for (size_t i = 0; i < nat0.size(); i++) m.map0[i] = (int32_t)m.nat2int0[nat0[i]];
}

}  // namespace

HostMesh *build_mesh(const double *xyz, int64_t nv, const int64_t *tet4, int64_t nt, int order, bool cube)
{
    if (nv < 4 || nt < 1 || !xyz || !tet4) throw Error(FEMPIC_EINVAL, "empty mesh");
    if (order != 1 && order != 2) throw Error(FEMPIC_EINVAL, "order must be 1 or 2");
    if (nv >= (int64_t)1 << 21) throw Error(FEMPIC_EINVAL, "more than 2^21 vertices");
    if (nt >= INT32_MAX / 20) throw Error(FEMPIC_EINVAL, "too many tets");
    auto *m = new HostMesh();
    try {
        m->order = order;
        m->nv = nv;
        m->nt = nt;
        m->xyz.assign(xyz, xyz + 3 * nv);
        m->tets.resize(4 * nt);
        for (int64_t t = 0; t < nt; t++) {
            int64_t v[4];
            for (int k = 0; k < 4; k++) {
                v[k] = tet4[4 * t + k];
                if (v[k] < 0 || v[k] >= nv) throw Error(FEMPIC_EMESH, "vertex id out of range");
            }
            std::sort(v, v + 4);
            for (int k = 0; k < 3; k++)
                if (v[k] == v[k + 1]) throw Error(FEMPIC_EMESH, "repeated vertex in a tet");
            for (int k = 0; k < 4; k++) m->tets[4 * t + k] = (int32_t)v[k];
        }
        topology(*m);
        geometry(*m);
        dofs(*m);
        m->is_cube = cube;
        m->dt_cfl = cfl_bound(*m);
    } catch (...) {
        delete m;
        throw;
    }
    return m;
}

HostMesh *build_cube(int N, double L, int order)
{
    // (N+1)^3 vertices must stay below the 2^21 cap of build_mesh; checked
    // here, before anything of the size of the cube is allocated
    if (N < 1 || N > CUBE_N_MAX || !(L > 0))
        throw Error(FEMPIC_EINVAL, "cube needs 1 <= N <= " + std::to_string(CUBE_N_MAX) + " and L > 0");
    const int64_t n1 = N + 1;
    std::vector<double> xyz(3 * n1 * n1 * n1);
    for (int64_t l = 0; l <= N; l++)
        for (int64_t j = 0; j <= N; j++)
            for (int64_t i = 0; i <= N; i++) {
                int64_t id = i + n1 * (j + n1 * l);
                xyz[3 * id] = i * L / N;
                xyz[3 * id + 1] = j * L / N;
                xyz[3 * id + 2] = l * L / N;
            }
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int64_t nt = 6LL * N * N * N;
    std::vector<int64_t> tets(4 * nt);
    for (int64_t l = 0; l < N; l++)
        for (int64_t j = 0; j < N; j++)
            for (int64_t i = 0; i < N; i++) {
                int64_t h = i + N * (j + N * l);
                for (int p = 0; p < 6; p++) {
                    int64_t c[3] = {i, j, l};
                    tets[4 * (6 * h + p)] = c[0] + n1 * (c[1] + n1 * c[2]);
                    for (int s = 0; s < 3; s++) {
                        c[perm[p][s]]++;
                        tets[4 * (6 * h + p) + s + 1] = c[0] + n1 * (c[1] + n1 * c[2]);
                    }
                }
            }
    HostMesh *m = build_mesh(xyz.data(), n1 * n1 * n1, tets.data(), nt, order, true);
    m->cube_N = N;
    m->cube_L = L;
    return m;
}

}  // namespace fempic
