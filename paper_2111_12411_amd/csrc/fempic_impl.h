// Internal declarations of the fempic library (host side).
#pragma once
#include <cstdint>
#include <string>
#include <vector>
#include <stdexcept>

#include "../../include/fempic.h"

namespace fempic {

constexpr double C_LIGHT = 299792458.0;
constexpr double MU0 = 1.25663706212e-6;
constexpr double EPS0 = 1.0 / (MU0 * C_LIGHT * C_LIGHT);

struct Error : std::runtime_error {
    int32_t code;
    Error(int32_t c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// Local entity tables of a tet with sorted vertices 0<1<2<3.
extern const int LOC_EDGE[6][2];  // (0,1),(0,2),(0,3),(1,2),(1,3),(2,3)
extern const int LOC_FACE[4][3];  // (0,1,2),(0,1,3),(0,2,3),(1,2,3); face f is opposite vertex 3-f

// Reference-element description of the order-k bases (Appendix).
// W1_i = (qc + qs * l_qv) (l_a grad l_b - l_b grad l_a)
struct W1Fn { int a, b, qv; double qs, qc; };
// W2_l = (qc + qs * l_qv) * 2 (l_a gb x gc + l_b gc x ga + l_c ga x gb)
struct W2Fn { int a, b, c, qv; double qs, qc; };
// W0_j = c1 * l_a * (l_b or (cs*l_a + cc))  -- see refelem.cpp
struct W0Fn { int a, b; double c1, cs, cc; };

struct RefElem {
    int order;
    int n0, n1, n2;
    std::vector<W1Fn> w1;
    std::vector<W2Fn> w2;
    std::vector<W0Fn> w0;
    std::vector<double> G;   // [n1][n0]  grad W0_j = sum_i G[i][j] W1_i
    std::vector<double> K;   // [n2][n1]  curl W1_j = sum_l K[l][j] W2_l
    std::vector<double> C1;  // [n1][n1][4][4] (1/6V) int phi_i^m phi_j^n
    std::vector<double> C2;  // [n2][n2][6][6]
    std::vector<double> F1;  // [4][n1][n1][4][4] (1/A) int over the face opposite vertex o of phi_i^m phi_j^n
    std::vector<double> glx, glw;  // Gauss-Legendre on [0,1], 2k+2 points
};
const RefElem &ref_elem(int order);

struct HostMesh {
    int order = 1;
    bool is_cube = false;
    int cube_N = 0;
    double cube_L = 1.0;
    int64_t nv = 0, nt = 0, ne = 0, nf = 0;
    std::vector<double> xyz;       // [nv][3]
    std::vector<int32_t> tets;     // [nt][4] sorted
    std::vector<int32_t> tet_edge; // [nt][6]
    std::vector<int32_t> tet_face; // [nt][4]
    std::vector<int32_t> nbr;      // [nt][4] across face opposite vertex m, -1 wall
    std::vector<double> geo;       // [nt][16]: m = 0..3: a_m, grad_m (x,y,z)
    std::vector<double> vol;       // [nt]
    std::vector<uint8_t> bedge, bface, bvert;
    // DoFs: natural numbering (documented in fempic.h) and internal numbering
    // (DoFs off the walls first, natural order kept within each group).
    int n1l = 0, n2l = 0, n0l = 0;
    int64_t N1 = 0, N2 = 0, N0 = 0, N1_int = 0, N0_int = 0;
    std::vector<int64_t> nat2int1, int2nat1, nat2int0, int2nat0;
    std::vector<int32_t> map1, map2, map0;  // [nt][n*l] internal ids
    double dt_cfl = 0.0;
};

HostMesh *build_mesh(const double *xyz, int64_t nv, const int64_t *tet4, int64_t nt, int order, bool cube = false);
// largest Kuhn cube: (N+1)^3 vertices below the 2^21 vertex cap of build_mesh
constexpr int CUBE_N_MAX = 126;
HostMesh *build_cube(int N, double L, int order);
double cfl_bound(const HostMesh &m);

// Element matrices of one tet: M1 (n1 x n1, without eps0), M2 (n2 x n2, without 1/mu0)
void element_mass(const HostMesh &m, int64_t t, double *M1, double *M2);

struct CSR {
    int64_t rows = 0, cols = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> idx;
    std::vector<double> val;
    int64_t nnz() const { return (int64_t)idx.size(); }
};

// The unknown W1 DoFs are the first n1s of the internal numbering: those off
// the walls (N1_int) with PEC walls, all of them (N1) with absorbing walls.
struct Operators {
    int64_t n1s = 0;
    CSR A;      // *eps + c dt^2 K^T *nu K (+ dt/2 *I)   (n1s x n1s)
    CSR Meps;   // *eps                      (n1s x n1s)
    CSR Mnu;    // *nu                       (N2 x N2)
    CSR K;      // curl                      (N2 x n1s)
    CSR Kt;     // K^T                       (n1s x N2)
    CSR Gt;     // gscale G^T                (N0_int x n1s)
    CSR Z;      // surface impedance *I      (n1s x n1s; absorbing walls only, else empty)
    // the smallest integer that makes every entry of G an integer (1 at order 1,
    // 3 at order 2): products with gscale G^T are then exact in double-double
    double gscale = 1.0;
    std::vector<double> Adiag_inv;
    // deposit scatter: for unknown W1 DoF j, the (tet*n1l + local) slots in tet order
    std::vector<int64_t> inc_ptr;
    std::vector<int32_t> inc_idx;
    // nodal scatter for rho~: interior W0 DoF j -> (tet*n0l + local)
    std::vector<int64_t> inc0_ptr;
    std::vector<int32_t> inc0_idx;
};

// A = *eps + c_dt2 dt^2 K^T *nu K (c_dt2 = (beta / gamma)^2 of the Newmark-beta scheme);
// absorbing: every W1 DoF is an unknown and A gains dt/2 *I (Sec. III-A) with the
// wall admittance 1/eta0
void assemble(const HostMesh &m, double dt, Operators &ops, double c_dt2 = 0.25, bool absorbing = false);

// Operators of the impressed-field projection (Sec. III-C): the curl over every
// W1 DoF, walls included (N2 x N1) and its transpose, and the face DoF ->
// (tet * n2l + local) incidence lists in tet order.
struct ImpressedOps {
    CSR K, Kt;
    std::vector<int64_t> inc2_ptr;
    std::vector<int32_t> inc2_idx;
};
void assemble_impressed(const HostMesh &m, ImpressedOps &io);

// collapsed Gauss-Legendre rule on the reference tet with n^3 points (the
// quadrature of the impressed field's moments): barycentric coordinates
// lam [n^3][4] and weights w [n^3] summing to 1
void impressed_rule(int n, std::vector<double> &lam, std::vector<double> &w);

// Device bytes a run allocates for a mesh of these sizes and n particles
// (operators with their nonzeros bounded per row for meshes of Kuhn-cube
// valence, fields, solver vectors, particle state, sort, queue and the initial
// spill pool).
struct FootprintSizes {
    int order;
    int64_t nt, n1, n1_int, n2, n0_int;
    bool absorbing = false;  // absorbing walls: all n1 W1 DoFs are unknowns, plus *I
};
size_t footprint_bytes(const FootprintSizes &z, int64_t n, bool mixed);
// sizes of the N^3 Kuhn cube with nt = 6 N^3 tets, N taken real (totals stand in for interior counts)
FootprintSizes kuhn_sizes(int order, double nt);

}  // namespace fempic
