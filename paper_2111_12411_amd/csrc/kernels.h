// Launch interface of the fempic HIP kernels (gfx950).
#pragma once
#include <hip/hip_runtime_api.h>
#include <cstdint>

namespace fempic {

struct GLRule {
    double x[8], w[8];  // Gauss-Legendre nodes / weights on [0,1]
};

struct DevMesh {
    int32_t nt;
    const double *geo;   // [nt][16] (a_m, grad_m) m = 0..3
    const int32_t *nbr;  // [nt][4] 4 nb + (face of nb shared with t) across the face opposite vertex m; -1 wall
    const int32_t *map1; // [nt][n1l] internal W1 ids (wall DoFs >= N1_int hold zero)
    const int32_t *map2; // [nt][n2l]
    const int32_t *map0; // [nt][n0l]
    // Kuhn cube locate
    int32_t cube_N;
    double cube_L;
};

// Particle state.  The position is held as the particle's barycentric
// coordinates l_1, l_2, l_3 in its tet (l_0 = 1 - l_1 - l_2 - l_3), FP64 like
// the velocity in both modes; the AB4 histories are R (double, or float in
// mixed mode): vh = v^{n-1} - v^n, v^{n-2} - v^n, v^{n-3} - v^n and
// ah = a^{n-1}, a^{n-2}, a^{n-3}, three components each; tet; id (load order).
//
// Layout: a particle's state is a row of 4-byte units, packed into 16-byte
// words, and the words are stored word-major: word k of row s at byte
// (k cap + s) 16.  Loads of one word by consecutive rows are contiguous, as in
// a structure of arrays, while one particle's state spans only NW words (8 in
// mixed mode, 13 in FP64) instead of one line per scalar: a particle read from
// a slot away from its neighbours (one that changed tet) costs NW lines.
struct PartLayout {
    int nw;                      // words per row
    int lam, tet, id, v, vh, ah; // first unit of each field
    int hs;                      // units per history value (1: float, 2: double)
};
// l_1..l_3, tet, id in words 0-1; v from unit 8; then vh, ah
constexpr PartLayout PART_MIXED{8, 0, 6, 7, 8, 14, 23, 1};
constexpr PartLayout PART_FP64{13, 0, 6, 7, 8, 14, 32, 2};
constexpr const PartLayout &part_layout(bool mixed) { return mixed ? PART_MIXED : PART_FP64; }
// byte offset of unit u of row s
constexpr int64_t part_off(int u, int64_t cap, int64_t s) { return ((int64_t)(u >> 2) * cap + s) * 16 + (u & 3) * 4; }

struct DevParticles {
    void *w;      // [nw][cap] 16-byte words (PartLayout)
    int64_t cap;
};
// the rows from s0 on, as a particle set of its own (same cap)
inline DevParticles part_rows(DevParticles p, int64_t s0) { return DevParticles{(char *)p.w + s0 * 16, p.cap}; }

// particle kernel: threads per block, most tets per block (order 1, 2), and the
// number of particles a block aims at (tets per block = that / particles per tet)
constexpr int PARTICLE_BLOCK = 256;
constexpr int PARTICLE_TPW_MAX_1 = 64;
constexpr int PARTICLE_TPW_MAX_2 = 16;
constexpr int PARTICLE_TARGET = 512;

struct StepParams {
    double qm;      // q / m
    double qw;      // q * w
    double dt;
    int32_t tpw;    // tets per workgroup in the particle kernel
    int32_t absorb; // 1: a particle that reaches a wall is removed there (else it reflects)
    int32_t boris;  // 1: Boris leapfrog with a straight path (no AB4 histories)
};

// step counters (device int64 each): crossings, reflections, spilled segments,
// error bits (or-ed), absorbed particles; the rest are zero
constexpr int NCNT = 8;
enum { CNT_CROSS = 0, CNT_REFL = 1, CNT_SPILL = 2, CNT_ERR = 3, CNT_ABSORB = 4 };
// pool.pid of an absorbed particle's last record: never placed in the next order
constexpr int32_t PID_ABSORBED = -1;

// device error flags (bit set)
enum : int32_t { ERR_CROSS = 1, ERR_POOL = 2, ERR_OUTSIDE = 4, ERR_NAN = 8 };

struct SpillPool {
    double *val;     // [cap][n1l]
    int32_t *tet;    // [cap]
    int64_t *tag;    // [cap]   (queued record << 8) | (last segment of the path << 7) | segment index; -1: unused slot
    int32_t *pid;    // [cap]   sorted particle index, set on the record of a path's last segment
    int32_t *count;  // [1] records appended past the fixed slots (atomic)
    int32_t *rcount; // [np] spill records of each queued record
    int64_t cap;
};

// particles whose path leaves the home tet during the step
struct ContRec {
    double lam[3];   // l_1..l_3 of tet t at s_lo (l_0 = 1 - l_1 - l_2 - l_3)
    double dp[12];   // path displacement r(s) - r(0) = sum_{d=1..4} dp[3(d-1) + c] s^d (after wall reflections so far)
    double s_lo;     // path parameter where the particle entered tet t
    int32_t i;       // sorted particle index
    int32_t t;       // current tet
    int32_t entry;   // entry face of t (its barycentric coordinate is zero at s_lo)
    int32_t ncross;  // face crossings so far
    int32_t pending; // face of t the path leaves through at s_lo, not yet crossed (-1: none)
    int32_t pad;
};

struct ContQueue {
    ContRec *rec;    // [np] a wave of k_particle writes its records at the start of its own particle range
    uint8_t *flag;   // [np + 16] 1 where rec holds a record
    int32_t *idx;    // [np] rec slots of the records, in slot order
    int32_t *count;  // [1] number of records (the total of the prefix sum)
    uint8_t *moved;  // [np] 1 where sorted particle i is queued (its path leaves the home tet)
    int32_t *nstay;  // [nt] particles of each tet that are not queued
};


// x: [3][cap] positions of n particles
hipError_t launch_locate_cube(const DevMesh &m, int64_t n, DevParticles p, int32_t *err, hipStream_t s);
// positions (held in the l_1..l_3 units, in the tet of the tet unit) replaced in
// place by l_1..l_3 of that tet
hipError_t launch_to_bary(const DevMesh &m, int64_t n, DevParticles p, hipStream_t s);
// keys[i] = tet of row i, i < n
hipError_t launch_tet_keys(DevParticles p, int64_t n, uint32_t *keys, hipStream_t s);
hipError_t launch_startup(int order, bool mixed, const DevMesh &m, const double *e, const double *b, const float *e32,
                          const float *b32, DevParticles p, int64_t n, double qm, double dt, hipStream_t s);

// stable LSD radix sort of (key, val) uint32 pairs on the low `bits` bits of key;
// in/out buffers alternate; returns the buffer index (0 or 1) that holds the result.
struct SortBuffers {
    uint32_t *key[2];
    uint32_t *val[2];
    uint32_t *hist;   // [256 * tiles]
    uint32_t *scan_tmp;  // scratch for the scan
    int64_t cap;
};
int64_t sort_hist_entries(int64_t n);
int64_t scan_tmp_entries(int64_t n);
// key_in (optional): keys of the first pass, read in place of sb.key[0].
// dn (optional): device count of the pairs, at most n; the launches are sized
// for n (the same holds for the dn arguments below)
hipError_t radix_sort(SortBuffers &sb, int64_t n, int bits, bool vals_are_iota, int *result_buf, hipStream_t s,
                      const uint32_t *key_in = nullptr, const int32_t *dn = nullptr);
// out[i] = in[perm[i]] for every particle array
hipError_t launch_permute(bool mixed, DevParticles in, DevParticles out, const uint32_t *perm, int64_t n,
                          hipStream_t s);
// order of np0 present and n new particles: next_perm[p + noff_new[t]] = perm[p]
// for present sorted position p in tet t (off[t] <= p < off[t+1]), and
// next_perm[off[t+1] + q] = slot0 + nval[q] for the q-th new particle in tet
// order (nkey = its tet); next_off[t] = off[t] + noff_new[t], t in [0, nt]
hipError_t launch_merge_order(int64_t np0, int64_t n, int32_t nt, const int32_t *off, const int32_t *noff_new,
                              const uint32_t *perm, const uint32_t *nkey, const uint32_t *nval, uint32_t slot0,
                              int32_t *next_off, uint32_t *next_perm, hipStream_t s);
// bucket offsets off[t] = first index with key >= t, for t in [0, nt]
hipError_t launch_offsets(const uint32_t *sorted_key, int64_t n, int32_t nt, int32_t *off, hipStream_t s,
                          const int32_t *dn = nullptr);
// exclusive scan of uint32 (in place allowed), total into *total (device)
hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, uint32_t *total, hipStream_t s,
                              const int32_t *dn = nullptr);

// Arguments of the particle kernels, kept in device memory (passed by pointer,
// so the kernels do not hold them all in scalar registers).
struct ParticleArgs {
    DevMesh m;
    const void *e, *b;        // field coefficients: double (FP64) or float (mixed)
    const uint32_t *perm;     // sorted position -> slot of the input state
    const int32_t *off;       // [nt+1] first sorted position of each tet
    DevParticles in, out;
    int64_t np;
    StepParams sp;
    GLRule gl;
    double *P;                // [nt][n1l] per-tet current moments of home segments
    SpillPool pool;
    ContQueue cq;
    unsigned long long *cnt;  // [NCNT] step counters
    unsigned long long *cntb; // [CONT_BLOCKS][NCNT] per-block counters of the continuation kernel
    unsigned long long *perr; // [1] particle-order error flag (launch_place)
};
hipError_t launch_particle(int order, bool mixed, bool boris, const ParticleArgs *dargs, int32_t nt, int32_t tpw,
                           hipStream_t s);
// fills cq.idx and *cq.count from cq.flag; tmp: device scratch of at least
// 2 (np / 4096 + 1) + scan_tmp_entries(np / 4096 + 1) entries
hipError_t launch_queue_index(const ContQueue &cq, int64_t np, uint32_t *tmp, hipStream_t s);
// blocks of the continuation kernel (one counter slot each in cntb)
constexpr int CONT_BLOCKS = 65536;
// nq_hint: expected queue length (sizes the grid; any length is processed)
hipError_t launch_continue(int order, bool mixed, bool boris, const ParticleArgs *dargs, int64_t nq_hint,
                           unsigned long long *cntb, unsigned long long *cnt, hipStream_t s);
// spill records in canonical order (queued record, then segment): key = tet,
// val = slot (| SREC_LAST); nslots: launch size, nq: device count of queued
// records (the slots in use are 2 nq plus the pool's appended count); kcap:
// capacity of key and val
hipError_t launch_spill_compact(const SpillPool &pool, int64_t nslots, const int32_t *nq, const uint32_t *pos,
                                uint32_t *key, uint32_t *val, int64_t kcap, hipStream_t s);
// sorted spill values: pool slot, with SREC_LAST set on the record of a path's last segment
constexpr uint32_t SREC_LAST = 0x80000000u;
// adds the spill records (values recval[cap][n1l]) to P; when cnt is set, also
// cnt[t] = nstay[t] + (last-segment records in t)
hipError_t launch_spill_reduce(int n1l, int32_t nt, const int32_t *soff, const uint32_t *sorted_rec,
                               const double *recval, int64_t cap, double *P, const int32_t *nstay, uint32_t *cnt,
                               hipStream_t s);
// Particle order of the next step without a sort.  Tet t's new bucket, from
// noff[t] (exclusive scan of cnt), holds the particles of its old bucket
// [off[t], off[t+1]) that were not queued (moved == 0, old order), then the
// queued particles whose path ends in t, in the order of their last-segment
// records among t's sorted spill records (queue order).  tpw: tets per block
// (at most the particle kernel's largest).  *err is set if a bucket does not
// come out at its size.  nrec = 0: no spill records (soff, srec unread).
hipError_t launch_place(int64_t np, int32_t nt, int32_t tpw, const int32_t *off, const uint8_t *moved,
                        const int32_t *soff, const uint32_t *srec, int64_t nrec, const int32_t *pid, int64_t cap,
                        const int32_t *noff, uint32_t *perm, unsigned long long *err, hipStream_t s);
hipError_t launch_scatter(const int64_t *ptr, const int32_t *idx, int64_t n, const double *P, double *out,
                          hipStream_t s);
hipError_t launch_rho_tet(int order, const DevMesh &m, const uint32_t *perm, const int32_t *off, DevParticles p,
                          double qw, double *Pr, hipStream_t s);

// linear algebra (FP64 unless noted)
struct DevCSR {
    int64_t rows, cols, nnz;
    const int64_t *ptr;
    const int32_t *idx;
    const double *val;
    const float *val32;  // optional FP32 copy
    int lanes;           // lanes per row in the SpMV
    // optional 2x2 block copy (rows 2R, 2R+1 x columns 2C, 2C+1), used by the
    // SpMV when present: bval[4k..4k+3] = block k row-major
    int64_t brows;
    const int64_t *bptr;
    const int32_t *bidx;
    const double *bval;
    const float *bval32;
};
// The field system's operator with PEC walls, A = eps0 M1 + c S / mu0, applied
// tet by tet without the assembled matrix: each tet's product from its gradients
// and volume (k_mf_elem), then each unknown DoF sums its tets' products in tet
// order (k_mf_sum).  The operands and geo/pe are in one precision (FP64 for
// mf_apply, FP32 for mf_apply32).
struct DevMF {
    int order;            // 1 or 2; 0: not in use (the assembled matrix is)
    int64_t nt, n1s;      // tets; unknown W1 DoFs (the internal ids below n1s)
    const int32_t *map1;  // [nt][n1l] internal W1 ids
    const void *geo;      // [nt][16]: grad l_0..l_3 (x, y, z), the volume, 3 unused
    const int64_t *ptr;   // per unknown DoF i: its incidences t n1l + l in [ptr[i], ptr[i+1]), tet-ascending
    const int32_t *idx;
    void *pe;             // [nt][n1l] the tets' products
    double kM, kC;        // eps0 and c / mu0 (c: the curl-curl term's coefficient times dt^2)
    // order 2 (required there; order 1 uses map1, ptr and idx): the two DoFs of an edge or
    // face are the unknowns 2j, 2j+1 at local positions 2i, 2i+1 of every tet they meet.
    // map1p [nt][n1l/2]: j of local pair i, -1 when not unknowns; ptr2: per pair j
    // the range [ptr2[j], ptr2[j+1]) of its tets (tet-ascending) in pe, which then
    // holds pairs of products; slot2 [nt][n1l/2]: where in pe the tet's pair i goes
    const int32_t *map1p;
    const int64_t *ptr2;
    const int32_t *slot2;
};
hipError_t mf_apply(const DevMF &mf, const double *x, double *y, hipStream_t s);
hipError_t mf_apply32(const DevMF &mf, const float *x, float *y, hipStream_t s);
hipError_t spmv(const DevCSR &A, const double *x, double *y, double alpha, double beta, const double *z,
                hipStream_t s);  // y = alpha A x + beta z (z may alias y or be null when beta == 0)
hipError_t spmv32(const DevCSR &A, const float *x, float *y, hipStream_t s);
hipError_t axpby(int64_t n, double a, const double *x, double b, const double *y, double *out, hipStream_t s);

// PCG pieces; scalars is a device double[16] block
// SC_RZ and SC_RZ + 10 hold r.z for even / odd iterations (parity argument `par`)
// The preconditioner is Jacobi (dinv[i] = 1/A_ii) or, when A carries its 2x2
// block copy, 2x2 block Jacobi (dinv[4j..4j+3]: inverse diagonal block of rows
// 2j, 2j+1); `block` of the init call must say which (A.bptr != nullptr).
enum { SC_RZ = 0, SC_PQ = 1, SC_RR = 4, SC_BB = 5 };
hipError_t pcg_init(int64_t n, const double *b, double *x, double *r, double *z, double *p, const double *dinv,
                    double *partial, double *scalars, bool block, hipStream_t s);
// mf (nullable): apply A tet by tet instead of the assembled matrix when mf->order != 0.
// partial: the product's dot partials at [0, 2048), the update's (r.z, r.r) pairs
// after them: at least 2048 + 2 ceil(n / 256) doubles.
hipError_t pcg_iter(const DevCSR &A, const DevMF *mf, int64_t n, double *x, double *r, double *z, double *p,
                    double *q, const double *dinv, double *partial, double *scalars, int par, hipStream_t s);
// FP32 inner PCG (mixed mode); vectors float, scalars double
hipError_t pcg32_init(int64_t n, const float *b, float *x, float *r, float *z, float *p, const float *dinv,
                      double *partial, double *scalars, bool block, hipStream_t s);
hipError_t pcg32_iter(const DevCSR &A, const DevMF *mf, int64_t n, float *x, float *r, float *z, float *p, float *q,
                      const float *dinv, double *partial, double *scalars, int par, hipStream_t s);
hipError_t cast_d2f(int64_t n, const double *in, float *out, double scale, hipStream_t s);
hipError_t add_f2d(int64_t n, const float *in, double scale, double *out, hipStream_t s);

// deterministic norms: out[k] = sum_i f_k(...) for the Gauss check; GtDe and Gtg
// are products with gscale G^T (gscale makes G's entries integers), divided here
hipError_t gauss_norms(int64_t n, const double *GtDe, const double *Gtg, const double *rho, const double *rho0,
                       double gscale, double *partial, double *out4, hipStream_t s);
hipError_t dot_det(int64_t n, const double *a, const double *b, double *partial, double *out, hipStream_t s);
// entries of the partial-sum buffer that gauss_norms and dot_det use at most
int64_t gauss_partial_entries();

// compensated running sum: hi = fl(hi + d) (the plain FP64 sum), lo += its rounding error
hipError_t add_comp(int64_t n, double *hi, double *lo, const double *d, hipStream_t s);
// y = A (x_hi + x_lo) accumulated as a compensated (double-double) dot product per
// row; the result as y_hi + y_lo (y_lo may be null: y_hi is the rounded result)
hipError_t spmv_dd(const DevCSR &A, const double *x_hi, const double *x_lo, double *y_hi, double *y_lo,
                   hipStream_t s);

// out = a1 (P1 x1) + a2 (P2 (x2 + x2lo)) + c1 v1 + c2 v2 in double-double (out_hi +
// out_lo; out_lo may be null); any of P1, P2 (same row count), x2lo, v1, v2 may be null
hipError_t combo_dd(int64_t rows, const DevCSR *P1, const double *x1, double a1, const DevCSR *P2, const double *x2,
                    const double *x2lo, double a2, const double *v1, double c1, const double *v2, double c2,
                    double *out_hi, double *out_lo, hipStream_t s);
// x += scale f, compensated (xlo += the rounding error of each addition)
hipError_t add_f2d_comp(int64_t n, const float *f, double scale, double *x, double *xlo, hipStream_t s);

// impressed field (Sec. III-C): per-tet moments Pf[t][n2l] of B sampled at the
// P points of the collapsed Gauss rule (lamq [P][4], wq [P] summing to 1),
// B [nt][P][3], times scale
hipError_t launch_impressed_rhs(int order, const DevMesh &m, int P, const double *lamq, const double *wq,
                                const double *B, double scale, double *Pf, hipStream_t s);
// out = a .* b
hipError_t mul(int64_t n, const double *a, const double *b, double *out, hipStream_t s);
// dinv = 1 / diag(A), or 1 / diag(A diag(Dinv)^-1 A^T) when Dinv is given (1 where
// not positive)
hipError_t jacobi(const DevCSR &A, const double *Dinv, double *dinv, hipStream_t s);

// Device scratch of the entry point that allocates nothing
// (fempic_gauss_residual_noalloc): NOALLOC_SCRATCH_BYTES on every device, held
// until the process ends.  noalloc_scratch gives its address on the current
// device (looked up on the first call per device, then kept).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)96 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
hipError_t noalloc_scratch(void **ptr);

}  // namespace fempic
