// Run: device state of one simulation and its step sequencing.
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "fempic_impl.h"
#include "kernels.h"

namespace fempic {

void set_error(const std::string &s);
// allocator of device buffers made from now on (both null: hipMalloc/hipFree)
void set_device_allocator(fempic_alloc_fn a, fempic_free_fn f, void *ctx);
// EINVAL for parameters outside what the library supports
void check_params(const fempic_params &p);

// Device bytes held by one run's buffers, their peak, and an optional cap
// (0: none).  A buffer made while an account is current (AccountScope on this
// thread) is charged to it until it is freed; a buffer that would take the
// account past its cap is refused with ENOMEM.
struct DevAccount {
    size_t bytes = 0, peak = 0, limit = 0;
};
// makes `a` the account of the buffers this thread allocates during the scope
struct AccountScope {
    explicit AccountScope(DevAccount *a);
    ~AccountScope();
    AccountScope(const AccountScope &) = delete;
    AccountScope &operator=(const AccountScope &) = delete;
    DevAccount *prev;
};

// device buffer; freed with the allocator that made it
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    fempic_free_fn fr = nullptr;  // null: hipFree
    void *fr_ctx = nullptr;
    DevAccount *acct = nullptr;   // charged account, if any
    DevBuf() = default;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), fr(o.fr), fr_ctx(o.fr_ctx), acct(o.acct)
    {
        o.p = nullptr;
        o.bytes = 0;
        o.fr = nullptr;
        o.fr_ctx = nullptr;
        o.acct = nullptr;
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    void alloc(size_t n);
    void release();
};

struct DevCSRBuf {
    DevBuf ptr, idx, val, val32, bptr, bidx, bval, bval32;
    DevCSR desc{};
};

struct PBufs {
    DevBuf w;  // the rows' 16-byte words (PartLayout)
    DevParticles d{};
};

class Run {
  public:
    // the run shares ownership of its mesh, so destroying the caller's mesh
    // handle while the run lives leaves the run intact
    // byte_limit: cap of the run's device bytes (0: none), see set_byte_limit
    Run(std::shared_ptr<const HostMesh> mesh, const fempic_params &p, hipStream_t s, size_t byte_limit = 0);
    ~Run();
    void load(const double *pos, const double *vel, int64_t n, double q, double m, double w);
    // append n particles of the loaded species (ids after the existing ones),
    // started like loaded ones; their charge joins the Gauss check's reference
    void inject(const double *pos, const double *vel, int64_t n);
    void step(int n_steps);
    void sync();
    void gauss(double out[3]);
    // the same check with its intermediates in the library's static device
    // scratch: allocates nothing (EINVAL when the mesh needs more than it holds)
    void gauss_noalloc(double out[3]);
    void fields_get(double *e, int64_t ne, double *b, int64_t nb);
    void fields_set(const double *e, int64_t ne, const double *b, int64_t nb);
    void deposit_get(double *dg, int64_t n);
    // y = A x (natural W1 numbering): the assembled FP64 matrix or the PCG iterations' form
    void field_matvec(const double *x, double *y, int64_t n, int form);
    void rho_get(double *rho, double *rho0, int64_t n);
    // impressed magnetic flux density: B sampled at the points of the n1d^3 rule
    // of every tet, projected (constrained: onto the divergence-free faces) and
    // kept as the run's impressed field; b_out (nullable) receives it
    void impressed_set(const double *B, int64_t n, int n1d, bool constrained, double *b_out, int64_t nb);
    void particles_get(double *pos, double *vel, int64_t *tet, int64_t n);
    void history_get(double *vh, double *ah, int64_t n);
    void save(const char *path);
    void restore(const char *path);
    void set_log(const char *path);
    static size_t footprint_estimate(const HostMesh &m, int64_t n, bool mixed, bool absorbing = false);
    // replay the particle phase's launches as HIP graphs (see particle_phase);
    // its per-kernel times are then not measured
    void set_phase_graphs(bool on);
    // refuse (ENOMEM) any allocation that would take the run's device bytes past `bytes` (0: no cap)
    void set_byte_limit(size_t bytes) { acct.limit = bytes; }
    const DevAccount &account() const { return acct; }
    // the operator of the PCG iterations: 0 assembled, 1 tet by tet, 2 tet by tet in DoF pairs
    int field_op() const { return mf.order == 0 ? 0 : (mf.map1p ? 2 : 1); }

    DevAccount acct;  // before every buffer member: destroyed after them
    std::shared_ptr<const HostMesh> mesh_hold;
    const HostMesh &m;
    fempic_params prm;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;  // the HIP device the run was made on
    bool mixed = false;
    int order = 1, n1l = 0, n2l = 0, n0l = 0;
    // absorbing walls (params.field_bc); n1s: the unknown W1 DoFs, the first n1s of
    // the internal numbering (N1_int with PEC walls, N1 with absorbing ones)
    bool absorbing = false;
    int64_t n1s = 0;
    GLRule gl{};
    DevMesh dm{};
    // statistics
    // np: particles in the run now; np_loaded: at load (absorbed ones leave np)
    int64_t np = 0, np_loaded = 0, steps_done = 0, last_cross = 0, last_refl = 0, last_spill = 0;
    int64_t last_absorb = 0, absorbed_total = 0;
    double last_particle_ms = 0, last_kernel_ms = 0, last_continue_ms = 0, last_field_ms = 0, last_relres = 0;
    int32_t last_iters = 0;
    int64_t last_phase_replays = 0;
    int64_t nnz_total = 0, a_nnz = 0, a_inc = 0;
    double gauss_last[3] = {0, 0, 0};  // the last evaluation that params.gauss_every asked for
    int64_t gauss_step = 0;

  private:
    void upload_csr(DevCSRBuf &d, const CSR &A, bool want32);
    void zero(DevBuf &b);
    size_t particle_bytes(int64_t n) const;
    void alloc_particles(int64_t n, int64_t cap = 0);
    // rows [s0, s0 + n) of a particle buffer set to / from a host image of them
    // (the device layout with n in place of cap)
    std::vector<char> rows_get(const PBufs &B, int64_t s0, int64_t n);
    void rows_put(PBufs &B, int64_t s0, int64_t n, const std::vector<char> &img);
    std::vector<char> rows_new(const double *pos, const double *vel, int64_t n, int64_t id0) const;
    void alloc_sort(SortBuffers &sb, int64_t cap, std::vector<DevBuf> &hold);
    void alloc_pool(int64_t cap);
    DevParticles P(int k) const;
    SpillPool pool() const;
    int key_bits() const;
    int tpw() const;
    const uint32_t *sort_current();
    void locate_host(const double *pos, int64_t n, int32_t *out);
    void compute_rho(double *dst, double *Pr = nullptr);
    const PBufs &gather_current();
    void gauss_with(double *Pr, double *rho, double *GtDe, double *Gtg, double *y1, double *y1_lo, double *partial,
                    double *out4, double out[3]);
    void particle_phase();
    void next_order(int64_t nrec, const uint32_t *srec);
    void commit_order();
    void merge_order(int64_t np0, int64_t base, int64_t n);
    // rows of the current buffer set that may hold a particle: [0, rows_used)
    int64_t rows_used = 0;
    void field_phase();
    void field_phase_three_level();
    void solve_fp64();
    void solve_mixed();
    double pcg64(const double *b, double tol2, double bb);
    // preconditioned CG on a symmetric positive semi-definite operator (consistent
    // right-hand side) from x = 0 until |r| <= rtol |b|; returns the relative residual
    double cg_general(int64_t n, const std::function<void(const double *, double *)> &apply, const double *dinv,
                      const double *b, double *x, double rtol, int maxit);
    // the field coefficients the particle kernels read: b (+ the impressed field),
    // cast to FP32 in mixed precision
    void refresh_gather_b();
    const void *gather_b() const;
    double residual_dd(const double *x, const double *x_lo, double *r);
    double solve_target() const;
    // the refined field solve's target relative residual (exact, in double-double)
    static constexpr double GAUSS_RTOL = 1e-17;
    double read_sc(int k);
    // 8 PCG iterations (FP64, or the FP32 inner solve) as one HIP graph replay,
    // captured on first use; eager launches when graphs are off
    void pcg_batch(bool fp32);
    bool use_graphs = true;
    hipGraphExec_t pcg_graph[2] = {nullptr, nullptr};
    // the particle phase's launches, from k_particle to the next order, as graphs
    // keyed by everything their launch parameters depend on (buffers of the
    // alternating step parity, launch bounds, counts)
    bool phase_graphs = false, phase_timed = true;
    std::map<std::vector<int64_t>, hipGraphExec_t> phase_graph;
    void clear_phase_graphs();

    DevBuf d_geo, d_nbr, d_map1, d_map2, d_map0;
    DevCSRBuf A, Meps, Mnu, K, Kt, Gt, Zi;  // Zi: surface impedance *I (absorbing walls)
    double gscale = 1.0;  // Gt holds gscale G^T
    DevBuf d_dinv, d_dinv32, d_inc_ptr, d_inc_idx, d_inc0_ptr, d_inc0_idx;
    // A applied tet by tet in the PCG iterations (order 0: the assembled matrix)
    DevBuf d_mfgeo, d_mfpe, d_mfmap, d_mfptr2, d_mfslot;
    DevMF mf{};
    DevBuf d_e, d_b, d_g, d_dg, d_e32, d_b32;
    // rounding errors of the running sums e and g (compensated summation), and
    // the low half of *eps e in the Gauss check
    DevBuf d_e_lo, d_g_lo, d_y1_lo;
    // three-level Newmark-beta (gamma, beta other than 1/2, 1/4): e^{n-1}, b^{n-1},
    // g^n - g^{n-1}, and whether they hold a step yet (else the history is at rest)
    bool three_level = false, have_prev = false;
    DevBuf d_eprev, d_bprev, d_dgprev, v_b2;
    DevBuf v_x, v_r, v_z, v_p, v_q, v_rhs, v_tmp, v_u;
    // double-double halves of the right-hand side and the solution, the FP64
    // solver's accumulated solution, *nu u; the three-level scheme's previous
    // increment e^n - e^{n-1} as hi + lo
    DevBuf v_rhs_lo, v_x_lo, v_xs, v_nu, d_dprev, d_dprev_lo;
    // impressed field (face coefficients, FP64) and b + it, which the gather reads
    // (FP64 runs) or which is cast to FP32 for it (mixed runs)
    bool has_imp = false;
    DevBuf d_bimp, d_bg;
    DevBuf f_x, f_r, f_z, f_p, f_q;
    DevBuf d_partial, d_sc, d_rho, d_rho0, d_GtDe, d_Gtg, d_y1;
    DevBuf d_P, d_Pr, d_off, d_soff, d_ctl, d_cntb, d_args;
    // d_ctl holds the step's control words, read back in one copy:
    // [0, 64) counters (int64 x NCNT), [64, 96) small (int32 x 8: 0 appended spill
    // slots, 2 spill records, 6 queued paths), [96, 104) particle-order error
    static constexpr int CTL_SMALL = 8 * NCNT, CTL_PERR = CTL_SMALL + 32, CTL_BYTES = CTL_PERR + 8;
    unsigned long long *p_cnt = nullptr, *p_perr = nullptr;
    int32_t *p_small = nullptr;
    DevBuf d_pool_val, d_pool_tet, d_pool_tag, d_pool_pid, d_rcount, d_rpos, d_cq, d_qflag, d_qtmp, d_qidx;
    // particle order: cur_perm (sorted position -> slot) and d_off describe the
    // current state while perm_valid; the particle phase builds the next ones
    DevBuf d_moved, d_nstay, d_noff, d_tcnt;
    const uint32_t *cur_perm = nullptr;
    uint32_t *next_perm = nullptr;
    bool perm_valid = false;
    bool counts_known = false;  // nq_last, nslot_last, nrec_last hold the last step's counts
    std::vector<DevBuf> hp_sort, hp_ssort;
    PBufs pb[2];
    int cur = 0;
    SortBuffers psort{}, ssort{};
    int64_t pool_cap = 0, nrec_last = 0, nslot_last = 0, nq_last = 0;
    double q = 0, mass = 1, w = 0;
    bool loaded = false;
    int32_t sticky = 0;
    std::string sticky_msg;
    void *h_pin = nullptr;
    std::FILE *log = nullptr;  // per-step JSON lines (set_log)
    void log_step(float particle_ms, float kernel_ms, float continue_ms, float field_ms, bool with_gauss);
    hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_c1 = nullptr, ev_c = nullptr, ev_d = nullptr, ev_e = nullptr;
};

}  // namespace fempic
