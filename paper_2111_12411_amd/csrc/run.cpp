// Run driver and C ABI of the fempic library: device state in HBM, per-step
// sequencing of the particle phase (sort, particle kernel, deterministic
// deposit reduction) and of the implicit field update (Jacobi-PCG in FP64,
// or FP32 PCG inside FP64 iterative refinement), the Gauss-law check, and
// host <-> device copies in the natural DoF numbering.
#include <hip/hip_runtime_api.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "fempic_impl.h"
#include "kernels.h"
#include "run.h"

namespace fempic {

thread_local std::string g_last_error;

void set_error(const std::string &s) { g_last_error = s; }

#define HIPCHECK(x)                                                                                     \
    do {                                                                                                \
        hipError_t err__ = (x);                                                                         \
        if (err__ != hipSuccess)                                                                        \
            throw Error(FEMPIC_EDEVICE, std::string(#x) + ": " + hipGetErrorString(err__));             \
    } while (0)

// a named range on the roctx timeline (rocprofv3 --marker-trace) for the
// lifetime of a scope; host side, so it spans issue and the waits inside
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

// ------------------------------------------------------------ device memory
// device allocator of new buffers: hipMalloc/hipFree, or the caller's pair
namespace {
std::mutex alloc_mu;
fempic_alloc_fn alloc_fn = nullptr;
fempic_free_fn free_fn = nullptr;
void *alloc_ctx = nullptr;
}  // namespace

void set_device_allocator(fempic_alloc_fn a, fempic_free_fn f, void *ctx)
{
    if ((a == nullptr) != (f == nullptr)) throw Error(FEMPIC_EINVAL, "allocator needs both functions, or neither");
    std::lock_guard<std::mutex> g(alloc_mu);
    alloc_fn = a;
    free_fn = f;
    alloc_ctx = a ? ctx : nullptr;
}

namespace {
thread_local DevAccount *cur_account = nullptr;
}
AccountScope::AccountScope(DevAccount *a) : prev(cur_account) { cur_account = a; }
AccountScope::~AccountScope() { cur_account = prev; }

// HIP calls that act on the whole device (allocation, frees and the device
// synchronisation before them, stream and pinned-memory creation and
// destruction, graph instantiation) and stream captures exclude each other
// across the threads of a process: such a call made while another thread has
// a capture open on its own stream can invalidate that capture.
std::mutex &device_mu()
{
    static std::mutex mu;
    return mu;
}

DevBuf::~DevBuf() { release(); }
void DevBuf::release()
{
    if (p && acct) acct->bytes -= bytes;
    acct = nullptr;
    if (p) {
        std::lock_guard<std::mutex> g(device_mu());
        if (fr) {
            // the caller's allocator may hand the memory out at once, so wait
            // for every queued use first (as hipFree does)
            (void)hipDeviceSynchronize();
            fr(p, fr_ctx);
        } else {
            (void)hipFree(p);
        }
    }
    p = nullptr;
    bytes = 0;
    fr = nullptr;
    fr_ctx = nullptr;
}
void DevBuf::alloc(size_t n)
{
    release();
    if (n == 0) n = 16;
    DevAccount *a_ = cur_account;
    if (a_ && a_->limit && a_->bytes + n > a_->limit)
        throw Error(FEMPIC_ENOMEM, "a buffer of " + std::to_string(n) + " bytes would take the run past its device "
                                   "byte limit of " + std::to_string(a_->limit));
    fempic_alloc_fn a;
    fempic_free_fn f;
    void *ctx;
    {
        std::lock_guard<std::mutex> g(alloc_mu);
        a = alloc_fn;
        f = free_fn;
        ctx = alloc_ctx;
    }
    std::lock_guard<std::mutex> g(device_mu());
    if (a) {
        p = a(n, ctx);
        if (!p) throw Error(FEMPIC_ENOMEM, "the installed allocator failed to provide " + std::to_string(n) + " bytes");
        if ((uintptr_t)p % 256) {
            f(p, ctx);
            p = nullptr;
            throw Error(FEMPIC_EINVAL, "the installed allocator returned memory that is not 256-byte aligned");
        }
        fr = f;
        fr_ctx = ctx;
    } else {
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            throw Error(FEMPIC_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
        }
    }
    bytes = n;
    if (a_) {
        acct = a_;
        a_->bytes += n;
        a_->peak = std::max(a_->peak, a_->bytes);
    }
}

template <typename T>
static void upload(DevBuf &b, const std::vector<T> &v, hipStream_t s)
{
    b.alloc(v.size() * sizeof(T));
    if (!v.empty()) HIPCHECK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

static int lanes_for(const CSR &A)
{
    double avg = A.rows ? (double)A.nnz() / A.rows : 1;
    if (avg <= 8) return 4;
    if (avg <= 20) return 8;
    if (avg <= 48) return 16;
    return 32;
}

void Run::upload_csr(DevCSRBuf &d, const CSR &A, bool want32)
{
    upload(d.ptr, A.ptr, stream);
    upload(d.idx, A.idx, stream);
    upload(d.val, A.val, stream);
    if (want32) {
        std::vector<float> v32(A.val.begin(), A.val.end());
        upload(d.val32, v32, stream);
        HIPCHECK(hipStreamSynchronize(stream));
    }
    d.desc.rows = A.rows;
    d.desc.cols = A.cols;
    d.desc.nnz = A.nnz();
    d.desc.ptr = (const int64_t *)d.ptr.p;
    d.desc.idx = (const int32_t *)d.idx.p;
    d.desc.val = (const double *)d.val.p;
    d.desc.val32 = want32 ? (const float *)d.val32.p : nullptr;
    d.desc.lanes = lanes_for(A);
    d.desc.brows = 0;
    d.desc.bptr = nullptr;
    d.desc.bidx = nullptr;
    d.desc.bval = nullptr;
    d.desc.bval32 = nullptr;
    // 2x2 block copy when the pattern is exactly blocked (order 2: the two DoFs of
    // an edge or a face are adjacent and couple with the same neighbours)
    if (A.rows % 2 || A.cols % 2 || A.rows == 0) return;
    const int64_t R = A.rows / 2;
    std::vector<int64_t> bptr(R + 1, 0);
    std::vector<int32_t> bidx;
    std::vector<double> bval;
    bidx.reserve(A.nnz() / 4);
    bval.reserve(A.nnz());
    std::vector<std::pair<int32_t, double>> r0, r1;
    for (int64_t b = 0; b < R; b++) {
        r0.clear();
        r1.clear();
        for (int64_t k = A.ptr[2 * b]; k < A.ptr[2 * b + 1]; k++) r0.emplace_back(A.idx[k], A.val[k]);
        for (int64_t k = A.ptr[2 * b + 1]; k < A.ptr[2 * b + 2]; k++) r1.emplace_back(A.idx[k], A.val[k]);
        std::sort(r0.begin(), r0.end());
        std::sort(r1.begin(), r1.end());
        if (r0.size() != r1.size() || r0.size() % 2) return;
        for (size_t k = 0; k < r0.size(); k += 2) {
            const int32_t c = r0[k].first;
            if (c % 2 || r0[k + 1].first != c + 1 || r1[k].first != c || r1[k + 1].first != c + 1) return;
            bidx.push_back(c / 2);
            bval.push_back(r0[k].second);
            bval.push_back(r0[k + 1].second);
            bval.push_back(r1[k].second);
            bval.push_back(r1[k + 1].second);
        }
        bptr[b + 1] = (int64_t)bidx.size();
    }
    upload(d.bptr, bptr, stream);
    upload(d.bidx, bidx, stream);
    upload(d.bval, bval, stream);
    if (want32) {
        std::vector<float> b32(bval.begin(), bval.end());
        upload(d.bval32, b32, stream);
    }
    HIPCHECK(hipStreamSynchronize(stream));  // the host vectors are freed on return
    d.desc.brows = R;
    d.desc.bptr = (const int64_t *)d.bptr.p;
    d.desc.bidx = (const int32_t *)d.bidx.p;
    d.desc.bval = (const double *)d.bval.p;
    d.desc.bval32 = want32 ? (const float *)d.bval32.p : nullptr;
}

Run::Run(std::shared_ptr<const HostMesh> mesh, const fempic_params &p, hipStream_t s, size_t byte_limit)
    : mesh_hold(std::move(mesh)), m(*mesh_hold), prm(p)
{
    acct.limit = byte_limit;
    AccountScope charge(&acct);
    HIPCHECK(hipGetDevice(&device));
    if (s) {
        stream = s;
        own_stream = false;
    } else {
        std::lock_guard<std::mutex> g(device_mu());
        HIPCHECK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        own_stream = true;
    }
    mixed = p.precision == FEMPIC_MIXED;
    order = m.order;
    n1l = m.n1l;
    n2l = m.n2l;
    n0l = m.n0l;
    const RefElem &R = ref_elem(order);
    for (int g = 0; g < (int)R.glx.size(); g++) {
        gl.x[g] = R.glx[g];
        gl.w[g] = R.glw[g];
    }
    // mesh tables
    upload(d_geo, m.geo, stream);
    {
        // device neighbour table: 4 nb + (face of nb shared with t), -1 at a wall
        std::vector<int32_t> nbx(m.nbr.size(), -1);
        for (int64_t t = 0; t < m.nt; t++)
            for (int f = 0; f < 4; f++) {
                const int32_t nb = m.nbr[4 * t + f];
                if (nb < 0) continue;
                int en = -1;
                for (int q = 0; q < 4; q++)
                    if (m.nbr[4 * (int64_t)nb + q] == (int32_t)t) en = q;
                if (en < 0) throw Error(FEMPIC_EMESH, "inconsistent neighbour table");
                nbx[4 * t + f] = 4 * nb + en;
            }
        upload(d_nbr, nbx, stream);
        HIPCHECK(hipStreamSynchronize(stream));  // nbx is freed at the end of this block
    }
    upload(d_map1, m.map1, stream);
    upload(d_map2, m.map2, stream);
    upload(d_map0, m.map0, stream);
    dm.nt = (int32_t)m.nt;
    dm.geo = (const double *)d_geo.p;
    dm.nbr = (const int32_t *)d_nbr.p;
    dm.map1 = (const int32_t *)d_map1.p;
    dm.map2 = (const int32_t *)d_map2.p;
    dm.map0 = (const int32_t *)d_map0.p;
    dm.cube_N = m.is_cube ? m.cube_N : 0;
    dm.cube_L = m.cube_L;
    // operators
    Operators ops;
    three_level = !(p.gamma == 0.5 && p.beta == 0.25);
    absorbing = p.field_bc == FEMPIC_FIELD_ABSORB;
    assemble(m, p.dt, ops, (p.beta / p.gamma) * (p.beta / p.gamma), absorbing);
    n1s = ops.n1s;
    upload_csr(A, ops.A, mixed);
    if (absorbing) upload_csr(Zi, ops.Z, false);
    upload_csr(Meps, ops.Meps, false);
    upload_csr(Mnu, ops.Mnu, false);
    upload_csr(K, ops.K, false);
    upload_csr(Kt, ops.Kt, false);
    upload_csr(Gt, ops.Gt, false);
    gscale = ops.gscale;
    {
        // preconditioner: inverse 2x2 diagonal blocks when A is 2x2-blocked, else 1/A_ii
        std::vector<double> dinv = ops.Adiag_inv;
        if (A.desc.bptr) {
            const CSR &Ah = ops.A;
            dinv.assign(2 * (size_t)Ah.rows, 0.0);
            for (int64_t j = 0; 2 * j < Ah.rows; j++) {
                double blk[2][2] = {{0, 0}, {0, 0}};
                for (int h = 0; h < 2; h++)
                    for (int64_t k = Ah.ptr[2 * j + h]; k < Ah.ptr[2 * j + h + 1]; k++)
                        if (Ah.idx[k] == 2 * j || Ah.idx[k] == 2 * j + 1) blk[h][Ah.idx[k] - 2 * j] = Ah.val[k];
                const double det = blk[0][0] * blk[1][1] - blk[0][1] * blk[1][0];
                if (!(det > 0.0)) throw Error(FEMPIC_EMESH, "system matrix has a singular diagonal block");
                dinv[4 * j] = blk[1][1] / det;
                dinv[4 * j + 1] = -blk[0][1] / det;
                dinv[4 * j + 2] = -blk[1][0] / det;
                dinv[4 * j + 3] = blk[0][0] / det;
            }
        }
        upload(d_dinv, dinv, stream);
        std::vector<float> d32(dinv.begin(), dinv.end());
        if (mixed) upload(d_dinv32, d32, stream);
        HIPCHECK(hipStreamSynchronize(stream));  // dinv and d32 are freed at the end of this block
    }
    upload(d_inc_ptr, ops.inc_ptr, stream);
    upload(d_inc_idx, ops.inc_idx, stream);
    upload(d_inc0_ptr, ops.inc0_ptr, stream);
    upload(d_inc0_idx, ops.inc0_idx, stream);
    // the PCG iterations apply A tet by tet (PEC walls; FEMPIC_MATFREE=0 keeps the
    // assembled matrix): per tet the gradients of l_0..l_3 and the volume, in the
    // precision of the iterations (FP32 inner solve in mixed precision)
    {
        const char *mfe = std::getenv("FEMPIC_MATFREE");
        const bool mf_on = !absorbing && !(mfe && std::strcmp(mfe, "0") == 0);
        mf = DevMF{};
        if (mf_on) {
            const int64_t nt = m.nt;
            std::vector<double> g64((size_t)nt * 16, 0.0);
            for (int64_t t = 0; t < nt; t++) {
                for (int v = 0; v < 4; v++)
                    for (int c = 0; c < 3; c++) g64[16 * t + 3 * v + c] = m.geo[16 * t + 4 * v + 1 + c];
                g64[16 * t + 12] = m.vol[t];
            }
            if (mixed) {
                std::vector<float> g32(g64.begin(), g64.end());
                upload(d_mfgeo, g32, stream);
                HIPCHECK(hipStreamSynchronize(stream));
                d_mfpe.alloc((size_t)nt * n1l * 4);
            } else {
                upload(d_mfgeo, g64, stream);
                HIPCHECK(hipStreamSynchronize(stream));
                d_mfpe.alloc((size_t)nt * n1l * 8);
            }
            const double c_dt2 = (p.beta / p.gamma) * (p.beta / p.gamma);
            mf = DevMF{order, nt, n1s, (const int32_t *)d_map1.p, d_mfgeo.p, (const int64_t *)d_inc_ptr.p,
                       (const int32_t *)d_inc_idx.p, d_mfpe.p, EPS0, c_dt2 * p.dt * p.dt / MU0,
                       nullptr, nullptr, nullptr};
            // order 2: pair the two DoFs of each edge and face when every tet lists
            // them as adjacent unknowns 2j, 2j+1 (the internal numbering does)
            if (order == 2 && n1s % 2 == 0) {
                const int np = n1l / 2;
                std::vector<int32_t> mp((size_t)nt * np);
                bool ok = true;
                for (int64_t t = 0; t < nt && ok; t++)
                    for (int i = 0; i < np; i++) {
                        const int32_t a = m.map1[(size_t)t * n1l + 2 * i], b = m.map1[(size_t)t * n1l + 2 * i + 1];
                        if (a < n1s || b < n1s) {
                            ok = ok && a % 2 == 0 && b == a + 1 && b < n1s;
                            mp[(size_t)t * np + i] = a / 2;
                        } else {
                            mp[(size_t)t * np + i] = -1;
                        }
                    }
                // per pair the incidences of its even DoF (the odd one's must be the next
                // positions), numbered in order: the position of each (tet, pair) in pe
                std::vector<int64_t> p2((size_t)n1s / 2 + 1, 0);
                std::vector<int32_t> sl((size_t)nt * np, -1);
                if (ok) {
                    int64_t pos = 0;
                    for (int64_t j = 0; j < n1s / 2 && ok; j++) {
                        const int64_t a0 = ops.inc_ptr[2 * j], a1 = ops.inc_ptr[2 * j + 1], b1 = ops.inc_ptr[2 * j + 2];
                        ok = a1 - a0 == b1 - a1;
                        for (int64_t q = 0; ok && q < a1 - a0; q++) {
                            const int32_t e = ops.inc_idx[a0 + q];  // t n1l + local
                            ok = e % 2 == 0 && ops.inc_idx[a1 + q] == e + 1 && sl[e / 2] < 0;
                            sl[e / 2] = (int32_t)pos++;
                        }
                        p2[j + 1] = pos;
                    }
                    for (int64_t t = 0; t < nt && ok; t++)
                        for (int i = 0; i < np; i++) ok = ok && (mp[(size_t)t * np + i] < 0) == (sl[(size_t)t * np + i] < 0);
                }
                if (ok) {
                    upload(d_mfmap, mp, stream);
                    upload(d_mfptr2, p2, stream);
                    upload(d_mfslot, sl, stream);
                    HIPCHECK(hipStreamSynchronize(stream));
                    mf.map1p = (const int32_t *)d_mfmap.p;
                    mf.ptr2 = (const int64_t *)d_mfptr2.p;
                    mf.slot2 = (const int32_t *)d_mfslot.p;
                }
            }
            // order 2 is applied in pairs only: without them the iterations keep the assembled matrix
            if (order == 2 && !mf.map1p) {
                mf = DevMF{};
                d_mfgeo.release();
                d_mfpe.release();
            }
        }
    }
    nnz_total = ops.A.nnz() + ops.Meps.nnz() + ops.Mnu.nnz() + ops.K.nnz() + ops.Kt.nnz() + ops.Gt.nnz();
    a_nnz = ops.A.nnz();
    a_inc = (int64_t)ops.inc_idx.size();
    // fields and solver vectors
    const int64_t N1 = m.N1, N1i = n1s, N2 = m.N2, N0i = m.N0_int;
    d_e.alloc(N1 * 8);
    d_b.alloc(N2 * 8);
    d_g.alloc(std::max<int64_t>(N1i, 1) * 8);
    d_dg.alloc(std::max<int64_t>(N1i, 1) * 8);
    for (auto *v : {&d_e_lo, &d_g_lo, &d_y1_lo}) v->alloc(std::max<int64_t>(N1i, 1) * 8);
    zero(d_e);
    zero(d_b);
    zero(d_g);
    zero(d_dg);
    zero(d_e_lo);
    zero(d_g_lo);
    if (mixed) {
        d_e32.alloc(N1 * 4);
        d_b32.alloc(N2 * 4);
        zero(d_e32);
        zero(d_b32);
    }
    for (auto *v : {&v_x, &v_r, &v_z, &v_p, &v_q, &v_rhs, &v_tmp, &v_rhs_lo, &v_x_lo, &v_xs})
        v->alloc(std::max<int64_t>(N1i, 1) * 8);
    v_nu.alloc(std::max<int64_t>(N2, 1) * 8);
    if (mixed)
        for (auto *v : {&f_x, &f_r, &f_z, &f_p, &f_q}) v->alloc(std::max<int64_t>(N1i, 1) * 4);
    v_u.alloc(std::max<int64_t>(N2, 1) * 8);
    if (three_level) {
        d_eprev.alloc(std::max<int64_t>(N1i, 1) * 8);
        d_bprev.alloc(std::max<int64_t>(N2, 1) * 8);
        d_dgprev.alloc(std::max<int64_t>(N1i, 1) * 8);
        d_dprev.alloc(std::max<int64_t>(N1i, 1) * 8);
        d_dprev_lo.alloc(std::max<int64_t>(N1i, 1) * 8);
        v_b2.alloc(std::max<int64_t>(N2, 1) * 8);
        zero(d_eprev);
        zero(d_bprev);
        zero(d_dgprev);
        zero(d_dprev);
        zero(d_dprev_lo);
    }
    const int64_t maxrows = std::max<int64_t>({N1i, N2, N0i, 1});
    d_partial.alloc((size_t)(maxrows / 4 + 1024) * 4 * 8);
    d_sc.alloc(64 * 8);
    zero(d_sc);
    d_rho.alloc(std::max<int64_t>(N0i, 1) * 8);
    d_rho0.alloc(std::max<int64_t>(N0i, 1) * 8);
    d_GtDe.alloc(std::max<int64_t>(N0i, 1) * 8);
    d_Gtg.alloc(std::max<int64_t>(N0i, 1) * 8);
    d_y1.alloc(std::max<int64_t>(N1i, 1) * 8);
    zero(d_rho0);
    d_P.alloc((size_t)m.nt * n1l * 8);
    d_Pr.alloc((size_t)m.nt * n0l * 8);
    d_off.alloc((size_t)(m.nt + 1) * 4);
    d_noff.alloc((size_t)(m.nt + 1) * 4);
    d_tcnt.alloc((size_t)std::max<int64_t>(m.nt, 1) * 4);
    d_nstay.alloc((size_t)std::max<int64_t>(m.nt, 1) * 4);
    d_soff.alloc((size_t)(m.nt + 1) * 4);
    d_ctl.alloc(128);
    zero(d_ctl);
    p_cnt = (unsigned long long *)d_ctl.p;
    p_small = (int32_t *)((char *)d_ctl.p + CTL_SMALL);
    p_perr = (unsigned long long *)((char *)d_ctl.p + CTL_PERR);
    d_cntb.alloc((size_t)CONT_BLOCKS * NCNT * 8);
    {
        std::lock_guard<std::mutex> g(device_mu());
        HIPCHECK(hipHostMalloc(&h_pin, 128 + sizeof(ParticleArgs) + 64, hipHostMallocDefault));
    }
    d_args.alloc(sizeof(ParticleArgs));
    for (auto *ev : {&ev_a, &ev_b, &ev_c1, &ev_c, &ev_d, &ev_e}) HIPCHECK(hipEventCreate(ev));
    // FEMPIC_GRAPHS=0 launches the PCG batches (and the particle phase) kernel by
    // kernel instead of replaying graphs; FEMPIC_PHASE_GRAPHS=1 replays the
    // particle phase as graphs (set_phase_graphs; the server's runs always do)
    const char *g = std::getenv("FEMPIC_GRAPHS");
    use_graphs = !(g && std::strcmp(g, "0") == 0);
    const char *pg = std::getenv("FEMPIC_PHASE_GRAPHS");
    phase_graphs = pg && std::strcmp(pg, "1") == 0;
    HIPCHECK(hipStreamSynchronize(stream));
}

Run::~Run()
{
    if (log) std::fclose(log);
    if (stream) (void)hipStreamSynchronize(stream);
    clear_phase_graphs();
    std::lock_guard<std::mutex> g(device_mu());
    for (auto &gx : pcg_graph)
        if (gx) (void)hipGraphExecDestroy(gx);
    for (auto ev : {ev_a, ev_b, ev_c1, ev_c, ev_d, ev_e})
        if (ev) (void)hipEventDestroy(ev);
    if (h_pin) (void)hipHostFree(h_pin);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
}

void Run::clear_phase_graphs()
{
    std::lock_guard<std::mutex> g(device_mu());
    for (auto &kv : phase_graph)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    phase_graph.clear();
}

void Run::set_phase_graphs(bool on)
{
    HIPCHECK(hipStreamSynchronize(stream));
    phase_graphs = on;
    if (!on) clear_phase_graphs();
}

void Run::zero(DevBuf &b)
{
    if (b.bytes) HIPCHECK(hipMemsetAsync(b.p, 0, b.bytes, stream));
}

void Run::sync()
{
    HIPCHECK(hipStreamSynchronize(stream));
    if (sticky) throw Error(sticky, sticky_msg);
}

size_t Run::particle_bytes(int64_t n) const { return (size_t)n * part_layout(mixed).nw * 16; }

namespace {
// a host image of particle rows: the device layout with the row count in place of cap
template <typename T>
T unit_get(const std::vector<char> &img, int64_t n, int u, int64_t s)
{
    T x;
    std::memcpy(&x, img.data() + part_off(u, n, s), sizeof x);
    return x;
}
template <typename T>
void unit_set(std::vector<char> &img, int64_t n, int u, int64_t s, T x)
{
    std::memcpy(img.data() + part_off(u, n, s), &x, sizeof x);
}
}  // namespace

std::vector<char> Run::rows_get(const PBufs &B, int64_t s0, int64_t n)
{
    const int nw = part_layout(mixed).nw;
    std::vector<char> img((size_t)std::max<int64_t>(n, 1) * nw * 16);
    for (int k = 0; k < nw && n > 0; k++)
        HIPCHECK(hipMemcpyAsync(img.data() + (size_t)k * n * 16, (const char *)B.w.p + ((size_t)k * B.d.cap + s0) * 16,
                                (size_t)n * 16, hipMemcpyDeviceToHost, stream));
    HIPCHECK(hipStreamSynchronize(stream));
    return img;
}

void Run::rows_put(PBufs &B, int64_t s0, int64_t n, const std::vector<char> &img)
{
    const int nw = part_layout(mixed).nw;
    for (int k = 0; k < nw && n > 0; k++)
        HIPCHECK(hipMemcpyAsync((char *)B.w.p + ((size_t)k * B.d.cap + s0) * 16, img.data() + (size_t)k * n * 16,
                                (size_t)n * 16, hipMemcpyHostToDevice, stream));
    HIPCHECK(hipStreamSynchronize(stream));
}

// image of n new particles: positions (in the l_1..l_3 units, until they are
// located), velocities and ids from id0; the rest zero
std::vector<char> Run::rows_new(const double *pos, const double *vel, int64_t n, int64_t id0) const
{
    const PartLayout &L = part_layout(mixed);
    std::vector<char> img((size_t)std::max<int64_t>(n, 1) * L.nw * 16, 0);
    for (int64_t i = 0; i < n; i++) {
        for (int c = 0; c < 3; c++) {
            unit_set<double>(img, n, L.lam + 2 * c, i, pos[3 * i + c]);
            unit_set<double>(img, n, L.v + 2 * c, i, vel[3 * i + c]);
        }
        unit_set<int32_t>(img, n, L.id, i, (int32_t)(id0 + i));
    }
    return img;
}

void Run::alloc_particles(int64_t n, int64_t cap_want)
{
    clear_phase_graphs();  // they name the old buffers
    np = n;
    np_loaded = n;
    const int64_t cap = std::max<int64_t>({n, cap_want, 1});
    for (int k = 0; k < 2; k++) {
        PBufs &B = pb[k];
        B.w.alloc(particle_bytes(cap));
        // rows start zero: unused units stay defined, and without AB4 (the Boris
        // push) the histories stay zero in both sets
        zero(B.w);
        B.d.w = B.w.p;
        B.d.cap = cap;
    }
    cur = 0;
    rows_used = n;
    perm_valid = false;
    counts_known = false;
    // particle sort
    alloc_sort(psort, cap, hp_sort);
    // spill pool
    pool_cap = std::max<int64_t>(cap + cap / 2, 1 << 16);
    alloc_pool(pool_cap);
    d_rcount.alloc(cap * 4);
    d_rpos.alloc(cap * 4);
    d_cq.alloc((size_t)cap * sizeof(ContRec));
    d_qflag.alloc(cap + 16);  // byte flags, read 16 at a time
    d_moved.alloc(cap);
    d_qtmp.alloc((2 * (cap / 4096 + 1) + scan_tmp_entries(cap / 4096 + 1)) * 4 + 64);
    d_qidx.alloc(cap * 4);
}

void Run::alloc_sort(SortBuffers &sb, int64_t cap, std::vector<DevBuf> &hold)
{
    hold.resize(6);
    for (int k = 0; k < 2; k++) {
        hold[k].alloc(cap * 4);
        hold[2 + k].alloc(cap * 4);
        sb.key[k] = (uint32_t *)hold[k].p;
        sb.val[k] = (uint32_t *)hold[2 + k].p;
    }
    const int64_t hn = sort_hist_entries(cap);
    hold[4].alloc(hn * 4);
    // the scans: histograms, particle flags, and per-tet bucket sizes
    hold[5].alloc(std::max({scan_tmp_entries(hn), scan_tmp_entries(cap), scan_tmp_entries(m.nt)}) * 4 + 64);
    sb.hist = (uint32_t *)hold[4].p;
    sb.scan_tmp = (uint32_t *)hold[5].p;
    sb.cap = cap;
}

void Run::alloc_pool(int64_t cap)
{
    if (cap >= (int64_t)SREC_LAST) throw Error(FEMPIC_ENOMEM, "spill pool beyond 2^31 records");
    clear_phase_graphs();  // they name the old pool
    pool_cap = cap;
    d_pool_val.alloc((size_t)cap * n1l * 8);
    d_pool_pid.alloc((size_t)cap * 4);
    d_pool_tet.alloc((size_t)cap * 4);
    d_pool_tag.alloc((size_t)cap * 8);
    alloc_sort(ssort, cap, hp_ssort);
}

DevParticles Run::P(int k) const { return pb[k].d; }

SpillPool Run::pool() const
{
    SpillPool sp;
    sp.val = (double *)d_pool_val.p;
    sp.tet = (int32_t *)d_pool_tet.p;
    sp.tag = (int64_t *)d_pool_tag.p;
    sp.pid = (int32_t *)d_pool_pid.p;
    sp.count = p_small;
    sp.rcount = (int32_t *)d_rcount.p;
    sp.cap = pool_cap;
    return sp;
}

int Run::key_bits() const
{
    int bits = 1;
    while (((int64_t)1 << bits) < m.nt) bits++;
    return bits;
}

// sort the current particles by tet: returns perm (sorted -> slot) and fills d_off
const uint32_t *Run::sort_current()
{
    if (perm_valid) return cur_perm;
    int res = 0;
    HIPCHECK(launch_tet_keys(pb[cur].d, np, psort.key[0], stream));
    HIPCHECK(radix_sort(psort, np, key_bits(), true, &res, stream, nullptr));
    HIPCHECK(launch_offsets(psort.key[res], np, (int32_t)m.nt, (int32_t *)d_off.p, stream));
    cur_perm = psort.val[res];
    perm_valid = true;
    return cur_perm;
}

// the particle order of the state the particle phase has just written: per
// tet, its particles that were not queued, then the queued ones whose path
// ended in it (srec: the tet-sorted spill records, at most nrec of them).
// Built into the buffers not in use; commit_order() makes it current.
void Run::next_order(int64_t nrec, const uint32_t *srec)
{
    HIPCHECK(exclusive_scan_u32((const uint32_t *)d_tcnt.p, (uint32_t *)d_noff.p, m.nt, psort.scan_tmp,
                                (uint32_t *)d_noff.p + m.nt, stream));
    HIPCHECK(launch_place(np, (int32_t)m.nt, tpw(), (const int32_t *)d_off.p, (const uint8_t *)d_moved.p,
                          (const int32_t *)d_soff.p, srec, nrec,
                          (const int32_t *)d_pool_pid.p, pool_cap, (const int32_t *)d_noff.p, next_perm,
                          p_perr, stream));
}

// The new rows [base, base + n) of the current buffer set join the current order
// of its np0 particles:
// each tet keeps its particles in their order and takes its new ones after
// them, in row order (what a stable sort of the appended state by tet gives).
// The keys of the new rows are sorted with the spill-record sort buffers.
void Run::merge_order(int64_t np0, int64_t base, int64_t n)
{
    sort_current();
    HIPCHECK(launch_tet_keys(part_rows(pb[cur].d, base), n, ssort.key[0], stream));
    int res = 0;
    HIPCHECK(radix_sort(ssort, n, key_bits(), true, &res, stream, nullptr));
    HIPCHECK(launch_offsets(ssort.key[res], n, (int32_t)m.nt, (int32_t *)d_soff.p, stream));
    next_perm = cur_perm == psort.val[0] ? psort.val[1] : psort.val[0];
    HIPCHECK(launch_merge_order(np0, n, (int32_t)m.nt, (const int32_t *)d_off.p, (const int32_t *)d_soff.p, cur_perm,
                                ssort.key[res], ssort.val[res], (uint32_t)base, (int32_t *)d_noff.p, next_perm, stream));
    commit_order();
}

void Run::commit_order()
{
    std::swap(d_off.p, d_noff.p);
    std::swap(d_off.bytes, d_noff.bytes);
    cur_perm = next_perm;
    perm_valid = true;
}

void Run::load(const double *pos, const double *vel, int64_t n, double q_, double mass_, double w_)
{
    Range rg("fempic load");
    AccountScope charge(&acct);
    if (n < 0 || (n > 0 && (!pos || !vel))) throw Error(FEMPIC_EINVAL, "bad particle arrays");
    if (!(mass_ > 0) || !std::isfinite(q_) || !std::isfinite(w_)) throw Error(FEMPIC_EINVAL, "bad species");
    if (n >= ((int64_t)1 << 31) / 2) throw Error(FEMPIC_EINVAL, "too many particles");
    for (int64_t k = 0; k < 3 * n; k++)
        if (!std::isfinite(pos[k]) || !std::isfinite(vel[k]))
            throw Error(FEMPIC_EINVAL, "particle " + std::to_string(k / 3) + " has a non-finite position or velocity");
    q = q_;
    mass = mass_;
    w = w_;
    alloc_particles(n);
    PBufs &B = pb[0];
    {
        std::vector<char> img = rows_new(pos, vel, n, 0);
        if (!m.is_cube) {
            std::vector<int32_t> tets(std::max<int64_t>(n, 1));
            locate_host(pos, n, tets.data());
            for (int64_t i = 0; i < n; i++) unit_set<int32_t>(img, n, part_layout(mixed).tet, i, tets[i]);
        }
        rows_put(B, 0, n, img);
    }
    if (m.is_cube) {
        HIPCHECK(hipMemsetAsync(p_small, 0, 4, stream));
        HIPCHECK(launch_locate_cube(dm, n, B.d, p_small, stream));
        int32_t err = 0;
        HIPCHECK(hipMemcpyAsync(&err, p_small, 4, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        if (err & ERR_OUTSIDE) throw Error(FEMPIC_EOUTSIDE, "a particle lies outside the mesh");
    }
    // the positions become barycentric coordinates in the located tets
    HIPCHECK(launch_to_bary(dm, n, B.d, stream));
    if (prm.pusher != FEMPIC_PUSH_BORIS) {
        // AB4 start-up from the current fields
        HIPCHECK(launch_startup(order, mixed, dm, (const double *)d_e.p, (const double *)gather_b(),
                                (const float *)d_e32.p, (const float *)d_b32.p, B.d, n, q / mass, prm.dt, stream));
    }
    // store the particles in tet order, so the first step reads them like every later one
    {
        const uint32_t *perm = sort_current();
        HIPCHECK(launch_permute(mixed, pb[0].d, pb[1].d, perm, n, stream));
        cur = 1;
        rows_used = n;
        perm_valid = false;
    }
    // Gauss reference charge
    compute_rho((double *)d_rho0.p);
    zero(d_g);
    zero(d_g_lo);
    HIPCHECK(hipStreamSynchronize(stream));
    have_prev = false;  // the three-level scheme starts from a history at rest
    absorbed_total = 0;
    last_absorb = 0;
    gauss_step = 0;
    for (double &g : gauss_last) g = 0.0;
    sticky = 0;
    loaded = true;
}

// Particle injection: the current state is gathered into the next step's order
// (tet-sorted rows [0, np)), grown into larger buffers when it must be, and the
// new particles are appended after it, located, given barycentric coordinates
// and started like loaded ones; the next step sorts the whole set.  Charge
// enters the run here, not through the deposit, so the Gauss check's reference
// rho~^0 takes the new particles' nodal charge (like that of the particles
// present at load): the check then measures the current of every particle since
// it appeared.
void Run::inject(const double *pos, const double *vel, int64_t n)
{
    sync();
    AccountScope charge(&acct);
    if (!loaded) throw Error(FEMPIC_EINVAL, "no particles loaded");
    if (n < 0 || (n > 0 && (!pos || !vel))) throw Error(FEMPIC_EINVAL, "bad particle arrays");
    if (np_loaded + n >= ((int64_t)1 << 31) / 2) throw Error(FEMPIC_EINVAL, "too many particles");
    for (int64_t k = 0; k < 3 * n; k++)
        if (!std::isfinite(pos[k]) || !std::isfinite(vel[k]))
            throw Error(FEMPIC_EINVAL, "particle " + std::to_string(k / 3) + " has a non-finite position or velocity");
    if (n == 0) return;
    // rho~ before and after, in the Gauss check's scratch vectors (N0_int each)
    DevBuf &rho_a = d_GtDe, &rho_b = d_Gtg;
    compute_rho((double *)rho_a.p);
    const int64_t np0 = np, np1 = np0 + n, id0 = np_loaded;
    // With room in the current buffer set the new rows go after every row that may
    // hold a particle (the last step wrote rows [0, rows_used); the particles it
    // absorbed left holes there) and are merged into the current particle order
    // (below); otherwise the state is gathered into tet order, grown, and the
    // next step sorts the whole set.
    int64_t base = rows_used;
    const bool room = base + n <= pb[cur].d.cap;
    if (!room) {
        gather_current();
        cur = 1 - cur;  // the gathered, tet-sorted rows are now the state
        base = np0;
    }
    if (!room) {
        // grow by half again, keeping the gathered rows
        PBufs old = std::move(pb[cur]);
        const int64_t oc = old.d.cap;
        const int64_t nl = np_loaded;
        alloc_particles(np0, np1 + np1 / 2);
        np_loaded = nl;
        const int64_t nc = pb[0].d.cap;
        PBufs &B = pb[0];
        for (int k = 0; k < part_layout(mixed).nw && np0 > 0; k++)
            HIPCHECK(hipMemcpyAsync((char *)B.w.p + (size_t)k * nc * 16, (const char *)old.w.p + (size_t)k * oc * 16,
                                    (size_t)np0 * 16, hipMemcpyDeviceToDevice, stream));
        HIPCHECK(hipStreamSynchronize(stream));  // old is freed at the end of this block
        cur = 0;
    }
    PBufs &B = pb[cur];
    {
        std::vector<char> img = rows_new(pos, vel, n, id0);
        if (!m.is_cube) {
            std::vector<int32_t> tets(n);
            locate_host(pos, n, tets.data());
            for (int64_t i = 0; i < n; i++) unit_set<int32_t>(img, n, part_layout(mixed).tet, i, tets[i]);
        }
        rows_put(B, base, n, img);
    }
    const DevParticles nw = part_rows(B.d, base);
    if (m.is_cube) {
        HIPCHECK(hipMemsetAsync(p_small, 0, 4, stream));
        HIPCHECK(launch_locate_cube(dm, n, nw, p_small, stream));
        int32_t err = 0;
        HIPCHECK(hipMemcpyAsync(&err, p_small, 4, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        if (err & ERR_OUTSIDE) throw Error(FEMPIC_EOUTSIDE, "an injected particle lies outside the mesh");
    }
    HIPCHECK(launch_to_bary(dm, n, nw, stream));
    if (prm.pusher != FEMPIC_PUSH_BORIS)
        HIPCHECK(launch_startup(order, mixed, dm, (const double *)d_e.p, (const double *)gather_b(),
                                (const float *)d_e32.p, (const float *)d_b32.p, nw, n, q / mass, prm.dt, stream));
    if (room) merge_order(np0, base, n);
    rows_used = base + n;
    np = np1;
    np_loaded = id0 + n;
    if (!room) perm_valid = false;
    counts_known = false;
    // rho~^0 += the new particles' charge (rho~ after minus rho~ before)
    compute_rho((double *)rho_b.p);
    HIPCHECK(axpby(m.N0_int, 1.0, (const double *)rho_b.p, -1.0, (const double *)rho_a.p, (double *)rho_b.p,
                   stream));
    HIPCHECK(axpby(m.N0_int, 1.0, (const double *)d_rho0.p, 1.0, (const double *)rho_b.p, (double *)d_rho0.p,
                   stream));
    HIPCHECK(hipStreamSynchronize(stream));
}

// uniform-bin point location for meshes that are not Kuhn cubes (host side, at load)
void Run::locate_host(const double *pos, int64_t n, int32_t *out)
{
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < m.nv; v++)
        for (int c = 0; c < 3; c++) {
            lo[c] = std::min(lo[c], m.xyz[3 * v + c]);
            hi[c] = std::max(hi[c], m.xyz[3 * v + c]);
        }
    const int nb = std::max(1, (int)std::cbrt((double)m.nt / 4.0));
    double h[3];
    for (int c = 0; c < 3; c++) h[c] = std::max(hi[c] - lo[c], 1e-300) / nb;
    std::vector<std::vector<int32_t>> bins((size_t)nb * nb * nb);
    auto bidx = [&](double x, int c) { return std::min(nb - 1, std::max(0, (int)std::floor((x - lo[c]) / h[c]))); };
    for (int64_t t = 0; t < m.nt; t++) {
        double bl[3] = {1e300, 1e300, 1e300}, bh[3] = {-1e300, -1e300, -1e300};
        for (int k = 0; k < 4; k++)
            for (int c = 0; c < 3; c++) {
                bl[c] = std::min(bl[c], m.xyz[3 * m.tets[4 * t + k] + c]);
                bh[c] = std::max(bh[c], m.xyz[3 * m.tets[4 * t + k] + c]);
            }
        int i0[3], i1[3];
        for (int c = 0; c < 3; c++) {
            i0[c] = bidx(bl[c], c);
            i1[c] = bidx(bh[c], c);
        }
        for (int a = i0[0]; a <= i1[0]; a++)
            for (int b = i0[1]; b <= i1[1]; b++)
                for (int c = i0[2]; c <= i1[2]; c++) bins[a + (size_t)nb * (b + (size_t)nb * c)].push_back((int32_t)t);
    }
    for (int64_t p = 0; p < n; p++) {
        const double *r = &pos[3 * p];
        for (int c = 0; c < 3; c++)
            if (!(r[c] >= lo[c] - 1e-12 && r[c] <= hi[c] + 1e-12))
                throw Error(FEMPIC_EOUTSIDE, "a particle lies outside the mesh");
        const auto &cand = bins[bidx(r[0], 0) + (size_t)nb * (bidx(r[1], 1) + (size_t)nb * bidx(r[2], 2))];
        double best = -1e300;
        int32_t bt = -1;
        for (int32_t t : cand) {
            const double *g = &m.geo[16 * (size_t)t];
            double mn = 1e300;
            for (int f = 0; f < 4; f++) mn = std::min(mn, g[4 * f] + g[4 * f + 1] * r[0] + g[4 * f + 2] * r[1] + g[4 * f + 3] * r[2]);
            if (mn > best || (mn == best && t < bt)) {
                best = mn;
                bt = t;
            }
        }
        if (bt < 0 || !(best >= -1e-10)) throw Error(FEMPIC_EOUTSIDE, "a particle lies outside the mesh");
        out[p] = bt;
    }
}

// nodal charge into dst (interior W0 DoFs), through per-tet partials in Pr (default: the run's)
void Run::compute_rho(double *dst, double *Pr)
{
    if (!Pr) Pr = (double *)d_Pr.p;
    const uint32_t *perm = sort_current();
    HIPCHECK(launch_rho_tet(order, dm, perm, (const int32_t *)d_off.p, pb[cur].d, q * w, Pr,
                            stream));
    HIPCHECK(launch_scatter((const int64_t *)d_inc0_ptr.p, (const int32_t *)d_inc0_idx.p, m.N0_int,
                            (const double *)Pr, dst, stream));
}

int Run::tpw() const
{
    const int tmax = order == 1 ? PARTICLE_TPW_MAX_1 : PARTICLE_TPW_MAX_2;
    const double ppt = m.nt ? (double)np / m.nt : 1.0;
    int t = (int)std::lround((double)PARTICLE_TARGET / std::max(ppt, 1e-9));
    return std::max(1, std::min(tmax, t));
}

void Run::particle_phase()
{
    Range rg("fempic particle phase (a1-a6)");
    AccountScope charge(&acct);  // the spill pool may grow
    HIPCHECK(hipEventRecord(ev_a, stream));
    const uint32_t *perm = sort_current();
    StepParams sp{q / mass, q * w, prm.dt, tpw(), prm.particle_bc == FEMPIC_ABSORB ? 1 : 0,
                  prm.pusher == FEMPIC_PUSH_BORIS ? 1 : 0};
    // The queue and spill stages run on counts that stay on the device: their
    // launches are sized by bounds from the previous step's counts (the largest
    // possible before the first), and the host reads the counts once, at the end
    // of the phase.  A step whose counts exceed the bounds, or that overflows
    // the spill pool, is redone: its input state is untouched until the commit.
    // With graphs the bounds are rounded up to at most 4 values per octave, so
    // that steps with similar counts replay the same graph.
    auto quant = [](int64_t x) {
        int e = 0;
        while ((int64_t)4 << e < x) e++;
        const int64_t q = std::max<int64_t>((int64_t)1 << e, 1024);
        return (x + q - 1) / q * q;
    };
    const bool graph = phase_graphs && use_graphs && counts_known;
    auto grow = [&](int64_t x) { return graph ? quant(x + x / 4 + 4096) : x + x / 4 + 4096; };
    int64_t nq_ub = counts_known ? std::min<int64_t>(np, grow(nq_last)) : np;
    int64_t nslot_ub = counts_known ? std::min<int64_t>(pool_cap, grow(nslot_last)) : pool_cap;
    int64_t nrec_ub = counts_known ? std::min<int64_t>(pool_cap, grow(nrec_last)) : pool_cap;
    const int64_t nq_hint = counts_known ? (graph ? quant(nq_last) : nq_last) : np / 8;
    next_perm = cur_perm == psort.val[0] ? psort.val[1] : psort.val[0];
    const int32_t *d_nq = p_small + 6, *d_nrec = p_small + 2;
    for (int attempt = 0;; attempt++) {
        if (attempt == 6) throw Error(FEMPIC_ENOMEM, "spill pool kept overflowing");
        // (k_particle clears the counters, the spill pool's append count and the order error flag)
        ParticleArgs *ha = (ParticleArgs *)((char *)h_pin + 128);
        ha->m = dm;
        ha->e = mixed ? (const void *)d_e32.p : (const void *)d_e.p;
        ha->b = gather_b();
        ha->perm = perm;
        ha->off = (const int32_t *)d_off.p;
        ha->in = pb[cur].d;
        ha->out = pb[1 - cur].d;
        ha->np = np;
        ha->sp = sp;
        ha->gl = gl;
        ha->P = (double *)d_P.p;
        ha->pool = pool();
        ha->cq = ContQueue{(ContRec *)d_cq.p, (uint8_t *)d_qflag.p, (int32_t *)d_qidx.p, p_small + 6,
                           (uint8_t *)d_moved.p, (int32_t *)d_nstay.p};
        ha->cnt = p_cnt;
        ha->perr = p_perr;
        ha->cntb = (unsigned long long *)d_cntb.p;
        HIPCHECK(hipMemcpyAsync(d_args.p, ha, sizeof(ParticleArgs), hipMemcpyHostToDevice, stream));
        // the phase's launches; timed: with events between the particle kernels
        auto launches = [&](bool timed) {
            if (timed) HIPCHECK(hipEventRecord(ev_b, stream));
            HIPCHECK(launch_particle(order, mixed, sp.boris != 0, (const ParticleArgs *)d_args.p, (int32_t)m.nt,
                                     sp.tpw, stream));
            if (timed) HIPCHECK(hipEventRecord(ev_c1, stream));
            // compact the queue written by k_particle, then continue the queued paths
            HIPCHECK(launch_queue_index(ha->cq, np, (uint32_t *)d_qtmp.p, stream));
            HIPCHECK(launch_continue(order, mixed, sp.boris != 0, (const ParticleArgs *)d_args.p, nq_hint,
                                     (unsigned long long *)d_cntb.p, p_cnt, stream));
            if (timed) HIPCHECK(hipEventRecord(ev_c, stream));
            // deterministic reduction of the spill pool: records in canonical order
            // (queued record, then segment), sorted by tet, summed per tet
            HIPCHECK(exclusive_scan_u32((const uint32_t *)d_rcount.p, (uint32_t *)d_rpos.p, nq_ub, psort.scan_tmp,
                                        (uint32_t *)(p_small + 2), stream, d_nq));
            HIPCHECK(launch_spill_compact(pool(), nslot_ub, d_nq, (const uint32_t *)d_rpos.p, ssort.key[0],
                                          ssort.val[0], ssort.cap, stream));
            int res = 0;
            HIPCHECK(radix_sort(ssort, nrec_ub, key_bits(), false, &res, stream, nullptr, d_nrec));
            HIPCHECK(launch_offsets(ssort.key[res], nrec_ub, (int32_t)m.nt, (int32_t *)d_soff.p, stream, d_nrec));
            const uint32_t *srec = ssort.val[res];
            HIPCHECK(launch_spill_reduce(n1l, (int32_t)m.nt, (const int32_t *)d_soff.p, srec,
                                         (const double *)d_pool_val.p, pool_cap, (double *)d_P.p,
                                         (const int32_t *)d_nstay.p, (uint32_t *)d_tcnt.p, stream));
            HIPCHECK(launch_scatter((const int64_t *)d_inc_ptr.p, (const int32_t *)d_inc_idx.p, n1s,
                                    (const double *)d_P.p, (double *)d_dg.p, stream));
            next_order(nrec_ub, srec);
        };
        phase_timed = !(graph && attempt == 0);
        if (phase_timed) {
            launches(true);
        } else {
            // kernels only; their launch parameters are all in the key
            const std::vector<int64_t> key{cur, (int64_t)(uintptr_t)cur_perm, (int64_t)(uintptr_t)next_perm,
                                           (int64_t)(uintptr_t)d_off.p, (int64_t)(uintptr_t)d_noff.p, nq_ub, nslot_ub,
                                           nrec_ub, nq_hint, np, sp.tpw, pool_cap};
            auto it = phase_graph.find(key);
            if (it == phase_graph.end()) {
                // keep few: a new set of bounds usually retires the older ones
                if (phase_graph.size() >= 8) clear_phase_graphs();
                std::lock_guard<std::mutex> lk(device_mu());  // (see device_mu)
                hipGraph_t g = nullptr;
                HIPCHECK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
                try {
                    launches(false);
                } catch (...) {
                    (void)hipStreamEndCapture(stream, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                HIPCHECK(hipStreamEndCapture(stream, &g));
                hipGraphExec_t gx = nullptr;
                const hipError_t e = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess)
                    throw Error(FEMPIC_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
                it = phase_graph.emplace(key, gx).first;
            }
            HIPCHECK(hipGraphLaunch(it->second, stream));
        }
        HIPCHECK(hipEventRecord(ev_d, stream));
        HIPCHECK(hipMemcpyAsync(h_pin, d_ctl.p, CTL_BYTES, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        const unsigned long long *c = (const unsigned long long *)h_pin;
        const int32_t *sm = (const int32_t *)((char *)h_pin + CTL_SMALL);
        const int64_t nq = sm[6];
        // spill slots in use: the fixed pair of every queued record, then the appended ones
        const int64_t nslots = 2 * nq + sm[0];
        const int64_t nrec = (uint32_t)sm[2];
        const unsigned long long errs = c[CNT_ERR];
        // a path over the crossing cap fails the step whatever else happened
        if (errs & ERR_CROSS) throw Error(FEMPIC_ECROSS, "a particle crossed more than 64 faces in one step");
        if (errs & ERR_POOL) {
            // grow the pool and redo the step
            alloc_pool(std::max<int64_t>(2 * pool_cap, nslots + nslots / 4 + 1024));
            nq_ub = std::max<int64_t>(nq_ub, nq);
            nslot_ub = std::min<int64_t>(pool_cap, nslots);
            nrec_ub = std::min<int64_t>(pool_cap, nrec);
            continue;
        }
        if (errs & ERR_NAN) throw Error(FEMPIC_EDEVICE, "non-finite particle position");
        if (nq > nq_ub || nslots > nslot_ub || nrec > nrec_ub) {
            nq_ub = nq;
            nslot_ub = nslots;
            nrec_ub = nrec;
            continue;
        }
        if (*(const unsigned long long *)((char *)h_pin + CTL_PERR))
            throw Error(FEMPIC_EDEVICE, "inconsistent particle order");
        last_cross = (int64_t)c[CNT_CROSS];
        last_refl = (int64_t)c[CNT_REFL];
        last_spill = (int64_t)c[CNT_SPILL];
        last_absorb = (int64_t)c[CNT_ABSORB];
        nslot_last = nslots;
        nq_last = nq;
        nrec_last = nrec;
        counts_known = true;
        break;
    }
    commit_order();
    cur = 1 - cur;
    rows_used = np;  // the step wrote rows [0, np) (holes where particles left)
    // particles absorbed at a wall are not in the new order
    np -= last_absorb;
    absorbed_total += last_absorb;
}

// Three-level Newmark-beta (Sec. III-B, eq. (maxnmb)) for gamma, beta other than
// 1/2, 1/4: M [gamma X^{n+1} + (1-2gamma) X^n + (gamma-1) X^{n-1}] / dt
// + S [beta X^{n+1} + an X^n + am X^{n-1}] = -(0, the same time stencil of g),
// an = 1/2 - 2beta + gamma, am = 1/2 + beta - gamma, X = (b, e), M = diag(*nu, *eps),
// S = [[0, *nu K], [-K^T *nu, 0]].  b^{n+1} is eliminated through the Faraday row:
//   A d = -((1-gamma)/gamma) [*eps (e^n - e^{n-1}) + (g^n - g^{n-1})] - (g^{n+1} - g^n)
//         + (dt/gamma) K^T *nu u,
//   u = B0 b^n + B1 b^{n-1} - (dt beta/gamma) K ((an + beta) e^n + am e^{n-1}),
//   A = *eps + (beta/gamma)^2 dt^2 K^T *nu K,  e^{n+1} = e^n + d,
//   b^{n+1} = -((1-2gamma) b^n + (gamma-1) b^{n-1}) / gamma
//             - (dt/gamma) K (beta e^{n+1} + an e^n + am e^{n-1}),
// with B0 = an - beta (1-2gamma)/gamma, B1 = am - beta (gamma-1)/gamma.  Before the
// first step the history is at rest (X^{-1} = X^n, no earlier current).
void Run::field_phase_three_level()
{
    Range rg("fempic field update, three-level Newmark-beta (a7)");
    const int64_t N1i = n1s, N2 = m.N2;
    const double dt = prm.dt, gm = prm.gamma, bt = prm.beta;
    const double an = 0.5 - 2.0 * bt + gm, am = 0.5 + bt - gm;
    const double B0 = an - bt * (1.0 - 2.0 * gm) / gm, B1 = am - bt * (gm - 1.0) / gm;
    double *e = (double *)d_e.p, *b = (double *)d_b.p, *dg = (double *)d_dg.p, *g = (double *)d_g.p;
    double *ep = (double *)d_eprev.p, *bp = (double *)d_bprev.p, *dgp = (double *)d_dgprev.p;
    double *w = (double *)v_tmp.p, *u = (double *)v_u.p, *rhs = (double *)v_rhs.p, *y = (double *)d_y1.p;
    double *b2 = (double *)v_b2.p, *d = (double *)v_x.p;
    double *dp = (double *)d_dprev.p, *dp_lo = (double *)d_dprev_lo.p;
    if (!have_prev) {
        HIPCHECK(axpby(N1i, 1.0, e, 0.0, e, ep, stream));
        HIPCHECK(axpby(N2, 1.0, b, 0.0, b, bp, stream));
        HIPCHECK(axpby(N1i, 0.0, dg, 0.0, dg, dgp, stream));
        HIPCHECK(axpby(N1i, 0.0, dg, 0.0, dg, dp, stream));
        HIPCHECK(axpby(N1i, 0.0, dg, 0.0, dg, dp_lo, stream));
        have_prev = true;
    }
    HIPCHECK(add_comp(N1i, g, (double *)d_g_lo.p, dg, stream));
    // u = B0 b + B1 b^{n-1} - (dt beta / gamma) K ((an + beta) e + am e^{n-1})
    HIPCHECK(axpby(N1i, an + bt, e, am, ep, w, stream));
    HIPCHECK(axpby(N2, B0, b, B1, bp, u, stream));
    HIPCHECK(spmv(K.desc, w, u, -dt * bt / gm, 1.0, u, stream));
    // rhs = (dt/gamma) K^T (*nu u) - ((1-gamma)/gamma) (*eps (e - e^{n-1}) + dg^{n-1}) - dg in
    // double-double, with e - e^{n-1} the previous increment kept as hi + lo
    HIPCHECK(spmv(Mnu.desc, u, (double *)v_nu.p, 1.0, 0.0, nullptr, stream));
    const double cprev = -(1.0 - gm) / gm;
    HIPCHECK(combo_dd(N1i, &Kt.desc, (const double *)v_nu.p, dt / gm, &Meps.desc, dp, dp_lo, cprev, dgp, cprev, dg,
                      -1.0, rhs, (double *)v_rhs_lo.p, stream));
    (void)y;
    if (mixed) solve_mixed();
    else solve_fp64();
    // b^{n+1} = -((1-2gamma) b + (gamma-1) b^{n-1}) / gamma - (dt/gamma) K ((beta + an) e + beta d + am e^{n-1})
    HIPCHECK(axpby(N1i, bt + an, e, bt, d, w, stream));
    HIPCHECK(axpby(N1i, 1.0, w, am, ep, w, stream));
    HIPCHECK(axpby(N2, -(1.0 - 2.0 * gm) / gm, b, -(gm - 1.0) / gm, bp, b2, stream));
    HIPCHECK(spmv(K.desc, w, b2, -dt / gm, 1.0, b2, stream));
    // shift the history, then the new fields
    HIPCHECK(axpby(N2, 1.0, b, 0.0, b, bp, stream));
    HIPCHECK(axpby(N2, 1.0, b2, 0.0, b2, b, stream));
    HIPCHECK(axpby(N1i, 1.0, e, 0.0, e, ep, stream));
    HIPCHECK(add_comp(N1i, e, (double *)d_e_lo.p, d, stream));
    HIPCHECK(axpby(N1i, 1.0, (const double *)d_e_lo.p, 1.0, (const double *)v_x_lo.p, (double *)d_e_lo.p, stream));
    HIPCHECK(axpby(N1i, 1.0, dg, 0.0, dg, dgp, stream));
    HIPCHECK(axpby(N1i, 1.0, d, 0.0, d, dp, stream));
    HIPCHECK(axpby(N1i, 1.0, (const double *)v_x_lo.p, 0.0, (const double *)v_x_lo.p, dp_lo, stream));
    if (mixed) HIPCHECK(cast_d2f(m.N1, e, (float *)d_e32.p, 1.0, stream));
    refresh_gather_b();
    HIPCHECK(hipEventRecord(ev_e, stream));
}

void Run::field_phase()
{
    if (three_level) return field_phase_three_level();
    Range rg("fempic field update (a7)");
    const int64_t N1i = n1s, N2 = m.N2;
    const double dt = prm.dt;
    double *e = (double *)d_e.p, *b = (double *)d_b.p, *dg = (double *)d_dg.p;
    // g += dg (compensated: d_g_lo keeps the rounding errors for the Gauss check)
    HIPCHECK(add_comp(N1i, (double *)d_g.p, (double *)d_g_lo.p, dg, stream));
    // u = b - dt/2 K e ; rhs = dt K^T (*nu u) - dg, the last step in double-double
    // (whatever *nu u rounds to, G^T K^T of it is zero)
    HIPCHECK(spmv(K.desc, e, (double *)v_u.p, -0.5 * dt, 1.0, b, stream));
    HIPCHECK(spmv(Mnu.desc, (const double *)v_u.p, (double *)v_nu.p, 1.0, 0.0, nullptr, stream));
    // (absorbing walls: - dt *I e as well, e = e + e_lo)
    HIPCHECK(combo_dd(N1i, &Kt.desc, (const double *)v_nu.p, dt, absorbing ? &Zi.desc : nullptr,
                      absorbing ? e : nullptr, absorbing ? (const double *)d_e_lo.p : nullptr, absorbing ? -dt : 0.0,
                      dg, -1.0, nullptr, 0.0, (double *)v_rhs.p, (double *)v_rhs_lo.p, stream));
    // solve A d = rhs (d = v_x + v_x_lo)
    if (mixed) solve_mixed();
    else solve_fp64();
    // b -= dt/2 K (2 e + d) ; e += d (compensated)
    HIPCHECK(axpby(N1i, 2.0, e, 1.0, (const double *)v_x.p, (double *)v_tmp.p, stream));
    HIPCHECK(spmv(K.desc, (const double *)v_tmp.p, b, -0.5 * dt, 1.0, b, stream));
    HIPCHECK(add_comp(N1i, e, (double *)d_e_lo.p, (const double *)v_x.p, stream));
    HIPCHECK(axpby(N1i, 1.0, (const double *)d_e_lo.p, 1.0, (const double *)v_x_lo.p, (double *)d_e_lo.p, stream));
    (void)N2;
    if (mixed) HIPCHECK(cast_d2f(m.N1, e, (float *)d_e32.p, 1.0, stream));
    refresh_gather_b();
    HIPCHECK(hipEventRecord(ev_e, stream));
}

double Run::read_sc(int k)
{
    HIPCHECK(hipMemcpyAsync(h_pin, (double *)d_sc.p + k, 8, hipMemcpyDeviceToHost, stream));
    HIPCHECK(hipStreamSynchronize(stream));
    return *(double *)h_pin;
}

// Eight PCG iterations: FP64 on v_*, or the FP32 inner solve on f_*.  The
// kernels and their arguments are the same for every batch (the iteration
// parity alternates 0, 1 within it), so the batch is captured once per run as a
// HIP graph and replayed; it holds kernels only.
void Run::pcg_batch(bool fp32)
{
    const int64_t n = n1s;
    double *sc = (double *)d_sc.p, *part = (double *)d_partial.p;
    auto launch = [&]() {
        for (int k = 0; k < 8; k++) {
            if (fp32)
                HIPCHECK(pcg32_iter(A.desc, &mf, n, (float *)f_x.p, (float *)f_r.p, (float *)f_z.p, (float *)f_p.p,
                                    (float *)f_q.p, (const float *)d_dinv32.p, part, sc, k & 1, stream));
            else
                HIPCHECK(pcg_iter(A.desc, &mf, n, (double *)v_x.p, (double *)v_r.p, (double *)v_z.p, (double *)v_p.p,
                                  (double *)v_q.p, (const double *)d_dinv.p, part, sc, k & 1, stream));
        }
    };
    if (!use_graphs) return launch();
    hipGraphExec_t &gx = pcg_graph[fp32 ? 1 : 0];
    if (!gx) {
        std::lock_guard<std::mutex> g(device_mu());  // (see device_mu)
        hipGraph_t graph = nullptr;
        HIPCHECK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        try {
            launch();
        } catch (...) {
            (void)hipStreamEndCapture(stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        HIPCHECK(hipStreamEndCapture(stream, &graph));
        const hipError_t e = hipGraphInstantiate(&gx, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            gx = nullptr;
            throw Error(FEMPIC_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
    }
    HIPCHECK(hipGraphLaunch(gx, stream));
}

// PCG (FP64) on A x = b from x = 0 until |r|^2 <= tol2 (or at the attainable
// accuracy); returns |r|^2 of the recurrence.  The iterate is v_x.
double Run::pcg64(const double *b, double tol2, double bb)
{
    const int64_t n = n1s;
    double *sc = (double *)d_sc.p, *part = (double *)d_partial.p;
    HIPCHECK(pcg_init(n, b, (double *)v_x.p, (double *)v_r.p, (double *)v_z.p, (double *)v_p.p,
                      (const double *)d_dinv.p, part, sc, A.desc.bptr != nullptr, stream));
    double rr = read_sc(SC_BB), best = rr;
    if (rr == 0.0) return 0.0;
    int stall = 0, it = 0;
    while (it < prm.pcg_maxit) {
        if (it + 8 <= prm.pcg_maxit) {
            pcg_batch(false);
            it += 8;
        } else {
            for (; it < prm.pcg_maxit; it++)
                HIPCHECK(pcg_iter(A.desc, &mf, n, (double *)v_x.p, (double *)v_r.p, (double *)v_z.p, (double *)v_p.p,
                                  (double *)v_q.p, (const double *)d_dinv.p, part, sc, it & 1, stream));
        }
        rr = read_sc(SC_RR);
        if (!(rr == rr)) throw Error(FEMPIC_ESOLVE, "field solve produced NaN");
        if (rr <= tol2) break;
        if (rr < 0.25 * best) {
            best = rr;
            stall = 0;
        } else if (++stall > 40 && rr <= 1e-24 * bb) {
            break;  // at the attainable accuracy
        }
    }
    last_iters += it;
    if (!(rr <= tol2) && !(rr <= 1e-24 * bb))
        throw Error(FEMPIC_ESOLVE, "PCG did not reach the tolerance: relres " + std::to_string(std::sqrt(rr / bb)));
    return rr;
}

// The residual of the refinement, r = (rhs + rhs_lo) - A (x + x_lo), in
// double-double, rounded into r; returns |r|^2.
double Run::residual_dd(const double *x, const double *x_lo, double *r)
{
    const int64_t n = n1s;
    HIPCHECK(combo_dd(n, nullptr, nullptr, 0.0, &A.desc, x, x_lo, -1.0, (const double *)v_rhs.p, 1.0,
                      (const double *)v_rhs_lo.p, 1.0, r, nullptr, stream));
    HIPCHECK(dot_det(n, r, r, (double *)d_partial.p, (double *)d_sc.p + 12, stream));
    return read_sc(12);
}

// Both solvers leave the solution as v_x + v_x_lo.  The right-hand side is
// v_rhs + v_rhs_lo (double-double), and the solve is refined against it with
// residuals in double-double down to gauss_rtol (below pcg_rtol): the part of
// the residual that reaches G^T is what each step would otherwise add to the
// Gauss residual, and at FP64 accuracy (1e-15 relative) it adds up, step after
// step, to more than 1e-12 over a thousand steps.
double Run::solve_target() const { return std::min(prm.pcg_rtol, GAUSS_RTOL); }

void Run::solve_fp64()
{
    Range rg("fempic pcg");
    const int64_t n = n1s;
    const double *rhs = (const double *)v_rhs.p;
    double *x = (double *)v_x.p, *xs = (double *)v_xs.p, *xlo = (double *)v_x_lo.p, *rc = (double *)v_tmp.p;
    HIPCHECK(dot_det(n, rhs, rhs, (double *)d_partial.p, (double *)d_sc.p + 12, stream));
    const double bb = read_sc(12);
    last_iters = 0;
    last_relres = 0;
    HIPCHECK(axpby(n, 0.0, rhs, 0.0, rhs, xlo, stream));
    if (bb == 0.0) {
        HIPCHECK(axpby(n, 0.0, rhs, 0.0, rhs, x, stream));
        return;
    }
    const double tgt2 = solve_target() * solve_target() * bb;
    pcg64(rhs, prm.pcg_rtol * prm.pcg_rtol * bb, bb);
    HIPCHECK(axpby(n, 1.0, x, 0.0, x, xs, stream));
    double rr = residual_dd(xs, xlo, rc);
    for (int cyc = 0; cyc < 4 && rr > tgt2; cyc++) {
        // correction A c = r to the reduction the target still needs (margin 4)
        const double red = std::max(1e-10, std::min(1e-1, 0.25 * std::sqrt(tgt2 / rr)));
        pcg64(rc, red * red * rr, rr);
        HIPCHECK(add_comp(n, xs, xlo, x, stream));
        rr = residual_dd(xs, xlo, rc);
    }
    HIPCHECK(axpby(n, 1.0, xs, 0.0, xs, x, stream));
    last_relres = std::sqrt(rr / bb);
    if (!(last_relres <= prm.pcg_rtol))
        throw Error(FEMPIC_ESOLVE, "PCG did not reach the tolerance: relres " + std::to_string(last_relres));
}

// FP32 PCG inside FP64 iterative refinement: x = 0, r = rhs; repeat: an inner
// FP32 solve of A c = r / |r|, x += |r| c (compensated into x + x_lo), r = the
// double-double residual, until |r| <= target |rhs|.
void Run::solve_mixed()
{
    Range rg("fempic pcg (FP32 inner, FP64 refinement)");
    const int64_t n = n1s;
    double *sc = (double *)d_sc.p, *part = (double *)d_partial.p;
    double *x = (double *)v_x.p, *xlo = (double *)v_x_lo.p, *r = (double *)v_r.p;
    const double *rhs = (const double *)v_rhs.p;
    HIPCHECK(dot_det(n, rhs, rhs, part, sc + 12, stream));
    const double bb = read_sc(12);
    last_iters = 0;
    last_relres = 0;
    HIPCHECK(axpby(n, 0.0, rhs, 0.0, rhs, x, stream));
    HIPCHECK(axpby(n, 0.0, rhs, 0.0, rhs, xlo, stream));
    HIPCHECK(axpby(n, 1.0, rhs, 0.0, rhs, r, stream));
    if (bb == 0.0) return;
    const double tgt = solve_target();
    double rr = bb;
    for (int outer = 0; outer < 12; outer++) {
        if (rr <= tgt * tgt * bb) break;
        const double scale = std::sqrt(rr);
        HIPCHECK(cast_d2f(n, r, (float *)f_q.p, 1.0 / scale, stream));
        HIPCHECK(pcg32_init(n, (const float *)f_q.p, (float *)f_x.p, (float *)f_r.p, (float *)f_z.p, (float *)f_p.p,
                            (const float *)d_dinv32.p, part, sc, A.desc.bptr != nullptr, stream));
        const double bb32 = read_sc(SC_BB);
        // the inner solve reduces its residual by 1e-5 (about what FP32 holds),
        // or by less on the last cycle: just what the target still needs, with
        // a margin of 4
        const double need = 0.25 * tgt * std::sqrt(bb / rr);
        const double red = std::max(1e-5, std::min(1.0, need));
        const double tol32 = red * red * bb32;
        int it = 0;
        double r32 = bb32;
        while (it < prm.pcg_maxit) {
            pcg_batch(true);
            it += 8;
            r32 = read_sc(SC_RR);
            if (!(r32 == r32)) throw Error(FEMPIC_ESOLVE, "FP32 inner solve produced NaN");
            if (r32 <= tol32) break;
        }
        last_iters += it;
        HIPCHECK(add_f2d_comp(n, (const float *)f_x.p, scale, x, xlo, stream));
        rr = residual_dd(x, xlo, r);
    }
    last_relres = std::sqrt(rr / bb);
    if (!(last_relres <= prm.pcg_rtol) && !(last_relres < 1e-12))
        throw Error(FEMPIC_ESOLVE, "refined solve did not reach the tolerance: relres " + std::to_string(last_relres));
}

void Run::step(int n_steps)
{
    if (!loaded) throw Error(FEMPIC_EINVAL, "no particles loaded");
    if (sticky) throw Error(sticky, sticky_msg);
    double pms = 0, kms = 0, cms = 0, fms = 0;
    int64_t replays = 0;
    try {
        for (int s = 0; s < n_steps; s++) {
            Range rg("fempic step");
            particle_phase();
            field_phase();
            HIPCHECK(hipEventSynchronize(ev_e));
            float t1 = 0, t2 = 0, t3 = 0, t4 = 0;
            HIPCHECK(hipEventElapsedTime(&t1, ev_a, ev_d));
            if (phase_timed) {  // (a replayed phase graph has no events between its kernels)
                HIPCHECK(hipEventElapsedTime(&t2, ev_b, ev_c1));
                HIPCHECK(hipEventElapsedTime(&t4, ev_c1, ev_c));
            } else {
                replays++;
            }
            HIPCHECK(hipEventElapsedTime(&t3, ev_d, ev_e));
            pms += t1;
            kms += t2;
            cms += t4;
            fms += t3;
            steps_done++;
            if (prm.gauss_every > 0 && steps_done % prm.gauss_every == 0) {
                gauss(gauss_last);
                gauss_step = steps_done;
            }
            if (log) log_step(t1, t2, t4, t3, gauss_step == steps_done);
        }
    } catch (Error &e) {
        sticky = e.code;
        sticky_msg = e.what();
        throw;
    }
    last_particle_ms = pms;
    last_phase_replays = replays;
    last_kernel_ms = kms;
    last_continue_ms = cms;
    last_field_ms = fms;
}

// the step log: one JSON object per line, appended and flushed after each step
void Run::set_log(const char *path)
{
    if (log) std::fclose(log);
    log = nullptr;
    if (path && *path) {
        log = std::fopen(path, "a");
        if (!log) throw Error(FEMPIC_EINVAL, std::string("cannot open step log ") + path);
    }
}

void Run::log_step(float particle_ms, float kernel_ms, float continue_ms, float field_ms, bool with_gauss)
{
    auto num = [](double v) {
        char b[32];
        if (std::isfinite(v)) std::snprintf(b, sizeof b, "%.17g", v);
        else std::snprintf(b, sizeof b, "null");
        return std::string(b);
    };
    std::string s = "{\"step\": " + std::to_string(steps_done) + ", \"n_particles\": " + std::to_string(np) +
                    ", \"particle_ms\": " + num(particle_ms) + ", \"particle_kernel_ms\": " + num(kernel_ms) +
                    ", \"continue_kernel_ms\": " + num(continue_ms) + ", \"field_ms\": " + num(field_ms) +
                    ", \"pcg_iters\": " + std::to_string(last_iters) + ", \"pcg_relres\": " + num(last_relres) +
                    ", \"crossings\": " + std::to_string(last_cross) + ", \"reflections\": " +
                    std::to_string(last_refl) + ", \"absorbed\": " + std::to_string(last_absorb) +
                    ", \"spills\": " + std::to_string(last_spill);
    if (with_gauss)
        s += ", \"gauss\": [" + num(gauss_last[0]) + ", " + num(gauss_last[1]) + ", " + num(gauss_last[2]) + "]";
    s += "}\n";
    if (std::fputs(s.c_str(), log) < 0 || std::fflush(log) != 0) throw Error(FEMPIC_EINVAL, "cannot write the step log");
}

void Run::gauss(double out[3])
{
    Range rg("fempic gauss residual (a8)");
    if (!loaded) throw Error(FEMPIC_EINVAL, "no particles loaded");
    gauss_with((double *)d_Pr.p, (double *)d_rho.p, (double *)d_GtDe.p, (double *)d_Gtg.p, (double *)d_y1.p,
               (double *)d_y1_lo.p, (double *)d_partial.p, (double *)d_sc.p + 16, out);
}

// The Gauss check with every intermediate in the library's static device
// scratch (kernels.hip): nothing is allocated, on the device or through the
// installed allocator.  Concurrent calls on one device share that scratch.
void Run::gauss_noalloc(double out[3])
{
    Range rg("fempic gauss residual without allocation (a8)");
    if (!loaded) throw Error(FEMPIC_EINVAL, "no particles loaded");
    int cur_dev = 0;
    HIPCHECK(hipGetDevice(&cur_dev));
    if (cur_dev != device) HIPCHECK(hipSetDevice(device));
    struct Restore {
        int dev, run_dev;
        ~Restore()
        {
            if (dev != run_dev) (void)hipSetDevice(dev);
        }
    } restore{cur_dev, device};
    void *base = nullptr;
    HIPCHECK(noalloc_scratch(&base));
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t n0 = (size_t)std::max<int64_t>(m.N0_int, 1), n1 = (size_t)std::max<int64_t>(n1s, 1);
    const size_t b_pr = al((size_t)m.nt * n0l * 8), b_v0 = al(n0 * 8), b_v1 = al(n1 * 8),
                 b_part = al((size_t)gauss_partial_entries() * 8);
    const size_t need = b_pr + 3 * b_v0 + 2 * b_v1 + b_part + 256;
    if (need > NOALLOC_SCRATCH_BYTES)
        throw Error(FEMPIC_EINVAL, "the Gauss check of this mesh needs " + std::to_string(need) +
                                       " bytes of scratch; the library's static scratch holds " +
                                       std::to_string(NOALLOC_SCRATCH_BYTES));
    char *p = (char *)base;
    double *Pr = (double *)p;
    double *rho = (double *)(p += b_pr);
    double *GtDe = (double *)(p += b_v0);
    double *Gtg = (double *)(p += b_v0);
    double *y1 = (double *)(p += b_v0);
    double *y1_lo = (double *)(p += b_v1);
    double *part = (double *)(p += b_v1);
    double *out4 = (double *)(p += b_part);
    gauss_with(Pr, rho, GtDe, Gtg, y1, y1_lo, part, out4, out);
}

// G^T *eps e and G^T g are sums of large terms that cancel down to the nodal
// charge change; they are evaluated from the compensated running sums (hi +
// lo) in double-double, so the check sees the scheme's Gauss residual, not the
// rounding of FP64 running sums and products.
void Run::gauss_with(double *Pr, double *rho, double *GtDe, double *Gtg, double *y1, double *y1_lo, double *partial,
                     double *out4, double out[3])
{
    compute_rho(rho, Pr);
    const int64_t N0i = m.N0_int;
    HIPCHECK(spmv_dd(Meps.desc, (const double *)d_e.p, (const double *)d_e_lo.p, y1, y1_lo, stream));
    HIPCHECK(spmv_dd(Gt.desc, y1, y1_lo, GtDe, nullptr, stream));
    HIPCHECK(spmv_dd(Gt.desc, (const double *)d_g.p, (const double *)d_g_lo.p, Gtg, nullptr, stream));
    HIPCHECK(gauss_norms(N0i, (const double *)GtDe, (const double *)Gtg, (const double *)rho,
                         (const double *)d_rho0.p, gscale, partial, out4, stream));
    HIPCHECK(hipMemcpyAsync(h_pin, out4, 32, hipMemcpyDeviceToHost, stream));
    sync();
    const double *v = (const double *)h_pin;
    double nrm = std::sqrt(v[3]);
    if (nrm == 0) nrm = 1.0;
    out[0] = std::sqrt(v[0]) / nrm;
    out[1] = std::sqrt(v[1]) / nrm;
    out[2] = std::sqrt(v[2]) / nrm;
}

void Run::fields_get(double *e, int64_t ne, double *b, int64_t nb)
{
    sync();
    if (e) {
        if (ne < m.N1) throw Error(FEMPIC_EINVAL, "e buffer too short");
        std::vector<double> ei(m.N1);
        HIPCHECK(hipMemcpy(ei.data(), d_e.p, m.N1 * 8, hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < m.N1; k++) e[m.int2nat1[k]] = ei[k];
    }
    if (b) {
        if (nb < m.N2) throw Error(FEMPIC_EINVAL, "b buffer too short");
        HIPCHECK(hipMemcpy(b, d_b.p, m.N2 * 8, hipMemcpyDeviceToHost));
    }
}

void Run::fields_set(const double *e, int64_t ne, const double *b, int64_t nb)
{
    sync();
    have_prev = false;  // new fields: the three-level scheme's history starts at rest
    if (e && ne >= m.N1)
        for (int64_t i = 0; i < m.N1; i++)
            if (!std::isfinite(e[i])) throw Error(FEMPIC_EINVAL, "non-finite e coefficient");
    if (b && nb >= m.N2)
        for (int64_t i = 0; i < m.N2; i++)
            if (!std::isfinite(b[i])) throw Error(FEMPIC_EINVAL, "non-finite b coefficient");
    if (e) {
        if (ne < m.N1) throw Error(FEMPIC_EINVAL, "e buffer too short");
        std::vector<double> ei(m.N1, 0.0);
        for (int64_t i = 0; i < m.N1; i++) {
            int64_t k = m.nat2int1[i];
            if (k < n1s) ei[k] = e[i];
        }
        HIPCHECK(hipMemcpy(d_e.p, ei.data(), m.N1 * 8, hipMemcpyHostToDevice));
        zero(d_e_lo);
        HIPCHECK(hipStreamSynchronize(stream));
    }
    if (b) {
        if (nb < m.N2) throw Error(FEMPIC_EINVAL, "b buffer too short");
        HIPCHECK(hipMemcpy(d_b.p, b, m.N2 * 8, hipMemcpyHostToDevice));
    }
    if (mixed) HIPCHECK(cast_d2f(m.N1, (const double *)d_e.p, (float *)d_e32.p, 1.0, stream));
    refresh_gather_b();
    HIPCHECK(hipStreamSynchronize(stream));
}

void Run::deposit_get(double *dg, int64_t n)
{
    sync();
    if (n < m.N1) throw Error(FEMPIC_EINVAL, "buffer too short");
    std::vector<double> d(std::max<int64_t>(n1s, 1));
    HIPCHECK(hipMemcpy(d.data(), d_dg.p, n1s * 8, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m.N1; i++) dg[i] = 0.0;
    for (int64_t k = 0; k < n1s; k++) dg[m.int2nat1[k]] = d[k];
}

void Run::field_matvec(const double *x, double *y, int64_t n, int form)
{
    sync();
    if (n < m.N1) throw Error(FEMPIC_EINVAL, "buffer too short");
    if (form != FEMPIC_OP_ASSEMBLED && form != FEMPIC_OP_ITERATION) throw Error(FEMPIC_EINVAL, "unknown operator form");
    std::vector<double> xi(std::max<int64_t>(n1s, 1), 0.0);
    for (int64_t i = 0; i < m.N1; i++) {
        if (!std::isfinite(x[i])) throw Error(FEMPIC_EINVAL, "non-finite x");
        const int64_t k = m.nat2int1[i];
        if (k < n1s) xi[k] = x[i];
    }
    // the solver's search-direction vectors hold nothing between steps
    std::vector<double> yi(xi.size(), 0.0);
    if (form == FEMPIC_OP_ITERATION && mixed) {
        std::vector<float> xf(xi.begin(), xi.end()), yf(xi.size());
        HIPCHECK(hipMemcpyAsync(f_p.p, xf.data(), n1s * 4, hipMemcpyHostToDevice, stream));
        if (mf.order) HIPCHECK(mf_apply32(mf, (const float *)f_p.p, (float *)f_q.p, stream));
        else HIPCHECK(spmv32(A.desc, (const float *)f_p.p, (float *)f_q.p, stream));
        HIPCHECK(hipMemcpyAsync(yf.data(), f_q.p, n1s * 4, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        for (int64_t k = 0; k < n1s; k++) yi[k] = yf[k];
    } else {
        HIPCHECK(hipMemcpyAsync(v_p.p, xi.data(), n1s * 8, hipMemcpyHostToDevice, stream));
        if (form == FEMPIC_OP_ITERATION && mf.order) HIPCHECK(mf_apply(mf, (const double *)v_p.p, (double *)v_q.p, stream));
        else HIPCHECK(spmv(A.desc, (const double *)v_p.p, (double *)v_q.p, 1.0, 0.0, nullptr, stream));
        HIPCHECK(hipMemcpyAsync(yi.data(), v_q.p, n1s * 8, hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
    }
    for (int64_t i = 0; i < m.N1; i++) y[i] = 0.0;
    for (int64_t k = 0; k < n1s; k++) y[m.int2nat1[k]] = yi[k];
}

// ------------------------------------------------------- impressed field
const void *Run::gather_b() const
{
    if (mixed) return d_b32.p;
    return has_imp ? d_bg.p : d_b.p;
}

void Run::refresh_gather_b()
{
    const double *b = (const double *)d_b.p;
    if (has_imp) {
        if (!d_bimp.p || !d_bg.p) throw Error(FEMPIC_EINVAL, "impressed field without its buffers");
        HIPCHECK(axpby(m.N2, 1.0, b, 1.0, (const double *)d_bimp.p, (double *)d_bg.p, stream));
        b = (const double *)d_bg.p;
    }
    if (mixed) HIPCHECK(cast_d2f(m.N2, b, (float *)d_b32.p, 1.0, stream));
}

double Run::cg_general(int64_t n, const std::function<void(const double *, double *)> &apply, const double *dinv,
                       const double *b, double *x, double rtol, int maxit)
{
    DevBuf r, z, p, q;
    for (DevBuf *v : {&r, &z, &p, &q}) v->alloc(std::max<int64_t>(n, 1) * 8);
    double *part = (double *)d_partial.p, *sc = (double *)d_sc.p;
    auto dot = [&](const double *a, const double *c) {
        HIPCHECK(dot_det(n, a, c, part, sc + 12, stream));
        return read_sc(12);
    };
    HIPCHECK(axpby(n, 0.0, b, 0.0, b, x, stream));
    HIPCHECK(axpby(n, 1.0, b, 0.0, b, (double *)r.p, stream));
    const double bb = dot(b, b);
    if (bb == 0.0) return 0.0;
    HIPCHECK(mul(n, dinv, (const double *)r.p, (double *)z.p, stream));
    HIPCHECK(axpby(n, 1.0, (const double *)z.p, 0.0, (const double *)z.p, (double *)p.p, stream));
    double rz = dot((const double *)r.p, (const double *)z.p), rr = bb;
    for (int it = 0; it < maxit && rr > rtol * rtol * bb; it++) {
        apply((const double *)p.p, (double *)q.p);
        const double pq = dot((const double *)p.p, (const double *)q.p);
        if (!(pq > 0.0)) break;  // the iterate has left the operator's range: at its accuracy
        const double al = rz / pq;
        HIPCHECK(axpby(n, 1.0, x, al, (const double *)p.p, x, stream));
        HIPCHECK(axpby(n, 1.0, (const double *)r.p, -al, (const double *)q.p, (double *)r.p, stream));
        HIPCHECK(mul(n, dinv, (const double *)r.p, (double *)z.p, stream));
        const double rz2 = dot((const double *)r.p, (const double *)z.p);
        rr = dot((const double *)r.p, (const double *)r.p);
        HIPCHECK(axpby(n, 1.0, (const double *)z.p, rz2 / rz, (const double *)p.p, (double *)p.p, stream));
        rz = rz2;
    }
    return std::sqrt(rr / bb);
}

// Projection of an impressed B onto the face space (Sec. III-C).  The moments
// f_l = <W2_l, B / mu0> come from B at the n1d^3 collapsed Gauss points of each
// tet.  Without the constraint, *nu b = f.  With it (eq. (conB)), b is the
// *nu-orthogonal projection onto the faces whose discrete divergence vanishes;
// on a simply connected box these are exactly the curls of edge fields, b = K a
// over every W1 DoF (walls included), so a solves K^T *nu K a = K^T f (CG on a
// semi-definite system with a consistent right-hand side) and b = K a is
// divergence-free by construction, as the saddle-point system's b is.
void Run::impressed_set(const double *B, int64_t n, int n1d, bool constrained, double *b_out, int64_t nb)
{
    sync();
    AccountScope charge(&acct);
    if (n1d < 1 || n1d > 8) throw Error(FEMPIC_EINVAL, "the rule takes 1 to 8 points per direction");
    const int P = n1d * n1d * n1d;
    if (!B || n < (int64_t)m.nt * P) throw Error(FEMPIC_EINVAL, "B must hold n_tet * n1d^3 points");
    if (b_out && nb < m.N2) throw Error(FEMPIC_EINVAL, "b buffer too short");
    for (int64_t k = 0; k < 3 * (int64_t)m.nt * P; k++)
        if (!std::isfinite(B[k])) throw Error(FEMPIC_EINVAL, "non-finite impressed B");
    const int64_t N2 = m.N2, N1 = m.N1, n2l = m.order == 2 ? 15 : 4;
    std::vector<double> lam, wq;
    impressed_rule(n1d, lam, wq);
    ImpressedOps io;
    assemble_impressed(m, io);
    DevBuf d_lam, d_w, d_B, d_Pf, d_ip, d_ii, d_f;
    upload(d_lam, lam, stream);
    upload(d_w, wq, stream);
    d_B.alloc((size_t)m.nt * P * 3 * 8);
    HIPCHECK(hipMemcpyAsync(d_B.p, B, (size_t)m.nt * P * 3 * 8, hipMemcpyHostToDevice, stream));
    d_Pf.alloc((size_t)m.nt * n2l * 8);
    upload(d_ip, io.inc2_ptr, stream);
    upload(d_ii, io.inc2_idx, stream);
    d_f.alloc(std::max<int64_t>(N2, 1) * 8);
    HIPCHECK(launch_impressed_rhs(m.order, dm, P, (const double *)d_lam.p, (const double *)d_w.p,
                                  (const double *)d_B.p, 1.0 / MU0, (double *)d_Pf.p, stream));
    HIPCHECK(launch_scatter((const int64_t *)d_ip.p, (const int32_t *)d_ii.p, N2, (const double *)d_Pf.p,
                            (double *)d_f.p, stream));
    HIPCHECK(hipStreamSynchronize(stream));
    d_B.release();
    d_Pf.release();
    if (!d_bimp.p) d_bimp.alloc(std::max<int64_t>(N2, 1) * 8);
    double *bi = (double *)d_bimp.p;
    DevBuf dnu;
    dnu.alloc(std::max<int64_t>(N2, 1) * 8);
    HIPCHECK(jacobi(Mnu.desc, nullptr, (double *)dnu.p, stream));
    const int maxit = std::max(prm.pcg_maxit, 1000);
    if (!constrained) {
        auto apply = [&](const double *x, double *y) { HIPCHECK(spmv(Mnu.desc, x, y, 1.0, 0.0, nullptr, stream)); };
        const double rel = cg_general(N2, apply, (const double *)dnu.p, (const double *)d_f.p, bi, 1e-14, maxit);
        if (!(rel <= 1e-12)) throw Error(FEMPIC_ESOLVE, "impressed-field projection: relres " + std::to_string(rel));
    } else {
        DevCSRBuf Ka, Kta;
        upload_csr(Ka, io.K, false);
        upload_csr(Kta, io.Kt, false);
        DevBuf rhs, a, dk, t2;
        for (DevBuf *v : {&rhs, &a, &dk}) v->alloc(std::max<int64_t>(N1, 1) * 8);
        t2.alloc(std::max<int64_t>(N2, 1) * 8);
        // K^T f, then K^T *nu K a = K^T f, Jacobi from the diagonal of K^T diag(*nu) K
        HIPCHECK(spmv(Kta.desc, (const double *)d_f.p, (double *)rhs.p, 1.0, 0.0, nullptr, stream));
        HIPCHECK(jacobi(Kta.desc, (const double *)dnu.p, (double *)dk.p, stream));
        auto apply = [&](const double *x, double *y) {
            HIPCHECK(spmv(Ka.desc, x, (double *)t2.p, 1.0, 0.0, nullptr, stream));
            HIPCHECK(spmv(Mnu.desc, (const double *)t2.p, bi, 1.0, 0.0, nullptr, stream));
            HIPCHECK(spmv(Kta.desc, bi, y, 1.0, 0.0, nullptr, stream));
        };
        const double rel = cg_general(N1, apply, (const double *)dk.p, (const double *)rhs.p, (double *)a.p, 1e-12,
                                      20 * maxit);
        if (!(rel <= 1e-8)) throw Error(FEMPIC_ESOLVE, "constrained impressed-field projection: relres " +
                                                           std::to_string(rel));
        HIPCHECK(spmv(Ka.desc, (const double *)a.p, bi, 1.0, 0.0, nullptr, stream));
    }
    if (!d_bg.p) d_bg.alloc(std::max<int64_t>(N2, 1) * 8);
    has_imp = true;
    refresh_gather_b();
    if (b_out) HIPCHECK(hipMemcpyAsync(b_out, bi, N2 * 8, hipMemcpyDeviceToHost, stream));
    HIPCHECK(hipStreamSynchronize(stream));
}

void Run::rho_get(double *rho, double *rho0, int64_t n)
{
    if (!loaded) throw Error(FEMPIC_EINVAL, "no particles loaded");
    sync();
    if (n < m.N0) throw Error(FEMPIC_EINVAL, "buffer too short");
    std::vector<double> d(std::max<int64_t>(m.N0_int, 1));
    auto out = [&](const void *src, double *dst) {
        if (!dst) return;
        if (m.N0_int) HIPCHECK(hipMemcpy(d.data(), src, m.N0_int * 8, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < m.N0; i++) dst[i] = 0.0;
        for (int64_t k = 0; k < m.N0_int; k++) dst[m.int2nat0[k]] = d[k];
    };
    if (rho) {
        compute_rho((double *)d_rho.p);
        HIPCHECK(hipStreamSynchronize(stream));
        out(d_rho.p, rho);
    }
    out(d_rho0.p, rho0);
}

// the current particles, gathered in the order the next step takes them into
// the buffer set that step writes (it overwrites them), and returned as that
// buffer set: rows [0, np) hold every particle still in the run
const PBufs &Run::gather_current()
{
    const uint32_t *perm = sort_current();
    HIPCHECK(launch_permute(mixed, pb[cur].d, pb[1 - cur].d, perm, np, stream));
    HIPCHECK(hipStreamSynchronize(stream));
    return pb[1 - cur];
}

void Run::particles_get(double *pos, double *vel, int64_t *tet, int64_t n)
{
    sync();
    if (n < np_loaded) throw Error(FEMPIC_EINVAL, "buffer too short");
    // particles absorbed at a wall: tet -1, position and velocity NaN
    const double nan = std::numeric_limits<double>::quiet_NaN();
    for (int64_t o = 0; o < np_loaded; o++) {
        for (int c = 0; c < 3; c++) {
            if (pos) pos[3 * o + c] = nan;
            if (vel) vel[3 * o + c] = nan;
        }
        if (tet) tet[o] = -1;
    }
    if (!loaded || np == 0) return;
    const std::vector<char> img = rows_get(gather_current(), 0, np);
    const PartLayout &L = part_layout(mixed);
    for (int64_t i = 0; i < np; i++) {
        const int64_t o = unit_get<int32_t>(img, np, L.id, i);
        const int32_t tt = unit_get<int32_t>(img, np, L.tet, i);
        // position from the barycentric coordinates: x_0 + sum_m l_m (x_m - x_0)
        const int32_t *tv = &m.tets[4 * (int64_t)tt];
        const double *x0 = &m.xyz[3 * tv[0]];
        for (int c = 0; c < 3; c++) {
            double r = x0[c];
            for (int k = 1; k < 4; k++)
                r += unit_get<double>(img, np, L.lam + 2 * (k - 1), i) * (m.xyz[3 * tv[k] + c] - x0[c]);
            if (pos) pos[3 * o + c] = r;
            if (vel) vel[3 * o + c] = unit_get<double>(img, np, L.v + 2 * c, i);
        }
        if (tet) tet[o] = tt;
    }
}

// ------------------------------------------------------------ checkpoint
// A checkpoint holds the state the next step reads, raw as it lies on the
// device: the particles in the order the next step takes them (tet order),
// with their velocity and AB4 histories in the run's storage precision; e, b,
// the accumulated current moments g and the reference charge rho~^0; the
// species, the step counter and the sizes that identify mesh and precision.
// A run restored from it on the same mesh with the same parameters takes the
// next steps bit for bit as the saved run does.
namespace {
constexpr char CKPT_MAGIC[8] = {'F', 'E', 'M', 'P', 'I', 'C', 'C', 'K'};
constexpr uint32_t CKPT_VERSION = 3;

struct CkptHeader {
    char magic[8];
    uint32_t version;
    int32_t precision, order, hist_bytes;
    int64_t nt, n1, n1_int, n2, n0_int, np, steps;
    double dt, q, mass, w;
    double gamma, beta;  // Newmark-beta parameters
    int32_t have_prev;   // three-level scheme: the field history below holds a step
    int32_t particle_bc;
    int64_t np_loaded;   // particles at load (ids are below it; absorbed ones are gone)
    int32_t has_imp;     // an impressed field follows the payload's fields
    int32_t pusher;      // FEMPIC_PUSH_AB4 or FEMPIC_PUSH_BORIS
};

// 64-bit FNV-1a over the payload taken as a stream of 8-byte words (a last
// partial word is zero-padded), so the value does not depend on how the payload
// is split into calls
struct Hash64 {
    uint64_t h = 1469598103934665603ull;
    unsigned char buf[8] = {};
    int nbuf = 0;
    void word(const unsigned char *c)
    {
        uint64_t wd;
        std::memcpy(&wd, c, 8);
        h = (h ^ wd) * 1099511628211ull;
    }
    void add(const void *p, size_t n)
    {
        const unsigned char *c = (const unsigned char *)p;
        size_t i = 0;
        while (nbuf && i < n) {
            buf[nbuf++] = c[i++];
            if (nbuf == 8) {
                word(buf);
                nbuf = 0;
            }
        }
        for (; i + 8 <= n; i += 8) word(c + i);
        while (i < n) buf[nbuf++] = c[i++];
    }
    uint64_t value() const
    {
        Hash64 t = *this;
        if (t.nbuf) {
            std::memset(t.buf + t.nbuf, 0, 8 - t.nbuf);
            t.word(t.buf);
        }
        return t.h;
    }
};

struct CkptFile {
    std::FILE *f = nullptr;
    std::string path;
    Hash64 hash;
    CkptFile(const char *p, const char *mode) : path(p)
    {
        f = std::fopen(p, mode);
        if (!f) throw Error(FEMPIC_EINVAL, "cannot open checkpoint " + path);
    }
    ~CkptFile()
    {
        if (f) std::fclose(f);
    }
    void write(const void *p, size_t n, bool hashed = true)
    {
        if (n && std::fwrite(p, 1, n, f) != n) throw Error(FEMPIC_EINVAL, "cannot write checkpoint " + path);
        if (hashed) hash.add(p, n);
    }
    void read(void *p, size_t n, bool hashed = true)
    {
        if (n && std::fread(p, 1, n, f) != n) throw Error(FEMPIC_EINVAL, "checkpoint " + path + " is truncated");
        if (hashed) hash.add(p, n);
    }
    void close_write()
    {
        const int r = std::fclose(f);
        f = nullptr;
        if (r != 0) throw Error(FEMPIC_EINVAL, "cannot write checkpoint " + path);
    }
};
}  // namespace

void Run::save(const char *path)
{
    Range rg("fempic checkpoint save");
    if (!path) throw Error(FEMPIC_EINVAL, "null path");
    if (!loaded) throw Error(FEMPIC_EINVAL, "no particles loaded");
    sync();
    // the particles in the next step's order, into the buffer set the next step writes
    const PBufs &S = gather_current();
    CkptHeader h{};
    std::memcpy(h.magic, CKPT_MAGIC, 8);
    h.version = CKPT_VERSION;
    h.precision = mixed ? FEMPIC_MIXED : FEMPIC_FP64;
    h.order = order;
    h.hist_bytes = mixed ? 4 : 8;
    h.nt = m.nt;
    h.n1 = m.N1;
    h.n1_int = n1s;
    h.n2 = m.N2;
    h.n0_int = m.N0_int;
    h.np = np;
    h.steps = steps_done;
    h.dt = prm.dt;
    h.q = q;
    h.mass = mass;
    h.w = w;
    h.gamma = prm.gamma;
    h.beta = prm.beta;
    h.have_prev = three_level && have_prev ? 1 : 0;
    h.particle_bc = prm.particle_bc;
    h.pusher = prm.pusher;
    h.np_loaded = np_loaded;
    h.has_imp = has_imp ? 1 : 0;
    CkptFile F(path, "wb");
    F.write(&h, sizeof h);
    std::vector<char> stage;
    auto put = [&](const void *d, size_t bytes) {
        stage.resize(std::max<size_t>(bytes, 1));
        if (bytes) HIPCHECK(hipMemcpy(stage.data(), d, bytes, hipMemcpyDeviceToHost));
        F.write(stage.data(), bytes);
    };
    {
        // the particles field by field (one column per scalar), from a host image of the rows
        const std::vector<char> img = rows_get(S, 0, np);
        const PartLayout &L = part_layout(mixed);
        const int rs = mixed ? 4 : 8;
        auto col = [&](int u, int bytes) {
            stage.resize(std::max<size_t>((size_t)np * bytes, 1));
            for (int64_t i = 0; i < np; i++) std::memcpy(&stage[(size_t)i * bytes], img.data() + part_off(u, np, i), bytes);
            F.write(stage.data(), (size_t)np * bytes);
        };
        for (int c = 0; c < 3; c++) col(L.lam + 2 * c, 8);
        for (int c = 0; c < 3; c++) col(L.v + 2 * c, 8);
        for (int c = 0; c < 9; c++) col(L.vh + L.hs * c, rs);
        for (int c = 0; c < 9; c++) col(L.ah + L.hs * c, rs);
        col(L.tet, 4);
        col(L.id, 4);
    }
    put(d_e.p, m.N1 * 8);
    put(d_b.p, m.N2 * 8);
    put(d_g.p, n1s * 8);
    put(d_rho0.p, m.N0_int * 8);
    put(d_e_lo.p, n1s * 8);
    put(d_g_lo.p, n1s * 8);
    if (h.have_prev) {
        put(d_eprev.p, n1s * 8);
        put(d_bprev.p, m.N2 * 8);
        put(d_dgprev.p, n1s * 8);
        put(d_dprev.p, n1s * 8);
        put(d_dprev_lo.p, n1s * 8);
    }
    if (h.has_imp) put(d_bimp.p, m.N2 * 8);
    const uint64_t sum = F.hash.value();
    F.write(&sum, 8, false);
    F.close_write();
}

void Run::restore(const char *path)
{
    Range rg("fempic checkpoint load");
    AccountScope charge(&acct);
    if (!path) throw Error(FEMPIC_EINVAL, "null path");
    HIPCHECK(hipStreamSynchronize(stream));
    CkptFile F(path, "rb");
    CkptHeader h{};
    F.read(&h, sizeof h);
    if (std::memcmp(h.magic, CKPT_MAGIC, 8) != 0 || h.version != CKPT_VERSION)
        throw Error(FEMPIC_EINVAL, "not a checkpoint of this library: " + F.path);
    if (h.precision != (mixed ? FEMPIC_MIXED : FEMPIC_FP64) || h.hist_bytes != (mixed ? 4 : 8))
        throw Error(FEMPIC_EINVAL, "checkpoint precision differs from the run's");
    if (h.order != order || h.nt != m.nt || h.n1 != m.N1 || h.n1_int != n1s || h.n2 != m.N2 ||
        h.n0_int != m.N0_int)
        throw Error(FEMPIC_EINVAL, "checkpoint is of another mesh, order or field wall condition");
    if (h.dt != prm.dt) throw Error(FEMPIC_EINVAL, "checkpoint time step differs from the run's");
    if (h.gamma != prm.gamma || h.beta != prm.beta)
        throw Error(FEMPIC_EINVAL, "checkpoint Newmark-beta parameters differ from the run's");
    if (h.have_prev != 0 && (h.have_prev != 1 || !three_level)) throw Error(FEMPIC_EINVAL, "checkpoint header is corrupt");
    if (h.has_imp != 0 && h.has_imp != 1) throw Error(FEMPIC_EINVAL, "checkpoint header is corrupt");
    if (h.np < 0 || h.np >= ((int64_t)1 << 31) / 2 || h.steps < 0 || h.np_loaded < h.np ||
        h.np_loaded >= ((int64_t)1 << 31) / 2)
        throw Error(FEMPIC_EINVAL, "checkpoint header is corrupt");
    if (h.particle_bc != prm.particle_bc) throw Error(FEMPIC_EINVAL, "checkpoint particle wall condition differs");
    if (h.pusher != prm.pusher) throw Error(FEMPIC_EINVAL, "checkpoint pusher differs");
    if (!(h.mass > 0) || !std::isfinite(h.q) || !std::isfinite(h.w))
        throw Error(FEMPIC_EINVAL, "checkpoint species is corrupt");
    const int64_t n = h.np;
    const size_t rs = mixed ? 4 : 8;
    {
        // the size the header implies, before anything is allocated for it
        const long here = std::ftell(F.f);
        const uint64_t want = (uint64_t)sizeof(CkptHeader) + (uint64_t)n * (6 * 8 + 18 * rs + 8) +
                              (uint64_t)(m.N1 + m.N2 + 3 * n1s + m.N0_int) * 8 +
                              (h.have_prev ? (uint64_t)(4 * n1s + m.N2) * 8 : 0) +
                              (h.has_imp ? (uint64_t)m.N2 * 8 : 0) + 8;
        if (here < 0 || std::fseek(F.f, 0, SEEK_END) != 0) throw Error(FEMPIC_EINVAL, "cannot read checkpoint " + F.path);
        const long size = std::ftell(F.f);
        if (size < 0 || (uint64_t)size != want || std::fseek(F.f, here, SEEK_SET) != 0)
            throw Error(FEMPIC_EINVAL, "checkpoint " + F.path + " is truncated or has the wrong size");
    }
    // read and check everything on the host before any of it reaches the device
    std::vector<double> x(3 * n), v(3 * n);
    std::vector<char> vh(9 * n * rs), ah(9 * n * rs);
    std::vector<int32_t> tet(n), id(n);
    std::vector<double> e(m.N1), b(m.N2), g(n1s), rho0(m.N0_int), e_lo(n1s), g_lo(n1s);
    F.read(x.data(), x.size() * 8);
    F.read(v.data(), v.size() * 8);
    F.read(vh.data(), vh.size());
    F.read(ah.data(), ah.size());
    F.read(tet.data(), n * 4);
    F.read(id.data(), n * 4);
    F.read(e.data(), e.size() * 8);
    F.read(b.data(), b.size() * 8);
    F.read(g.data(), g.size() * 8);
    F.read(rho0.data(), rho0.size() * 8);
    F.read(e_lo.data(), e_lo.size() * 8);
    F.read(g_lo.data(), g_lo.size() * 8);
    std::vector<double> ep, bp, dgp, dpv, dpl;
    if (h.have_prev) {
        ep.resize(n1s);
        bp.resize(m.N2);
        dgp.resize(n1s);
        dpv.resize(n1s);
        dpl.resize(n1s);
        F.read(ep.data(), ep.size() * 8);
        F.read(bp.data(), bp.size() * 8);
        F.read(dgp.data(), dgp.size() * 8);
        F.read(dpv.data(), dpv.size() * 8);
        F.read(dpl.data(), dpl.size() * 8);
    }
    std::vector<double> bim;
    if (h.has_imp) {
        bim.resize(m.N2);
        F.read(bim.data(), bim.size() * 8);
    }
    const uint64_t want = F.hash.value();
    uint64_t sum = 0;
    F.read(&sum, 8, false);
    if (sum != want) throw Error(FEMPIC_EINVAL, "checkpoint checksum mismatch: " + F.path);
    for (double a : x)
        if (!std::isfinite(a)) throw Error(FEMPIC_EINVAL, "checkpoint holds a non-finite position");
    for (double a : v)
        if (!std::isfinite(a)) throw Error(FEMPIC_EINVAL, "checkpoint holds a non-finite velocity");
    for (const std::vector<double> *f : {&e, &b, &ep, &bp, &dpv, &dpl, &bim})
        for (double a : *f)
            if (!std::isfinite(a)) throw Error(FEMPIC_EINVAL, "checkpoint holds a non-finite field coefficient");
    for (const std::vector<char> *hv : {&vh, &ah})
        for (size_t k = 0; k < hv->size(); k += rs) {
            double a;
            if (mixed) {
                float f;
                std::memcpy(&f, hv->data() + k, 4);
                a = f;
            } else {
                std::memcpy(&a, hv->data() + k, 8);
            }
            if (!std::isfinite(a)) throw Error(FEMPIC_EINVAL, "checkpoint holds a non-finite history value");
        }
    std::vector<char> seen(std::max<int64_t>(h.np_loaded, 1), 0);
    for (int64_t i = 0; i < n; i++) {
        if (tet[i] < 0 || tet[i] >= m.nt) throw Error(FEMPIC_EINVAL, "checkpoint holds a tet outside the mesh");
        if (id[i] < 0 || id[i] >= h.np_loaded || seen[id[i]])
            throw Error(FEMPIC_EINVAL, "checkpoint particle ids are corrupt");
        seen[id[i]] = 1;
    }
    q = h.q;
    mass = h.mass;
    w = h.w;
    alloc_particles(n);
    {
        const PartLayout &L = part_layout(mixed);
        std::vector<char> img((size_t)std::max<int64_t>(n, 1) * L.nw * 16, 0);
        auto col = [&](int u, const char *src, int bytes) {
            for (int64_t i = 0; i < n; i++) std::memcpy(img.data() + part_off(u, n, i), src + (size_t)i * bytes, bytes);
        };
        for (int c = 0; c < 3; c++) col(L.lam + 2 * c, (const char *)&x[c * n], 8);
        for (int c = 0; c < 3; c++) col(L.v + 2 * c, (const char *)&v[c * n], 8);
        for (int c = 0; c < 9; c++) col(L.vh + L.hs * c, &vh[c * n * rs], (int)rs);
        for (int c = 0; c < 9; c++) col(L.ah + L.hs * c, &ah[c * n * rs], (int)rs);
        col(L.tet, (const char *)tet.data(), 4);
        col(L.id, (const char *)id.data(), 4);
        rows_put(pb[0], 0, n, img);
        rows_used = n;
    }
    auto get = [&](void *d, const void *src, size_t bytes) {
        if (bytes) HIPCHECK(hipMemcpy(d, src, bytes, hipMemcpyHostToDevice));
    };
    get(d_e.p, e.data(), e.size() * 8);
    get(d_b.p, b.data(), b.size() * 8);
    get(d_g.p, g.data(), g.size() * 8);
    get(d_rho0.p, rho0.data(), rho0.size() * 8);
    get(d_e_lo.p, e_lo.data(), e_lo.size() * 8);
    get(d_g_lo.p, g_lo.data(), g_lo.size() * 8);
    if (h.have_prev) {
        get(d_eprev.p, ep.data(), ep.size() * 8);
        get(d_bprev.p, bp.data(), bp.size() * 8);
        get(d_dgprev.p, dgp.data(), dgp.size() * 8);
        get(d_dprev.p, dpv.data(), dpv.size() * 8);
        get(d_dprev_lo.p, dpl.data(), dpl.size() * 8);
    }
    have_prev = h.have_prev != 0;
    has_imp = h.has_imp != 0;
    if (has_imp) {
        if (!d_bimp.p) d_bimp.alloc(std::max<int64_t>(m.N2, 1) * 8);
        if (!d_bg.p) d_bg.alloc(std::max<int64_t>(m.N2, 1) * 8);
        get(d_bimp.p, bim.data(), bim.size() * 8);
    }
    np_loaded = h.np_loaded;
    absorbed_total = h.np_loaded - h.np;
    last_absorb = 0;
    if (mixed) HIPCHECK(cast_d2f(m.N1, (const double *)d_e.p, (float *)d_e32.p, 1.0, stream));
    refresh_gather_b();
    HIPCHECK(hipStreamSynchronize(stream));
    steps_done = h.steps;
    gauss_step = 0;
    for (double &g : gauss_last) g = 0.0;
    sticky = 0;
    loaded = true;
}

void Run::history_get(double *vh, double *ah, int64_t n)
{
    sync();
    if (prm.pusher == FEMPIC_PUSH_BORIS) throw Error(FEMPIC_EINVAL, "the Boris push keeps no AB4 history");
    if (n < np_loaded) throw Error(FEMPIC_EINVAL, "buffer too short");
    const double nan = std::numeric_limits<double>::quiet_NaN();
    for (int64_t k = 0; k < 9 * np_loaded; k++) {
        if (vh) vh[k] = nan;
        if (ah) ah[k] = nan;
    }
    if (!loaded || np == 0) return;
    const std::vector<char> img = rows_get(gather_current(), 0, np);
    const PartLayout &L = part_layout(mixed);
    auto hist = [&](int u0, int c, int64_t i) {
        return mixed ? (double)unit_get<float>(img, np, u0 + c, i) : unit_get<double>(img, np, u0 + 2 * c, i);
    };
    for (int64_t i = 0; i < np; i++) {
        const int64_t o = unit_get<int32_t>(img, np, L.id, i);
        for (int c = 0; c < 9; c++) {
            // the device keeps v^{n-j} - v^n; the caller gets v^{n-j}
            if (vh) vh[9 * o + c] = hist(L.vh, c, i) + unit_get<double>(img, np, L.v + 2 * (c % 3), i);
            if (ah) ah[9 * o + c] = hist(L.ah, c, i);
        }
    }
}

// Mirrors what the constructor, load and the first particle phase allocate.
// The operators' nonzeros are bounded per row by what Kuhn cubes reach as N
// grows (order 1: A 16, K 3, G^T 14; order 2: about 44, 12 and 24), with a margin.
size_t footprint_bytes(const FootprintSizes &z, int64_t n, bool mixed)
{
    const bool k2 = z.order == 2;
    const double n1l = k2 ? 20 : 6, n2l = k2 ? 15 : 4, n0l = k2 ? 10 : 4;
    const double nt = (double)z.nt, N1 = (double)z.n1, N1i = (double)(z.absorbing ? z.n1 : z.n1_int),
                 N2 = (double)z.n2, N0i = (double)z.n0_int;
    const double nnzA = N1i * (k2 ? 46.0 : 17.0), nnzK = N2 * (k2 ? 13.0 : 3.0), nnzG = N0i * (k2 ? 25.0 : 15.0),
                 nnzNu = N2 * (k2 ? 24.0 : 7.0);
    auto csr = [](double rows, double nnz) { return (rows + 1) * 8 + nnz * 12 + 256; };
    // A and *eps, with 2x2 block copies at order 2; K, K^T, *nu, G^T
    double ops = 2 * csr(N1i, nnzA) + (mixed ? nnzA * 4 : 0) + csr(N2, nnzK) + csr(N1i, nnzK) + csr(N2, nnzNu) +
                 csr(N0i, nnzG);
    if (k2) ops += 2 * ((N1i / 2 + 1) * 8 + nnzA * 9 + 256) + (mixed ? nnzA * 4 : 0);
    // the surface impedance matrix: a wall DoF meets the DoFs of its wall faces
    if (z.absorbing) ops += csr(N1i, (N1 - (double)z.n1_int) * (k2 ? 16.0 : 5.0));
    const double precond = (k2 ? 2 : 1) * N1i * (8 + (mixed ? 4 : 0));
    const double inc = (N1i + 1) * 8 + nt * n1l * 4 + (N0i + 1) * 8 + nt * n0l * 4;
    const double mesh = nt * (16 * 8 + 16 + (n1l + n2l + n0l) * 4);
    // the operator applied tet by tet (PEC walls): geometry and per-tet products
    const double matfree = z.absorbing ? 0.0
                                       : nt * (16 + n1l) * (mixed ? 4 : 8) +
                                             (k2 ? 2 * nt * n1l / 2 * 4 + (N1i / 2 + 1) * 8 : 0);
    double vecs = (N1 + N2) * 8 + 5 * N1i * 8 + (mixed ? (N1 + N2) * 4 : 0) + 8 * N1i * 8 +
                  (mixed ? 5 * N1i * 4 : 0) + N2 * 8 + 4 * N0i * 8;
    vecs += 5 * N1i * 8 + N2 * 8;  // double-double halves, *nu u, the previous increment
    vecs += (std::max({N1i, N2, N0i, 1.0}) / 4 + 1024) * 32 + 512;
    const double tets = nt * (n1l + n0l) * 8 + 5 * (nt + 1) * 4 + (double)CONT_BLOCKS * NCNT * 8 + 4096;
    const double cap = (double)std::max<int64_t>(n, 1);
    const double parts = 2 * cap * part_layout(mixed).nw * 16;
    auto sorts = [&](double c) {
        const double hn = (double)sort_hist_entries((int64_t)c);
        const double tmp = (double)std::max({scan_tmp_entries((int64_t)hn), scan_tmp_entries((int64_t)c),
                                             scan_tmp_entries(z.nt)});
        return 4 * c * 4 + hn * 4 + tmp * 4 + 64;
    };
    const double pool_cap = std::max(cap + std::floor(cap / 2), 65536.0);
    const double pool = pool_cap * (n1l * 8 + 16) + sorts(pool_cap);
    const double queue = cap * (4 + 4 + sizeof(ContRec) + 1 + 4) + cap + 16 +
                         (2 * (cap / 4096 + 1) + (double)scan_tmp_entries((int64_t)(cap / 4096 + 1))) * 4 + 64;
    // every buffer is at least 16 bytes; a generous allowance for the few dozen small ones
    const double small = 64 * 1024;
    return (size_t)(ops + precond + inc + mesh + matfree + vecs + tets + parts + sorts(cap) + pool + queue + small);
}

FootprintSizes kuhn_sizes(int order, double nt)
{
    const double N = std::cbrt(std::max(nt, 1.0) / 6.0);
    const double V = std::pow(N + 1.0, 3), T = 6.0 * N * N * N;
    const double E = 3.0 * N * (N + 1.0) * (N + 1.0) + 3.0 * N * N * (N + 1.0) + N * N * N;
    const double F = 12.0 * N * N * N + 6.0 * N * N;
    const double N1 = order == 1 ? E : 2 * E + 2 * F, N2 = order == 1 ? F : 3 * F + 3 * T;
    const double N0 = order == 1 ? V : V + E;
    auto up = [](double x) { return (int64_t)std::ceil(x); };
    return FootprintSizes{order, up(T), up(N1), up(N1), up(N2), up(N0)};
}

size_t Run::footprint_estimate(const HostMesh &m, int64_t n, bool mixed, bool absorbing)
{
    return footprint_bytes(FootprintSizes{m.order, m.nt, m.N1, m.N1_int, m.N2, m.N0_int, absorbing}, n, mixed);
}

void check_params(const fempic_params &p)
{
    if (p.precision != FEMPIC_FP64 && p.precision != FEMPIC_MIXED) throw Error(FEMPIC_EINVAL, "bad precision");
    if (!(p.dt > 0) || !std::isfinite(p.dt)) throw Error(FEMPIC_EINVAL, "dt must be positive");
    // the unconditionally stable members of the Newmark-beta family: 2 beta >= gamma >= 1/2
    if (!std::isfinite(p.gamma) || !std::isfinite(p.beta) || !(p.gamma >= 0.5) || !(2.0 * p.beta >= p.gamma) ||
        p.gamma > 1e6)
        throw Error(FEMPIC_EINVAL, "Newmark-beta needs 2 beta >= gamma >= 1/2");
    if (!(p.pcg_rtol > 0) || p.pcg_maxit < 1) throw Error(FEMPIC_EINVAL, "bad solver settings");
    if (p.particle_bc != FEMPIC_REFLECT && p.particle_bc != FEMPIC_ABSORB)
        throw Error(FEMPIC_EINVAL, "unsupported particle boundary condition");
    if (p.gauss_every < 0) throw Error(FEMPIC_EINVAL, "gauss_every must be >= 0");
    if (p.pusher != FEMPIC_PUSH_AB4 && p.pusher != FEMPIC_PUSH_BORIS) throw Error(FEMPIC_EINVAL, "unknown pusher");
    if (p.field_bc != FEMPIC_FIELD_PEC && p.field_bc != FEMPIC_FIELD_ABSORB)
        throw Error(FEMPIC_EINVAL, "unknown field boundary condition");
    if (p.field_bc == FEMPIC_FIELD_ABSORB && !(p.gamma == 0.5 && p.beta == 0.25))
        throw Error(FEMPIC_EINVAL, "absorbing walls need the trapezoidal scheme (gamma, beta = 1/2, 1/4)");
}

}  // namespace fempic

// =================================================================== C ABI
using namespace fempic;

struct fempic_mesh_s {
    std::shared_ptr<const HostMesh> m;  // runs made on the mesh hold it too
};
struct fempic_run_s {
    std::unique_ptr<Run> r;
};

#define API_BEGIN try {
#define API_END                                     \
    }                                               \
    catch (const Error &e) {                        \
        set_error(e.what());                        \
        return e.code;                              \
    }                                               \
    catch (const std::bad_alloc &) {                \
        set_error("host allocation failed");        \
        return FEMPIC_ENOMEM;                       \
    }                                               \
    catch (const std::exception &e) {              \
        set_error(e.what());                        \
        return FEMPIC_EINVAL;                       \
    }                                               \
    catch (...) {                                   \
        set_error("unknown failure");               \
        return FEMPIC_EINVAL;                       \
    }                                               \
    set_error("");                                  \
    return FEMPIC_OK;

extern "C" {

const char *fempic_last_error(void) { return g_last_error.c_str(); }

int32_t fempic_mesh_create(const double *xyz, int64_t n_vert, const int64_t *tet4, int64_t n_tet, int32_t order,
                           fempic_mesh *out)
{
    API_BEGIN
    if (!out) throw Error(FEMPIC_EINVAL, "null out");
    std::shared_ptr<const HostMesh> m(build_mesh(xyz, n_vert, tet4, n_tet, order));
    *out = new fempic_mesh_s{std::move(m)};
    API_END
}

int32_t fempic_mesh_create_cube(int32_t N, double L, int32_t order, fempic_mesh *out)
{
    API_BEGIN
    if (!out) throw Error(FEMPIC_EINVAL, "null out");
    std::shared_ptr<const HostMesh> m(build_cube(N, L, order));
    *out = new fempic_mesh_s{std::move(m)};
    API_END
}

int32_t fempic_mesh_destroy(fempic_mesh mesh)
{
    delete mesh;
    return FEMPIC_OK;
}

int32_t fempic_mesh_info(fempic_mesh mesh, fempic_mesh_info_t *out)
{
    API_BEGIN
    if (!mesh || !out) throw Error(FEMPIC_EINVAL, "null argument");
    const HostMesh &m = *mesh->m;
    fempic_mesh_info_t i{};
    i.n_vert = m.nv;
    i.n_edge = m.ne;
    i.n_face = m.nf;
    i.n_tet = m.nt;
    i.n1 = m.N1;
    i.n1_int = m.N1_int;
    i.n2 = m.N2;
    i.n0 = m.N0;
    i.n0_int = m.N0_int;
    i.order = m.order;
    i.n1_loc = m.n1l;
    i.n2_loc = m.n2l;
    i.n0_loc = m.n0l;
    i.dt_cfl = m.dt_cfl;
    *out = i;
    API_END
}

int32_t fempic_run_create(fempic_mesh mesh, const fempic_params *params, void *hip_stream, fempic_run *out)
{
    API_BEGIN
    if (!mesh || !params || !out) throw Error(FEMPIC_EINVAL, "null argument");
    const fempic_params &p = *params;
    check_params(p);
    auto *h = new fempic_run_s();
    try {
        h->r.reset(new Run(mesh->m, p, (hipStream_t)hip_stream));
    } catch (...) {
        delete h;
        throw;
    }
    *out = h;
    API_END
}

int32_t fempic_run_destroy(fempic_run run)
{
    delete run;
    return FEMPIC_OK;
}

int32_t fempic_particles_load(fempic_run run, const double *pos, const double *vel, int64_t n, double q, double m,
                              double w)
{
    API_BEGIN
    if (!run) throw Error(FEMPIC_EINVAL, "null run");
    run->r->load(pos, vel, n, q, m, w);
    API_END
}

int32_t fempic_step(fempic_run run, int32_t n_steps)
{
    API_BEGIN
    if (!run || n_steps < 0) throw Error(FEMPIC_EINVAL, "bad argument");
    run->r->step(n_steps);
    API_END
}

int32_t fempic_sync(fempic_run run)
{
    API_BEGIN
    if (!run) throw Error(FEMPIC_EINVAL, "null run");
    run->r->sync();
    API_END
}

int32_t fempic_gauss_residual(fempic_run run, double out[3])
{
    API_BEGIN
    if (!run || !out) throw Error(FEMPIC_EINVAL, "null argument");
    double v[3];
    run->r->gauss(v);
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
    API_END
}

int32_t fempic_gauss_residual_noalloc(fempic_run run, double out[3])
{
    API_BEGIN
    if (!run || !out) throw Error(FEMPIC_EINVAL, "null argument");
    double v[3];
    run->r->gauss_noalloc(v);
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
    API_END
}

int32_t fempic_fields_get(fempic_run run, double *e, int64_t ne, double *b, int64_t nb)
{
    API_BEGIN
    if (!run) throw Error(FEMPIC_EINVAL, "null run");
    run->r->fields_get(e, ne, b, nb);
    API_END
}

int32_t fempic_fields_set(fempic_run run, const double *e, int64_t ne, const double *b, int64_t nb)
{
    API_BEGIN
    if (!run) throw Error(FEMPIC_EINVAL, "null run");
    run->r->fields_set(e, ne, b, nb);
    API_END
}

int32_t fempic_deposit_get(fempic_run run, double *dg, int64_t n)
{
    API_BEGIN
    if (!run || !dg) throw Error(FEMPIC_EINVAL, "null argument");
    run->r->deposit_get(dg, n);
    API_END
}

int32_t fempic_field_matvec(fempic_run run, const double *x, double *y, int64_t n, int32_t form)
{
    API_BEGIN
    if (!run || !x || !y) throw Error(FEMPIC_EINVAL, "null argument");
    run->r->field_matvec(x, y, n, form);
    API_END
}

int32_t fempic_impressed_points(fempic_mesh mesh, int32_t n1d, double *xyz, int64_t n)
{
    API_BEGIN
    if (!mesh) throw Error(FEMPIC_EINVAL, "null mesh");
    if (n1d < 1 || n1d > 8) throw Error(FEMPIC_EINVAL, "the rule takes 1 to 8 points per direction");
    const HostMesh &m = *mesh->m;
    std::vector<double> lam, w;
    impressed_rule(n1d, lam, w);
    const int64_t P = (int64_t)w.size();
    if (!xyz || n < m.nt * P) throw Error(FEMPIC_EINVAL, "xyz must hold n_tet * n1d^3 points");
    for (int64_t t = 0; t < m.nt; t++) {
        const int32_t *v = &m.tets[4 * t];
        for (int64_t q = 0; q < P; q++)
            for (int c = 0; c < 3; c++) {
                double r = 0.0;
                for (int k = 0; k < 4; k++) r += lam[4 * q + k] * m.xyz[3 * v[k] + c];
                xyz[3 * (t * P + q) + c] = r;
            }
    }
    API_END
}

int32_t fempic_impressed_set(fempic_run run, const double *B, int64_t n, int32_t n1d, int32_t constrained,
                             double *b_out, int64_t nb)
{
    API_BEGIN
    if (!run) throw Error(FEMPIC_EINVAL, "null run");
    run->r->impressed_set(B, n, n1d, constrained != 0, b_out, nb);
    API_END
}

int32_t fempic_particles_inject(fempic_run run, const double *pos, const double *vel, int64_t n)
{
    API_BEGIN
    if (!run) throw Error(FEMPIC_EINVAL, "null run");
    run->r->inject(pos, vel, n);
    API_END
}

int32_t fempic_rho_get(fempic_run run, double *rho, double *rho0, int64_t n)
{
    API_BEGIN
    if (!run) throw Error(FEMPIC_EINVAL, "null run");
    run->r->rho_get(rho, rho0, n);
    API_END
}

int32_t fempic_particles_get(fempic_run run, double *pos, double *vel, int64_t *tet, int64_t n)
{
    API_BEGIN
    if (!run) throw Error(FEMPIC_EINVAL, "null run");
    run->r->particles_get(pos, vel, tet, n);
    API_END
}

int32_t fempic_history_get(fempic_run run, double *vh, double *ah, int64_t n)
{
    API_BEGIN
    if (!run) throw Error(FEMPIC_EINVAL, "null run");
    run->r->history_get(vh, ah, n);
    API_END
}

int32_t fempic_run_save(fempic_run run, const char *path)
{
    API_BEGIN
    if (!run) throw Error(FEMPIC_EINVAL, "null run");
    run->r->save(path);
    API_END
}

int32_t fempic_run_load(fempic_run run, const char *path)
{
    API_BEGIN
    if (!run) throw Error(FEMPIC_EINVAL, "null run");
    run->r->restore(path);
    API_END
}

int32_t fempic_run_set_log(fempic_run run, const char *path)
{
    API_BEGIN
    if (!run) throw Error(FEMPIC_EINVAL, "null run");
    run->r->set_log(path);
    API_END
}

int32_t fempic_set_allocator(fempic_alloc_fn alloc, fempic_free_fn release, void *ctx)
{
    API_BEGIN
    set_device_allocator(alloc, release, ctx);
    API_END
}

int32_t fempic_stats(fempic_run run, fempic_stats_t *out)
{
    API_BEGIN
    if (!run || !out) throw Error(FEMPIC_EINVAL, "null argument");
    const Run &r = *run->r;
    fempic_stats_t s{};
    s.steps = r.steps_done;
    s.n_particles = r.np;
    s.n_loaded = r.np_loaded;
    s.absorbed = r.last_absorb;
    s.absorbed_total = r.absorbed_total;
    s.particle_ms = r.last_particle_ms;
    s.particle_kernel_ms = r.last_kernel_ms;
    s.continue_kernel_ms = r.last_continue_ms;
    s.field_ms = r.last_field_ms;
    s.pcg_iters = r.last_iters;
    s.pcg_relres = r.last_relres;
    s.crossings = r.last_cross;
    s.reflections = r.last_refl;
    s.spills = r.last_spill;
    for (int k = 0; k < 3; k++) s.gauss[k] = r.gauss_last[k];
    s.gauss_step = r.gauss_step;
    s.a_rows = r.n1s;
    s.a_nnz = r.a_nnz;
    s.device_bytes = (int64_t)r.account().bytes;
    s.device_peak_bytes = (int64_t)r.account().peak;
    s.phase_replays = r.last_phase_replays;
    s.field_op = r.field_op();
    s.a_inc = r.a_inc;
    *out = s;
    API_END
}

int32_t fempic_footprint_mesh(fempic_mesh mesh, int64_t n_particles, int32_t precision, size_t *bytes)
{
    API_BEGIN
    if (!mesh || !bytes || n_particles < 0 || (precision != FEMPIC_FP64 && precision != FEMPIC_MIXED))
        throw Error(FEMPIC_EINVAL, "bad argument");
    *bytes = Run::footprint_estimate(*mesh->m, n_particles, precision == FEMPIC_MIXED);
    API_END
}

int32_t fempic_footprint(int32_t order, int64_t n_tet, int64_t n_particles, int32_t precision, size_t *bytes)
{
    API_BEGIN
    if (!bytes || (order != 1 && order != 2) || n_tet < 1 || n_particles < 0 ||
        (precision != FEMPIC_FP64 && precision != FEMPIC_MIXED))
        throw Error(FEMPIC_EINVAL, "bad argument");
    *bytes = footprint_bytes(kuhn_sizes(order, (double)n_tet), n_particles, precision == FEMPIC_MIXED);
    API_END
}

}  // extern "C"
