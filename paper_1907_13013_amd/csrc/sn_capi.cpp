// C ABI of the slab S_N / FPSA library: handle management, validation,
// device residency of the setup data, and the solver drivers.
#include "snfpsa.h"
#include "snfpsa_diag.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "setup_math.hpp"
#include "sn_adjoint.hpp"
#include "sn_batch_host.hpp"
#include "sn_kernels.hpp"
#include "sn_krylov.hpp"

using namespace snfpsa;

static_assert(FP_CELLMATS == FP_CELL_MATS, "host and device factor layouts differ");
static_assert(SN_KERNEL_COUNT == KID_COUNT, "kernel ids of the header and the kernels differ");

namespace {

thread_local std::string g_err;

sn_status fail(sn_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

struct HipError {
    hipError_t e;
    std::string where;
};

#define HIPCHK(call)                                                                 \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) throw HipError{e_, std::string(#call)};                \
    } while (0)

// Per-kernel HIP-event timing (enabled on request): every launch records its
// own dispatch begin/end into an event pair on its stream; resolved lazily.
struct EventTimer final : KernelTimer {
    struct Rec {
        int id;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    int64_t launches[KID_COUNT] = {};
    double total_ms[KID_COUNT] = {};

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) throw HipError{hipErrorOutOfMemory, "hipEventCreate"};
        return e;
    }
    bool events(int id, hipEvent_t *start, hipEvent_t *stop) override {
        if (pending.size() >= 8192) resolve();  // before handing out new events
        *start = get();
        *stop = get();
        pending.push_back({id, *start, *stop});
        return true;
    }
    void resolve() {
        for (Rec &r : pending) {
            float ms = 0.f;
            (void)hipEventSynchronize(r.b);
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                launches[r.id] += 1;
                total_ms[r.id] += ms;
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }
    ~EventTimer() override {
        resolve();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

struct Slab {
    int K = 0, N = 0, L = 0, NH = 0, L1 = 0;
    int64_t cell_off = 0, psi_off = 0, phi_off = 0, exit_off = 0;
    // device tables
    double *mu = nullptr, *inv_absmu = nullptr, *w = nullptr, *Mt = nullptr, *Vt = nullptr;
    double *h = nullptr, *sigma_t = nullptr, *sigma_s = nullptr;
    double *psi_left = nullptr, *psi_right = nullptr;
    // Fokker-Planck factors
    double *cellmats = nullptr, *psi_fwd = nullptr, *psi_bwd = nullptr;
    double *theta_fwd = nullptr, *theta_bwd = nullptr;
    double *EsrcT = nullptr, *PhisrcT = nullptr, *PhiinfT = nullptr;
    std::vector<int32_t> seg_begin, seg_type;
    int chunk = 0, nchunks = 0;
    // source maps without the cell's sigma_s (shared factorisations): the
    // correction GEMMs scale phi_half - phi_old by sigma_s2 = [K][2][L+1]
    bool fold_ss = true;
    double *sigma_s2 = nullptr;
    // sweep tiling
    int TC = 0, S = 0, sub = 0, ntiles = 0;
};

// Sweep tiling of a slab: 256 threads = S sub-chunks x N angles; the
// default takes about 128 tiles per slab (their carries are formed inside
// the apply kernel), at most 32 cells per tile (64 for N < 8) so that a
// tile's source and moments fit in LDS for the fused solve sweep.  The
// autotuner also tries half (policy 1) and twice (policy 2) that tile width.
constexpr int kTilePolicies = 3;

void set_tiling(Slab &b, int policy) {
    b.S = std::max(1, 256 / b.N);
    const int want = (b.K + 127) / 128;
    const int cap = b.N >= 8 ? 32 : 64;
    int tc = std::max(b.S, std::min(cap, ((want + b.S - 1) / b.S) * b.S));
    if (policy == 1) tc = std::max(b.S, ((tc / 2) / b.S) * b.S);
    if (policy == 2) tc = std::max(b.S, std::min(cap, 2 * tc));
    b.TC = tc;
    b.sub = (b.TC + b.S - 1) / b.S;
    b.ntiles = (b.K + b.TC - 1) / b.TC;
}

// Per-solve workspace sized for the largest slab.  An FP64 handle with
// several slabs holds up to kSlots of them, each with its own stream, so
// that independent slabs iterate concurrently (slot 0 uses the caller's
// stream).
struct Workspace {
    double *q = nullptr, *psi = nullptr, *phiA = nullptr, *phiB = nullptr, *phi_half = nullptr;
    double *s = nullptr, *pvec = nullptr, *inflow = nullptr, *e_fwd = nullptr, *e_bwd = nullptr;
    double *fvec = nullptr, *gvec = nullptr, *bvec = nullptr;
    double *part_f = nullptr, *part_b = nullptr;
    double *subA = nullptr, *subB = nullptr, *tileA = nullptr, *tileB = nullptr;
    double *carry = nullptr, *sweep_exit = nullptr;
    double *grpA = nullptr, *grpB = nullptr;
    unsigned long long *hist = nullptr;       // device, per-iteration stopping-test values
    unsigned long long *hist_host = nullptr;  // pinned
    int hist_cap = 0;
    hipStream_t stream = nullptr;             // null for slot 0 (the caller's stream)
    hipEvent_t done = nullptr;                // marks the end of the slot's queued batch
};
constexpr int kSlots = 8;

}  // namespace

// ---------------------------------------------------------------------------
// Multi-slab FP64 solve in batched launches.  Every kernel of an SI or FPSA
// iteration runs as one launch per kernel variant over all slabs of the
// handle (each slab and cell-type segment one descriptor, see MultiLaunch),
// so an iteration of hundreds of slabs costs a dozen launches instead of a
// dozen per slab.  Each slab keeps its own workspace, iterates, and column
// of a stopping-test ring; a slab whose test has passed is skipped by every
// later launch.  The launches read the iteration number from a device
// counter (advanced by the last launch of the iteration), so one set of
// descriptors serves the whole solve.  Blocks are interleaved across slabs,
// with slabs that share Fokker-Planck factors next to each other, so a
// shared factor read by one slab's block is in cache for the others'.
// ---------------------------------------------------------------------------
namespace {

struct F64Plan {
    int method = 0;
    const void *qext = nullptr;
    bool bc = true;
    const unsigned long long *hist = nullptr;
    double tol = 0.0;     // grouped Fokker-Planck launches test their slabs' convergence
    std::vector<MultiLaunch> launches;
    void *dev = nullptr;   // every launch's descriptors and block table (one allocation)
    void *dev2 = nullptr;  // the grouped launches' per-slab vector tables
    hipGraphExec_t exec = nullptr;  // one captured iteration (launches + counter step)
};

struct F64Batch {
    std::vector<Workspace> ws;  // per-slab views into mem
    double *phiA = nullptr, *phiB = nullptr, *phi_half = nullptr;  // [phi_len] each, slab b at phi_off
    void *mem = nullptr;
    int *iter = nullptr;
    std::vector<F64Plan> plans;  // most recently used last
    static constexpr size_t kPlans = 4;
    // graph capture and replay run on this stream, ordered after and
    // before the caller's stream by gev
    hipStream_t gstream = nullptr;
    hipEvent_t gev = nullptr;
    static void drop(F64Plan &p) {
        if (p.exec) (void)hipGraphExecDestroy(p.exec);
        if (p.dev) (void)hipFree(p.dev);
        if (p.dev2) (void)hipFree(p.dev2);
        p.exec = nullptr;
        p.dev = nullptr;
        p.dev2 = nullptr;
    }
    void release() {
        for (F64Plan &p : plans) drop(p);
        plans.clear();
        if (mem) (void)hipFree(mem);
        if (iter) (void)hipFree(iter);
        if (gstream) (void)hipStreamDestroy(gstream);
        if (gev) (void)hipEventDestroy(gev);
        mem = nullptr;
        iter = nullptr;
        gstream = nullptr;
        gev = nullptr;
    }
};

// phases of one iteration, in order; a slab's kernels fall into them in
// its own sequence, and one launch per kernel variant and phase serves all
// slabs
enum {
    PH_SCATTER = 0,   // unfused slabs: source GEMM
    PH_SWEEP_AGG,     // tile aggregates (fused: with the tile's source)
    PH_SCAN_GROUPS,   // long slabs: tile-group maps
    PH_SCAN_CARRY,    // long slabs: tile carry-ins
    PH_SWEEP_APPLY,   // sweep (fused: with the tile's moments, SI: and the stopping test)
    PH_MOMENTS,       // unfused slabs: moments GEMM
    PH_FP_SOURCE,     // FPSA: Fokker-Planck source per segment
    PH_FP_MATVEC,
    PH_FP_CHAIN,
    PH_FP_CARRY,
    PH_FP_FIXUP,
    PH_FP_UPDATE,     // FPSA: corrected moments per segment
    PH_STOP,          // FPSA with several segments: the stopping test
    PH_COUNT
};

struct PlanItem {
    LaunchShape sh;
    int kind = 0;  // 0 GEMM, 1 sweep, 2 Fokker-Planck, 3 stopping test, 4 grouped Fokker-Planck
    GemmArgs g;
    SweepArgs sw;
    FPArgs f;
    StopArgs st;
    FPGroupArgs fg;
    size_t vec_off = 0;  // kind 4: the group's FPSlabVecs in the plan's vector table
    IterPatch p;
    uintptr_t order = 0;  // items of one launch are ordered by this key
};

}  // namespace


struct sn_handle_s {
    int device = 0;
    int fp_scheme = 0;
    int precision = SN_F64;
    bool has_fp = false;                      // Fokker-Planck factors built
    BatchData *batch = nullptr;               // SN_F32 / SN_BF16X3 handles
    std::vector<Slab> slabs;
    int64_t psi_len = 0, phi_len = 0, exit_len = 0;
    std::vector<void *> allocs;
    std::vector<Workspace> ws;                // ws[0]: every call; ws[1..]: concurrent slabs in sn_solve
    hipEvent_t ev_order = nullptr;            // orders the slot streams after the caller's stream
    // adjoint workspace, allocated on first use: the transformed adjoint
    // source of every slab, one slab's adjoint angular flux, per-cell sums
    double *adj_q = nullptr, *adj_y = nullptr, *jpart = nullptr;
    size_t ws_psi_slab = 0, ws_cells_slab = 0;
    // GMRES workspace, allocated on first use: Krylov basis [(m+1)][n], two
    // work vectors, a zero vector, dot partial sums, coefficients
    double *kr_V = nullptr, *kr_w = nullptr, *kr_t = nullptr, *kr_zero = nullptr;
    double *kr_part = nullptr, *kr_coef = nullptr, *kr_host = nullptr;
    GmresState *kr_state = nullptr, *kr_state_host = nullptr;  // device cycle state, pinned mirror
    size_t kr_ld = 0;
    size_t ws_phi_slab = 0;
    unsigned long long *hist = nullptr;       // device, per-iteration stopping-test values
    unsigned long long *hist_host = nullptr;  // pinned
    int hist_cap = 0;
    EventTimer *timer = nullptr;              // null unless kernel timing is on
    // multi-slab FP64 solves in batched launches (built on first use), and
    // whether sn_solve uses them
    F64Batch *f64b = nullptr;
    bool batched_solve = true;
    // sweep tile autotuner of FP64 handles: the policy kept and the measured
    // time of one solve sweep per candidate (see set_tiling)
    int tile_choice = 0;
    double tile_ms[kTilePolicies] = {0.0, 0.0, 0.0};
    // exit-current tables: w_n mu_n for mu_n > 0 (zero for mu_n < 0) laid
    // out like psi_exit [sum N_b], and the slab offsets into it [slabs + 1]
    double *exit_wmu = nullptr;
    long long *exit_offs = nullptr;

    // builds exit_wmu / exit_offs from the descriptor's angle counts
    void build_exit_tables(const sn_problem_desc *d, hipStream_t st) {
        dvec wmu;
        std::vector<long long> offs(1, 0);
        for (int b = 0; b < d->num_slabs; ++b) {
            dvec mu, w;
            gauss_legendre(d->N[b], mu, w);
            for (int n = 0; n < d->N[b]; ++n) wmu.push_back(mu[n] > 0.0 ? w[n] * mu[n] : 0.0);
            offs.push_back(offs.back() + d->N[b]);
        }
        exit_wmu = upload(wmu, st);
        exit_offs = upload(offs, st);
    }

    template <typename T>
    T *dalloc(size_t count) {
        void *p = nullptr;
        if (count == 0) count = 1;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) throw std::bad_alloc();
        allocs.push_back(p);
        return static_cast<T *>(p);
    }
    template <typename T>
    T *upload(const std::vector<T> &v, hipStream_t st) {
        T *p = dalloc<T>(v.size());
        if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
        return p;
    }
    void release() {
        delete timer;
        timer = nullptr;
        if (f64b) {
            f64b->release();
            delete f64b;
            f64b = nullptr;
        }
        delete batch;
        batch = nullptr;
        for (void *p : allocs) (void)hipFree(p);
        allocs.clear();
        if (hist) (void)hipFree(hist);
        hist = nullptr;
        if (hist_host) (void)hipHostFree(hist_host);
        hist_host = nullptr;
        hist_cap = 0;
        if (kr_host) (void)hipHostFree(kr_host);
        kr_host = nullptr;
        if (kr_state_host) (void)hipHostFree(kr_state_host);
        kr_state_host = nullptr;
        for (Workspace &w : ws) {
            if (w.hist) (void)hipFree(w.hist);
            if (w.hist_host) (void)hipHostFree(w.hist_host);
            if (w.stream) (void)hipStreamDestroy(w.stream);
            if (w.done) (void)hipEventDestroy(w.done);
        }
        ws.clear();
        if (ev_order) (void)hipEventDestroy(ev_order);
        ev_order = nullptr;
    }
    // per-iteration history buffers, grown on demand (synchronises the device)
    void ensure_hist(Workspace &w, int n) {
        if (n <= w.hist_cap) return;
        (void)hipDeviceSynchronize();
        if (w.hist) (void)hipFree(w.hist);
        if (w.hist_host) (void)hipHostFree(w.hist_host);
        w.hist = nullptr;
        w.hist_host = nullptr;
        w.hist_cap = 0;
        HIPCHK(hipMalloc((void **)&w.hist, (size_t)n * sizeof(unsigned long long)));
        HIPCHK(hipHostMalloc((void **)&w.hist_host, (size_t)n * sizeof(unsigned long long), hipHostMallocDefault));
        w.hist_cap = n;
    }
    void ensure_hist(int n) {
        if (n <= hist_cap) return;
        (void)hipDeviceSynchronize();
        if (hist) (void)hipFree(hist);
        if (hist_host) (void)hipHostFree(hist_host);
        hist = nullptr;
        hist_host = nullptr;
        hist_cap = 0;
        HIPCHK(hipMalloc((void **)&hist, (size_t)n * sizeof(unsigned long long)));
        HIPCHK(hipHostMalloc((void **)&hist_host, (size_t)n * sizeof(unsigned long long), hipHostMallocDefault));
        hist_cap = n;
    }
};

namespace {

bool finite_all(const double *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

sn_status check_handle(sn_handle h) {
    if (!h) return fail(SN_E_STATE, "NULL handle");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SN_E_HIP, "hipGetDevice failed");
    if (dev != h->device) return fail(SN_E_STATE, "current device differs from the handle's device");
    return SN_OK;
}

SweepArgs sweep_args(const Workspace &W, const Slab &b, const double *q, double *psi, bool with_bc,
                     SkipTest skip = SkipTest()) {
    SweepArgs a;
    a.K = b.K; a.N = b.N; a.TC = b.TC; a.S = b.S; a.sub = b.sub; a.ntiles = b.ntiles;
    a.q = q; a.psi = psi;
    a.h = b.h; a.sigma_t = b.sigma_t; a.mu = b.mu; a.inv_absmu = b.inv_absmu;
    a.psi_left = with_bc ? b.psi_left : nullptr;
    a.psi_right = with_bc ? b.psi_right : nullptr;
    a.subA = W.subA; a.subB = W.subB; a.tileA = W.tileA; a.tileB = W.tileB;
    a.carry = W.carry; a.exit = W.sweep_exit;
    a.grpA = W.grpA; a.grpB = W.grpB;
    a.skip = skip;
    return a;
}

// phi [2K][L+1] = psi [2K][N] x Vt [N][L+1]
struct FusedStop {
    const double *ref = nullptr;
    unsigned long long *slot = nullptr;
};

void set_stop(GemmArgs &g, const FusedStop *fs) {
    if (!fs) return;
    g.stop_ref = fs->ref;
    g.stop_slot = fs->slot;
}

GemmArgs moments_args(const Slab &b, const double *psi, double *phi, SkipTest skip = SkipTest(),
                      const FusedStop *fs = nullptr) {
    GemmArgs g;
    g.skip = skip;
    set_stop(g, fs);
    g.rows = 2 * b.K; g.ncols = b.L1;
    g.A1 = psi; g.lda1 = b.N; g.k1 = b.N;
    g.B1 = b.Vt;
    g.C = phi; g.ldc = b.L1;
    return g;
}

void moments(const Slab &b, const double *psi, double *phi, hipStream_t st, KernelTimer *tm,
             SkipTest skip = SkipTest(), const FusedStop *fs = nullptr) {
    launch_gemm(moments_args(b, psi, phi, skip, fs), st, tm);
}

// q [2K][N] = (phi .* sigma_s) [2K][L+1] x Mt [L+1][N] + q_ext
GemmArgs scatter_args(const Slab &b, const double *phi, const double *qext, double *q, SkipTest skip = SkipTest()) {
    GemmArgs g;
    g.skip = skip;
    g.rows = 2 * b.K; g.ncols = b.N;
    g.A1 = phi; g.lda1 = b.L1; g.k1 = b.L1;
    g.S = b.sigma_s; g.s_div = 2; g.lds = b.L1;
    g.B1 = b.Mt;
    g.Cin = qext; g.ldcin = b.N;
    g.C = q; g.ldc = b.N;
    return g;
}

void scatter(const Slab &b, const double *phi, const double *qext, double *q, hipStream_t st,
             KernelTimer *tm, SkipTest skip = SkipTest()) {
    launch_gemm(scatter_args(b, phi, qext, q, skip), st, tm);
}

// The kernels of one slab's correction phi_new = phi_half + D F^{-1} S
// (phi_half - phi_old): per cell-type segment the Fokker-Planck source
// s = (phi_half - phi_old) E (gemm_fp_source), the interface recurrences,
// and per segment the update (gemm_fp_update), which carries the stopping
// test when the slab has one segment.
GemmArgs fp_source_args(const Workspace &W, const Slab &b, const double *phi_half, const double *phi_old,
                        size_t sg, SkipTest skip) {
    const int L2 = 2 * b.L1, N = b.N;
    const size_t et = (size_t)L2 * N;
    const int j0 = b.seg_begin[sg], j1 = b.seg_begin[sg + 1], t = b.seg_type[sg];
    GemmArgs g;
    g.skip = skip;
    g.rows = j1 - j0; g.ncols = N;
    g.A1 = phi_half + (size_t)j0 * L2; g.A1sub = phi_old + (size_t)j0 * L2;
    g.lda1 = L2; g.k1 = L2;
    if (!b.fold_ss) {
        g.S = b.sigma_s2 + (size_t)j0 * L2; g.s_div = 1; g.lds = L2;
    }
    g.B1 = b.EsrcT + t * et;
    g.C = W.s + (size_t)j0 * N; g.ldc = N;
    g.kid = KID_GEMM_FP_SOURCE;
    return g;
}

FPArgs fp_args(const Workspace &W, const Slab &b, SkipTest skip) {
    FPArgs f;
    f.K = b.K; f.NH = b.NH; f.chunk = b.chunk; f.nchunks = b.nchunks;
    f.cellmats = b.cellmats;
    f.psi_fwd = b.psi_fwd; f.psi_bwd = b.psi_bwd;
    f.theta_fwd = b.theta_fwd; f.theta_bwd = b.theta_bwd;
    f.part_f = W.part_f; f.part_b = W.part_b;
    f.carry_parts = fp_carry_parts(b.nchunks, b.NH);
    f.s = W.s; f.pvec = W.pvec; f.inflow = W.inflow;
    f.fvec = W.fvec; f.gvec = W.gvec; f.bvec = W.bvec;
    f.e_fwd = W.e_fwd; f.e_bwd = W.e_bwd;
    f.skip = skip;
    return f;
}

GemmArgs fp_update_args(const Workspace &W, const Slab &b, const double *phi_half, const double *phi_old,
                        double *phi_new, size_t sg, SkipTest skip, const FusedStop *fs) {
    const int L2 = 2 * b.L1, N = b.N;
    const size_t pt = (size_t)L2 * L2, it = (size_t)N * L2;
    const int j0 = b.seg_begin[sg], j1 = b.seg_begin[sg + 1], t = b.seg_type[sg];
    GemmArgs g;
    g.skip = skip;
    g.rows = j1 - j0; g.ncols = L2;
    g.A1 = phi_half + (size_t)j0 * L2; g.A1sub = phi_old + (size_t)j0 * L2;
    g.lda1 = L2; g.k1 = L2;
    if (!b.fold_ss) {
        g.S = b.sigma_s2 + (size_t)j0 * L2; g.s_div = 1; g.lds = L2;
    }
    g.B1 = b.PhisrcT + t * pt;
    g.A2 = W.inflow + (size_t)j0 * N; g.lda2 = N; g.k2 = N;
    g.B2 = b.PhiinfT + t * it;
    g.Cin = phi_half + (size_t)j0 * L2; g.ldcin = L2;
    g.C = phi_new + (size_t)j0 * L2; g.ldc = L2;
    g.kid = KID_GEMM_FP_UPDATE;
    if (fs && b.seg_begin.size() == 2) {
        // single segment: the stopping test rides on the update GEMM
        FusedStop f2 = *fs;
        set_stop(g, &f2);
    }
    return g;
}

void correct(sn_handle H, const Workspace &W, const Slab &b, const double *phi_half, const double *phi_old,
             double *phi_new, hipStream_t st, SkipTest skip = SkipTest(),
             const FusedStop *fs = nullptr, bool timed = true) {
    KernelTimer *const tm = timed ? H->timer : nullptr;
    const int L2 = 2 * b.L1;
    FPArgs f = fp_args(W, b, skip);
    if (b.seg_begin.size() == 2 && fp_fusable(b.NH, L2)) {
        // one cell type: the source GEMM rides on the additive-term kernel
        const int t = b.seg_type[0];
        f.L2 = L2;
        f.src_half = phi_half;
        f.src_old = phi_old;
        f.src_sigma = b.fold_ss ? nullptr : b.sigma_s2;
        f.src_E = b.EsrcT + (size_t)t * L2 * b.N;
    } else {
        for (size_t sg = 0; sg + 1 < b.seg_begin.size(); ++sg)
            launch_gemm(fp_source_args(W, b, phi_half, phi_old, sg, skip), st, tm);
    }
    launch_fp_recurrences(f, st, tm);
    for (size_t sg = 0; sg + 1 < b.seg_begin.size(); ++sg)
        launch_gemm(fp_update_args(W, b, phi_half, phi_old, phi_new, sg, skip, fs), st, tm);
}

}  // namespace

// Per-slab workspaces of the batched solve in one allocation (256-byte
// aligned sub-arrays), or SN_E_NOMEM when they exceed the budget (half the
// free device memory, at most 32 GiB); the caller then solves slab by slab.
static sn_status f64_batch_workspace(sn_handle h) {
    if (h->f64b) return SN_OK;
    const size_t ns = h->slabs.size();
    std::vector<size_t> offs;
    size_t total = 0;
    auto take = [&](size_t n) {
        offs.push_back(total);
        total += ((n + 31) & ~(size_t)31) * sizeof(double);
    };
    take((size_t)h->phi_len);  // phiA
    take((size_t)h->phi_len);  // phiB
    take((size_t)h->phi_len);  // phi_half
    for (const Slab &b : h->slabs) {
        const size_t K = b.K, N = b.N, NH = b.NH, P = (size_t)b.nchunks;
        const size_t parts = (size_t)fp_carry_parts(b.nchunks, b.NH);
        const size_t nt = (size_t)b.ntiles;
        take(K * 2 * N);                                            // q
        take(sweep_fusable(b.N, b.L1, b.TC) ? 0 : K * 2 * N);       // psi (unfused slabs)
        take(K * N);                                                // s
        take(K * N);                                                // inflow
        for (int i = 0; i < 4; ++i) take((K + 1) * NH);             // pvec, bvec, fvec, gvec
        take((P + 1) * NH);                                         // e_fwd
        take((P + 1) * NH);                                         // e_bwd
        take((P + 1) * parts * NH);                                 // part_f
        take((P + 1) * parts * NH);                                 // part_b
        take(nt * b.S * N);                                         // subA
        take(nt * b.S * N);                                         // subB
        take(nt * N);                                               // tileA
        take(nt * N);                                               // tileB
        take(nt * N);                                               // carry
        take(((nt + 63) / 64) * N);                                 // grpA
        take(((nt + 63) / 64) * N);                                 // grpB
        take(N);                                                    // sweep_exit
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
    if (total > std::min<size_t>(free_b / 2, (size_t)32 << 30)) return SN_E_NOMEM;
    F64Batch *B = new (std::nothrow) F64Batch();
    if (!B) return SN_E_NOMEM;
    if (hipMalloc(&B->mem, total) != hipSuccess || hipMalloc((void **)&B->iter, sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        B->release();
        delete B;
        return SN_E_NOMEM;
    }
    char *base = static_cast<char *>(B->mem);
    size_t k = 0;
    auto next = [&]() { return reinterpret_cast<double *>(base + offs[k++]); };
    B->phiA = next();
    B->phiB = next();
    B->phi_half = next();
    B->ws.resize(ns);
    for (size_t i = 0; i < ns; ++i) {
        const Slab &b = h->slabs[i];
        Workspace &W = B->ws[i];
        W.phiA = B->phiA + b.phi_off;
        W.phiB = B->phiB + b.phi_off;
        W.phi_half = B->phi_half + b.phi_off;
        W.q = next();
        W.psi = next();
        W.s = next();
        W.inflow = next();
        W.pvec = next();
        W.bvec = next();
        W.fvec = next();
        W.gvec = next();
        W.e_fwd = next();
        W.e_bwd = next();
        W.part_f = next();
        W.part_b = next();
        W.subA = next();
        W.subB = next();
        W.tileA = next();
        W.tileB = next();
        W.carry = next();
        W.grpA = next();
        W.grpB = next();
        W.sweep_exit = next();
    }
    h->f64b = B;
    return SN_OK;
}

// Descriptors of one iteration of every slab, grouped into launches.
template <class A>
static void plan_group(const std::vector<const PlanItem *> &items, const A PlanItem::*field,
                       std::vector<char> &blob, std::vector<std::pair<size_t, size_t>> &where,
                       std::vector<MultiLaunch> &out) {
    // entries in key order; blocks interleaved across entries
    std::vector<const PlanItem *> v(items);
    std::stable_sort(v.begin(), v.end(), [](const PlanItem *a, const PlanItem *b) { return a->order < b->order; });
    std::vector<MultiEntry<A>> ent(v.size());
    int maxb = 0;
    unsigned lds = 0;
    for (size_t i = 0; i < v.size(); ++i) {
        ent[i].a = v[i]->*field;
        ent[i].p = v[i]->p;
        ent[i].gx = v[i]->sh.gx;
        ent[i].flag = v[i]->sh.v2;
        maxb = std::max(maxb, v[i]->sh.gx * v[i]->sh.gy);
        lds = std::max(lds, v[i]->sh.lds);
    }
    std::vector<BlockRef> refs;
    for (int local = 0; local < maxb; ++local)
        for (size_t i = 0; i < v.size(); ++i)
            if (local < v[i]->sh.gx * v[i]->sh.gy) refs.push_back(BlockRef{(int)i, local});
    auto put = [&](const void *p, size_t n) {
        const size_t off = (blob.size() + 255) & ~(size_t)255;
        blob.resize(off + n);
        std::memcpy(blob.data() + off, p, n);
        return off;
    };
    MultiLaunch L;
    L.shape = v[0]->sh;
    L.nblocks = (int)refs.size();
    L.lds = lds;
    const size_t e_off = put(ent.data(), ent.size() * sizeof(MultiEntry<A>));
    const size_t r_off = put(refs.data(), refs.size() * sizeof(BlockRef));
    where.emplace_back(e_off, r_off);
    out.push_back(L);
}

static sn_status f64_plan(sn_handle h, int method, const double *q_ext, bool problem_bc, double tol,
                          F64Plan **out) {
    F64Batch &B = *h->f64b;
    for (size_t e = 0; e < B.plans.size(); ++e) {
        const F64Plan &p = B.plans[e];
        if (p.method == method && p.qext == q_ext && p.bc == problem_bc && p.hist == h->hist && p.tol == tol) {
            std::rotate(B.plans.begin() + e, B.plans.begin() + e + 1, B.plans.end());
            *out = &B.plans.back();
            return SN_OK;
        }
    }
    const int ns = (int)h->slabs.size();
    // slabs sharing one factorisation (same factor arrays and sizes; padded
    // half-width <= 64) run their recurrences as groups of at most
    // kFPGroupMax slabs
    std::vector<int> group_of(ns, -1);
    std::vector<std::vector<int>> groups;
    if (method == SN_FPSA) {
        std::map<std::tuple<const double *, const double *, int, int, int>, std::vector<int>> by_key;
        for (int bi = 0; bi < ns; ++bi) {
            const Slab &b = h->slabs[bi];
            if (b.NH > 64) continue;
            by_key[std::make_tuple((const double *)b.cellmats, (const double *)b.psi_fwd, b.K, b.NH, b.chunk)]
                .push_back(bi);
        }
        for (auto &kv : by_key) {
            if (kv.second.size() < 2) continue;
            const size_t cap = kFPGroupMax;
            for (size_t i0 = 0; i0 < kv.second.size(); i0 += cap) {
                std::vector<int> grp(kv.second.begin() + i0, kv.second.begin() + std::min(kv.second.size(), i0 + cap));
                if (grp.size() < 2) continue;
                for (int bi : grp) group_of[bi] = (int)groups.size();
                groups.push_back(std::move(grp));
            }
        }
    }
    std::vector<FPSlabVecs> vecs;
    std::vector<PlanItem> items;
    items.reserve((size_t)ns * 16);
    std::vector<int> phase;
    auto add = [&](int ph, const PlanItem &it) {
        items.push_back(it);
        phase.push_back(ph);
    };
    for (int bi = 0; bi < ns; ++bi) {
        const Slab &b = h->slabs[bi];
        const Workspace &W = B.ws[bi];
        const double *qe = q_ext ? q_ext + b.psi_off : nullptr;
        const size_t nphi = (size_t)b.K * 2 * b.L1;
        IterPatch base;
        base.phiA = W.phiA;
        base.phiB = W.phiB;
        base.hist = h->hist + bi;
        base.hist_stride = ns;
        base.flags = PATCH_SKIP;
        // placeholders for the iteration-relative pointers (the kernels
        // replace them): the first iteration's, so that every shape decision
        // sees the fields it tests
        double *cur = W.phiA, *nxt = W.phiB;
        unsigned long long *slot = h->hist + bi;
        const bool fuse = sweep_fusable(b.N, b.L1, b.TC);
        if (!fuse) {
            PlanItem it;
            it.kind = 0;
            it.g = scatter_args(b, cur, qe, W.q);
            it.sh = gemm_shape(it.g);
            it.p = base;
            it.p.flags |= PATCH_A1_CUR;
            it.order = (uintptr_t)bi;
            add(PH_SCATTER, it);
        }
        {
            SweepArgs a = sweep_args(W, b, W.q, W.psi, problem_bc);
            PlanItem it;
            it.kind = 1;
            it.p = base;
            if (fuse) {
                a.src_phi = cur; a.src_sigma_s = b.sigma_s; a.src_Mt = b.Mt; a.src_qext = qe;
                a.q_out = W.q; a.L1 = b.L1;
                a.mom_Vt = b.Vt; a.write_psi = false;
                it.p.flags |= PATCH_SRC_CUR;
                if (method == SN_FPSA) {
                    a.mom_out = W.phi_half;
                } else {
                    a.mom_out = nxt; a.mom_ref = cur; a.mom_slot = slot;
                    it.p.flags |= PATCH_MOM_NXT | PATCH_MOM_STOP;
                }
            }
            it.sw = a;
            it.order = (uintptr_t)bi;
            LaunchShape sh[4];
            const int n = sweep_shapes(a, sh);
            for (int i = 0; i < n; ++i) {
                it.sh = sh[i];
                add(sh[i].kernel == MK_SWEEP_AGG ? PH_SWEEP_AGG
                    : sh[i].kernel == MK_SCAN_GROUPS ? PH_SCAN_GROUPS
                    : sh[i].kernel == MK_SCAN_CARRY ? PH_SCAN_CARRY : PH_SWEEP_APPLY, it);
            }
        }
        if (!fuse) {
            PlanItem it;
            it.kind = 0;
            it.p = base;
            if (method == SN_FPSA) {
                it.g = moments_args(b, W.psi, W.phi_half);
            } else {
                FusedStop fs;
                fs.ref = cur;
                fs.slot = slot;
                it.g = moments_args(b, W.psi, nxt, SkipTest(), &fs);
                it.p.flags |= PATCH_C_NXT | PATCH_STOP;
            }
            it.sh = gemm_shape(it.g);
            it.order = (uintptr_t)bi;
            add(PH_MOMENTS, it);
        }
        if (method != SN_FPSA) continue;
        const bool single = b.seg_begin.size() == 2;
        for (size_t sg = 0; sg + 1 < b.seg_begin.size(); ++sg) {
            PlanItem it;
            it.kind = 0;
            it.g = fp_source_args(W, b, W.phi_half, cur, sg, SkipTest());
            it.sh = gemm_shape(it.g);
            it.p = base;
            it.p.flags |= PATCH_A1SUB_CUR;
            it.p.off = (long long)b.seg_begin[sg] * 2 * b.L1;
            it.order = (uintptr_t)bi;
            add(PH_FP_SOURCE, it);
        }
        if (group_of[bi] < 0) {
            PlanItem it;
            it.kind = 2;
            it.f = fp_args(W, b, SkipTest());
            it.p = base;
            it.order = (uintptr_t)b.cellmats;  // slabs sharing factors side by side
            LaunchShape sh[4];
            fp_shapes(it.f, sh);
            const int ph[4] = {PH_FP_MATVEC, PH_FP_CHAIN, PH_FP_CARRY, PH_FP_FIXUP};
            for (int i = 0; i < 4; ++i) {
                it.sh = sh[i];
                add(ph[i], it);
            }
        } else if (groups[group_of[bi]][0] == bi) {
            // the group's recurrences, emitted with its first slab
            const std::vector<int> &grp = groups[group_of[bi]];
            PlanItem it;
            it.kind = 4;
            it.fg.f = fp_args(W, b, SkipTest());
            it.fg.nslab = (int)grp.size();
            it.fg.hist_stride = ns;
            it.fg.tol = tol;
            it.vec_off = vecs.size();
            for (int sb : grp) {
                const Workspace &V = B.ws[sb];
                FPSlabVecs v;
                v.s = V.s; v.fvec = V.fvec; v.gvec = V.gvec; v.pvec = V.pvec; v.bvec = V.bvec; v.inflow = V.inflow;
                v.e_fwd = V.e_fwd; v.e_bwd = V.e_bwd; v.part_f = V.part_f; v.part_b = V.part_b;
                v.hist = h->hist + sb;
                vecs.push_back(v);
            }
            it.p = base;
            it.p.flags = 0;
            it.order = (uintptr_t)bi;
            LaunchShape sh[4];
            fp_group_shapes(it.fg.f, sh);
            const int ph[4] = {PH_FP_MATVEC, PH_FP_CHAIN, PH_FP_CARRY, PH_FP_FIXUP};
            for (int i = 0; i < 4; ++i) {
                it.sh = sh[i];
                add(ph[i], it);
            }
        }
        for (size_t sg = 0; sg + 1 < b.seg_begin.size(); ++sg) {
            FusedStop fs;
            fs.ref = cur;
            fs.slot = slot;
            PlanItem it;
            it.kind = 0;
            it.g = fp_update_args(W, b, W.phi_half, cur, nxt, sg, SkipTest(), &fs);
            it.sh = gemm_shape(it.g);
            it.p = base;
            it.p.flags |= PATCH_A1SUB_CUR | PATCH_C_NXT | (single ? PATCH_STOP : 0u);
            it.p.off = (long long)b.seg_begin[sg] * 2 * b.L1;
            it.order = (uintptr_t)bi;
            add(PH_FP_UPDATE, it);
        }
        if (!single) {
            PlanItem it;
            it.kind = 3;
            it.st.a = nxt;
            it.st.b = cur;
            it.st.n = nphi;
            it.st.slot = slot;
            it.sh = stop_shape(nphi);
            it.p = base;
            it.p.flags |= PATCH_STOPTEST;
            it.order = (uintptr_t)bi;
            add(PH_STOP, it);
        }
    }
    // group by phase and kernel variant
    F64Plan plan;
    plan.method = method;
    plan.qext = q_ext;
    plan.bc = problem_bc;
    plan.hist = h->hist;
    plan.tol = tol;
    if (!vecs.empty()) {
        if (hipMalloc(&plan.dev2, vecs.size() * sizeof(FPSlabVecs)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SN_E_NOMEM, "device allocation of the batched solve's vector tables failed");
        }
        if (hipMemcpy(plan.dev2, vecs.data(), vecs.size() * sizeof(FPSlabVecs), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(plan.dev2);
            return fail(SN_E_HIP, "copying the batched solve's vector tables failed");
        }
        for (PlanItem &it : items)
            if (it.kind == 4) it.fg.v = static_cast<const FPSlabVecs *>(plan.dev2) + it.vec_off;
    }
    std::vector<char> blob;
    std::vector<std::pair<size_t, size_t>> where;
    for (int ph = 0; ph < PH_COUNT; ++ph) {
        std::map<std::tuple<int, int, int, int>, std::vector<const PlanItem *>> groups;
        for (size_t i = 0; i < items.size(); ++i) {
            if (phase[i] != ph) continue;
            const LaunchShape &s = items[i].sh;
            if (s.gx * s.gy <= 0) continue;
            groups[std::make_tuple(s.kernel, s.v1, s.v2, s.block)].push_back(&items[i]);
        }
        for (auto &kv : groups) {
            switch (kv.second[0]->kind) {
                case 0: plan_group(kv.second, &PlanItem::g, blob, where, plan.launches); break;
                case 1: plan_group(kv.second, &PlanItem::sw, blob, where, plan.launches); break;
                case 2: plan_group(kv.second, &PlanItem::f, blob, where, plan.launches); break;
                case 4: plan_group(kv.second, &PlanItem::fg, blob, where, plan.launches); break;
                default: plan_group(kv.second, &PlanItem::st, blob, where, plan.launches); break;
            }
        }
    }
    if (hipMalloc(&plan.dev, std::max<size_t>(blob.size(), 1)) != hipSuccess) {
        (void)hipGetLastError();
        F64Batch::drop(plan);
        return fail(SN_E_NOMEM, "device allocation of the batched solve's launch tables failed");
    }
    if (hipMemcpy(plan.dev, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
        F64Batch::drop(plan);
        return fail(SN_E_HIP, "copying the batched solve's launch tables failed");
    }
    for (size_t i = 0; i < plan.launches.size(); ++i) {
        plan.launches[i].entries = static_cast<char *>(plan.dev) + where[i].first;
        plan.launches[i].refs = reinterpret_cast<const BlockRef *>(static_cast<char *>(plan.dev) + where[i].second);
    }
    if (B.plans.size() == F64Batch::kPlans) {
        F64Batch::drop(B.plans.front());
        B.plans.erase(B.plans.begin());
    }
    B.plans.push_back(std::move(plan));
    *out = &B.plans.back();
    return SN_OK;
}

// SI / FPSA of every slab of a multi-slab FP64 handle in batched launches;
// same arguments and results as the slab-by-slab path of solve_impl.
static sn_status solve_batched_f64(sn_handle h, int32_t method, double tol, int32_t max_iter, const double *q_ext,
                                   double *phi, double *psi_exit, int32_t *iters, double *resid_hist,
                                   hipStream_t st, bool problem_bc) {
    const int ns = (int)h->slabs.size();
    F64Batch &B = *h->f64b;
    F64Plan *plan = nullptr;
    try {
        h->ensure_hist(kHistRing * ns);
    } catch (const HipError &e) {
        return fail(SN_E_HIP, std::string("HIP error in ") + e.where + ": " + hipGetErrorString(e.e));
    }
    sn_status ps = f64_plan(h, method, q_ext, problem_bc, tol, &plan);
    if (ps != SN_OK) return ps;
    std::vector<int> its(ns, 0);
    std::vector<char> bad(ns, 0);
    try {
        HIPCHK(hipMemcpyAsync(B.phiA, phi, (size_t)h->phi_len * sizeof(double), hipMemcpyDeviceToDevice, st));
        static const int one = 1;
        HIPCHK(hipMemcpyAsync(B.iter, &one, sizeof(int), hipMemcpyHostToDevice, st));
        // with kernel timing off, one iteration is captured into a graph
        // (once per plan) and replayed on the handle's stream
        const bool graph = h->timer == nullptr;
        hipStream_t rs = st;
        if (graph) {
            if (!B.gstream) {
                HIPCHK(hipStreamCreateWithFlags(&B.gstream, hipStreamNonBlocking));
                HIPCHK(hipEventCreateWithFlags(&B.gev, hipEventDisableTiming));
            }
            rs = B.gstream;
            HIPCHK(hipEventRecord(B.gev, st));
            HIPCHK(hipStreamWaitEvent(rs, B.gev, 0));
            if (!plan->exec) {
                hipGraph_t gr = nullptr;
                HIPCHK(hipStreamBeginCapture(rs, hipStreamCaptureModeThreadLocal));
                for (const MultiLaunch &L : plan->launches) launch_multi(L, B.iter, rs, nullptr);
                launch_iter_step(B.iter, rs);
                const hipError_t ec = hipStreamEndCapture(rs, &gr);
                if (ec != hipSuccess) {
                    if (gr) (void)hipGraphDestroy(gr);
                    HIPCHK(ec);
                }
                const hipError_t ei = hipGraphInstantiate(&plan->exec, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                HIPCHK(ei);
            }
        }
        int remaining = ns, launched = 0, batch = 2;
        auto passes = [&](double v) { return v <= tol || !std::isfinite(v); };
        // ring rows of iterations m0 + 1 .. m0 + nb as at most two row ranges
        auto ring_ranges = [&](int m0, int nb, auto &&fn) {
            const int r0 = (int)hist_row(m0 + 1);
            const int c0 = std::min(nb, kHistRing - r0);
            fn(r0, c0);
            if (nb > c0) fn(0, nb - c0);
        };
        while (launched < max_iter && remaining > 0) {
            const int nb = std::min(batch, max_iter - launched);
            ring_ranges(launched, nb, [&](int r, int c) {
                HIPCHK(hipMemsetAsync(h->hist + (size_t)r * ns, 0, (size_t)c * ns * sizeof(unsigned long long), rs));
            });
            for (int i = 0; i < nb; ++i) {
                if (graph) {
                    HIPCHK(hipGraphLaunch(plan->exec, rs));
                    continue;
                }
                for (const MultiLaunch &L : plan->launches) launch_multi(L, B.iter, rs, h->timer);
                launch_iter_step(B.iter, rs);
            }
            ring_ranges(launched, nb, [&](int r, int c) {
                HIPCHK(hipMemcpyAsync(h->hist_host + (size_t)r * ns, h->hist + (size_t)r * ns,
                                      (size_t)c * ns * sizeof(unsigned long long), hipMemcpyDeviceToHost, rs));
            });
            HIPCHK(hipStreamSynchronize(rs));
            for (int b = 0; b < ns; ++b) {
                if (its[b]) continue;
                for (int i = 0; i < nb; ++i) {
                    double v;
                    std::memcpy(&v, &h->hist_host[hist_row(launched + i + 1) * ns + b], sizeof(double));
                    if (resid_hist) resid_hist[(size_t)b * max_iter + launched + i] = v;
                    if (passes(v)) {
                        its[b] = launched + i + 1;
                        bad[b] = !std::isfinite(v);
                        --remaining;
                        break;
                    }
                }
            }
            launched += nb;
            batch = std::min(2 * batch, kHistBatch);
        }
        if (rs != st) {
            HIPCHK(hipEventRecord(B.gev, rs));
            HIPCHK(hipStreamWaitEvent(st, B.gev, 0));
        }
        sn_status result = SN_OK;
        for (int b = 0; b < ns; ++b) {
            const Slab &sl = h->slabs[b];
            const Workspace &W = B.ws[b];
            if (!its[b]) {
                its[b] = max_iter;
                result = SN_NOT_CONVERGED;
            }
            iters[b] = its[b];
            const double *fin = (its[b] & 1) ? W.phiB : W.phiA;
            HIPCHK(hipMemcpyAsync(phi + sl.phi_off, fin, (size_t)sl.K * 2 * sl.L1 * sizeof(double),
                                  hipMemcpyDeviceToDevice, st));
            if (psi_exit)
                launch_exit_flux(sl.N, W.sweep_exit, method == SN_FPSA ? W.bvec : nullptr,
                                 method == SN_FPSA ? W.pvec + (size_t)sl.K * sl.NH : nullptr, psi_exit + sl.exit_off,
                                 st, h->timer);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        for (int b = 0; b < ns; ++b)
            if (bad[b]) return fail(SN_E_NONFINITE, "non-finite stopping-test value in slab " + std::to_string(b));
        return result;
    } catch (const HipError &e) {
        // leave the graph stream usable after a failure inside a capture
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (B.gstream && hipStreamIsCapturing(B.gstream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
            hipGraph_t gr = nullptr;
            (void)hipStreamEndCapture(B.gstream, &gr);
            if (gr) (void)hipGraphDestroy(gr);
        }
        (void)hipGetLastError();
        return fail(SN_E_HIP, std::string("HIP error in ") + e.where + ": " + hipGetErrorString(e.e));
    }
}

// Sweep tile autotuner of an FP64 handle: every candidate tiling (set_tiling)
// is timed on the solve's sweep (fused source and moments where the slab
// takes them) of up to sixteen of the handle's slabs, one warm-up and three
// timed passes with HIP events, and the fastest is kept for every slab.
static void set_tiling_all(sn_handle H, int policy) {
    for (Slab &b : H->slabs) set_tiling(b, policy);
}

static void autotune_tiles(sn_handle H, hipStream_t st) {
    Workspace &W = H->ws[0];
    HIPCHK(hipMemsetAsync(W.phiA, 0, H->ws_phi_slab * sizeof(double), st));
    const int nmeas = std::min<int>(16, (int)H->slabs.size());
    auto run = [&]() {
        for (int bi = 0; bi < nmeas; ++bi) {
            const Slab &b = H->slabs[bi];
            SweepArgs a = sweep_args(W, b, W.q, W.psi, true);
            if (sweep_fusable(b.N, b.L1, b.TC)) {
                a.src_phi = W.phiA; a.src_sigma_s = b.sigma_s; a.src_Mt = b.Mt; a.src_qext = nullptr;
                a.q_out = W.q; a.L1 = b.L1;
                a.mom_Vt = b.Vt; a.write_psi = false; a.mom_out = W.phi_half;
                launch_sweep(a, false, st, nullptr);
            } else {
                scatter(b, W.phiA, nullptr, W.q, st, nullptr);
                launch_sweep(a, false, st, nullptr);
                moments(b, W.psi, W.phi_half, st, nullptr);
            }
        }
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        throw HipError{hipErrorOutOfMemory, "hipEventCreate"};
    }
    int best = 0;
    hipError_t err = hipSuccess;
    for (int pol = 0; pol < kTilePolicies && err == hipSuccess; ++pol) {
        set_tiling_all(H, pol);
        run();
        err = hipEventRecord(e0, st);
        for (int rep = 0; rep < 3; ++rep) run();
        if (err == hipSuccess) err = hipEventRecord(e1, st);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        H->tile_ms[pol] = ms / 3.0;
        if (H->tile_ms[pol] < H->tile_ms[best]) best = pol;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(err);
    HIPCHK(hipGetLastError());
    H->tile_choice = best;
    set_tiling_all(H, best);
}

// ===========================================================================
extern "C" {

const char *sn_last_error(void) { return g_err.c_str(); }

sn_status sn_setup(const sn_problem_desc *d, void *stream, sn_handle *out) {
    g_err.clear();
    if (!d || !out) return fail(SN_E_INVALID, "NULL descriptor or output pointer");
    *out = nullptr;
    if (d->num_slabs < 1) return fail(SN_E_INVALID, "num_slabs must be >= 1");
    if (!d->K || !d->N || !d->L || !d->h || !d->sigma_t || !d->sigma_s)
        return fail(SN_E_INVALID, "descriptor arrays K, N, L, h, sigma_t, sigma_s are required");
    if (d->fp_scheme != SN_FP_WFD && d->fp_scheme != SN_FP_MPD && d->fp_scheme != SN_FP_NONE)
        return fail(SN_E_INVALID, "fp_scheme must be SN_FP_WFD, SN_FP_MPD or SN_FP_NONE");
    if (d->precision != SN_F64 && d->precision != SN_F32 && d->precision != SN_BF16X3)
        return fail(SN_E_INVALID, "precision must be SN_F64, SN_F32 or SN_BF16X3");
    if (d->fp_coefficients != SN_FP_CELL && d->fp_coefficients != SN_FP_MEAN)
        return fail(SN_E_INVALID, "fp_coefficients must be SN_FP_CELL or SN_FP_MEAN");
    int64_t cells = 0, sslen = 0, halves = 0;
    for (int b = 0; b < d->num_slabs; ++b) {
        const int K = d->K[b], N = d->N[b], L = d->L[b];
        if (K < 1) return fail(SN_E_INVALID, "slab " + std::to_string(b) + ": K must be >= 1");
        if (N < 2 || N % 2 || N > 256)
            return fail(SN_E_INVALID, "slab " + std::to_string(b) + ": N must be even, 2 <= N <= 256");
        if (L < 0 || L >= N)
            return fail(SN_E_INVALID, "slab " + std::to_string(b) + ": need 0 <= L <= N-1");
        cells += K;
        sslen += (int64_t)K * (L + 1);
        halves += N / 2;
    }
    if (!finite_all(d->h, cells) || !finite_all(d->sigma_t, cells) || !finite_all(d->sigma_s, sslen) ||
        (d->psi_left && !finite_all(d->psi_left, halves)) ||
        (d->psi_right && !finite_all(d->psi_right, halves)))
        return fail(SN_E_NONFINITE, "non-finite value in the problem description");
    {
        int64_t c = 0, so = 0;
        for (int b = 0; b < d->num_slabs; ++b) {
            const int L1 = d->L[b] + 1;
            for (int j = 0; j < d->K[b]; ++j, ++c) {
                const double *ss = d->sigma_s + so + (int64_t)j * L1;
                if (!(d->h[c] > 0.0)) return fail(SN_E_INVALID, "cell width must be > 0");
                if (!(d->sigma_t[c] > 0.0)) return fail(SN_E_INVALID, "sigma_t must be > 0");
                if (d->sigma_t[c] - ss[0] < 0.0) return fail(SN_E_INVALID, "sigma_a = sigma_t - sigma_s0 must be >= 0");
                if (L1 > 1 && ss[0] - ss[1] < 0.0)
                    return fail(SN_E_INVALID, "sigma_tr = sigma_s0 - sigma_s1 must be >= 0");
            }
            so += (int64_t)d->K[b] * L1;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    sn_handle H = new (std::nothrow) sn_handle_s();
    if (!H) return fail(SN_E_NOMEM, "host allocation failed");
    try {
        HIPCHK(hipGetDevice(&H->device));
        HIPCHK(scratch_attach(H->device));  // the allocation-free entry point's scratch on this device
        H->fp_scheme = d->fp_scheme;
        H->precision = d->precision;
        H->has_fp = d->precision == SN_F64 && d->fp_scheme != SN_FP_NONE;
        if (d->precision != SN_F64) {
            // batched FP32 / split-BF16 handle: batch tables only
            std::string msg;
            const sn_status bs = batch_setup(d, st, &H->batch, msg);
            if (bs != SN_OK) {
                H->release();
                delete H;
                return fail(bs, msg);
            }
            for (int bi = 0; bi < d->num_slabs; ++bi) {
                Slab b;
                b.K = d->K[bi]; b.N = d->N[bi]; b.L = d->L[bi]; b.NH = b.N / 2; b.L1 = b.L + 1;
                H->slabs.push_back(b);
            }
            H->psi_len = H->batch->psi_len;
            H->phi_len = H->batch->phi_len;
            H->exit_len = H->batch->exit_len;
            H->build_exit_tables(d, st);
            HIPCHK(hipStreamSynchronize(st));
            *out = H;
            return SN_OK;
        }
        // SN_FP_MEAN: per slab the width-weighted means of sigma_a and
        // sigma_tr, rounded to two significant digits; slabs with equal
        // (K, N, L, widths, rounded means) share one factorisation.  The
        // distinct factorisations are computed up front on host threads.
        std::vector<std::vector<double>> mean_key(d->num_slabs);
        std::map<std::vector<double>, FPFactors> mean_factors;
        std::map<std::vector<double>, int> fp_cache;  // key -> first slab holding its device factors
        if (H->has_fp && d->fp_coefficients == SN_FP_MEAN) {
            auto round2 = [](double x) {
                if (!(x > 0.0)) return 0.0;
                const double e = std::pow(10.0, std::floor(std::log10(x)) - 1.0);
                return std::round(x / e) * e;
            };
            std::vector<std::pair<std::vector<double>, int64_t>> jobs;  // key, first cell
            int64_t cc = 0, ss = 0;
            for (int bi = 0; bi < d->num_slabs; ++bi) {
                const int K = d->K[bi], L1 = d->L[bi] + 1;
                double hs = 0.0, sa = 0.0, str = 0.0;
                for (int j = 0; j < K; ++j) {
                    const double *sr = d->sigma_s + ss + (int64_t)j * L1;
                    const double hh = d->h[cc + j];
                    sa += hh * (d->sigma_t[cc + j] - sr[0]);
                    str += hh * (sr[0] - (L1 > 1 ? sr[1] : 0.0));
                    hs += hh;
                }
                std::vector<double> key = {(double)K, (double)d->N[bi], (double)d->L[bi], round2(sa / hs),
                                           round2(str / hs)};
                key.insert(key.end(), d->h + cc, d->h + cc + K);
                if (mean_factors.find(key) == mean_factors.end()) {
                    mean_factors.emplace(key, FPFactors());
                    jobs.emplace_back(key, cc);
                }
                mean_key[bi] = std::move(key);
                cc += K;
                ss += (int64_t)K * L1;
            }
            std::atomic<int> next(0), failed(0);
            auto work = [&]() {
                for (int jb; (jb = next.fetch_add(1)) < (int)jobs.size();) {
                    const std::vector<double> &key = jobs[jb].first;
                    const int K = (int)key[0], N = (int)key[1], L = (int)key[2];
                    dvec mu, w;
                    gauss_legendre(N, mu, w);
                    const dvec A = (d->fp_scheme == SN_FP_WFD) ? wfd_laplacian(N, mu, w) : mpd_laplacian(N, mu, w);
                    const dvec sa(K, key[3]), str(K, key[4]);
                    if (!build_fp_factors_coef(K, N, L, d->h + jobs[jb].second, sa.data(), str.data(), nullptr, mu, w,
                                               A, mean_factors.at(key)))
                        failed.store(1);
                }
            };
            const int nthr = (int)std::min<size_t>(jobs.size(), std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
            std::vector<std::thread> pool;
            for (int t = 1; t < nthr; ++t) pool.emplace_back(work);
            work();
            for (std::thread &t : pool) t.join();
            if (failed.load()) {
                H->release();
                delete H;
                return fail(SN_E_INVALID, "Fokker-Planck operator with the slab-mean coefficients is singular");
            }
        }
        // per-cell factorisations of up to kFactorGroup slabs, computed together
        constexpr int kFactorGroup = 16;
        std::vector<FPFactors> group_factors(kFactorGroup);
        int64_t c = 0, so = 0, half = 0, psi_off = 0, phi_off = 0, exit_off = 0;
        size_t ws_q = 0, ws_phi = 0, ws_s = 0, ws_p = 0, ws_e = 0, ws_sub = 0, ws_tile = 0, ws_n = 0, ws_grp = 0;
        size_t ws_part = 0;
        for (int bi = 0; bi < d->num_slabs; ++bi) {
            Slab b;
            b.K = d->K[bi]; b.N = d->N[bi]; b.L = d->L[bi]; b.NH = b.N / 2; b.L1 = b.L + 1;
            b.cell_off = c; b.psi_off = psi_off; b.phi_off = phi_off; b.exit_off = exit_off;
            dvec mu, w;
            gauss_legendre(b.N, mu, w);
            dvec P = legendre_table(b.N, b.L, mu);
            dvec Mt((size_t)b.L1 * b.N), Vt((size_t)b.N * b.L1), inv(b.N);
            for (int l = 0; l < b.L1; ++l)
                for (int n = 0; n < b.N; ++n) {
                    Mt[(size_t)l * b.N + n] = 0.5 * (2 * l + 1) * P[(size_t)l * b.N + n];
                    Vt[(size_t)n * b.L1 + l] = w[n] * P[(size_t)l * b.N + n];
                }
            for (int n = 0; n < b.N; ++n) inv[n] = 1.0 / std::fabs(mu[n]);
            b.mu = H->upload(mu, st);
            b.inv_absmu = H->upload(inv, st);
            b.w = H->upload(w, st);
            b.Mt = H->upload(Mt, st);
            b.Vt = H->upload(Vt, st);
            b.h = H->upload(dvec(d->h + c, d->h + c + b.K), st);
            b.sigma_t = H->upload(dvec(d->sigma_t + c, d->sigma_t + c + b.K), st);
            b.sigma_s = H->upload(dvec(d->sigma_s + so, d->sigma_s + so + (int64_t)b.K * b.L1), st);
            b.psi_left = d->psi_left ? H->upload(dvec(d->psi_left + half, d->psi_left + half + b.NH), st) : nullptr;
            b.psi_right = d->psi_right ? H->upload(dvec(d->psi_right + half, d->psi_right + half + b.NH), st) : nullptr;
            if (H->has_fp) {
                const bool mean = d->fp_coefficients == SN_FP_MEAN;
                if (mean) {
                    auto it = fp_cache.find(mean_key[bi]);
                    if (it != fp_cache.end()) {
                        const Slab &o = H->slabs[it->second];
                        b.cellmats = o.cellmats; b.psi_fwd = o.psi_fwd; b.psi_bwd = o.psi_bwd;
                        b.theta_fwd = o.theta_fwd; b.theta_bwd = o.theta_bwd;
                        b.EsrcT = o.EsrcT; b.PhisrcT = o.PhisrcT; b.PhiinfT = o.PhiinfT;
                        b.seg_begin = o.seg_begin; b.seg_type = o.seg_type;
                        b.chunk = o.chunk; b.nchunks = o.nchunks;
                        b.fold_ss = false;
                    }
                    dvec s2((size_t)b.K * 2 * b.L1);
                    for (int j = 0; j < b.K; ++j)
                        for (int nu = 0; nu < 2; ++nu)
                            for (int l = 0; l < b.L1; ++l)
                                s2[((size_t)j * 2 + nu) * b.L1 + l] = d->sigma_s[so + (int64_t)j * b.L1 + l];
                    b.sigma_s2 = H->upload(s2, st);
                }
                if (!mean || !b.cellmats) {
                    // Fokker-Planck factorisation (FP64, host): per-cell
                    // coefficients are factored for a group of slabs at a
                    // time on host threads, so that only one group's host
                    // factors are held at once
                    FPFactors Fc;
                    if (!mean) {
                        if (bi % kFactorGroup == 0) {
                            const int g1 = std::min(d->num_slabs, bi + kFactorGroup);
                            std::vector<int64_t> cc(g1 - bi), ss(g1 - bi);
                            int64_t c2 = c, s2 = so;
                            for (int k = bi; k < g1; ++k) {
                                cc[k - bi] = c2;
                                ss[k - bi] = s2;
                                c2 += d->K[k];
                                s2 += (int64_t)d->K[k] * (d->L[k] + 1);
                            }
                            std::atomic<int> next(bi), failed(-1);
                            auto work = [&]() {
                                for (int k; (k = next.fetch_add(1)) < g1;) {
                                    const int N = d->N[k];
                                    dvec m2, w2;
                                    gauss_legendre(N, m2, w2);
                                    const dvec A = (d->fp_scheme == SN_FP_WFD) ? wfd_laplacian(N, m2, w2)
                                                                               : mpd_laplacian(N, m2, w2);
                                    if (!build_fp_factors(d->K[k], N, d->L[k], d->h + cc[k - bi], d->sigma_t + cc[k - bi],
                                                          d->sigma_s + ss[k - bi], m2, w2, A, group_factors[k - bi]))
                                        failed.store(k);
                                }
                            };
                            const int nthr = std::max(1, std::min(g1 - bi, (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
                            std::vector<std::thread> pool;
                            for (int t = 1; t < nthr; ++t) pool.emplace_back(work);
                            work();
                            for (std::thread &t : pool) t.join();
                            if (failed.load() >= 0) {
                                const int k = failed.load();
                                H->release();
                                delete H;
                                return fail(SN_E_INVALID, "Fokker-Planck operator is singular for slab " + std::to_string(k));
                            }
                        }
                        Fc = std::move(group_factors[bi % kFactorGroup]);
                        group_factors[bi % kFactorGroup] = FPFactors();
                    }
                    FPFactors &F = mean ? mean_factors.at(mean_key[bi]) : Fc;
                    b.fold_ss = F.folded_sigma_s;
                    if (mean) fp_cache.emplace(mean_key[bi], bi);
                    {
                        // device layout: all six matrices transposed, so that the
                        // threads of one cell (one per row) read consecutive addresses
                        // and a chain step's matrix copies verbatim into LDS
                        const size_t M2 = (size_t)b.NH * b.NH;
                        dvec dev(F.cellmats.size());
                        for (int j = 0; j < b.K; ++j)
                            for (int m = 0; m < FP_CELL_MATS; ++m) {
                                const double *src = &F.cellmats[((size_t)j * FP_CELL_MATS + m) * M2];
                                double *dst = &dev[((size_t)j * FP_CELL_MATS + m) * M2];
                                for (int r = 0; r < b.NH; ++r)
                                    for (int cc = 0; cc < b.NH; ++cc)
                                        dst[(size_t)cc * b.NH + r] = src[(size_t)r * b.NH + cc];
                            }
                        b.cellmats = H->upload(dev, st);
                    }
                    {
                        // prefix and transfer products, transposed per matrix
                        const size_t M2 = (size_t)b.NH * b.NH;
                        auto transposed = [&](const dvec &src) {
                            dvec dst(src.size());
                            for (size_t m = 0; m < src.size() / std::max<size_t>(M2, 1); ++m)
                                for (int r = 0; r < b.NH; ++r)
                                    for (int cc = 0; cc < b.NH; ++cc)
                                        dst[m * M2 + (size_t)cc * b.NH + r] = src[m * M2 + (size_t)r * b.NH + cc];
                            return dst;
                        };
                        b.psi_fwd = H->upload(transposed(F.psi_fwd), st);
                        b.psi_bwd = H->upload(transposed(F.psi_bwd), st);
                        b.theta_fwd = H->upload(transposed(F.theta_fwd), st);
                        b.theta_bwd = H->upload(transposed(F.theta_bwd), st);
                    }
                    b.EsrcT = H->upload(F.EsrcT, st);
                    b.PhisrcT = H->upload(F.PhisrcT, st);
                    b.PhiinfT = H->upload(F.PhiinfT, st);
                    b.seg_begin = F.seg_begin;
                    b.seg_type = F.seg_type;
                    b.chunk = F.chunk;
                    b.nchunks = F.nchunks;
                    if (mean) F = FPFactors();  // uploaded; the host copy is no longer needed
                }
            }
            // sweep tiling (the autotuner may change it below): the
            // workspace holds the tiles of every candidate
            size_t max_tiles = 0;
            for (int pol = kTilePolicies - 1; pol >= 0; --pol) {
                set_tiling(b, pol);
                max_tiles = std::max(max_tiles, (size_t)b.ntiles);
            }
            // workspace sizes
            ws_q = std::max(ws_q, (size_t)b.K * 2 * b.N);
            ws_phi = std::max(ws_phi, (size_t)b.K * 2 * b.L1);
            ws_s = std::max(ws_s, (size_t)b.K * b.N);
            ws_p = std::max(ws_p, (size_t)(b.K + 1) * b.NH);
            ws_e = std::max(ws_e, (size_t)(b.nchunks + 1) * b.NH);
            ws_part = std::max(ws_part, (size_t)(b.nchunks + 1) * fp_carry_parts(b.nchunks, b.NH) * b.NH);
            ws_sub = std::max(ws_sub, max_tiles * b.S * b.N);
            ws_tile = std::max(ws_tile, max_tiles * b.N);
            ws_grp = std::max(ws_grp, ((max_tiles + 63) / 64) * b.N);
            ws_n = std::max(ws_n, (size_t)b.N);
            H->ws_psi_slab = std::max(H->ws_psi_slab, (size_t)b.K * 2 * b.N);
            H->ws_cells_slab = std::max(H->ws_cells_slab, (size_t)b.K);
            H->ws_phi_slab = std::max(H->ws_phi_slab, (size_t)b.K * 2 * b.L1);
            c += b.K;
            so += (int64_t)b.K * b.L1;
            half += b.NH;
            psi_off += (int64_t)b.K * 2 * b.N;
            phi_off += (int64_t)b.K * 2 * b.L1;
            exit_off += b.N;
            H->slabs.push_back(std::move(b));
        }
        H->psi_len = psi_off;
        H->phi_len = phi_off;
        H->exit_len = exit_off;
        H->build_exit_tables(d, st);
        // slots: one per concurrently iterated slab, within a memory budget
        {
            const size_t per = sizeof(double) * (2 * ws_q + 3 * ws_phi + 2 * ws_s + 4 * ws_p + 2 * ws_e +
                                                 2 * ws_part + 2 * ws_sub + 3 * ws_tile + 2 * ws_grp + ws_n);
            const size_t budget = (size_t)8 << 30;
            const int nslot = (int)std::max<size_t>(
                1, std::min<size_t>({(size_t)kSlots, (size_t)d->num_slabs, budget / std::max<size_t>(per, 1)}));
            H->ws.resize(nslot);
            for (int g = 0; g < nslot; ++g) {
                Workspace &W = H->ws[g];
                W.q = H->dalloc<double>(ws_q);
                W.psi = H->dalloc<double>(ws_q);
                W.phiA = H->dalloc<double>(ws_phi);
                W.phiB = H->dalloc<double>(ws_phi);
                W.phi_half = H->dalloc<double>(ws_phi);
                W.s = H->dalloc<double>(ws_s);
                W.inflow = H->dalloc<double>(ws_s);
                W.pvec = H->dalloc<double>(ws_p);
                W.bvec = H->dalloc<double>(ws_p);
                W.fvec = H->dalloc<double>(ws_p);
                W.gvec = H->dalloc<double>(ws_p);
                W.e_fwd = H->dalloc<double>(ws_e);
                W.e_bwd = H->dalloc<double>(ws_e);
                W.part_f = H->dalloc<double>(ws_part);
                W.part_b = H->dalloc<double>(ws_part);
                W.subA = H->dalloc<double>(ws_sub);
                W.subB = H->dalloc<double>(ws_sub);
                W.tileA = H->dalloc<double>(ws_tile);
                W.tileB = H->dalloc<double>(ws_tile);
                W.carry = H->dalloc<double>(ws_tile);
                W.grpA = H->dalloc<double>(ws_grp);
                W.grpB = H->dalloc<double>(ws_grp);
                W.sweep_exit = H->dalloc<double>(ws_n);
                if (g > 0) HIPCHK(hipStreamCreateWithFlags(&W.stream, hipStreamNonBlocking));
                HIPCHK(hipEventCreateWithFlags(&W.done, hipEventDisableTiming));
            }
            if (nslot > 1) HIPCHK(hipEventCreateWithFlags(&H->ev_order, hipEventDisableTiming));
        }
        autotune_tiles(H, st);
        HIPCHK(hipStreamSynchronize(st));
    } catch (const HipError &e) {
        H->release();
        delete H;
        return fail(SN_E_HIP, std::string("HIP error in ") + e.where + ": " + hipGetErrorString(e.e));
    } catch (const std::bad_alloc &) {
        H->release();
        delete H;
        return fail(SN_E_NOMEM, "device or host allocation failed in sn_setup");
    }
    *out = H;
    return SN_OK;
}

sn_status sn_destroy(sn_handle h) {
    if (!h) return fail(SN_E_STATE, "NULL handle");
    (void)hipDeviceSynchronize();
    h->release();
    delete h;
    return SN_OK;
}

sn_status sn_slab_info(sn_handle h, int32_t slab, int32_t *info) {
    if (!h) return fail(SN_E_STATE, "NULL handle");
    if (!info || slab < 0 || slab >= (int32_t)h->slabs.size()) return fail(SN_E_INVALID, "bad slab index");
    const Slab &b = h->slabs[slab];
    info[0] = b.K; info[1] = b.N; info[2] = b.L;
    info[3] = b.chunk; info[4] = b.nchunks; info[5] = b.ntiles;
    info[6] = h->batch ? 0 : b.TC;
    return SN_OK;
}

sn_status sn_sizes(sn_handle h, int64_t *psi_len, int64_t *phi_len, int64_t *exit_len) {
    if (!h) return fail(SN_E_STATE, "NULL handle");
    if (psi_len) *psi_len = h->psi_len;
    if (phi_len) *phi_len = h->phi_len;
    if (exit_len) *exit_len = h->exit_len;
    return SN_OK;
}

static sn_status sweep_impl(sn_handle h, const void *qv, void *psiv, double *phi, int32_t bc_mode,
                            void *stream, bool adjoint) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (!qv) return fail(SN_E_INVALID, "q is required");
    if (!adjoint && bc_mode != SN_BC_PROBLEM && bc_mode != SN_BC_ZERO)
        return fail(SN_E_INVALID, "bc_mode must be SN_BC_PROBLEM or SN_BC_ZERO");
    hipStream_t st = (hipStream_t)stream;
    if (h->batch) {
        if (adjoint) return fail(SN_E_STATE, "the adjoint sweep needs an SN_F64 handle");
        batch_sweep(*h->batch, (const float *)qv, (float *)psiv, phi, bc_mode == SN_BC_PROBLEM, nullptr, st,
                    h->timer);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(SN_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
        return SN_OK;
    }
    const double *q = (const double *)qv;
    const Workspace &W = h->ws[0];
    double *psi = (double *)psiv;
    for (const Slab &b : h->slabs) {
        double *out = psi ? psi + b.psi_off : W.psi;
        SweepArgs a = sweep_args(W, b, q + b.psi_off, out, !adjoint && bc_mode == SN_BC_PROBLEM);
        launch_sweep(a, adjoint, st, h->timer);
        if (phi) moments(b, out, phi + b.phi_off, st, h->timer);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SN_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return SN_OK;
}

sn_status sn_sweep(sn_handle h, const void *q, void *psi, double *phi, int32_t bc_mode, void *stream) {
    return sweep_impl(h, q, psi, phi, bc_mode, stream, false);
}

sn_status sn_sweep_adjoint(sn_handle h, const double *q_adj, double *psi_adj, double *phi_adj,
                           void *stream) {
    return sweep_impl(h, q_adj, psi_adj, phi_adj, SN_BC_ZERO, stream, true);
}

sn_status sn_scatter_source(sn_handle h, const double *phi, const void *q_extv, void *q_outv,
                            void *stream) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (!phi || !q_outv) return fail(SN_E_INVALID, "phi and q_out are required");
    hipStream_t st = (hipStream_t)stream;
    if (h->batch) {
        batch_scatter(*h->batch, phi, (const float *)q_extv, (float *)q_outv, st, h->timer);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(SN_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
        return SN_OK;
    }
    const double *q_ext = (const double *)q_extv;
    double *q_out = (double *)q_outv;
    for (const Slab &b : h->slabs)
        scatter(b, phi + b.phi_off, q_ext ? q_ext + b.psi_off : nullptr, q_out + b.psi_off, st, h->timer);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SN_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return SN_OK;
}

sn_status fpsa_correct(sn_handle h, const double *phi_half, const double *phi_old, double *phi_new,
                       void *stream) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (!phi_half || !phi_old || !phi_new) return fail(SN_E_INVALID, "phi_half, phi_old, phi_new are required");
    if (phi_new == phi_half || phi_new == phi_old) return fail(SN_E_INVALID, "phi_new may not alias its inputs");
    if (!h->has_fp) return fail(SN_E_STATE, "the handle has no Fokker-Planck factors (SN_F64 with a scheme needed)");
    hipStream_t st = (hipStream_t)stream;
    const Workspace &W = h->ws[0];
    for (const Slab &b : h->slabs)
        correct(h, W, b, phi_half + b.phi_off, phi_old + b.phi_off, phi_new + b.phi_off, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SN_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return SN_OK;
}

// Work vectors of one slab's correction (the workspace fields correct()
// uses), carved out of one base pointer; offsets in doubles, each sub-array
// starting on 256 bytes.  Returns the doubles needed.
static size_t correct_scratch_layout(const Slab &b, double *base, Workspace *W) {
    const size_t NH = (size_t)b.NH, N = (size_t)b.N, K = (size_t)b.K;
    const size_t parts = (size_t)fp_carry_parts(b.nchunks, b.NH);
    size_t off = 0;
    auto take = [&](double *&dst, size_t n) {
        if (W) dst = base + off;
        off += (n + 31) & ~(size_t)31;
    };
    Workspace tmp;
    Workspace &w = W ? *W : tmp;
    take(w.s, K * N);
    take(w.inflow, K * N);
    take(w.pvec, (K + 1) * NH);
    take(w.bvec, (K + 1) * NH);
    take(w.fvec, (K + 1) * NH);
    take(w.gvec, (K + 1) * NH);
    take(w.e_fwd, ((size_t)b.nchunks + 1) * NH);
    take(w.e_bwd, ((size_t)b.nchunks + 1) * NH);
    take(w.part_f, ((size_t)b.nchunks + 1) * parts * NH);
    take(w.part_b, ((size_t)b.nchunks + 1) * parts * NH);
    return off;
}

sn_status fpsa_correct_noalloc(sn_handle h, const double *phi_half, const double *phi_old, double *phi_new,
                               void *stream) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (!phi_half || !phi_old || !phi_new) return fail(SN_E_INVALID, "phi_half, phi_old, phi_new are required");
    if (phi_new == phi_half || phi_new == phi_old) return fail(SN_E_INVALID, "phi_new may not alias its inputs");
    if (!h->has_fp) return fail(SN_E_STATE, "the handle has no Fokker-Planck factors (SN_F64 with a scheme needed)");
    double *base = scratch_device_ptr(h->device);
    if (!base) return fail(SN_E_STATE, "the scratch of this device was not attached at setup");
    const size_t cap = kScratchBytes / sizeof(double);
    for (size_t bi = 0; bi < h->slabs.size(); ++bi) {
        const size_t need = correct_scratch_layout(h->slabs[bi], nullptr, nullptr);
        if (need > cap)
            return fail(SN_E_INVALID, "slab " + std::to_string(bi) + " needs " + std::to_string(need * sizeof(double)) +
                                          " bytes of scratch; fpsa_correct_noalloc has " +
                                          std::to_string(kScratchBytes) + " (use fpsa_correct)");
    }
    hipStream_t st = (hipStream_t)stream;
    // slabs one after the other on the stream, each reusing the scratch
    for (const Slab &b : h->slabs) {
        Workspace W;
        correct_scratch_layout(b, base, &W);
        correct(h, W, b, phi_half + b.phi_off, phi_old + b.phi_off, phi_new + b.phi_off, st, SkipTest(), nullptr,
                false);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SN_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return SN_OK;
}

// ---------------------------------------------------------------------------
// Restarted GMRES on the moment form of the transport problem (the outer
// Krylov solver the paper compares with FPSA, Sec. 4):
//   (I - K) phi = b,   K phi = D L^{-1} M Sigma phi  (zero inflow, no source),
//   b = D L^{-1} (q_ext + inflow),
// left-preconditioned by the FPSA correction P = I + D F^{-1} M Sigma
// (precond) or unpreconditioned.  P (b - (I - K) x) is exactly one FPSA step
// from x minus x, so the residual GMRES minimises (2-norm) bounds the
// stopping-test value of eq:iterate (max norm) that SI / FPSA use: the same
// tolerance means the same test.  Each application of (I - K) is one sweep
// (plus one Fokker-Planck solve); iters counts sweeps.  Classical
// Gram-Schmidt with one reorthogonalisation pass; Givens rotations and the
// small triangular solve on the host.  The returned phi is one FPSA (SI)
// step from the final iterate.
// ---------------------------------------------------------------------------
constexpr int kGmresRestart = kGmresMaxRestart;

static sn_status gmres_workspace(sn_handle h) {
    if (h->kr_V) return SN_OK;
    const int m = kGmresRestart;
    const size_t n = h->ws_phi_slab;
    try {
        h->kr_ld = (n + 31) & ~(size_t)31;
        h->kr_V = h->dalloc<double>((size_t)(m + 1) * h->kr_ld);
        h->kr_w = h->dalloc<double>(n);
        h->kr_t = h->dalloc<double>(n);
        h->kr_zero = h->dalloc<double>(n);
        h->kr_part = h->dalloc<double>((size_t)krylov_gs_blocks(n) * (m + 1));
        h->kr_coef = h->dalloc<double>((size_t)3 * (m + 2));
        HIPCHK(hipMemset(h->kr_zero, 0, n * sizeof(double)));
        HIPCHK(hipHostMalloc((void **)&h->kr_host, (size_t)3 * (m + 2) * sizeof(double), hipHostMallocDefault));
        h->kr_state = reinterpret_cast<GmresState *>(h->dalloc<double>((sizeof(GmresState) + 7) / 8));
        HIPCHK(hipHostMalloc((void **)&h->kr_state_host, sizeof(GmresState), hipHostMallocDefault));
    } catch (const std::bad_alloc &) {
        return fail(SN_E_NOMEM, "device allocation of the GMRES workspace failed");
    } catch (const HipError &e) {
        return fail(SN_E_HIP, std::string("HIP error in ") + e.where + ": " + hipGetErrorString(e.e));
    }
    return SN_OK;
}

static sn_status gmres_solve(sn_handle h, bool precond, double tol, int32_t max_iter, const double *q_ext,
                             double *phi, double *psi_exit, int32_t *iters, double *resid_hist, hipStream_t st,
                             bool problem_bc) {
    sn_status ws = gmres_workspace(h);
    if (ws != SN_OK) return ws;
    const int m = kGmresRestart;
    Workspace &W = h->ws[0];
    sn_status result = SN_OK;
    try {
        for (size_t bi = 0; bi < h->slabs.size(); ++bi) {
            const Slab &b = h->slabs[bi];
            const size_t n = (size_t)b.K * 2 * b.L1, ld = h->kr_ld;
            const double *qe = q_ext ? q_ext + b.psi_off : nullptr;
            double *x = phi + b.phi_off;
            const bool fuse = sweep_fusable(b.N, b.L1, b.TC);
            // mom = D L^{-1} (M Sigma src + qext), inflow per with_bc
            auto sweep_moments = [&](const double *src, const double *qx, bool with_bc, double *mom,
                                     SkipTest sk = SkipTest()) {
                if (fuse) {
                    SweepArgs a = sweep_args(W, b, W.q, W.psi, with_bc, sk);
                    a.src_phi = src; a.src_sigma_s = b.sigma_s; a.src_Mt = b.Mt; a.src_qext = qx;
                    a.q_out = W.q; a.L1 = b.L1;
                    a.mom_Vt = b.Vt; a.write_psi = false; a.mom_out = mom;
                    launch_sweep(a, false, st, h->timer);
                } else {
                    scatter(b, src, qx, W.q, st, h->timer, sk);
                    launch_sweep(sweep_args(W, b, W.q, W.psi, with_bc, sk), false, st, h->timer);
                    moments(b, W.psi, mom, st, h->timer, sk);
                }
            };
            // V_0 = P (b - (I - K) x); kr_w = x + V_0 (one FPSA / SI step)
            auto residual = [&]() {
                sweep_moments(x, qe, problem_bc, W.phi_half);
                if (precond) {
                    correct(h, W, b, W.phi_half, x, h->kr_w, st);
                    launch_vec_sub(n, h->kr_w, x, h->kr_V, st, h->timer);
                } else {
                    HIPCHK(hipMemcpyAsync(h->kr_w, W.phi_half, n * sizeof(double), hipMemcpyDeviceToDevice, st));
                    launch_vec_sub(n, W.phi_half, x, h->kr_V, st, h->timer);
                }
            };
            auto fetch = [&](int count) {
                HIPCHK(hipMemcpyAsync(h->kr_host, h->kr_coef, count * sizeof(double), hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
            };
            std::vector<double> H((size_t)(m + 1) * m), g(m + 1), y(m);
            int sweeps = 0;
            bool converged = false, nonfinite = false;
            while (true) {
                residual();
                ++sweeps;
                launch_multi_dot(n, 1, h->kr_V, ld, h->kr_V, h->kr_part, h->kr_coef, st, h->timer);
                fetch(1);
                const double beta = std::sqrt(h->kr_host[0]);
                if (resid_hist) resid_hist[bi * (size_t)max_iter + sweeps - 1] = beta;
                if (!std::isfinite(beta)) { nonfinite = true; break; }
                if (beta <= tol) { converged = true; break; }
                if (sweeps >= max_iter) break;
                launch_vec_scale(n, h->kr_V, 1.0 / beta, h->kr_V, st, h->timer);
                // the cycle's Arnoldi steps are queued in batches; each step's
                // sweep and correction are gated on the device state (a
                // finished cycle skips them), and the host reads the state
                // once per batch instead of once per step
                GmresState &hs = *h->kr_state_host;
                std::memset(&hs, 0, sizeof(GmresState));
                hs.g[0] = beta;
                hs.gate = beta;
                HIPCHK(hipMemcpyAsync(h->kr_state, &hs, sizeof(GmresState), hipMemcpyHostToDevice, st));
                SkipTest sk;
                sk.prev = reinterpret_cast<const unsigned long long *>(&h->kr_state->gate);
                sk.tol = tol;
                double *c1 = h->kr_coef, *c2 = h->kr_coef + (m + 2), *c3 = h->kr_coef + 2 * (m + 2);
                int j = 0, ran = 0, batch = 4;
                // leave room for the sweep that evaluates the updated iterate
                while (j < m && sweeps < max_iter - 1) {
                    const int nb = std::min({batch, m - j, max_iter - 1 - sweeps});
                    for (int jj = j; jj < j + nb; ++jj) {
                        double *vj = h->kr_V + (size_t)jj * ld;
                        // w = P (I - K) v_j
                        sweep_moments(vj, nullptr, false, W.phi_half, sk);
                        launch_vec_sub(n, vj, W.phi_half, h->kr_t, st, h->timer);
                        if (precond)
                            correct(h, W, b, h->kr_t, h->kr_zero, h->kr_w, st, sk);
                        else
                            HIPCHK(hipMemcpyAsync(h->kr_w, h->kr_t, n * sizeof(double), hipMemcpyDeviceToDevice, st));
                        // two classical Gram-Schmidt passes, then the norm
                        launch_multi_dot(n, jj + 1, h->kr_V, ld, h->kr_w, h->kr_part, c1, st, h->timer);
                        launch_axpy_dot(n, jj + 1, h->kr_V, ld, c1, h->kr_w, h->kr_part, c2, st, h->timer);
                        launch_axpy_norm(n, jj + 1, h->kr_V, ld, c2, h->kr_w, h->kr_part, c3, st, h->timer);
                        launch_gmres_arnoldi(h->kr_state, jj, m, c1, c2, c3, tol, st, h->timer);
                        launch_vec_scale_dev(n, h->kr_w, &h->kr_state->inv_hn, h->kr_V + (size_t)(jj + 1) * ld, st,
                                             h->timer);
                    }
                    HIPCHK(hipMemcpyAsync(&hs, h->kr_state, sizeof(GmresState), hipMemcpyDeviceToHost, st));
                    HIPCHK(hipStreamSynchronize(st));
                    // steps whose sweep ran; each one that completed its
                    // rotation recorded its residual
                    for (int k = ran; k < hs.ran; ++k) {
                        ++sweeps;
                        if (resid_hist && k < hs.jn) resid_hist[bi * (size_t)max_iter + sweeps - 1] = hs.res[k];
                    }
                    ran = hs.ran;
                    if (hs.done) break;
                    j += nb;
                    // the steps still needed, from the recent contraction
                    int nextb = std::min(2 * batch, m);
                    if (j >= 2) {
                        const int d = std::min(j - 1, 4);
                        const double rl = hs.res[j - 1], r0 = hs.res[j - 1 - d];
                        const double rho = std::pow(rl / r0, 1.0 / d);
                        if (rho > 0.0 && rho < 1.0 && rl > tol)
                            nextb = (int)std::max(1.0, std::min((double)m, std::ceil(std::log(tol / rl) / std::log(rho))));
                    }
                    batch = nextb;
                }
                nonfinite = hs.nonfinite != 0;
                const int jn = hs.jn;
                for (int i = 0; i < jn; ++i) g[i] = hs.g[i];
                for (int r = 0; r < jn; ++r)
                    for (int c = 0; c < jn; ++c) H[(size_t)r * m + c] = hs.H[r * m + c];
                if (nonfinite) break;
                // y = R^{-1} g, x += V y
                for (int i = jn - 1; i >= 0; --i) {
                    double sacc = g[i];
                    for (int k = i + 1; k < jn; ++k) sacc -= H[(size_t)i * m + k] * y[k];
                    y[i] = sacc / H[(size_t)i * m + i];
                }
                HIPCHK(hipMemcpyAsync(h->kr_coef, y.data(), jn * sizeof(double), hipMemcpyHostToDevice, st));
                launch_multi_axpy(n, jn, h->kr_V, ld, h->kr_coef, 1.0, x, st, h->timer);
                HIPCHK(hipStreamSynchronize(st));  // y is a host temporary
            }
            iters[bi] = sweeps;  // <= max_iter
            // phi <- the FPSA (SI) step from the final iterate, computed by residual()
            HIPCHK(hipMemcpyAsync(x, h->kr_w, n * sizeof(double), hipMemcpyDeviceToDevice, st));
            if (psi_exit)
                launch_exit_flux(b.N, W.sweep_exit, precond ? W.bvec : nullptr,
                                 precond ? W.pvec + (size_t)b.K * b.NH : nullptr, psi_exit + b.exit_off, st,
                                 h->timer);
            if (nonfinite) {
                HIPCHK(hipStreamSynchronize(st));
                return fail(SN_E_NONFINITE, "non-finite GMRES residual in slab " + std::to_string(bi));
            }
            if (!converged) result = SN_NOT_CONVERGED;
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
    } catch (const HipError &e) {
        return fail(SN_E_HIP, std::string("HIP error in ") + e.where + ": " + hipGetErrorString(e.e));
    }
    return result;
}

static sn_status solve_impl(sn_handle h, int32_t method, double tol, int32_t max_iter, const void *q_extv,
                            double *phi, void *psi_exitv, int32_t *iters, double *resid_hist, void *stream,
                            bool problem_bc) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (method != SN_SI && method != SN_FPSA && method != SN_FPSA_GMRES && method != SN_GMRES)
        return fail(SN_E_INVALID, "method must be SN_SI, SN_FPSA, SN_FPSA_GMRES or SN_GMRES");
    if (!phi || !iters) return fail(SN_E_INVALID, "phi and iters are required");
    if (max_iter < 1) return fail(SN_E_INVALID, "max_iter must be >= 1");
    if (!(tol >= 0.0)) return fail(SN_E_INVALID, "tol must be >= 0");
    if ((method == SN_FPSA || method == SN_FPSA_GMRES) && !h->has_fp)
        return fail(SN_E_STATE, "FPSA needs an SN_F64 handle with a Fokker-Planck scheme");
    hipStream_t st = (hipStream_t)stream;
    if (h->batch && (method == SN_FPSA_GMRES || method == SN_GMRES))
        return fail(SN_E_STATE, "GMRES needs an SN_F64 handle");
    if (method == SN_FPSA_GMRES || method == SN_GMRES)
        return gmres_solve(h, method == SN_FPSA_GMRES, tol, max_iter, (const double *)q_extv, phi,
                           (double *)psi_exitv, iters, resid_hist, st, problem_bc);
    if (h->batch) {
        try {
            h->ensure_hist(kHistRing * h->batch->nslab);
        } catch (const HipError &e) {
            return fail(SN_E_HIP, std::string("HIP error in ") + e.where + ": " + hipGetErrorString(e.e));
        }
        std::string msg;
        const sn_status r = batch_solve_si(*h->batch, tol, max_iter, (const float *)q_extv, phi, (float *)psi_exitv,
                                           iters, resid_hist, h->hist, h->hist_host, st, h->timer, msg);
        if (r < 0) return fail(r, msg);
        return r;
    }
    const double *q_ext = (const double *)q_extv;
    double *psi_exit = (double *)psi_exitv;
    if (h->slabs.size() >= 2 && h->batched_solve && f64_batch_workspace(h) == SN_OK)
        return solve_batched_f64(h, method, tol, max_iter, q_ext, phi, psi_exit, iters, resid_hist, st, problem_bc);
    sn_status result = SN_OK;
    // Slabs are independent: up to ws.size() of them iterate at once, slab
    // i of the queue on slot g with its own workspace and stream (slot 0 on
    // the caller's stream).  Per slab, iterations are queued in batches
    // without host synchronisation; iteration m's kernels are gated on
    // iteration m-1's stopping-test value (SkipTest), so once the test
    // passes on the device the remaining queued iterations do nothing.  The
    // batch size follows the observed contraction rate.
    struct SlotRun {
        int slab = -1, launched = 0, batch = 2, its = 0, pending = 0;
        bool nonfinite = false;
    };
    const int G = std::min<int>((int)h->ws.size(), (int)h->slabs.size());
    std::vector<SlotRun> run(G);
    auto passes = [&](double d) { return d <= tol || !std::isfinite(d); };
    int bad_slab = -1;
    try {
        for (int g = 0; g < G; ++g) h->ensure_hist(h->ws[g], max_iter);
        auto stream_of = [&](int g) { return g == 0 ? st : h->ws[g].stream; };
        if (G > 1) {
            HIPCHK(hipEventRecord(h->ev_order, st));
            for (int g = 1; g < G; ++g) HIPCHK(hipStreamWaitEvent(h->ws[g].stream, h->ev_order, 0));
        }
        size_t next = 0;
        auto start = [&](int g) {
            SlotRun &r = run[g];
            r = SlotRun();
            if (next >= h->slabs.size()) return;
            r.slab = (int)next++;
            const Slab &b = h->slabs[r.slab];
            Workspace &W = h->ws[g];
            launch_solve_reset(W.hist, max_iter, stream_of(g));
            HIPCHK(hipMemcpyAsync(W.phiA, phi + b.phi_off, (size_t)b.K * 2 * b.L1 * sizeof(double),
                                  hipMemcpyDeviceToDevice, stream_of(g)));
        };
        // queue the next batch of iterations of slot g and the copy of their
        // stopping-test values
        auto enqueue = [&](int g) {
            SlotRun &r = run[g];
            const Slab &b = h->slabs[r.slab];
            Workspace &W = h->ws[g];
            const hipStream_t sg = stream_of(g);
            const size_t nphi = (size_t)b.K * 2 * b.L1;
            double *buf[2] = {W.phiA, W.phiB};
            const double *qe = q_ext ? q_ext + b.psi_off : nullptr;
            const bool fuse = sweep_fusable(b.N, b.L1, b.TC);
            const int nb = std::min(r.batch, max_iter - r.launched);
            for (int i = 0; i < nb; ++i) {
                const int m = r.launched + i + 1;
                double *cur = buf[(m - 1) & 1], *nxt = buf[m & 1];
                SkipTest sk;
                sk.prev = m > 1 ? W.hist + (m - 2) : nullptr;
                sk.tol = tol;
                FusedStop fs;
                fs.ref = cur;
                fs.slot = W.hist + (m - 1);
                if (fuse) {
                    // the sweep forms its tiles' source from cur and their
                    // moments (SI: the next iterate and its stopping test)
                    SweepArgs a = sweep_args(W, b, W.q, W.psi, problem_bc, sk);
                    a.src_phi = cur; a.src_sigma_s = b.sigma_s; a.src_Mt = b.Mt; a.src_qext = qe;
                    a.q_out = W.q; a.L1 = b.L1;
                    a.mom_Vt = b.Vt; a.write_psi = false;
                    if (method == SN_FPSA) {
                        a.mom_out = W.phi_half;
                    } else {
                        a.mom_out = nxt; a.mom_ref = cur; a.mom_slot = fs.slot;
                    }
                    launch_sweep(a, false, sg, h->timer);
                    if (method == SN_FPSA) {
                        correct(h, W, b, W.phi_half, cur, nxt, sg, sk, &fs);
                        if (b.seg_begin.size() != 2)
                            launch_stopping_test(nxt, cur, nphi, fs.slot, sk, sg, h->timer);
                    }
                    continue;
                }
                scatter(b, cur, qe, W.q, sg, h->timer, sk);
                SweepArgs a = sweep_args(W, b, W.q, W.psi, problem_bc, sk);
                launch_sweep(a, false, sg, h->timer);
                if (method == SN_FPSA) {
                    moments(b, W.psi, W.phi_half, sg, h->timer, sk);
                    correct(h, W, b, W.phi_half, cur, nxt, sg, sk, &fs);
                    if (b.seg_begin.size() != 2)
                        launch_stopping_test(nxt, cur, nphi, fs.slot, sk, sg, h->timer);
                } else {
                    moments(b, W.psi, nxt, sg, h->timer, sk, &fs);
                }
            }
            HIPCHK(hipMemcpyAsync(W.hist_host + r.launched, W.hist + r.launched, nb * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, sg));
            r.pending = nb;
        };
        // after slot g's stream has drained: look for the passing test, or
        // size the next batch; true when the slab is finished
        auto process = [&](int g) {
            SlotRun &r = run[g];
            Workspace &W = h->ws[g];
            const int nb = r.pending;
            for (int i = 0; i < nb && r.its == 0; ++i) {
                double d;
                std::memcpy(&d, &W.hist_host[r.launched + i], sizeof(double));
                if (passes(d)) {
                    r.its = r.launched + i + 1;
                    r.nonfinite = !std::isfinite(d);
                }
            }
            r.launched += nb;
            if (r.its || r.launched >= max_iter) return true;
            // predict the iterations still needed from the recent contraction rate
            double hl, h0;
            std::memcpy(&hl, &W.hist_host[r.launched - 1], sizeof(double));
            const int d = std::min(r.launched - 1, 8);
            int nextb = std::min(2 * r.batch, 256);
            if (d >= 1) {
                std::memcpy(&h0, &W.hist_host[r.launched - 1 - d], sizeof(double));
                const double rho = std::pow(hl / h0, 1.0 / d);
                if (rho > 0.0 && rho < 1.0 && hl > tol) {
                    const double rem = std::log(tol / hl) / std::log(rho);
                    nextb = (int)std::min(4096.0, std::max(1.0, std::ceil(0.9 * rem)));
                }
            }
            r.batch = nextb;
            return false;
        };
        auto finish = [&](int g) {
            SlotRun &r = run[g];
            const Slab &b = h->slabs[r.slab];
            Workspace &W = h->ws[g];
            const hipStream_t sg = stream_of(g);
            const bool converged = r.its > 0;
            const int its = converged ? r.its : max_iter;
            iters[r.slab] = its;
            if (resid_hist)
                for (int m = 0; m < its; ++m)
                    std::memcpy(&resid_hist[r.slab * (size_t)max_iter + m], &W.hist_host[m], sizeof(double));
            double *fin = (its & 1) ? W.phiB : W.phiA;
            HIPCHK(hipMemcpyAsync(phi + b.phi_off, fin, (size_t)b.K * 2 * b.L1 * sizeof(double),
                                  hipMemcpyDeviceToDevice, sg));
            if (psi_exit)
                launch_exit_flux(b.N, W.sweep_exit, method == SN_FPSA ? W.bvec : nullptr,
                                 method == SN_FPSA ? W.pvec + (size_t)b.K * b.NH : nullptr,
                                 psi_exit + b.exit_off, sg, h->timer);
            if (r.nonfinite && bad_slab < 0) bad_slab = r.slab;
            if (!converged) result = SN_NOT_CONVERGED;
        };
        // each slot's next batch is queued as soon as its previous one has
        // been read back, independently of the other slots
        auto submit = [&](int g) {
            enqueue(g);
            HIPCHK(hipEventRecord(h->ws[g].done, stream_of(g)));
        };
        for (int g = 0; g < G; ++g) {
            start(g);
            if (run[g].slab >= 0) submit(g);
        }
        while (true) {
            bool any = false, progressed = false;
            for (int g = 0; g < G; ++g) {
                if (run[g].slab < 0) continue;
                any = true;
                const hipError_t q = hipEventQuery(h->ws[g].done);
                if (q == hipErrorNotReady) continue;
                HIPCHK(q);
                progressed = true;
                if (process(g)) {
                    finish(g);
                    start(g);
                }
                if (run[g].slab >= 0) submit(g);
            }
            if (!any) break;
            if (!progressed) std::this_thread::yield();
        }
        HIPCHK(hipGetLastError());
        for (int g = 0; g < G; ++g) HIPCHK(hipStreamSynchronize(stream_of(g)));
    } catch (const HipError &e) {
        return fail(SN_E_HIP, std::string("HIP error in ") + e.where + ": " + hipGetErrorString(e.e));
    }
    if (bad_slab >= 0) return fail(SN_E_NONFINITE, "non-finite stopping-test value in slab " + std::to_string(bad_slab));
    return result;
}

sn_status sn_solve(sn_handle h, int32_t method, double tol, int32_t max_iter, const void *q_ext,
                   double *phi, void *psi_exit, int32_t *iters, double *resid_hist, void *stream) {
    return solve_impl(h, method, tol, max_iter, q_ext, phi, psi_exit, iters, resid_hist, stream, true);
}

static sn_status ensure_adjoint_workspace(sn_handle h) {
    if (h->adj_q) return SN_OK;
    try {
        h->adj_q = h->dalloc<double>((size_t)h->psi_len);
        h->adj_y = h->dalloc<double>(h->ws_psi_slab);
        h->jpart = h->dalloc<double>(h->ws_cells_slab);
    } catch (const std::bad_alloc &) {
        return fail(SN_E_NOMEM, "device allocation of the adjoint workspace failed");
    }
    return SN_OK;
}

static sn_status f64_handle(sn_handle h, const char *what) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (h->batch) return fail(SN_E_STATE, std::string(what) + " needs an SN_F64 handle");
    return SN_OK;
}

sn_status sn_update_cross_sections(sn_handle h, const double *sigma_t, const double *sigma_s, void *stream) {
    sn_status cs = f64_handle(h, "sn_update_cross_sections");
    if (cs != SN_OK) return cs;
    if (!sigma_t || !sigma_s) return fail(SN_E_INVALID, "sigma_t and sigma_s are required");
    int64_t c = 0, so = 0;
    for (const Slab &b : h->slabs) {
        if (!finite_all(sigma_t + c, b.K) || !finite_all(sigma_s + so, (size_t)b.K * b.L1))
            return fail(SN_E_NONFINITE, "non-finite cross section");
        for (int j = 0; j < b.K; ++j) {
            const double *ss = sigma_s + so + (int64_t)j * b.L1;
            if (!(sigma_t[c + j] > 0.0)) return fail(SN_E_INVALID, "sigma_t must be > 0");
            if (sigma_t[c + j] - ss[0] < 0.0) return fail(SN_E_INVALID, "sigma_a = sigma_t - sigma_s0 must be >= 0");
            if (h->has_fp && b.L1 > 1 && ss[0] - ss[1] < 0.0)
                return fail(SN_E_INVALID, "sigma_tr = sigma_s0 - sigma_s1 must be >= 0");
        }
        c += b.K;
        so += (int64_t)b.K * b.L1;
    }
    hipStream_t st = (hipStream_t)stream;
    try {
        c = 0;
        so = 0;
        for (const Slab &b : h->slabs) {
            HIPCHK(hipMemcpyAsync(b.sigma_t, sigma_t + c, (size_t)b.K * sizeof(double), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(b.sigma_s, sigma_s + so, (size_t)b.K * b.L1 * sizeof(double),
                                  hipMemcpyHostToDevice, st));
            if (b.sigma_s2) {
                dvec s2((size_t)b.K * 2 * b.L1);
                for (int j = 0; j < b.K; ++j)
                    for (int nu = 0; nu < 2; ++nu)
                        for (int l = 0; l < b.L1; ++l)
                            s2[((size_t)j * 2 + nu) * b.L1 + l] = sigma_s[so + (int64_t)j * b.L1 + l];
                HIPCHK(hipMemcpyAsync(b.sigma_s2, s2.data(), s2.size() * sizeof(double), hipMemcpyHostToDevice, st));
                HIPCHK(hipStreamSynchronize(st));  // s2 is a host temporary
            }
            c += b.K;
            so += (int64_t)b.K * b.L1;
        }
        HIPCHK(hipStreamSynchronize(st));
    } catch (const HipError &e) {
        return fail(SN_E_HIP, std::string("HIP error in ") + e.where + ": " + hipGetErrorString(e.e));
    }
    return SN_OK;
}

sn_status sn_solve_adjoint(sn_handle h, int32_t method, double tol, int32_t max_iter, const double *c,
                           double *phi_y, int32_t *iters, double *resid_hist, void *stream) {
    sn_status cs = f64_handle(h, "sn_solve_adjoint");
    if (cs != SN_OK) return cs;
    if (!c) return fail(SN_E_INVALID, "c is required");
    cs = ensure_adjoint_workspace(h);
    if (cs != SN_OK) return cs;
    hipStream_t st = (hipStream_t)stream;
    for (const Slab &b : h->slabs)
        launch_adjoint_source(b.K, b.N, b.h, b.w, c + b.psi_off, h->adj_q + b.psi_off, st, h->timer);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SN_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return solve_impl(h, method, tol, max_iter, h->adj_q, phi_y, nullptr, iters, resid_hist, stream, false);
}

sn_status sn_response_gradient(sn_handle h, const double *q_ext, const double *phi, const double *c,
                               const double *phi_y, double *J, double *g_sigma_t, double *g_sigma_s,
                               void *stream) {
    sn_status cs = f64_handle(h, "sn_response_gradient");
    if (cs != SN_OK) return cs;
    if (!phi || !c || !phi_y || !J || !g_sigma_t || !g_sigma_s)
        return fail(SN_E_INVALID, "phi, c, phi_y, J, g_sigma_t and g_sigma_s are required");
    cs = ensure_adjoint_workspace(h);
    if (cs != SN_OK) return cs;
    hipStream_t st = (hipStream_t)stream;
    Workspace &W = h->ws[0];
    for (size_t bi = 0; bi < h->slabs.size(); ++bi) {
        const Slab &b = h->slabs[bi];
        // converged states are kept as moments only: each angular flux is
        // regenerated by one sweep of its converged scattering source
        scatter(b, phi + b.phi_off, q_ext ? q_ext + b.psi_off : nullptr, W.q, st, h->timer);
        launch_sweep(sweep_args(W, b, W.q, W.psi, true), false, st, h->timer);
        launch_adjoint_source(b.K, b.N, b.h, b.w, c + b.psi_off, h->adj_q + b.psi_off, st, h->timer);
        scatter(b, phi_y + b.phi_off, h->adj_q + b.psi_off, W.q, st, h->timer);
        launch_sweep(sweep_args(W, b, W.q, h->adj_y, false), false, st, h->timer);
        GradArgs g;
        g.K = b.K; g.N = b.N; g.L1 = b.L1;
        g.h = b.h; g.w = b.w;
        g.psi = W.psi; g.y = h->adj_y; g.c = c + b.psi_off;
        g.phi = phi + b.phi_off; g.phi_y = phi_y + b.phi_off;
        g.g_sigma_t = g_sigma_t + b.cell_off;
        g.g_sigma_s = g_sigma_s + b.phi_off / 2;  // [sum K (L+1)]
        g.jpart = h->jpart;
        launch_grad_cells(g, st, h->timer);
        launch_sum(b.K, h->jpart, J + bi, st, h->timer);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SN_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return SN_OK;
}

sn_status sn_exit_current_weights(sn_handle h, double *c, void *stream) {
    sn_status cs = f64_handle(h, "sn_exit_current_weights");
    if (cs != SN_OK) return cs;
    if (!c) return fail(SN_E_INVALID, "c is required");
    hipStream_t st = (hipStream_t)stream;
    for (const Slab &b : h->slabs) launch_exit_weights(b.K, b.N, b.mu, b.w, c + b.psi_off, st, h->timer);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SN_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return SN_OK;
}

sn_status sn_exit_current(sn_handle h, const void *psi_exit, double *J, void *stream) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (!psi_exit || !J) return fail(SN_E_INVALID, "psi_exit and J are required");
    launch_exit_current((int)h->slabs.size(), h->exit_offs, h->exit_wmu, psi_exit, h->batch != nullptr, J,
                        (hipStream_t)stream, h->timer);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SN_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return SN_OK;
}

// Mixed-precision iterative refinement: FP32 (or split-BF16) batched source
// iterations corrected by FP64 residuals (see snfpsa.h).
sn_status sn_solve_refined(sn_handle lo, sn_handle hi, double tol, double tol_lo, double inner_rel,
                           int32_t max_steps, int32_t max_iter, const double *q_ext, double *phi, int32_t *steps,
                           int32_t *inner_iters, double *resid, void *stream) {
    sn_status cs = check_handle(lo);
    if (cs != SN_OK) return cs;
    cs = check_handle(hi);
    if (cs != SN_OK) return cs;
    if (!lo->batch) return fail(SN_E_STATE, "the low-precision handle must be SN_F32 or SN_BF16X3");
    if (hi->batch) return fail(SN_E_STATE, "the residual handle must be SN_F64");
    if (lo->slabs.size() != hi->slabs.size() || lo->phi_len != hi->phi_len || lo->psi_len != hi->psi_len)
        return fail(SN_E_INVALID, "the two handles describe different slabs");
    for (size_t b = 0; b < lo->slabs.size(); ++b)
        if (lo->slabs[b].K != hi->slabs[b].K || lo->slabs[b].N != hi->slabs[b].N || lo->slabs[b].L != hi->slabs[b].L)
            return fail(SN_E_INVALID, "the two handles describe different slabs");
    if (!phi || !steps) return fail(SN_E_INVALID, "phi and steps are required");
    if (!(tol >= 0.0) || !(tol_lo >= 0.0) || !(inner_rel > 0.0 && inner_rel < 1.0))
        return fail(SN_E_INVALID, "need tol >= 0, tol_lo >= 0 and 0 < inner_rel < 1");
    if (max_steps < 1 || max_iter < 1) return fail(SN_E_INVALID, "max_steps and max_iter must be >= 1");
    const int ns = (int)lo->slabs.size();
    hipStream_t st = (hipStream_t)stream;
    const size_t n = (size_t)hi->phi_len, npsi = (size_t)hi->psi_len;
    double *r = nullptr, *u = nullptr, *part = nullptr, *dmax = nullptr, *dmax_h = nullptr;
    float *qlo = nullptr, *qc = nullptr;
    auto release = [&]() {
        (void)hipStreamSynchronize(st);
        for (void *p : {(void *)r, (void *)u, (void *)part, (void *)dmax, (void *)qlo, (void *)qc})
            if (p) (void)hipFree(p);
        if (dmax_h) (void)hipHostFree(dmax_h);
    };
    sn_status result = SN_NOT_CONVERGED;
    std::string msg;
    try {
        HIPCHK(hipMalloc((void **)&r, n * sizeof(double)));
        HIPCHK(hipMalloc((void **)&u, n * sizeof(double)));
        HIPCHK(hipMalloc((void **)&part, (size_t)krylov_dot_blocks(n) * sizeof(double)));
        HIPCHK(hipMalloc((void **)&dmax, sizeof(double)));
        HIPCHK(hipMalloc((void **)&qc, npsi * sizeof(float)));
        HIPCHK(hipHostMalloc((void **)&dmax_h, sizeof(double), hipHostMallocDefault));
        if (q_ext) {
            HIPCHK(hipMalloc((void **)&qlo, npsi * sizeof(float)));
            launch_narrow(npsi, q_ext, qlo, st, lo->timer);
        }
        lo->ensure_hist(kHistRing * ns);
        std::vector<int32_t> its(ns, 0);
        if (inner_iters) std::fill(inner_iters, inner_iters + ns, 0);
        // low-precision solve of the problem itself
        sn_status ls = batch_solve_si(*lo->batch, tol_lo, max_iter, qlo, phi, nullptr, its.data(), nullptr, lo->hist,
                                      lo->hist_host, st, lo->timer, msg, true);
        if (ls < 0) {
            release();
            return fail(ls, msg);
        }
        if (inner_iters)
            for (int b = 0; b < ns; ++b) inner_iters[b] += its[b];
        Workspace &W = hi->ws[0];
        int s = 0;
        while (true) {
            // FP64 residual r = D L^{-1}(M Sigma phi + q_ext + inflow) - phi
            for (const Slab &b : hi->slabs) {
                scatter(b, phi + b.phi_off, q_ext ? q_ext + b.psi_off : nullptr, W.q, st, hi->timer);
                launch_sweep(sweep_args(W, b, W.q, W.psi, true), false, st, hi->timer);
                moments(b, W.psi, W.phi_half, st, hi->timer);
                launch_vec_sub((size_t)b.K * 2 * b.L1, W.phi_half, phi + b.phi_off, r + b.phi_off, st, hi->timer);
            }
            launch_absmax(n, r, part, dmax, st, hi->timer);
            HIPCHK(hipMemcpyAsync(dmax_h, dmax, sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            const double rn = *dmax_h;
            if (resid) resid[s] = rn;
            ++s;
            if (!std::isfinite(rn)) {
                release();
                return fail(SN_E_NONFINITE, "non-finite residual in the refinement");
            }
            if (rn <= tol) {
                result = SN_OK;
                break;
            }
            if (s >= max_steps) break;
            // correction: u = K u + K r in low precision (zero inflow), then
            // phi += r + u, so that the correction solves (I - K) d = r
            batch_scatter(*lo->batch, r, nullptr, qc, st, lo->timer);
            HIPCHK(hipMemsetAsync(u, 0, n * sizeof(double), st));
            ls = batch_solve_si(*lo->batch, inner_rel * rn, max_iter, qc, u, nullptr, its.data(), nullptr, lo->hist,
                                lo->hist_host, st, lo->timer, msg, false);
            if (ls < 0) {
                release();
                return fail(ls, msg);
            }
            if (inner_iters)
                for (int b = 0; b < ns; ++b) inner_iters[b] += its[b];
            launch_add2(n, r, u, phi, st, hi->timer);
        }
        *steps = s;
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        release();
        return fail(SN_E_HIP, std::string("HIP error in ") + e.where + ": " + hipGetErrorString(e.e));
    }
    release();
    return result;
}

sn_status sn_sweep_tuning(sn_handle h, int32_t *choice, double *ms) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (!choice) return fail(SN_E_INVALID, "choice is required");
    if (!h->batch) {
        *choice = h->tile_choice;
        if (ms)
            for (int c = 0; c < 4; ++c) ms[c] = c < kTilePolicies ? h->tile_ms[c] : 0.0;
        return SN_OK;
    }
    *choice = h->batch->tune_choice;
    if (ms)
        for (int c = 0; c < 4; ++c) ms[c] = h->batch->tune_ms[c];
    return SN_OK;
}

sn_status sn_set_sweep_choice(sn_handle h, int32_t choice) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (!h->batch) {
        if (choice < 0 || choice >= kTilePolicies) return fail(SN_E_INVALID, "choice must be 0..2 for an SN_F64 handle");
        (void)hipDeviceSynchronize();
        set_tiling_all(h, choice);
        h->tile_choice = choice;
        // the batched solve's workspace and launch tables follow the tiling
        if (h->f64b) {
            h->f64b->release();
            delete h->f64b;
            h->f64b = nullptr;
        }
        return SN_OK;
    }
    if (choice < 0 || choice > 3) return fail(SN_E_INVALID, "choice must be 0..3");
    h->batch->tune_choice = choice;
    h->batch->nitems_dm = h->batch->cand_n[choice];
    h->batch->items_dm = h->batch->cand_items[choice];
    return SN_OK;
}

sn_status sn_scan_tuning(sn_handle h, int32_t *seg_cells, double *ms) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (!h->batch) return fail(SN_E_STATE, "sn_scan_tuning needs an SN_F32 or SN_BF16X3 handle");
    if (!seg_cells) return fail(SN_E_INVALID, "seg_cells is required");
    const BatchData &B = *h->batch;
    const bool any = B.nlong_chains > 0;
    *seg_cells = any ? kSegCandidates[B.seg_choice] : 0;
    if (ms)
        for (int c = 0; c < 3; ++c) ms[c] = any ? B.seg_ms[c] : 0.0;
    return SN_OK;
}

sn_status sn_set_scan_choice(sn_handle h, int32_t choice) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (!h->batch) return fail(SN_E_STATE, "sn_set_scan_choice needs an SN_F32 or SN_BF16X3 handle");
    if (choice < 0 || choice > 2) return fail(SN_E_INVALID, "choice must be 0..2");
    batch_set_seg_choice(*h->batch, choice);
    return SN_OK;
}

sn_status sn_fused_iteration(sn_handle h, int32_t *enabled, int32_t *available) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (!h->batch) return fail(SN_E_STATE, "sn_fused_iteration needs an SN_F32 or SN_BF16X3 handle");
    if (enabled) *enabled = h->batch->use_fused ? 1 : 0;
    if (available) *available = h->batch->fused_ok ? 1 : 0;
    return SN_OK;
}

sn_status sn_set_fused_iteration(sn_handle h, int32_t enable) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (!h->batch) return fail(SN_E_STATE, "sn_set_fused_iteration needs an SN_F32 or SN_BF16X3 handle");
    if (enable && !h->batch->fused_ok)
        return fail(SN_E_STATE, "the fused iteration needs slabs of at most 131072 cells and classes at most 128 wide");
    h->batch->use_fused = enable != 0;
    return SN_OK;
}

sn_status sn_set_graph_replay(sn_handle h, int32_t enable) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (!h->batch) return fail(SN_E_STATE, "sn_set_graph_replay needs an SN_F32 or SN_BF16X3 handle");
    h->batch->use_graphs = enable != 0;
    return SN_OK;
}

sn_status sn_set_batched_solve(sn_handle h, int32_t enable) {
    sn_status cs = f64_handle(h, "sn_set_batched_solve");
    if (cs != SN_OK) return cs;
    h->batched_solve = enable != 0;
    return SN_OK;
}

sn_status sn_set_kernel_timing(sn_handle h, int32_t enable) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    delete h->timer;
    h->timer = nullptr;
    if (enable) h->timer = new (std::nothrow) EventTimer();
    if (enable && !h->timer) return fail(SN_E_NOMEM, "host allocation failed");
    return SN_OK;
}

sn_status sn_get_kernel_timing(sn_handle h, int32_t kernel_id, const char **name, int64_t *launches,
                               double *total_ms) {
    sn_status cs = check_handle(h);
    if (cs != SN_OK) return cs;
    if (kernel_id < 0 || kernel_id >= KID_COUNT) return fail(SN_E_INVALID, "kernel id out of range");
    if (name) *name = kernel_name(kernel_id);
    int64_t n = 0;
    double ms = 0.0;
    if (h->timer) {
        try {
            h->timer->resolve();
        } catch (const HipError &e) {
            return fail(SN_E_HIP, e.where);
        }
        n = h->timer->launches[kernel_id];
        ms = h->timer->total_ms[kernel_id];
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    return SN_OK;
}

// ---------------------------------------------------------------------------
// Host diagnostics (snfpsa_diag.h): setup math only, no device work.
// ---------------------------------------------------------------------------
sn_status sn_diag_quadrature(int32_t N, double *mu, double *w) {
    if (N < 1 || !mu || !w) return fail(SN_E_INVALID, "bad arguments");
    dvec m, ww;
    gauss_legendre(N, m, ww);
    std::copy(m.begin(), m.end(), mu);
    std::copy(ww.begin(), ww.end(), w);
    return SN_OK;
}

sn_status sn_diag_laplacian(int32_t N, int32_t scheme, double *A) {
    if (N < 2 || !A) return fail(SN_E_INVALID, "bad arguments");
    dvec m, ww;
    gauss_legendre(N, m, ww);
    dvec M = scheme == SN_FP_WFD ? wfd_laplacian(N, m, ww) : mpd_laplacian(N, m, ww);
    std::copy(M.begin(), M.end(), A);
    return SN_OK;
}

struct sn_diag_fp_s {
    FPFactors F;
};

sn_status sn_diag_fp_factor(int32_t K, int32_t N, int32_t L, const double *h, const double *sigma_t,
                            const double *sigma_s, int32_t scheme, int32_t chunk, sn_diag_fp *out) {
    if (!out || K < 1 || N < 2 || N % 2 || L < 0 || L >= N) return fail(SN_E_INVALID, "bad arguments");
    dvec m, ww;
    gauss_legendre(N, m, ww);
    dvec A = scheme == SN_FP_WFD ? wfd_laplacian(N, m, ww) : mpd_laplacian(N, m, ww);
    sn_diag_fp p = new (std::nothrow) sn_diag_fp_s();
    if (!p) return fail(SN_E_NOMEM, "host allocation failed");
    if (!build_fp_factors(K, N, L, h, sigma_t, sigma_s, m, ww, A, p->F, chunk)) {
        delete p;
        return fail(SN_E_INVALID, "singular Fokker-Planck cell block");
    }
    *out = p;
    return SN_OK;
}

sn_status sn_diag_fp_info(sn_diag_fp p, int32_t *info) {
    if (!p || !info) return fail(SN_E_INVALID, "bad arguments");
    info[0] = p->F.chunk;
    info[1] = p->F.nchunks;
    info[2] = p->F.ntypes;
    info[3] = (int32_t)p->F.seg_type.size();
    return SN_OK;
}

sn_status sn_diag_fp_get(sn_diag_fp p, int32_t which, void *dst) {
    if (!p || !dst) return fail(SN_E_INVALID, "bad arguments");
    const FPFactors &F = p->F;
    switch (which) {
        case 0: std::copy(F.cellmats.begin(), F.cellmats.end(), (double *)dst); break;
        case 1: std::copy(F.chunk_fwd.begin(), F.chunk_fwd.end(), (double *)dst); break;
        case 2: std::copy(F.chunk_bwd.begin(), F.chunk_bwd.end(), (double *)dst); break;
        case 3: std::copy(F.EsrcT.begin(), F.EsrcT.end(), (double *)dst); break;
        case 4: std::copy(F.PhisrcT.begin(), F.PhisrcT.end(), (double *)dst); break;
        case 5: std::copy(F.PhiinfT.begin(), F.PhiinfT.end(), (double *)dst); break;
        case 6: std::copy(F.seg_begin.begin(), F.seg_begin.end(), (int32_t *)dst); break;
        case 7: std::copy(F.seg_type.begin(), F.seg_type.end(), (int32_t *)dst); break;
        case 8: std::copy(F.psi_fwd.begin(), F.psi_fwd.end(), (double *)dst); break;
        case 9: std::copy(F.psi_bwd.begin(), F.psi_bwd.end(), (double *)dst); break;
        case 10: std::copy(F.theta_fwd.begin(), F.theta_fwd.end(), (double *)dst); break;
        case 11: std::copy(F.theta_bwd.begin(), F.theta_bwd.end(), (double *)dst); break;
        default: return fail(SN_E_INVALID, "unknown array id");
    }
    return SN_OK;
}

sn_status sn_diag_fp_free(sn_diag_fp p) {
    delete p;
    return SN_OK;
}

}  // extern "C"
