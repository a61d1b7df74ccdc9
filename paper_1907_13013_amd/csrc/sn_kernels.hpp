// Kernel argument blocks and launchers of the slab S_N / FPSA library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace snfpsa {

// Convergence gating of a queued iteration: its kernels do nothing when the
// previous iteration's stopping-test value (IEEE bits in *prev) passed the
// test or is not finite.  A skipped iteration leaves its own slot at zero,
// so every later queued iteration is skipped as well.
struct SkipTest {
    const unsigned long long *prev = nullptr;  // null: never skip
    double tol = 0.0;
};

// C = Cin + ((A1 - A1sub) .* S) x B1 + A2 x B2   (row-major, FP64)
struct GemmArgs {
    int rows = 0, ncols = 0;
    const double *A1 = nullptr, *A1sub = nullptr;
    int lda1 = 0, k1 = 0;
    const double *S = nullptr;  // row-group scale, may be null
    int s_div = 1, lds = 0;
    const double *B1 = nullptr;  // [k1][ncols]
    const double *A2 = nullptr;  // may be null
    int lda2 = 0, k2 = 0;
    const double *B2 = nullptr;  // [k2][ncols]
    const double *Cin = nullptr;
    int ldcin = 0;
    double *C = nullptr;
    int ldc = 0;
    SkipTest skip;
    // optional fused stopping test on the result: *stop_slot = max |C - ref|
    // (ref with leading dimension ldc, IEEE bits folded with atomicMax)
    const double *stop_ref = nullptr;
    unsigned long long *stop_slot = nullptr;
    int kid = -1;  // timing identity of the launch (-1: KID_GEMM)
};

// One slab's sweep: q/psi [K][2][N]; workspace arrays sized by ntiles.
struct SweepArgs {
    int K = 0, N = 0, TC = 0, S = 0, sub = 0, ntiles = 0;
    const double *q = nullptr;
    double *psi = nullptr;
    const double *h = nullptr, *sigma_t = nullptr;
    const double *mu = nullptr, *inv_absmu = nullptr;
    const double *psi_left = nullptr, *psi_right = nullptr;  // null = vacuum
    double *subA = nullptr, *subB = nullptr;    // [ntiles][S][N]
    double *tileA = nullptr, *tileB = nullptr;  // [ntiles][N]
    double *carry = nullptr;                    // [ntiles][N] (long slabs only)
    double *grpA = nullptr, *grpB = nullptr;    // [ceil(ntiles / 64)][N] tile-group maps (long slabs only)
    double *exit = nullptr;                     // [N] far-face outflow (may be null)
    SkipTest skip;
    // Optional fusions (forward sweep, 8 <= N <= 64, L1 <= 64, TC <= 32):
    // the aggregate pass forms the tile's scattering source
    //   q = (src_phi .* src_sigma_s) x src_Mt + src_qext   -> q_out (then read by apply)
    // and the apply pass the tile's moments  mom_out = psi x mom_Vt, with an
    // optional stopping test against mom_ref folded into *mom_slot.
    const double *src_phi = nullptr;      // [K][2][L1]
    const double *src_sigma_s = nullptr;  // [K][L1]
    const double *src_Mt = nullptr;       // [L1][N]
    const double *src_qext = nullptr;     // [K][2][N] or null
    double *q_out = nullptr;              // [K][2][N]
    int L1 = 0;
    const double *mom_Vt = nullptr;       // [N][L1]
    double *mom_out = nullptr;            // [K][2][L1]
    const double *mom_ref = nullptr;
    unsigned long long *mom_slot = nullptr;
    bool write_psi = true;
};

// Whether a slab's sweep can carry the fused source / moments GEMMs.
bool sweep_fusable(int N, int L1, int TC);

// Matrices per cell of the factorised Fokker-Planck operator, in order:
// G, Hm (forward elimination), Gb, Hb (backward elimination), and for the
// interface at the cell's left face W, W rho and sig.
constexpr int FP_CELLMATS = 7;

// One slab's Fokker-Planck interface recurrences (two-sided Riccati form).
// All matrices are stored transposed (element (r, c) at c*NH + r) so that
// the threads of one cell, one per row, read consecutive addresses.
struct FPArgs {
    int K = 0, NH = 0, chunk = 0, nchunks = 0;
    const double *cellmats = nullptr;   // [K][FP_CELLMATS][NH][NH]
    const double *psi_fwd = nullptr;    // [K][NH][NH] within-chunk prefix products (G)
    const double *psi_bwd = nullptr;    // [K][NH][NH] within-chunk prefix products (Gb)
    const double *theta_fwd = nullptr;  // chunk transfer products, see setup_math.hpp
    const double *theta_bwd = nullptr;
    const double *s = nullptr;          // [K][N]  (s+ | s-)
    double *fvec = nullptr;             // [K][NH] forward additive terms  Hm s- + s+
    double *gvec = nullptr;             // [K][NH] backward additive terms Hb s+ + s-
    double *pvec = nullptr;             // [K+1][NH] p_loc_j; p_K = a_K at [K]
    double *bvec = nullptr;             // [K+1][NH] q_loc_j; b_0 at [0] after the fix-up
    double *inflow = nullptr;           // [K][N]  (a_j | b_{j+1})
    double *e_fwd = nullptr, *e_bwd = nullptr;      // [nchunks][NH] chunk end values
    double *part_f = nullptr, *part_b = nullptr;    // [nchunks+1][parts][NH] carry partial sums
    int carry_parts = 1;                            // parts per carry row
    SkipTest skip;
};

// Number of partial sums per carry row used by launch_fp_recurrences.
int fp_carry_parts(int nchunks, int NH);

// Kernel identities for the optional per-launch timing.
enum KernelId {
    KID_GEMM = 0,
    KID_SWEEP_AGGREGATE,
    KID_SWEEP_SCAN,
    KID_SWEEP_APPLY,
    KID_ABSDIFF,
    KID_FP_MATVEC,
    KID_FP_CHAIN,
    KID_FP_CARRY,
    KID_FP_FIXUP,
    KID_EXIT,
    KID_SWEEP_BATCH,
    KID_SRC_BATCH,
    KID_MOM_BATCH,
    KID_ADJOINT,
    KID_KRYLOV,
    KID_GEMM_FP_SOURCE,   // gemm_f64_mfma launched for the Fokker-Planck source
    KID_GEMM_FP_UPDATE,   // gemm_f64_mfma launched for the correction update
    KID_COUNT
};
const char *kernel_name(int id);

// Supplies a start/stop event pair for one launch of kernel `id`; the launch
// then records its own dispatch begin and end into them
// (hipExtLaunchKernelGGL), so the pair times the kernel itself and not the
// surrounding stream markers.  May be null; returning false skips timing.
struct KernelTimer {
    virtual ~KernelTimer() = default;
    virtual bool events(int id, hipEvent_t *start, hipEvent_t *stop) = 0;
};

void launch_gemm(const GemmArgs &g, hipStream_t s, KernelTimer *t);
void launch_sweep(const SweepArgs &a, bool adjoint, hipStream_t s, KernelTimer *t);
// *slot = max |a - b| (IEEE bits, atomicMax); gated by skip.
void launch_stopping_test(const double *a, const double *b, size_t n, unsigned long long *slot,
                          SkipTest skip, hipStream_t s, KernelTimer *t);
void launch_solve_reset(unsigned long long *hist, int max_iter, hipStream_t s);
void launch_fp_recurrences(const FPArgs &f, hipStream_t s, KernelTimer *t);
void launch_exit_flux(int N, const double *sweep_exit, const double *b0, const double *pK,
                      double *out, hipStream_t s, KernelTimer *t);

// Fixed per-device scratch of the allocation-free entry point: capacity in
// bytes; scratch_attach(device) (the device current) resolves its device
// address once per device, scratch_device_ptr(device) returns it (null
// before the attach).
constexpr size_t kScratchBytes = (size_t)64 << 20;
hipError_t scratch_attach(int device);
double *scratch_device_ptr(int device);

}  // namespace snfpsa
