// Kernel argument blocks and launchers of the slab S_N / FPSA library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace snfpsa {

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
    double *carry = nullptr;                    // [ntiles][N]
    double *exit = nullptr;                     // [N] far-face outflow (may be null)
};

// One slab's Fokker-Planck interface recurrences.
struct FPArgs {
    int K = 0, NH = 0, chunk = 0, nchunks = 0;
    const double *cellmats = nullptr;   // [K][6][NH][NH]
    const double *chunk_fwd = nullptr;  // [nchunks][NH][NH]
    const double *chunk_bwd = nullptr;
    const double *s = nullptr;          // [K][N]  (s+ | s-)
    double *pvec = nullptr;             // [K+1][NH]
    double *inflow = nullptr;           // [K][N]  (a_j | b_{j+1})
    double *e_fwd = nullptr, *e_bwd = nullptr;  // [nchunks][NH]
    double *b0 = nullptr;               // [NH] correction outflow at z0
};

// Kernel identities for the optional per-launch timing.
enum KernelId {
    KID_GEMM = 0,
    KID_SWEEP_AGGREGATE,
    KID_SWEEP_SCAN,
    KID_SWEEP_APPLY,
    KID_ABSDIFF,
    KID_FP_FWD_LOCAL,
    KID_FP_FWD_FIX,
    KID_FP_BWD_LOCAL,
    KID_FP_BWD_FIX,
    KID_EXIT,
    KID_COUNT
};
const char *kernel_name(int id);

// Records begin/end of a launch on its stream (HIP events); may be null.
struct KernelTimer {
    virtual ~KernelTimer() = default;
    virtual void begin(int id, hipStream_t s) = 0;
    virtual void end(int id, hipStream_t s) = 0;
};

void launch_gemm(const GemmArgs &g, hipStream_t s, KernelTimer *t);
void launch_sweep(const SweepArgs &a, bool adjoint, hipStream_t s, KernelTimer *t);
void launch_absdiff_max(const double *a, const double *b, size_t n, unsigned long long *out,
                        hipStream_t s, KernelTimer *t);
void launch_fp_recurrences(const FPArgs &f, hipStream_t s, KernelTimer *t);
void launch_exit_flux(int N, const double *sweep_exit, const double *b0, const double *pK,
                      double *out, hipStream_t s, KernelTimer *t);

}  // namespace snfpsa
