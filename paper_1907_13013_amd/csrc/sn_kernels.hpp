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
    // Fused Fokker-Planck source of a slab with one cell type
    // (launch_fp_recurrences only; the multi-slab launches leave src_half
    // null): the additive-term kernel forms s = (phi_half - phi_old)
    // [.* sigma] x E itself instead of reading s.
    int L2 = 0;                                     // 2 (L + 1): the moment row of a cell
    const double *src_half = nullptr, *src_old = nullptr;   // [K][L2]
    const double *src_sigma = nullptr;              // [K][L2] or null (folded into the table)
    const double *src_E = nullptr;                  // [L2][N]
};

// Whether launch_fp_recurrences can form the Fokker-Planck source inside its
// additive-term kernel for a slab of NH = N/2 and L2 = 2 (L + 1).
bool fp_fusable(int NH, int L2);

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
    KID_FUSED_AGG,        // batched fused iteration: aggregate pass
    KID_FUSED_SCAN,       // batched fused iteration: tile-map scan
    KID_FUSED_APPLY,      // batched fused iteration: apply pass with the moments
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

// ---------------------------------------------------------------------------
// Batched launches over many slabs (the multi-slab FP64 solve): one launch of
// a kernel variant serves every slab (and cell-type segment) that uses it.
// Block i of such a launch serves descriptor refs[i].entry at its local
// block refs[i].local (local % gx, local / gx for two-dimensional grids).
// A descriptor holds the slab's arguments as for a single launch plus the
// fields that follow the iteration number m, read from a device counter, so
// that one set of launches serves every iteration and can be captured in a
// graph: iteration m reads the iterate phiA / phiB[(m - 1) & 1], writes
// [m & 1], and uses row hist_row(m) of the slab's stopping-test ring.
// ---------------------------------------------------------------------------
constexpr int kHistRing = 128;   // rows of a stopping-test ring
constexpr int kHistBatch = 64;   // iterations queued between read-backs
static_assert((kHistRing & (kHistRing - 1)) == 0 && kHistRing >= 2 * kHistBatch, "history ring");
__host__ __device__ inline size_t hist_row(int m) { return (size_t)((m - 1) & (kHistRing - 1)); }

struct BlockRef {
    int entry, local;
};
enum : unsigned {
    PATCH_SKIP = 1u,        // skip.prev = the previous iteration's slot (none at m = 1)
    PATCH_SRC_CUR = 2u,     // sweep: src_phi = current iterate
    PATCH_MOM_NXT = 4u,     // sweep: mom_out = next iterate
    PATCH_MOM_STOP = 8u,    // sweep: mom_ref = current iterate, mom_slot = this iteration's slot
    PATCH_A1_CUR = 16u,     // GEMM: A1 = current iterate
    PATCH_A1SUB_CUR = 32u,  // GEMM: A1sub = current iterate
    PATCH_C_NXT = 64u,      // GEMM: C = next iterate
    PATCH_STOP = 128u,      // GEMM: stop_ref = current iterate, stop_slot = this iteration's slot
    PATCH_STOPTEST = 256u   // stopping test: a = next, b = current iterate, slot = this iteration's
};
struct IterPatch {
    double *phiA = nullptr, *phiB = nullptr;  // the slab's two iterate buffers
    unsigned long long *hist = nullptr;       // the slab's column of the stopping-test ring
    int hist_stride = 0;                      // ring row stride (slots)
    long long off = 0;                        // offset of the entry's rows in the iterates
    unsigned flags = 0;                       // PATCH_* fields the iteration sets
};
template <class A>
struct MultiEntry {
    A a;
    IterPatch p;
    int gx = 1;    // blocks in x of the entry's own grid
    int flag = 0;  // sweep apply: the carry-in is formed in the kernel
};

// Stopping test of one slab (eq:iterate): *slot = max |a - b| over n values.
struct StopArgs {
    const double *a = nullptr, *b = nullptr;
    size_t n = 0;
    unsigned long long *slot = nullptr;
    SkipTest skip;
};

// Slabs that share one Fokker-Planck factorisation (slab-mean
// coefficients) run the interface recurrences as a group: one block applies
// each shared matrix to the vectors of every slab of the group, so the
// factors are read once per group instead of once per slab.  Each slab
// keeps its own vectors; the group is skipped once every slab's stopping
// test has passed (a slab whose test passed earlier recomputes the same
// values from its unchanged inputs).
constexpr int kFPGroupMax = 32;  // slabs per group
struct FPSlabVecs {
    const double *s = nullptr;
    double *fvec = nullptr, *gvec = nullptr, *pvec = nullptr, *bvec = nullptr, *inflow = nullptr;
    double *e_fwd = nullptr, *e_bwd = nullptr, *part_f = nullptr, *part_b = nullptr;
    const unsigned long long *hist = nullptr;  // the slab's column of the stopping-test ring
};
struct FPGroupArgs {
    FPArgs f;                         // shared factors and sizes (its vector fields unused)
    const FPSlabVecs *v = nullptr;    // [nslab] device
    int nslab = 0;
    int hist_stride = 0;
    double tol = 0.0;
};

// Kernel variants, and one launch of a slab: the variant, its grid, block
// and dynamic LDS, and the timing identity.
enum MultiKernel {
    MK_GEMM = 0,      // gemm_f64_mfma<v1>
    MK_GEMM_TALL,     // gemm_f64_tall
    MK_SWEEP_AGG,     // sweep_aggregate<v1>
    MK_SCAN_GROUPS,   // sweep_scan_groups
    MK_SCAN_CARRY,    // sweep_scan_carry
    MK_SWEEP_APPLY,   // sweep_apply<v1>, v2 = in-kernel carry
    MK_STOP,          // stopping_test
    MK_FP_MATVEC,     // fp_matvec<v1>
    MK_FP_CHAIN,      // v2: 0 fp_chain_ring<v1>, 1 fp_chain_staged<v1, true>, 2 <v1, false>, 3 fp_chain_any
    MK_FP_CARRY,      // fp_carry<v1>
    MK_FP_FIXUP,      // fp_fixup<v1>
    MK_GFP_MATVEC,    // grouped forms (FPGroupArgs entries), v1 = NHP <= 64
    MK_GFP_CHAIN,
    MK_GFP_CARRY,
    MK_GFP_FIXUP
};
struct LaunchShape {
    int kernel = 0, v1 = 0, v2 = 0;
    int gx = 1, gy = 1;
    unsigned lds = 0;
    int block = 256;
    int kid = 0;
};
LaunchShape gemm_shape(const GemmArgs &g);
// forward sweeps: aggregate, [scan groups, scan carry,] apply; returns the count
int sweep_shapes(const SweepArgs &s, LaunchShape out[4]);
// matvec, chain, carry, fix-up
void fp_shapes(const FPArgs &f, LaunchShape out[4]);
LaunchShape stop_shape(size_t n);
// grouped matvec, chain, carry, fix-up of a group's shared factorisation
// (NH <= 64)
void fp_group_shapes(const FPArgs &f, LaunchShape out[4]);

// One batched launch: entries is a device array of MultiEntry<A> of the
// kernel's argument type (GemmArgs, SweepArgs, FPArgs or StopArgs), refs the
// per-block table; lds the largest dynamic LDS of its entries.
struct MultiLaunch {
    LaunchShape shape;
    const void *entries = nullptr;
    const BlockRef *refs = nullptr;
    int nblocks = 0;
    unsigned lds = 0;
};
void launch_multi(const MultiLaunch &L, const int *iter, hipStream_t s, KernelTimer *t);
// iter[0] += 1 (the end of one batched iteration)
void launch_iter_step(int *iter, hipStream_t s);

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
