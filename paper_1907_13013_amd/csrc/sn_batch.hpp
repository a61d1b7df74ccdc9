// Batched (many-slab) kernels of the slab S_N library: the FP32 sweep of
// every angle of every slab in one launch, and the scattering-source and
// moment GEMMs of all slabs of a quadrature class on FP32 MFMA (or split
// BF16), with per-slab stopping tests and per-slab convergence gating.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sn_kernels.hpp"

namespace snfpsa {

// Per-slab metadata of a batched handle (device array, one per slab).
struct BatchSlab {
    int K = 0, N = 0, L1 = 0, cls = 0;     // cls: index of the (N, L1) class
    long long cell_off = 0;                // first cell in the concatenated cell arrays
    long long psi_off = 0;                 // first element of q / psi ([cell][node][angle])
    long long phi_off = 0;                 // first element of phi ([cell][node][l])
    long long ss_off = 0;                  // first element of sigma_s ([cell][l])
    int quad_off = 0;                      // first entry of the slab's mu / 1/|mu| tables
    int bc_off = 0;                        // first of the slab's N/2 inflow values
    int exit_off = 0;                      // first of the slab's N exit values
    int ab_off = 0;                        // first tile-map entry of the fused iteration (tile t: + 2 t N)
};

// Work item of the batched sweep: one wavefront serves the angles
// [angle0, angle0 + min(N, 64)) of `count` slabs of equal N (slab_list
// entries first .. first + count - 1), lanes slab-major; kmax = the largest
// K among them.  A second group of the same N and angle block (first2,
// count2, kmax2; count2 = 0: none) is swept after the first, so that pairing
// long with short groups gives every wavefront about the same number of
// cells.
// pad > 0 (direction-major list only): each group is one slab of N <= 16
// swept in pad = 64/N cell segments by the wavefront.
struct SweepItem {
    int first, count, angle0, kmax;
    int first2, count2, kmax2, pad;
};

// Per-slab convergence gate: work of slab b is skipped when prev[b] (the
// IEEE bits of its previous stopping-test value) passed the test or is not
// finite.  prev == null: never skip.  With iter set (graph replay of the
// solve's iteration), prev is hist + (*iter - 2) * ns instead, none for
// *iter == 1.
struct SlabGate {
    const unsigned long long *prev = nullptr;
    double tol = 0.0;
    const int *iter = nullptr;
    unsigned long long *hist = nullptr;    // [kHistRing][ns] stopping-test ring
    int ns = 0;
};

struct BatchSweepArgs {
    int nitems = 0;
    const SweepItem *items = nullptr;
    const int *slab_list = nullptr;
    const BatchSlab *slabs = nullptr;
    const float *q = nullptr;              // [sum 2 K N]
    float *psi = nullptr;                  // [sum 2 K N]
    const float2 *cellpar = nullptr;       // [cells] {h, sigma_t h}
    const double *mu = nullptr, *inv_absmu = nullptr;
    const double *psi_left = nullptr, *psi_right = nullptr;  // [sum N/2] or null (vacuum)
    float *exit = nullptr;                 // [sum N] far-face outflow or null
    SlabGate gate;
    bool dirmajor = false;                 // q / psi in the direction-major layout (below)
};

// Direction-major layout of a slab's q / psi (the batched solve's internal
// workspace): [dir][cell][a][node] with dir = 0 for the N/2 negative cosines
// and 1 for the positive ones, a the angle within its half; element
// (cell, node, n) of a slab sits at
//   dir * K * N + cell * N + 2 * (n - dir * N/2) + node.
// Each sweep direction then streams contiguous memory and a cell's two
// nodes are adjacent.
__host__ __device__ inline long long dm_index(int K, int N, int cell, int node, int n) {
    const int dir = n >= N / 2 ? 1 : 0;
    return (long long)dir * K * N + (long long)cell * N + 2 * (n - dir * (N / 2)) + node;
}

// Long slabs (K >= kLongCells) in the direction-major solve sweep: each
// (slab, 64-angle block) chain is cut into segments of about kSegCells
// cells, one wavefront each.  Pass 1 composes a segment's affine cell maps,
// a per-chain scan forms every segment's carry-in, pass 2 re-sweeps.
constexpr int kLongCells = 16384;
// candidate segment lengths of the long-slab scan (the autotuner keeps the
// fastest on the handle's own long slabs; 1024 without long slabs)
constexpr int kSegCandidates[3] = {512, 1024, 2048};

struct LongSeg {
    int slab, angle0, c0, c1;   // cells [c0, c1) of angles angle0 .. angle0+63
    int first, nseg, seg, pad;  // first = index of segment 0 of this chain
};

struct BatchLongArgs {
    int nsegs = 0, nchains = 0;
    const LongSeg *segs = nullptr;
    const int *chain_first = nullptr;      // [nchains] index of each chain's segment 0
    const BatchSlab *slabs = nullptr;
    const float *q = nullptr;              // direction-major
    float *psi = nullptr;
    const float2 *cellpar = nullptr;
    const double *mu = nullptr, *inv_absmu = nullptr;
    const double *psi_left = nullptr, *psi_right = nullptr;
    float *exit = nullptr;
    float2 *segAB = nullptr;               // [nsegs][64] segment maps
    float *carry = nullptr;                // [nsegs][64] segment carry-ins
    SlabGate gate;
};

void launch_sweep_long(const BatchLongArgs &a, hipStream_t s, KernelTimer *t);

// Padded width of a class GEMM: the smallest power of two >= 16 and >= both
// the angle count N and the moment count L1.
int class_width(int N, int L1);

typedef short short4_t __attribute__((ext_vector_type(4)));

// One row tile of a class GEMM: up to 64 node rows of one slab.
struct GemmTile {
    int slab, row0;
};

// Per-tile copy of the slab fields that the persistent class GEMMs address
// by (one 32-byte record per tile, read by four lanes, instead of a
// tile -> slab chain of dependent loads); offsets in 16-byte vectors (the
// persistent kernels run only on classes whose slabs start every row on 16
// bytes).
struct alignas(16) TileMeta {
    unsigned psi4, phi4, ss4;              // psi_off / 4, phi_off / 4, sigma_s base / 4
    int K, slab, row0;                     // the slab's cells, index, the tile's first row
    // sigma_s row of slab cell c: float4 vector ss4 + c * ss_step.  A tile
    // whose cells all have the same row has ss_step 0 and ss4 at that row
    // (every cell reads one cached row); otherwise ss4 = ss_off / 4 and
    // ss_step = L1 / 4
    int ss_step;
    int pad;
};
static_assert(sizeof(TileMeta) == 32 && alignof(TileMeta) == 16, "TileMeta is read as four 8-byte quarters");

// q = (phi .* sigma_s) x Mt + q_ext  over the tiles of one (N, L1) class,
// phi FP64 in, q FP32 out; split = true: split-BF16 products (hi x hi +
// hi x lo + lo x hi) with FP32 accumulation, else FP32 MFMA.
struct BatchSrcArgs {
    int ntiles = 0, N = 0, L1 = 0;
    const GemmTile *tiles = nullptr;
    const BatchSlab *slabs = nullptr;
    const double *phi = nullptr;           // [sum 2 K L1] FP64 moments, or
    const float *phi32 = nullptr;          // the same in FP32 (the solve's iterates; phi null)
    const float *sigma_s = nullptr;        // [sum K L1]
    const float *Mt = nullptr;             // [L1][N] of the class
    // split-BF16 tables of the class: Mt = hi + lo (bf16 round-to-nearest-
    // even), in MFMA fragment order [W/16][N][4] x 4 values, entry
    // (kb, n, j) holding rows k = 16 kb + 4 j .. 16 kb + 4 j + 3 of column n
    // (zero for k >= L1), W = max(32, class_width(N, L1))
    const short4_t *Mt_hi = nullptr, *Mt_lo = nullptr;
    const float *q_ext = nullptr;          // [sum 2 K N] or null (always [cell][node][angle])
    float *q = nullptr;
    SlabGate gate;
    bool dirmajor = false;                 // q written in the direction-major layout
    // graph replay: the FP32 input is buf[(*gate.iter - 1) & 1]
    const float *buf0 = nullptr, *buf1 = nullptr;
    // > 0: grid of the persistent kernel (FP32 iterates, direction-major q,
    // class eligible, see persistent_gemm_blocks), FP32 or split-BF16; the
    // persistent kernels read the tiles through meta ([ntiles])
    int pblocks = 0, pblocks_split = 0;
    const TileMeta *meta = nullptr;
};

// phi = psi x Vt (FP32 MFMA, FP64 or FP32 out) over the tiles of one class,
// with the per-slab stopping test max |phi - ref| (evaluated in FP64) folded
// into slot[slab] when a reference is set.
struct BatchMomArgs {
    int ntiles = 0, N = 0, L1 = 0;
    const GemmTile *tiles = nullptr;
    const BatchSlab *slabs = nullptr;
    const float *psi = nullptr;
    const float *Vt = nullptr;             // [N][L1] of the class
    double *phi = nullptr;                 // FP64 output, or
    float *phi32 = nullptr;                // FP32 output (the solve's iterates; phi and ref null)
    const double *ref = nullptr;
    const float *ref32 = nullptr;          // stopping-test reference of FP32 iterates
    unsigned long long *slot = nullptr;    // [num_slabs]
    SlabGate gate;
    bool dirmajor = false;                 // psi read in the direction-major layout
    // graph replay (gate.iter set): FP32 output buf[*iter & 1], reference
    // buf[(*iter - 1) & 1], slot gate.hist + (*iter - 1) * ns
    float *buf0 = nullptr, *buf1 = nullptr;
    int pblocks = 0;                       // as in BatchSrcArgs
    const TileMeta *meta = nullptr;
};

// Fused source iteration (handles whose slabs all have at most
// kFusedMaxCells cells and whose classes are at most 128 wide with 16-byte
// rows).
// A slab's cells are cut into tiles of kFusedCells (the class GEMMs'
// 64-row tiles).  The aggregate pass forms each tile's scattering source on
// MFMA in LDS and runs every angle's LD recurrence over each half of the tile
// (two thread halves at once) from a zero inflow: the half's outgoing flux is
// alpha x + beta for inflow x.  The scan composes these maps along each
// (slab, angle) into every half-tile's inflow and the far-face exit.  The
// apply pass forms the source again, sweeps both halves from their inflows
// with the fluxes kept in LDS, and takes the new iterate's
// moments on MFMA with the per-slab stopping test: q and psi never reach
// HBM.
constexpr int kFusedCells = 32;
// Longest slab of the fused iteration: its scan walks a slab's tiles in
// series (8192 half-tile maps per angle at most, a fraction of a millisecond).
constexpr int kFusedMaxCells = 131072;

// Per-tile record of the fused passes (offsets in 16-byte vectors as in
// TileMeta; cell0 = first cell of the tile in the concatenated cell arrays;
// ab = first of the tile's 2 N tile-map entries: angle n's maps of its
// lower and upper halves at ab + 2 n and ab + 2 n + 1).
struct alignas(16) FusedTile {
    unsigned phi4, psi4, ss4;
    int ss_step;
    int K, slab, row0, cell0;
    int quad_off, ab, iso, pad;            // iso: the tile's q_ext is isotropic (its e0 rows are used)
};
static_assert(sizeof(FusedTile) == 48, "FusedTile layout");

struct BatchFusedArgs {
    int ntiles = 0, N = 0, L1 = 0;
    const FusedTile *tiles = nullptr;
    const float *phi32 = nullptr;          // current iterate (gate.iter null)
    float *out32 = nullptr;                // next iterate (apply pass)
    // graph replay (gate.iter set): current buf[(*iter - 1) & 1], next
    // buf[*iter & 1], stopping-test slots gate.hist + hist_row(*iter) ns
    const float *buf0 = nullptr, *buf1 = nullptr;
    const float *sigma_s = nullptr, *Mt = nullptr, *Vt = nullptr;
    // three-piece BF16 tables of the class: Mt and Vt as p0 + p1 + p2, each
    // piece in the fragment order of BatchSrcArgs' split tables (Vt's entry
    // (kb, l, j) holding rows n = 16 kb + 4 j .. + 3 of column l).  FP32
    // handles form both products from three pieces (FP32 rounding; FP32
    // MFMA from Mt / Vt at 32 wide); split handles (split) the source from
    // two (the split-BF16 precision) and the moments on FP32 MFMA.
    const short4_t *Mt3[3] = {nullptr, nullptr, nullptr};
    const short4_t *Vt3[3] = {nullptr, nullptr, nullptr};
    bool split = false;
    const float *q_ext = nullptr;          // [cell][node][angle] or null
    // isotropic external source per node row ([sum 2 K]), read for tiles
    // with iso set instead of q_ext
    const float *e0 = nullptr;
    const float2 *cellpar = nullptr;
    const float *sinv = nullptr;           // sign(mu) / |mu| per quadrature entry
    float *alpha = nullptr, *beta = nullptr;   // aggregate pass out
    const float *carry = nullptr;              // apply pass in
    unsigned long long *slot = nullptr;
    SlabGate gate;
};

struct BatchFusedScanArgs {
    int nslabs = 0;
    const BatchSlab *slabs = nullptr;
    const double *mu = nullptr;
    const double *psi_left = nullptr, *psi_right = nullptr;
    float *exit = nullptr;
    const float *alpha = nullptr, *beta = nullptr;
    float *carry = nullptr;
    SlabGate gate;
};

// Isotropy test of q_ext per fused tile: iso[tile] = 1 and e0 = the common
// value of each node row when every row of the tile has one value over its
// angles (then the aggregate and apply passes read e0 instead of q_ext).
struct BatchIsoArgs {
    int ntiles = 0, N = 0;
    FusedTile *tiles = nullptr;
    const float *q_ext = nullptr;
    float *e0 = nullptr;
};

// true when an (N, L1) class can run the fused passes (16-byte rows given)
bool fused_class_ok(int N, int L1);
// aggregate (apply = false) or apply pass over the tiles of one class
void launch_fused_pass(const BatchFusedArgs &a, bool apply, hipStream_t s, KernelTimer *t);
void launch_fused_scan(const BatchFusedScanArgs &a, hipStream_t s, KernelTimer *t);
void launch_fused_iso(const BatchIsoArgs &a, hipStream_t s);

void launch_sweep_batch(const BatchSweepArgs &a, hipStream_t s, KernelTimer *t);
// Grid of the persistent class GEMMs of an (N, L1) class (kind 0: FP32
// source, 1: moments, 2: split-BF16 source): resident blocks per CU x CUs,
// capped at the number of row units; 0 when the class has no persistent
// kernel of that kind (width above 256, above 128 for the moments, or rows
// not 16-byte aligned: vec4 false).  Host call, outside any stream
// capture.
int persistent_gemm_blocks(int N, int L1, int kind, bool vec4, int ntiles);
void launch_src_batch(const BatchSrcArgs &a, bool split_bf16, hipStream_t s, KernelTimer *t);
void launch_mom_batch(const BatchMomArgs &a, hipStream_t s, KernelTimer *t);
// out rows of each slab from bufs[its[slab] & 1] (per tile), converting the
// final iterate selection of a batched solve into one array
void launch_select_final(int ntiles, const GemmTile *tiles, const BatchSlab *slabs, int L1,
                         const int *its, const float *bufA, const float *bufB, double *out, hipStream_t s);
// out = (float) in, n elements
void launch_to_f32(size_t n, const double *in, float *out, hipStream_t s);
// *iter += 1 (the last node of a replayed iteration)
void launch_iter_advance(int *iter, hipStream_t s);

}  // namespace snfpsa
