// Host side of the batched FP32 / split-BF16 path: setup of the batch
// tables and the sweep, scattering-source and source-iteration drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sn_batch.hpp"
#include "snfpsa.h"

namespace snfpsa {

struct BatchClass {
    int N = 0, L1 = 0;
    float *Mt = nullptr, *Vt = nullptr;    // [L1][N], [N][L1]
    short4_t *Mt_hi = nullptr, *Mt_lo = nullptr;  // split-BF16 Mt (split handles only)
    GemmTile *tiles = nullptr;             // row tiles of all slabs of the class
    TileMeta *meta = nullptr;              // the same with their slab fields (persistent GEMMs)
    FusedTile *ftiles = nullptr;           // the same for the fused iteration (null: class not eligible)
    short4_t *Mt3[3] = {nullptr, nullptr, nullptr};  // three-piece BF16 Mt and Vt (fused classes)
    short4_t *Vt3[3] = {nullptr, nullptr, nullptr};
    int ntiles = 0;
    // grids of the persistent FP32 source / moment and split-BF16 source
    // GEMMs (0: none)
    int pblocks_src = 0, pblocks_mom = 0, pblocks_split = 0;
};

struct BatchData {
    int nslab = 0;
    bool split_bf16 = false;
    std::vector<BatchSlab> host_slabs;
    std::vector<BatchClass> classes;
    BatchSlab *slabs = nullptr;
    int *slab_list = nullptr;
    SweepItem *items = nullptr;            // [cell][node][angle] layout (sn_sweep)
    int nitems = 0;
    SweepItem *items_dm = nullptr;         // direction-major layout (the solve), short slabs
    int nitems_dm = 0;
    // autotuned decomposition of the solve's sweep: candidate c has pairing
    // (c & 1) == 0 and small-N segmentation (c & 2) == 0; tune_ms[c] its
    // measured sweep time, tune_choice the one kept
    SweepItem *cand_items[4] = {nullptr, nullptr, nullptr, nullptr};
    int cand_n[4] = {0, 0, 0, 0};
    double tune_ms[4] = {0, 0, 0, 0};
    int tune_choice = 0;
    // one solve iteration as a HIP graph with iteration-relative addressing
    // (the current iteration in iter_dev), replayed once per iteration;
    // recaptured when an argument it bakes in changes
    // (captured and replayed on gstream, which is ordered after the caller's
    // stream by gev), cached per set of baked-in arguments
    struct GraphEntry {
        const void *key[6];
        double tol;
        bool bc;
        hipGraphExec_t exec;
    };
    bool use_graphs = true;
    bool persistent_gemms = true;          // persistent FP32 class GEMMs where eligible
    int *iter_dev = nullptr;
    hipStream_t gstream = nullptr;
    hipEvent_t gev = nullptr;
    std::vector<GraphEntry> graphs;        // most recently used last
    static constexpr size_t kGraphCache = 4;
    LongSeg *long_segs = nullptr;          // segments of the long slabs (the solve)
    int *long_chain_first = nullptr;
    int nlong_segs = 0, nlong_chains = 0;
    float2 *long_ab = nullptr;             // sized for the candidate with most segments
    float *long_carry = nullptr;
    // autotuned segment length of the long-slab scan: candidate c cuts the
    // chains into segments of about kSegCandidates[c] cells; seg_ms[c] its
    // measured sweep time, seg_choice the one kept
    LongSeg *cand_segs[3] = {nullptr, nullptr, nullptr};
    int *cand_chain_first[3] = {nullptr, nullptr, nullptr};
    int cand_nsegs[3] = {0, 0, 0};
    double seg_ms[3] = {0, 0, 0};
    int seg_choice = 1;
    // fused iteration (see launch_fused_pass): available when every class
    // is eligible and no slab has more than kFusedMaxCells cells; on by default
    // then.  Tile maps alpha / beta and inflows carry ([ab_len] each),
    // isotropic external source e0 ([2 cells]).
    bool fused_ok = false, use_fused = false;
    int64_t ab_len = 0;
    float *alpha = nullptr, *beta = nullptr, *carry = nullptr, *e0 = nullptr;
    float2 *cellpar = nullptr;
    float *sigma_s = nullptr;
    double *mu = nullptr, *inv_absmu = nullptr;
    float *sinv = nullptr;                 // sign(mu) / |mu| in FP32 (the fused passes)
    double *psi_left = nullptr, *psi_right = nullptr;
    int64_t psi_len = 0, phi_len = 0, exit_len = 0;
    // workspace
    float *q = nullptr, *psi = nullptr;
    float *phiA = nullptr, *phiB = nullptr;   // the solve's FP32 iterates
    int *its = nullptr;                    // [nslab] device, final selection
    std::vector<void *> allocs;

    ~BatchData();
};

// Builds the batch tables from a validated description (FP32 storage of
// q / psi / sigma_s, FP64 phi).  Throws std::bad_alloc or HipError-like
// failures through the returned status; msg receives the reason.
sn_status batch_setup(const sn_problem_desc *d, hipStream_t st, BatchData **out, std::string &msg);

// Selects candidate c (0..2) of the long-slab segment lengths.
void batch_set_seg_choice(BatchData &B, int c);

// psi = L^{-1} q for every slab (FP32 q / psi); phi (nullable, FP64)
// receives the moments.
void batch_sweep(BatchData &B, const float *q, float *psi, double *phi, bool problem_bc, float *exit,
                 hipStream_t st, KernelTimer *t);
void batch_scatter(BatchData &B, const double *phi, const float *q_ext, float *q, hipStream_t st, KernelTimer *t);

// Source iteration of every slab (each stopping on its own) from phi^0 in
// phi; see sn_solve.  hist (device) / hist_host (pinned) hold the
// stopping-test ring, kHistRing * nslab entries each.
sn_status batch_solve_si(BatchData &B, double tol, int32_t max_iter, const float *q_ext, double *phi,
                         float *psi_exit, int32_t *iters, double *resid_hist, unsigned long long *hist,
                         unsigned long long *hist_host, hipStream_t st, KernelTimer *t, std::string &msg,
                         bool problem_bc = true);

}  // namespace snfpsa
