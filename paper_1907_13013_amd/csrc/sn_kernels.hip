// HIP kernels (gfx950, wave64) of the slab S_N / FPSA library.
//
//   gemm_f64_mfma      scattering source / moments / FP correction maps as
//                      FP64 MFMA GEMMs (v_mfma_f64_16x16x4f64), LDS-staged
//                      with register prefetch of the next K chunk
//   sweep_*            LD transport sweep (eq:trsi, L = mu d/dz + sigma_t) as
//                      an affine scan over cells, one lane per angle
//   stopping_test      FP64 max|phi^{m+1} - phi^m| (eq:iterate) into a
//                      per-iteration history, with the convergence flag that
//                      turns later iterations' kernels into no-ops
//   fp_*               FP correction: forward/backward interface recurrences
//                      of the factorised LD x S_N Fokker-Planck operator
//                      (eq:correct with F of eq:fpop)
#include "sn_kernels.hpp"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

namespace snfpsa {

typedef double d4 __attribute__((ext_vector_type(4)));

// Kernel launch, timed by its own dispatch timestamps when a timer is set.
#define LAUNCH(id, t, kernel, grid, block, shm, st, ...)                                       \
    do {                                                                                       \
        hipEvent_t ev0_ = nullptr, ev1_ = nullptr;                                             \
        if ((t) && (t)->events((id), &ev0_, &ev1_))                                            \
            hipExtLaunchKernelGGL(kernel, grid, block, shm, st, ev0_, ev1_, 0, __VA_ARGS__);   \
        else                                                                                   \
            hipLaunchKernelGGL(kernel, grid, block, shm, st, __VA_ARGS__);                     \
    } while (0)

const char *kernel_name(int id) {
    static const char *names[KID_COUNT] = {"gemm_f64_mfma", "sweep_aggregate", "sweep_scan",
                                           "sweep_apply",   "stopping_test",   "fp_matvec",
                                           "fp_chain",      "fp_carry",        "fp_fixup",
                                           "exit_flux",     "sweep_batch_f32", "src_batch",
                                           "mom_batch",     "adjoint_aux",     "krylov",
                                           "gemm_fp_source", "gemm_fp_update", "fused_aggregate",
                                           "fused_scan",    "fused_apply"};
    return (id >= 0 && id < KID_COUNT) ? names[id] : "";
}

__device__ __forceinline__ bool skipped(const SkipTest &t) {
    if (!t.prev) return false;
    const double d = __longlong_as_double((long long)*t.prev);
    return d <= t.tol || !isfinite(d);
}

// Iteration-relative fields of a batched launch's descriptor (see
// MultiEntry): iteration m reads buffer (m - 1) & 1 and writes buffer m & 1
// of the slab's iterates, offset by the entry's rows.
__device__ __forceinline__ double *iter_buf(const IterPatch &p, int k) { return ((k & 1) ? p.phiB : p.phiA) + p.off; }
__device__ __forceinline__ unsigned long long *iter_slot(const IterPatch &p, int m) {
    return p.hist + hist_row(m) * (size_t)p.hist_stride;
}
__device__ __forceinline__ void patch_skip(SkipTest &sk, const IterPatch &p, int m) {
    if (p.flags & PATCH_SKIP) sk.prev = m > 1 ? iter_slot(p, m - 1) : nullptr;
}
__device__ __forceinline__ void apply_patch(SweepArgs &s, const IterPatch &p, int m) {
    patch_skip(s.skip, p, m);
    if (p.flags & PATCH_SRC_CUR) s.src_phi = iter_buf(p, m - 1);
    if (p.flags & PATCH_MOM_NXT) s.mom_out = iter_buf(p, m);
    if (p.flags & PATCH_MOM_STOP) {
        s.mom_ref = iter_buf(p, m - 1);
        s.mom_slot = iter_slot(p, m);
    }
}
__device__ __forceinline__ void apply_patch(GemmArgs &g, const IterPatch &p, int m) {
    patch_skip(g.skip, p, m);
    if (p.flags & PATCH_A1_CUR) g.A1 = iter_buf(p, m - 1);
    if (p.flags & PATCH_A1SUB_CUR) g.A1sub = iter_buf(p, m - 1);
    if (p.flags & PATCH_C_NXT) g.C = iter_buf(p, m);
    if (p.flags & PATCH_STOP) {
        g.stop_ref = iter_buf(p, m - 1);
        g.stop_slot = iter_slot(p, m);
    }
}
__device__ __forceinline__ void apply_patch(FPArgs &f, const IterPatch &p, int m) { patch_skip(f.skip, p, m); }
__device__ __forceinline__ void apply_patch(StopArgs &a, const IterPatch &p, int m) {
    patch_skip(a.skip, p, m);
    if (p.flags & PATCH_STOPTEST) {
        a.a = iter_buf(p, m);
        a.b = iter_buf(p, m - 1);
        a.slot = iter_slot(p, m);
    }
}

// ---------------------------------------------------------------------------
// Stopping test (eq:iterate) reduction shared by the stand-alone kernel and
// the fused GEMM epilogue: each block folds its maximum of |x - y| into the
// iteration's slot as the IEEE bit pattern of a non-negative double (ordered
// like unsigned integers; NaN sorts above +Inf, so a NaN anywhere surfaces
// as NaN).  The test itself is applied by the next iteration's kernels and
// by the host.  Called by all threads of the block.
// ---------------------------------------------------------------------------
__device__ void stop_block_reduce(unsigned long long m, unsigned long long *slot) {
    __shared__ unsigned long long red[16];
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    const int nw = (blockDim.x + 63) / 64;
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < nw; ++i) m = red[i] > m ? red[i] : m;
        atomicMax(slot, m);
    }
}

__device__ __forceinline__ unsigned long long absdiff_bits(double x, double y) {
    return (unsigned long long)__double_as_longlong(fabs(x - y));
}

// ---------------------------------------------------------------------------
// FP64 MFMA GEMM:  C = Cin + (A1 - A1sub) .* S  x B1  +  A2 x B2
// Row-major operands; S (optional) scales A1 column-wise per row group:
// A1[m][k] *= S[(m / s_div) * lds + k].  A 256-thread block computes a
// 16 x 64 tile, wave w the 16 x 16 block at columns 16w.. (one accumulator).
// K (the concatenation of the A1 and A2 segments) is consumed in chunks of
// 64 staged through LDS; the next chunk's global loads are issued before the
// current chunk's MFMAs.
// MFMA 16x16x4 f64 operand layout: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element r of lane l is D[l/16 + 4*r][l%16]
// (rows interleaved with stride 4, unlike the f32 16x16x4 variant).
// ---------------------------------------------------------------------------
constexpr int GM = 16, GN = 64, GK = 64;
constexpr int AS_LD = GK + 2;
// Wide form (GNW = 128, for large row counts with 64 < ncols <= 128): one
// block covers all columns, so A is read once instead of once per 64
// columns; wave w computes the 16 x 32 block at columns 32 w (two
// accumulators), and the chunks stream (NQ = 0) to keep the B chunk's
// registers within budget.
constexpr int GNWIDE = 128;
constexpr int kWideRows = 4096;   // smaller products keep twice the blocks
template <int GNW>
struct GemmGeom {
    static constexpr int BS_LD = GNW == GN ? GN + 16 : GNW + 2;
    static constexpr int CT = GNW / 64;   // 16-column tiles per wave
};

// A chunk's operands as loaded: A (and A1sub, S when present) and B, raw.
// The loads are unconditional at clamped addresses (the segment's optional
// operands under block-uniform branches), and the subtraction, scale and
// masks are applied when the chunk is staged: a loaded value is never used
// right after its load, so all of a chunk's loads are in flight together.
template <int GNW>
struct GemmChunk {
    double a[GM * GK / 256], asub[GM * GK / 256], s[GM * GK / 256], b[GK * GNW / 256];
};

struct GemmSeg {
    int k0, kt;
    bool sub, scaled;
};

__device__ __forceinline__ GemmSeg gemm_seg(const GemmArgs &g, int q, int nq1) {
    GemmSeg sg;
    const bool second = q >= nq1;
    sg.k0 = (second ? q - nq1 : q) * GK;
    sg.kt = second ? g.k2 : g.k1;
    sg.sub = !second && g.A1sub;
    sg.scaled = !second && g.S;
    return sg;
}

template <int GNW>
__device__ __forceinline__ void gemm_load_chunk(const GemmArgs &g, int q, int nq1, int m0, int n0,
                                                int tid, GemmChunk<GNW> &rc) {
    const bool second = q >= nq1;
    const GemmSeg sg = gemm_seg(g, q, nq1);
    const double *A = second ? g.A2 : g.A1;
    const double *B = second ? g.B2 : g.B1;
    const int lda = second ? g.lda2 : g.lda1;
#pragma unroll
    for (int i = 0; i < GM * GK / 256; ++i) {
        const int idx = tid + 256 * i;
        const int m = min(m0 + idx / GK, g.rows - 1), k = min(sg.k0 + idx % GK, sg.kt - 1);
        rc.a[i] = A[(size_t)m * lda + k];
        if (sg.sub) rc.asub[i] = g.A1sub[(size_t)m * lda + k];
        if (sg.scaled) rc.s[i] = g.S[(size_t)(m / g.s_div) * g.lds + k];
    }
#pragma unroll
    for (int i = 0; i < GK * GNW / 256; ++i) {
        const int idx = tid + 256 * i;
        const int k = min(sg.k0 + idx / GNW, sg.kt - 1), n = min(n0 + idx % GNW, g.ncols - 1);
        rc.b[i] = B[(size_t)k * g.ncols + n];
    }
}

// NQ > 0: all NQ chunks of K are loaded into registers before the first is
// staged, so the block waits on memory once; NQ = 0: chunks are streamed
// with a one-chunk register prefetch (any K).
template <int NQ, int GNW>
__device__ __forceinline__ void gemm_f64_mfma_body(GemmArgs g, const int bx_, const int by_) {
    constexpr int CT = GemmGeom<GNW>::CT, BS_LD = GemmGeom<GNW>::BS_LD;
    if (skipped(g.skip)) return;
    __shared__ double As[GM * AS_LD];
    __shared__ double Bs[GK * BS_LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = bx_ * GM, n0 = by_ * GNW;
    const int cw = wave * 16 * CT;
    const int nq1 = g.A1 ? (g.k1 + GK - 1) / GK : 0;
    const int nq = NQ > 0 ? NQ : nq1 + (g.A2 ? (g.k2 + GK - 1) / GK : 0);
    d4 acc[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    constexpr int NR = NQ > 0 ? NQ : 1;
    GemmChunk<GNW> rc[NR];
    if constexpr (NQ > 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) gemm_load_chunk(g, q, nq1, m0, n0, tid, rc[q]);
    } else {
        if (nq > 0) gemm_load_chunk(g, 0, nq1, m0, n0, tid, rc[0]);
    }
    // epilogue operands do not depend on the product: fetch them up front
    double cin[CT][4], ref[CT][4];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        const int col = n0 + cw + 16 * t + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = m0 + (lane >> 4) + 4 * r;
            const bool ok = row < g.rows && col < g.ncols;
            cin[t][r] = (ok && g.Cin) ? g.Cin[(size_t)row * g.ldcin + col] : 0.0;
            ref[t][r] = (ok && g.stop_ref) ? g.stop_ref[(size_t)row * g.ldc + col] : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < (NQ > 0 ? NQ : nq); ++q) {
        GemmChunk<GNW> &cur = rc[NQ > 0 ? q : 0];
        const GemmSeg sg = gemm_seg(g, q, nq1);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < GM * GK / 256; ++i) {
            const int idx = tid + 256 * i;
            const int r = idx / GK, kk = idx % GK;
            double v = cur.a[i];
            if (sg.sub) v -= cur.asub[i];
            if (sg.scaled) v *= cur.s[i];
            As[r * AS_LD + kk] = (m0 + r < g.rows && sg.k0 + kk < sg.kt) ? v : 0.0;
        }
        // B rows past the segment meet zero A columns and B columns past
        // ncols feed unstored outputs: the clamped values need no mask
#pragma unroll
        for (int i = 0; i < GK * GNW / 256; ++i) {
            const int idx = tid + 256 * i;
            Bs[(idx / GNW) * BS_LD + idx % GNW] = cur.b[i];
        }
        __syncthreads();
        if constexpr (NQ == 0) {
            if (q + 1 < nq) gemm_load_chunk(g, q + 1, nq1, m0, n0, tid, rc[0]);
        }
#pragma unroll
        for (int kq = 0; kq < GK / 4; ++kq) {
            const double a = As[(lane & 15) * AS_LD + kq * 4 + (lane >> 4)];
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const double b = Bs[(kq * 4 + (lane >> 4)) * BS_LD + cw + 16 * t + (lane & 15)];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
            }
        }
    }
    unsigned long long dmax = 0ull;
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        const int col = n0 + cw + 16 * t + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = m0 + (lane >> 4) + 4 * r;
            if (row < g.rows && col < g.ncols) {
                const double v = acc[t][r] + cin[t][r];
                g.C[(size_t)row * g.ldc + col] = v;
                if (g.stop_ref) {
                    const unsigned long long d = absdiff_bits(v, ref[t][r]);
                    dmax = d > dmax ? d : dmax;
                }
            }
        }
    }
    if (g.stop_ref) stop_block_reduce(dmax, g.stop_slot);
}

template <int NQ>
__global__ void __launch_bounds__(256) gemm_f64_mfma(GemmArgs g) {
    gemm_f64_mfma_body<NQ, GN>(g, (int)blockIdx.x, (int)blockIdx.y);
}

__global__ void __launch_bounds__(256) gemm_f64_wide(GemmArgs g) {
    gemm_f64_mfma_body<0, GNWIDE>(g, (int)blockIdx.x, (int)blockIdx.y);
}

template <int NQ>
__global__ void __launch_bounds__(256) gemm_f64_mfma_multi(const MultiEntry<GemmArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<GemmArgs> &e = E[r.entry];
    GemmArgs a = e.a;
    apply_patch(a, e.p, *iter);
    gemm_f64_mfma_body<NQ, GN>(a, r.local % e.gx, r.local / e.gx);
}

__global__ void __launch_bounds__(256) gemm_f64_wide_multi(const MultiEntry<GemmArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<GemmArgs> &e = E[r.entry];
    GemmArgs a = e.a;
    apply_patch(a, e.p, *iter);
    gemm_f64_mfma_body<0, GNWIDE>(a, r.local % e.gx, r.local / e.gx);
}


// ---------------------------------------------------------------------------
// Tall FP64 GEMM for large slabs (thousands of row tiles, K and the column
// count >= 256, no A2 / A1sub): C = Cin + (A1 .* S) x B1.  A block computes
// 64 rows x 256 columns, wave w the 64 x 64 block at columns 64 w (sixteen
// 16 x 16 accumulators), so each A element staged in LDS serves 256 columns
// and each B fragment 64 rows.  K runs in chunks of 16: the next chunk's A
// rows and B fragments are loaded into registers while the current chunk's
// MFMAs run, and A goes through two LDS buffers.  Operand layout as in
// gemm_f64_mfma.
// ---------------------------------------------------------------------------
constexpr int TT_ROWS = 64, TT_COLS = 256, TT_KC = 16, TT_LD = TT_KC + 1;

__device__ __forceinline__ void gemm_f64_tall_body(GemmArgs g, const int bx_, const int by_) {
    if (skipped(g.skip)) return;
    __shared__ double As[2][TT_ROWS * TT_LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = bx_ * TT_ROWS;
    const int c0 = by_ * TT_COLS + wave * 64;
    const bool wave_on = c0 < g.ncols;
    const int nchunk = (g.k1 + TT_KC - 1) / TT_KC;
    // A chunk: thread t holds row t/4, k = 4 (t%4) .. +3 of the chunk.  The
    // loads are unconditional (clamped addresses; without S the scale reads
    // A again and is not applied) and the scale and the mask for k >= k1 are
    // applied when the values are staged, so that issuing the next chunk's
    // loads never waits for them.
    const int ar = tid >> 2, ak = (tid & 3) * 4;
    const int arow = min(m0 + ar, g.rows - 1);
    const bool scaled = g.S != nullptr;
    const double *sp = scaled ? g.S : g.A1;
    const size_t srow = scaled ? (size_t)(arow / g.s_div) * g.lds : (size_t)arow * g.lda1;
    auto load_a = [&](int kc, double (&ra)[4], double (&rs)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kcl = min(kc * TT_KC + ak + i, g.k1 - 1);
            ra[i] = g.A1[(size_t)arow * g.lda1 + kcl];
            rs[i] = sp[srow + kcl];
        }
    };
    // B fragments: k-step s of the chunk, column block cb of the wave;
    // clamped entries are finite and meet zero A (k >= k1) or feed unstored
    // outputs (col >= ncols), so they need no mask
    auto load_b = [&](int kc, double (&rb)[4][4]) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const int k = kc * TT_KC + 4 * s4 + (lane >> 4), col = c0 + cb * 16 + (lane & 15);
                rb[s4][cb] = g.B1[(size_t)min(k, g.k1 - 1) * g.ncols + min(col, g.ncols - 1)];
            }
    };
    d4 acc[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
    // A rows of chunk kc sit in set A for even kc, set B for odd kc
    double raA[4], rsA[4], raB[4], rsB[4], bcur[4][4], bnext[4][4];
    // the epilogue's first operand (Cin, else the stopping-test reference)
    // is requested with the last chunk for all of the wave's outputs, so
    // that its latency hides behind the products; a second one (a launch
    // with both) is loaded per 16-row block in the epilogue
    const double *eop = g.Cin ? g.Cin : g.stop_ref;
    const int lde = g.Cin ? g.ldcin : g.ldc;
    auto stage_a = [&](int kc, const double (&ra)[4], const double (&rs)[4]) {
        double *Ab = As[kc & 1];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = kc * TT_KC + ak + i;
            const double v = scaled ? ra[i] * rs[i] : ra[i];
            Ab[ar * TT_LD + ak + i] = (k < g.k1 && m0 + ar < g.rows) ? v : 0.0;
        }
    };
    auto products = [&](int kc) {
        const double *Ab = As[kc & 1];
        if (wave_on) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const double a = Ab[(rb * 16 + (lane & 15)) * TT_LD + 4 * s4 + (lane >> 4)];
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bcur[s4][cb], acc[rb][cb], 0, 0, 0);
                }
        }
    };
    // A (streamed from memory) is requested two chunks ahead, B (shared by
    // every block, cache resident) one chunk ahead; each step requests B
    // before A, so that waiting for a chunk's B in the in-order load counter
    // never waits for the A loaded after it
    load_a(0, raA, rsA);
    load_b(0, bcur);
    load_a(min(1, nchunk - 1), raB, rsB);
    auto step = [&](int kc, double (&ra)[4], double (&rs)[4]) {
        stage_a(kc, ra, rs);
        __syncthreads();
        load_b(kc + 1, bnext);
        load_a(min(kc + 2, nchunk - 1), ra, rs);  // into the set just staged
        products(kc);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) bcur[s4][cb] = bnext[s4][cb];
    };
    // two chunks per trip (straight-line, so the compiler's load counting
    // stays exact across the sets)
    int kc = 0;
#pragma unroll 1
    for (; kc + 2 < nchunk; kc += 2) {
        step(kc, raA, rsA);
        step(kc + 1, raB, rsB);
    }
    if (kc + 1 < nchunk) step(kc, raA, rsA);
    // the last chunk (no next chunk to fetch) requests the epilogue's
    // operand for all of the wave's outputs
    double pre[4][4][4];
    if ((nchunk - 1) & 1)
        stage_a(nchunk - 1, raB, rsB);
    else
        stage_a(nchunk - 1, raA, rsA);
    __syncthreads();
    // the last chunk's B fragments (requested a chunk ago) land before the
    // epilogue loads are issued, so that its products never wait behind them
    // in the in-order load counter (s_waitcnt vmcnt(0), other counters free)
    __builtin_amdgcn_s_waitcnt(0x0F70);
    if (eop) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = min(m0 + rb * 16 + (lane >> 4) + 4 * r, g.rows - 1);
                    const int col = min(c0 + cb * 16 + (lane & 15), g.ncols - 1);
                    pre[rb][cb][r] = eop[(size_t)row * lde + col];
                }
    }
    products(nchunk - 1);
    // epilogue, one 16-row block at a time (operands absent from the launch
    // are neither loaded nor used: uniform branches)
    unsigned long long dmax = 0ull;
    if (wave_on) {
        const bool has_cin = g.Cin != nullptr, has_ref = g.stop_ref != nullptr;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            double ci[4][4], rf[4][4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    ci[cb][r] = has_cin ? pre[rb][cb][r] : 0.0;
                    rf[cb][r] = has_cin ? 0.0 : pre[rb][cb][r];
                }
            if (has_cin && has_ref) {
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = min(m0 + rb * 16 + (lane >> 4) + 4 * r, g.rows - 1);
                        const int col = min(c0 + cb * 16 + (lane & 15), g.ncols - 1);
                        rf[cb][r] = g.stop_ref[(size_t)row * g.ldc + col];
                    }
            }
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + rb * 16 + (lane >> 4) + 4 * r;
                    const int col = c0 + cb * 16 + (lane & 15);
                    const double v = acc[rb][cb][r] + ci[cb][r];
                    if (row < g.rows && col < g.ncols) {
                        g.C[(size_t)row * g.ldc + col] = v;
                        if (g.stop_ref) {
                            const unsigned long long d = absdiff_bits(v, rf[cb][r]);
                            dmax = d > dmax ? d : dmax;
                        }
                    }
                }
        }
    }
    if (g.stop_ref) stop_block_reduce(dmax, g.stop_slot);
}

__global__ void __launch_bounds__(256) gemm_f64_tall(GemmArgs g) {
    gemm_f64_tall_body(g, (int)blockIdx.x, (int)blockIdx.y);
}

__global__ void __launch_bounds__(256) gemm_f64_tall_multi(const MultiEntry<GemmArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<GemmArgs> &e = E[r.entry];
    GemmArgs a = e.a;
    apply_patch(a, e.p, *iter);
    gemm_f64_tall_body(a, r.local % e.gx, r.local / e.gx);
}


static bool gemm_tall_fits(const GemmArgs &g) {
    return !g.A2 && !g.A1sub && g.A1 && g.rows >= 4096 && g.k1 >= 64 && g.ncols >= TT_COLS;
}

LaunchShape gemm_shape(const GemmArgs &g) {
    LaunchShape sh;
    sh.kid = g.kid >= 0 ? g.kid : KID_GEMM;
    if (gemm_tall_fits(g)) {
        sh.kernel = MK_GEMM_TALL;
        sh.gx = (g.rows + TT_ROWS - 1) / TT_ROWS;
        sh.gy = (g.ncols + TT_COLS - 1) / TT_COLS;
        return sh;
    }
    const int nq = (g.A1 ? (g.k1 + GK - 1) / GK : 0) + (g.A2 ? (g.k2 + GK - 1) / GK : 0);
    sh.kernel = MK_GEMM;
    sh.gx = (g.rows + GM - 1) / GM;
    if (g.ncols > GN && g.ncols <= GNWIDE && g.rows >= kWideRows) {
        // one block over all columns: A read once (v2 = 1: gemm_f64_wide)
        sh.v2 = 1;
        sh.gy = 1;
        return sh;
    }
    sh.v1 = (nq >= 1 && nq <= 4) ? nq : 0;
    sh.gy = (g.ncols + GN - 1) / GN;
    return sh;
}

void launch_gemm(const GemmArgs &g, hipStream_t s, KernelTimer *t) {
    if (g.rows <= 0 || g.ncols <= 0) return;
    const LaunchShape sh = gemm_shape(g);
    const dim3 grid(sh.gx, sh.gy);
    if (sh.kernel == MK_GEMM_TALL) {
        LAUNCH(sh.kid, t, gemm_f64_tall, grid, dim3(256), 0, s, g);
        return;
    }
    if (sh.v2 == 1) {
        LAUNCH(sh.kid, t, gemm_f64_wide, grid, dim3(256), 0, s, g);
        return;
    }
    switch (sh.v1) {
        case 1: LAUNCH(sh.kid, t, gemm_f64_mfma<1>, grid, dim3(256), 0, s, g); break;
        case 2: LAUNCH(sh.kid, t, gemm_f64_mfma<2>, grid, dim3(256), 0, s, g); break;
        case 3: LAUNCH(sh.kid, t, gemm_f64_mfma<3>, grid, dim3(256), 0, s, g); break;
        case 4: LAUNCH(sh.kid, t, gemm_f64_mfma<4>, grid, dim3(256), 0, s, g); break;
        default: LAUNCH(sh.kid, t, gemm_f64_mfma<0>, grid, dim3(256), 0, s, g); break;
    }
}

// ---------------------------------------------------------------------------
// LD sweep as an affine scan.
//
// For angle n and cell j with tau = sigma_t h / |mu|, the LD cell equations
// close to  psi_out = a psi_in + b  with
//   a = (6 - 2 tau) / (6 + 4 tau + tau^2),
//   b = ((6 + 4 tau) g_out + (6 - 2 tau) g_in) / (6 + 4 tau + tau^2),
//   psi at the inflow-side node = ((6+4tau)(g_in + psi_in) - (6+2tau) g_out)/den,
// where, for the forward sweep, g_in = h/(6|mu|)(2 q_in + q_out) and
// g_out = h/(6|mu|)(q_in + 2 q_out) (q_in / q_out = source at the inflow-side
// / outflow-side node; mu > 0 enters through the left node).  The transpose
// (adjoint) sweep has the same recurrence run in the opposite direction with
// g = y at the nodes and output (h/(6|mu|)) [[2,1],[1,2]] applied after.
// Affine maps compose as (a2,b2) o (a1,b1) = (a2 a1, a2 b1 + b2).
//
// Kernels: per tile of TC cells, per-(sub-chunk, angle) aggregates; then the
// apply pass, which derives each tile's carry-in from the aggregates of the
// tiles before it (or, for long slabs, from a separate per-angle scan over
// tiles) and re-sweeps each sub-chunk.  Thread t of a 256-thread block
// serves angle t % N and sub-chunk t / N.
// ---------------------------------------------------------------------------
constexpr int SWEEP_INKERNEL_TILES = 128;

struct CellCoef {
    double a, b, gin, gout, tau, den_inv;
};

__device__ __forceinline__ CellCoef cell_coef(double inv_absmu, double hj, double stj,
                                              double yin, double yout, bool adjoint) {
    CellCoef c;
    c.tau = stj * hj * inv_absmu;
    c.den_inv = 1.0 / (6.0 + c.tau * (4.0 + c.tau));
    if (adjoint) {
        c.gin = yin;
        c.gout = yout;
    } else {
        const double f = hj * inv_absmu * (1.0 / 6.0);
        c.gin = f * (2.0 * yin + yout);
        c.gout = f * (yin + 2.0 * yout);
    }
    c.a = (6.0 - 2.0 * c.tau) * c.den_inv;
    c.b = ((6.0 + 4.0 * c.tau) * c.gout + (6.0 - 2.0 * c.tau) * c.gin) * c.den_inv;
    return c;
}

// Direction of the recurrence for angle n: +1 left-to-right, -1 right-to-left.
__device__ __forceinline__ int sweep_dir(double mu, bool adjoint) {
    return ((mu > 0.0) != adjoint) ? 1 : -1;
}

__device__ __forceinline__ double boundary_inflow(const SweepArgs &s, int n, bool adjoint) {
    if (adjoint) return 0.0;
    const double mu = s.mu[n];
    if (mu > 0.0) return s.psi_left ? s.psi_left[n - s.N / 2] : 0.0;
    return s.psi_right ? s.psi_right[n] : 0.0;
}

// Fused sweep tiles.  A tile of TC <= 32 cells has R = 2 (c1 - c0) <= 64
// node rows; its GEMM operands are staged in LDS zero-padded to NP columns
// (NP in {16, 32, 64}, NP >= N and NP >= L1) at row stride NP + 1.
//
// tile_prefetch / tile_gemm: C = A x B with A [R][NP] and B [NP][NP] in LDS
// on FP64 MFMA; the four waves take the 16 x 16 output blocks (at most 16)
// in turn.  tile_prefetch evaluates pre(row, col) for every output position
// the calling lane will own (clamped to row < R and col < nc, so pre may
// issue global loads without branches); tile_gemm hands each element with
// row < R and col < nc to out(row, col, v, pre value).
template <int NP, class Pre>
__device__ __forceinline__ void tile_prefetch(int R, int nc, double (&pv)[4][4], Pre &&pre) {
    constexpr int NCT = NP / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kl = lane >> 4;
    const int ntile = ((R + 15) / 16) * NCT;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = min(wave + 4 * i, ntile - 1);
        const int r0 = (t / NCT) * 16, c0 = (t % NCT) * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) pv[i][r] = pre(min(r0 + kl + 4 * r, R - 1), min(c0 + (lane & 15), nc - 1));
    }
}

// tile_products computes the lane's output blocks into acc (block i of
// wave w is output tile w + 4 i), reading A and B only; tile_scatter then
// hands them to out.  Between the two the caller may reuse A's storage.
template <int NP>
__device__ __forceinline__ void tile_products(const double *A, int R, const double *B, d4 (&acc)[4]) {
    constexpr int NCT = NP / 16, LD = NP + 1, NK = NP / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kl = lane >> 4;
    const int ntile = ((R + 15) / 16) * NCT;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = wave + 4 * i;
        if (t >= ntile) break;
        const int r0 = (t / NCT) * 16, c0 = (t % NCT) * 16;
        const int ar = min(r0 + (lane & 15), R - 1), bc = c0 + (lane & 15);
        double a[NK], b[NK];
#pragma unroll
        for (int u = 0; u < NK; ++u) {
            a[u] = A[ar * LD + 4 * u + kl];
            b[u] = B[(4 * u + kl) * LD + bc];
        }
        acc[i] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < NK; ++u) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc[i], 0, 0, 0);
    }
}

template <int NP, class Out>
__device__ __forceinline__ void tile_scatter(int R, int nc, const d4 (&acc)[4], const double (&pv)[4][4], Out &&out) {
    constexpr int NCT = NP / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kl = lane >> 4;
    const int ntile = ((R + 15) / 16) * NCT;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = wave + 4 * i;
        if (t >= ntile) break;
        const int r0 = (t / NCT) * 16, bc = (t % NCT) * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = r0 + kl + 4 * r;
            if (row < R && bc < nc) out(row, bc, acc[i][r], pv[i][r]);
        }
    }
}

template <int NP, class Out>
__device__ __forceinline__ void tile_gemm(const double *A, int R, const double *B, int nc,
                                          const double (&pv)[4][4], Out &&out) {
    d4 acc[4];
    tile_products<NP>(A, R, B, acc);
    tile_scatter<NP>(R, nc, acc, pv, out);
}

// Copies a rows x NP block into LDS at row stride NP + 1 with element
// (r, c) = get(r, c) for c < cols and 0 for cols <= c < NP (rows <= 64, so
// at most 16 elements per thread).  Load indices past the block are clamped,
// so the loads carry no branches and all are issued before the first store.
template <int NP, class Get>
__device__ __forceinline__ void stage_block(double *dst, int rows, int cols, Get &&get) {
    const int n = rows * NP, t = threadIdx.x;
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int idx = min(t + 256 * u, n - 1);
        v[u] = get(idx / NP, min(idx % NP, cols - 1));
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int idx = t + 256 * u;
        if (idx < n) dst[(idx / NP) * (NP + 1) + idx % NP] = (idx % NP) < cols ? v[u] : 0.0;
    }
}

// padded width of a fusable slab, 0 if the sweep cannot carry the GEMMs
static int fuse_width(int N, int L1, int TC) {
    if (N < 8 || N > 64 || L1 > 64 || TC > 32) return 0;
    const int w = N > L1 ? N : L1;
    return w <= 16 ? 16 : (w <= 32 ? 32 : 64);
}

bool sweep_fusable(int N, int L1, int TC) { return fuse_width(N, L1, TC) > 0; }

// dynamic LDS of the fused sweep kernels (doubles)
static size_t fused_aggregate_lds(const SweepArgs &s, int NP) {
    return ((size_t)2 * s.TC + NP) * (NP + 1);
}
static size_t fused_apply_lds(const SweepArgs &s, int NP) {
    return ((size_t)2 * s.TC + NP) * (NP + 1);
}

// Cells are processed in groups of SWEEP_BATCH: the group's sources and
// cross sections are loaded before the dependent recurrence runs over it.
constexpr int SWEEP_BATCH = 8;

// NP > 0: fused source (q of the tile from phi by MFMA, see SweepArgs).
template <int NP>
__device__ __forceinline__ void sweep_aggregate_body(SweepArgs s, bool adjoint, const int bx_, const int by_) {
    if (skipped(s.skip)) return;
    extern __shared__ double dyn[];
    __shared__ double shA[256], shB[256];
    const int N = s.N, S = s.S;
    const int t = threadIdx.x, n = t % N, sc = t / N;
    const int tile = bx_;
    const int c0 = tile * s.TC, c1 = min(s.K, c0 + s.TC);
    constexpr bool fused = NP > 0;
    constexpr int ldq = NP + 1;
    double *qt = dyn;  // fused: the tile's source [2 TC][NP+1], over the A operand
    if constexpr (fused) {
        // q = (phi .* sigma_s) x Mt + q_ext for the tile's R node rows
        const int L1 = s.L1, R = 2 * (c1 - c0);
        double *At = dyn;
        double *Bt = At + (size_t)2 * s.TC * ldq;
        const bool has = s.src_qext != nullptr;
        const double *qe = has ? s.src_qext : s.q_out;  // a valid address either way
        double pv[4][4];
        tile_prefetch<NP>(R, N, pv, [&](int row, int col) { return qe[((size_t)c0 * 2 + row) * N + col]; });
        stage_block<NP>(At, R, L1, [&](int r, int l) {
            return s.src_phi[((size_t)c0 * 2 + r) * L1 + l] * s.src_sigma_s[(size_t)(c0 + r / 2) * L1 + l];
        });
        stage_block<NP>(Bt, NP, N, [&](int r, int c) { return s.src_Mt[(size_t)min(r, L1 - 1) * N + c]; });
        __syncthreads();
        // rows of Bt past L1 hold Mt's last row: zero them (A is zero there
        // too, but 0 x finite is what keeps the padding exact)
        for (int idx = t; idx < (NP - L1) * NP; idx += 256) Bt[(L1 + idx / NP) * ldq + idx % NP] = 0.0;
        __syncthreads();
        d4 acc[4];
        tile_products<NP>(At, R, Bt, acc);
        __syncthreads();  // every wave is done reading At, which qt overwrites
        tile_scatter<NP>(R, N, acc, pv, [&](int row, int col, double v, double e) {
            v += has ? e : 0.0;
            qt[row * ldq + col] = v;
            s.q_out[((size_t)c0 * 2 + row) * N + col] = v;
        });
        __syncthreads();
    }
    double A = 1.0, B = 0.0;
    if (sc < S) {
        const double mu = s.mu[n], inv = s.inv_absmu[n];
        const int dir = sweep_dir(mu, adjoint);
        const int j0 = c0 + sc * s.sub, j1 = min(c1, c0 + (sc + 1) * s.sub);
        const int in_node = dir > 0 ? 0 : 1;
        const int len = j1 - j0;
        for (int i0 = 0; i0 < len; i0 += SWEEP_BATCH) {
            double yin[SWEEP_BATCH], yout[SWEEP_BATCH], hh[SWEEP_BATCH], st[SWEEP_BATCH];
#pragma unroll
            for (int u = 0; u < SWEEP_BATCH; ++u) {
                const int i = min(i0 + u, len - 1);
                const int j = dir > 0 ? j0 + i : j1 - 1 - i;
                if constexpr (fused) {
                    yin[u] = qt[((j - c0) * 2 + in_node) * ldq + n];
                    yout[u] = qt[((j - c0) * 2 + (1 - in_node)) * ldq + n];
                } else {
                    yin[u] = s.q[((size_t)j * 2 + in_node) * N + n];
                    yout[u] = s.q[((size_t)j * 2 + (1 - in_node)) * N + n];
                }
                hh[u] = s.h[j];
                st[u] = s.sigma_t[j];
            }
#pragma unroll
            for (int u = 0; u < SWEEP_BATCH; ++u) {
                if (i0 + u < len) {
                    const CellCoef c = cell_coef(inv, hh[u], st[u], yin[u], yout[u], adjoint);
                    B = c.a * B + c.b;
                    A = c.a * A;
                }
            }
        }
        s.subA[((size_t)tile * S + sc) * N + n] = A;
        s.subB[((size_t)tile * S + sc) * N + n] = B;
    }
    shA[t] = A;
    shB[t] = B;
    __syncthreads();
    if (sc == 0) {
        const int dir = sweep_dir(s.mu[n], adjoint);
        double TA = 1.0, TB = 0.0;
        for (int i = 0; i < S; ++i) {
            const int ss = dir > 0 ? i : S - 1 - i;
            const double a = shA[ss * N + n], b = shB[ss * N + n];
            TB = a * TB + b;
            TA = a * TA;
        }
        s.tileA[(size_t)tile * N + n] = TA;
        s.tileB[(size_t)tile * N + n] = TB;
    }
}

template <int NP>
__global__ void __launch_bounds__(256) sweep_aggregate(SweepArgs s, bool adjoint) {
    sweep_aggregate_body<NP>(s, adjoint, (int)blockIdx.x, (int)blockIdx.y);
}

template <int NP>
__global__ void __launch_bounds__(256) sweep_aggregate_multi(const MultiEntry<SweepArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<SweepArgs> &e = E[r.entry];
    SweepArgs a = e.a;
    apply_patch(a, e.p, *iter);
    sweep_aggregate_body<NP>(a, false, r.local, 0);
}


// Long slabs: the carry-in of every tile, per angle, in two passes over
// groups of SCAN_GROUP consecutive tiles in the angle's sweep order (lane =
// angle, one block per 64 angles and group).  sweep_scan_groups composes
// each group's tile maps; sweep_scan_carry folds the maps of the groups
// before its own onto the boundary inflow, then walks its group writing each
// tile's carry-in (and, in the last group, the exit flux).  The chain a lane
// waits through is at most ntiles / SCAN_GROUP + SCAN_GROUP maps long instead
// of ntiles.  Loads go eight at a time, at clamped addresses, before they are
// folded.
constexpr int SCAN_GROUP = 64;

__device__ __forceinline__ int scan_tile(int ii, int dir, int ntiles) { return dir > 0 ? ii : ntiles - 1 - ii; }

__device__ __forceinline__ void sweep_scan_groups_body(SweepArgs s, bool adjoint, const int bx_, const int by_) {
    if (skipped(s.skip)) return;
    const int N = s.N;
    const int n = bx_ * 64 + threadIdx.x;
    if (n >= N) return;
    const int dir = sweep_dir(s.mu[n], adjoint);
    const int g = by_;
    const int i0 = g * SCAN_GROUP, i1 = min(s.ntiles, i0 + SCAN_GROUP);
    double A = 1.0, B = 0.0;
    for (int ib = i0; ib < i1; ib += 8) {
        double a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int tile = scan_tile(min(ib + u, i1 - 1), dir, s.ntiles);
            a[u] = s.tileA[(size_t)tile * N + n];
            b[u] = s.tileB[(size_t)tile * N + n];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (ib + u < i1) {
                B = a[u] * B + b[u];
                A = a[u] * A;
            }
        }
    }
    s.grpA[(size_t)g * N + n] = A;
    s.grpB[(size_t)g * N + n] = B;
}

__global__ void __launch_bounds__(64) sweep_scan_groups(SweepArgs s, bool adjoint) {
    sweep_scan_groups_body(s, adjoint, (int)blockIdx.x, (int)blockIdx.y);
}

__global__ void __launch_bounds__(64) sweep_scan_groups_multi(const MultiEntry<SweepArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<SweepArgs> &e = E[r.entry];
    SweepArgs a = e.a;
    apply_patch(a, e.p, *iter);
    sweep_scan_groups_body(a, false, r.local % e.gx, r.local / e.gx);
}


__device__ __forceinline__ void sweep_scan_carry_body(SweepArgs s, bool adjoint, const int bx_, const int by_) {
    if (skipped(s.skip)) return;
    const int N = s.N;
    const int n = bx_ * 64 + threadIdx.x;
    if (n >= N) return;
    const int dir = sweep_dir(s.mu[n], adjoint);
    const int g = by_;
    const int i0 = g * SCAN_GROUP, i1 = min(s.ntiles, i0 + SCAN_GROUP);
    double x = boundary_inflow(s, n, adjoint);
    for (int gb = 0; gb < g; gb += 8) {
        double a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int gg = min(gb + u, g - 1);
            a[u] = s.grpA[(size_t)gg * N + n];
            b[u] = s.grpB[(size_t)gg * N + n];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (gb + u < g) x = a[u] * x + b[u];
    }
    for (int ib = i0; ib < i1; ib += 8) {
        double a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int tile = scan_tile(min(ib + u, i1 - 1), dir, s.ntiles);
            a[u] = s.tileA[(size_t)tile * N + n];
            b[u] = s.tileB[(size_t)tile * N + n];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (ib + u < i1) {
                s.carry[(size_t)scan_tile(ib + u, dir, s.ntiles) * N + n] = x;
                x = a[u] * x + b[u];
            }
        }
    }
    if (i1 == s.ntiles && s.exit) s.exit[n] = x;
}

__global__ void __launch_bounds__(64) sweep_scan_carry(SweepArgs s, bool adjoint) {
    sweep_scan_carry_body(s, adjoint, (int)blockIdx.x, (int)blockIdx.y);
}

__global__ void __launch_bounds__(64) sweep_scan_carry_multi(const MultiEntry<SweepArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<SweepArgs> &e = E[r.entry];
    SweepArgs a = e.a;
    apply_patch(a, e.p, *iter);
    sweep_scan_carry_body(a, false, r.local % e.gx, r.local / e.gx);
}


// Every load that does not depend on the carry (the tile aggregates before
// this tile, this tile's sub-chunk aggregates, the first batch of sweep
// inputs, and in fused mode Vt and the stopping-test reference) is issued
// at the start, so the block waits on memory about once before the sweep.
// NP > 0: fused moments (and stopping test) of the swept tile, see SweepArgs.
template <int NP>
__device__ __forceinline__ void sweep_apply_body(SweepArgs s, bool adjoint, bool inkernel_carry, const int bx_, const int by_) {
    if (skipped(s.skip)) return;
    extern __shared__ double dyn[];
    __shared__ double shA[256], shB[256], subA[256], subB[256];
    const int N = s.N, S = s.S;
    const int t = threadIdx.x, n = t % N, sc = t / N;
    const bool live = sc < S;
    const int tile = bx_;
    const int c0 = tile * s.TC, c1 = min(s.K, c0 + s.TC);
    const double mu = s.mu[n], inv = s.inv_absmu[n];
    const int dir = sweep_dir(mu, adjoint);
    constexpr bool fused = NP > 0;
    constexpr int ldp = NP + 1;
    double *pt = dyn;                                  // fused: swept tile [2 TC][NP+1]
    double *Vs = dyn + (size_t)2 * s.TC * ldp;         // fused: Vt [NP][NP+1]
    // this tile's sub-chunk aggregates (S x N <= 256 values, one per thread)
    const double sa = live ? s.subA[((size_t)tile * S + sc) * N + n] : 1.0;
    const double sb = live ? s.subB[((size_t)tile * S + sc) * N + n] : 0.0;
    // first batch of the sweep inputs
    const int j0 = c0 + sc * s.sub, j1 = min(c1, c0 + (sc + 1) * s.sub);
    const int in_node = dir > 0 ? 0 : 1;
    const int len = live ? j1 - j0 : 0;
    double yin[SWEEP_BATCH], yout[SWEEP_BATCH], hh[SWEEP_BATCH], st[SWEEP_BATCH];
    auto load_batch = [&](int i0) {
#pragma unroll
        for (int u = 0; u < SWEEP_BATCH; ++u) {
            const int i = min(i0 + u, max(len - 1, 0));
            const int j = min(dir > 0 ? j0 + i : j1 - 1 - i, s.K - 1);
            yin[u] = s.q[((size_t)j * 2 + in_node) * N + n];
            yout[u] = s.q[((size_t)j * 2 + (1 - in_node)) * N + n];
            hh[u] = s.h[j];
            st[u] = s.sigma_t[j];
        }
    };
    load_batch(0);
    // fused: Vt staged, stopping-test references fetched for the tile GEMM,
    // the swept tile's padding columns cleared
    double pv[4][4];
    const int L1 = s.L1, R = 2 * (c1 - c0);
    const bool stop = fused && s.mom_ref != nullptr;
    if constexpr (fused) {
        stage_block<NP>(Vs, NP, L1, [&](int r, int c) { return s.mom_Vt[(size_t)min(r, N - 1) * L1 + c]; });
        const double *ref = stop ? s.mom_ref : s.mom_out;  // a valid address either way
        tile_prefetch<NP>(R, L1, pv, [&](int row, int col) { return ref[((size_t)c0 * 2 + row) * L1 + col]; });
        for (int idx = t; idx < R * (NP - N); idx += 256)
            pt[(idx / (NP - N)) * ldp + N + idx % (NP - N)] = 0.0;
    }
    double x;
    if (inkernel_carry) {
        // tiles before this one in sweep order, split into S contiguous runs,
        // folded in batches of 16
        const int P = dir > 0 ? tile : s.ntiles - 1 - tile;
        const int Q = (P + S - 1) / S;
        double A = 1.0, B = 0.0;
        if (live) {
            const int i0 = sc * Q, i1 = min(P, i0 + Q);
            for (int i = i0; i < i1; i += 16) {
                double a[16], b[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int ii = min(i + u, i1 - 1);
                    const int tt = dir > 0 ? ii : s.ntiles - 1 - ii;
                    a[u] = s.tileA[(size_t)tt * N + n];
                    b[u] = s.tileB[(size_t)tt * N + n];
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    if (i + u < i1) {
                        B = a[u] * B + b[u];
                        A = a[u] * A;
                    }
                }
            }
        }
        shA[t] = A;
        shB[t] = B;
        subA[t] = sa;
        subB[t] = sb;
        __syncthreads();
        x = boundary_inflow(s, n, adjoint);
        for (int i = 0; i < S; ++i) x = shA[i * N + n] * x + shB[i * N + n];
        if (live && sc == 0 && s.exit && P == s.ntiles - 1) {
            // last tile in sweep order: its outflow is the far-face exit flux
            const double TA = s.tileA[(size_t)tile * N + n], TB = s.tileB[(size_t)tile * N + n];
            s.exit[n] = TA * x + TB;
        }
    } else {
        subA[t] = sa;
        subB[t] = sb;
        __syncthreads();
        x = s.carry[(size_t)tile * N + n];
    }
    if (live) {
        if (dir > 0) {
            for (int i = 0; i < sc; ++i) x = subA[i * N + n] * x + subB[i * N + n];
        } else {
            for (int i = S - 1; i > sc; --i) x = subA[i * N + n] * x + subB[i * N + n];
        }
        for (int i0 = 0; i0 < len; i0 += SWEEP_BATCH) {
            if (i0 > 0) load_batch(i0);
#pragma unroll
            for (int u = 0; u < SWEEP_BATCH; ++u) {
                if (i0 + u < len) {
                    const int j = dir > 0 ? j0 + i0 + u : j1 - 1 - i0 - u;
                    const size_t iin = ((size_t)j * 2 + in_node) * N + n;
                    const size_t iout = ((size_t)j * 2 + (1 - in_node)) * N + n;
                    const CellCoef c = cell_coef(inv, hh[u], st[u], yin[u], yout[u], adjoint);
                    const double vout = c.a * x + c.b;
                    const double vin =
                        ((6.0 + 4.0 * c.tau) * (c.gin + x) - (6.0 + 2.0 * c.tau) * c.gout) * c.den_inv;
                    if (adjoint) {
                        // x = (h/(6|mu|)) [[2,1],[1,2]] zeta  (node order in/out is symmetric)
                        const double f = hh[u] * inv * (1.0 / 6.0);
                        s.psi[iin] = f * (2.0 * vin + vout);
                        s.psi[iout] = f * (vin + 2.0 * vout);
                    } else {
                        if (s.write_psi) {
                            s.psi[iin] = vin;
                            s.psi[iout] = vout;
                        }
                        if constexpr (fused) {
                            pt[((j - c0) * 2 + in_node) * ldp + n] = vin;
                            pt[((j - c0) * 2 + (1 - in_node)) * ldp + n] = vout;
                        }
                    }
                    x = vout;
                }
            }
        }
    }
    if constexpr (fused) {
        // moments of the tile (and the stopping test) on the swept values;
        // rows of Vs past N hold Vt's last row: zero them first
        for (int idx = t; idx < (NP - N) * NP; idx += 256) Vs[(N + idx / NP) * ldp + idx % NP] = 0.0;
        __syncthreads();
        unsigned long long dmax = 0ull;
        tile_gemm<NP>(pt, R, Vs, L1, pv, [&](int row, int col, double v, double rv) {
            s.mom_out[((size_t)c0 * 2 + row) * L1 + col] = v;
            if (stop) {
                const unsigned long long d = absdiff_bits(v, rv);
                dmax = d > dmax ? d : dmax;
            }
        });
        if (stop) stop_block_reduce(dmax, s.mom_slot);
    }
}

template <int NP>
__global__ void __launch_bounds__(256) sweep_apply(SweepArgs s, bool adjoint, bool inkernel_carry) {
    sweep_apply_body<NP>(s, adjoint, inkernel_carry, (int)blockIdx.x, (int)blockIdx.y);
}

template <int NP>
__global__ void __launch_bounds__(256) sweep_apply_multi(const MultiEntry<SweepArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<SweepArgs> &e = E[r.entry];
    SweepArgs a = e.a;
    apply_patch(a, e.p, *iter);
    sweep_apply_body<NP>(a, false, e.flag != 0, r.local, 0);
}


int sweep_shapes(const SweepArgs &s, LaunchShape out[4]) {
    const bool ink = s.ntiles <= SWEEP_INKERNEL_TILES;
    const int np = (s.src_phi || s.mom_out) ? fuse_width(s.N, s.L1, s.TC) : 0;
    int k = 0;
    LaunchShape a;
    a.kernel = MK_SWEEP_AGG;
    a.kid = KID_SWEEP_AGGREGATE;
    a.gx = s.ntiles;
    if (np > 0 && s.src_phi) {
        a.v1 = np;
        a.lds = (unsigned)(fused_aggregate_lds(s, np) * sizeof(double));
    }
    out[k++] = a;
    if (!ink) {
        LaunchShape g;
        g.kernel = MK_SCAN_GROUPS;
        g.kid = KID_SWEEP_SCAN;
        g.gx = (s.N + 63) / 64;
        g.gy = (s.ntiles + SCAN_GROUP - 1) / SCAN_GROUP;
        g.block = 64;
        out[k++] = g;
        g.kernel = MK_SCAN_CARRY;
        out[k++] = g;
    }
    LaunchShape p;
    p.kernel = MK_SWEEP_APPLY;
    p.kid = KID_SWEEP_APPLY;
    p.gx = s.ntiles;
    p.v2 = ink ? 1 : 0;
    if (np > 0 && s.mom_out) {
        p.v1 = np;
        p.lds = (unsigned)(fused_apply_lds(s, np) * sizeof(double));
    }
    out[k++] = p;
    return k;
}

template <int NP>
static void launch_sweep_agg(const LaunchShape &sh, const SweepArgs &s, bool adjoint, hipStream_t st,
                             KernelTimer *t) {
    LAUNCH(sh.kid, t, sweep_aggregate<NP>, dim3(sh.gx), dim3(256), sh.lds, st, s, adjoint);
}
template <int NP>
static void launch_sweep_app(const LaunchShape &sh, const SweepArgs &s, bool adjoint, hipStream_t st,
                             KernelTimer *t) {
    LAUNCH(sh.kid, t, sweep_apply<NP>, dim3(sh.gx), dim3(256), sh.lds, st, s, adjoint, sh.v2 != 0);
}

void launch_sweep(const SweepArgs &s0, bool adjoint, hipStream_t st, KernelTimer *t) {
    if (s0.K <= 0) return;
    SweepArgs s = s0;
    if (adjoint) {  // the transposed sweep carries no fused GEMMs
        s.src_phi = nullptr;
        s.mom_out = nullptr;
    }
    LaunchShape sh[4];
    const int n = sweep_shapes(s, sh);
    for (int i = 0; i < n; ++i) {
        const LaunchShape &x = sh[i];
        switch (x.kernel) {
            case MK_SWEEP_AGG:
                switch (x.v1) {
                    case 16: launch_sweep_agg<16>(x, s, adjoint, st, t); break;
                    case 32: launch_sweep_agg<32>(x, s, adjoint, st, t); break;
                    case 64: launch_sweep_agg<64>(x, s, adjoint, st, t); break;
                    default: launch_sweep_agg<0>(x, s, adjoint, st, t); break;
                }
                break;
            case MK_SCAN_GROUPS:
                LAUNCH(x.kid, t, sweep_scan_groups, dim3(x.gx, x.gy), dim3(64), 0, st, s, adjoint);
                break;
            case MK_SCAN_CARRY:
                LAUNCH(x.kid, t, sweep_scan_carry, dim3(x.gx, x.gy), dim3(64), 0, st, s, adjoint);
                break;
            default:
                switch (x.v1) {
                    case 16: launch_sweep_app<16>(x, s, adjoint, st, t); break;
                    case 32: launch_sweep_app<32>(x, s, adjoint, st, t); break;
                    case 64: launch_sweep_app<64>(x, s, adjoint, st, t); break;
                    default: launch_sweep_app<0>(x, s, adjoint, st, t); break;
                }
                break;
        }
    }
}

// ---------------------------------------------------------------------------
// Stopping test (eq:iterate): hist[it-1] = max_i |a_i - b_i| as the IEEE bit
// pattern of a non-negative double (ordered like unsigned integers; NaN
// sorts above +Inf, so a NaN anywhere surfaces as NaN).  The last block to
// finish evaluates the test and sets the convergence flag.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void stopping_test_body(const double *a, const double *b, size_t n,
                                                   unsigned long long *slot, SkipTest skip, int bx, int nbx) {
    if (skipped(skip)) return;
    unsigned long long m = 0ull;
    const size_t stride = (size_t)nbx * blockDim.x;
    for (size_t i0 = (size_t)bx * blockDim.x + threadIdx.x; i0 < n; i0 += 8 * stride) {
        double x[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const size_t i = min(i0 + u * stride, n - 1);
            x[u] = a[i];
            y[u] = b[i];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const unsigned long long v = absdiff_bits(x[u], y[u]);
            m = v > m ? v : m;
        }
    }
    stop_block_reduce(m, slot);
}

__global__ void __launch_bounds__(256) stopping_test(const double *a, const double *b, size_t n,
                                                     unsigned long long *slot, SkipTest skip) {
    stopping_test_body(a, b, n, slot, skip, (int)blockIdx.x, (int)gridDim.x);
}

__global__ void __launch_bounds__(256) stopping_test_multi(const MultiEntry<StopArgs> *E, const BlockRef *br,
                                                           const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<StopArgs> &e = E[r.entry];
    StopArgs a = e.a;
    apply_patch(a, e.p, *iter);
    stopping_test_body(a.a, a.b, a.n, a.slot, a.skip, r.local, e.gx);
}

__global__ void solve_reset(unsigned long long *hist, int max_iter) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < max_iter) hist[i] = 0ull;
}

void launch_solve_reset(unsigned long long *hist, int max_iter, hipStream_t s) {
    const int n = std::max(max_iter, 1);
    hipLaunchKernelGGL(solve_reset, dim3((n + 255) / 256), dim3(256), 0, s, hist, max_iter);
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point (fpsa_correct_noalloc): one
// fixed array per device, resident from the code object's load until the
// process ends.  Host code never passes the array's name to a kernel (that
// is a host-side stand-in, not a device address): scratch_attach resolves
// the device address once per device, with that device current, and every
// later use goes through scratch_device_ptr.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
double *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mutex;
}  // namespace

hipError_t scratch_attach(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double *>(p);
    return hipSuccess;
}

double *scratch_device_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch_ptr[device];
}

LaunchShape stop_shape(size_t n) {
    LaunchShape sh;
    sh.kernel = MK_STOP;
    sh.kid = KID_ABSDIFF;
    sh.gx = (int)std::max<size_t>(1, std::min<size_t>((n + 2047) / 2048, 256));
    return sh;
}

void launch_stopping_test(const double *a, const double *b, size_t n, unsigned long long *slot,
                          SkipTest skip, hipStream_t s, KernelTimer *t) {
    if (n == 0) return;
    const LaunchShape sh = stop_shape(n);
    LAUNCH(sh.kid, t, stopping_test, dim3(sh.gx), dim3(256), 0, s, a, b, n, slot, skip);
}

// ---------------------------------------------------------------------------
// Fokker-Planck interface recurrences (see setup_math.hpp):
//   forward  p_{j+1} = G_j p_j + f_j,  f_j = Hm_j s-_j + s+_j,   p_0 = 0
//   backward b_j = U_j b_{j+1} + g_j,  g_j = Y_j p_j + X_j s-_j,  b_K = 0
//            a_j = rho_j b_j + p_j
// Cells are cut into chunks.  The only dependent chain is fp_chain, which
// runs every chunk from a zero carry (all chunks in parallel) and records
// the local values and the chunk's end value.  fp_carry then forms each
// chunk's true carry-in as a sum of independent matvecs with the
// precomputed chunk transfer products, and fp_fixup adds the carry's
// contribution through the precomputed within-chunk prefix products and
// applies the next matvec (g_j, or a_j and the inflow vector) in the same
// pass.  Every kernel is instantiated for a padded row length NHP (a power
// of two >= NH) so its loads can be issued together before the FMAs that
// consume them.
// ---------------------------------------------------------------------------

// sum_c M[r][c] x[c] for a transposed NH x NH matrix: MT points at element
// (r, 0), consecutive columns are NH apart.  Loads of a batch of up to 32
// columns are all issued before the first FMA.
template <int NHP>
__device__ __forceinline__ double tdot(const double *__restrict__ MT, const double *__restrict__ x, int NH) {
    constexpr int BT = NHP < 32 ? NHP : (NHP > 64 ? 16 : 32);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c0 = 0; c0 < NHP; c0 += BT) {
        double m[BT], xv[BT];
#pragma unroll
        for (int c = 0; c < BT; ++c) {
            const int cc = min(c0 + c, NH - 1);
            m[c] = MT[(size_t)cc * NH];
            xv[c] = x[cc];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < BT; ++c) s[c & 3] = fma(c0 + c < NH ? m[c] : 0.0, xv[c], s[c & 3]);
    }
    return (s[0] + s[1]) + (s[2] + s[3]);
}

// Additive terms of both eliminations, one thread per (direction, cell, row):
// f_j = Hm_j s-_j + s+_j (forward) and g_j = Hb_j s+_j + s-_j (backward).
template <int NHP>
__device__ __forceinline__ void fp_matvec_body(FPArgs f, const int bx_, const int by_) {
    if (skipped(f.skip)) return;
    const int NH = f.NH, N = 2 * NH;
    const size_t M2 = (size_t)NH * NH;
    const size_t per = (size_t)f.K * NH;
    size_t gid = (size_t)bx_ * blockDim.x + threadIdx.x;
    if (gid >= 2 * per) return;
    const bool fwd = gid < per;
    if (!fwd) gid -= per;
    const int j = (int)(gid / NH), r = (int)(gid % NH);
    const double *Mt = f.cellmats + (size_t)j * FP_CELLMATS * M2 + (fwd ? 1 : 3) * M2 + r;
    const double *sj = f.s + (size_t)j * N;
    const double *x = fwd ? sj + NH : sj;      // s- or s+
    const double add = fwd ? sj[r] : sj[NH + r];
    (fwd ? f.fvec : f.gvec)[(size_t)j * NH + r] = tdot<NHP>(Mt, x, NH) + add;
}

template <int NHP>
__global__ void __launch_bounds__(256) fp_matvec(FPArgs f) {
    fp_matvec_body<NHP>(f, (int)blockIdx.x, (int)blockIdx.y);
}

template <int NHP>
__global__ void __launch_bounds__(256) fp_matvec_multi(const MultiEntry<FPArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<FPArgs> &e = E[r.entry];
    FPArgs a = e.a;
    apply_patch(a, e.p, *iter);
    fp_matvec_body<NHP>(a, r.local, 0);
}


// Moment-difference rows [c0, c0 + nrows) of a slab's [K][L2] arrays staged
// for the fused source: As[r][k] = (half - old) [.* sigma] at row stride
// LDA.  Each thread issues the loads of a batch of eight elements before it
// stores any, so a block waits on memory once per batch.
__device__ __forceinline__ void stage_diff_rows(const FPArgs &f, int c0, int nrows, double *As, int LDA) {
    const int L2 = f.L2, n = nrows * L2;
    const bool sig = f.src_sigma != nullptr;
    for (int base = 0; base < n; base += 256 * 8) {
        double h[8], o[8], sg[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = min(base + (int)threadIdx.x + 256 * u, n - 1);
            const size_t g = (size_t)c0 * L2 + e;
            h[u] = f.src_half[g];
            o[u] = f.src_old[g];
            sg[u] = sig ? f.src_sigma[g] : 1.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + (int)threadIdx.x + 256 * u;
            if (e < n) As[(e / L2) * LDA + e % L2] = sig ? (h[u] - o[u]) * sg[u] : h[u] - o[u];
        }
    }
}

// acc[t] += A x B over the k range [0, KP) for NT 16 x 16 output tiles that
// share their 16 rows: A's row for this lane at Ar (LDS, zero past the data,
// KP a multiple of 4), B element (k, column t) from getb (global memory,
// cached).  B fragments are fetched one batch of BK k-steps ahead of the
// MFMAs that use them, so the fetch latency overlaps the products.
template <int NT, class GetB>
__device__ __forceinline__ void mfma_rows_gb(const double *Ar, int KP, GetB &&getb, d4 (&acc)[NT]) {
    constexpr int BK = 8;
    const int kl = (threadIdx.x & 63) >> 4;
    double bc[NT][BK], bn[NT][BK];
    auto fetch = [&](int k0, double (&dst)[NT][BK]) {
#pragma unroll
        for (int u = 0; u < BK; ++u) {
            const int k = min(k0 + 4 * u + kl, KP - 1);
#pragma unroll
            for (int t = 0; t < NT; ++t) dst[t][u] = getb(k, t);
        }
    };
    fetch(0, bc);
    for (int k0 = 0; k0 < KP; k0 += 4 * BK) {
        if (k0 + 4 * BK < KP) fetch(k0 + 4 * BK, bn);
#pragma unroll
        for (int u = 0; u < BK; ++u) {
            if (k0 + 4 * u < KP) {
                const double a = Ar[k0 + 4 * u + kl];
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bc[t][u], acc[t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int u = 0; u < BK; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) bc[t][u] = bn[t][u];
    }
}

// Fused source and additive terms (FPArgs::src_half set): a block of
// CPB = 256 / NHP cells forms their source rows s_j = (phi_half_j -
// phi_old_j) [.* sigma_j] x E on FP64 MFMA (the difference rows staged in
// LDS, zero-padded to RT * 16 rows and to a multiple of 4 columns; E
// fragments read from global memory, where every block finds them in
// cache), keeps them in LDS, and then forms f_j and g_j as fp_matvec does,
// thread (cell, row) both of them.
template <int NHP>
__device__ __forceinline__ void fp_matvec_src_body(FPArgs f, const int bx_) {
    if (skipped(f.skip)) return;
    constexpr int CPB = 256 / NHP, RT = (CPB + 15) / 16;
    extern __shared__ double fsm[];
    const int NH = f.NH, N = 2 * NH, L2 = f.L2, KP = (L2 + 3) & ~3, LDA = KP + 1;
    const size_t M2 = (size_t)NH * NH;
    double *As = fsm;                               // [RT * 16][LDA]
    double *Ss = fsm + (size_t)RT * 16 * LDA;       // [CPB][N]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j0 = bx_ * CPB, nc = min(CPB, f.K - j0);
    // zero padding (rows past the block's cells, columns L2 .. KP - 1), then
    // the data rows
    for (int idx = tid; idx < RT * 16 * KP; idx += 256) {
        const int r = idx / KP, k = idx % KP;
        if (r >= nc || k >= L2) As[r * LDA + k] = 0.0;
    }
    stage_diff_rows(f, j0, nc, As, LDA);
    __syncthreads();
    const int nct = (N + 15) / 16, kl = lane >> 4;
    for (int tt = wave; tt < RT * nct; tt += 4) {
        const int rt = tt / nct, col = (tt % nct) * 16 + (lane & 15), colc = min(col, N - 1);
        d4 acc[1] = {d4{0.0, 0.0, 0.0, 0.0}};
        mfma_rows_gb<1>(As + (rt * 16 + (lane & 15)) * LDA, KP,
                        [&](int k, int) { return f.src_E[(size_t)min(k, L2 - 1) * N + colc]; }, acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = rt * 16 + kl + 4 * r;
            if (row < CPB && col < N) Ss[row * N + col] = acc[0][r];
        }
    }
    __syncthreads();
    const int jl = tid / NHP, r = tid % NHP;
    if (jl >= nc || r >= NH) return;
    const int j = j0 + jl;
    const double *sj = Ss + jl * N;
    const double *cm = f.cellmats + (size_t)j * FP_CELLMATS * M2 + r;
    f.fvec[(size_t)j * NH + r] = tdot<NHP>(cm + M2, sj + NH, NH) + sj[r];
    f.gvec[(size_t)j * NH + r] = tdot<NHP>(cm + 3 * M2, sj, NH) + sj[NH + r];
}

template <int NHP>
__global__ void __launch_bounds__(256) fp_matvec_src(FPArgs f) {
    fp_matvec_src_body<NHP>(f, (int)blockIdx.x);
}

// One chain step for lane r with a runtime row length (NH > 64 path); the
// matrix is stored transposed, so row r is strided by NH.
__device__ __forceinline__ double chain_row(const double *Mcol, const double *v, double a, int NH) {
    double s0 = a, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int c = 0;
    for (; c + 3 < NH; c += 4) {
        s0 = fma(Mcol[(size_t)c * NH], v[c], s0);
        s1 = fma(Mcol[(size_t)(c + 1) * NH], v[c + 1], s1);
        s2 = fma(Mcol[(size_t)(c + 2) * NH], v[c + 2], s2);
        s3 = fma(Mcol[(size_t)(c + 3) * NH], v[c + 3], s3);
    }
    for (; c < NH; ++c) s0 = fma(Mcol[(size_t)c * NH], v[c], s0);
    return (s0 + s1) + (s2 + s3);
}

// Staged chain for small or padded NH (NH <= NHP, NHP a power of two <= 64).
// Step matrices (stored transposed) are zero-padded to NHP x NHP in LDS with
// stride NHP+1, so lane r's reads of row r are conflict-free.  Wave 0 runs
// the chain on one LDS buffer while waves 1-3 fill the other with the next
// B steps; index math is compile-time and each producer issues all of its
// loads before it writes any of them.
template <int NHP>
struct ChainGeom {
    static constexpr int LD = NHP + 1;
    static constexpr int MS = NHP * LD + NHP;       // doubles per step in LDS
    static constexpr int PER = NHP * NHP + NHP;     // elements per step
    static constexpr int PER2 = PER / 2;            // 16-byte pairs per step
    static constexpr int B0 = (18432 - 2 * NHP) / (2 * MS);
    static constexpr int B = B0 < 1 ? 1 : (B0 > 64 ? 64 : B0);
    static constexpr int PRODUCERS = 192;
    static constexpr int U = (B * PER + PRODUCERS - 1) / PRODUCERS;    // scalar loads
    static constexpr int U2 = (B * PER2 + PRODUCERS - 1) / PRODUCERS;  // pair loads
};

// One chain step of lane r: a + sum_c M[r][c] v[c] with M^T in LDS at
// stride LDT (Mcol = &M^T[0][r]), the column entries and the vector read in
// full before the FMAs.
template <int NHP, int LDT>
__device__ __forceinline__ double chain_row_t(const double *Mcol, const double *v, double a) {
    constexpr int BT = NHP < 32 ? NHP : (NHP > 64 ? 16 : 32);
    double s[4] = {a, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c0 = 0; c0 < NHP; c0 += BT) {
        double m[BT], x[BT];
#pragma unroll
        for (int c = 0; c < BT; ++c) {
            m[c] = Mcol[(c0 + c) * LDT];
            x[c] = v[c0 + c];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < BT; ++c) s[c & 3] = fma(m[c], x[c], s[c & 3]);
    }
    return (s[0] + s[1]) + (s[2] + s[3]);
}

// Chain kernels run both eliminations in one grid of 2 * nchunks blocks:
// blocks [0, nchunks) the forward chunks, the rest the backward ones.
__device__ __forceinline__ int chain_dir(const FPArgs &f, int bx, int &c) {
    const int forward = bx < f.nchunks;
    c = forward ? bx : bx - f.nchunks;
    return forward;
}

template <int NHP, bool EXACT>
__device__ __forceinline__ void fp_chain_staged_body(FPArgs f, const int bx_, const int by_) {
    using G = ChainGeom<NHP>;
    if (skipped(f.skip)) return;
    __shared__ double buf[2][G::B * G::MS];
    __shared__ __attribute__((aligned(16))) double vec[2][NHP];
    const int NH = f.NH;
    int c;
    const int forward = chain_dir(f, bx_, c);
    const int j0 = c * f.chunk, j1 = min(f.K, j0 + f.chunk);
    const int T = j1 - j0;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid < 2 * NHP) vec[tid / NHP][tid % NHP] = 0.0;
    const int nsub = (T + G::B - 1) / G::B;
    const double *cell_M = f.cellmats + (forward ? 0 : 2) * (size_t)NH * NH;
    const double *cell_a = forward ? f.fvec : f.gvec;

    // cell of step t of this chunk
    auto cell_of = [&](int t) { return forward ? j0 + t : j1 - 1 - t; };

    // producers (tid 64..255) copy the steps of block sb into dst; steps past
    // the end of the chunk repeat its last step (never consumed)
    auto stage = [&](int sb, double *dst) {
        const int p = tid - 64;
        const int tb = sb * G::B;
        const int last = min(G::B, T - tb) - 1;
        if constexpr (EXACT) {
            double2 v[G::U2];
            int off[G::U2];
#pragma unroll
            for (int u = 0; u < G::U2; ++u) {
                const int e = min(p + u * G::PRODUCERS, G::B * G::PER2 - 1);
                const int k = e / G::PER2, w2 = e % G::PER2;
                const int j = cell_of(tb + min(k, last));
                const bool mat = w2 < NHP * NHP / 2;
                const double *src = mat ? cell_M + (size_t)j * FP_CELLMATS * NHP * NHP + 2 * w2
                                        : cell_a + (size_t)j * NHP + 2 * (w2 - NHP * NHP / 2);
                v[u] = *reinterpret_cast<const double2 *>(src);
                off[u] = k * G::MS + (mat ? (2 * w2 / NHP) * G::LD + (2 * w2) % NHP
                                          : NHP * G::LD + 2 * (w2 - NHP * NHP / 2));
            }
#pragma unroll
            for (int u = 0; u < G::U2; ++u) {
                dst[off[u]] = v[u].x;
                dst[off[u] + 1] = v[u].y;
            }
        } else {
            double v[G::U];
            int off[G::U];
            const size_t M2 = (size_t)NH * NH;
#pragma unroll
            for (int u = 0; u < G::U; ++u) {
                const int e = min(p + u * G::PRODUCERS, G::B * G::PER - 1);
                const int k = e / G::PER, w = e % G::PER;
                const int j = cell_of(tb + min(k, last));
                const bool mat = w < NHP * NHP;
                const int r = w / NHP, col = w % NHP, vi = w - NHP * NHP;
                const bool valid = mat ? (r < NH && col < NH) : (vi < NH);
                const int rr = min(r, NH - 1), c2 = min(col, NH - 1), v2 = min(max(vi, 0), NH - 1);
                // LDS (r, col) <- M^T[r][col], stored at r * NH + col
                const double *src = mat ? cell_M + (size_t)j * FP_CELLMATS * M2 + (size_t)rr * NH + c2
                                        : cell_a + (size_t)j * NH + v2;
                v[u] = *src;
                v[u] = valid ? v[u] : 0.0;
                off[u] = k * G::MS + (mat ? r * G::LD + col : NHP * G::LD + vi);
            }
#pragma unroll
            for (int u = 0; u < G::U; ++u) dst[off[u]] = v[u];
        }
    };

    if (wave != 0 && nsub > 0) stage(0, buf[0]);
    __syncthreads();
    int cur = 0;
    for (int sb = 0; sb < nsub; ++sb) {
        if (wave != 0) {
            if (sb + 1 < nsub) stage(sb + 1, buf[(sb + 1) & 1]);
        } else {
            const int tb = sb * G::B, ns = min(G::B, T - tb);
            const double *base = buf[sb & 1];
            for (int k = 0; k < ns; ++k) {
                const double *M = base + k * G::MS;
                const int j = cell_of(tb + k);
                if (lane < NHP) {
                    const double *vc = vec[cur];
                    // forward: p_loc before the step; backward: b_loc after it
                    if (forward && lane < NH) f.pvec[(size_t)j * NH + lane] = vc[lane];
                    const double v = chain_row_t<NHP, G::LD>(M + lane, vc, M[NHP * G::LD + lane]);
                    vec[cur ^ 1][lane] = v;
                    if (!forward && lane < NH) f.bvec[(size_t)j * NH + lane] = v;
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                cur ^= 1;
            }
        }
        __syncthreads();
    }
    if (wave == 0 && lane < NH) (forward ? f.e_fwd : f.e_bwd)[(size_t)c * NH + lane] = vec[cur][lane];
}

template <int NHP, bool EXACT>
__global__ void __launch_bounds__(256) fp_chain_staged(FPArgs f) {
    fp_chain_staged_body<NHP, EXACT>(f, (int)blockIdx.x, (int)blockIdx.y);
}

template <int NHP, bool EXACT>
__global__ void __launch_bounds__(256) fp_chain_staged_multi(const MultiEntry<FPArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<FPArgs> &e = E[r.entry];
    FPArgs a = e.a;
    apply_patch(a, e.p, *iter);
    fp_chain_staged_body<NHP, EXACT>(a, r.local, 0);
}


// Ring-staged chain for NH == NHP in {8, 16, 32, 64}.  A chain step needs
// the step matrix (stored transposed, NHP*NHP doubles) and the additive
// vector (NHP doubles).  Waves 1-3 copy them straight into an LDS ring of R
// step slots with direct-to-LDS loads (global_load_lds_dwordx4: lane l of
// one instruction writes bytes [16 l, 16 l + 16) after the wave-uniform LDS
// base), keeping R-1 steps in flight, while wave 0 runs the chain out of the
// ring.  All four waves meet at one barrier per step.  Before that barrier a
// producer waits until the loads of the next step have landed: it issues the
// same, compile-time number of load instructions for every step (steps past
// the end of the chunk load 16 bytes per instruction into a free slot), so
// the wait is a fixed vmcnt.  The consumer's lanes split each row in
// 64 / NHP column groups and combine them with cross-lane shuffles.
template <int NHP>
struct RingGeom {
    static constexpr int SLOT = NHP * NHP + NHP;          // doubles per step
    static constexpr int PIECES = SLOT / 2;               // 16-byte pieces per step
    static constexpr int IMAX = (PIECES + 191) / 192;     // loads per producer wave per step
    static constexpr int RB = 153600 / (SLOT * 8);        // slots that fit in LDS
    static constexpr int RV = 63 / IMAX + 2;              // (R - 2) * IMAX <= 63 (vmcnt range)
    static constexpr int R0 = RB < RV ? RB : RV;
    static constexpr int R = R0 > 32 ? 32 : R0;
    static_assert(R >= 3, "ring too small");
    static constexpr int SPLIT = 64 / NHP;                // lanes per row
    static constexpr int CPL = NHP / SPLIT;               // columns per lane
};

// s_waitcnt vmcnt(n) with lgkmcnt and expcnt left alone (gfx9 encoding:
// vmcnt bits [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8]).
template <int n>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(n >= 0 && n <= 63, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14));
}

// s_barrier plus a compiler-only memory barrier (no fence instructions), so
// that no LDS access or LDS-bound load is moved across it.
__device__ __forceinline__ void ring_barrier() {
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void glb_void_t;

template <int NHP, int PW>
__device__ __forceinline__ void ring_producer(const FPArgs &f, int forward, int j0, int j1,
                                              double *ring) {
    using G = RingGeom<NHP>;
    constexpr int NI = (G::PIECES - PW * 64 + 191) / 192;  // this wave's loads per step
    const int lane = threadIdx.x & 63;
    const int T = j1 - j0;
    const size_t M2 = (size_t)NHP * NHP;
    const double *cell_M = f.cellmats + (forward ? 0 : 2) * M2;
    const double *cell_a = forward ? f.fvec : f.gvec;
    auto issue = [&](int t) {
        const int tc = t < T ? t : T - 1;
        const int j = forward ? j0 + tc : j1 - 1 - tc;
        double *slot = ring + (size_t)(t % G::R) * G::SLOT;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int base = k * 192 + PW * 64;       // first piece of this instruction
            const int i = base + lane;
            if (i < G::PIECES && (t < T || lane == 0)) {
                const double *src = i < NHP * NHP / 2 ? cell_M + (size_t)j * FP_CELLMATS * M2 + 2 * i
                                                      : cell_a + (size_t)j * NHP + 2 * (i - NHP * NHP / 2);
                __builtin_amdgcn_global_load_lds((glb_void_t *)src, (lds_void_t *)(slot + 2 * base), 16, 0, 0);
            }
        }
    };
#pragma unroll 1
    for (int t = 0; t < G::R; ++t) issue(t);
    if constexpr (NI > 0) wait_vmcnt<(G::R - 1) * NI>();
    ring_barrier();
#pragma unroll 1
    for (int s = 0; s < T; ++s) {
        if constexpr (NI > 0) wait_vmcnt<(G::R - 2) * NI>();
        ring_barrier();
        issue(s + G::R);
    }
    wait_vmcnt<0>();
}

template <int NHP>
__device__ __forceinline__ void fp_chain_ring_body(FPArgs f, const int bx_, const int by_) {
    using G = RingGeom<NHP>;
    if (skipped(f.skip)) return;
    __shared__ __attribute__((aligned(16))) double ring[G::R * G::SLOT];
    __shared__ double vec[2][NHP];
    int c;
    const int forward = chain_dir(f, bx_, c);
    const int j0 = c * f.chunk, j1 = min(f.K, j0 + f.chunk);
    const int T = j1 - j0;
    if (T <= 0) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave == 1) {
        ring_producer<NHP, 0>(f, forward, j0, j1, ring);
        return;
    }
    if (wave == 2) {
        ring_producer<NHP, 1>(f, forward, j0, j1, ring);
        return;
    }
    if (wave == 3) {
        ring_producer<NHP, 2>(f, forward, j0, j1, ring);
        return;
    }
    // wave 0: the chain
    const int r = lane % NHP, h = lane / NHP;
    if (lane < NHP) vec[0][lane] = 0.0;
    ring_barrier();
    int cur = 0;
#pragma unroll 1
    for (int s = 0; s < T; ++s) {
        const double *slot = ring + (size_t)(s % G::R) * G::SLOT;
        const int j = forward ? j0 + s : j1 - 1 - s;
        const double *vc = vec[cur];
        double m[G::CPL], x[G::CPL];
#pragma unroll
        for (int q = 0; q < G::CPL; ++q) {
            const int cc = h * G::CPL + q;
            m[q] = slot[cc * NHP + r];
            x[q] = vc[cc];
        }
        const double a = slot[NHP * NHP + r];
        const double vold = vc[r];
        __builtin_amdgcn_sched_barrier(0);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < G::CPL; ++q) acc[q & 3] = fma(m[q], x[q], acc[q & 3]);
        double v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
#pragma unroll
        for (int off = NHP; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
        v += a;
        if (h == 0) {
            // forward: p_loc before the step; backward: b_loc after it
            if (forward) f.pvec[(size_t)j * NHP + r] = vold;
            else f.bvec[(size_t)j * NHP + r] = v;
            vec[cur ^ 1][r] = v;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        cur ^= 1;
        ring_barrier();
    }
    if (lane < NHP) (forward ? f.e_fwd : f.e_bwd)[(size_t)c * NHP + lane] = vec[cur][lane];
}

template <int NHP>
__global__ void __launch_bounds__(256) fp_chain_ring(FPArgs f) {
    fp_chain_ring_body<NHP>(f, (int)blockIdx.x, (int)blockIdx.y);
}

template <int NHP>
__global__ void __launch_bounds__(256) fp_chain_ring_multi(const MultiEntry<FPArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<FPArgs> &e = E[r.entry];
    FPArgs a = e.a;
    apply_patch(a, e.p, *iter);
    fp_chain_ring_body<NHP>(a, r.local, 0);
}


// Runtime-NH chain (NH > 64): one wave, rows read from global memory.
__device__ __forceinline__ void fp_chain_any_body(FPArgs f, const int bx_, const int by_) {
    if (skipped(f.skip)) return;
    extern __shared__ double smem[];
    const int NH = f.NH;
    const size_t M2 = (size_t)NH * NH;
    int c;
    const int forward = chain_dir(f, bx_, c);
    const int j0 = c * f.chunk, j1 = min(f.K, j0 + f.chunk);
    const int lane = threadIdx.x;
    double *vec = smem;  // [2][NH]
    for (int r = lane; r < 2 * NH; r += 64) vec[r] = 0.0;
    __syncthreads();
    int cur = 0;
    for (int t = 0; t < j1 - j0; ++t) {
        const int j = forward ? j0 + t : j1 - 1 - t;
        const double *M = f.cellmats + (size_t)j * FP_CELLMATS * M2 + (forward ? 0 : 2) * M2;
        const double *a = (forward ? f.fvec : f.gvec) + (size_t)j * NH;
        const double *vc = vec + cur * NH;
        double *vn = vec + (cur ^ 1) * NH;
        for (int r = lane; r < NH; r += 64) {
            if (forward) f.pvec[(size_t)j * NH + r] = vc[r];
            const double v = chain_row(M + r, vc, a[r], NH);
            vn[r] = v;
            if (!forward) f.bvec[(size_t)j * NH + r] = v;
        }
        __syncthreads();
        cur ^= 1;
    }
    for (int r = lane; r < NH; r += 64) (forward ? f.e_fwd : f.e_bwd)[(size_t)c * NH + r] = vec[cur * NH + r];
}

__global__ void __launch_bounds__(64) fp_chain_any(FPArgs f) {
    fp_chain_any_body(f, (int)blockIdx.x, (int)blockIdx.y);
}

__global__ void __launch_bounds__(64) fp_chain_any_multi(const MultiEntry<FPArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<FPArgs> &e = E[r.entry];
    FPArgs a = e.a;
    apply_patch(a, e.p, *iter);
    fp_chain_any_body(a, r.local, 0);
}


// Chunk carry-ins.  Forward rows c = 0..P:  carry_c = e_{c-1} +
// sum_{c' <= c-2} ThF_{c,c'} e_{c'} (carry_0 = 0; carry_P = p_K).
// Backward rows c = 0..P-1:  carry'_c = e'_{c+1} + sum_{c' >= c+2}
// ThB_{c,c'} e'_{c'} (carry'_{P-1} = q_K = 0).
// Grid (row, part) with the P+1 forward rows first, then the P backward
// rows: a block sums up to GRP = 256/NHP of a row's transfer terms, one term
// per thread group, into a partial vector.  The partials and the identity
// term are added (in part order) by fp_fixup, after the kernel boundary has
// made them visible, so no block here waits for another.
__device__ __forceinline__ int carry_terms(int forward, int c, int P) {
    const int a = forward ? c : P - 1 - c;  // mirrored row index
    return a - 1 > 0 ? a - 1 : 0;
}

template <int NHP>
__device__ __forceinline__ void fp_carry_body(FPArgs f, const int bx_, const int by_) {
    if (skipped(f.skip)) return;
    constexpr int GRP = 256 / NHP;
    __shared__ double red[256];
    const int NH = f.NH, P = f.nchunks;
    const size_t M2 = (size_t)NH * NH;
    const int forward = (int)bx_ <= P;
    const int c = forward ? (int)bx_ : (int)bx_ - (P + 1), part = by_;
    const int a = forward ? c : P - 1 - c;
    const int nterms = carry_terms(forward, c, P);
    const int nparts = max(1, (nterms + GRP - 1) / GRP);
    if (part >= nparts) return;
    const int tid = threadIdx.x, r = tid % NHP, g = tid / NHP;
    const double *e = forward ? f.e_fwd : f.e_bwd;
    double acc = 0.0;
    const int ap = part * GRP + g;                  // mirrored c'
    if (r < NH && ap < nterms) {
        const size_t row0 = (size_t)(a - 1) * (a - 2) / 2;
        const int cp = forward ? ap : P - 1 - ap;
        const double *T = (forward ? f.theta_fwd : f.theta_bwd) + (row0 + ap) * M2 + r;
        acc = tdot<NHP>(T, e + (size_t)cp * NH, NH);
    }
    red[tid] = acc;
    __syncthreads();
    if (g == 0 && r < NH) {
        double sum = 0.0;
        for (int gg = 0; gg < GRP; ++gg) sum += red[gg * NHP + r];
        (forward ? f.part_f : f.part_b)[((size_t)c * f.carry_parts + part) * NH + r] = sum;
    }
}

template <int NHP>
__global__ void __launch_bounds__(256) fp_carry(FPArgs f) {
    fp_carry_body<NHP>(f, (int)blockIdx.x, (int)blockIdx.y);
}

template <int NHP>
__global__ void __launch_bounds__(256) fp_carry_multi(const MultiEntry<FPArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<FPArgs> &e = E[r.entry];
    FPArgs a = e.a;
    apply_patch(a, e.p, *iter);
    fp_carry_body<NHP>(a, r.local % e.gx, r.local / e.gx);
}


// carry of row c (see fp_carry): partial sums in part order + identity term
__device__ __forceinline__ double carry_value(const FPArgs &f, int forward, int c, int r) {
    const int P = f.nchunks, NH = f.NH;
    const int nterms = carry_terms(forward, c, P);
    int grp = 256;
    {
        int nhp = 2;
        while (nhp < NH) nhp *= 2;
        grp = 256 / nhp;
    }
    const int nparts = max(1, (nterms + grp - 1) / grp);
    const double *prow = (forward ? f.part_f : f.part_b) + (size_t)c * f.carry_parts * NH + r;
    // the chunk end value and eight partial sums at a time are requested
    // (clamped addresses) before any is added, so the sum costs one memory
    // round trip per eight parts instead of one per part
    const int a = forward ? c : P - 1 - c;
    const int ce = min(max(forward ? c - 1 : c + 1, 0), P - 1);
    const double e = (forward ? f.e_fwd : f.e_bwd)[(size_t)ce * NH + r];
    double sum = 0.0;
    for (int p0 = 0; p0 < nparts; p0 += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = prow[(size_t)min(p0 + u, nparts - 1) * NH];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (p0 + u < nparts) sum += v[u];
    }
    if (a >= 1) sum += e;
    return sum;
}

// Fix-up and combination at interface j (the left face of cell j), one
// thread per (cell, row), CPB = 256/NHP cells per block:
//   p_j = p_loc_j + PsiF_j carry_c(j),   q_j = q_loc_j + PsiB_j carry'_c(j)
//   a_j = W_j p_j + (W rho)_j q_j,       b_j = sig_j a_j + q_j
// The inflow of cell j is (a_j | b_{j+1}) with b_K = 0.  b_0 (into bvec[0])
// and a_K = p_K (into pvec[K]) are kept for the exit flux.  The prologue
// forms the carries of the chunks the block touches from fp_carry's partial
// sums; the vectors of a cell are shared through LDS.
template <int NHP>
__device__ __forceinline__ void fp_fixup_body(FPArgs f, const int bx_, const int by_) {
    if (skipped(f.skip)) return;
    constexpr int CPB = 256 / NHP;
    constexpr int CMAX = CPB / 4 + 2;               // chunks per block (chunk >= 4)
    __shared__ double psh[CPB][NHP], qsh[CPB][NHP], ash[CPB][NHP];
    __shared__ double cfs[CMAX + 1][NHP], cbs[CMAX][NHP];
    const int NH = f.NH, N = 2 * NH;
    const size_t M2 = (size_t)NH * NH;
    const int tid = threadIdx.x, jl = tid / NHP, r = tid % NHP;
    const int jfirst = bx_ * CPB, jlast = min(f.K, jfirst + CPB) - 1;
    const int c_lo = jfirst / f.chunk, c_hi = jlast / f.chunk;
    const int nc = c_hi - c_lo + 1;
    const bool last_block = jlast == f.K - 1;
    for (int idx = tid; idx < (nc + 1) * NH; idx += blockDim.x) {
        const int k = idx / NH, rr = idx % NH;
        if (k < nc) {
            cfs[k][rr] = carry_value(f, 1, c_lo + k, rr);
            cbs[k][rr] = carry_value(f, 0, c_lo + k, rr);
        } else if (last_block) {
            cfs[nc][rr] = carry_value(f, 1, f.nchunks, rr);  // p_K
        }
    }
    __syncthreads();
    const int j = jfirst + jl;
    const bool live = j < f.K && r < NH;
    const double *cm = f.cellmats + (size_t)j * FP_CELLMATS * M2 + r;
    double q = 0.0;
    if (live) {
        const int k = j / f.chunk - c_lo;
        const double p = f.pvec[(size_t)j * NH + r] + tdot<NHP>(f.psi_fwd + (size_t)j * M2 + r, cfs[k], NH);
        q = f.bvec[(size_t)j * NH + r] + tdot<NHP>(f.psi_bwd + (size_t)j * M2 + r, cbs[k], NH);
        psh[jl][r] = p;
        qsh[jl][r] = q;
    }
    __syncthreads();
    double a = 0.0;
    if (live) {
        a = tdot<NHP>(cm + 4 * M2, psh[jl], NH) + tdot<NHP>(cm + 5 * M2, qsh[jl], NH);
        ash[jl][r] = a;
    }
    __syncthreads();
    if (!live) return;
    const double b = tdot<NHP>(cm + 6 * M2, ash[jl], NH) + q;
    f.inflow[(size_t)j * N + r] = a;
    if (j >= 1) f.inflow[(size_t)(j - 1) * N + NH + r] = b;
    if (j == f.K - 1) {
        f.inflow[(size_t)j * N + NH + r] = 0.0;
        f.pvec[(size_t)f.K * NH + r] = cfs[nc][r];
    }
    if (j == 0) f.bvec[r] = b;
}

template <int NHP>
__global__ void __launch_bounds__(256) fp_fixup(FPArgs f) {
    fp_fixup_body<NHP>(f, (int)blockIdx.x, (int)blockIdx.y);
}

template <int NHP>
__global__ void __launch_bounds__(256) fp_fixup_multi(const MultiEntry<FPArgs> *E, const BlockRef *br, const int *iter) {
    const BlockRef r = br[blockIdx.x];
    const MultiEntry<FPArgs> &e = E[r.entry];
    FPArgs a = e.a;
    apply_patch(a, e.p, *iter);
    fp_fixup_body<NHP>(a, r.local, 0);
}

int fp_carry_parts(int nchunks, int NH) {
    int nhp = 2;
    while (nhp < NH) nhp *= 2;
    const int grp = 256 / nhp;
    return std::max(1, (std::max(nchunks - 1, 0) + grp - 1) / grp);
}

// padded row length of the recurrences' kernels
static int fp_nhp(int NH) {
    int nhp = 2;
    while (nhp < NH && nhp < 128) nhp *= 2;
    return nhp;
}

void fp_shapes(const FPArgs &f, LaunchShape out[4]) {
    const int NHP = fp_nhp(f.NH);
    LaunchShape m;
    m.kernel = MK_FP_MATVEC;
    m.v1 = NHP;
    m.kid = KID_FP_MATVEC;
    m.gx = (int)((2 * (size_t)f.K * f.NH + 255) / 256);
    LaunchShape c;
    c.kernel = MK_FP_CHAIN;
    c.v1 = NHP;
    c.kid = KID_FP_CHAIN;
    c.gx = 2 * f.nchunks;
    if (NHP >= 8 && NHP <= 64) {
        c.v2 = f.NH == NHP ? 0 : 2;
    } else if (NHP <= 64) {
        c.v2 = f.NH == NHP ? 1 : 2;
    } else {
        c.v2 = 3;
        c.block = 64;
        c.lds = (unsigned)(2 * f.NH * sizeof(double));
    }
    LaunchShape k;
    k.kernel = MK_FP_CARRY;
    k.v1 = NHP;
    k.kid = KID_FP_CARRY;
    k.gx = 2 * f.nchunks + 1;
    k.gy = f.carry_parts;
    LaunchShape x;
    x.kernel = MK_FP_FIXUP;
    x.v1 = NHP;
    x.kid = KID_FP_FIXUP;
    x.gx = (f.K + 256 / NHP - 1) / (256 / NHP);
    if (f.src_half) {
        // fused source: CPB cells per block, A rows and source rows in LDS
        const int cpb = 256 / NHP, rt = (cpb + 15) / 16, kp = (f.L2 + 3) & ~3;
        m.v2 = 1;
        m.gx = (f.K + cpb - 1) / cpb;
        m.lds = (unsigned)(((size_t)rt * 16 * (kp + 1) + (size_t)cpb * 2 * f.NH) * sizeof(double));
    }
    out[0] = m;
    out[1] = c;
    out[2] = k;
    out[3] = x;
}

bool fp_fusable(int NH, int L2) {
    const int nhp = fp_nhp(NH);
    return nhp >= 8 && nhp <= 64 && L2 >= 2 && L2 <= 256;
}

template <int NHP>
static void fp_launch_all(const LaunchShape (&sh)[4], const FPArgs &f, hipStream_t s, KernelTimer *t) {
    if constexpr (NHP >= 8 && NHP <= 64) {
        if (sh[0].v2 == 1)
            LAUNCH(sh[0].kid, t, fp_matvec_src<NHP>, dim3(sh[0].gx), dim3(256), sh[0].lds, s, f);
        else
            LAUNCH(sh[0].kid, t, fp_matvec<NHP>, dim3(sh[0].gx), dim3(256), 0, s, f);
    } else {
        LAUNCH(sh[0].kid, t, fp_matvec<NHP>, dim3(sh[0].gx), dim3(256), 0, s, f);
    }
    const dim3 ch_grid(sh[1].gx);
    if constexpr (NHP >= 8 && NHP <= 64) {
        if (sh[1].v2 == 0)
            LAUNCH(sh[1].kid, t, fp_chain_ring<NHP>, ch_grid, dim3(256), 0, s, f);
        else
            LAUNCH(sh[1].kid, t, (fp_chain_staged<NHP, false>), ch_grid, dim3(256), 0, s, f);
    } else if constexpr (NHP <= 64) {
        if (sh[1].v2 == 1)
            LAUNCH(sh[1].kid, t, (fp_chain_staged<NHP, true>), ch_grid, dim3(256), 0, s, f);
        else
            LAUNCH(sh[1].kid, t, (fp_chain_staged<NHP, false>), ch_grid, dim3(256), 0, s, f);
    } else {
        LAUNCH(sh[1].kid, t, fp_chain_any, ch_grid, dim3(64), sh[1].lds, s, f);
    }
    LAUNCH(sh[2].kid, t, fp_carry<NHP>, dim3(sh[2].gx, sh[2].gy), dim3(256), 0, s, f);
    LAUNCH(sh[3].kid, t, fp_fixup<NHP>, dim3(sh[3].gx), dim3(256), 0, s, f);
}

void launch_fp_recurrences(const FPArgs &f, hipStream_t s, KernelTimer *t) {
    // the caller sets the fused fields only where fp_fusable(NH, L2) holds
    if (f.K <= 0 || f.NH <= 0) return;
    LaunchShape sh[4];
    fp_shapes(f, sh);
    switch (sh[0].v1) {
        case 2: fp_launch_all<2>(sh, f, s, t); break;
        case 4: fp_launch_all<4>(sh, f, s, t); break;
        case 8: fp_launch_all<8>(sh, f, s, t); break;
        case 16: fp_launch_all<16>(sh, f, s, t); break;
        case 32: fp_launch_all<32>(sh, f, s, t); break;
        case 64: fp_launch_all<64>(sh, f, s, t); break;
        default: fp_launch_all<128>(sh, f, s, t); break;
    }
}

// ---------------------------------------------------------------------------
// Exit angular flux: sweep outflow plus (FPSA) the correction's outflow.
// out[n] for mu_n < 0 is at z0, for mu_n > 0 at z1 (angle order ascending).
// ---------------------------------------------------------------------------
__global__ void exit_flux(int N, const double *sweep_exit, const double *b0, const double *pK,
                          double *out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int NH = N / 2;
    double v = sweep_exit[n];
    if (n < NH) {
        if (b0) v += b0[n];
    } else {
        if (pK) v += pK[n - NH];
    }
    out[n] = v;
}

void launch_exit_flux(int N, const double *sweep_exit, const double *b0, const double *pK,
                      double *out, hipStream_t s, KernelTimer *t) {
    LAUNCH(KID_EXIT, t, exit_flux, dim3((N + 63) / 64), dim3(64), 0, s, N, sweep_exit, b0, pK, out);
}

// ---------------------------------------------------------------------------
// Grouped interface recurrences (FPGroupArgs): the slabs of a group share
// the factorisation, so each block loads a shared matrix once and applies
// it to every slab's vector.  Thread t serves row r = t % NHP for the slabs
// s = t / NHP, t / NHP + 256 / NHP, ...; matrices are staged in LDS row by
// row at stride NHP + 1 (stored transposed in memory, (r, c) at c NH + r),
// and a slab's vector is read from LDS by all rows at once (broadcast).
// The same recurrences as fp_matvec / fp_chain / fp_carry / fp_fixup, with
// the same partial-sum layout, so carry_value reads either.
// ---------------------------------------------------------------------------
constexpr int GFP_SC = 16;  // slabs whose vectors one matvec block stages at a time

// every slab of the group has passed its stopping test at iteration m - 1
__device__ __forceinline__ bool gfp_done(const FPGroupArgs &g, int m) {
    if (m <= 1) return false;
    for (int s = 0; s < g.nslab; ++s) {
        const double d = __longlong_as_double((long long)g.v[s].hist[hist_row(m - 1) * (size_t)g.hist_stride]);
        if (d > g.tol && isfinite(d)) return false;
    }
    return true;
}

// dst[r * (NHP + 1) + c] = M(r, c) for r, c < NH (transposed source), zero padding
template <int NHP>
__device__ __forceinline__ void gfp_stage(double *dst, const double *MT, int NH) {
    for (int idx = threadIdx.x; idx < NHP * NHP; idx += 256) {
        const int c = idx / NHP, r = idx % NHP;
        dst[r * (NHP + 1) + c] = (r < NH && c < NH) ? MT[(size_t)c * NH + r] : 0.0;
    }
}

// a FPArgs view of slab s of the group (its vectors, the shared factors)
__device__ __forceinline__ FPArgs gfp_slab(const FPGroupArgs &g, int s) {
    FPArgs f = g.f;
    const FPSlabVecs &v = g.v[s];
    f.s = v.s; f.fvec = v.fvec; f.gvec = v.gvec; f.pvec = v.pvec; f.bvec = v.bvec; f.inflow = v.inflow;
    f.e_fwd = v.e_fwd; f.e_bwd = v.e_bwd; f.part_f = v.part_f; f.part_b = v.part_b;
    return f;
}

// f_j = Hm_j s-_j + s+_j and g_j = Hb_j s+_j + s-_j of every slab; one
// block per cell
template <int NHP>
__global__ void __launch_bounds__(256) gfp_matvec(const MultiEntry<FPGroupArgs> *E, const BlockRef *br,
                                                  const int *iter) {
    const BlockRef rf = br[blockIdx.x];
    const FPGroupArgs g = E[rf.entry].a;
    if (gfp_done(g, *iter)) return;
    constexpr int NL = 256 / NHP;
    __shared__ double Ms[2][NHP * (NHP + 1)];
    __shared__ double sv[GFP_SC][2 * NHP];
    const int NH = g.f.NH, N = 2 * NH;
    const size_t M2 = (size_t)NH * NH;
    const int j = rf.local;
    const int t = threadIdx.x, r = t % NHP, lane = t / NHP;
    const double *cm = g.f.cellmats + (size_t)j * FP_CELLMATS * M2;
    gfp_stage<NHP>(Ms[0], cm + 1 * M2, NH);  // Hm
    gfp_stage<NHP>(Ms[1], cm + 3 * M2, NH);  // Hb
    for (int s0 = 0; s0 < g.nslab; s0 += GFP_SC) {
        const int sc = min(GFP_SC, g.nslab - s0);
        for (int idx = t; idx < sc * N; idx += 256) sv[idx / N][idx % N] = g.v[s0 + idx / N].s[(size_t)j * N + idx % N];
        __syncthreads();
        if (r < NH) {
            for (int s = lane; s < sc; s += NL) {
                double f0 = 0.0, f1 = 0.0, g0 = 0.0, g1 = 0.0;
#pragma unroll
                for (int c = 0; c < NHP; c += 2) {
                    if (c < NH) {
                        f0 = fma(Ms[0][r * (NHP + 1) + c], sv[s][NH + c], f0);
                        g0 = fma(Ms[1][r * (NHP + 1) + c], sv[s][c], g0);
                    }
                    if (c + 1 < NH) {
                        f1 = fma(Ms[0][r * (NHP + 1) + c + 1], sv[s][NH + c + 1], f1);
                        g1 = fma(Ms[1][r * (NHP + 1) + c + 1], sv[s][c + 1], g1);
                    }
                }
                g.v[s0 + s].fvec[(size_t)j * NH + r] = (f0 + f1) + sv[s][r];
                g.v[s0 + s].gvec[(size_t)j * NH + r] = (g0 + g1) + sv[s][NH + r];
            }
        }
        __syncthreads();
    }
}

// both local chains of one chunk (block per chunk and direction) for every
// slab: the step matrix and the slabs' additive terms of the next step are
// loaded into registers while the current step runs from LDS
template <int NHP>
__global__ void __launch_bounds__(256) gfp_chain(const MultiEntry<FPGroupArgs> *E, const BlockRef *br,
                                                 const int *iter) {
    const BlockRef rf = br[blockIdx.x];
    const FPGroupArgs g = E[rf.entry].a;
    if (gfp_done(g, *iter)) return;
    constexpr int NL = 256 / NHP, LDM = NHP + 1;
    constexpr int SMAX = kFPGroupMax;
    constexpr int GU = (NHP * NHP + 255) / 256;   // matrix entries per thread
    constexpr int AU = (SMAX * NHP + 255) / 256;  // additive entries per thread
    __shared__ double Gs[NHP * LDM];
    __shared__ double As[SMAX * NHP];
    __shared__ double Vs[2][SMAX * NHP];
    const int NH = g.f.NH, S = g.nslab;
    const size_t M2 = (size_t)NH * NH;
    int c;
    const int forward = chain_dir(g.f, rf.local, c);
    const int j0 = c * g.f.chunk, j1 = min(g.f.K, j0 + g.f.chunk), T = j1 - j0;
    const int t = threadIdx.x, r = t % NHP, lane = t / NHP;
    for (int idx = t; idx < SMAX * NHP; idx += 256) Vs[0][idx] = 0.0;
    auto cell_of = [&](int k) { return forward ? j0 + k : j1 - 1 - k; };
    double gr[GU], ar[AU];
    // step k's matrix entries (transposed source, clamped indices) and
    // additive terms into registers
    auto fetch = [&](int k) {
        const int j = cell_of(min(k, T - 1));
        const double *M = g.f.cellmats + (size_t)j * FP_CELLMATS * M2 + (forward ? 0 : 2) * M2;
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int idx = min(t + 256 * u, NHP * NHP - 1);
            const int cc = idx / NHP, rr = idx % NHP;
            gr[u] = M[(size_t)min(cc, NH - 1) * NH + min(rr, NH - 1)];
        }
#pragma unroll
        for (int u = 0; u < AU; ++u) {
            const int idx = min(t + 256 * u, SMAX * NHP - 1);
            const int s = min(idx / NHP, S - 1), rr = min(idx % NHP, NH - 1);
            ar[u] = (forward ? g.v[s].fvec : g.v[s].gvec)[(size_t)j * NH + rr];
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int idx = t + 256 * u;
            if (idx < NHP * NHP) {
                const int cc = idx / NHP, rr = idx % NHP;
                Gs[rr * LDM + cc] = (rr < NH && cc < NH) ? gr[u] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < AU; ++u) {
            const int idx = t + 256 * u;
            if (idx < SMAX * NHP) As[idx] = ar[u];
        }
    };
    if (T > 0) fetch(0);
    int cur = 0;
    for (int k = 0; k < T; ++k) {
        __syncthreads();  // the previous step's readers of Gs / As are done
        store();
        if (k + 1 < T) fetch(k + 1);
        __syncthreads();
        const int j = cell_of(k);
        if (r < NH) {
            double grow[NHP];
#pragma unroll
            for (int cc = 0; cc < NHP; ++cc) grow[cc] = Gs[r * LDM + cc];
            for (int s = lane; s < S; s += NL) {
                const double *vo = &Vs[cur][s * NHP];
                double a0 = As[s * NHP + r], a1 = 0.0;
#pragma unroll
                for (int cc = 0; cc < NHP; cc += 2) {
                    if (cc < NH) a0 = fma(grow[cc], vo[cc], a0);
                    if (cc + 1 < NH) a1 = fma(grow[cc + 1], vo[cc + 1], a1);
                }
                const double v = a0 + a1;
                // forward: p_loc before the step; backward: b_loc after it
                if (forward) g.v[s].pvec[(size_t)j * NH + r] = vo[r];
                else g.v[s].bvec[(size_t)j * NH + r] = v;
                Vs[cur ^ 1][s * NHP + r] = v;
            }
        }
        cur ^= 1;
    }
    __syncthreads();
    if (r < NH)
        for (int s = lane; s < S; s += NL) (forward ? g.v[s].e_fwd : g.v[s].e_bwd)[(size_t)c * NH + r] = Vs[cur][s * NHP + r];
}

// chunk carry partial sums of every slab (the rows, parts and term split of
// fp_carry): part p of row c sums the transfer terms p GRP .. p GRP + GRP - 1
template <int NHP>
__global__ void __launch_bounds__(256) gfp_carry(const MultiEntry<FPGroupArgs> *E, const BlockRef *br,
                                                 const int *iter) {
    const BlockRef rf = br[blockIdx.x];
    const MultiEntry<FPGroupArgs> &e = E[rf.entry];
    const FPGroupArgs g = e.a;
    if (gfp_done(g, *iter)) return;
    constexpr int GRP = 256 / NHP, NL = 256 / NHP, LDM = NHP + 1;
    constexpr int SMAX = kFPGroupMax;
    constexpr int SPT = (SMAX + NL - 1) / NL;  // slabs per thread
    __shared__ double Ts[NHP * LDM];
    __shared__ double Es[SMAX * NHP];
    const int NH = g.f.NH, P = g.f.nchunks, S = g.nslab;
    const size_t M2 = (size_t)NH * NH;
    const int bx = rf.local % e.gx, part = rf.local / e.gx;
    const int forward = bx <= P;
    const int c = forward ? bx : bx - (P + 1);
    const int a = forward ? c : P - 1 - c;
    const int nterms = carry_terms(forward, c, P);
    const int nparts = max(1, (nterms + GRP - 1) / GRP);
    if (part >= nparts) return;
    const int t = threadIdx.x, r = t % NHP, lane = t / NHP;
    double acc[SPT];
#pragma unroll
    for (int i = 0; i < SPT; ++i) acc[i] = 0.0;
    const int ap0 = part * GRP, ap1 = min(nterms, ap0 + GRP);
    for (int ap = ap0; ap < ap1; ++ap) {
        const size_t row0 = (size_t)(a - 1) * (a - 2) / 2;
        const int cp = forward ? ap : P - 1 - ap;
        const double *T = (forward ? g.f.theta_fwd : g.f.theta_bwd) + (row0 + ap) * M2;
        __syncthreads();
        gfp_stage<NHP>(Ts, T, NH);
        for (int idx = t; idx < S * NH; idx += 256) {
            const int s = idx / NH, k = idx % NH;
            Es[s * NHP + k] = (forward ? g.v[s].e_fwd : g.v[s].e_bwd)[(size_t)cp * NH + k];
        }
        __syncthreads();
        if (r < NH) {
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
                const int s = lane + NL * i;
                if (s < S) {
                    double x = acc[i];
#pragma unroll
                    for (int cc = 0; cc < NHP; ++cc)
                        if (cc < NH) x = fma(Ts[r * LDM + cc], Es[s * NHP + cc], x);
                    acc[i] = x;
                }
            }
        }
    }
    if (r < NH) {
#pragma unroll
        for (int i = 0; i < SPT; ++i) {
            const int s = lane + NL * i;
            if (s < S) (forward ? g.v[s].part_f : g.v[s].part_b)[((size_t)c * g.f.carry_parts + part) * NH + r] = acc[i];
        }
    }
}

// fix-up and combination at the interfaces of every slab, one block per run
// of up to GFP_CELLS cells inside one chunk (the chunk's carries are formed
// once per block and slab):
//   p = p_loc + PsiF carry, q = q_loc + PsiB carry', a = W p + W rho q,
//   b = sig a + q; inflow (a_j | b_{j+1}), b_0 and p_K as fp_fixup
constexpr int GFP_CELLS = 8;

__host__ __device__ inline int gfp_fixup_runs(int chunk) { return (chunk + GFP_CELLS - 1) / GFP_CELLS; }

template <int NHP>
__global__ void __launch_bounds__(256) gfp_fixup(const MultiEntry<FPGroupArgs> *E, const BlockRef *br,
                                                 const int *iter) {
    const BlockRef rf = br[blockIdx.x];
    const FPGroupArgs g = E[rf.entry].a;
    if (gfp_done(g, *iter)) return;
    constexpr int NL = 256 / NHP, LDM = NHP + 1, SMAX = kFPGroupMax;
    __shared__ double Ms[2][NHP * LDM];
    __shared__ double X[SMAX * NHP], Y[SMAX * NHP], Z[SMAX * NHP], Q[SMAX * NHP], Av[SMAX * NHP];
    const int NH = g.f.NH, N = 2 * NH, K = g.f.K, S = g.nslab;
    const size_t M2 = (size_t)NH * NH;
    const int runs = gfp_fixup_runs(g.f.chunk);
    const int ch = rf.local / runs, run = rf.local % runs;
    const int jb = ch * g.f.chunk + run * GFP_CELLS;
    const int je = min(min(K, (ch + 1) * g.f.chunk), jb + GFP_CELLS);
    if (jb >= je) return;
    const int t = threadIdx.x, r = t % NHP, lane = t / NHP;
    // carries of the chunk per slab: X forward, Y backward; p_K with the last cell
    if (r < NH) {
        for (int s = lane; s < S; s += NL) {
            const FPArgs f = gfp_slab(g, s);
            X[s * NHP + r] = carry_value(f, 1, ch, r);
            Y[s * NHP + r] = carry_value(f, 0, ch, r);
            if (je == K) f.pvec[(size_t)K * NH + r] = carry_value(f, 1, g.f.nchunks, r);
        }
    }
    for (int j = jb; j < je; ++j) {
        const double *cm = g.f.cellmats + (size_t)j * FP_CELLMATS * M2;
        __syncthreads();  // the previous cell's readers of Ms are done
        gfp_stage<NHP>(Ms[0], g.f.psi_fwd + (size_t)j * M2, NH);
        gfp_stage<NHP>(Ms[1], g.f.psi_bwd + (size_t)j * M2, NH);
        __syncthreads();
        // p = p_loc + PsiF carry into Z, q = q_loc + PsiB carry' into Q
        if (r < NH) {
            for (int s = lane; s < S; s += NL) {
                double p = g.v[s].pvec[(size_t)j * NH + r], q = g.v[s].bvec[(size_t)j * NH + r];
#pragma unroll
                for (int cc = 0; cc < NHP; ++cc)
                    if (cc < NH) {
                        p = fma(Ms[0][r * LDM + cc], X[s * NHP + cc], p);
                        q = fma(Ms[1][r * LDM + cc], Y[s * NHP + cc], q);
                    }
                Z[s * NHP + r] = p;
                Q[s * NHP + r] = q;
            }
        }
        __syncthreads();
        gfp_stage<NHP>(Ms[0], cm + 4 * M2, NH);  // W
        gfp_stage<NHP>(Ms[1], cm + 5 * M2, NH);  // W rho
        __syncthreads();
        // a = W p + W rho q into Av
        if (r < NH) {
            for (int s = lane; s < S; s += NL) {
                double a = 0.0;
#pragma unroll
                for (int cc = 0; cc < NHP; ++cc)
                    if (cc < NH) a = fma(Ms[0][r * LDM + cc], Z[s * NHP + cc], fma(Ms[1][r * LDM + cc], Q[s * NHP + cc], a));
                Av[s * NHP + r] = a;
                g.v[s].inflow[(size_t)j * N + r] = a;
            }
        }
        __syncthreads();
        gfp_stage<NHP>(Ms[0], cm + 6 * M2, NH);  // sig
        __syncthreads();
        // b = sig a + q
        if (r < NH) {
            for (int s = lane; s < S; s += NL) {
                double b = Q[s * NHP + r];
#pragma unroll
                for (int cc = 0; cc < NHP; ++cc)
                    if (cc < NH) b = fma(Ms[0][r * LDM + cc], Av[s * NHP + cc], b);
                double *inflow = g.v[s].inflow;
                if (j >= 1) inflow[(size_t)(j - 1) * N + NH + r] = b;
                if (j == K - 1) inflow[(size_t)j * N + NH + r] = 0.0;
                if (j == 0) g.v[s].bvec[r] = b;
            }
        }
    }
}

void fp_group_shapes(const FPArgs &f, LaunchShape out[4]) {
    const int NHP = fp_nhp(f.NH);
    LaunchShape m;
    m.kernel = MK_GFP_MATVEC;
    m.v1 = NHP;
    m.kid = KID_FP_MATVEC;
    m.gx = f.K;
    LaunchShape c = m;
    c.kernel = MK_GFP_CHAIN;
    c.kid = KID_FP_CHAIN;
    c.gx = 2 * f.nchunks;
    LaunchShape k = m;
    k.kernel = MK_GFP_CARRY;
    k.kid = KID_FP_CARRY;
    k.gx = 2 * f.nchunks + 1;
    k.gy = f.carry_parts;
    LaunchShape x = m;
    x.kernel = MK_GFP_FIXUP;
    x.kid = KID_FP_FIXUP;
    x.gx = f.nchunks * gfp_fixup_runs(f.chunk);
    out[0] = m;
    out[1] = c;
    out[2] = k;
    out[3] = x;
}

template <int NHP>
static void launch_multi_gfp(const MultiLaunch &L, const int *iter, hipStream_t s, KernelTimer *t) {
    const dim3 grid(L.nblocks);
    const LaunchShape &sh = L.shape;
    const MultiEntry<FPGroupArgs> *E = static_cast<const MultiEntry<FPGroupArgs> *>(L.entries);
    switch (sh.kernel) {
        case MK_GFP_MATVEC: LAUNCH(sh.kid, t, gfp_matvec<NHP>, grid, dim3(256), 0, s, E, L.refs, iter); break;
        case MK_GFP_CHAIN: LAUNCH(sh.kid, t, gfp_chain<NHP>, grid, dim3(256), 0, s, E, L.refs, iter); break;
        case MK_GFP_CARRY: LAUNCH(sh.kid, t, gfp_carry<NHP>, grid, dim3(256), 0, s, E, L.refs, iter); break;
        default: LAUNCH(sh.kid, t, gfp_fixup<NHP>, grid, dim3(256), 0, s, E, L.refs, iter); break;
    }
}

// ---------------------------------------------------------------------------
// Batched launches (see MultiLaunch): one grid of L.nblocks blocks over the
// per-block table.
// ---------------------------------------------------------------------------
template <class A>
static const MultiEntry<A> *multi_entries(const MultiLaunch &L) {
    return static_cast<const MultiEntry<A> *>(L.entries);
}

template <int NHP>
static void launch_multi_fp(const MultiLaunch &L, const int *iter, hipStream_t s, KernelTimer *t) {
    const dim3 grid(L.nblocks);
    const LaunchShape &sh = L.shape;
    const MultiEntry<FPArgs> *E = multi_entries<FPArgs>(L);
    switch (sh.kernel) {
        case MK_FP_MATVEC: LAUNCH(sh.kid, t, fp_matvec_multi<NHP>, grid, dim3(256), 0, s, E, L.refs, iter); break;
        case MK_FP_CHAIN:
            if constexpr (NHP >= 8 && NHP <= 64) {
                if (sh.v2 == 0)
                    LAUNCH(sh.kid, t, fp_chain_ring_multi<NHP>, grid, dim3(256), 0, s, E, L.refs, iter);
                else
                    LAUNCH(sh.kid, t, (fp_chain_staged_multi<NHP, false>), grid, dim3(256), 0, s, E, L.refs, iter);
            } else if constexpr (NHP <= 64) {
                if (sh.v2 == 1)
                    LAUNCH(sh.kid, t, (fp_chain_staged_multi<NHP, true>), grid, dim3(256), 0, s, E, L.refs, iter);
                else
                    LAUNCH(sh.kid, t, (fp_chain_staged_multi<NHP, false>), grid, dim3(256), 0, s, E, L.refs, iter);
            } else {
                LAUNCH(sh.kid, t, fp_chain_any_multi, grid, dim3(64), L.lds, s, E, L.refs, iter);
            }
            break;
        case MK_FP_CARRY: LAUNCH(sh.kid, t, fp_carry_multi<NHP>, grid, dim3(256), 0, s, E, L.refs, iter); break;
        default: LAUNCH(sh.kid, t, fp_fixup_multi<NHP>, grid, dim3(256), 0, s, E, L.refs, iter); break;
    }
}

void launch_multi(const MultiLaunch &L, const int *iter, hipStream_t s, KernelTimer *t) {
    if (L.nblocks <= 0) return;
    const dim3 grid(L.nblocks);
    const LaunchShape &sh = L.shape;
    switch (sh.kernel) {
        case MK_GEMM: {
            const MultiEntry<GemmArgs> *E = multi_entries<GemmArgs>(L);
            if (sh.v2 == 1) {
                LAUNCH(sh.kid, t, gemm_f64_wide_multi, grid, dim3(256), 0, s, E, L.refs, iter);
                break;
            }
            switch (sh.v1) {
                case 1: LAUNCH(sh.kid, t, gemm_f64_mfma_multi<1>, grid, dim3(256), 0, s, E, L.refs, iter); break;
                case 2: LAUNCH(sh.kid, t, gemm_f64_mfma_multi<2>, grid, dim3(256), 0, s, E, L.refs, iter); break;
                case 3: LAUNCH(sh.kid, t, gemm_f64_mfma_multi<3>, grid, dim3(256), 0, s, E, L.refs, iter); break;
                case 4: LAUNCH(sh.kid, t, gemm_f64_mfma_multi<4>, grid, dim3(256), 0, s, E, L.refs, iter); break;
                default: LAUNCH(sh.kid, t, gemm_f64_mfma_multi<0>, grid, dim3(256), 0, s, E, L.refs, iter); break;
            }
            break;
        }
        case MK_GEMM_TALL:
            LAUNCH(sh.kid, t, gemm_f64_tall_multi, grid, dim3(256), 0, s, multi_entries<GemmArgs>(L), L.refs, iter);
            break;
        case MK_SWEEP_AGG: {
            const MultiEntry<SweepArgs> *E = multi_entries<SweepArgs>(L);
            switch (sh.v1) {
                case 16: LAUNCH(sh.kid, t, sweep_aggregate_multi<16>, grid, dim3(256), L.lds, s, E, L.refs, iter); break;
                case 32: LAUNCH(sh.kid, t, sweep_aggregate_multi<32>, grid, dim3(256), L.lds, s, E, L.refs, iter); break;
                case 64: LAUNCH(sh.kid, t, sweep_aggregate_multi<64>, grid, dim3(256), L.lds, s, E, L.refs, iter); break;
                default: LAUNCH(sh.kid, t, sweep_aggregate_multi<0>, grid, dim3(256), 0, s, E, L.refs, iter); break;
            }
            break;
        }
        case MK_SCAN_GROUPS:
            LAUNCH(sh.kid, t, sweep_scan_groups_multi, grid, dim3(64), 0, s, multi_entries<SweepArgs>(L), L.refs, iter);
            break;
        case MK_SCAN_CARRY:
            LAUNCH(sh.kid, t, sweep_scan_carry_multi, grid, dim3(64), 0, s, multi_entries<SweepArgs>(L), L.refs, iter);
            break;
        case MK_SWEEP_APPLY: {
            const MultiEntry<SweepArgs> *E = multi_entries<SweepArgs>(L);
            switch (sh.v1) {
                case 16: LAUNCH(sh.kid, t, sweep_apply_multi<16>, grid, dim3(256), L.lds, s, E, L.refs, iter); break;
                case 32: LAUNCH(sh.kid, t, sweep_apply_multi<32>, grid, dim3(256), L.lds, s, E, L.refs, iter); break;
                case 64: LAUNCH(sh.kid, t, sweep_apply_multi<64>, grid, dim3(256), L.lds, s, E, L.refs, iter); break;
                default: LAUNCH(sh.kid, t, sweep_apply_multi<0>, grid, dim3(256), 0, s, E, L.refs, iter); break;
            }
            break;
        }
        case MK_STOP:
            LAUNCH(sh.kid, t, stopping_test_multi, grid, dim3(256), 0, s, multi_entries<StopArgs>(L), L.refs, iter);
            break;
        case MK_GFP_MATVEC:
        case MK_GFP_CHAIN:
        case MK_GFP_CARRY:
        case MK_GFP_FIXUP:
            switch (sh.v1) {
                case 2: launch_multi_gfp<2>(L, iter, s, t); break;
                case 4: launch_multi_gfp<4>(L, iter, s, t); break;
                case 8: launch_multi_gfp<8>(L, iter, s, t); break;
                case 16: launch_multi_gfp<16>(L, iter, s, t); break;
                case 32: launch_multi_gfp<32>(L, iter, s, t); break;
                default: launch_multi_gfp<64>(L, iter, s, t); break;
            }
            break;
        default:
            switch (sh.v1) {
                case 2: launch_multi_fp<2>(L, iter, s, t); break;
                case 4: launch_multi_fp<4>(L, iter, s, t); break;
                case 8: launch_multi_fp<8>(L, iter, s, t); break;
                case 16: launch_multi_fp<16>(L, iter, s, t); break;
                case 32: launch_multi_fp<32>(L, iter, s, t); break;
                case 64: launch_multi_fp<64>(L, iter, s, t); break;
                default: launch_multi_fp<128>(L, iter, s, t); break;
            }
            break;
    }
}

__global__ void iter_step(int *iter) {
    if (threadIdx.x == 0) iter[0] += 1;
}

void launch_iter_step(int *iter, hipStream_t s) { hipLaunchKernelGGL(iter_step, dim3(1), dim3(64), 0, s, iter); }

}  // namespace snfpsa
