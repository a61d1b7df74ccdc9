// Batched (many-slab) kernels, gfx950.
//
//   sweep_batch_*     LD transport sweep of every (slab, angle) in one launch:
//                     one wavefront per work item (a block of up to 64
//                     angles of one slab, or all angles of 64/N slabs of
//                     equal N, then a second, shorter group of the same
//                     kind), each lane running its angle's recurrence over
//                     the slab's cells with batches of cells in flight
//   src_batch         scattering source q = (phi .* sigma_s) M^T + q_ext of
//                     64 node rows per block on FP32 MFMA, or as split-BF16
//                     products with FP32 accumulation
//   mom_batch         moments phi = psi V of 64 node rows per block on FP32
//                     MFMA, FP64 out, with the per-slab stopping test
//   select_final      per-slab copy of the final iterate of a batched solve
#include "sn_batch.hpp"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

namespace snfpsa {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

#define LAUNCH(id, t, kernel, grid, block, shm, st, ...)                                       \
    do {                                                                                       \
        hipEvent_t ev0_ = nullptr, ev1_ = nullptr;                                             \
        if ((t) && (t)->events((id), &ev0_, &ev1_))                                            \
            hipExtLaunchKernelGGL(kernel, grid, block, shm, st, ev0_, ev1_, 0, __VA_ARGS__);   \
        else                                                                                   \
            hipLaunchKernelGGL(kernel, grid, block, shm, st, __VA_ARGS__);                     \
    } while (0)

__device__ __forceinline__ bool slab_done(const SlabGate &g, int slab) {
    const unsigned long long *prev = g.prev;
    if (g.iter) {
        const int m = *g.iter;
        prev = m > 1 ? g.hist + hist_row(m - 1) * g.ns : nullptr;
    }
    if (!prev) return false;
    const double d = __longlong_as_double((long long)prev[slab]);
    return d <= g.tol || !isfinite(d);
}

// ---------------------------------------------------------------------------
// Batched FP32 sweep.  Lane (slot, a) of a work item serves angle
// angle0 + a of slab slab_list[first + slot].  A lane's cells are visited in
// its sweep direction (mu > 0 left to right); per cell it reads the two
// nodal sources and {h, sigma_t h}, and writes the two nodal fluxes.  Cells
// go in batches of SB; the next batch's loads are issued before the current
// batch is computed.  Loads past a lane's last cell are clamped to valid
// cells and their results dropped.
// ---------------------------------------------------------------------------
template <int SB>
struct CellBatch {
    float qi[SB], qo[SB];
    float2 cp[SB];
};

// Sweeps one group of a work item (see SweepItem) with the calling wavefront.
template <int SB>
__device__ __forceinline__ void sweep_group(const BatchSweepArgs &a, int first, int count, int angle0, int kmax) {
    const int lane = threadIdx.x & 63;
    const BatchSlab s0 = a.slabs[a.slab_list[first]];
    const int Nw = s0.N < 64 ? s0.N : 64;           // lanes per slab
    const int slot = lane / Nw, n = angle0 + lane % Nw;
    bool active = slot < count && n < s0.N;
    const int slab = a.slab_list[first + (active ? slot : 0)];
    const BatchSlab m = active ? a.slabs[slab] : s0;
    if (active && slab_done(a.gate, slab)) active = false;
    const int N = m.N, K = m.K;
    const int nn = active ? n : 0;
    const double mu = a.mu[m.quad_off + nn];
    const float inv = (float)a.inv_absmu[m.quad_off + nn];
    const bool fwd = mu > 0.0;
    const int in_node = fwd ? 0 : 1;
    float x = 0.0f;
    if (fwd) {
        if (a.psi_left) x = (float)a.psi_left[m.bc_off + nn - N / 2];
    } else {
        if (a.psi_right) x = (float)a.psi_right[m.bc_off + nn];
    }
    const float *qb = a.q + m.psi_off + nn;
    float *pb = a.psi + m.psi_off + nn;
    const float2 *cpb = a.cellpar + m.cell_off;
    const int Ka = active ? K : 0;
    const size_t stride = 2 * (size_t)N;
    auto cell_of = [&](int i) {
        const int ic = min(i, K - 1);
        return fwd ? ic : K - 1 - ic;
    };
    auto load = [&](CellBatch<SB> &b, int i0) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int j = cell_of(i0 + u);
            b.qi[u] = qb[j * stride + in_node * N];
            b.qo[u] = qb[j * stride + (1 - in_node) * N];
            b.cp[u] = cpb[j];
        }
    };
    auto run = [&](const CellBatch<SB> &b, int i0) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            if (i0 + u < Ka) {
                const int j = fwd ? i0 + u : K - 1 - i0 - u;
                const float h = b.cp[u].x, tau = b.cp[u].y * inv;
                const float f = h * inv * (1.0f / 6.0f);
                const float gin = f * (2.0f * b.qi[u] + b.qo[u]);
                const float gout = f * (b.qi[u] + 2.0f * b.qo[u]);
                const float den_inv = __builtin_amdgcn_rcpf(6.0f + tau * (4.0f + tau));
                const float vout = ((6.0f - 2.0f * tau) * x + (6.0f + 4.0f * tau) * gout + (6.0f - 2.0f * tau) * gin) *
                                   den_inv;
                const float vin = ((6.0f + 4.0f * tau) * (gin + x) - (6.0f + 2.0f * tau) * gout) * den_inv;
                pb[j * stride + in_node * N] = vin;
                pb[j * stride + (1 - in_node) * N] = vout;
                x = vout;
            }
        }
    };
    CellBatch<SB> b0, b1;
    load(b0, 0);
    for (int i0 = 0; i0 < kmax; i0 += 2 * SB) {
        load(b1, i0 + SB);
        run(b0, i0);
        load(b0, i0 + 2 * SB);
        run(b1, i0 + SB);
    }
    if (active && a.exit) a.exit[m.exit_off + n] = x;
}

template <int SB>
__global__ void __launch_bounds__(256) sweep_batch_f32(BatchSweepArgs a) {
    const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= a.nitems) return;
    const SweepItem it = a.items[item];
    sweep_group<SB>(a, it.first, it.count, it.angle0, it.kmax);
    if (it.count2 > 0) sweep_group<SB>(a, it.first2, it.count2, it.angle0, it.kmax2);
}

// Direction-major variant: a lane's cells are contiguous runs of N floats
// (its two nodes adjacent), one 8-byte load of the source and one 8-byte
// store of the flux per cell; three batches of cells in flight.
typedef float v2f __attribute__((ext_vector_type(2)));

template <int SB>
struct CellBatchDM {
    v2f qv[SB];
    float2 cp[SB];
};

// Sweeps one group of a work item (see SweepItem) with the calling wavefront.
template <int SB>
__device__ __forceinline__ void sweep_group_dm(const BatchSweepArgs &a, int first, int count, int angle0, int kmax) {
    const int lane = threadIdx.x & 63;
    const BatchSlab s0 = a.slabs[a.slab_list[first]];
    const int Nw = s0.N < 64 ? s0.N : 64;
    const int slot = lane / Nw, n = angle0 + lane % Nw;
    bool active = slot < count && n < s0.N;
    const int slab = a.slab_list[first + (active ? slot : 0)];
    const BatchSlab m = active ? a.slabs[slab] : s0;
    if (active && slab_done(a.gate, slab)) active = false;
    const int N = m.N, K = m.K;
    const int nn = active ? n : 0;
    const double mu = a.mu[m.quad_off + nn];
    const float inv = (float)a.inv_absmu[m.quad_off + nn];
    const bool fwd = mu > 0.0;
    float x = 0.0f;
    if (fwd) {
        if (a.psi_left) x = (float)a.psi_left[m.bc_off + nn - N / 2];
    } else {
        if (a.psi_right) x = (float)a.psi_right[m.bc_off + nn];
    }
    const long long base = m.psi_off + dm_index(K, N, 0, 0, nn);
    // q is read once and psi written once per sweep: non-temporal accesses
    const v2f *qb = reinterpret_cast<const v2f *>(a.q + base);
    v2f *pb = reinterpret_cast<v2f *>(a.psi + base);
    const bool nt = N >= 32;
    const int cs = N / 2;  // cell stride in float2
    const float2 *cpb = a.cellpar + m.cell_off;
    const int Ka = active ? K : 0;
    auto cell_of = [&](int i) {
        const int ic = min(i, K - 1);
        return fwd ? ic : K - 1 - ic;
    };
    auto load = [&](CellBatchDM<SB> &b, int i0) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int j = cell_of(i0 + u);
            // N < 32: a cell's data per direction is less than a cache line and
            // the next cell reads the rest of it, so keep those loads cached
            b.qv[u] = nt ? __builtin_nontemporal_load(qb + (long long)j * cs) : qb[(long long)j * cs];
            b.cp[u] = cpb[j];
        }
    };
    auto run = [&](const CellBatchDM<SB> &b, int i0) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            if (i0 + u < Ka) {
                const int j = fwd ? i0 + u : K - 1 - i0 - u;
                const float qi = fwd ? b.qv[u].x : b.qv[u].y, qo = fwd ? b.qv[u].y : b.qv[u].x;
                const float h = b.cp[u].x, tau = b.cp[u].y * inv;
                const float f = h * inv * (1.0f / 6.0f);
                const float gin = f * (2.0f * qi + qo);
                const float gout = f * (qi + 2.0f * qo);
                const float den_inv = __builtin_amdgcn_rcpf(6.0f + tau * (4.0f + tau));
                const float vout =
                    ((6.0f - 2.0f * tau) * x + (6.0f + 4.0f * tau) * gout + (6.0f - 2.0f * tau) * gin) * den_inv;
                const float vin = ((6.0f + 4.0f * tau) * (gin + x) - (6.0f + 2.0f * tau) * gout) * den_inv;
                const v2f o = fwd ? v2f{vin, vout} : v2f{vout, vin};
                if (nt)
                    __builtin_nontemporal_store(o, pb + (long long)j * cs);
                else
                    pb[(long long)j * cs] = o;
                x = vout;
            }
        }
    };
    CellBatchDM<SB> b0, b1, b2;
    load(b0, 0);
    load(b1, SB);
    for (int i0 = 0; i0 < kmax; i0 += 3 * SB) {
        load(b2, i0 + 2 * SB);
        run(b0, i0);
        load(b0, i0 + 3 * SB);
        run(b1, i0 + SB);
        load(b1, i0 + 4 * SB);
        run(b2, i0 + 2 * SB);
    }
    if (active && a.exit) a.exit[m.exit_off + n] = x;
}

// Segmented direction-major sweep of one small-N slab (N <= 16) by one
// wavefront: its cells are split into nseg = 64/N contiguous segments, lane
// (segment, angle).  Pass 1 composes each segment's affine cell maps
// (x_out = A x_in + B); the segment maps are exchanged by cross-lane
// shuffles so that every segment forms its carry-in from the boundary
// inflow; pass 2 re-sweeps the segment from that carry and writes psi.  The
// chain of a lane is 2 K / nseg cells instead of K.
template <int SB>
__device__ __forceinline__ void sweep_group_dm_seg(const BatchSweepArgs &a, int first, int nseg) {
    const int lane = threadIdx.x & 63;
    const int slab = a.slab_list[first];
    const BatchSlab m = a.slabs[slab];
    const int N = m.N, K = m.K;
    const int seg = lane / N, n = lane % N;
    const bool active = seg < nseg && !slab_done(a.gate, slab);
    const int sg = seg < nseg ? seg : nseg - 1;
    const int c0 = (int)((long long)K * sg / nseg), c1 = (int)((long long)K * (sg + 1) / nseg);
    const int len = active ? c1 - c0 : 0;
    const int smax = (K + nseg - 1) / nseg;  // longest segment (wave-uniform)
    const double mu = a.mu[m.quad_off + n];
    const float inv = (float)a.inv_absmu[m.quad_off + n];
    const bool fwd = mu > 0.0;
    float x0 = 0.0f;
    if (fwd) {
        if (a.psi_left) x0 = (float)a.psi_left[m.bc_off + n - N / 2];
    } else {
        if (a.psi_right) x0 = (float)a.psi_right[m.bc_off + n];
    }
    const long long base = m.psi_off + dm_index(K, N, 0, 0, n);
    const v2f *qb = reinterpret_cast<const v2f *>(a.q + base);
    v2f *pb = reinterpret_cast<v2f *>(a.psi + base);
    const int cs = N / 2;
    const float2 *cpb = a.cellpar + m.cell_off;
    auto cell_of = [&](int i) {
        const int ic = min(i, max(len - 1, 0));
        return max(min(fwd ? c0 + ic : c1 - 1 - ic, K - 1), 0);  // empty segments: any valid cell
    };
    auto load = [&](CellBatchDM<SB> &b, int i0) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int j = cell_of(i0 + u);
            b.qv[u] = qb[(long long)j * cs];
            b.cp[u] = cpb[j];
        }
    };
    // pass 1: segment map
    float A = 1.0f, B = 0.0f;
    auto agg = [&](const CellBatchDM<SB> &b, int i0) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            if (i0 + u < len) {
                const float qi = fwd ? b.qv[u].x : b.qv[u].y, qo = fwd ? b.qv[u].y : b.qv[u].x;
                const float h = b.cp[u].x, tau = b.cp[u].y * inv;
                const float f = h * inv * (1.0f / 6.0f);
                const float gin = f * (2.0f * qi + qo);
                const float gout = f * (qi + 2.0f * qo);
                const float den_inv = __builtin_amdgcn_rcpf(6.0f + tau * (4.0f + tau));
                const float ac = (6.0f - 2.0f * tau) * den_inv;
                const float bc = ((6.0f + 4.0f * tau) * gout + (6.0f - 2.0f * tau) * gin) * den_inv;
                B = ac * B + bc;
                A = ac * A;
            }
        }
    };
    float x = 0.0f;
    auto run = [&](const CellBatchDM<SB> &b, int i0) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            if (i0 + u < len) {
                const int j = fwd ? c0 + i0 + u : c1 - 1 - i0 - u;
                const float qi = fwd ? b.qv[u].x : b.qv[u].y, qo = fwd ? b.qv[u].y : b.qv[u].x;
                const float h = b.cp[u].x, tau = b.cp[u].y * inv;
                const float f = h * inv * (1.0f / 6.0f);
                const float gin = f * (2.0f * qi + qo);
                const float gout = f * (qi + 2.0f * qo);
                const float den_inv = __builtin_amdgcn_rcpf(6.0f + tau * (4.0f + tau));
                const float vout =
                    ((6.0f - 2.0f * tau) * x + (6.0f + 4.0f * tau) * gout + (6.0f - 2.0f * tau) * gin) * den_inv;
                const float vin = ((6.0f + 4.0f * tau) * (gin + x) - (6.0f + 2.0f * tau) * gout) * den_inv;
                pb[(long long)j * cs] = fwd ? v2f{vin, vout} : v2f{vout, vin};
                x = vout;
            }
        }
    };
    auto pass = [&](auto &&body) {
        CellBatchDM<SB> b0, b1, b2;
        load(b0, 0);
        load(b1, SB);
        for (int i0 = 0; i0 < smax; i0 += 3 * SB) {
            load(b2, i0 + 2 * SB);
            body(b0, i0);
            load(b0, i0 + 3 * SB);
            body(b1, i0 + SB);
            load(b1, i0 + 4 * SB);
            body(b2, i0 + 2 * SB);
        }
    };
    pass(agg);
    // carry-in: compose the maps of the segments before this one in sweep order
    x = x0;
    for (int t = 0; t < nseg; ++t) {
        const float At = __shfl(A, t * N + n, 64), Bt = __shfl(B, t * N + n, 64);
        const bool before = fwd ? t < sg : false;
        if (before) x = At * x + Bt;
    }
    for (int t = nseg - 1; t >= 0; --t) {
        const float At = __shfl(A, t * N + n, 64), Bt = __shfl(B, t * N + n, 64);
        const bool before = fwd ? false : t > sg;
        if (before) x = At * x + Bt;
    }
    pass(run);
    if (active && a.exit && (fwd ? sg == nseg - 1 : sg == 0)) a.exit[m.exit_off + n] = x;
}

template <int SB>
__global__ void __launch_bounds__(256) sweep_batch_dm(BatchSweepArgs a) {
    const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= a.nitems) return;
    const SweepItem it = a.items[item];
    if (it.pad > 0) {
        // small N: one slab per group, pad = number of cell segments
        sweep_group_dm_seg<SB>(a, it.first, it.pad);
        if (it.count2 > 0) sweep_group_dm_seg<SB>(a, it.first2, it.pad);
        return;
    }
    sweep_group_dm<SB>(a, it.first, it.count, it.angle0, it.kmax);
    if (it.count2 > 0) sweep_group_dm<SB>(a, it.first2, it.count2, it.angle0, it.kmax2);
}

void launch_sweep_batch(const BatchSweepArgs &a, hipStream_t s, KernelTimer *t) {
    if (a.nitems <= 0) return;
    const dim3 grid((unsigned)((a.nitems + 3) / 4));
    // direction-major: batches of 16 cells, 48 cells in flight per lane at
    // one wavefront per SIMD (297 registers); on the 4096-slab batch this
    // streams faster than 24 in flight at two wavefronts per SIMD (fewer
    // concurrent streams, each deeper).  The [cell][node][angle] layout
    // likewise: two batches of 32 cells (322 registers).  The long-slab
    // passes keep batches of 8 (on the 2^20-cell slab, batches of 12 to 32
    // at lower occupancy are up to 9 % slower).
    if (a.dirmajor)
        LAUNCH(KID_SWEEP_BATCH, t, sweep_batch_dm<16>, grid, dim3(256), 0, s, a);
    else
        LAUNCH(KID_SWEEP_BATCH, t, sweep_batch_f32<32>, grid, dim3(256), 0, s, a);  // one wavefront per SIMD
}

// ---------------------------------------------------------------------------
// Long-slab segmented sweep (direction-major layout, see LongSeg).
// ---------------------------------------------------------------------------
struct LaneSetup {
    bool active, fwd;
    int n, N, K;
    float inv, x0;
    long long base;
};

__device__ __forceinline__ LaneSetup long_lane(const BatchLongArgs &a, const LongSeg &sg) {
    LaneSetup L;
    const int lane = threadIdx.x & 63;
    const BatchSlab m = a.slabs[sg.slab];
    L.N = m.N;
    L.K = m.K;
    const int n = sg.angle0 + lane;
    L.active = n < m.N && !slab_done(a.gate, sg.slab);
    L.n = n < m.N ? n : m.N - 1;
    const double mu = a.mu[m.quad_off + L.n];
    L.inv = (float)a.inv_absmu[m.quad_off + L.n];
    L.fwd = mu > 0.0;
    L.x0 = 0.0f;
    if (L.fwd) {
        if (a.psi_left) L.x0 = (float)a.psi_left[m.bc_off + L.n - m.N / 2];
    } else {
        if (a.psi_right) L.x0 = (float)a.psi_right[m.bc_off + L.n];
    }
    L.base = m.psi_off + dm_index(m.K, m.N, 0, 0, L.n);
    return L;
}

// pass 1 (agg) or pass 2 (write): one segment of one chain per wavefront
template <int SB, bool WRITE>
__global__ void __launch_bounds__(256) sweep_long_pass(BatchLongArgs a) {
    const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= a.nsegs) return;
    const int lane = threadIdx.x & 63;
    const LongSeg sg = a.segs[item];
    const LaneSetup L = long_lane(a, sg);
    const BatchSlab m = a.slabs[sg.slab];
    const v2f *qb = reinterpret_cast<const v2f *>(a.q + L.base);
    v2f *pb = reinterpret_cast<v2f *>(a.psi + L.base);
    const int cs = L.N / 2;
    const float2 *cpb = a.cellpar + m.cell_off;
    const int len = L.active ? sg.c1 - sg.c0 : 0;
    const int smax = sg.c1 - sg.c0;
    const bool fwd = L.fwd;
    const float inv = L.inv;
    auto cell_of = [&](int i) {
        const int ic = min(i, smax - 1);
        return fwd ? sg.c0 + ic : sg.c1 - 1 - ic;
    };
    auto load = [&](CellBatchDM<SB> &b, int i0) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int j = cell_of(i0 + u);
            b.qv[u] = __builtin_nontemporal_load(qb + (long long)j * cs);
            b.cp[u] = cpb[j];
        }
    };
    float A = 1.0f, B = 0.0f;
    float x = WRITE ? a.carry[(size_t)item * 64 + lane] : 0.0f;
    auto body = [&](const CellBatchDM<SB> &b, int i0) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            if (i0 + u < len) {
                const float qi = fwd ? b.qv[u].x : b.qv[u].y, qo = fwd ? b.qv[u].y : b.qv[u].x;
                const float h = b.cp[u].x, tau = b.cp[u].y * inv;
                const float f = h * inv * (1.0f / 6.0f);
                const float gin = f * (2.0f * qi + qo);
                const float gout = f * (qi + 2.0f * qo);
                const float den_inv = __builtin_amdgcn_rcpf(6.0f + tau * (4.0f + tau));
                const float ac = (6.0f - 2.0f * tau) * den_inv;
                const float bc = ((6.0f + 4.0f * tau) * gout + (6.0f - 2.0f * tau) * gin) * den_inv;
                if constexpr (WRITE) {
                    const int j = fwd ? sg.c0 + i0 + u : sg.c1 - 1 - i0 - u;
                    const float vout = ac * x + bc;
                    const float vin = ((6.0f + 4.0f * tau) * (gin + x) - (6.0f + 2.0f * tau) * gout) * den_inv;
                    __builtin_nontemporal_store(fwd ? v2f{vin, vout} : v2f{vout, vin}, pb + (long long)j * cs);
                    x = vout;
                } else {
                    B = ac * B + bc;
                    A = ac * A;
                }
            }
        }
    };
    CellBatchDM<SB> b0, b1, b2;
    load(b0, 0);
    load(b1, SB);
    for (int i0 = 0; i0 < smax; i0 += 3 * SB) {
        load(b2, i0 + 2 * SB);
        body(b0, i0);
        load(b0, i0 + 3 * SB);
        body(b1, i0 + SB);
        load(b1, i0 + 4 * SB);
        body(b2, i0 + 2 * SB);
    }
    if constexpr (!WRITE) a.segAB[(size_t)item * 64 + lane] = float2{A, B};
}

// carry-ins of every segment of a chain, in the chain's sweep direction;
// the segment maps are read 16 at a time ahead of the fold
__global__ void __launch_bounds__(256) sweep_long_scan(BatchLongArgs a) {
    const int chain = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (chain >= a.nchains) return;
    const int lane = threadIdx.x & 63;
    const int first = a.chain_first[chain];
    const LongSeg s0 = a.segs[first];
    const LaneSetup L = long_lane(a, s0);
    const int ns = s0.nseg;
    float x = L.x0;
    for (int t0 = 0; t0 < ns; t0 += 16) {
        float2 ab[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int t = min(t0 + u, ns - 1);
            const int sidx = L.fwd ? t : ns - 1 - t;
            ab[u] = a.segAB[(size_t)(first + sidx) * 64 + lane];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (t0 + u < ns) {
                const int sidx = L.fwd ? t0 + u : ns - 1 - t0 - u;
                a.carry[(size_t)(first + sidx) * 64 + lane] = x;
                x = ab[u].x * x + ab[u].y;
            }
        }
    }
    if (L.active && a.exit) a.exit[a.slabs[s0.slab].exit_off + L.n] = x;
}

void launch_sweep_long(const BatchLongArgs &a, hipStream_t s, KernelTimer *t) {
    if (a.nsegs <= 0) return;
    const dim3 g1((unsigned)((a.nsegs + 3) / 4)), g2((unsigned)((a.nchains + 3) / 4));
    LAUNCH(KID_SWEEP_BATCH, t, (sweep_long_pass<8, false>), g1, dim3(256), 0, s, a);
    LAUNCH(KID_SWEEP_BATCH, t, sweep_long_scan, g2, dim3(256), 0, s, a);
    LAUNCH(KID_SWEEP_BATCH, t, (sweep_long_pass<8, true>), g1, dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------
// Class GEMMs.  MFMA f32 16x16x4 (and bf16 16x16x16)
// layouts: lane l supplies A[l%16][k(l)] and B[k(l)][l%16]; accumulator
// element r of lane l is D[4 (l/16) + r][l%16].
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned short bf16_rne(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

constexpr int TM = 64;

// FP32 class GEMMs: k-steps per B prefetch (KC) and the occupancy asked of
// the compiler.  From W = 64 on, eight-step chunks keep the kernels within
// 168 VGPRs, so three 64-row tiles share a CU (two with sixteen-step
// chunks): one tile's staging then overlaps two others' products.
constexpr int gemm_kc(int W) { return W >= 64 ? 8 : (W / 4 < 16 ? W / 4 : 16); }
constexpr int gemm_waves(int W) { return W >= 64 ? 3 : 1; }
// split-BF16 source GEMM: k-blocks of 16 per B prefetch, fragments staged
// per pass (four-block prefetches keep W >= 128 at two waves per SIMD)
constexpr int SPLIT_KC = 4, SPLIT_FP = 4;

// Padded width W (16 .. 256, a power of two >= the GEMM's K and column
// counts) of a class GEMM; its tiles are staged in LDS at row stride
// W + 4, which spreads the 16 rows x 4 k of an MFMA operand read over all
// banks.
int class_width(int a, int b) {
    const int m = a > b ? a : b;
    int w = 16;
    while (w < m) w *= 2;
    return w;
}

// Stages the TM x W tile with element (r, c) = get(r, c) for r < rows and
// c < cols, zero elsewhere, into LDS at row stride W + 4.  Every thread
// issues all of its loads (clamped to valid positions, no branches) before
// its first store; W = 128 and 256 go in two and four passes (registers).
template <int W, class Get>
__device__ __forceinline__ void stage_tile(float *dst, int rows, int cols, Get &&get) {
    constexpr int CH = W >= 64 ? W / 64 : 1;   // 64-wide column chunks
    constexpr int CW = W >= 64 ? 64 : W;       // lanes per row
    constexpr int RPW = 64 / CW;               // rows per wave per pass
    constexpr int PASSES = W == 256 ? 4 : (W == 128 ? 2 : 1);
    constexpr int RG = TM / (4 * RPW * PASSES); // row groups per pass
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane % CW, rl = lane / CW;
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
        float v[RG][CH];
#pragma unroll
        for (int i = 0; i < RG; ++i)
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int r = ((ps * RG + i) * 4 + wave) * RPW + rl;
                v[i][c] = get(min(r, rows - 1), min(cl + CW * c, cols - 1));
            }
#pragma unroll
        for (int i = 0; i < RG; ++i)
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int r = ((ps * RG + i) * 4 + wave) * RPW + rl, cc = cl + CW * c;
                dst[r * (W + 4) + cc] = (r < rows && cc < cols) ? v[i][c] : 0.0f;
            }
    }
}

// the source GEMMs' moments: FP64 (boundary calls) or FP32 (the solve's
// iterates), a template parameter so that the loads stay unconditional
template <typename PhiT>
__device__ __forceinline__ const PhiT *src_phi(const BatchSrcArgs &g);
template <>
__device__ __forceinline__ const double *src_phi<double>(const BatchSrcArgs &g) { return g.phi; }
template <>
__device__ __forceinline__ const float *src_phi<float>(const BatchSrcArgs &g) {
    if (g.gate.iter) return ((*g.gate.iter - 1) & 1) ? g.buf1 : g.buf0;
    return g.phi32;
}

// Source GEMM epilogue: lane (col, kl) holds rows 16 rb + 4 kl + r of
// column col; adds the prefetched external source and stores q.
__device__ __forceinline__ void src_epilogue(const BatchSrcArgs &g, const BatchSlab &m, const GemmTile &tl, int rows,
                                             int col, int kl, const f4 (&acc)[4], const float (&e)[4][4]) {
    const int N = g.N;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rl = rb * 16 + 4 * kl + r;
            if (rl < rows && col < N) {
                const int row = tl.row0 + rl;
                const size_t od = g.dirmajor ? m.psi_off + dm_index(m.K, N, row >> 1, row & 1, col)
                                             : m.psi_off + (size_t)row * N + col;
                g.q[od] = acc[rb][r] + (g.q_ext ? e[rb][r] : 0.0f);
            }
        }
}

// Source GEMM: block = one tile of TM = 64 node rows of one slab; the A rows
// (phi .* sigma_s, rounded to FP32) are staged in LDS; wave w computes output
// column blocks w, w+4, ... of 16 columns for all four 16-row blocks, so every
// B fragment it reads serves 64 rows.  A column block's B fragments and its
// external-source values are loaded before its products start.
template <int W, typename PhiT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(gemm_waves(W), 8))) src_batch(BatchSrcArgs g) {
    extern __shared__ float sm_src[];
    constexpr int LD = W + 4;
    const int tile = blockIdx.x;
    const GemmTile tl = g.tiles[tile];
    if (slab_done(g.gate, tl.slab)) return;
    const BatchSlab m = g.slabs[tl.slab];
    const PhiT *ph = src_phi<PhiT>(g);
    const int N = g.N, L1 = g.L1;
    const int rows = min(TM, 2 * m.K - tl.row0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float *As = sm_src;  // [TM][W+4]
    stage_tile<W>(As, rows, L1, [&](int r, int l) {
        const long long row = tl.row0 + r;
        return (float)ph[m.phi_off + row * L1 + l] * g.sigma_s[m.ss_off + (row / 2) * L1 + l];
    });
    __syncthreads();
    const int ar = lane & 15, kl = lane >> 4;
    // external source; without one the loads stay unconditional but all
    // read q[0] (one cached line) and their values are not used
    const float *qe = g.q_ext ? g.q_ext : g.q;
    const size_t emask = g.q_ext ? ~(size_t)0 : 0;
    // steps t = (column block wave + 4 (t / NCH), K chunk t % NCH) of KC
    // k-steps each; the next step's B fragments are loaded before the
    // current step's products
    constexpr int KC = gemm_kc(W), NCH = W / 4 / KC;
    const int ncb = (N + 15) / 16;
    const int T = (ncb > wave ? (ncb - wave + 3) / 4 : 0) * NCH;
    auto load_b = [&](int t, float (&bf)[KC]) {
        const int colc = min((wave + 4 * (t / NCH)) * 16 + ar, N - 1), c = t % NCH;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            // k >= L1 meets zero A columns: a clamped (finite) B value
            // needs no select, which would wait for the load here
            const int kk = 4 * (c * KC + k) + kl;
            bf[k] = g.Mt[(size_t)min(kk, L1 - 1) * N + colc];
        }
    };
    float bnext[KC];
    if (T > 0) load_b(0, bnext);
    f4 acc[4];
    float e[4][4];
#pragma unroll 1
    for (int t = 0; t < T; ++t) {
        const int cb = wave + 4 * (t / NCH), c = t % NCH;
        const int col = cb * 16 + ar;
        float bf[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) bf[k] = bnext[k];
        if (c == 0) {
            const int colc = min(col, N - 1);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                acc[rb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = tl.row0 + min(rb * 16 + 4 * kl + r, rows - 1);
                    e[rb][r] = qe[(m.psi_off + (size_t)row * N + colc) & emask];
                }
            }
        }
        if (t + 1 < T) load_b(t + 1, bnext);
#pragma unroll
        for (int k = 0; k < KC; ++k)
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(As[(rb * 16 + ar) * LD + 4 * (c * KC + k) + kl], bf[k],
                                                               acc[rb], 0, 0, 0);
        if (c == NCH - 1) src_epilogue(g, m, tl, rows, col, kl, acc, e);
    }
}

// Split-BF16 source GEMM: x = hi + lo with hi = bf16(x), lo = bf16(x - hi),
// and A B ~ Ahi Bhi + Ahi Blo + Alo Bhi, three bf16 16x16x16 MFMAs with FP32
// accumulation.  The A tile is split once while it is staged, straight into
// MFMA fragment order: fragment (rb, kb) holds rows 16 rb .. 16 rb + 15 and
// k = 16 kb .. 16 kb + 15, lane l's four values A[16 rb + l%16][16 kb +
// 4 (l/16) + i] packed in 8 bytes at slot l, so each operand is one
// conflict-free 8-byte LDS read.  B comes split from setup in the same
// fragment order ([kb][column][l/16], see the class tables).
template <int W, typename PhiT>
__global__ void __launch_bounds__(256) src_batch_split(BatchSrcArgs g) {
    extern __shared__ s4 sm_split[];
    constexpr int KB = W / 16;
    s4 *Ahi = sm_split;            // [4][KB][64]
    s4 *Alo = sm_split + 4 * KB * 64;
    const int tile = blockIdx.x;
    const GemmTile tl = g.tiles[tile];
    if (slab_done(g.gate, tl.slab)) return;
    const BatchSlab m = g.slabs[tl.slab];
    const PhiT *ph = src_phi<PhiT>(g);
    const int N = g.N, L1 = g.L1;
    const int rows = min(TM, 2 * m.K - tl.row0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ar = lane & 15, kl = lane >> 4;
    // wave w stages fragments w, w + 4, ... (KB of them), FP at a time with
    // every load of a pass issued before its first conversion
    {
        constexpr int FP = KB < SPLIT_FP ? KB : SPLIT_FP;
        const int r = min(ar, 15);
#pragma unroll 1
        for (int f0 = 0; f0 < KB; f0 += FP) {
            float v[FP][4];
#pragma unroll
            for (int j = 0; j < FP; ++j) {
                const int f = 4 * (f0 + j) + wave;       // fragment index rb * KB + kb
                const int rl = (f / KB) * 16 + r;
                const long long row = tl.row0 + min(rl, rows - 1);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = (f % KB) * 16 + 4 * kl + i;
                    const int kc = min(k, L1 - 1);
                    v[j][i] = (float)ph[m.phi_off + row * L1 + kc] * g.sigma_s[m.ss_off + (row / 2) * L1 + kc];
                }
            }
#pragma unroll
            for (int j = 0; j < FP; ++j) {
                const int f = 4 * (f0 + j) + wave;
                const int rl = (f / KB) * 16 + r;
                s4 h, lo;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = (f % KB) * 16 + 4 * kl + i;
                    const float x = (rl < rows && k < L1) ? v[j][i] : 0.0f;
                    const unsigned short xh = bf16_rne(x);
                    h[i] = (short)xh;
                    lo[i] = (short)bf16_rne(x - bf16_to_f32(xh));
                }
                Ahi[f * 64 + lane] = h;
                Alo[f * 64 + lane] = lo;
            }
        }
    }
    __syncthreads();
    // external source; without one the loads stay unconditional but all
    // read q[0] (one cached line) and their values are not used
    const float *qe = g.q_ext ? g.q_ext : g.q;
    const size_t emask = g.q_ext ? ~(size_t)0 : 0;
    const s4 *Bh = g.Mt_hi, *Bl = g.Mt_lo;
    // steps as in src_batch: (column block, chunk of KC k-blocks of 16)
    constexpr int KC = KB < SPLIT_KC ? KB : SPLIT_KC, NCH = KB / KC;
    const int ncb = (N + 15) / 16;
    const int T = (ncb > wave ? (ncb - wave + 3) / 4 : 0) * NCH;
    auto load_b = [&](int t, s4 (&bh)[KC], s4 (&bl)[KC]) {
        const int colc = min((wave + 4 * (t / NCH)) * 16 + ar, N - 1), c = t % NCH;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const size_t o = ((size_t)(c * KC + k) * N + colc) * 4 + kl;
            bh[k] = Bh[o];
            bl[k] = Bl[o];
        }
    };
    s4 bhn[KC], bln[KC];
    if (T > 0) load_b(0, bhn, bln);
    f4 acc[4];
    float e[4][4];
#pragma unroll 1
    for (int t = 0; t < T; ++t) {
        const int cb = wave + 4 * (t / NCH), c = t % NCH;
        const int col = cb * 16 + ar;
        s4 bh[KC], bl[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            bh[k] = bhn[k];
            bl[k] = bln[k];
        }
        if (c == 0) {
            const int colc = min(col, N - 1);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                acc[rb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = tl.row0 + min(rb * 16 + 4 * kl + r, rows - 1);
                    e[rb][r] = qe[(m.psi_off + (size_t)row * N + colc) & emask];
                }
            }
        }
        if (t + 1 < T) load_b(t + 1, bhn, bln);
#pragma unroll
        for (int k = 0; k < KC; ++k)
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int f = rb * KB + c * KC + k;
                const s4 ah = Ahi[f * 64 + lane], al = Alo[f * 64 + lane];
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh[k], acc[rb], 0, 0, 0);
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl[k], acc[rb], 0, 0, 0);
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh[k], acc[rb], 0, 0, 0);
            }
        if (c == NCH - 1) src_epilogue(g, m, tl, rows, col, kl, acc, e);
    }
}

// Row units of the persistent kernels: W <= 128 stages whole 64-row tiles
// (two 32-row blocks), W = 256 half tiles (one block), which keeps its 128
// B registers per lane within budget.  Unit u is part u % NP of tile u / NP.
template <int W>
struct PUnit {
    static constexpr int RB = W >= 256 ? 1 : 2;  // 32-row blocks per unit
    static constexpr int ROWS = 32 * RB;
    static constexpr int NP = TM / ROWS;         // units per tile
};

template <int W, typename PhiT>
__global__ void src_batch_p(BatchSrcArgs g);  // persistent FP32 source GEMM (below)
template <int W, typename PhiT>
__global__ void src_batch_sp(BatchSrcArgs g);  // persistent split-BF16 source GEMM (below)

template <int W, typename PhiT>
static void launch_src_wt(const BatchSrcArgs &a, bool split, hipStream_t s, KernelTimer *t) {
    if (split) {
        const std::uint32_t lds = (std::uint32_t)(2 * 4 * (W / 16) * 64 * sizeof(s4));
        LAUNCH(KID_SRC_BATCH, t, (src_batch_split<W, PhiT>), dim3((unsigned)a.ntiles), dim3(256), lds, s, a);
    } else {
        const std::uint32_t lds = (std::uint32_t)(TM * (W + 4) * sizeof(float));
        LAUNCH(KID_SRC_BATCH, t, (src_batch<W, PhiT>), dim3((unsigned)a.ntiles), dim3(256), lds, s, a);
    }
}

template <int W>
static void launch_src_w(const BatchSrcArgs &a, bool split, hipStream_t s, KernelTimer *t) {
    if constexpr (W <= 256) {
        constexpr int WS = W < 32 ? 32 : W;  // W = 16 classes: the 32-wide kernel
        if (a.pblocks_split > 0 && split && a.meta) {
            const std::uint32_t lds = (std::uint32_t)(2 * PUnit<WS>::ROWS * (WS + 4) * sizeof(short));
            if (a.phi32)
                LAUNCH(KID_SRC_BATCH, t, (src_batch_sp<WS, float>), dim3((unsigned)a.pblocks_split), dim3(2 * WS), lds, s, a);
            else
                LAUNCH(KID_SRC_BATCH, t, (src_batch_sp<WS, double>), dim3((unsigned)a.pblocks_split), dim3(2 * WS), lds, s, a);
            return;
        }
    }
    if constexpr (W <= 256) {
        // W = 16 classes run the 32-wide kernel (half its columns zero)
        constexpr int WP = W < 32 ? 32 : W;
        if (a.pblocks > 0 && !split && a.meta) {
            const std::uint32_t lds = (std::uint32_t)(PUnit<WP>::ROWS * (WP + 4) * sizeof(float));
            if (a.phi32)
                LAUNCH(KID_SRC_BATCH, t, (src_batch_p<WP, float>), dim3((unsigned)a.pblocks), dim3(2 * WP), lds, s, a);
            else
                LAUNCH(KID_SRC_BATCH, t, (src_batch_p<WP, double>), dim3((unsigned)a.pblocks), dim3(2 * WP), lds, s, a);
            return;
        }
    }
    if (a.phi32)
        launch_src_wt<W, float>(a, split, s, t);
    else
        launch_src_wt<W, double>(a, split, s, t);
}

void launch_src_batch(const BatchSrcArgs &a, bool split_bf16, hipStream_t s, KernelTimer *t) {
    if (a.ntiles <= 0) return;
    switch (class_width(a.N, a.L1)) {
        case 16: launch_src_w<16>(a, split_bf16, s, t); break;
        case 32: launch_src_w<32>(a, split_bf16, s, t); break;
        case 64: launch_src_w<64>(a, split_bf16, s, t); break;
        case 128: launch_src_w<128>(a, split_bf16, s, t); break;
        default: launch_src_w<256>(a, split_bf16, s, t); break;
    }
}

// Moments GEMM: block = one tile of TM node rows; the psi rows are staged in
// LDS; waves as in src_batch, with the stopping-test references loaded
// before the products.
__device__ void slab_max_reduce(unsigned long long m, unsigned long long *slot) {
    __shared__ unsigned long long red[4];
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 4; ++i) m = red[i] > m ? red[i] : m;
        atomicMax(slot, m);
    }
}

// the moments GEMM's output and stopping-test reference: FP64 (boundary
// calls) or FP32 (the solve's iterates)
template <typename PhiT>
struct MomIO;
template <>
struct MomIO<double> {
    __device__ static double *out(const BatchMomArgs &g) { return g.phi; }
    __device__ static const double *ref(const BatchMomArgs &g) { return g.ref; }
};
template <>
struct MomIO<float> {
    __device__ static float *out(const BatchMomArgs &g) {
        if (g.gate.iter) return (*g.gate.iter & 1) ? g.buf1 : g.buf0;
        return g.phi32;
    }
    __device__ static const float *ref(const BatchMomArgs &g) {
        if (g.gate.iter) return ((*g.gate.iter - 1) & 1) ? g.buf1 : g.buf0;
        return g.ref32;
    }
};

template <int W, typename PhiT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(gemm_waves(W), 8))) mom_batch(BatchMomArgs g) {
    extern __shared__ float sm_mom[];
    constexpr int LD = W + 4;
    const int tile = blockIdx.x;
    const GemmTile tl = g.tiles[tile];
    if (slab_done(g.gate, tl.slab)) return;
    const BatchSlab m = g.slabs[tl.slab];
    const int N = g.N, L1 = g.L1;
    const int rows = min(TM, 2 * m.K - tl.row0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float *Ps = sm_mom;  // [TM][W+4]
    if (g.dirmajor)
        stage_tile<W>(Ps, rows, N, [&](int r, int c) {
            const int row = tl.row0 + r;
            return g.psi[m.psi_off + dm_index(m.K, N, row >> 1, row & 1, c)];
        });
    else
        stage_tile<W>(Ps, rows, N, [&](int r, int c) { return g.psi[m.psi_off + (size_t)(tl.row0 + r) * N + c]; });
    __syncthreads();
    unsigned long long dmax = 0ull;
    const int ar = lane & 15, kl = lane >> 4;
    PhiT *out = MomIO<PhiT>::out(g);
    const PhiT *refp = MomIO<PhiT>::ref(g);
    const bool stop = refp != nullptr;
    // stopping-test reference; without a test the loads all read out[0]
    // (one cached line) and their values are not used
    const PhiT *ref = stop ? refp : out;
    const size_t emask = stop ? ~(size_t)0 : 0;
    // steps as in src_batch: (column block of moments, chunk of KC k-steps)
    constexpr int KC = gemm_kc(W), NCH = W / 4 / KC;
    const int ncb = (L1 + 15) / 16;
    const int T = (ncb > wave ? (ncb - wave + 3) / 4 : 0) * NCH;
    auto load_b = [&](int t, float (&bf)[KC]) {
        const int colc = min((wave + 4 * (t / NCH)) * 16 + ar, L1 - 1), c = t % NCH;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int kk = 4 * (c * KC + k) + kl;
            bf[k] = g.Vt[(size_t)min(kk, N - 1) * L1 + colc];  // as in src_batch
        }
    };
    float bnext[KC];
    if (T > 0) load_b(0, bnext);
    f4 acc[4];
    double e[4][4];
#pragma unroll 1
    for (int t = 0; t < T; ++t) {
        const int cb = wave + 4 * (t / NCH), c = t % NCH;
        const int col = cb * 16 + ar;
        float bf[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) bf[k] = bnext[k];
        if (c == 0) {
            const int colc = min(col, L1 - 1);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                acc[rb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = tl.row0 + min(rb * 16 + 4 * kl + r, rows - 1);
                    const size_t o = m.phi_off + (size_t)row * L1 + colc;
                    e[rb][r] = (double)ref[o & emask];
                }
            }
        }
        if (t + 1 < T) load_b(t + 1, bnext);
#pragma unroll
        for (int k = 0; k < KC; ++k)
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ps[(rb * 16 + ar) * LD + 4 * (c * KC + k) + kl], bf[k],
                                                               acc[rb], 0, 0, 0);
        if (c == NCH - 1) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rl = rb * 16 + 4 * kl + r;
                    if (rl < rows && col < L1) {
                        const size_t o = m.phi_off + (size_t)(tl.row0 + rl) * L1 + col;
                        const double v = (double)acc[rb][r];
                        out[o] = (PhiT)v;
                        if (stop) {
                            const unsigned long long d =
                                (unsigned long long)__double_as_longlong(fabs(v - e[rb][r]));
                            dmax = d > dmax ? d : dmax;
                        }
                    }
                }
        }
    }
    if (stop) {
        unsigned long long *slot = g.gate.iter ? g.gate.hist + hist_row(*g.gate.iter) * g.gate.ns : g.slot;
        slab_max_reduce(dmax, slot + tl.slab);
    }
}


// ---------------------------------------------------------------------------
// Persistent class GEMMs for the solve's FP32 iterates (W = 16 .. 256,
// direction-major q / psi, rows 16-byte aligned).  A block of W / 32 waves
// (wave w owns output columns 32 w .. 32 w + 31 of a row unit, as one 32 x 32
// accumulator per 32 rows; see PUnit) keeps its B fragments in registers for
// its whole life and walks the units blockIdx.x, blockIdx.x + gridDim.x, ...;
// the next unit's operands are requested as 16-byte loads into registers
// right after the current unit is staged, so a wave's memory latency is
// hidden behind its own products and not only behind other blocks'.  Per
// unit a wave requests, in order, its epilogue operands, then the next unit:
// the epilogue waits only for its own operands.  The prefetch is issued
// unconditionally (clamped to the last unit) so that the wait count is the
// same on every path.
//
// Products: MFMA f32 32x32x2 (lane l supplies A[l%32][l/32] and
// B[l/32][l%32]; accumulator element j of lane l is D[8 (j/4) + 4 (l/32) +
// j%4][l%32]).  Two independent 32 x 32 accumulators per wave keep the
// matrix pipe busy where four 16 x 16 chains leave it waiting on their own
// results (measured: 16x16x4 with four chains per wave reaches ~60-80 % of
// the FP32 matrix peak, 32x32x2 with two ~95 %).  Lane group g = l/32 takes
// the contiguous k range g W/2 .. g W/2 + W/2 - 1 (the MFMA sums its two k
// over the groups, so any assignment that A and B share gives the product),
// so one 16-byte LDS read feeds four steps; the row stride W + 4 (4 mod 32
// words) keeps eight lanes' reads on distinct banks.
// ---------------------------------------------------------------------------
typedef float f16v __attribute__((ext_vector_type(16)));

// Four consecutive moments as loaded (FP32 iterates of the solve, or FP64
// at the boundary call), converted to FP32 only when staged, so that a
// prefetch never waits at its own load.
template <typename T>
struct Raw4;
template <>
struct Raw4<float> {
    float4 v;
    __device__ void load(const float *p) { v = *reinterpret_cast<const float4 *>(p); }
    __device__ float4 get() const { return v; }
};
template <>
struct Raw4<double> {
    double2 a, b;
    __device__ void load(const double *p) {
        a = reinterpret_cast<const double2 *>(p)[0];
        b = reinterpret_cast<const double2 *>(p)[1];
    }
    __device__ float4 get() const { return float4{(float)a.x, (float)a.y, (float)b.x, (float)b.y}; }
};


template <int NW>
__device__ void slab_max_reduce_w(unsigned long long m, unsigned long long *slot) {
    __shared__ unsigned long long red[NW];
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NW; ++i) m = red[i] > m ? red[i] : m;
        atomicMax(slot, m);
    }
}

// acc[rb] += A[32 rb .. 32 rb + 31][:] x B over RB row blocks of an LDS
// tile (row stride LD), lane group g on k = g KH .. g KH + KH - 1
template <int LD, int KH, int RB>
__device__ __forceinline__ void mfma32_tile(const float *A, int r32, int g, const float (&breg)[KH], f16v (&acc)[RB]) {
#pragma unroll
    for (int kq = 0; kq < KH / 4; ++kq) {
        float4 av[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
            av[rb] = *reinterpret_cast<const float4 *>(&A[(rb * 32 + r32) * LD + g * KH + 4 * kq]);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rb].x, breg[4 * kq], acc[rb], 0, 0, 0);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
            acc[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rb].y, breg[4 * kq + 1], acc[rb], 0, 0, 0);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
            acc[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rb].z, breg[4 * kq + 2], acc[rb], 0, 0, 0);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
            acc[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rb].w, breg[4 * kq + 3], acc[rb], 0, 0, 0);
    }
}


// tile row of accumulator element j of row block rb for lane group g
__device__ __forceinline__ int acc32_row(int rb, int j, int g) { return rb * 32 + 8 * (j / 4) + 4 * g + (j % 4); }

// Unit pipeline of the persistent class GEMMs.  Block b walks units
// u_k = b + k G.  While unit u_k's products run, the block issues the
// operand loads of u_{k+1} (addresses from its descriptor, already in LDS),
// the gate value of u_{k+1}, and the descriptor of u_{k+3} into registers,
// which the next iteration writes to a four-entry LDS ring: nothing loaded
// in an iteration is used before the next one, so no product waits on
// memory (a descriptor consumed where it is loaded would be moved to scalar
// registers at once, and that wait would also cover the operand prefetch).
// The gate's previous stopping-test values are resolved once per launch.
__device__ __forceinline__ const unsigned long long *gate_prev(const SlabGate &g) {
    if (g.iter) {
        const int m = *g.iter;
        return m > 1 ? g.hist + hist_row(m - 1) * g.ns : nullptr;
    }
    return g.prev;
}
// the gate value of `slab` (prev null: a valid word of `any`, ignored)
__device__ __forceinline__ unsigned long long gate_bits(const unsigned long long *prev, const TileMeta *any, int slab) {
    const unsigned long long *p = prev ? prev : reinterpret_cast<const unsigned long long *>(any);
    return p[prev ? slab : 0];
}
__device__ __forceinline__ bool gate_done(const unsigned long long *prev, unsigned long long bits, double tol) {
    if (!prev) return false;
    const double d = __longlong_as_double((long long)bits);
    return d <= tol || !isfinite(d);
}
// q element of tile row `row`, angle col: direction-major in the solve,
// [cell][node][angle] at the boundary call
__device__ __forceinline__ size_t q_index_m(const BatchSrcArgs &g, const TileMeta &m, int row, int col) {
    const size_t off = 4 * (size_t)m.psi4;
    return g.dirmajor ? off + dm_index(m.K, g.N, row >> 1, row & 1, col) : off + (size_t)row * g.N + col;
}

template <int W, typename PhiT>
__global__ void __launch_bounds__(2 * W) __attribute__((amdgpu_waves_per_eu(2, 8))) src_batch_p(BatchSrcArgs g) {
    extern __shared__ float sm_srcp[];
    constexpr int NT = 2 * W, LD = W + 4, KH = W / 2;
    constexpr int RB = PUnit<W>::RB, UR = PUnit<W>::ROWS, NP = PUnit<W>::NP;
    constexpr int Q = W / 4;          // 16-byte vectors per A row
    constexpr int CSTEP = NT / Q;     // cells staged per pass (8)
    constexpr int CI = UR / 2 / CSTEP;  // passes over the unit's cells
    float *As = sm_srcp;              // [UR][W+4]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r32 = lane & 31, lg = lane >> 5;
    const int N = g.N, L1 = g.L1;
    const PhiT *ph = src_phi<PhiT>(g);
    // external source; without one the loads stay unconditional but all
    // read q[0] (one cached line) and their values are not used
    const float *qe = g.q_ext ? g.q_ext : g.q;
    const size_t emask = g.q_ext ? ~(size_t)0 : 0;
    const bool active = wave * 32 < N;          // the wave's columns exist
    const int col = wave * 32 + r32, colc = min(col, N - 1);
    // B fragments; clamped entries are finite and meet zero A columns or
    // feed unstored outputs
    float breg[KH];
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) breg[kk] = g.Mt[(size_t)min(lg * KH + kk, L1 - 1) * N + colc];
    const int l4 = tid % Q, cg = tid / Q;
    const bool lval = 4 * l4 < L1;
    const int l4c = lval ? l4 : L1 / 4 - 1;
    Raw4<PhiT> pf0[CI], pf1[CI];
    float4 ps[CI];  // phi rows 2c, 2c+1 and sigma_s row c
    auto prefetch = [&](const TileMeta &m, int unit) {
        const int c0 = (m.row0 + (unit % NP) * UR) / 2;
#pragma unroll
        for (int i = 0; i < CI; ++i) {
            const long long cell = min(c0 + cg + CSTEP * i, m.K - 1);
            const PhiT *p = ph + 4 * (size_t)m.phi4 + cell * 2 * L1 + 4 * l4c;
            pf0[i].load(p);
            pf1[i].load(p + L1);
            ps[i] = reinterpret_cast<const float4 *>(g.sigma_s + 4 * (size_t)m.ss4)[cell * m.ss_step + l4c];
        }
    };
    const TileMeta *meta = g.meta;
    const unsigned long long *prev = gate_prev(g.gate);
    const int nunits = g.ntiles * NP, G = (int)gridDim.x;
    if ((int)blockIdx.x >= nunits) return;
    __shared__ TileMeta dring[4];
    const uint2 *mq = reinterpret_cast<const uint2 *>(meta);
    const int qtr = tid & 3;
    auto unit_of = [&](int k) { return min((int)blockIdx.x + k * G, nunits - 1); };
    auto desc = [&](int k) { return mq[4 * (unit_of(k) / NP) + qtr]; };  // quarter of descriptor k
    {
        const uint2 d0 = desc(0), d1 = desc(1);
        if (tid < 4) {
            reinterpret_cast<uint2 *>(&dring[0])[qtr] = d0;
            reinterpret_cast<uint2 *>(&dring[1])[qtr] = d1;
        }
    }
    uint2 dpend = desc(2);
    __syncthreads();
    unsigned long long gb;
    {
        const TileMeta m0 = dring[0];
        prefetch(m0, unit_of(0));
        gb = gate_bits(prev, meta, m0.slab);
    }
#pragma unroll 1
    for (int k = 0;; ++k) {
        const int unit = (int)blockIdx.x + k * G;
        if (unit >= nunits) break;
        __syncthreads();  // the previous tile's products are done with As
        if (tid < 4) reinterpret_cast<uint2 *>(&dring[(k + 2) & 3])[qtr] = dpend;
#pragma unroll
        for (int i = 0; i < CI; ++i) {
            const int c = cg + CSTEP * i;
            const float4 f0 = pf0[i].get(), f1 = pf1[i].get();
            float4 a0, a1;
            a0.x = f0.x * ps[i].x; a0.y = f0.y * ps[i].y; a0.z = f0.z * ps[i].z; a0.w = f0.w * ps[i].w;
            a1.x = f1.x * ps[i].x; a1.y = f1.y * ps[i].y; a1.z = f1.z * ps[i].z; a1.w = f1.w * ps[i].w;
            if (!lval) a0 = a1 = float4{0.f, 0.f, 0.f, 0.f};
            *reinterpret_cast<float4 *>(&As[(2 * c) * LD + 4 * l4]) = a0;
            *reinterpret_cast<float4 *>(&As[(2 * c + 1) * LD + 4 * l4]) = a1;
        }
        __syncthreads();
        const TileMeta mc = dring[k & 3], mn = dring[(k + 1) & 3];
        const int row0 = mc.row0 + (unit % NP) * UR;
        const int rows = min(UR, 2 * mc.K - row0);  // <= 0: the part past a short tile
        const bool skip = rows <= 0 || gate_done(prev, gb, g.gate.tol);
        const bool work = active && !skip;
        float e[RB][16];
        if (work) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int row = row0 + min(acc32_row(rb, j, lg), rows - 1);
                    e[rb][j] = qe[(4 * (size_t)mc.psi4 + (size_t)row * N + colc) & emask];
                }
        }
        prefetch(mn, unit_of(k + 1));
        dpend = desc(k + 3);
        const unsigned long long gbn = gate_bits(prev, meta, mn.slab);
        if (work) {
            f16v acc[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int j = 0; j < 16; ++j) acc[rb][j] = 0.f;
            mfma32_tile<LD, KH, RB>(As, r32, lg, breg, acc);
            if (col < N) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        const int rl = acc32_row(rb, j, lg);
                        if (rl < rows) {
                            const int row = row0 + rl;
                            g.q[q_index_m(g, mc, row, col)] = acc[rb][j] + (g.q_ext ? e[rb][j] : 0.0f);
                        }
                    }
            }
        }
        gb = gbn;
    }
}

template <int W>
__global__ void __launch_bounds__(2 * W) __attribute__((amdgpu_waves_per_eu(2, 8))) mom_batch_p(BatchMomArgs g) {
    extern __shared__ float sm_momp[];
    constexpr int NT = 2 * W, NW = W / 32, LD = W + 4, KH = W / 2;
    constexpr int RB = PUnit<W>::RB, UR = PUnit<W>::ROWS, NP = PUnit<W>::NP;
    constexpr int PR = W / 2;         // angle pairs per cell (one 16-byte vector: 2 nodes x 2 angles)
    constexpr int CSTEP = NT / PR;    // cells staged per pass (4)
    constexpr int CI = UR / 2 / CSTEP;
    float *Ps = sm_momp;              // [UR][W+4]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r32 = lane & 31, lg = lane >> 5;
    const int N = g.N, L1 = g.L1;
    float *out = MomIO<float>::out(g);
    const float *refp = MomIO<float>::ref(g);
    const bool stop = refp != nullptr;
    // stopping-test reference; without a test the loads all read out[0]
    // (one cached line) and their values are not used
    const float *ref = stop ? refp : out;
    const size_t emask = stop ? ~(size_t)0 : 0;
    const bool active = wave * 32 < L1;
    const int col = wave * 32 + r32, colc = min(col, L1 - 1);
    float breg[KH];
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) breg[kk] = g.Vt[(size_t)min(lg * KH + kk, N - 1) * L1 + colc];
    // angle pair (n, n + 1) of this thread in the direction-major layout:
    // half dir, index a within it; pairs beyond N stage zeros
    const int pi = tid % PR, cg = tid / PR;
    const int n = 2 * pi;
    const bool nval = n < N;
    const int nc = nval ? n : N - 2;
    const int dir = nc >= N / 2 ? 1 : 0;
    const int a = nc - dir * (N / 2);
    float4 pf[CI];
    auto prefetch = [&](const TileMeta &m, int unit) {
        const int c0 = (m.row0 + (unit % NP) * UR) / 2;
        const float *base = g.psi + 4 * (size_t)m.psi4 + (long long)dir * m.K * N + 2 * a;
#pragma unroll
        for (int i = 0; i < CI; ++i) {
            const long long cell = min(c0 + cg + CSTEP * i, m.K - 1);
            pf[i] = *reinterpret_cast<const float4 *>(base + cell * N);
        }
    };
    const TileMeta *meta = g.meta;
    const unsigned long long *prev = gate_prev(g.gate);
    // this iteration's stopping-test slots
    unsigned long long *slots = g.gate.iter ? g.gate.hist + hist_row(*g.gate.iter) * g.gate.ns : g.slot;
    const int nunits = g.ntiles * NP, G = (int)gridDim.x;
    if ((int)blockIdx.x >= nunits) return;
    __shared__ TileMeta dring[4];
    const uint2 *mq = reinterpret_cast<const uint2 *>(meta);
    const int qtr = tid & 3;
    auto unit_of = [&](int k) { return min((int)blockIdx.x + k * G, nunits - 1); };
    auto desc = [&](int k) { return mq[4 * (unit_of(k) / NP) + qtr]; };  // quarter of descriptor k
    {
        const uint2 d0 = desc(0), d1 = desc(1);
        if (tid < 4) {
            reinterpret_cast<uint2 *>(&dring[0])[qtr] = d0;
            reinterpret_cast<uint2 *>(&dring[1])[qtr] = d1;
        }
    }
    uint2 dpend = desc(2);
    __syncthreads();
    unsigned long long gb;
    {
        const TileMeta m0 = dring[0];
        prefetch(m0, unit_of(0));
        gb = gate_bits(prev, meta, m0.slab);
    }
#pragma unroll 1
    for (int k = 0;; ++k) {
        const int unit = (int)blockIdx.x + k * G;
        if (unit >= nunits) break;
        __syncthreads();  // the previous tile's products are done with Ps
        if (tid < 4) reinterpret_cast<uint2 *>(&dring[(k + 2) & 3])[qtr] = dpend;
#pragma unroll
        for (int i = 0; i < CI; ++i) {
            const int c = cg + CSTEP * i;
            const float4 v = nval ? pf[i] : float4{0.f, 0.f, 0.f, 0.f};
            // vector element 2 t + nd is (node nd, angle n + t)
            *reinterpret_cast<float2 *>(&Ps[(2 * c) * LD + n]) = float2{v.x, v.z};
            *reinterpret_cast<float2 *>(&Ps[(2 * c + 1) * LD + n]) = float2{v.y, v.w};
        }
        __syncthreads();
        const TileMeta mc = dring[k & 3], mn = dring[(k + 1) & 3];
        const int row0 = mc.row0 + (unit % NP) * UR;
        const int rows = min(UR, 2 * mc.K - row0);  // <= 0: the part past a short tile
        const bool skip = rows <= 0 || gate_done(prev, gb, g.gate.tol);
        const bool work = active && !skip;
        float e[RB][16];
        if (work) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int row = row0 + min(acc32_row(rb, j, lg), rows - 1);
                    e[rb][j] = ref[(4 * (size_t)mc.phi4 + (size_t)row * L1 + colc) & emask];
                }
        }
        prefetch(mn, unit_of(k + 1));
        dpend = desc(k + 3);
        const unsigned long long gbn = gate_bits(prev, meta, mn.slab);
        unsigned long long dmax = 0ull;
        if (!skip && active) {
            f16v acc[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int j = 0; j < 16; ++j) acc[rb][j] = 0.f;
            mfma32_tile<LD, KH, RB>(Ps, r32, lg, breg, acc);
            if (col < L1) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        const int rl = acc32_row(rb, j, lg);
                        if (rl < rows) {
                            const size_t o = 4 * (size_t)mc.phi4 + (size_t)(row0 + rl) * L1 + col;
                            const double v = (double)acc[rb][j];
                            out[o] = (float)v;
                            if (stop) {
                                const unsigned long long d =
                                    (unsigned long long)__double_as_longlong(fabs(v - (double)e[rb][j]));
                                dmax = d > dmax ? d : dmax;
                            }
                        }
                    }
            }
        }
        if (stop && !skip) slab_max_reduce_w<NW>(dmax, slots + mc.slab);  // skip is uniform over the block
        gb = gbn;
    }
}


// Split-BF16 source GEMM in the persistent form of src_batch_p (W = 16 ..
// 256 in row units as there, W = 16 classes on the 32-wide kernel): the staged A = phi .* sigma_s is split into bf16 hi + lo while it is
// written to LDS (two [UR][W+4] bf16 arrays, row stride 66 words at W = 128,
// so sixteen lanes' 8-byte reads hit distinct banks), the split B fragments
// come from the class tables (entry (k0 / 16, n, (k0 % 16) / 4) holds
// k = k0 .. k0 + 3 of column n) into registers, and each step of four k
// runs A_hi B_hi + A_hi B_lo + A_lo B_hi as three MFMA 32x32x8 bf16 with
// FP32 accumulation (lane l supplies A[l%32][4 (l/32) + i] and
// B[4 (l/32) + i][l%32], i < 4; output layout as the f32 32x32 MFMA).
template <int W, typename PhiT>
__global__ void __launch_bounds__(2 * W) __attribute__((amdgpu_waves_per_eu(2, 8))) src_batch_sp(BatchSrcArgs g) {
    extern __shared__ short sm_srcsp[];
    constexpr int NT = 2 * W, LDH = W + 4, KH = W / 2, NS = KH / 4;
    constexpr int RB = PUnit<W>::RB, UR = PUnit<W>::ROWS, NP = PUnit<W>::NP;
    constexpr int Q = W / 4, CSTEP = NT / Q, CI = UR / 2 / CSTEP;
    short *Ahi = sm_srcsp, *Alo = sm_srcsp + UR * LDH;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r32 = lane & 31, lg = lane >> 5;
    const int N = g.N, L1 = g.L1;
    const PhiT *ph = src_phi<PhiT>(g);
    // external source; without one the loads stay unconditional but all
    // read q[0] (one cached line) and their values are not used
    const float *qe = g.q_ext ? g.q_ext : g.q;
    const size_t emask = g.q_ext ? ~(size_t)0 : 0;
    const bool active = wave * 32 < N;
    const int col = wave * 32 + r32, colc = min(col, N - 1);
    s4 bh[NS], bl[NS];
#pragma unroll
    for (int st = 0; st < NS; ++st) {
        const int k0 = lg * KH + 4 * st;
        const size_t o = ((size_t)(k0 / 16) * N + colc) * 4 + (k0 % 16) / 4;
        bh[st] = g.Mt_hi[o];
        bl[st] = g.Mt_lo[o];
    }
    const int l4 = tid % Q, cg = tid / Q;
    const bool lval = 4 * l4 < L1;
    const int l4c = lval ? l4 : L1 / 4 - 1;
    Raw4<PhiT> pf0[CI], pf1[CI];
    float4 ps[CI];
    auto prefetch = [&](const TileMeta &m, int unit) {
        const int c0 = (m.row0 + (unit % NP) * UR) / 2;
#pragma unroll
        for (int i = 0; i < CI; ++i) {
            const long long cell = min(c0 + cg + CSTEP * i, m.K - 1);
            const PhiT *p = ph + 4 * (size_t)m.phi4 + cell * 2 * L1 + 4 * l4c;
            pf0[i].load(p);
            pf1[i].load(p + L1);
            ps[i] = reinterpret_cast<const float4 *>(g.sigma_s + 4 * (size_t)m.ss4)[cell * m.ss_step + l4c];
        }
    };
    auto split_store = [&](int row, float4 a) {
        const float x[4] = {a.x, a.y, a.z, a.w};
        s4 h, lo;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const unsigned short xh = bf16_rne(x[i]);
            h[i] = (short)xh;
            lo[i] = (short)bf16_rne(x[i] - bf16_to_f32(xh));
        }
        *reinterpret_cast<s4 *>(&Ahi[row * LDH + 4 * l4]) = h;
        *reinterpret_cast<s4 *>(&Alo[row * LDH + 4 * l4]) = lo;
    };
    const TileMeta *meta = g.meta;
    const unsigned long long *prev = gate_prev(g.gate);
    const int nunits = g.ntiles * NP, G = (int)gridDim.x;
    if ((int)blockIdx.x >= nunits) return;
    __shared__ TileMeta dring[4];
    const uint2 *mq = reinterpret_cast<const uint2 *>(meta);
    const int qtr = tid & 3;
    auto unit_of = [&](int k) { return min((int)blockIdx.x + k * G, nunits - 1); };
    auto desc = [&](int k) { return mq[4 * (unit_of(k) / NP) + qtr]; };  // quarter of descriptor k
    {
        const uint2 d0 = desc(0), d1 = desc(1);
        if (tid < 4) {
            reinterpret_cast<uint2 *>(&dring[0])[qtr] = d0;
            reinterpret_cast<uint2 *>(&dring[1])[qtr] = d1;
        }
    }
    uint2 dpend = desc(2);
    __syncthreads();
    unsigned long long gb;
    {
        const TileMeta m0 = dring[0];
        prefetch(m0, unit_of(0));
        gb = gate_bits(prev, meta, m0.slab);
    }
#pragma unroll 1
    for (int k = 0;; ++k) {
        const int unit = (int)blockIdx.x + k * G;
        if (unit >= nunits) break;
        __syncthreads();  // the previous tile's products are done with Ahi / Alo
        if (tid < 4) reinterpret_cast<uint2 *>(&dring[(k + 2) & 3])[qtr] = dpend;
#pragma unroll
        for (int i = 0; i < CI; ++i) {
            const int c = cg + CSTEP * i;
            const float4 f0 = pf0[i].get(), f1 = pf1[i].get();
            float4 a0, a1;
            a0.x = f0.x * ps[i].x; a0.y = f0.y * ps[i].y; a0.z = f0.z * ps[i].z; a0.w = f0.w * ps[i].w;
            a1.x = f1.x * ps[i].x; a1.y = f1.y * ps[i].y; a1.z = f1.z * ps[i].z; a1.w = f1.w * ps[i].w;
            if (!lval) a0 = a1 = float4{0.f, 0.f, 0.f, 0.f};
            split_store(2 * c, a0);
            split_store(2 * c + 1, a1);
        }
        __syncthreads();
        const TileMeta mc = dring[k & 3], mn = dring[(k + 1) & 3];
        const int row0 = mc.row0 + (unit % NP) * UR;
        const int rows = min(UR, 2 * mc.K - row0);  // <= 0: the part past a short tile
        const bool skip = rows <= 0 || gate_done(prev, gb, g.gate.tol);
        const bool work = active && !skip;
        float e[RB][16];
        if (work) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int row = row0 + min(acc32_row(rb, j, lg), rows - 1);
                    e[rb][j] = qe[(4 * (size_t)mc.psi4 + (size_t)row * N + colc) & emask];
                }
        }
        prefetch(mn, unit_of(k + 1));
        dpend = desc(k + 3);
        const unsigned long long gbn = gate_bits(prev, meta, mn.slab);
        if (work) {
            f16v acc[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int j = 0; j < 16; ++j) acc[rb][j] = 0.f;
#pragma unroll
            for (int st = 0; st < NS; ++st) {
                s4 ah[RB], al[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const int o = (rb * 32 + r32) * LDH + lg * KH + 4 * st;
                    ah[rb] = *reinterpret_cast<const s4 *>(&Ahi[o]);
                    al[rb] = *reinterpret_cast<const s4 *>(&Alo[o]);
                }
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[rb], bh[st], acc[rb], 0, 0, 0);
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[rb], bl[st], acc[rb], 0, 0, 0);
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al[rb], bh[st], acc[rb], 0, 0, 0);
                }
            }
            if (col < N) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        const int rl = acc32_row(rb, j, lg);
                        if (rl < rows) {
                            const int row = row0 + rl;
                            g.q[q_index_m(g, mc, row, col)] = acc[rb][j] + (g.q_ext ? e[rb][j] : 0.0f);
                        }
                    }
            }
        }
        gb = gbn;
    }
}

// ---------------------------------------------------------------------------
// Fused source iteration.  Block = one tile of kFusedCells cells (64 node
// rows) of one slab, 2W threads (W / 32 waves, wave w on output columns
// 32 w .. 32 w + 31 of the 32x32x2 FP32 MFMA products, as in the class
// GEMMs).  One LDS array [64][W+4] holds in turn A = phi .* sigma_s, the
// source q (angle columns, zero past N) and, in the apply pass, the fluxes
// psi that replace q in place; threads n and W + n (n < N) run angle n's
// recurrence over the two halves of the tile's cells.
// ---------------------------------------------------------------------------
bool fused_class_ok(int N, int L1) { return class_width(N, L1) <= 128 && N % 4 == 0 && L1 % 4 == 0 && N >= 4; }

// Products of the fused passes from BF16 pieces of the FP32 operands:
// x = p0 + p1 + p2 with p0 = bf16(x), p1 = bf16(x - p0), p2 = bf16(x - p0 -
// p1) (each difference exact in FP32).  A is staged as NP piece arrays
// [64][W+8] bf16 in LDS (16-byte aligned rows, 4 words mod 32 apart so the
// eight lanes of a 16-byte read phase hit distinct banks), B pieces come
// from the class tables into registers, and each step of eight k runs the
// cross products p_i q_j with i + j < NP on MFMA 32x32x16 bf16 (lane l
// supplies A[l%32][k] and B[k][l%32] for eight k of its group's range) with
// FP32 accumulation: NP = 3, six products, rounds like FP32 (the terms left
// out are below 2^-24 of the result); NP = 2, three products, the
// split-BF16 precision.  Output layout as the f32 32x32 MFMA.
template <int NP, int LDH>
__device__ __forceinline__ void store_pieces(short *P, int row, int v, float4 a) {
    const float x[4] = {a.x, a.y, a.z, a.w};
    s4 pc[NP];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float r = x[t];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const unsigned short h = bf16_rne(r);
            pc[q][t] = (short)h;
            r -= bf16_to_f32(h);
        }
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) *reinterpret_cast<s4 *>(&P[q * 64 * LDH + row * LDH + 4 * v]) = pc[q];
}

// b[q][st]: piece q of this lane's B values k = lg KH + 8 st .. + 7 of
// column c (class table entries (k0 / 16, c, (k0 % 16) / 4) and the next)
template <int NP, int NS8, int KH>
__device__ __forceinline__ void load_pieces(const short4_t *const (&T)[3], int ncols, int c, int lg,
                                            bf8 (&b)[NP][NS8]) {
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int st = 0; st < NS8; ++st) {
            const int k0 = lg * KH + 8 * st;
            b[q][st] = *reinterpret_cast<const bf8 *>(&T[q][((k0 / 16) * ncols + c) * 4 + (k0 % 16) / 4]);
        }
}

// acc[rb] += A[32 rb + l%32][:] B over the pieces
template <int NP, int RB, int NS8, int KH, int LDH>
__device__ __forceinline__ void pieces_product(const short *P, int r32, int lg, const bf8 (&b)[NP][NS8],
                                               f16v (&acc)[RB]) {
#pragma unroll
    for (int st = 0; st < NS8; ++st) {
        bf8 a[NP][RB];
#pragma unroll
        for (int q = 0; q < NP; ++q)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                a[q][rb] = *reinterpret_cast<const bf8 *>(&P[q * 64 * LDH + (rb * 32 + r32) * LDH + lg * KH + 8 * st]);
#pragma unroll
        for (int i = 0; i < NP; ++i)
#pragma unroll
            for (int j = 0; i + j < NP; ++j)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][rb], b[j][st], acc[rb], 0, 0, 0);
    }
}

// waves per SIMD the register budget is sized for: three for the 128-wide
// passes with three pieces (their 52 KB of LDS fit three blocks per CU) and
// the apply passes from 64 wide (staged rows or the moments' B fragments
// held through the recurrence), four for the others
template <int W, bool APPLY, int SPS>
struct FusedOcc {
    static constexpr int value = ((W == 128 && SPS == 3) || (APPLY && W >= 64)) ? 3 : 4;
};

// SPS: pieces of the source product.  FP32 handles take three for the
// source and the moments (SPS = 3), or at 32 wide form both on FP32 MFMA
// (SPS = 0: 32x32x2 f32, B fragments in registers; the pieces' staging
// costs more than their products save there); split-BF16 handles (SPS = 2)
// take two for the source and form the moments on FP32 MFMA, so that their
// iterates still settle at FP32 rounding.
template <int W, bool APPLY, int SPS>
__global__ void __launch_bounds__(2 * W) __attribute__((amdgpu_waves_per_eu(FusedOcc<W, APPLY, SPS>::value, 8)))
fused_tile(BatchFusedArgs g) {
    extern __shared__ float sm_fz[];
    constexpr int NT = 2 * W, NW = W / 32, LD = W + 4, KH = W / 2, RB = 2;
    constexpr int Q = W / 4;                // 16-byte vectors per A row
    constexpr int CSTEP = NT / Q;           // cells staged per pass (8)
    constexpr int CI = kFusedCells / CSTEP; // passes (4)
    constexpr int LDH = W + 8, NS8 = KH / 8;
    float *As = sm_fz;                                            // [64][W+4] FP32: q, then psi, then phi
    short *P = reinterpret_cast<short *>(sm_fz);                  // [SPS][64][W+8] bf16 pieces (the same bytes)
    float2 *cps = reinterpret_cast<float2 *>(P + (SPS == 3 ? 3 : 2) * 64 * LDH);  // [kFusedCells] {h, sigma_t h}
    const FusedTile tl = g.tiles[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r32 = lane & 31, lg = lane >> 5;
    const int N = g.N, L1 = g.L1;
    const int c0 = tl.row0 / 2;
    const int nc = min(kFusedCells, tl.K - c0), rows = 2 * nc;
    const float *ph = g.gate.iter ? (((*g.gate.iter - 1) & 1) ? g.buf1 : g.buf0) : g.phi32;
    const float *phb = ph + 4 * (size_t)tl.phi4 + (size_t)tl.row0 * L1;  // the tile's first row
    const bool iso = g.e0 && tl.iso;
    // the recurrence's per-angle values, requested first: thread (hf, n)
    // sweeps angle n over half hf of the tile's cells in sweep order (the
    // inflows of both halves arrive as one 8-byte word; one is used)
    const int hf = tid / W, n = tid - hf * W, na = min(n, N - 1);
    const float sinv_n = g.sinv[tl.quad_off + na];
    const float2 cin = APPLY ? *reinterpret_cast<const float2 *>(g.carry + tl.ab + 2 * na) : float2{0.0f, 0.0f};
    // A = phi .* sigma_s, rows of cells past the slab's end zero; an
    // isotropic external source e0 is added to column 0 as 2 e0 (the
    // l = 0 row of Mt is 1/2).  The slab's convergence gate is resolved
    // after these loads are requested.  Thread (l4, cg) stages columns
    // 4 l4 .. 4 l4 + 3 of rows 2c, 2c + 1 for c = cg + 8 i; up to 64-wide
    // apply passes keep these rows (the current iterate) in registers for
    // the stopping test, written out in the same layout.
    constexpr bool KEEP = APPLY && W < 128;
    const int l4 = tid % Q, cg = tid / Q;
    const bool lval = 4 * l4 < L1;
    float4 f0[CI], f1[CI];
    {
        const int l4c = lval ? l4 : L1 / 4 - 1;
        const float4 *ssb = reinterpret_cast<const float4 *>(g.sigma_s + 4 * (size_t)tl.ss4);
        float4 sv[CI];
        float2 ev[CI];
        const float *e0 = g.e0 ? g.e0 : g.sigma_s;  // read only when iso
#pragma unroll
        for (int i = 0; i < CI; ++i) {
            const int c = min(cg + CSTEP * i, nc - 1);
            const float *p = phb + (c * 2 * L1 + 4 * l4c);
            f0[i] = *reinterpret_cast<const float4 *>(p);
            f1[i] = *reinterpret_cast<const float4 *>(p + L1);
            sv[i] = ssb[(long long)(c0 + c) * tl.ss_step + l4c];
            ev[i] = *reinterpret_cast<const float2 *>(e0 + (iso ? 2 * (size_t)(tl.cell0 + c) : 0));
        }
        if (slab_done(g.gate, tl.slab)) return;  // uniform over the block
#pragma unroll
        for (int i = 0; i < CI; ++i) {
            const int c = cg + CSTEP * i;
            float4 a0, a1;
            a0.x = f0[i].x * sv[i].x; a0.y = f0[i].y * sv[i].y; a0.z = f0[i].z * sv[i].z; a0.w = f0[i].w * sv[i].w;
            a1.x = f1[i].x * sv[i].x; a1.y = f1[i].y * sv[i].y; a1.z = f1[i].z * sv[i].z; a1.w = f1[i].w * sv[i].w;
            if (iso && l4 == 0) {
                a0.x += 2.0f * ev[i].x;
                a1.x += 2.0f * ev[i].y;
            }
            if (!lval || c >= nc) a0 = a1 = float4{0.f, 0.f, 0.f, 0.f};
            if constexpr (SPS == 0) {
                *reinterpret_cast<float4 *>(&As[(2 * c) * LD + 4 * l4]) = a0;
                *reinterpret_cast<float4 *>(&As[(2 * c + 1) * LD + 4 * l4]) = a1;
            } else {
                store_pieces<SPS, LDH>(P, 2 * c, l4, a0);
                store_pieces<SPS, LDH>(P, 2 * c + 1, l4, a1);
            }
        }
    }
    if (tid < kFusedCells) cps[tid] = g.cellpar[tl.cell0 + min(tid, nc - 1)];
    const int col = wave * 32 + r32;
    const int colc = min(col, N - 1), colm = min(col, L1 - 1);
    f16v acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[rb][j] = 0.f;
    float breg[SPS != 3 ? KH : 1];  // FP32 B fragments (SPS = 0: Mt, then Vt; SPS = 2: Vt)
    if constexpr (SPS == 0) {
#pragma unroll
        for (int kk = 0; kk < KH; ++kk) breg[kk] = g.Mt[min(lg * KH + kk, L1 - 1) * N + colc];
        __syncthreads();
        mfma32_tile<LD, KH, RB>(As, r32, lg, breg, acc);
    } else {
        bf8 b[SPS][NS8];
        load_pieces<SPS, NS8, KH>(g.Mt3, N, colc, lg, b);
        __syncthreads();
        pieces_product<SPS, RB, NS8, KH, LDH>(P, r32, lg, b, acc);
    }
    __syncthreads();  // every wave is done with A
    // q into the same array (angle columns past N zero: the moments product
    // meets them with clamped Vt rows)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int j = 0; j < 16; ++j) As[acc32_row(rb, j, lg) * LD + col] = col < N ? acc[rb][j] : 0.0f;
    // FP32 moments: their B fragments, requested before the recurrence (not
    // hoisted above the source product)
    if (APPLY && SPS != 3) {
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int kk = 0; kk < KH; ++kk) breg[kk] = g.Vt[min(lg * KH + kk, N - 1) * L1 + colm];
    }
    // a per-angle external source, added in 16-byte vectors of its rows
    if (g.q_ext && !iso) {
        __syncthreads();
        const float4 *qe = reinterpret_cast<const float4 *>(g.q_ext + 4 * (size_t)tl.psi4 + (size_t)tl.row0 * N);
        const int nq = N / 4;
        for (int i = tid; i < rows * nq; i += NT) {
            const int row = i / nq, v = i - row * nq;
            const float4 e = qe[i];
            float4 *d = reinterpret_cast<float4 *>(&As[row * LD + 4 * v]);
            float4 q = *d;
            q.x += e.x; q.y += e.y; q.z += e.z; q.w += e.w;
            *d = q;
        }
    }
    __syncthreads();
    // LD recurrence of angle n over half hf of the tile's cells in its sweep
    // direction (the same arithmetic as the batched sweep): the aggregate
    // pass from a zero inflow, keeping the product of the inflow factors, the
    // apply pass from the half's inflow.  The half's map entry is
    // ab + 2 n + p with p its spatial position (0: the lower cells).
    const bool fwd = sinv_n > 0.0f;
    const float inv = fabsf(sinv_n);
    const int in_node = fwd ? 0 : 1;
    const int hs = (nc + 1) / 2, ub = hf ? hs : 0, ue = hf ? nc : hs;
    const int p = fwd ? hf : 1 - hf;
    if (n < N) {
        float x = p ? cin.y : cin.x, al = 1.0f;
        // groups of 8 cells: the group's LDS reads first, then its chain
        constexpr int GC = 8;
#pragma unroll 1
        for (int u0 = ub; u0 < ue; u0 += GC) {
            float qiv[GC], qov[GC];
            float2 cpv[GC];
#pragma unroll
            for (int v = 0; v < GC; ++v) {
                const int uu = min(u0 + v, ue - 1), c = fwd ? uu : nc - 1 - uu;
                qiv[v] = As[(2 * c + in_node) * LD + n];
                qov[v] = As[(2 * c + 1 - in_node) * LD + n];
                cpv[v] = cps[c];
            }
#pragma unroll
            for (int v = 0; v < GC; ++v) {
                if (u0 + v >= ue) break;
                const int c = fwd ? u0 + v : nc - 1 - u0 - v;
                const float qi = qiv[v], qo = qov[v];
                const float2 cp = cpv[v];
                const float h = cp.x, tau = cp.y * inv;
                const float f = h * inv * (1.0f / 6.0f);
                const float gin = f * (2.0f * qi + qo);
                const float gout = f * (qi + 2.0f * qo);
                const float den_inv = __builtin_amdgcn_rcpf(6.0f + tau * (4.0f + tau));
                const float vout = ((6.0f - 2.0f * tau) * x + (6.0f + 4.0f * tau) * gout + (6.0f - 2.0f * tau) * gin) *
                                   den_inv;
                if (APPLY) {
                    As[(2 * c + in_node) * LD + n] = ((6.0f + 4.0f * tau) * (gin + x) - (6.0f + 2.0f * tau) * gout) *
                                                      den_inv;
                    As[(2 * c + 1 - in_node) * LD + n] = vout;
                } else {
                    al *= (6.0f - 2.0f * tau) * den_inv;
                }
                x = vout;
            }
        }
        if (!APPLY) {
            g.alpha[tl.ab + 2 * n + p] = al;
            g.beta[tl.ab + 2 * n + p] = x;
        }
    }
    if (!APPLY) return;
    constexpr int PER = 64 * Q / NT;  // 16-byte vectors per thread
    // the 128-wide passes' stopping-test reference rows (the current
    // iterate) in the layout of the output pass below, requested before the
    // moments product (two pieces) or after it (three, whose registers they
    // would exceed during it)
    const int nl = L1 / 4, nvec = rows * nl;
    constexpr bool PRE = !KEEP;
    const float4 *pb = reinterpret_cast<const float4 *>(phb);
    float4 po[PER];
    auto request_ref = [&]() {
#pragma unroll
        for (int u = 0; u < PER; ++u) po[u] = pb[min(tid + u * NT, nvec - 1)];
    };
    if (PRE && SPS != 3) request_ref();
    __syncthreads();
    // moments phi = psi Vt of the tile's rows
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[rb][j] = 0.f;
    if constexpr (SPS == 3) {
        // psi as three pieces in the same bytes (read whole, then written)
        {
            float4 pv[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int i = tid + u * NT, row = i / Q, v = i - row * Q;
                pv[u] = *reinterpret_cast<const float4 *>(&As[row * LD + 4 * v]);
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int i = tid + u * NT, row = i / Q, v = i - row * Q;
                store_pieces<3, LDH>(P, row, v, pv[u]);
            }
        }
        bf8 b[3][NS8];
        load_pieces<3, NS8, KH>(g.Vt3, L1, colm, lg, b);
        __syncthreads();
        pieces_product<3, RB, NS8, KH, LDH>(P, r32, lg, b, acc);
        if (PRE) request_ref();
    } else {
        mfma32_tile<LD, KH, RB>(As, r32, lg, breg, acc);
    }
    __syncthreads();  // every wave is done with psi
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int j = 0; j < 16; ++j) As[acc32_row(rb, j, lg) * LD + col] = acc[rb][j];
    __syncthreads();
    // the new iterate out in 16-byte vectors, with the stopping test
    // max |phi_new - phi_old| (in FP64) against the current iterate
    float *out = g.gate.iter ? ((*g.gate.iter & 1) ? const_cast<float *>(g.buf1) : const_cast<float *>(g.buf0))
                             : g.out32;
    unsigned long long *slots = g.gate.iter ? g.gate.hist + hist_row(*g.gate.iter) * g.gate.ns : g.slot;
    float4 *ob = reinterpret_cast<float4 *>(out + 4 * (size_t)tl.phi4 + (size_t)tl.row0 * L1);
    unsigned long long dmax = 0ull;
    auto test = [&](float4 nv, float4 o) {
        const double d = fmax(fmax(fabs((double)nv.x - (double)o.x), fabs((double)nv.y - (double)o.y)),
                              fmax(fabs((double)nv.z - (double)o.z), fabs((double)nv.w - (double)o.w)));
        const unsigned long long b = (unsigned long long)__double_as_longlong(d);
        dmax = b > dmax ? b : dmax;
    };
    if constexpr (KEEP) {
        if (lval) {
#pragma unroll
            for (int i = 0; i < CI; ++i) {
                const int c = cg + CSTEP * i;
                if (c < nc) {
                    const float4 n0 = *reinterpret_cast<const float4 *>(&As[(2 * c) * LD + 4 * l4]);
                    const float4 n1 = *reinterpret_cast<const float4 *>(&As[(2 * c + 1) * LD + 4 * l4]);
                    ob[(2 * c) * nl + l4] = n0;
                    ob[(2 * c + 1) * nl + l4] = n1;
                    test(n0, f0[i]);
                    test(n1, f1[i]);
                }
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = tid + u * NT;
            if (i >= nvec) break;
            const int row = i / nl, v = i - row * nl;
            const float4 nv = *reinterpret_cast<const float4 *>(&As[row * LD + 4 * v]);
            ob[i] = nv;
            test(nv, PRE ? po[u] : pb[i]);
        }
    }
    if (slots) slab_max_reduce_w<NW>(dmax, slots + tl.slab);
}

// Inflow of every half-tile: per (slab, angle) the half-tile maps in sweep
// order, x_in(next) = alpha x_in + beta from the face inflow; the last
// outflow is the far-face exit.  A tile's two maps of one angle are adjacent
// (lower half first) and move as one 8-byte word; batches of 16 tiles are
// loaded one batch ahead.
__global__ void __launch_bounds__(128) fused_scan(BatchFusedScanArgs a) {
    const int slab = blockIdx.x, n = threadIdx.x;
    const BatchSlab m = a.slabs[slab];
    if (n >= m.N || slab_done(a.gate, slab)) return;
    const int N = m.N, T = (m.K + kFusedCells - 1) / kFusedCells;
    const bool fwd = a.mu[m.quad_off + n] > 0.0;
    float x = 0.0f;
    if (fwd) {
        if (a.psi_left) x = (float)a.psi_left[m.bc_off + n - N / 2];
    } else {
        if (a.psi_right) x = (float)a.psi_right[m.bc_off + n];
    }
    const float2 *al = reinterpret_cast<const float2 *>(a.alpha + m.ab_off) + n;
    const float2 *be = reinterpret_cast<const float2 *>(a.beta + m.ab_off) + n;
    float2 *cr = reinterpret_cast<float2 *>(a.carry + m.ab_off) + n;
    constexpr int B = 16;
    auto tile_of = [&](int i) { return fwd ? min(i, T - 1) : max(T - 1 - i, 0); };
    float2 a0[B], b0[B], a1[B], b1[B];
    auto load = [&](float2 (&av)[B], float2 (&bv)[B], int i0) {
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const size_t t = (size_t)tile_of(i0 + u) * N;
            av[u] = al[t];
            bv[u] = be[t];
        }
    };
    auto run = [&](const float2 (&av)[B], const float2 (&bv)[B], int i0) {
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (i0 + u < T) {
                float2 c;
                if (fwd) {
                    c.x = x;
                    x = av[u].x * x + bv[u].x;
                    c.y = x;
                    x = av[u].y * x + bv[u].y;
                } else {
                    c.y = x;
                    x = av[u].y * x + bv[u].y;
                    c.x = x;
                    x = av[u].x * x + bv[u].x;
                }
                cr[(size_t)tile_of(i0 + u) * N] = c;
            }
    };
    load(a0, b0, 0);
    for (int i0 = 0; i0 < T; i0 += 2 * B) {
        load(a1, b1, i0 + B);
        run(a0, b0, i0);
        load(a0, b0, i0 + 2 * B);
        run(a1, b1, i0 + B);
    }
    if (a.exit) a.exit[m.exit_off + n] = x;
}

// Isotropy of q_ext per tile: block = one tile; the tile's rows are read
// in 16-byte vectors, each compared with its row's first value.
__global__ void __launch_bounds__(256) fused_iso(BatchIsoArgs a) {
    FusedTile &tl = a.tiles[blockIdx.x];
    const int N = a.N, tid = threadIdx.x;
    const int rows = 2 * min(kFusedCells, tl.K - tl.row0 / 2);
    const float *q = a.q_ext + 4 * (size_t)tl.psi4 + (size_t)tl.row0 * N;
    const float4 *q4 = reinterpret_cast<const float4 *>(q);
    const int nv = rows * (N / 4);
    bool same = true;
    for (int i = tid; i < nv; i += 256) {
        const float4 v = q4[i];
        const float f = q[(4 * i / N) * N];
        same = same && v.x == f && v.y == f && v.z == f && v.w == f;
    }
    if (tid < rows) a.e0[2 * (size_t)tl.cell0 + tid] = q[tid * N];
    const int all = __syncthreads_and(same ? 1 : 0);
    if (tid == 0) tl.iso = all;
}

template <int W>
static void launch_fused_w(const BatchFusedArgs &a, bool apply, hipStream_t s, KernelTimer *t) {
    // piece arrays [2 or 3][64][W+8] bf16 (they cover the [64][W+4] FP32 array)
    const int sps = a.split ? 2 : (W == 32 ? 0 : 3);
    const std::uint32_t lds =
        (std::uint32_t)((sps == 3 ? 3 : 2) * 64 * (W + 8) * sizeof(short) + kFusedCells * sizeof(float2));
    const dim3 grid((unsigned)a.ntiles), block(2 * W);
    if (sps == 2) {
        if (apply)
            LAUNCH(KID_FUSED_APPLY, t, (fused_tile<W, true, 2>), grid, block, lds, s, a);
        else
            LAUNCH(KID_FUSED_AGG, t, (fused_tile<W, false, 2>), grid, block, lds, s, a);
    } else if (sps == 0) {
        if constexpr (W == 32) {
            if (apply)
                LAUNCH(KID_FUSED_APPLY, t, (fused_tile<W, true, 0>), grid, block, lds, s, a);
            else
                LAUNCH(KID_FUSED_AGG, t, (fused_tile<W, false, 0>), grid, block, lds, s, a);
        }
    } else {
        if constexpr (W > 32) {
            if (apply)
                LAUNCH(KID_FUSED_APPLY, t, (fused_tile<W, true, 3>), grid, block, lds, s, a);
            else
                LAUNCH(KID_FUSED_AGG, t, (fused_tile<W, false, 3>), grid, block, lds, s, a);
        }
    }
}

void launch_fused_pass(const BatchFusedArgs &a, bool apply, hipStream_t s, KernelTimer *t) {
    if (a.ntiles <= 0) return;
    switch (class_width(a.N, a.L1)) {
        case 16:
        case 32: launch_fused_w<32>(a, apply, s, t); break;
        case 64: launch_fused_w<64>(a, apply, s, t); break;
        default: launch_fused_w<128>(a, apply, s, t); break;
    }
}

void launch_fused_scan(const BatchFusedScanArgs &a, hipStream_t s, KernelTimer *t) {
    if (a.nslabs <= 0) return;
    LAUNCH(KID_FUSED_SCAN, t, fused_scan, dim3((unsigned)a.nslabs), dim3(128), 0, s, a);
}

void launch_fused_iso(const BatchIsoArgs &a, hipStream_t s) {
    if (a.ntiles <= 0) return;
    hipLaunchKernelGGL(fused_iso, dim3((unsigned)a.ntiles), dim3(256), 0, s, a);
}

int persistent_gemm_blocks(int N, int L1, int kind, bool vec4, int ntiles) {
    const int w = std::max(32, class_width(N, L1));  // W = 16 classes run the 32-wide kernels
    // W = 256: the sources only (the persistent moments kernel, one 32-row
    // chain per wave there, measured slower than the tile-per-block one)
    if (!vec4 || ntiles <= 0 || w > 256 || (kind == 1 && w > 128)) return 0;
    const bool mom = kind == 1;
    size_t lds = (size_t)(w == 256 ? PUnit<256>::ROWS : TM) * (w + 4) * sizeof(float);
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipSuccess;
    if (kind == 2) {
        // split-BF16 source (the class tables are built at least 32 wide)
        lds = (size_t)2 * (w == 256 ? PUnit<256>::ROWS : TM) * (w + 4) * sizeof(short);
        e = w == 32    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (src_batch_sp<32, float>), 64, lds)
            : w == 64  ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (src_batch_sp<64, float>), 128, lds)
            : w == 128 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (src_batch_sp<128, float>), 256, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (src_batch_sp<256, float>), 512, lds);
    } else if (w == 32)
        e = mom ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mom_batch_p<32>, 64, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (src_batch_p<32, float>), 64, lds);
    else if (w == 64)
        e = mom ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mom_batch_p<64>, 128, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (src_batch_p<64, float>), 128, lds);
    else if (w == 128)
        e = mom ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mom_batch_p<128>, 256, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (src_batch_p<128, float>), 256, lds);
    else
        e = mom ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mom_batch_p<256>, 512, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (src_batch_p<256, float>), 512, lds);
    if (e != hipSuccess || per_cu <= 0 || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
        (void)hipGetLastError();
        return 0;
    }
    const int units = w == 256 ? 2 * ntiles : ntiles;
    return std::min(units, per_cu * cus);
}

template <int W>
static void launch_mom_w(const BatchMomArgs &a, hipStream_t s, KernelTimer *t) {
    const std::uint32_t lds = (std::uint32_t)(TM * (W + 4) * sizeof(float));
    if constexpr (W <= 256) {
        constexpr int WP = W < 32 ? 32 : W;  // as in launch_src_w
        if (a.pblocks > 0 && a.phi32 && a.dirmajor && a.meta) {
            const std::uint32_t ldsp = (std::uint32_t)(PUnit<WP>::ROWS * (WP + 4) * sizeof(float));
            LAUNCH(KID_MOM_BATCH, t, mom_batch_p<WP>, dim3((unsigned)a.pblocks), dim3(2 * WP), ldsp, s, a);
            return;
        }
    }
    if (a.phi32)
        LAUNCH(KID_MOM_BATCH, t, (mom_batch<W, float>), dim3((unsigned)a.ntiles), dim3(256), lds, s, a);
    else
        LAUNCH(KID_MOM_BATCH, t, (mom_batch<W, double>), dim3((unsigned)a.ntiles), dim3(256), lds, s, a);
}

void launch_mom_batch(const BatchMomArgs &a, hipStream_t s, KernelTimer *t) {
    if (a.ntiles <= 0) return;
    switch (class_width(a.N, a.L1)) {
        case 16: launch_mom_w<16>(a, s, t); break;
        case 32: launch_mom_w<32>(a, s, t); break;
        case 64: launch_mom_w<64>(a, s, t); break;
        case 128: launch_mom_w<128>(a, s, t); break;
        default: launch_mom_w<256>(a, s, t); break;
    }
}

__global__ void select_final(const GemmTile *tiles, const BatchSlab *slabs, int L1, const int *its,
                             const float *bufA, const float *bufB, double *out) {
    const GemmTile tl = tiles[blockIdx.x];
    const BatchSlab m = slabs[tl.slab];
    const int rows = min(TM, 2 * m.K - tl.row0);
    const float *src = (its[tl.slab] & 1) ? bufB : bufA;
    for (int idx = threadIdx.x; idx < rows * L1; idx += blockDim.x) {
        const size_t o = m.phi_off + (size_t)tl.row0 * L1 + idx;
        out[o] = (double)src[o];
    }
}

void launch_select_final(int ntiles, const GemmTile *tiles, const BatchSlab *slabs, int L1, const int *its,
                         const float *bufA, const float *bufB, double *out, hipStream_t s) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(select_final, dim3((unsigned)ntiles), dim3(256), 0, s, tiles, slabs, L1, its, bufA, bufB,
                       out);
}

__global__ void __launch_bounds__(256) to_f32(size_t n, const double *in, float *out) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) out[i] = (float)in[i];
}

void launch_to_f32(size_t n, const double *in, float *out, hipStream_t s) {
    if (n == 0) return;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(to_f32, dim3(grid), dim3(256), 0, s, n, in, out);
}

__global__ void iter_advance(int *iter) {
    if (threadIdx.x == 0) iter[0] += 1;
}

void launch_iter_advance(int *iter, hipStream_t s) { hipLaunchKernelGGL(iter_advance, dim3(1), dim3(64), 0, s, iter); }

}  // namespace snfpsa
