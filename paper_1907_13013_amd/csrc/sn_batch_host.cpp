// Host side of the batched FP32 / split-BF16 path.
#include "sn_batch_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <stdexcept>
#include <utility>

#include "setup_math.hpp"

namespace snfpsa {

namespace {

struct HipFail : std::runtime_error {
    explicit HipFail(const std::string &w) : std::runtime_error(w) {}
};

#define BCHK(x)                                                                                    \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) throw HipFail(std::string(#x) + ": " + hipGetErrorString(e_));       \
    } while (0)

template <typename T>
T *balloc(BatchData &B, size_t n) {
    void *p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) throw std::bad_alloc();
    B.allocs.push_back(p);
    return static_cast<T *>(p);
}

// bf16 bits of x, round to nearest even (finite x)
unsigned short bf16_bits(float x) {
    unsigned int u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

float bf16_value(unsigned short h) {
    const unsigned int u = (unsigned int)h << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

// Split-BF16 tables of Mt [L1][N] in the fragment order of the split source
// GEMM: entry (kb, n, j) packs Mt[16 kb + 4 j + i][n], i = 0..3, zero-padded
// to W rows.
void split_tables(const std::vector<float> &Mt, int N, int L1, int W, std::vector<short4_t> &hi,
                  std::vector<short4_t> &lo) {
    const int KB = W / 16;
    hi.assign((size_t)KB * N * 4, short4_t{0, 0, 0, 0});
    lo.assign(hi.size(), short4_t{0, 0, 0, 0});
    for (int kb = 0; kb < KB; ++kb)
        for (int n = 0; n < N; ++n)
            for (int j = 0; j < 4; ++j) {
                const size_t o = ((size_t)kb * N + n) * 4 + j;
                for (int i = 0; i < 4; ++i) {
                    const int k = 16 * kb + 4 * j + i;
                    const float x = k < L1 ? Mt[(size_t)k * N + n] : 0.0f;
                    const unsigned short h = bf16_bits(x);
                    hi[o][i] = (short)h;
                    lo[o][i] = (short)bf16_bits(x - bf16_value(h));
                }
            }
}

// Three-piece BF16 tables of M [nk][ncols] in the fragment order of
// split_tables: M = p0 + p1 + p2 with p0 = bf16(x), p1 = bf16(x - p0),
// p2 = bf16(x - p0 - p1) (each difference exact in FP32).
void split3_tables(const std::vector<float> &M, int ncols, int nk, int W, std::vector<short4_t> (&p)[3]) {
    const int KB = W / 16;
    for (auto &v : p) v.assign((size_t)KB * ncols * 4, short4_t{0, 0, 0, 0});
    for (int kb = 0; kb < KB; ++kb)
        for (int c = 0; c < ncols; ++c)
            for (int j = 0; j < 4; ++j) {
                const size_t o = ((size_t)kb * ncols + c) * 4 + j;
                for (int i = 0; i < 4; ++i) {
                    const int k = 16 * kb + 4 * j + i;
                    float x = k < nk ? M[(size_t)k * ncols + c] : 0.0f;
                    for (int q = 0; q < 3; ++q) {
                        const unsigned short h = bf16_bits(x);
                        p[q][o][i] = (short)h;
                        x -= bf16_value(h);
                    }
                }
            }
}

template <typename T>
T *bupload(BatchData &B, const std::vector<T> &v, hipStream_t st) {
    T *p = balloc<T>(B, v.size());
    if (!v.empty()) BCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return p;
}

}  // namespace

BatchData::~BatchData() {
    for (GraphEntry &g : graphs) (void)hipGraphExecDestroy(g.exec);
    if (gev) (void)hipEventDestroy(gev);
    if (gstream) (void)hipStreamDestroy(gstream);
    for (void *p : allocs) (void)hipFree(p);
}

static BatchSweepArgs sweep_args(BatchData &B, const float *q, float *psi, bool problem_bc, float *exit);

// The long-slab passes of the direction-major sweep with the segment list
// of candidate c (see BatchData::seg_choice).
static BatchLongArgs long_args(BatchData &B, int c, const float *q, float *psi, bool problem_bc, float *exit,
                               SlabGate gate) {
    BatchLongArgs l;
    l.nsegs = B.cand_nsegs[c]; l.nchains = B.nlong_chains;
    l.segs = B.cand_segs[c]; l.chain_first = B.cand_chain_first[c]; l.slabs = B.slabs;
    l.q = q; l.psi = psi; l.cellpar = B.cellpar; l.mu = B.mu; l.inv_absmu = B.inv_absmu;
    l.psi_left = problem_bc ? B.psi_left : nullptr;
    l.psi_right = problem_bc ? B.psi_right : nullptr;
    l.exit = exit;
    l.segAB = B.long_ab; l.carry = B.long_carry; l.gate = gate;
    return l;
}

void batch_set_seg_choice(BatchData &B, int c) {
    B.seg_choice = c;
    B.nlong_segs = B.cand_nsegs[c];
    B.long_segs = B.cand_segs[c];
    B.long_chain_first = B.cand_chain_first[c];
}

// Autotuner of the solve's sweep decomposition: the direction-major work
// list is built four ways (long/short group pairing on or off, N <= 16
// slabs segmented or not) and each is timed on this handle's own batch
// (one warm-up and three timed sweeps of a zero source, HIP events); the
// fastest is kept.  The choice depends on the mix of N and K, the number of
// work items against the wavefronts the part holds at once, and the tail.
static void tune_solve_sweep(BatchData &B, hipStream_t st) {
    BCHK(hipMemsetAsync(B.q, 0, (size_t)B.psi_len * sizeof(float), st));
    hipEvent_t e0, e1;
    BCHK(hipEventCreate(&e0));
    BCHK(hipEventCreate(&e1));
    int best = 0;
    for (int c = 0; c < 4; ++c) {
        BatchSweepArgs a = sweep_args(B, B.q, B.psi, false, nullptr);
        a.dirmajor = true;
        a.nitems = B.cand_n[c];
        a.items = B.cand_items[c];
        launch_sweep_batch(a, st, nullptr);
        BCHK(hipEventRecord(e0, st));
        for (int r = 0; r < 3; ++r) launch_sweep_batch(a, st, nullptr);
        BCHK(hipEventRecord(e1, st));
        BCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        BCHK(hipEventElapsedTime(&ms, e0, e1));
        B.tune_ms[c] = ms / 3.0;
        if (B.tune_ms[c] < B.tune_ms[best]) best = c;
    }
    B.tune_choice = best;
    B.nitems_dm = B.cand_n[best];
    B.items_dm = B.cand_items[best];
    // the long slabs' scan: each candidate segment length timed the same way
    if (B.nlong_chains > 0) {
        int bs = 0;
        for (int c = 0; c < 3; ++c) {
            const BatchLongArgs l = long_args(B, c, B.q, B.psi, false, nullptr, SlabGate());
            launch_sweep_long(l, st, nullptr);
            BCHK(hipEventRecord(e0, st));
            for (int r = 0; r < 3; ++r) launch_sweep_long(l, st, nullptr);
            BCHK(hipEventRecord(e1, st));
            BCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            BCHK(hipEventElapsedTime(&ms, e0, e1));
            B.seg_ms[c] = ms / 3.0;
            if (B.seg_ms[c] < B.seg_ms[bs]) bs = c;
        }
        batch_set_seg_choice(B, bs);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

sn_status batch_setup(const sn_problem_desc *d, hipStream_t st, BatchData **out, std::string &msg) {
    BatchData *B = new (std::nothrow) BatchData();
    if (!B) {
        msg = "host allocation failed";
        return SN_E_NOMEM;
    }
    try {
        const int ns = d->num_slabs;
        B->nslab = ns;
        B->split_bf16 = d->precision == SN_BF16X3;
        // quadrature per distinct N, classes per distinct (N, L+1)
        std::map<int, int> quad_of;
        std::vector<double> mu_all, inv_all;
        std::map<std::pair<int, int>, int> cls_of;
        std::vector<std::vector<float>> Mt_h, Vt_h;
        int64_t cells = 0, psi_off = 0, phi_off = 0, ss_off = 0, ab_off = 0;
        int half = 0, exit_off = 0;
        B->host_slabs.resize(ns);
        for (int b = 0; b < ns; ++b) {
            const int K = d->K[b], N = d->N[b], L1 = d->L[b] + 1;
            auto qi = quad_of.find(N);
            std::vector<double> mu, w;
            gauss_legendre(N, mu, w);
            if (qi == quad_of.end()) {
                qi = quad_of.emplace(N, (int)mu_all.size()).first;
                for (int n = 0; n < N; ++n) {
                    mu_all.push_back(mu[n]);
                    inv_all.push_back(1.0 / std::fabs(mu[n]));
                }
            }
            auto ci = cls_of.find({N, L1});
            if (ci == cls_of.end()) {
                ci = cls_of.emplace(std::make_pair(N, L1), (int)Mt_h.size()).first;
                std::vector<double> P = legendre_table(N, L1 - 1, mu);
                std::vector<float> Mt((size_t)L1 * N), Vt((size_t)N * L1);
                for (int l = 0; l < L1; ++l)
                    for (int n = 0; n < N; ++n) {
                        Mt[(size_t)l * N + n] = (float)(0.5 * (2 * l + 1) * P[(size_t)l * N + n]);
                        Vt[(size_t)n * L1 + l] = (float)(w[n] * P[(size_t)l * N + n]);
                    }
                Mt_h.push_back(std::move(Mt));
                Vt_h.push_back(std::move(Vt));
            }
            BatchSlab &m = B->host_slabs[b];
            m.K = K; m.N = N; m.L1 = L1; m.cls = ci->second;
            m.cell_off = cells; m.psi_off = psi_off; m.phi_off = phi_off; m.ss_off = ss_off;
            m.quad_off = qi->second; m.bc_off = half; m.exit_off = exit_off;
            m.ab_off = (int)std::min<int64_t>(ab_off, INT32_MAX);
            ab_off += 2 * (int64_t)((K + kFusedCells - 1) / kFusedCells) * N;
            cells += K;
            psi_off += (int64_t)K * 2 * N;
            phi_off += (int64_t)K * 2 * L1;
            ss_off += (int64_t)K * L1;
            half += N / 2;
            exit_off += N;
        }
        B->psi_len = psi_off;
        B->phi_len = phi_off;
        B->exit_len = exit_off;
        // classes: tables and row tiles (64 node rows, never straddling a slab)
        std::vector<std::vector<GemmTile>> tiles(Mt_h.size());
        for (int b = 0; b < ns; ++b) {
            const BatchSlab &m = B->host_slabs[b];
            for (int r0 = 0; r0 < 2 * m.K; r0 += 64) tiles[m.cls].push_back(GemmTile{b, r0});
        }
        B->classes.resize(Mt_h.size());
        for (auto &kv : cls_of) {
            BatchClass &c = B->classes[kv.second];
            c.N = kv.first.first;
            c.L1 = kv.first.second;
            c.Mt = bupload(*B, Mt_h[kv.second], st);
            if (B->split_bf16) {
                std::vector<short4_t> hi, lo;
                // at least 32 wide: the persistent split kernel runs W = 16
                // classes 32 wide (the tile-per-block kernel reads the first
                // class_width / 16 blocks, laid out the same)
                split_tables(Mt_h[kv.second], c.N, c.L1, std::max(32, class_width(c.N, c.L1)), hi, lo);
                c.Mt_hi = bupload(*B, hi, st);
                c.Mt_lo = bupload(*B, lo, st);
            }
            c.Vt = bupload(*B, Vt_h[kv.second], st);
            c.tiles = bupload(*B, tiles[kv.second], st);
            c.ntiles = (int)tiles[kv.second].size();
            // the persistent GEMMs read rows as 16-byte vectors: every slab
            // of the class must start its phi, sigma_s and psi rows on a
            // 16-byte boundary
            bool vec4 = c.N % 4 == 0 && c.L1 % 4 == 0;
            for (const BatchSlab &m : B->host_slabs)
                if (m.cls == kv.second && (m.phi_off % 4 || m.ss_off % 4 || m.psi_off % 4)) vec4 = false;
            // offsets in 16-byte vectors must fit 32 bits
            for (const BatchSlab &m : B->host_slabs)
                if (m.cls == kv.second && (m.psi_off / 4 > 0xffffffffLL || m.phi_off / 4 > 0xffffffffLL))
                    vec4 = false;
            if (vec4) {
                std::vector<TileMeta> meta;
                meta.reserve(tiles[kv.second].size());
                for (const GemmTile &tl : tiles[kv.second]) {
                    const BatchSlab &m = B->host_slabs[tl.slab];
                    // cells of one region share their sigma_s row: a tile
                    // inside one region reads a single row
                    const int c0 = tl.row0 / 2, c1 = std::min(m.K, c0 + 32);
                    const double *r0 = d->sigma_s + m.ss_off + (int64_t)c0 * m.L1;
                    bool same = true;
                    for (int c = c0 + 1; c < c1 && same; ++c)
                        same = std::memcmp(r0, d->sigma_s + m.ss_off + (int64_t)c * m.L1, sizeof(double) * m.L1) == 0;
                    const int64_t ss4 = same ? (m.ss_off + (int64_t)c0 * m.L1) / 4 : m.ss_off / 4;
                    meta.push_back(TileMeta{(unsigned)(m.psi_off / 4), (unsigned)(m.phi_off / 4), (unsigned)ss4, m.K,
                                            tl.slab, tl.row0, same ? 0 : m.L1 / 4, 0});
                }
                c.meta = bupload(*B, meta, st);
                if (fused_class_ok(c.N, c.L1) && cells < INT32_MAX && ab_off < INT32_MAX) {
                    std::vector<FusedTile> ft;
                    ft.reserve(meta.size());
                    for (size_t i = 0; i < meta.size(); ++i) {
                        const TileMeta &tm = meta[i];
                        const BatchSlab &m = B->host_slabs[tm.slab];
                        ft.push_back(FusedTile{tm.phi4, tm.psi4, tm.ss4, tm.ss_step, tm.K, tm.slab, tm.row0,
                                               (int)(m.cell_off + tm.row0 / 2), m.quad_off,
                                               m.ab_off + 2 * (tm.row0 / (2 * kFusedCells)) * m.N, 0, 0});
                    }
                    c.ftiles = bupload(*B, ft, st);
                    const int w = std::max(32, class_width(c.N, c.L1));
                    std::vector<short4_t> pm[3], pv[3];
                    split3_tables(Mt_h[kv.second], c.N, c.L1, w, pm);
                    split3_tables(Vt_h[kv.second], c.L1, c.N, w, pv);
                    for (int q = 0; q < 3; ++q) {
                        c.Mt3[q] = bupload(*B, pm[q], st);
                        c.Vt3[q] = bupload(*B, pv[q], st);
                    }
                }
            }
            c.pblocks_src = persistent_gemm_blocks(c.N, c.L1, 0, vec4, c.ntiles);
            c.pblocks_mom = persistent_gemm_blocks(c.N, c.L1, 1, vec4, c.ntiles);
            c.pblocks_split = B->split_bf16 ? persistent_gemm_blocks(c.N, c.L1, 2, vec4, c.ntiles) : 0;
        }
        // the fused iteration: every class eligible, no long slab
        B->fused_ok = true;
        for (const BatchClass &c : B->classes) B->fused_ok = B->fused_ok && c.ftiles;
        for (const BatchSlab &m : B->host_slabs) B->fused_ok = B->fused_ok && m.K <= kFusedMaxCells;
        if (B->fused_ok) {
            B->ab_len = ab_off;
            B->alpha = balloc<float>(*B, (size_t)ab_off);
            B->beta = balloc<float>(*B, (size_t)ab_off);
            B->carry = balloc<float>(*B, (size_t)ab_off);
            B->e0 = balloc<float>(*B, 2 * (size_t)cells);
            B->use_fused = true;
        }
        // sweep work items: slabs grouped by N, longest first; N < 64 packs
        // 64/N slabs of neighbouring lengths into one wavefront
        std::vector<int> order(ns);
        for (int b = 0; b < ns; ++b) order[b] = b;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            const BatchSlab &a = B->host_slabs[x], &c = B->host_slabs[y];
            if (a.N != c.N) return a.N < c.N;
            return a.K > c.K;
        });
        // segmented: slabs of N <= 16 are swept one per wavefront in 64/N
        // cell segments (direction-major kernel only)
        // dm: the solve's direction-major list (long slabs excluded);
        // pair: pair long with short groups; seg_small: N <= 16 slabs swept
        // in cell segments (direction-major list only)
        auto build_items = [&](bool dm, bool pair, bool seg_small) {
            const bool segmented = dm;
            std::vector<SweepItem> items;
            for (size_t i = 0; i < order.size();) {
                const int N = B->host_slabs[order[i]].N;
                size_t j = i;
                while (j < order.size() && B->host_slabs[order[j]].N == N) ++j;
                const bool seg = dm && seg_small && N <= 16;
                // long slabs (sorted first within their N) go to the segmented
                // long-slab sweep of the direction-major path
                if (segmented)
                    while (i < j && B->host_slabs[order[i]].K >= kLongCells) ++i;
                if (i == j) continue;
                // groups of this N, longest first (slabs are sorted by K)
                std::vector<SweepItem> grp;
                if (N >= 64 || seg) {
                    for (size_t k = i; k < j; ++k)
                        grp.push_back(SweepItem{(int)k, 1, 0, B->host_slabs[order[k]].K, 0, 0, 0, seg ? 64 / N : 0});
                } else {
                    const int P = 64 / N;
                    for (size_t k = i; k < j; k += P) {
                        const int cnt = (int)std::min<size_t>(P, j - k);
                        grp.push_back(SweepItem{(int)k, cnt, 0, B->host_slabs[order[k]].K, 0, 0, 0, 0});
                    }
                }
                // pair the g-th longest with the g-th shortest group
                const size_t ng = grp.size();
                for (size_t g = 0; g < (ng + 1) / 2; ++g) {
                    if (!pair) break;
                    SweepItem it = grp[g];
                    const size_t o = ng - 1 - g;
                    if (o != g) {
                        it.first2 = grp[o].first;
                        it.count2 = grp[o].count;
                        it.kmax2 = grp[o].kmax;
                    }
                    for (int a0 = 0; a0 < (seg ? 1 : N); a0 += 64) {
                        it.angle0 = a0;
                        items.push_back(it);
                    }
                }
                if (!pair)
                    for (SweepItem it : grp)
                        for (int a0 = 0; a0 < (seg ? 1 : N); a0 += 64) {
                            it.angle0 = a0;
                            items.push_back(it);
                        }
                i = j;
            }
            // longest work first (segmented groups count their shorter chains)
            auto work = [](const SweepItem &x) {
                const int k = x.kmax + x.kmax2;
                return x.pad > 0 ? 2 * k / x.pad : k;
            };
            std::stable_sort(items.begin(), items.end(),
                             [&](const SweepItem &x, const SweepItem &y) { return work(x) > work(y); });
            return items;
        };
        {
            // long slabs: chains of (slab, 64-angle block) cut into segments
            // of about len cells, one list per candidate length
            size_t max_segs = 0;
            for (int c = 0; c < 3; ++c) {
                const int len = kSegCandidates[c];
                std::vector<LongSeg> segs;
                std::vector<int> chain_first;
                for (int b = 0; b < ns; ++b) {
                    const BatchSlab &m = B->host_slabs[b];
                    if (m.K < kLongCells) continue;
                    const int nseg = (m.K + len - 1) / len;
                    for (int a0 = 0; a0 < m.N; a0 += 64) {
                        const int first = (int)segs.size();
                        chain_first.push_back(first);
                        for (int sgi = 0; sgi < nseg; ++sgi) {
                            const int c0 = (int)((long long)m.K * sgi / nseg);
                            const int c1 = (int)((long long)m.K * (sgi + 1) / nseg);
                            segs.push_back(LongSeg{b, a0, c0, c1, first, nseg, sgi, 0});
                        }
                    }
                }
                B->nlong_chains = (int)chain_first.size();
                B->cand_nsegs[c] = (int)segs.size();
                max_segs = std::max(max_segs, segs.size());
                if (!segs.empty()) {
                    B->cand_segs[c] = bupload(*B, segs, st);
                    B->cand_chain_first[c] = bupload(*B, chain_first, st);
                }
            }
            if (max_segs) {
                B->long_ab = balloc<float2>(*B, max_segs * 64);
                B->long_carry = balloc<float>(*B, max_segs * 64);
            }
            B->seg_choice = 1;
            B->nlong_segs = B->cand_nsegs[1];
            B->long_segs = B->cand_segs[1];
            B->long_chain_first = B->cand_chain_first[1];
            std::vector<SweepItem> items = build_items(false, true, false);
            B->nitems = (int)items.size();
            B->items = bupload(*B, items, st);
            for (int c = 0; c < 4; ++c) {
                const std::vector<SweepItem> l = build_items(true, (c & 1) == 0, (c & 2) == 0);
                B->cand_items[c] = bupload(*B, l, st);
                B->cand_n[c] = (int)l.size();
            }
            B->nitems_dm = B->cand_n[0];
            B->items_dm = B->cand_items[0];
        }
        B->slab_list = bupload(*B, order, st);
        B->slabs = bupload(*B, B->host_slabs, st);
        B->mu = bupload(*B, mu_all, st);
        B->inv_absmu = bupload(*B, inv_all, st);
        {
            std::vector<float> sinv(mu_all.size());
            for (size_t i = 0; i < mu_all.size(); ++i) sinv[i] = (float)(mu_all[i] > 0.0 ? inv_all[i] : -inv_all[i]);
            B->sinv = bupload(*B, sinv, st);
        }
        // cell parameters and cross sections (FP32)
        {
            std::vector<float2> cp((size_t)cells);
            for (int64_t c = 0; c < cells; ++c) cp[c] = float2{(float)d->h[c], (float)(d->sigma_t[c] * d->h[c])};
            B->cellpar = bupload(*B, cp, st);
            std::vector<float> ss((size_t)ss_off);
            for (int64_t i = 0; i < ss_off; ++i) ss[i] = (float)d->sigma_s[i];
            B->sigma_s = bupload(*B, ss, st);
        }
        if (d->psi_left) B->psi_left = bupload(*B, std::vector<double>(d->psi_left, d->psi_left + half), st);
        if (d->psi_right) B->psi_right = bupload(*B, std::vector<double>(d->psi_right, d->psi_right + half), st);
        B->q = balloc<float>(*B, (size_t)psi_off);
        B->psi = balloc<float>(*B, (size_t)psi_off);
        B->phiA = balloc<float>(*B, (size_t)phi_off);
        B->phiB = balloc<float>(*B, (size_t)phi_off);
        B->its = balloc<int>(*B, (size_t)ns);
        B->iter_dev = balloc<int>(*B, 1);
        BCHK(hipStreamSynchronize(st));
        tune_solve_sweep(*B, st);
    } catch (const std::bad_alloc &) {
        delete B;
        msg = "device or host allocation failed in the batch setup";
        return SN_E_NOMEM;
    } catch (const HipFail &e) {
        delete B;
        msg = std::string("HIP error in the batch setup: ") + e.what();
        return SN_E_HIP;
    }
    *out = B;
    return SN_OK;
}

static BatchSweepArgs sweep_args(BatchData &B, const float *q, float *psi, bool problem_bc, float *exit) {
    BatchSweepArgs a;
    a.nitems = B.nitems;
    a.items = B.items;  // the direction-major list is set by the solve
    a.slab_list = B.slab_list;
    a.slabs = B.slabs;
    a.q = q;
    a.psi = psi;
    a.cellpar = B.cellpar;
    a.mu = B.mu;
    a.inv_absmu = B.inv_absmu;
    a.psi_left = problem_bc ? B.psi_left : nullptr;
    a.psi_right = problem_bc ? B.psi_right : nullptr;
    a.exit = exit;
    return a;
}

// phi (FP64) or phi32 (FP32, with its reference ref32) receives the moments
static void moments(BatchData &B, const float *psi, double *phi, const double *ref, float *phi32, const float *ref32,
                    unsigned long long *slot, SlabGate gate, bool dirmajor, hipStream_t st, KernelTimer *t,
                    float *buf0 = nullptr, float *buf1 = nullptr) {
    for (const BatchClass &c : B.classes) {
        BatchMomArgs g;
        g.ntiles = c.ntiles; g.N = c.N; g.L1 = c.L1;
        g.tiles = c.tiles; g.slabs = B.slabs;
        g.psi = psi; g.Vt = c.Vt; g.phi = phi; g.ref = ref; g.slot = slot; g.gate = gate;
        g.phi32 = phi32; g.ref32 = ref32;
        g.buf0 = buf0; g.buf1 = buf1;
        g.dirmajor = dirmajor;
        g.pblocks = B.persistent_gemms ? c.pblocks_mom : 0;
        g.meta = c.meta;
        launch_mom_batch(g, st, t);
    }
}

// moments in FP64 (phi) or FP32 (phi32, phi null)
static void source(BatchData &B, const double *phi, const float *phi32, const float *q_ext, float *q, SlabGate gate,
                   bool dirmajor, hipStream_t st, KernelTimer *t, const float *buf0 = nullptr,
                   const float *buf1 = nullptr) {
    for (const BatchClass &c : B.classes) {
        BatchSrcArgs g;
        g.ntiles = c.ntiles; g.N = c.N; g.L1 = c.L1;
        g.tiles = c.tiles; g.slabs = B.slabs;
        g.phi = phi; g.phi32 = phi32; g.sigma_s = B.sigma_s; g.Mt = c.Mt; g.q_ext = q_ext; g.q = q; g.gate = gate;
        g.Mt_hi = c.Mt_hi; g.Mt_lo = c.Mt_lo;
        g.buf0 = buf0; g.buf1 = buf1;
        g.dirmajor = dirmajor;
        g.pblocks = B.persistent_gemms ? c.pblocks_src : 0;
        g.pblocks_split = B.persistent_gemms ? c.pblocks_split : 0;
        g.meta = c.meta;
        launch_src_batch(g, B.split_bf16, st, t);
    }
}

// the fused passes of one class; cur / nxt / slot as in the unfused
// iteration (all null while capturing: read from gate.iter then)
static BatchFusedArgs fused_args(BatchData &B, const BatchClass &c, const float *cur, float *nxt,
                                 unsigned long long *slot, const float *q_ext, const SlabGate &gate, bool rel,
                                 const float *buf0, const float *buf1) {
    BatchFusedArgs g;
    g.ntiles = c.ntiles; g.N = c.N; g.L1 = c.L1;
    g.tiles = c.ftiles;
    g.phi32 = rel ? nullptr : cur;
    g.out32 = rel ? nullptr : nxt;
    g.buf0 = buf0; g.buf1 = buf1;
    g.sigma_s = B.sigma_s; g.Mt = c.Mt; g.Vt = c.Vt;
    g.split = B.split_bf16;
    for (int q = 0; q < 3; ++q) {
        g.Mt3[q] = c.Mt3[q];
        g.Vt3[q] = c.Vt3[q];
    }
    g.q_ext = q_ext;
    g.e0 = q_ext ? B.e0 : nullptr;
    g.cellpar = B.cellpar; g.sinv = B.sinv;
    g.alpha = B.alpha; g.beta = B.beta; g.carry = B.carry;
    g.slot = rel ? nullptr : slot;
    g.gate = gate;
    return g;
}

void batch_sweep(BatchData &B, const float *q, float *psi, double *phi, bool problem_bc, float *exit,
                 hipStream_t st, KernelTimer *t) {
    float *out = psi ? psi : B.psi;
    launch_sweep_batch(sweep_args(B, q, out, problem_bc, exit), st, t);
    if (phi) moments(B, out, phi, nullptr, nullptr, nullptr, nullptr, SlabGate(), false, st, t);
}

void batch_scatter(BatchData &B, const double *phi, const float *q_ext, float *q, hipStream_t st, KernelTimer *t) {
    source(B, phi, nullptr, q_ext, q, SlabGate(), false, st, t);
}

sn_status batch_solve_si(BatchData &B, double tol, int32_t max_iter, const float *q_ext, double *phi,
                         float *psi_exit, int32_t *iters, double *resid_hist, unsigned long long *hist,
                         unsigned long long *hist_host, hipStream_t st, KernelTimer *t, std::string &msg,
                         bool problem_bc) {
    const int ns = B.nslab;
    const size_t nphi = (size_t)B.phi_len;
    // the iterates are kept in FP32 (half the GEMM traffic of FP64); the
    // stopping test compares them in FP64, and the final iterate is widened
    // back into phi
    float *buf[2] = {B.phiA, B.phiB};
    try {
        launch_to_f32(nphi, phi, buf[0], st);
        // (the fused passes read q_ext in 16-byte vectors)
        const bool fused = B.use_fused && reinterpret_cast<uintptr_t>(q_ext) % 16 == 0;

        if (fused && q_ext)
            for (const BatchClass &c : B.classes) {
                BatchIsoArgs ia;
                ia.ntiles = c.ntiles; ia.N = c.N; ia.tiles = c.ftiles; ia.q_ext = q_ext; ia.e0 = B.e0;
                launch_fused_iso(ia, st);
            }
        std::vector<int> its(ns, 0);
        std::vector<char> bad(ns, 0);
        int remaining = ns, launched = 0, batch = 2;
        auto passes = [&](double v) { return v <= tol || !std::isfinite(v); };
        // run stream: the caller's, or the graph stream while replaying
        hipStream_t rs = st;
        // the kernels of iteration m (gate/slot/buffers from m), or of the
        // current iteration read from iter_dev (graph capture, m = 0)
        auto iteration = [&](int m) {
            const bool rel = m == 0;
            const float *cur = rel ? buf[0] : buf[(m - 1) & 1];
            float *nxt = rel ? buf[0] : buf[m & 1];
            SlabGate gate;
            gate.tol = tol;
            if (rel) {
                gate.iter = B.iter_dev;
                gate.hist = hist;
                gate.ns = ns;
            } else {
                gate.prev = m > 1 ? hist + hist_row(m - 1) * ns : nullptr;
            }
            KernelTimer *tt = rel ? nullptr : t;
            if (fused) {
                unsigned long long *slot = rel ? nullptr : hist + hist_row(m) * ns;
                auto passes = [&](bool apply) {
                    for (const BatchClass &c : B.classes)
                        launch_fused_pass(fused_args(B, c, cur, nxt, slot, q_ext, gate, rel, buf[0], buf[1]), apply,
                                          rs, tt);
                };
                passes(false);
                BatchFusedScanArgs sa;
                sa.nslabs = ns; sa.slabs = B.slabs; sa.mu = B.mu;
                sa.psi_left = problem_bc ? B.psi_left : nullptr;
                sa.psi_right = problem_bc ? B.psi_right : nullptr;
                sa.exit = psi_exit;
                sa.alpha = B.alpha; sa.beta = B.beta; sa.carry = B.carry;
                sa.gate = gate;
                launch_fused_scan(sa, rs, tt);
                passes(true);
                if (rel) launch_iter_advance(B.iter_dev, rs);
                return;
            }
            // the iteration's q / psi live in the direction-major layout
            source(B, nullptr, cur, q_ext, B.q, gate, true, rs, tt, rel ? buf[0] : nullptr, rel ? buf[1] : nullptr);
            BatchSweepArgs a = sweep_args(B, B.q, B.psi, problem_bc, psi_exit);
            a.gate = gate;
            a.dirmajor = true;
            a.nitems = B.nitems_dm;
            a.items = B.items_dm;
            launch_sweep_batch(a, rs, tt);
            if (B.nlong_segs) launch_sweep_long(long_args(B, B.seg_choice, B.q, B.psi, problem_bc, psi_exit, gate), rs, tt);
            moments(B, B.psi, nullptr, nullptr, nxt, cur, rel ? nullptr : hist + hist_row(m) * ns, gate, true, rs,
                    tt, rel ? buf[0] : nullptr, rel ? buf[1] : nullptr);
            if (rel) launch_iter_advance(B.iter_dev, rs);
        };
        // graph of one iteration, captured when first needed (kernel timing
        // off) on the library's own stream, and replayed once per iteration
        bool graph = B.use_graphs && t == nullptr;
        hipGraphExec_t exec = nullptr;
        if (graph) {
            if (!B.gstream) {
                BCHK(hipStreamCreateWithFlags(&B.gstream, hipStreamNonBlocking));
                BCHK(hipEventCreateWithFlags(&B.gev, hipEventDisableTiming));
            }
            BCHK(hipEventRecord(B.gev, st));
            BCHK(hipStreamWaitEvent(B.gstream, B.gev, 0));
            rs = B.gstream;
            const void *key[6] = {q_ext, psi_exit, hist, B.items_dm, B.long_segs, fused ? B.alpha : nullptr};
            for (size_t e = 0; e < B.graphs.size(); ++e) {
                const BatchData::GraphEntry &g = B.graphs[e];
                if (g.tol == tol && g.bc == problem_bc && std::equal(key, key + 6, g.key)) {
                    exec = g.exec;
                    std::rotate(B.graphs.begin() + e, B.graphs.begin() + e + 1, B.graphs.end());
                    break;
                }
            }
            if (!exec) {
                hipGraph_t gr = nullptr;
                BCHK(hipStreamBeginCapture(rs, hipStreamCaptureModeThreadLocal));
                iteration(0);
                BCHK(hipStreamEndCapture(rs, &gr));
                const hipError_t ei = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                BCHK(ei);
                if (B.graphs.size() == BatchData::kGraphCache) {
                    (void)hipGraphExecDestroy(B.graphs.front().exec);
                    B.graphs.erase(B.graphs.begin());
                }
                BatchData::GraphEntry g;
                std::copy(key, key + 6, g.key);
                g.tol = tol;
                g.bc = problem_bc;
                g.exec = exec;
                B.graphs.push_back(g);
            }
            static const int one = 1;
            BCHK(hipMemcpyAsync(B.iter_dev, &one, sizeof(int), hipMemcpyHostToDevice, rs));
        }
        // ring rows of iterations m0 + 1 .. m0 + nb as at most two contiguous
        // row ranges (first row, count)
        auto ring_ranges = [&](int m0, int nb, auto &&fn) {
            const int r0 = (int)hist_row(m0 + 1);
            const int c0 = std::min(nb, kHistRing - r0);
            fn(r0, c0);
            if (nb > c0) fn(0, nb - c0);
        };
        while (launched < max_iter && remaining > 0) {
            const int nb = std::min(batch, max_iter - launched);
            ring_ranges(launched, nb, [&](int r, int c) {
                BCHK(hipMemsetAsync(hist + (size_t)r * ns, 0, (size_t)c * ns * sizeof(unsigned long long), rs));
            });
            for (int i = 0; i < nb; ++i) {
                if (graph) {
                    BCHK(hipGraphLaunch(exec, rs));
                    continue;
                }
                iteration(launched + i + 1);
            }
            ring_ranges(launched, nb, [&](int r, int c) {
                BCHK(hipMemcpyAsync(hist_host + (size_t)r * ns, hist + (size_t)r * ns,
                                    (size_t)c * ns * sizeof(unsigned long long), hipMemcpyDeviceToHost, rs));
            });
            BCHK(hipStreamSynchronize(rs));
            for (int b = 0; b < ns; ++b) {
                if (its[b]) continue;
                for (int i = 0; i < nb; ++i) {
                    double v;
                    std::memcpy(&v, &hist_host[hist_row(launched + i + 1) * ns + b], sizeof(double));
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
            BCHK(hipEventRecord(B.gev, rs));
            BCHK(hipStreamWaitEvent(st, B.gev, 0));
        }
        sn_status result = SN_OK;
        for (int b = 0; b < ns; ++b) {
            if (!its[b]) {
                its[b] = max_iter;
                result = SN_NOT_CONVERGED;
            }
            iters[b] = its[b];
        }
        BCHK(hipMemcpyAsync(B.its, its.data(), ns * sizeof(int), hipMemcpyHostToDevice, st));
        for (const BatchClass &c : B.classes)
            launch_select_final(c.ntiles, c.tiles, B.slabs, c.L1, B.its, buf[0], buf[1], phi, st);
        BCHK(hipGetLastError());
        BCHK(hipStreamSynchronize(st));
        for (int b = 0; b < ns; ++b)
            if (bad[b]) {
                msg = "non-finite stopping-test value in slab " + std::to_string(b);
                return SN_E_NONFINITE;
            }
        return result;
    } catch (const HipFail &e) {
        // leave the graph stream usable after a failure inside a capture
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (B.gstream && hipStreamIsCapturing(B.gstream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
            hipGraph_t gr = nullptr;
            (void)hipStreamEndCapture(B.gstream, &gr);
            if (gr) (void)hipGraphDestroy(gr);
        }
        (void)hipGetLastError();
        msg = std::string("HIP error in the batched solve: ") + e.what();
        return SN_E_HIP;
    }
}

}  // namespace snfpsa
