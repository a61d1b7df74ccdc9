// HIP kernels (gfx950, wave64) of the slab S_N / FPSA library.
//
//   gemm_f64_mfma      scattering source / moments / FP correction maps as
//                      FP64 MFMA GEMMs (v_mfma_f64_16x16x4f64), LDS-staged
//   sweep_*            LD transport sweep (eq:trsi, L = mu d/dz + sigma_t) as
//                      an affine scan over cells, one lane per angle
//   absdiff_max        FP64 stopping test max|phi^{m+1} - phi^m| (eq:iterate)
//   fp_*               FP correction: chunked forward/backward interface
//                      recurrences of the factorised LD x S_N Fokker-Planck
//                      operator (eq:correct with F of eq:fpop)
#include "sn_kernels.hpp"

#include <hip/hip_runtime.h>

namespace snfpsa {

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// FP64 MFMA GEMM:  C = Cin + (A1 - A1sub) .* S  x B1  +  A2 x B2
// Row-major operands; S (optional) scales A1 column-wise per row group:
// A1[m][k] *= S[(m / s_div) * lds + k].  Tile 64 x 64 per 256-thread block,
// each wave owns 16 rows x 64 columns (four 16x16 accumulators).
// MFMA 16x16x4 f64 operand layout: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element r of lane l is D[l/16 + 4*r][l%16]
// (rows interleaved with stride 4, unlike the f32 16x16x4 variant).
// ---------------------------------------------------------------------------
constexpr int GT_M = 64, GT_N = 64, GT_K = 16;
constexpr int AS_LD = GT_K + 1, BS_LD = GT_N + 16;

__global__ void __launch_bounds__(256) gemm_f64_mfma(GemmArgs g) {
    __shared__ double As[GT_M * AS_LD];
    __shared__ double Bs[GT_K * BS_LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * GT_M, n0 = blockIdx.y * GT_N;
    d4 acc[4];
    for (int j = 0; j < 4; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};

    for (int seg = 0; seg < 2; ++seg) {
        const double *A = seg ? g.A2 : g.A1;
        if (!A) continue;
        const double *Asub = seg ? nullptr : g.A1sub;
        const double *S = seg ? nullptr : g.S;
        const double *B = seg ? g.B2 : g.B1;
        const int lda = seg ? g.lda2 : g.lda1;
        const int kt = seg ? g.k2 : g.k1;
        for (int k0 = 0; k0 < kt; k0 += GT_K) {
            __syncthreads();
            for (int idx = tid; idx < GT_M * GT_K; idx += 256) {
                const int r = idx / GT_K, kk = idx % GT_K;
                const int m = m0 + r, k = k0 + kk;
                double v = 0.0;
                if (m < g.rows && k < kt) {
                    v = A[(size_t)m * lda + k];
                    if (Asub) v -= Asub[(size_t)m * lda + k];
                    if (S) v *= S[(size_t)(m / g.s_div) * g.lds + k];
                }
                As[r * AS_LD + kk] = v;
            }
            for (int idx = tid; idx < GT_K * GT_N; idx += 256) {
                const int kk = idx / GT_N, c = idx % GT_N;
                const int k = k0 + kk, n = n0 + c;
                Bs[kk * BS_LD + c] = (k < kt && n < g.ncols) ? B[(size_t)k * g.ncols + n] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int kq = 0; kq < GT_K / 4; ++kq) {
                const double a = As[(wave * 16 + (lane & 15)) * AS_LD + kq * 4 + (lane >> 4)];
#pragma unroll
                for (int jt = 0; jt < 4; ++jt) {
                    const double b = Bs[(kq * 4 + (lane >> 4)) * BS_LD + jt * 16 + (lane & 15)];
                    acc[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[jt], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {
        const int col = n0 + jt * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = m0 + wave * 16 + (lane >> 4) + 4 * r;
            if (row < g.rows && col < g.ncols) {
                double v = acc[jt][r];
                if (g.Cin) v += g.Cin[(size_t)row * g.ldcin + col];
                g.C[(size_t)row * g.ldc + col] = v;
            }
        }
    }
}

#define TIMED(id, t, s, launch)         \
    do {                                \
        if (t) (t)->begin((id), (s));   \
        launch;                         \
        if (t) (t)->end((id), (s));     \
    } while (0)

const char *kernel_name(int id) {
    static const char *names[KID_COUNT] = {"gemm_f64_mfma",  "sweep_aggregate", "sweep_scan_tiles",
                                           "sweep_apply",    "absdiff_max",     "fp_forward_local",
                                           "fp_forward_fix", "fp_backward_local", "fp_backward_fix",
                                           "exit_flux"};
    return (id >= 0 && id < KID_COUNT) ? names[id] : "";
}

void launch_gemm(const GemmArgs &g, hipStream_t s, KernelTimer *t) {
    if (g.rows <= 0 || g.ncols <= 0) return;
    dim3 grid((g.rows + GT_M - 1) / GT_M, (g.ncols + GT_N - 1) / GT_N);
    TIMED(KID_GEMM, t, s, hipLaunchKernelGGL(gemm_f64_mfma, grid, dim3(256), 0, s, g));
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
// Three kernels: per tile of TC cells, per-(sub-chunk, angle) aggregates;
// a per-angle scan over tiles giving each tile's carry-in; and the apply
// pass that re-sweeps each sub-chunk from its carry-in.  Thread t of a
// 256-thread block serves angle t % N and sub-chunk t / N.
// ---------------------------------------------------------------------------
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

__global__ void __launch_bounds__(256) sweep_aggregate(SweepArgs s, bool adjoint) {
    __shared__ double shA[256], shB[256];
    const int N = s.N, S = s.S;
    const int t = threadIdx.x, n = t % N, sc = t / N;
    const int tile = blockIdx.x;
    const int c0 = tile * s.TC, c1 = min(s.K, c0 + s.TC);
    double A = 1.0, B = 0.0;
    if (sc < S) {
        const double mu = s.mu[n], inv = s.inv_absmu[n];
        const int dir = sweep_dir(mu, adjoint);
        const int j0 = c0 + sc * s.sub, j1 = min(c1, c0 + (sc + 1) * s.sub);
        const int in_node = dir > 0 ? 0 : 1;
        for (int i = 0; i < j1 - j0; ++i) {
            const int j = dir > 0 ? j0 + i : j1 - 1 - i;
            const double yin = s.q[((size_t)j * 2 + in_node) * N + n];
            const double yout = s.q[((size_t)j * 2 + (1 - in_node)) * N + n];
            const CellCoef c = cell_coef(inv, s.h[j], s.sigma_t[j], yin, yout, adjoint);
            B = c.a * B + c.b;
            A = c.a * A;
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

__global__ void sweep_scan_tiles(SweepArgs s, bool adjoint) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= s.N) return;
    const int N = s.N, NH = N / 2;
    const double mu = s.mu[n];
    const int dir = sweep_dir(mu, adjoint);
    double x = 0.0;
    if (!adjoint) {
        if (mu > 0.0 && s.psi_left) x = s.psi_left[n - NH];
        if (mu < 0.0 && s.psi_right) x = s.psi_right[n];
    }
    for (int i = 0; i < s.ntiles; ++i) {
        const int tile = dir > 0 ? i : s.ntiles - 1 - i;
        s.carry[(size_t)tile * N + n] = x;
        x = s.tileA[(size_t)tile * N + n] * x + s.tileB[(size_t)tile * N + n];
    }
    if (s.exit) s.exit[n] = x;
}

__global__ void __launch_bounds__(256) sweep_apply(SweepArgs s, bool adjoint) {
    const int N = s.N, S = s.S;
    const int t = threadIdx.x, n = t % N, sc = t / N;
    if (sc >= S) return;
    const int tile = blockIdx.x;
    const int c0 = tile * s.TC, c1 = min(s.K, c0 + s.TC);
    const double mu = s.mu[n], inv = s.inv_absmu[n];
    const int dir = sweep_dir(mu, adjoint);
    double x = s.carry[(size_t)tile * N + n];
    if (dir > 0) {
        for (int i = 0; i < sc; ++i)
            x = s.subA[((size_t)tile * S + i) * N + n] * x + s.subB[((size_t)tile * S + i) * N + n];
    } else {
        for (int i = S - 1; i > sc; --i)
            x = s.subA[((size_t)tile * S + i) * N + n] * x + s.subB[((size_t)tile * S + i) * N + n];
    }
    const int j0 = c0 + sc * s.sub, j1 = min(c1, c0 + (sc + 1) * s.sub);
    const int in_node = dir > 0 ? 0 : 1;
    for (int i = 0; i < j1 - j0; ++i) {
        const int j = dir > 0 ? j0 + i : j1 - 1 - i;
        const size_t iin = ((size_t)j * 2 + in_node) * N + n;
        const size_t iout = ((size_t)j * 2 + (1 - in_node)) * N + n;
        const double hj = s.h[j];
        const CellCoef c = cell_coef(inv, hj, s.sigma_t[j], s.q[iin], s.q[iout], adjoint);
        const double vout = c.a * x + c.b;
        const double vin = ((6.0 + 4.0 * c.tau) * (c.gin + x) - (6.0 + 2.0 * c.tau) * c.gout) * c.den_inv;
        if (adjoint) {
            // x = (h/(6|mu|)) [[2,1],[1,2]] zeta  (node order in/out is symmetric)
            const double f = hj * inv * (1.0 / 6.0);
            s.psi[iin] = f * (2.0 * vin + vout);
            s.psi[iout] = f * (vin + 2.0 * vout);
        } else {
            s.psi[iin] = vin;
            s.psi[iout] = vout;
        }
        x = vout;
    }
}

void launch_sweep(const SweepArgs &s, bool adjoint, hipStream_t st, KernelTimer *t) {
    if (s.K <= 0) return;
    TIMED(KID_SWEEP_AGGREGATE, t, st,
          hipLaunchKernelGGL(sweep_aggregate, dim3(s.ntiles), dim3(256), 0, st, s, adjoint));
    TIMED(KID_SWEEP_SCAN, t, st,
          hipLaunchKernelGGL(sweep_scan_tiles, dim3((s.N + 63) / 64), dim3(64), 0, st, s, adjoint));
    TIMED(KID_SWEEP_APPLY, t, st,
          hipLaunchKernelGGL(sweep_apply, dim3(s.ntiles), dim3(256), 0, st, s, adjoint));
}

// ---------------------------------------------------------------------------
// Stopping test: out = max(out, max_i |a_i - b_i|) as the IEEE bit pattern of
// a non-negative double (ordered like unsigned integers; NaN sorts above
// +Inf, so a NaN anywhere surfaces as NaN).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) absdiff_max(const double *a, const double *b, size_t n,
                                                   unsigned long long *out) {
    __shared__ unsigned long long red[4];
    unsigned long long m = 0ull;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const double d = fabs(a[i] - b[i]);
        const unsigned long long u = (unsigned long long)__double_as_longlong(d);
        m = u > m ? u : m;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 4; ++i) m = red[i] > m ? red[i] : m;
        red[0] = m;
        atomicMax(out, red[0]);
    }
}

__global__ void zero_u64(unsigned long long *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

void launch_absdiff_max(const double *a, const double *b, size_t n, unsigned long long *out,
                        hipStream_t s, KernelTimer *t) {
    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, s, out, 1);
    if (n == 0) return;
    int blocks = (int)std::min<size_t>((n + 255) / 256, 1024);
    TIMED(KID_ABSDIFF, t, s, hipLaunchKernelGGL(absdiff_max, dim3(blocks), dim3(256), 0, s, a, b, n, out));
}

// ---------------------------------------------------------------------------
// Fokker-Planck interface recurrences (see setup_math.hpp):
//   forward  p_{j+1} = G_j p_j + Hm_j s-_j + s+_j,          p_0 = 0
//   backward b_j = U_j b_{j+1} + Y_j p_j + X_j s-_j,          b_K = 0
//            a_j = rho_j b_j + p_j
// Cells are cut into chunks; a "local" pass runs each chunk from a zero
// carry and records its end value, and a "fix" pass folds the preceding
// chunks' end values through the precomputed chunk products to obtain the
// true carry-in, then re-runs the chunk and stores the results.  One
// 64-lane wave per chunk; lane r owns rows r and r + 64 of each NH x NH
// matvec, the vectors live in LDS.
// ---------------------------------------------------------------------------
constexpr int FP_MAX_NH = 128;

__device__ __forceinline__ double rowdot(const double *__restrict__ Mrow,
                                         const double *__restrict__ v, int NH) {
    double s0 = 0.0, s1 = 0.0;
    int c = 0;
    for (; c + 1 < NH; c += 2) {
        s0 = fma(Mrow[c], v[c], s0);
        s1 = fma(Mrow[c + 1], v[c + 1], s1);
    }
    if (c < NH) s0 = fma(Mrow[c], v[c], s0);
    return s0 + s1;
}

__global__ void __launch_bounds__(64) fp_forward(FPArgs f, bool fix) {
    __shared__ double pv[FP_MAX_NH], sm[FP_MAX_NH], tmp[FP_MAX_NH];
    const int NH = f.NH, N = 2 * NH, lane = threadIdx.x;
    const size_t M2 = (size_t)NH * NH;
    const int c = blockIdx.x;
    const int j0 = c * f.chunk, j1 = min(f.K, j0 + f.chunk);
    for (int r = lane; r < NH; r += 64) pv[r] = 0.0;
    __syncthreads();
    if (fix) {
        for (int cc = 0; cc < c; ++cc) {
            const double *Phi = f.chunk_fwd + (size_t)cc * M2;
            for (int r = lane; r < NH; r += 64)
                tmp[r] = rowdot(Phi + (size_t)r * NH, pv, NH) + f.e_fwd[(size_t)cc * NH + r];
            __syncthreads();
            for (int r = lane; r < NH; r += 64) pv[r] = tmp[r];
            __syncthreads();
        }
    }
    for (int j = j0; j < j1; ++j) {
        const double *cm = f.cellmats + (size_t)j * 6 * M2;
        const double *sj = f.s + (size_t)j * N;
        for (int r = lane; r < NH; r += 64) {
            sm[r] = sj[NH + r];
            if (fix) f.pvec[(size_t)j * NH + r] = pv[r];
        }
        __syncthreads();
        for (int r = lane; r < NH; r += 64)
            tmp[r] = rowdot(cm + (size_t)r * NH, pv, NH) + rowdot(cm + M2 + (size_t)r * NH, sm, NH) +
                     sj[r];
        __syncthreads();
        for (int r = lane; r < NH; r += 64) pv[r] = tmp[r];
        __syncthreads();
    }
    for (int r = lane; r < NH; r += 64) {
        if (!fix) f.e_fwd[(size_t)c * NH + r] = pv[r];
        else if (j1 == f.K) f.pvec[(size_t)f.K * NH + r] = pv[r];
    }
}

__global__ void __launch_bounds__(64) fp_backward(FPArgs f, bool fix) {
    __shared__ double bv[FP_MAX_NH], pj[FP_MAX_NH], sm[FP_MAX_NH], tmp[FP_MAX_NH];
    const int NH = f.NH, N = 2 * NH, lane = threadIdx.x;
    const size_t M2 = (size_t)NH * NH;
    const int c = blockIdx.x;
    const int j0 = c * f.chunk, j1 = min(f.K, j0 + f.chunk);
    for (int r = lane; r < NH; r += 64) bv[r] = 0.0;
    __syncthreads();
    if (fix) {
        for (int cc = f.nchunks - 1; cc > c; --cc) {
            const double *Phi = f.chunk_bwd + (size_t)cc * M2;
            for (int r = lane; r < NH; r += 64)
                tmp[r] = rowdot(Phi + (size_t)r * NH, bv, NH) + f.e_bwd[(size_t)cc * NH + r];
            __syncthreads();
            for (int r = lane; r < NH; r += 64) bv[r] = tmp[r];
            __syncthreads();
        }
    }
    for (int j = j1 - 1; j >= j0; --j) {
        const double *cm = f.cellmats + (size_t)j * 6 * M2;
        const double *sj = f.s + (size_t)j * N;
        for (int r = lane; r < NH; r += 64) {
            sm[r] = sj[NH + r];
            pj[r] = f.pvec[(size_t)j * NH + r];
            if (fix) f.inflow[(size_t)j * N + NH + r] = bv[r];  // b_{j+1} enters cell j
        }
        __syncthreads();
        for (int r = lane; r < NH; r += 64)
            tmp[r] = rowdot(cm + 2 * M2 + (size_t)r * NH, bv, NH) +
                     rowdot(cm + 3 * M2 + (size_t)r * NH, pj, NH) +
                     rowdot(cm + 4 * M2 + (size_t)r * NH, sm, NH);
        __syncthreads();
        for (int r = lane; r < NH; r += 64) bv[r] = tmp[r];
        __syncthreads();
        if (fix) {
            for (int r = lane; r < NH; r += 64) {
                const double a = rowdot(cm + 5 * M2 + (size_t)r * NH, bv, NH) + pj[r];
                f.inflow[(size_t)j * N + r] = a;              // a_j enters cell j
                if (j == 0 && f.b0) f.b0[r] = bv[r];          // b_0 leaves the slab at z0
            }
            __syncthreads();
        }
    }
    if (!fix)
        for (int r = lane; r < NH; r += 64) f.e_bwd[(size_t)c * NH + r] = bv[r];
}

void launch_fp_recurrences(const FPArgs &f, hipStream_t s, KernelTimer *t) {
    if (f.K <= 0 || f.NH <= 0) return;
    TIMED(KID_FP_FWD_LOCAL, t, s, hipLaunchKernelGGL(fp_forward, dim3(f.nchunks), dim3(64), 0, s, f, false));
    TIMED(KID_FP_FWD_FIX, t, s, hipLaunchKernelGGL(fp_forward, dim3(f.nchunks), dim3(64), 0, s, f, true));
    TIMED(KID_FP_BWD_LOCAL, t, s, hipLaunchKernelGGL(fp_backward, dim3(f.nchunks), dim3(64), 0, s, f, false));
    TIMED(KID_FP_BWD_FIX, t, s, hipLaunchKernelGGL(fp_backward, dim3(f.nchunks), dim3(64), 0, s, f, true));
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
    TIMED(KID_EXIT, t, s,
          hipLaunchKernelGGL(exit_flux, dim3((N + 63) / 64), dim3(64), 0, s, N, sweep_exit, b0, pK, out));
}

}  // namespace snfpsa
