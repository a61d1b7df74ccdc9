// Adjoint source, per-cell gradient and summation kernels; the operator
// identities they rest on are stated in sn_adjoint.hpp.
#include "sn_adjoint.hpp"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace snfpsa {

#define LAUNCH(id, t, kernel, grid, block, shm, st, ...)                                       \
    do {                                                                                       \
        hipEvent_t ev0_ = nullptr, ev1_ = nullptr;                                             \
        if ((t) && (t)->events((id), &ev0_, &ev1_))                                            \
            hipExtLaunchKernelGGL(kernel, grid, block, shm, st, ev0_, ev1_, 0, __VA_ARGS__);   \
        else                                                                                   \
            hipLaunchKernelGGL(kernel, grid, block, shm, st, __VA_ARGS__);                     \
    } while (0)

// one thread per (cell, angle)
__global__ void __launch_bounds__(256) adjoint_source(int K, int N, const double *h, const double *w,
                                                      const double *c, double *q_y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)K * N) return;
    const int k = (int)(i / N), n = (int)(i % N);
    const double *ck = c + (size_t)k * 2 * N;
    const double iw = 1.0 / w[n];
    const double c0 = ck[N - 1 - n] * iw, c1 = ck[N + N - 1 - n] * iw;
    const double f = 2.0 / h[k];  // Mass^{-1} = (2/h) [[2,-1],[-1,2]]
    double *qk = q_y + (size_t)k * 2 * N;
    qk[n] = f * (2.0 * c0 - c1);
    qk[N + n] = f * (2.0 * c1 - c0);
}

void launch_adjoint_source(int K, int N, const double *h, const double *w, const double *c, double *q_y,
                           hipStream_t s, KernelTimer *t) {
    const long long n = (long long)K * N;
    if (n <= 0) return;
    LAUNCH(KID_ADJOINT, t, adjoint_source, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, K, N, h, w, c, q_y);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// one wavefront per cell, four cells per block
__global__ void __launch_bounds__(256) grad_cells(GradArgs a) {
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= a.K) return;
    const int N = a.N, L1 = a.L1;
    const double *ps = a.psi + (size_t)k * 2 * N, *ys = a.y + (size_t)k * 2 * N, *cs = a.c + (size_t)k * 2 * N;
    double gt = 0.0, jp = 0.0;
    for (int n = lane; n < N; n += 64) {
        const double p0 = ps[n], p1 = ps[N + n];
        const double y0 = ys[N - 1 - n], y1 = ys[N + N - 1 - n];
        gt += a.w[n] * (y0 * (2.0 * p0 + p1) + y1 * (p0 + 2.0 * p1));
        jp += cs[n] * p0 + cs[N + n] * p1;
    }
    gt = wave_sum(gt);
    jp = wave_sum(jp);
    const double m6 = a.h[k] / 6.0;
    if (lane == 0) {
        a.g_sigma_t[k] = -m6 * gt;
        a.jpart[k] = jp;
    }
    const double *f = a.phi + (size_t)k * 2 * L1, *fy = a.phi_y + (size_t)k * 2 * L1;
    for (int l = lane; l < L1; l += 64) {
        const double x0 = fy[l], x1 = fy[L1 + l], p0 = f[l], p1 = f[L1 + l];
        const double sgn = (l & 1) ? -1.0 : 1.0;
        a.g_sigma_s[(size_t)k * L1 + l] =
            sgn * 0.5 * (2 * l + 1) * m6 * (x0 * (2.0 * p0 + p1) + x1 * (p0 + 2.0 * p1));
    }
}

void launch_grad_cells(const GradArgs &a, hipStream_t s, KernelTimer *t) {
    if (a.K <= 0) return;
    LAUNCH(KID_ADJOINT, t, grad_cells, dim3((unsigned)((a.K + 3) / 4)), dim3(256), 0, s, a);
}

__global__ void __launch_bounds__(1024) sum_kernel(int n, const double *x, double *out) {
    __shared__ double red[16];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) v += x[i];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int i = 0; i < 16; ++i) r += red[i];
        *out = r;
    }
}

void launch_sum(int n, const double *x, double *out, hipStream_t s, KernelTimer *t) {
    LAUNCH(KID_ADJOINT, t, sum_kernel, dim3(1), dim3(1024), 0, s, n, x, out);
}

// one thread per (cell, node, angle) of one slab
__global__ void __launch_bounds__(256) exit_weights(int K, int N, const double *mu, const double *w, double *c) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)K * 2 * N) return;
    const int n = (int)(i % N);
    const long long kn = i / N;  // cell * 2 + node
    c[i] = (kn == 2LL * K - 1 && n >= N / 2) ? w[n] * mu[n] : 0.0;
}

void launch_exit_weights(int K, int N, const double *mu, const double *w, double *c, hipStream_t s,
                         KernelTimer *t) {
    const long long n = (long long)K * 2 * N;
    if (n <= 0) return;
    LAUNCH(KID_ADJOINT, t, exit_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, K, N, mu, w, c);
}

// one wavefront per slab, four slabs per block
template <typename T>
__global__ void __launch_bounds__(256) exit_current(int nslab, const long long *off, const double *wmu,
                                                    const T *psi_exit, double *J) {
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= nslab) return;
    double v = 0.0;
    for (long long i = off[b] + lane; i < off[b + 1]; i += 64) v += wmu[i] * (double)psi_exit[i];
    v = wave_sum(v);
    if (lane == 0) J[b] = v;
}

void launch_exit_current(int nslab, const long long *off, const double *wmu, const void *psi_exit,
                         bool exit_f32, double *J, hipStream_t s, KernelTimer *t) {
    if (nslab <= 0) return;
    const dim3 grid((unsigned)((nslab + 3) / 4));
    if (exit_f32)
        LAUNCH(KID_ADJOINT, t, exit_current<float>, grid, dim3(256), 0, s, nslab, off, wmu,
               (const float *)psi_exit, J);
    else
        LAUNCH(KID_ADJOINT, t, exit_current<double>, grid, dim3(256), 0, s, nslab, off, wmu,
               (const double *)psi_exit, J);
}

}  // namespace snfpsa
