// Vector kernels of the GMRES outer solver; see sn_krylov.hpp.
#include "sn_krylov.hpp"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

namespace snfpsa {

#define LAUNCH(id, t, kernel, grid, block, shm, st, ...)                                       \
    do {                                                                                       \
        hipEvent_t ev0_ = nullptr, ev1_ = nullptr;                                             \
        if ((t) && (t)->events((id), &ev0_, &ev1_))                                            \
            hipExtLaunchKernelGGL(kernel, grid, block, shm, st, ev0_, ev1_, 0, __VA_ARGS__);   \
        else                                                                                   \
            hipLaunchKernelGGL(kernel, grid, block, shm, st, __VA_ARGS__);                     \
    } while (0)

static unsigned grid_for(size_t n) { return (unsigned)std::min<size_t>((n + 255) / 256, 2048); }

__global__ void __launch_bounds__(256) vec_sub(size_t n, const double *a, const double *b, double *out) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) out[i] = a[i] - b[i];
}

void launch_vec_sub(size_t n, const double *a, const double *b, double *out, hipStream_t s, KernelTimer *t) {
    LAUNCH(KID_KRYLOV, t, vec_sub, dim3(grid_for(n)), dim3(256), 0, s, n, a, b, out);
}

__global__ void __launch_bounds__(256) vec_scale(size_t n, const double *x, double alpha, double *out) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) out[i] = alpha * x[i];
}

void launch_vec_scale(size_t n, const double *x, double alpha, double *out, hipStream_t s, KernelTimer *t) {
    LAUNCH(KID_KRYLOV, t, vec_scale, dim3(grid_for(n)), dim3(256), 0, s, n, x, alpha, out);
}

constexpr int kDotChunk = 4096;  // elements per block of multi_dot

int krylov_dot_blocks(size_t n) { return (int)std::max<size_t>(1, (n + kDotChunk - 1) / kDotChunk); }

__device__ __forceinline__ double block_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// block b: partial[b * k + j] = sum over its chunk of V_j . w
__global__ void __launch_bounds__(256) multi_dot_partial(size_t n, int k, const double *V, size_t ld, const double *w,
                                                         double *partial) {
    __shared__ double red[4];
    const size_t i0 = (size_t)blockIdx.x * kDotChunk, i1 = min(n, i0 + kDotChunk);
    for (int j = 0; j < k; ++j) {
        const double *v = V + (size_t)j * ld;
        double acc = 0.0;
        for (size_t i = i0 + threadIdx.x; i < i1; i += 256) acc += v[i] * w[i];
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * k + j] = s;
    }
}

__global__ void reduce_partials(int nb, int k, const double *partial, double *out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[(size_t)b * k + j];
    out[j] = s;
}

void launch_multi_dot(size_t n, int k, const double *V, size_t ld, const double *w, double *partial, double *out,
                      hipStream_t s, KernelTimer *t) {
    const int nb = krylov_dot_blocks(n);
    LAUNCH(KID_KRYLOV, t, multi_dot_partial, dim3((unsigned)nb), dim3(256), 0, s, n, k, V, ld, w, partial);
    LAUNCH(KID_KRYLOV, t, reduce_partials, dim3((unsigned)((k + 63) / 64)), dim3(64), 0, s, nb, k, partial, out);
}

__global__ void __launch_bounds__(256) multi_axpy(size_t n, int k, const double *V, size_t ld, const double *coef,
                                                  double sign, double *w) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s += coef[j] * V[(size_t)j * ld + i];
        w[i] += sign * s;
    }
}

void launch_multi_axpy(size_t n, int k, const double *V, size_t ld, const double *coef, double sign, double *w,
                       hipStream_t s, KernelTimer *t) {
    LAUNCH(KID_KRYLOV, t, multi_axpy, dim3(grid_for(n)), dim3(256), 0, s, n, k, V, ld, coef, sign, w);
}

__global__ void __launch_bounds__(256) absmax_partial(size_t n, const double *x, double *partial) {
    __shared__ double red[4];
    const size_t i0 = (size_t)blockIdx.x * kDotChunk, i1 = min(n, i0 + kDotChunk);
    double m = 0.0;
    for (size_t i = i0 + threadIdx.x; i < i1; i += 256) m = fmax(m, fabs(x[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ void absmax_final(int nb, const double *partial, double *out) {
    if (threadIdx.x != 0) return;
    double m = 0.0;
    for (int b = 0; b < nb; ++b) m = fmax(m, partial[b]);
    *out = m;
}

void launch_absmax(size_t n, const double *x, double *partial, double *out, hipStream_t s, KernelTimer *t) {
    const int nb = krylov_dot_blocks(n);
    LAUNCH(KID_KRYLOV, t, absmax_partial, dim3((unsigned)nb), dim3(256), 0, s, n, x, partial);
    LAUNCH(KID_KRYLOV, t, absmax_final, dim3(1), dim3(64), 0, s, nb, partial, out);
}

__global__ void __launch_bounds__(256) add2(size_t n, const double *a, const double *b, double *x) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) x[i] += a[i] + b[i];
}

void launch_add2(size_t n, const double *a, const double *b, double *x, hipStream_t s, KernelTimer *t) {
    LAUNCH(KID_KRYLOV, t, add2, dim3(grid_for(n)), dim3(256), 0, s, n, a, b, x);
}

__global__ void __launch_bounds__(256) narrow(size_t n, const double *in, float *out) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) out[i] = (float)in[i];
}

void launch_narrow(size_t n, const double *in, float *out, hipStream_t s, KernelTimer *t) {
    LAUNCH(KID_KRYLOV, t, narrow, dim3(grid_for(n)), dim3(256), 0, s, n, in, out);
}

}  // namespace snfpsa
