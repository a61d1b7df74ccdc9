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

__global__ void __launch_bounds__(256) vec_scale_dev(size_t n, const double *x, const double *alpha, double *out) {
    const double a = *alpha;
    if (a == 0.0) return;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) out[i] = a * x[i];
}

void launch_vec_scale_dev(size_t n, const double *x, const double *alpha, double *out, hipStream_t s,
                          KernelTimer *t) {
    LAUNCH(KID_KRYLOV, t, vec_scale_dev, dim3(grid_for(n)), dim3(256), 0, s, n, x, alpha, out);
}

__global__ void gmres_arnoldi(GmresState *st, int j, int m, const double *c1, const double *c2, const double *c3,
                              double tol) {
    if (threadIdx.x != 0 || st->done) return;
    st->ran += 1;
    double *H = st->H;
    for (int i = 0; i <= j; ++i) H[i * m + j] = c1[i] + c2[i];
    const double hn = sqrt(c3[0]);
    H[(j + 1) * m + j] = hn;
    for (int i = 0; i < j; ++i) {
        const double a0 = H[i * m + j], a1 = H[(i + 1) * m + j];
        H[i * m + j] = st->cs[i] * a0 + st->sn[i] * a1;
        H[(i + 1) * m + j] = -st->sn[i] * a0 + st->cs[i] * a1;
    }
    const double a0 = H[j * m + j], a1 = H[(j + 1) * m + j];
    const double r = hypot(a0, a1);
    if (r == 0.0) {
        // exhausted Krylov space: the cycle keeps columns 0 .. j-1
        st->done = 1;
        st->gate = 0.0;
        st->inv_hn = 0.0;
        return;
    }
    st->cs[j] = r > 0.0 ? a0 / r : 1.0;
    st->sn[j] = r > 0.0 ? a1 / r : 0.0;
    H[j * m + j] = r;
    H[(j + 1) * m + j] = 0.0;
    st->g[j + 1] = -st->sn[j] * st->g[j];
    st->g[j] = st->cs[j] * st->g[j];
    const double res = fabs(st->g[j + 1]);
    st->res[j] = res;
    st->jn = j + 1;
    if (!isfinite(res) || !isfinite(hn)) {
        st->nonfinite = 1;
        st->done = 1;
        st->gate = __longlong_as_double(0x7ff8000000000000ll);
        st->inv_hn = 0.0;
        return;
    }
    if (res <= tol || hn == 0.0) {
        st->done = 1;
        st->gate = 0.0;
        st->inv_hn = 0.0;
        return;
    }
    st->gate = res;
    st->inv_hn = 1.0 / hn;
}

void launch_gmres_arnoldi(GmresState *st, int j, int m, const double *c1, const double *c2, const double *c3,
                          double tol, hipStream_t s, KernelTimer *t) {
    LAUNCH(KID_KRYLOV, t, gmres_arnoldi, dim3(1), dim3(64), 0, s, st, j, m, c1, c2, c3, tol);
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

// Gram-Schmidt kernels: one element per thread, 256 per block.  A block
// forms, for every basis row j < k, the sum of its elements' products in a
// fixed order (a wave's butterfly, then the four waves in order) into
// partial[b * k + j]; reduce_partials then sums the blocks' values of row j
// in a fixed order (block j, a strided pass and the same block sum).
int krylov_gs_blocks(size_t n) { return (int)std::max<size_t>(1, (n + 255) / 256); }

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// red[wave][j] -> partial[b * k + j] (called by all threads, after the
// waves have written red)
__device__ __forceinline__ void store_partials(const double (*red)[kGmresMaxRestart + 2], int k, double *partial) {
    __syncthreads();
    const int j = threadIdx.x;
    if (j < k) partial[(size_t)blockIdx.x * k + j] = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
}

// partial[b * k + j] = sum over block b's elements of V_j[i] w[i]
__global__ void __launch_bounds__(256) multi_dot_partial(size_t n, int k, const double *V, size_t ld, const double *w,
                                                         double *partial) {
    __shared__ double red[4][kGmresMaxRestart + 2];
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const bool ok = i < n;
    const size_t ic = ok ? i : n - 1;
    const double wi = ok ? w[ic] : 0.0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll 4
    for (int j = 0; j < k; ++j) {
        const double v = wave_sum(wi * V[(size_t)j * ld + ic]);
        if (lane == 0) red[wave][j] = v;
    }
    store_partials(red, k, partial);
}

// w -= sum_j coef[j] V_j, then (dots) partial[b * k + j] = the block's part
// of V_j . w, or (!dots) partial[b] = the block's part of w . w
__global__ void __launch_bounds__(256) axpy_then_dot(size_t n, int k, const double *V, size_t ld,
                                                     const double *coef, double *w, bool dots, double *partial) {
    __shared__ double red[4][kGmresMaxRestart + 2];
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const bool ok = i < n;
    const size_t ic = ok ? i : n - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v[kGmresMaxRestart + 1];
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kGmresMaxRestart + 1; ++j)
        if (j < k) {
            v[j] = V[(size_t)j * ld + ic];
            s += coef[j] * v[j];
        }
    const double wn = ok ? w[ic] - s : 0.0;
    if (ok) w[i] = wn;
    if (dots) {
#pragma unroll
        for (int j = 0; j < kGmresMaxRestart + 1; ++j)
            if (j < k) {
                const double d = wave_sum(v[j] * wn);
                if (lane == 0) red[wave][j] = d;
            }
        store_partials(red, k, partial);
    } else {
        const double d = wave_sum(wn * wn);
        if (lane == 0) red[wave][0] = d;
        store_partials(red, 1, partial);
    }
}

__global__ void __launch_bounds__(256) reduce_partials(int nb, int k, const double *partial, double *out) {
    __shared__ double red[4];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += partial[(size_t)b * k + j];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[j] = s;
}

void launch_multi_dot(size_t n, int k, const double *V, size_t ld, const double *w, double *partial, double *out,
                      hipStream_t s, KernelTimer *t) {
    const int nb = krylov_gs_blocks(n);
    LAUNCH(KID_KRYLOV, t, multi_dot_partial, dim3((unsigned)nb), dim3(256), 0, s, n, k, V, ld, w, partial);
    LAUNCH(KID_KRYLOV, t, reduce_partials, dim3((unsigned)k), dim3(256), 0, s, nb, k, partial, out);
}

void launch_axpy_dot(size_t n, int k, const double *V, size_t ld, const double *coef, double *w, double *partial,
                     double *out, hipStream_t s, KernelTimer *t) {
    const int nb = krylov_gs_blocks(n);
    LAUNCH(KID_KRYLOV, t, axpy_then_dot, dim3((unsigned)nb), dim3(256), 0, s, n, k, V, ld, coef, w, true, partial);
    LAUNCH(KID_KRYLOV, t, reduce_partials, dim3((unsigned)k), dim3(256), 0, s, nb, k, partial, out);
}

void launch_axpy_norm(size_t n, int k, const double *V, size_t ld, const double *coef, double *w, double *partial,
                      double *out, hipStream_t s, KernelTimer *t) {
    const int nb = krylov_gs_blocks(n);
    LAUNCH(KID_KRYLOV, t, axpy_then_dot, dim3((unsigned)nb), dim3(256), 0, s, n, k, V, ld, coef, w, false, partial);
    LAUNCH(KID_KRYLOV, t, reduce_partials, dim3(1u), dim3(256), 0, s, nb, 1, partial, out);
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
