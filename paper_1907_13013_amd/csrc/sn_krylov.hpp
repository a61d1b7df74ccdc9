// Vector kernels of the restarted GMRES outer solver (FP64, one slab's
// moment vectors of length n; the Krylov basis is stored row by row, row j
// at V + j * ld).
#pragma once

#include <hip/hip_runtime.h>

#include "sn_kernels.hpp"

namespace snfpsa {

// out = a - b
void launch_vec_sub(size_t n, const double *a, const double *b, double *out, hipStream_t s, KernelTimer *t);
// out = alpha x
void launch_vec_scale(size_t n, const double *x, double alpha, double *out, hipStream_t s, KernelTimer *t);
// out[j] = <V_j, w> for j < k, in a fixed summation order (block partial
// sums, then one thread per j over the blocks); partial holds
// krylov_dot_blocks(n) * k doubles.
int krylov_dot_blocks(size_t n);
void launch_multi_dot(size_t n, int k, const double *V, size_t ld, const double *w, double *partial, double *out,
                      hipStream_t s, KernelTimer *t);
// w += sign * sum_{j<k} coef[j] V_j (coef on the device)
void launch_multi_axpy(size_t n, int k, const double *V, size_t ld, const double *coef, double sign, double *w,
                       hipStream_t s, KernelTimer *t);

// out[0] = max |x_i| (block partial maxima, then one thread over the blocks)
void launch_absmax(size_t n, const double *x, double *partial, double *out, hipStream_t s, KernelTimer *t);
// x += a + b
void launch_add2(size_t n, const double *a, const double *b, double *x, hipStream_t s, KernelTimer *t);
// out = (float) in
void launch_narrow(size_t n, const double *in, float *out, hipStream_t s, KernelTimer *t);

}  // namespace snfpsa
