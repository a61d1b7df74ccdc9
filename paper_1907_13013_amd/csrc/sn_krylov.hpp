// Vector kernels of the restarted GMRES outer solver (FP64, one slab's
// moment vectors of length n; the Krylov basis is stored row by row, row j
// at V + j * ld).
#pragma once

#include <hip/hip_runtime.h>

#include "sn_kernels.hpp"

namespace snfpsa {

// Longest GMRES restart cycle (Arnoldi steps).
constexpr int kGmresMaxRestart = 30;

// out = a - b
void launch_vec_sub(size_t n, const double *a, const double *b, double *out, hipStream_t s, KernelTimer *t);
// out = alpha x
void launch_vec_scale(size_t n, const double *x, double alpha, double *out, hipStream_t s, KernelTimer *t);
// Blocks of the absmax reduction (4096 elements each) and of the
// Gram-Schmidt kernels (256 elements each).
int krylov_dot_blocks(size_t n);
int krylov_gs_blocks(size_t n);
// out[j] = <V_j, w> for j < k <= kGmresMaxRestart + 1, in a fixed summation
// order (block partial sums, then one block per j over them); partial holds
// krylov_gs_blocks(n) * k doubles.
void launch_multi_dot(size_t n, int k, const double *V, size_t ld, const double *w, double *partial, double *out,
                      hipStream_t s, KernelTimer *t);
// w -= sum_{j<k} coef[j] V_j, then out[j] = <V_j, w> (one pass over V;
// the second Gram-Schmidt pass's coefficients)
void launch_axpy_dot(size_t n, int k, const double *V, size_t ld, const double *coef, double *w, double *partial,
                     double *out, hipStream_t s, KernelTimer *t);
// w -= sum_{j<k} coef[j] V_j, then out[0] = <w, w>
void launch_axpy_norm(size_t n, int k, const double *V, size_t ld, const double *coef, double *w, double *partial,
                      double *out, hipStream_t s, KernelTimer *t);
// w += sign * sum_{j<k} coef[j] V_j (coef on the device)
void launch_multi_axpy(size_t n, int k, const double *V, size_t ld, const double *coef, double sign, double *w,
                       hipStream_t s, KernelTimer *t);

// Device state of one GMRES restart cycle (at most kGmresMaxRestart
// Arnoldi steps): the Hessenberg matrix H [(m+1)][m] (row-major, stride m),
// the Givens rotations, the rotated right-hand side g, and the flags with
// which the cycle's queued steps gate themselves.
struct GmresState {
    double H[(kGmresMaxRestart + 1) * kGmresMaxRestart];
    double cs[kGmresMaxRestart], sn[kGmresMaxRestart], g[kGmresMaxRestart + 1];
    double res[kGmresMaxRestart];   // |g[j+1]| after step j
    double gate;                    // SkipTest value of the next step: the last residual, 0 once finished, NaN if not finite
    double inv_hn;                  // 1 / h[j+1][j] for the next basis vector, 0 once finished
    int jn;                         // columns of H in use
    int ran;                        // steps whose sweep ran (not skipped)
    int done, nonfinite;
};
// Arnoldi step j of a cycle of length m, one thread: unless the cycle has
// finished, H[:, j] = c1 + c2 (the two Gram-Schmidt passes' coefficients),
// h[j+1][j] = sqrt(c3), the previous rotations applied, the new rotation
// formed and g rotated; the cycle finishes when |g[j+1]| <= tol, when
// h[j+1][j] = 0, when the rotation's norm is 0 (the Krylov space is
// exhausted: column j is dropped) or when a value is not finite.
void launch_gmres_arnoldi(GmresState *st, int j, int m, const double *c1, const double *c2, const double *c3,
                          double tol, hipStream_t s, KernelTimer *t);
// out = (*alpha) x, nothing when *alpha == 0 (alpha on the device)
void launch_vec_scale_dev(size_t n, const double *x, const double *alpha, double *out, hipStream_t s,
                          KernelTimer *t);

// out[0] = max |x_i| (block partial maxima, then one thread over the blocks)
void launch_absmax(size_t n, const double *x, double *partial, double *out, hipStream_t s, KernelTimer *t);
// x += a + b
void launch_add2(size_t n, const double *a, const double *b, double *x, hipStream_t s, KernelTimer *t);
// out = (float) in
void launch_narrow(size_t n, const double *in, float *out, hipStream_t s, KernelTimer *t);

}  // namespace snfpsa
