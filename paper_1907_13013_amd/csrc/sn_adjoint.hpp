// Kernels of the adjoint solve and of the response gradient (FP64 handles).
//
// The transport operator of eq:treq discretised by LD x S_N with a
// symmetric quadrature satisfies A^T = X A X^{-1}, X = W R: W = diag(w_n)
// over angles and R the angle reflection n -> N-1-n (mu -> -mu).  So the
// adjoint lambda' of A^T lambda' = c is W R y with y the FORWARD solution of
// A y = R W^{-1} c (zero inflow), whose nodal source is q_y = Mass^{-1}
// R W^{-1} c per cell.  The response J = <c, psi> then has
//   dJ/dsigma_t(k)    = - sum_{nu,nu',n} Mass_k[nu][nu'] w_n y(k,nu,N-1-n) psi(k,nu',n)
//   dJ/dsigma_{s,l}(k) = (2l+1)/2 (-1)^l sum_{nu,nu'} Mass_k[nu][nu'] phi_y(k,nu,l) phi(k,nu',l)
// with Mass_k = (h_k/6) [[2,1],[1,2]] and phi_y the moments of y.
#pragma once

#include <hip/hip_runtime.h>

#include "sn_kernels.hpp"

namespace snfpsa {

// q_y[k][nu][n] = (Mass_k^{-1} c~)[nu], c~[nu] = c[k][nu][N-1-n] / w[n]
void launch_adjoint_source(int K, int N, const double *h, const double *w, const double *c, double *q_y,
                           hipStream_t s, KernelTimer *t);

// Per cell: g_sigma_t[k], g_sigma_s[k][l] (formulas above) and
// jpart[k] = sum_{nu,n} c psi; one wavefront per cell.
struct GradArgs {
    int K = 0, N = 0, L1 = 0;
    const double *h = nullptr, *w = nullptr;
    const double *psi = nullptr, *y = nullptr, *c = nullptr;     // [K][2][N]
    const double *phi = nullptr, *phi_y = nullptr;               // [K][2][L1]
    double *g_sigma_t = nullptr;                                 // [K]
    double *g_sigma_s = nullptr;                                 // [K][L1]
    double *jpart = nullptr;                                     // [K]
};
void launch_grad_cells(const GradArgs &a, hipStream_t s, KernelTimer *t);

// out = sum_{i < n} x[i] (one block, fixed summation order)
void launch_sum(int n, const double *x, double *out, hipStream_t s, KernelTimer *t);

// c[k][nu][n] = w_n mu_n at the right node (nu = 1) of the last cell for
// mu_n > 0, zero elsewhere: the response weights of the partial current
// leaving the slab through its right face (one slab, [K][2][N]).
void launch_exit_weights(int K, int N, const double *mu, const double *w, double *c, hipStream_t s,
                         KernelTimer *t);

// J[b] = sum_{i in [off[b], off[b+1])} wmu[i] * psi_exit[i] for every slab
// b < nslab (one wavefront per slab, fixed summation order); psi_exit is
// double (FP64 handles) or float (batched handles), accumulated in FP64.
void launch_exit_current(int nslab, const long long *off, const double *wmu, const void *psi_exit,
                         bool exit_f32, double *J, hipStream_t s, KernelTimer *t);

}  // namespace snfpsa
