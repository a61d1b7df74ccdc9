/*
 * snfpsa.h -- C ABI of the MI355X (gfx950) slab S_N / Fokker-Planck synthetic
 * acceleration library.
 *
 * Method: Patel, Warsa, Prinja, "Acceleration of the S_N equations with
 * highly anisotropic scattering using the Fokker-Planck equation".
 *   - problem statement: Sec. 2, eq:trans, eq:trans-equation-bc, eq:treq;
 *   - source iteration: Sec. 2.1, eq:trsi;
 *   - FPSA predict / correct / stopping test: Sec. 2.1, eq:predict,
 *     eq:correct, eq:iterate, with the Fokker-Planck operator eq:fpop;
 *   - angular Laplacians: Sec. 2.2, WFD eq:fp-wdd, eq:sph-weights, eq:w_wfd;
 *     MPD eq:fp-mpd.
 * The spatial scheme is linear discontinuous (LD) Galerkin (Sec. 2.2 names
 * it without equations): nodal, upwind faces, consistent mass
 * (h/6)[[2,1],[1,2]]; the Fokker-Planck correction uses the same LD scheme
 * with removal sigma_a I - (sigma_tr/2) A, A the WFD or MPD matrix, and zero
 * inflow on both faces.  The S_N quadrature is Gauss-Legendre, mu ascending,
 * weights summing to 2.
 *
 * Conventions
 *   Status: every call returns sn_status.  Negative = error, outputs
 *     undefined, message via sn_last_error() (thread-local).  No C++
 *     exception crosses this boundary.
 *   Ownership: the caller owns every pointer it passes.  The handle owns the
 *     quadrature, tables, cross sections, Fokker-Planck factors and its
 *     workspace; sn_destroy frees them.  No caller pointer is kept past the
 *     call (or, for asynchronous calls, past stream-ordered completion).
 *   Streams: `stream` is a hipStream_t (NULL = default stream).  sn_sweep,
 *     sn_scatter_source, fpsa_correct and sn_sweep_adjoint are asynchronous
 *     on `stream`; sn_setup and sn_solve synchronise.  One handle may be
 *     used by one stream at a time (it owns one workspace).
 *   Device arrays: contiguous, resident on the handle's device.  phi is
 *     always double.  q, psi, q_ext and psi_exit are double for SN_F64
 *     handles and float for SN_F32 / SN_BF16X3 handles (hence void * in the
 *     signatures).  Slabs are concatenated in descriptor order:
 *       psi, q : [sum_b K_b * 2 * N_b]  laid out [cell][node][angle]
 *                (node 0 = left LD node, 1 = right; angle fastest, mu
 *                ascending)
 *       phi    : [sum_b K_b * 2 * (L_b+1)] laid out [cell][node][l]
 *   Limits: N even, 2 <= N <= 256; 0 <= L <= N-1.
 */
#ifndef SNFPSA_H
#define SNFPSA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sn_handle_s *sn_handle;

typedef enum {
    SN_OK = 0,
    SN_NOT_CONVERGED = 1, /* iteration limit hit; outputs hold the last iterate */
    SN_E_INVALID = -1,    /* bad argument / shape / cross sections          */
    SN_E_NOMEM = -2,      /* host or device allocation failed                */
    SN_E_HIP = -3,        /* HIP runtime error                               */
    SN_E_NONFINITE = -4,  /* NaN/Inf in an input or in the iteration         */
    SN_E_STATE = -5       /* handle misuse (NULL handle, wrong device)       */
} sn_status;

/* Precision of a handle.
 *   SN_F64     everything in FP64 (sweeps, scattering GEMMs, FP correction).
 *   SN_F32     FP32 sweeps and q / psi storage; scattering source and moments
 *              on FP32 MFMA with FP32 accumulation; the quadrature / Legendre
 *              tables built in FP64 and rounded once.  phi passed in and out
 *              of every call is FP64; inside sn_solve the iterates are kept
 *              in FP32 and the stopping test is evaluated in FP64.  All slabs
 *              run batched (one launch per phase for the whole handle).
 *              Source iteration only.
 *   SN_BF16X3  as SN_F32 with the scattering source as split-BF16 products
 *              (hi*hi + hi*lo + lo*hi on BF16 MFMA, FP32 accumulation).      */
typedef enum { SN_F64 = 0, SN_F32 = 1, SN_BF16X3 = 2 } sn_precision;
/* SN_FP_NONE: no Fokker-Planck factorisation (source iteration only); used
 * for large batches whose factors would not fit. */
typedef enum { SN_FP_WFD = 0, SN_FP_MPD = 1, SN_FP_NONE = 2 } sn_fp_scheme;
/* Coefficients of the Fokker-Planck operator F_h behind FPSA.
 *   SN_FP_CELL  each cell's own sigma_a and sigma_tr (eq:fpop as stated).
 *   SN_FP_MEAN  per slab, the width-weighted means of sigma_a and sigma_tr
 *               over its cells, rounded to two significant digits; slabs
 *               with equal K, N, L, cell widths and rounded means share one
 *               factorisation (distinct ones are built on host threads).
 *               F only preconditions the iteration: for any nonsingular F
 *               the fixed point of eq:predict + eq:correct is the transport
 *               solution, and the residual F acts on keeps each cell's own
 *               sigma_s.  For slabs heterogeneous from cell to cell (not
 *               region by region, where a mean F can make FPSA diverge),
 *               whose per-cell factors would not fit in memory. */
typedef enum { SN_FP_CELL = 0, SN_FP_MEAN = 1 } sn_fp_coefficients;
/* Outer solvers.  SN_SI: source iteration (eq:trsi).  SN_FPSA: eq:predict +
 * eq:correct.  SN_FPSA_GMRES: restarted GMRES(30) on the moment form
 * (I - K) phi = b of the same discrete problem (K = one sweep of the
 * scattering source, b = one sweep of q_ext and the inflows), left-
 * preconditioned by the FPSA correction I + D F_h^{-1} S (the paper's
 * FPSA-preconditioned GMRES, Sec. 4).  SN_GMRES: the same without the
 * preconditioner. */
typedef enum { SN_SI = 0, SN_FPSA = 1, SN_FPSA_GMRES = 2, SN_GMRES = 3 } sn_method;
enum { SN_BC_PROBLEM = 0, SN_BC_ZERO = 1 };

/* Problem description; every pointer is HOST memory, FP64, read during
 * sn_setup only.
 *   num_slabs           number of independent slabs (>= 1)
 *   K[b], N[b], L[b]    cells, angles (even), scattering order of slab b
 *   h, sigma_t          [sum K]   cell widths and total cross sections (> 0)
 *   sigma_s             [sum_b K_b (L_b+1)] Legendre moments sigma_{s,l} of
 *                       each cell, normalised as in eq:treq (the scattering
 *                       source is sum_l (2l+1)/2 sigma_{s,l} P_l(mu) phi_l);
 *                       sigma_a = sigma_t - sigma_{s,0} >= 0 required
 *   psi_left            [sum N_b/2] inflow at z0 for the positive cosines
 *   psi_right           [sum N_b/2] inflow at z1 for the negative cosines
 *                       (both in ascending-mu order; NULL = vacuum)
 *   fp_scheme           SN_FP_WFD or SN_FP_MPD angular Laplacian, or
 *                       SN_FP_NONE (no FPSA; implied for SN_F32 / SN_BF16X3)
 *   precision           SN_F64, SN_F32 or SN_BF16X3
 *   fp_coefficients     SN_FP_CELL or SN_FP_MEAN (zero = SN_FP_CELL)        */
typedef struct {
    int32_t num_slabs;
    const int32_t *K;
    const int32_t *N;
    const int32_t *L;
    const double *h;
    const double *sigma_t;
    const double *sigma_s;
    const double *psi_left;
    const double *psi_right;
    int32_t fp_scheme;
    int32_t precision;
    int32_t fp_coefficients;
} sn_problem_desc;

/* Builds the quadrature and Legendre tables (Sec. 2.2), copies the cross
 * sections to the device and, for SN_F64 handles with a Fokker-Planck
 * scheme, factors the LD x S_N Fokker-Planck operator of every slab (eq:fpop
 * with eq:fp-mpd-oper / eq:wd-eq-oper) once, in FP64.  The factorisation is
 * the setup the paper excludes from its timings.
 * Errors: SN_E_INVALID (shapes, N odd or > 256, L >= N, h <= 0,
 * sigma_t <= 0, sigma_a < 0, sigma_tr < 0), SN_E_NONFINITE, SN_E_NOMEM,
 * SN_E_HIP.  Synchronises `stream`. */
sn_status sn_setup(const sn_problem_desc *desc, void *stream, sn_handle *out);

/* Frees everything the handle owns (after synchronising its device). */
sn_status sn_destroy(sn_handle h);

/* Message of the last negative status on this thread ("" if none). */
const char *sn_last_error(void);

/* psi = L_h^{-1} q (eq:trsi with L = mu d/dz + sigma_t): one LD transport
 * sweep of every angle of every slab.  bc_mode SN_BC_PROBLEM uses the
 * descriptor's inflows, SN_BC_ZERO vacuum.  psi (nullable) receives the
 * nodal angular flux, phi (nullable) its moments phi_l = sum_n w_n P_l(mu_n)
 * psi_n for l <= L (eq:phi-mom).  Asynchronous. */
sn_status sn_sweep(sn_handle h, const void *q, void *psi, double *phi,
                   int32_t bc_mode, void *stream);

/* q_out = sum_l (2l+1)/2 sigma_{s,l} P_l(mu_n) phi_l + q_ext at every cell
 * and LD node (the scattering source of eq:treq); q_ext nullable.
 * Asynchronous. */
sn_status sn_scatter_source(sn_handle h, const double *phi, const void *q_ext,
                            void *q_out, void *stream);

/* One FPSA correction (eq:correct) in moment form:
 *   phi_new = phi_half + D F_h^{-1} S (phi_half - phi_old)
 * where S is the scattering source above, F_h the LD x S_N Fokker-Planck
 * operator with zero inflow, D the discrete-to-moment map for l <= L.
 * phi_new may not alias phi_half or phi_old.  SN_F64 handles with a
 * Fokker-Planck scheme only (else SN_E_STATE).  Asynchronous. */
sn_status fpsa_correct(sn_handle h, const double *phi_half, const double *phi_old,
                       double *phi_new, void *stream);

/* fpsa_correct for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same correction, the same kernels and the same result as
 * fpsa_correct, with the Fokker-Planck work vectors of each slab (its
 * source, both interface vectors, the chains' local values, the chunk end
 * values and carry partial sums: about (2 K N + 2 (K + 1) N + small) doubles
 * per slab) taken from a fixed scratch array of 64 MiB per device
 * (resident from the library's load until the process ends, its address
 * resolved once per device by sn_setup) instead of the handle's workspace.
 * The call allocates nothing and records no per-kernel timing events.
 * The caller passes phi_half, phi_old and phi_new as for fpsa_correct.
 * Slabs run one after the other on `stream`, reusing the scratch; no part of
 * it needs to start at zero.  Every call on a device shares that device's
 * scratch, so calls that overlap on one device (different streams, or
 * different handles on concurrent streams) race: serialise them.
 * Errors: as fpsa_correct, and SN_E_INVALID when a slab needs more than
 * 64 MiB of scratch (the message states how much; use fpsa_correct).
 * Asynchronous. */
sn_status fpsa_correct_noalloc(sn_handle h, const double *phi_half, const double *phi_old,
                               double *phi_new, void *stream);

/* Source iteration (SN_SI, eq:trsi) or FPSA (SN_FPSA, eq:predict +
 * eq:correct) until max |phi^{m+1}_l - phi^m_l| <= tol over all cells, nodes
 * and l <= L of a slab (eq:iterate; FP64), each slab stopping on its own.
 *   q_ext      nullable device [cell][node][angle] source
 *   phi        device; in: phi^0, out: last iterate
 *   psi_exit   nullable device [sum N_b]: outgoing angular flux at the slab
 *              faces, angle order ascending (mu<0 entries at z0, mu>0 at z1)
 *   iters      host [num_slabs]: iterations taken (one sweep each)
 *   resid_hist nullable host [num_slabs * max_iter]: stopping-test value of
 *              every iteration (entries past iters[b] are left untouched)
 * SN_FPSA needs an SN_F64 handle with a Fokker-Planck scheme (else
 * SN_E_STATE).  For the GMRES methods the test is the 2-norm of the
 * (preconditioned) residual P (b - (I - K) phi), which bounds the max-norm
 * change of one FPSA (SI) step from phi, so tol means what it means for
 * SN_FPSA (SN_SI); iters counts sweeps, resid_hist holds the residual norm
 * after each sweep, and phi returns one FPSA (SI) step from the final
 * iterate.  GMRES needs an SN_F64 handle; SN_FPSA_GMRES a Fokker-Planck
 * scheme.  SN_F32 / SN_BF16X3 handles iterate all slabs together, each
 * slab's kernels skipped once its own test has passed.
 * Returns SN_OK, SN_NOT_CONVERGED (limit hit; outputs valid) or an error
 * (SN_E_NONFINITE if the iteration produced NaN/Inf).  Synchronises. */
sn_status sn_solve(sn_handle h, int32_t method, double tol, int32_t max_iter,
                   const void *q_ext, double *phi, void *psi_exit,
                   int32_t *iters, double *resid_hist, void *stream);

/* Exact transpose of the zero-inflow sweep operator q -> psi of sn_sweep
 * (angles swept in the opposite direction with transposed LD cell blocks):
 * for all x, y:  <y, sweep(x)> = <sweep_adjoint(y), x>  (plain dot product
 * over [cell][node][angle]).  psi_adj nullable; phi_adj (nullable) receives
 * the moments of psi_adj as in sn_sweep.  SN_F64 handles only.
 * Asynchronous. */
sn_status sn_sweep_adjoint(sn_handle h, const double *q_adj, double *psi_adj,
                           double *phi_adj, void *stream);

/* Replaces the cross sections used by the sweep and the scattering source
 * (host FP64 arrays laid out as in sn_problem_desc, validated the same way)
 * and keeps the quadrature and the Fokker-Planck factors: FPSA then
 * converges to the transport solution of the new cross sections with the
 * old operator as its preconditioner (SN_FP_CELL factors keep the old
 * sigma_s in their source maps too).  For parameter studies and finite
 * differences without a new factorisation.  SN_F64 handles only (else
 * SN_E_STATE).  Synchronises. */
sn_status sn_update_cross_sections(sn_handle h, const double *sigma_t, const double *sigma_s,
                                   void *stream);

/* Adjoint of the transport solution for a linear response
 *   J_b = <c, psi>  (plain dot product over slab b's [cell][node][angle]
 *                    entries; psi the solution of sn_solve's problem)
 * The discrete operator A = L_h - S_h of eq:treq (LD x S_N, symmetric
 * Gauss-Legendre quadrature) satisfies A^T = X A X^{-1} with X = W R,
 * W = diag(w_n), R the reflection mu_n -> -mu_n (n -> N-1-n), as
 * transposing the upwind LD cell equations reverses their direction.  The
 * adjoint lambda = W R y therefore follows from the FORWARD problem
 *   A y = R W^{-1} c   (zero inflow; nodal source Mass^{-1} R W^{-1} c)
 * solved here by SN_SI or SN_FPSA exactly as sn_solve does (same kernels,
 * same preconditioner, same stopping test applied to phi_y).
 *   c      device [cell][node][angle] response weights; for the exit
 *          current through z1: c = w_n mu_n at the right node of the last
 *          cell for mu_n > 0, zero elsewhere
 *   phi_y  device [cell][node][l]; in: initial guess (zero, or a previous
 *          adjoint: warm start), out: the moments of y
 *   iters, resid_hist as in sn_solve.
 * SN_F64 handles only; SN_FPSA needs a Fokker-Planck scheme.  Returns as
 * sn_solve.  Synchronises. */
sn_status sn_solve_adjoint(sn_handle h, int32_t method, double tol, int32_t max_iter,
                           const double *c, double *phi_y, int32_t *iters, double *resid_hist,
                           void *stream);

/* Response and its gradient with respect to every cell's cross sections,
 * from the converged moments of the forward solve (phi, with its q_ext and
 * the descriptor's inflows) and of the adjoint (phi_y, same c).  Only
 * moments are kept between the calls: psi and y are regenerated here by one
 * sweep each of their converged scattering sources.  With
 * Mass_k = (h_k/6) [[2,1],[1,2]]:
 *   J[b]                = <c, psi> over slab b
 *   g_sigma_t[k]        = dJ/dsigma_t(k) at fixed sigma_s
 *                       = - sum_{nu,nu',n} Mass_k[nu][nu'] w_n y(k,nu,N-1-n) psi(k,nu',n)
 *   g_sigma_s[k][l]     = dJ/dsigma_{s,l}(k)
 *                       = (2l+1)/2 (-1)^l sum_{nu,nu'} Mass_k[nu][nu'] phi_y(k,nu,l) phi(k,nu',l)
 * Device outputs: J [num_slabs], g_sigma_t [sum K], g_sigma_s
 * [sum K (L+1)].  q_ext nullable.  The derivatives are those of the
 * discrete solution; their accuracy follows the two solves' stopping
 * tests.  SN_F64 handles only.  Asynchronous. */
sn_status sn_response_gradient(sn_handle h, const double *q_ext, const double *phi, const double *c,
                               const double *phi_y, double *J, double *g_sigma_t, double *g_sigma_s,
                               void *stream);

/* Response weights of the partial current leaving each slab through its
 * right face z1 (the exit current differentiated by sn_solve_adjoint /
 * sn_response_gradient):
 *   c[k][nu][n] = w_n mu_n   for the last cell k = K-1, right LD node
 *                            nu = 1 and mu_n > 0,
 *   c[k][nu][n] = 0          elsewhere,
 * with the handle's Gauss-Legendre quadrature (so <c, psi> is
 * sum_{mu_n > 0} w_n mu_n psi_n(z1), the outgoing partial current of
 * Sec. 2's slab problem).  c: device FP64 [cell][node][angle], psi_len
 * entries, caller-owned, fully overwritten.  SN_F64 handles only (else
 * SN_E_STATE).  Asynchronous. */
sn_status sn_exit_current_weights(sn_handle h, double *c, void *stream);

/* Exit current of every slab from the outgoing face fluxes that sn_solve
 * returns in psi_exit:
 *   J[b] = sum_{mu_n > 0} w_n mu_n psi_exit[b][n]
 * (the mu_n > 0 entries of psi_exit are the angular flux leaving through
 * z1; the same quantity as <c, psi> with c from sn_exit_current_weights).
 * psi_exit: device [sum N_b], double for SN_F64 handles, float for
 * SN_F32 / SN_BF16X3 handles; J: device FP64 [num_slabs], accumulated in
 * FP64 in a fixed order.  Both caller-owned.  Asynchronous. */
sn_status sn_exit_current(sn_handle h, const void *psi_exit, double *J, void *stream);

/* Mixed-precision iterative refinement of the transport solution: the
 * batched low-precision handle lo (SN_F32 / SN_BF16X3) does the source
 * iterations, the FP64 handle hi (same slabs, any scheme) the residuals.
 *   1. phi <- low-precision source iteration from phi to tol_lo;
 *   2. r = D L^{-1}(M Sigma phi + q_ext + inflow) - phi in FP64 (one FP64
 *      sweep: the change one source iteration would make);
 *   3. stop if max |r| <= tol (the test of eq:iterate, in FP64);
 *   4. u = fixed point of u = D L^{-1} M Sigma (u + r) with zero inflow, by
 *      low-precision source iteration to inner_rel * max |r|; then
 *      phi += r + u, which solves (I - K) d = r for the correction d;
 *   5. back to 2.
 * Each step gains about the low precision's digits, so a few steps reach
 * FP64 accuracy while the source iterations run in FP32.
 *   q_ext       nullable device FP64 [cell][node][angle] source
 *   phi         device FP64; in: initial guess, out: refined solution
 *   steps       host: residual evaluations done (<= max_steps)
 *   inner_iters nullable host [num_slabs]: low-precision iterations, summed
 *   resid       nullable host [max_steps]: max |r| of each step
 * Allocates its work arrays (two phi-sized FP64, one or two psi-sized FP32)
 * for the call.  SN_OK when max |r| <= tol, SN_NOT_CONVERGED after
 * max_steps (phi valid), SN_E_STATE for the wrong handle kinds, SN_E_INVALID
 * if the handles describe different slabs.  Synchronises. */
sn_status sn_solve_refined(sn_handle lo, sn_handle hi, double tol, double tol_lo, double inner_rel,
                           int32_t max_steps, int32_t max_iter, const double *q_ext, double *phi,
                           int32_t *steps, int32_t *inner_iters, double *resid, void *stream);

/* Autotuner report of the sweep's decomposition.  *choice receives the
 * candidate kept (the fastest), ms[4] (nullable) the measured time of one
 * sweep per candidate (0 for a candidate that does not exist).
 *   Batched (SN_F32 / SN_BF16X3) handles: at setup the solve's sweep
 *   decomposition is built four ways and each is timed on the handle's own
 *   slabs; candidate c pairs long with short slab groups when (c & 1) == 0
 *   and sweeps N <= 16 slabs in cell segments when (c & 2) == 0.
 *   SN_F64 handles: the width of the sweep tiles (the cells one block
 *   scans, from which the scan's carries are formed) is chosen among three
 *   candidates, the default of about 128 tiles per slab (c = 0), half that
 *   width (c = 1) and twice it (c = 2), each rounded to the sweep's
 *   sub-chunk count and at most 32 cells (64 for N < 8); each is timed at
 *   setup on the solve's sweep (with its fused source and moments) of up to
 *   16 of the handle's slabs, and every slab takes the fastest.
 * Tiling changes no result: the scan's associativity is exact up to FP64
 * rounding order. */
sn_status sn_sweep_tuning(sn_handle h, int32_t *choice, double *ms);

/* Overrides the autotuner's choice with candidate choice (meaning as
 * above): 0..3 for batched handles, 0..2 for SN_F64 handles; for
 * reproducible decompositions and for testing every candidate.  On an
 * SN_F64 handle it synchronises the device and frees the batched solve's
 * workspace and captured graphs (rebuilt on the next solve).  SN_E_INVALID
 * outside that range. */
sn_status sn_set_sweep_choice(sn_handle h, int32_t choice);

/* Scan-width autotuner of a batched (SN_F32 / SN_BF16X3) handle.  Slabs of
 * at least 16384 cells are swept in the solve as chains of segments (per
 * slab and block of 64 angles): a first pass composes each segment's
 * affine cell maps, a scan over the chain forms the segments' carry-ins and
 * a second pass re-sweeps them.  At setup the segment length is chosen
 * among 512 (c = 0), 1024 (c = 1) and 2048 cells (c = 2) by timing one
 * warm-up and three sweeps of the handle's long slabs with each; the
 * fastest is kept.  *seg_cells receives its length (0 when the handle has
 * no such slab), ms[3] (nullable) the measured time per candidate (0
 * without long slabs).  Segment lengths change results by FP32 rounding
 * order only.  SN_E_STATE for SN_F64 handles. */
sn_status sn_scan_tuning(sn_handle h, int32_t *seg_cells, double *ms);

/* Overrides the scan-width choice of a batched handle with candidate
 * choice (0..2, as above); the solve's captured graphs follow the choice.
 * SN_E_INVALID outside 0..2, SN_E_STATE for SN_F64 handles. */
sn_status sn_set_scan_choice(sn_handle h, int32_t choice);

/* Fused source iteration of a batched (SN_F32 / SN_BF16X3) handle (eq:trsi
 * with the transport sweep of eq:treq, Sec. 2): instead of a scattering-
 * source GEMM, a sweep and a moments GEMM that pass q and psi through
 * device memory, each iteration runs three launches per class: per tile
 * of 32 cells of one slab, an aggregate pass forms the tile's source in LDS
 * on MFMA and composes the LD cell maps of every angle over each half of
 * the tile into the half's affine map (outflow = alpha inflow + beta); a
 * scan over each slab's half-tiles gives every half-tile its inflow and the
 * far-face exit; an apply pass forms the source again, sweeps both halves
 * from their inflows and writes the moments of the new iterate with the
 * stopping test.  An external source whose values
 * are equal over the angles of every node row of a tile is read as one
 * value per row.  Available when no slab has more than 131072 cells and
 * every (N, L+1) class has N and L+1 multiples of 4 with both at most 128
 * (and 16-byte aligned rows); then on by default.  SN_F32 handles form
 * both products on BF16 MFMA from three BF16 pieces of each FP32 operand
 * (x = p0 + p1 + p2; the six cross products that carry more than 2^-24 of
 * the result, FP32 accumulation), which rounds like FP32; SN_BF16X3 handles
 * form the source from two pieces (three products, the split-BF16
 * precision) and the moments on FP32 MFMA.  Results differ from the
 * unfused iteration by rounding only.  A q_ext that is not 16-byte aligned
 * takes the unfused iteration.
 * *enabled / *available receive the state (either nullable). */
sn_status sn_fused_iteration(sn_handle h, int32_t *enabled, int32_t *available);

/* Switches the fused iteration of a batched handle on (enable != 0) or off.
 * SN_E_STATE for SN_F64 handles and for enable != 0 where it is not
 * available. */
sn_status sn_set_fused_iteration(sn_handle h, int32_t enable);

/* Graph replay of a batched (SN_F32 / SN_BF16X3) handle's solve, on by
 * default.  When on and kernel timing is off, sn_solve captures the kernels
 * of one source iteration into a HIP graph once (they address the current
 * iteration through a device counter) and replays it once per iteration on
 * a stream the handle owns, ordered after and before the caller's stream by
 * events; up to four graphs (per source, exit buffer, tolerance, boundary
 * mode and sweep decomposition) stay cached on the handle.  The results are
 * those of the eager launches, bit for bit.  enable = 0 launches every
 * kernel from the host instead.  SN_E_STATE for SN_F64 handles. */
sn_status sn_set_graph_replay(sn_handle h, int32_t enable);

/* Multi-slab FP64 solves in batched launches, on by default.  When on,
 * sn_solve and sn_solve_adjoint (SN_SI, SN_FPSA) on an SN_F64 handle with
 * two or more slabs run every kernel of an iteration as one launch per
 * kernel variant over all slabs (and cell-type segments), each slab with its
 * own workspace, iterates and stopping test, skipped by every launch after
 * its test has passed; slabs that share Fokker-Planck factors
 * (SN_FP_MEAN) have their blocks side by side so that the shared factors
 * are read from cache.  The results are those of the slab-by-slab solve:
 * the same iteration counts, with moments that agree to FP64 rounding (the
 * same kernels, whose batched instances the compiler may contract
 * differently; measured within 1e-11 of the largest moment).
 * With kernel timing off, one iteration is captured into a HIP graph (once
 * per source, method and boundary mode, four kept per handle) and replayed
 * on a stream the handle owns, ordered after and before the caller's stream
 * by events.  The per-slab workspaces (about 3 phi + 4 psi values per
 * slab) are allocated on the first such solve; if they would exceed half
 * the free device memory (at most 32 GiB) the solve runs slab by slab.
 * enable = 0 always solves slab by slab (up to eight slabs at a time on
 * their own streams).  SN_E_STATE for batched (SN_F32 / SN_BF16X3)
 * handles. */
sn_status sn_set_batched_solve(sn_handle h, int32_t enable);

/* Per-kernel timing.  While enabled, every kernel the library launches is
 * bracketed by HIP events recorded on its launch stream; totals accumulate
 * per kernel until timing is switched off or on again (which resets them).
 * Reading resolves the recorded events (waits for them).  Off by default;
 * costs two event records per launch when on.
 * kernel_id in [0, SN_KERNEL_COUNT); *name receives a static string. */
#define SN_KERNEL_COUNT 20
sn_status sn_set_kernel_timing(sn_handle h, int32_t enable);
sn_status sn_get_kernel_timing(sn_handle h, int32_t kernel_id, const char **name,
                               int64_t *launches, double *total_ms);

/* Layout of slab b (host helper, no device work): info[0..5] = K, N, L,
 * cells per chunk and number of chunks of the Fokker-Planck recurrences,
 * number of sweep tiles, cells per sweep tile (SN_F64 handles). */
sn_status sn_slab_info(sn_handle h, int32_t slab, int32_t *info);

/* Sizes of the concatenated device arrays (host helper, no device work). */
sn_status sn_sizes(sn_handle h, int64_t *psi_len, int64_t *phi_len,
                   int64_t *exit_len);

#ifdef __cplusplus
}
#endif
#endif /* SNFPSA_H */
