/*
 * snfpsa_diag.h -- host-only diagnostics of the library's setup math.
 *
 * These calls expose what sn_setup computes on the host (quadrature, angular
 * Laplacians, and the factorised Fokker-Planck operator) so that the setup
 * can be checked on a machine without a GPU.  They launch no device work
 * and no solver call uses them.  All arrays are host memory, FP64 unless
 * stated, row-major.
 */
#ifndef SNFPSA_DIAG_H
#define SNFPSA_DIAG_H

#include <stdint.h>

#include "snfpsa.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Gauss-Legendre nodes (ascending) and weights (sum 2) used by sn_setup. */
sn_status sn_diag_quadrature(int32_t N, double *mu, double *w);

/* N x N angular Laplacian: scheme SN_FP_WFD (eq:w_wfd, nu = -2) or
 * SN_FP_MPD (eq:fp-mpd). */
sn_status sn_diag_laplacian(int32_t N, int32_t scheme, double *A);

/* Factorisation of one slab's LD x S_N Fokker-Planck operator (the
 * two-sided interface-Riccati form used by fpsa_correct: forward
 * a = rho b + p, backward b = sig a + q, combined per interface).  h, sigma_t [K],
 * sigma_s [K][L+1]; chunk <= 0 picks the default chunk length. */
typedef struct sn_diag_fp_s *sn_diag_fp;
sn_status sn_diag_fp_factor(int32_t K, int32_t N, int32_t L, const double *h,
                            const double *sigma_t, const double *sigma_s,
                            int32_t scheme, int32_t chunk, sn_diag_fp *out);
/* info[4] = {chunk, nchunks, ntypes, nsegments} */
sn_status sn_diag_fp_info(sn_diag_fp p, int32_t *info);
/* which: 0 cellmats [K][7][N/2][N/2] (G, Hm, Gb, Hb, W, W rho, sig)
 *        1 forward chunk products [nchunks][N/2][N/2]
 *        2 backward chunk products [nchunks][N/2][N/2]
 *        3 EsrcT [ntypes][2(L+1)][N]
 *        4 PhisrcT [ntypes][2(L+1)][2(L+1)]
 *        5 PhiinfT [ntypes][N][2(L+1)]
 *        6 segment starts, int32 [nsegments+1]
 *        7 segment types, int32 [nsegments]
 *        8 within-chunk forward prefix products PsiF [K][N/2][N/2]
 *        9 within-chunk backward prefix products PsiB [K][N/2][N/2] (of Gb)
 *       10 forward chunk transfer products ThF [nchunks(nchunks-1)/2][N/2][N/2]
 *       11 backward chunk transfer products ThB [nchunks(nchunks-1)/2][N/2][N/2] */
sn_status sn_diag_fp_get(sn_diag_fp p, int32_t which, void *dst);
sn_status sn_diag_fp_free(sn_diag_fp p);

#ifdef __cplusplus
}
#endif
#endif /* SNFPSA_DIAG_H */
