// Host-side FP64 setup math of the slab S_N / FPSA library: quadrature,
// Legendre tables, angular Laplacians and the factorisation of the LD x S_N
// Fokker-Planck correction operator.  Runs once per sn_setup (the paper
// excludes this setup from its solver timings, Sec. 4).
#pragma once

#include <cstdint>
#include <vector>

namespace snfpsa {

using dvec = std::vector<double>;

// Gauss-Legendre rule on [-1,1], nodes ascending, weights summing to 2.
void gauss_legendre(int N, dvec &mu, dvec &w);

// P[l*N + n] = P_l(mu_n) for l = 0..L.
dvec legendre_table(int N, int L, const dvec &mu);

// Angular Laplacians of Sec. 2.2 (row-major N x N).
//   WFD: eq:fp-wdd / eq:sph-weights / eq:w_wfd with gamma_{1/2} = 0 and the
//        normalisation nu = -2 (so gamma_{N+1/2} = 0 and gamma > 0 inside).
//   MPD: eq:fp-mpd, F = V^{-1} diag(-l(l+1)) V; for Gauss-Legendre V^{-1} is
//        the moment-to-discrete map M_{n,l} = (2l+1)/2 P_l(mu_n) exactly.
dvec wfd_laplacian(int N, const dvec &mu, const dvec &w);
dvec mpd_laplacian(int N, const dvec &mu, const dvec &w);

// Factorised LD x S_N Fokker-Planck operator of one slab.
//
// Cell equations (both LD test functions, all N angles at once):
//   D_j u_j = Mass_j r_j + J [a_j ; b_{j+1}],   u_j = [U_L(0..N-1); U_R(0..N-1)]
// with removal T = sigma_a I - (sigma_tr/2) A and inflows a_j (the N/2
// positive-cosine fluxes entering cell j through its left face) and b_{j+1}
// (the N/2 negative-cosine fluxes entering through its right face); zero
// inflow at both slab faces.  Eliminating the cell interiors leaves, per
// cell, the interface relations
//   a_{j+1} = T_j a_j + R_j b_{j+1} + s+_j,   b_j = R'_j a_j + T'_j b_{j+1} + s-_j,
// which are solved by a forward Riccati recursion a_j = rho_j b_j + p_j
// followed by a backward substitution for b_j:
//   p_{j+1} = G_j p_j + Hm_j s-_j + s+_j
//   b_j     = U_j b_{j+1} + Y_j p_j + X_j s-_j,    a_j = rho_j b_j + p_j.
// G, Hm, U, Y, X, rho are fixed by the operator and precomputed here; only
// the vectors change per application.
struct FPFactors {
    int K = 0, N = 0, L = 0, NH = 0;
    int chunk = 0, nchunks = 0;
    // per cell: 6 matrices NH x NH, order [G, Hm, U, Y, X, rho]
    dvec cellmats;                    // [K][6][NH][NH]
    // chunk products: forward G_{j1}...G_{j0}, backward U_{j0}...U_{j1}
    dvec chunk_fwd, chunk_bwd;        // [nchunks][NH][NH]
    // Parallel completion of the chunked recurrences.  With p_loc / b_loc
    // the chain values of a chunk started from a zero carry:
    //   p_j = p_loc_j + PsiF_j carry_c,  PsiF_j = G_{j-1} ... G_{j0} (I at j0)
    //   b_j = b_loc_j + PsiB_j carry'_c, PsiB_j = U_j ... U_{j1-1}
    //   carry_c  = sum_{c'<c} ThF_{c,c'} e_{c'},  ThF_{c,c'} = Phi_{c-1}...Phi_{c'+1}
    //   carry'_c = sum_{c'>c} ThB_{c,c'} e'_{c'}, ThB_{c,c'} = Phi'_{c+1}...Phi'_{c'-1}
    // (carry_c = p at the first interface of chunk c, carry'_c = b at the
    // interface after its last cell; the nearest-neighbour terms are I).
    dvec psi_fwd, psi_bwd;            // [K][NH][NH]
    dvec theta_fwd;                   // ThF_{c,c'} for 0 <= c' <= c-2, c = 2..nchunks,
                                      //   at index (c-1)(c-2)/2 + c'
    dvec theta_bwd;                   // ThB_{c,c'} for c+2 <= c' <= nchunks-1, c = -1..nchunks-3,
                                      //   stored like ThF with c -> nchunks-1-c
    // cell types (runs of identical cells): type index + per-type matrices
    std::vector<int32_t> seg_begin;   // [nseg+1] cell ranges of equal type
    std::vector<int32_t> seg_type;    // [nseg]
    int ntypes = 0;
    // per type, stored as GEMM right operands (row-major K x Ncols):
    //   EsrcT  [2(L+1)][N]     source of the interface problem: s = [s+; s-]
    //   PhisrcT[2(L+1)][2(L+1)] moments of the zero-inflow cell solution
    //   PhiinfT[N][2(L+1)]      moments of the response to [a_j; b_{j+1}]
    dvec EsrcT, PhisrcT, PhiinfT;
};

// sigma_s is [K][L+1] for this slab; sigma_a = sigma_t - sigma_s0,
// sigma_tr = sigma_s0 - sigma_s1.  Returns false if a cell block is
// singular.
bool build_fp_factors(int K, int N, int L, const double *h, const double *sigma_t,
                      const double *sigma_s, const dvec &mu, const dvec &w,
                      const dvec &A, FPFactors &out, int chunk_hint = 0);

}  // namespace snfpsa
