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
// inflow at both slab faces (a_0 = 0, b_K = 0).  Eliminating the cell
// interiors leaves, per cell, the interface relations
//   a_{j+1} = T_j a_j + R_j b_{j+1} + s+_j,   b_j = R'_j a_j + T'_j b_{j+1} + s-_j.
// They are solved by two independent Riccati eliminations and a local
// combination at each interface k:
//   from the left   a_k = rho_k b_k + p_k,    p_{j+1} = G_j p_j + Hm_j s-_j + s+_j
//   from the right  b_k = sig_k a_k + q_k,    q_j = Gb_j q_{j+1} + Hb_j s+_j + s-_j
//   a_k = W_k p_k + (W rho)_k q_k,  b_k = sig_k a_k + q_k,  W_k = (I - rho_k sig_k)^{-1}
// with rho_0 = 0, p_0 = 0, sig_K = 0, q_K = 0 and
//   G_j = T_j (I - rho_j R'_j)^{-1},   Hm_j = G_j rho_j,   rho_{j+1} = R_j + Hm_j T'_j,
//   Gb_j = T'_j (I - sig_{j+1} R_j)^{-1}, Hb_j = Gb_j sig_{j+1}, sig_j = R'_j + Hb_j T_j.
// All matrices are fixed by the operator and precomputed here; only the
// vectors change per application.
constexpr int FP_CELL_MATS = 7;  // per cell: G, Hm, Gb, Hb, W, W rho, sig

struct FPFactors {
    int K = 0, N = 0, L = 0, NH = 0;
    int chunk = 0, nchunks = 0;
    bool folded_sigma_s = true;       // EsrcT / PhisrcT include the cell's sigma_s
    // per cell j (interface j for W, W rho, sig): FP_CELL_MATS matrices NH x NH
    dvec cellmats;                    // [K][FP_CELL_MATS][NH][NH]
    // chunk products: forward G_{j1}...G_{j0}, backward Gb_{j0}...Gb_{j1}
    dvec chunk_fwd, chunk_bwd;        // [nchunks][NH][NH]
    // Parallel completion of the chunked recurrences.  With p_loc / q_loc
    // the chain values of a chunk started from a zero carry:
    //   p_j = p_loc_j + PsiF_j carry_c,  PsiF_j = G_{j-1} ... G_{j0} (I at j0)
    //   q_j = q_loc_j + PsiB_j carry'_c, PsiB_j = Gb_j ... Gb_{j1-1}
    //   carry_c  = sum_{c'<c} ThF_{c,c'} e_{c'},  ThF_{c,c'} = Phi_{c-1}...Phi_{c'+1}
    //   carry'_c = sum_{c'>c} ThB_{c,c'} e'_{c'}, ThB_{c,c'} = Phi'_{c+1}...Phi'_{c'-1}
    // (carry_c = p at the first interface of chunk c, carry'_c = q at the
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
// singular.  The FPSA residual's scattering matrix is folded into the
// source maps (EsrcT, PhisrcT act on phi_half - phi_old).
bool build_fp_factors(int K, int N, int L, const double *h, const double *sigma_t,
                      const double *sigma_s, const dvec &mu, const dvec &w,
                      const dvec &A, FPFactors &out, int chunk_hint = 0);

// The same from the removal coefficients of F directly: sigma_a, sigma_tr
// [K].  sigma_s (nullable) as above; null leaves the scattering out of the
// source maps, which then act on Sigma (phi_half - phi_old) formed by the
// caller, and cell types depend on (h, sigma_a, sigma_tr) only.
bool build_fp_factors_coef(int K, int N, int L, const double *h, const double *sigma_a,
                           const double *sigma_tr, const double *sigma_s, const dvec &mu,
                           const dvec &w, const dvec &A, FPFactors &out, int chunk_hint = 0);

}  // namespace snfpsa
