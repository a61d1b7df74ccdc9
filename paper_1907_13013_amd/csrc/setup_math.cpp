// Host FP64 setup math: quadrature, Legendre tables, WFD/MPD Laplacians and
// the two-sided interface (Riccati) factorisation of the LD x S_N
// Fokker-Planck operator.  See setup_math.hpp for the formulation.
#include "setup_math.hpp"

#include <cmath>
#include <map>
#include <stdexcept>

namespace snfpsa {

namespace {

constexpr double kPi = 3.14159265358979323846;

// P_n(x) and P_{n-1}(x) by the three-term recurrence.
void legendre_pair(int n, double x, double &pn, double &pnm1) {
    double a = 1.0, b = x;
    if (n == 0) { pn = 1.0; pnm1 = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
        a = b;
        b = c;
    }
    pn = b;
    pnm1 = a;
}

// Row-major dense helpers on n x n (or general) matrices.
void matmul(int m, int k, int n, const double *A, const double *B, double *C) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int t = 0; t < k; ++t) s += A[(size_t)i * k + t] * B[(size_t)t * n + j];
            C[(size_t)i * n + j] = s;
        }
}

// In-place inverse by Gauss-Jordan elimination with partial pivoting.
bool invert(int n, double *A) {
    std::vector<double> M((size_t)n * 2 * n, 0.0);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) M[(size_t)i * 2 * n + j] = A[(size_t)i * n + j];
        M[(size_t)i * 2 * n + n + i] = 1.0;
    }
    const int w2 = 2 * n;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        double best = std::fabs(M[(size_t)c * w2 + c]);
        for (int r = c + 1; r < n; ++r) {
            double v = std::fabs(M[(size_t)r * w2 + c]);
            if (v > best) { best = v; piv = r; }
        }
        if (!(best > 0.0)) return false;
        if (piv != c)
            for (int j = 0; j < w2; ++j) std::swap(M[(size_t)c * w2 + j], M[(size_t)piv * w2 + j]);
        const double inv = 1.0 / M[(size_t)c * w2 + c];
        for (int j = 0; j < w2; ++j) M[(size_t)c * w2 + j] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = M[(size_t)r * w2 + c];
            if (f == 0.0) continue;
            for (int j = 0; j < w2; ++j) M[(size_t)r * w2 + j] -= f * M[(size_t)c * w2 + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = M[(size_t)i * w2 + n + j];
    return true;
}

}  // namespace

void gauss_legendre(int N, dvec &mu, dvec &w) {
    mu.assign(N, 0.0);
    w.assign(N, 0.0);
    for (int i = 1; i <= N; ++i) {
        // Tricomi's asymptotic guess for the i-th largest root, then Newton.
        double x = (1.0 - 1.0 / (8.0 * N * N) + 1.0 / (8.0 * N * N * N)) *
                   std::cos(kPi * (4.0 * i - 1.0) / (4.0 * N + 2.0));
        double pn = 0, pm = 0, dp = 1;
        for (int it = 0; it < 60; ++it) {
            legendre_pair(N, x, pn, pm);
            dp = N * (pm - x * pn) / (1.0 - x * x);
            const double dx = pn / dp;
            x -= dx;
            if (std::fabs(dx) <= 1e-17 * std::fabs(x) + 1e-300) break;
        }
        legendre_pair(N, x, pn, pm);
        const double one_m_x2 = (1.0 - x) * (1.0 + x);  // accurate near |x| = 1
        dp = N * (pm - x * pn) / one_m_x2;
        mu[N - i] = x;
        w[N - i] = 2.0 / (one_m_x2 * dp * dp);
    }
    // symmetrise: the rule is exactly symmetric about 0
    for (int i = 0; i < N / 2; ++i) {
        const double m = 0.5 * (mu[N - 1 - i] - mu[i]);
        const double ww = 0.5 * (w[N - 1 - i] + w[i]);
        mu[i] = -m;
        mu[N - 1 - i] = m;
        w[i] = w[N - 1 - i] = ww;
    }
    if (N % 2) mu[N / 2] = 0.0;
}

dvec legendre_table(int N, int L, const dvec &mu) {
    dvec P((size_t)(L + 1) * N);
    for (int n = 0; n < N; ++n) {
        double a = 1.0, b = mu[n];
        P[n] = 1.0;
        if (L >= 1) P[(size_t)N + n] = b;
        for (int l = 2; l <= L; ++l) {
            double c = ((2 * l - 1) * mu[n] * b - (l - 1) * a) / l;
            P[(size_t)l * N + n] = c;
            a = b;
            b = c;
        }
    }
    return P;
}

dvec wfd_laplacian(int N, const dvec &mu, const dvec &w) {
    // gamma[i] = gamma_{i+1/2} in 1-based notation: gamma[0] = gamma_{1/2} = 0
    dvec gamma(N + 1, 0.0);
    for (int n = 0; n < N; ++n) gamma[n + 1] = gamma[n] - 2.0 * mu[n] * w[n];
    gamma[N] = 0.0;
    dvec W((size_t)N * N, 0.0);
    for (int n = 0; n < N; ++n) {
        const double down = (n > 0) ? gamma[n] / (mu[n] - mu[n - 1]) : 0.0;
        const double up = (n + 1 < N) ? gamma[n + 1] / (mu[n + 1] - mu[n]) : 0.0;
        if (n > 0) W[(size_t)n * N + n - 1] = down / w[n];
        if (n + 1 < N) W[(size_t)n * N + n + 1] = up / w[n];
        W[(size_t)n * N + n] = -(down + up) / w[n];
    }
    return W;
}

dvec mpd_laplacian(int N, const dvec &mu, const dvec &w) {
    dvec P = legendre_table(N, N - 1, mu);
    dvec F((size_t)N * N, 0.0);
    // F[n][m] = sum_l (2l+1)/2 P_l(mu_n) (-l(l+1)) P_l(mu_m) w_m
    for (int n = 0; n < N; ++n)
        for (int m = 0; m < N; ++m) {
            double s = 0.0;
            for (int l = 0; l < N; ++l)
                s += 0.5 * (2 * l + 1) * P[(size_t)l * N + n] * (-(double)l * (l + 1)) * P[(size_t)l * N + m];
            F[(size_t)n * N + m] = s * w[m];
        }
    return F;
}

bool build_fp_factors(int K, int N, int L, const double *h, const double *sigma_t,
                      const double *sigma_s, const dvec &mu, const dvec &w, const dvec &A,
                      FPFactors &out, int chunk_hint) {
    const int L1 = L + 1;
    dvec sa(K), str(K);
    for (int j = 0; j < K; ++j) {
        const double *ss = sigma_s + (size_t)j * L1;
        sa[j] = sigma_t[j] - ss[0];
        str[j] = ss[0] - (L1 > 1 ? ss[1] : 0.0);
    }
    return build_fp_factors_coef(K, N, L, h, sa.data(), str.data(), sigma_s, mu, w, A, out, chunk_hint);
}

bool build_fp_factors_coef(int K, int N, int L, const double *h, const double *sigma_a,
                           const double *sigma_tr, const double *sigma_s, const dvec &mu, const dvec &w,
                           const dvec &A, FPFactors &out, int chunk_hint) {
    const int NH = N / 2, N2 = 2 * N, L1 = L + 1, L2 = 2 * L1;
    out.K = K; out.N = N; out.L = L; out.NH = NH;
    out.folded_sigma_s = sigma_s != nullptr;
    dvec P = legendre_table(N, L, mu);

    // ---- cell types: runs of cells with identical (h, sigma_a, sigma_tr and,
    // when it is folded into the source maps, sigma_s row)
    std::map<std::vector<double>, int> type_of;
    std::vector<std::vector<double>> keys;
    out.seg_begin.clear();
    out.seg_type.clear();
    std::vector<int> cell_type(K);
    const int nkey = 3 + (sigma_s ? L1 : 0);
    for (int j = 0; j < K; ++j) {
        std::vector<double> key(nkey);
        key[0] = h[j];
        key[1] = sigma_a[j];
        key[2] = sigma_tr[j];
        if (sigma_s)
            for (int l = 0; l < L1; ++l) key[3 + l] = sigma_s[(size_t)j * L1 + l];
        auto it = type_of.find(key);
        int t;
        if (it == type_of.end()) {
            t = (int)keys.size();
            type_of.emplace(key, t);
            keys.push_back(key);
        } else {
            t = it->second;
        }
        cell_type[j] = t;
        if (j == 0 || cell_type[j - 1] != t) {
            out.seg_begin.push_back(j);
            out.seg_type.push_back(t);
        }
    }
    out.seg_begin.push_back(K);
    const int ntypes = (int)keys.size();
    out.ntypes = ntypes;

    // ---- per type: cell block, responses, source and moment maps
    std::vector<dvec> Tc(ntypes), Rc(ntypes), Rpc(ntypes), Tpc(ntypes);
    out.EsrcT.assign((size_t)ntypes * L2 * N, 0.0);
    out.PhisrcT.assign((size_t)ntypes * L2 * L2, 0.0);
    out.PhiinfT.assign((size_t)ntypes * N * L2, 0.0);
    dvec D((size_t)N2 * N2), Pm((size_t)N2 * N), Q((size_t)N2 * N2), Qp((size_t)N2 * L2);
    for (int t = 0; t < ntypes; ++t) {
        const double hh = keys[t][0], sa = keys[t][1], str = keys[t][2];
        // D: LD cell block with removal T = sa I - (str/2) A
        for (int n = 0; n < N; ++n)
            for (int m = 0; m < N; ++m) {
                const double T = (n == m ? sa : 0.0) - 0.5 * str * A[(size_t)n * N + m];
                D[(size_t)n * N2 + m] = hh / 3.0 * T;
                D[(size_t)n * N2 + N + m] = hh / 6.0 * T;
                D[(size_t)(N + n) * N2 + m] = hh / 6.0 * T;
                D[(size_t)(N + n) * N2 + N + m] = hh / 3.0 * T;
            }
        for (int n = 0; n < N; ++n) {
            const double m = mu[n];
            D[(size_t)n * N2 + n] += std::fabs(m) / 2.0;
            D[(size_t)n * N2 + N + n] += m / 2.0;
            D[(size_t)(N + n) * N2 + n] -= m / 2.0;
            D[(size_t)(N + n) * N2 + N + n] += std::fabs(m) / 2.0;
        }
        if (!invert(N2, D.data())) return false;  // D now holds D^{-1}
        // Pm = D^{-1} J: inflow columns [a (angles NH..N-1) ; b (angles 0..NH-1)]
        for (int r = 0; r < N2; ++r) {
            for (int i = 0; i < NH; ++i) {
                const int na = NH + i, nb = i;
                Pm[(size_t)r * N + i] = D[(size_t)r * N2 + na] * mu[na];            // row L_na, +mu
                Pm[(size_t)r * N + NH + i] = D[(size_t)r * N2 + N + nb] * (-mu[nb]); // row R_nb, |mu|
            }
        }
        // Q = D^{-1} Mass, Mass per angle (h/6)[[2,1],[1,2]] on (L,R)
        for (int r = 0; r < N2; ++r)
            for (int n = 0; n < N; ++n) {
                const double dl = D[(size_t)r * N2 + n], dr = D[(size_t)r * N2 + N + n];
                Q[(size_t)r * N2 + n] = hh / 6.0 * (2.0 * dl + dr);
                Q[(size_t)r * N2 + N + n] = hh / 6.0 * (dl + 2.0 * dr);
            }
        // Qp = Q (I2 x M Sigma): column (nu, l)
        for (int r = 0; r < N2; ++r)
            for (int nu = 0; nu < 2; ++nu)
                for (int l = 0; l < L1; ++l) {
                    double s = 0.0;
                    for (int n = 0; n < N; ++n)
                        s += Q[(size_t)r * N2 + nu * N + n] * 0.5 * (2 * l + 1) * P[(size_t)l * N + n];
                    Qp[(size_t)r * L2 + nu * L1 + l] = sigma_s ? s * keys[t][3 + l] : s;
                }
        // interface responses; outgoing rows: a_out = U_R at angles NH..N-1,
        // b_out = U_L at angles 0..NH-1
        Tc[t].assign((size_t)NH * NH, 0); Rc[t].assign((size_t)NH * NH, 0);
        Rpc[t].assign((size_t)NH * NH, 0); Tpc[t].assign((size_t)NH * NH, 0);
        for (int i = 0; i < NH; ++i) {
            const int ra = N + NH + i, rb = i;
            for (int c = 0; c < NH; ++c) {
                Tc[t][(size_t)i * NH + c] = Pm[(size_t)ra * N + c];
                Rc[t][(size_t)i * NH + c] = Pm[(size_t)ra * N + NH + c];
                Rpc[t][(size_t)i * NH + c] = Pm[(size_t)rb * N + c];
                Tpc[t][(size_t)i * NH + c] = Pm[(size_t)rb * N + NH + c];
            }
        }
        double *Es = &out.EsrcT[(size_t)t * L2 * N];
        for (int i = 0; i < NH; ++i)
            for (int col = 0; col < L2; ++col) {
                Es[(size_t)col * N + i] = Qp[(size_t)(N + NH + i) * L2 + col];
                Es[(size_t)col * N + NH + i] = Qp[(size_t)i * L2 + col];
            }
        double *Ps = &out.PhisrcT[(size_t)t * L2 * L2];
        double *Pi = &out.PhiinfT[(size_t)t * N * L2];
        for (int nu = 0; nu < 2; ++nu)
            for (int l = 0; l < L1; ++l) {
                const int row = nu * L1 + l;
                for (int col = 0; col < L2; ++col) {
                    double s = 0.0;
                    for (int n = 0; n < N; ++n)
                        s += P[(size_t)l * N + n] * w[n] * Qp[(size_t)(nu * N + n) * L2 + col];
                    Ps[(size_t)col * L2 + row] = s;
                }
                for (int col = 0; col < N; ++col) {
                    double s = 0.0;
                    for (int n = 0; n < N; ++n)
                        s += P[(size_t)l * N + n] * w[n] * Pm[(size_t)(nu * N + n) * N + col];
                    Pi[(size_t)col * L2 + row] = s;
                }
            }
    }

    // ---- Riccati eliminations from both faces
    const size_t M2 = (size_t)NH * NH;
    const size_t CM = FP_CELL_MATS * M2;
    out.cellmats.assign((size_t)K * CM, 0.0);
    dvec rho_all((size_t)(K + 1) * M2, 0.0), sig(M2, 0.0), tmp(M2), tmp2(M2), Mg(M2);
    for (int j = 0; j < K; ++j) {
        const int t = cell_type[j];
        const double *rho = &rho_all[(size_t)j * M2];
        double *G = &out.cellmats[(size_t)j * CM], *Hm = G + M2;
        // G = T (I - rho R')^{-1}, Hm = G rho, rho_{j+1} = R + Hm T'
        matmul(NH, NH, NH, rho, Rpc[t].data(), tmp.data());
        for (size_t e = 0; e < M2; ++e) Mg[e] = -tmp[e];
        for (int i = 0; i < NH; ++i) Mg[(size_t)i * NH + i] += 1.0;
        if (!invert(NH, Mg.data())) return false;
        matmul(NH, NH, NH, Tc[t].data(), Mg.data(), G);
        matmul(NH, NH, NH, G, rho, Hm);
        matmul(NH, NH, NH, Hm, Tpc[t].data(), tmp.data());
        double *rn = &rho_all[(size_t)(j + 1) * M2];
        for (size_t e = 0; e < M2; ++e) rn[e] = Rc[t][e] + tmp[e];
    }
    for (int j = K - 1; j >= 0; --j) {
        const int t = cell_type[j];
        double *cm = &out.cellmats[(size_t)j * CM];
        double *Gb = cm + 2 * M2, *Hb = cm + 3 * M2, *W = cm + 4 * M2, *Wr = cm + 5 * M2, *S = cm + 6 * M2;
        // sig holds sig_{j+1}: Gb = T' (I - sig R)^{-1}, Hb = Gb sig, sig_j = R' + Hb T
        matmul(NH, NH, NH, sig.data(), Rc[t].data(), tmp.data());
        for (size_t e = 0; e < M2; ++e) Mg[e] = -tmp[e];
        for (int i = 0; i < NH; ++i) Mg[(size_t)i * NH + i] += 1.0;
        if (!invert(NH, Mg.data())) return false;
        matmul(NH, NH, NH, Tpc[t].data(), Mg.data(), Gb);
        matmul(NH, NH, NH, Gb, sig.data(), Hb);
        matmul(NH, NH, NH, Hb, Tc[t].data(), tmp.data());
        for (size_t e = 0; e < M2; ++e) sig[e] = Rpc[t][e] + tmp[e];
        // interface j: W = (I - rho_j sig_j)^{-1}, W rho_j, sig_j
        const double *rho = &rho_all[(size_t)j * M2];
        matmul(NH, NH, NH, rho, sig.data(), tmp.data());
        for (size_t e = 0; e < M2; ++e) W[e] = -tmp[e];
        for (int i = 0; i < NH; ++i) W[(size_t)i * NH + i] += 1.0;
        if (!invert(NH, W)) return false;
        matmul(NH, NH, NH, W, rho, Wr);
        std::copy(sig.begin(), sig.end(), S);
    }

    // ---- chunk products for the chunked recurrences
    // chunk length ~ sqrt(K/2) balances the local pass (chunk steps) against
    // the fix pass (up to K/chunk fold steps + chunk steps)
    int chunk = chunk_hint > 0 ? chunk_hint : (int)std::lround(std::sqrt(0.5 * K));
    if (chunk < 4) chunk = 4;
    if (chunk > K) chunk = K;
    out.chunk = chunk;
    out.nchunks = (K + chunk - 1) / chunk;
    out.chunk_fwd.assign((size_t)out.nchunks * M2, 0.0);
    out.chunk_bwd.assign((size_t)out.nchunks * M2, 0.0);
    for (int c = 0; c < out.nchunks; ++c) {
        const int j0 = c * chunk, j1 = std::min(K, j0 + chunk) - 1;
        dvec F(M2, 0.0), B(M2, 0.0);
        for (int i = 0; i < NH; ++i) F[(size_t)i * NH + i] = B[(size_t)i * NH + i] = 1.0;
        for (int j = j0; j <= j1; ++j) {
            matmul(NH, NH, NH, &out.cellmats[(size_t)j * CM], F.data(), tmp.data());
            F.swap(tmp);
        }
        for (int j = j1; j >= j0; --j) {
            matmul(NH, NH, NH, &out.cellmats[(size_t)j * CM + 2 * M2], B.data(), tmp2.data());
            B.swap(tmp2);
        }
        std::copy(F.begin(), F.end(), out.chunk_fwd.begin() + (size_t)c * M2);
        std::copy(B.begin(), B.end(), out.chunk_bwd.begin() + (size_t)c * M2);
    }

    // ---- within-chunk prefix products
    out.psi_fwd.assign((size_t)K * M2, 0.0);
    out.psi_bwd.assign((size_t)K * M2, 0.0);
    for (int c = 0; c < out.nchunks; ++c) {
        const int j0 = c * chunk, j1 = std::min(K, j0 + chunk);
        dvec Pf(M2, 0.0);
        for (int i = 0; i < NH; ++i) Pf[(size_t)i * NH + i] = 1.0;
        for (int j = j0; j < j1; ++j) {
            std::copy(Pf.begin(), Pf.end(), out.psi_fwd.begin() + (size_t)j * M2);
            matmul(NH, NH, NH, &out.cellmats[(size_t)j * CM], Pf.data(), tmp.data());
            Pf.swap(tmp);
        }
        dvec Pb(M2, 0.0);
        for (int i = 0; i < NH; ++i) Pb[(size_t)i * NH + i] = 1.0;
        for (int j = j1 - 1; j >= j0; --j) {
            matmul(NH, NH, NH, &out.cellmats[(size_t)j * CM + 2 * M2], Pb.data(), tmp.data());
            Pb.swap(tmp);
            std::copy(Pb.begin(), Pb.end(), out.psi_bwd.begin() + (size_t)j * M2);
        }
    }

    // ---- chunk-to-chunk transfer products
    // forward: carry_c for c = 0..NC (carry_P = p_K).  ThF_{c,c'} for c' <= c-2.
    const int NC = out.nchunks;
    auto tri = [](int a) { return (size_t)(a - 1) * (a - 2) / 2; };  // first index of row a
    out.theta_fwd.assign(tri(NC + 1) * M2, 0.0);
    for (int c = 2; c <= NC; ++c) {
        // ThF_{c,c'} = Phi_{c-1} ... Phi_{c'+1}; build from c' = c-2 downwards
        dvec Th(M2);
        std::copy(out.chunk_fwd.begin() + (size_t)(c - 1) * M2, out.chunk_fwd.begin() + (size_t)c * M2,
                  Th.begin());
        for (int cp = c - 2; cp >= 0; --cp) {
            std::copy(Th.begin(), Th.end(), out.theta_fwd.begin() + (tri(c) + cp) * M2);
            if (cp > 0) {
                matmul(NH, NH, NH, Th.data(), &out.chunk_fwd[(size_t)cp * M2], tmp.data());
                Th.swap(tmp);
            }
        }
    }
    // backward: carry'_c for c = -1..NC-1 (carry'_{NC-1} = b_K = 0, carry'_{-1} = b_0).
    // Mirror index a = NC-1-c (a = 0..NC): ThB_{c,c'} for c' >= c+2 stored at
    // tri(a) + (NC-1-c') with c' from c+2 .. NC-1.
    out.theta_bwd.assign(tri(NC + 1) * M2, 0.0);
    for (int c = -1; c <= NC - 3; ++c) {
        const int a = NC - 1 - c;
        // ThB_{c,c'} = Phi'_{c+1} ... Phi'_{c'-1}; build from c' = c+2 upwards
        dvec Th(M2);
        std::copy(out.chunk_bwd.begin() + (size_t)(c + 1) * M2, out.chunk_bwd.begin() + (size_t)(c + 2) * M2,
                  Th.begin());
        for (int cp = c + 2; cp <= NC - 1; ++cp) {
            std::copy(Th.begin(), Th.end(), out.theta_bwd.begin() + (tri(a) + (NC - 1 - cp)) * M2);
            if (cp < NC - 1) {
                matmul(NH, NH, NH, Th.data(), &out.chunk_bwd[(size_t)cp * M2], tmp.data());
                Th.swap(tmp);
            }
        }
    }
    return true;
}

}  // namespace snfpsa
