// Drives the library's host setup math (quadrature, Legendre tables, WFD
// and MPD Laplacians, the interface factorisation of the Fokker-Planck
// operator, chunk and transfer products, cell types) for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer; the same functions the
// C ABI's sn_setup and the sn_diag_* calls run on the host.  Exit status 0
// when every factorisation succeeded and its arrays have their documented
// sizes.
#include <cmath>
#include <cstdio>
#include <vector>

#include "setup_math.hpp"

using namespace snfpsa;

#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);  \
            return 1;                                                                \
        }                                                                            \
    } while (0)

static int one(int K, int N, int L, int regions, int chunk, int scheme) {
    dvec mu, w;
    gauss_legendre(N, mu, w);
    CHECK((int)mu.size() == N && (int)w.size() == N);
    const dvec P = legendre_table(N, L, mu);
    CHECK(P.size() == (size_t)(L + 1) * N);
    const dvec A = scheme == 0 ? wfd_laplacian(N, mu, w) : mpd_laplacian(N, mu, w);
    CHECK(A.size() == (size_t)N * N);
    std::vector<double> h(K), st(K), ss((size_t)K * (L + 1));
    for (int k = 0; k < K; ++k) {
        const int reg = (k * regions) / K;
        h[k] = 0.05 + 0.01 * reg;
        st[k] = 0.5 + reg;
        double gl = 1.0;
        for (int l = 0; l <= L; ++l, gl *= 0.9) ss[(size_t)k * (L + 1) + l] = (0.9 - 0.05 * reg) * st[k] * gl;
    }
    FPFactors F;
    CHECK(build_fp_factors(K, N, L, h.data(), st.data(), ss.data(), mu, w, A, F, chunk));
    const size_t M2 = (size_t)(N / 2) * (N / 2);
    CHECK(F.cellmats.size() == (size_t)K * FP_CELL_MATS * M2);
    CHECK(F.psi_fwd.size() == (size_t)K * M2 && F.psi_bwd.size() == (size_t)K * M2);
    CHECK(F.nchunks >= 1 && (int)F.seg_type.size() + 1 == (int)F.seg_begin.size());
    for (double v : F.cellmats) CHECK(std::isfinite(v));
    std::vector<double> sa(K), str(K);
    for (int k = 0; k < K; ++k) {
        sa[k] = st[k] - ss[(size_t)k * (L + 1)];
        str[k] = ss[(size_t)k * (L + 1)] - (L >= 1 ? ss[(size_t)k * (L + 1) + 1] : 0.0);
    }
    FPFactors G;
    CHECK(build_fp_factors_coef(K, N, L, h.data(), sa.data(), str.data(), nullptr, mu, w, A, G, chunk));
    CHECK(!G.folded_sigma_s);
    return 0;
}

int main() {
    // K = 1, N = 2; ragged chunks; N from 2 to 64; both Laplacians
    const int cases[][6] = {{1, 2, 1, 1, 0, 0}, {7, 4, 3, 2, 3, 1}, {23, 8, 7, 3, 5, 0},
                            {40, 16, 15, 4, 0, 1}, {64, 32, 31, 2, 0, 0}, {33, 64, 20, 3, 6, 1},
                            {19, 6, 5, 2, 4, 0}};
    for (const auto &c : cases)
        if (one(c[0], c[1], c[2], c[3], c[4], c[5])) return 1;
    std::printf("setup driver ok\n");
    return 0;
}
