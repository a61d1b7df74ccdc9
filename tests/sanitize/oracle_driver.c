/* Drives the FP64 oracle (oracle/sn_oracle.c) through every exported
 * function on small slabs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: any out-of-bounds access, use after free,
 * leak or undefined operation aborts the run.  Exit status 0 when every
 * call returned its success code. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int or_gauss_legendre(int N, double *mu, double *w);
void or_legendre(int N, int L, const double *mu, double *P);
void or_wfd_matrix(int N, const double *mu, const double *w, double *W);
int or_mpd_matrix(int N, const double *mu, const double *w, double *F);
void or_moments(int K, int N, int L, const double *mu, const double *w, const double *psi, double *phi);
void or_scatter_source(int K, int N, int L, const double *mu, const double *sigma_s, const double *phi,
                       const double *q_ext, double *q);
void or_sweep(int K, int N, const double *mu, const double *h, const double *sigma_t, const double *q,
              const double *psi_left, const double *psi_right, double *psi);
void or_sweep_adjoint(int K, int N, const double *mu, const double *h, const double *sigma_t, const double *y,
                      double *x);
int or_solve(int K, int N, int L, const double *h, const double *sigma_t, const double *sigma_s,
             const double *psi_left, const double *psi_right, const double *q_ext, int method, int scheme,
             double tol, int max_iter, double *phi, double *psi_out, int *iters, double *resid_hist);
int or_fpsa_correct(int K, int N, int L, const double *h, const double *sigma_t, const double *sigma_s, int scheme,
                    const double *phi_half, const double *phi_old, double *phi_new, double *U_out);
int or_fp_solve(int K, int N, const double *h, const double *sigma_a, const double *sigma_tr, int scheme,
                const double *r, double *U);
int or_adjoint_solve(int K, int N, int L, const double *h, const double *sigma_t, const double *sigma_s,
                     const double *c, double tol, int max_iter, double *lam, int *iters);
void or_response_gradient(int K, int N, int L, const double *psi, const double *lambda, double *g_sigma_t,
                          double *g_sigma_s);
void or_last_timing(double *factor_s, double *iterate_s);
void or_set_threads(int n);
int or_get_threads(void);

static double *arr(size_t n, double v)
{
    double *a = (double *)malloc(sizeof(double) * (n ? n : 1));
    for (size_t i = 0; i < n; ++i) a[i] = v;
    return a;
}

static double urand(unsigned *s)
{
    *s = *s * 1103515245u + 12345u;
    return ((*s >> 8) & 0xffff) / 65536.0;
}

#define CHECK(cond)                                                      \
    do {                                                                 \
        if (!(cond)) {                                                   \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                    \
        }                                                                \
    } while (0)

static int one_slab(int K, int N, int L, unsigned seed)
{
    unsigned s = seed;
    size_t nq = (size_t)K * 2 * N, np = (size_t)K * 2 * (L + 1);
    double *mu = arr(N, 0), *w = arr(N, 0), *P = arr((size_t)(L + 1) * N, 0), *A = arr((size_t)N * N, 0);
    CHECK(or_gauss_legendre(N, mu, w) == 0);
    or_legendre(N, L, mu, P);
    or_wfd_matrix(N, mu, w, A);
    CHECK(or_mpd_matrix(N, mu, w, A) == 0);
    double *h = arr(K, 0.1), *st = arr(K, 0), *ss = arr((size_t)K * (L + 1), 0);
    for (int k = 0; k < K; ++k) {
        st[k] = 0.5 + 2.0 * urand(&s);
        double c = 0.5 + 0.4 * urand(&s), g = 0.9;
        double gl = 1.0;
        for (int l = 0; l <= L; ++l, gl *= g) ss[(size_t)k * (L + 1) + l] = c * st[k] * gl;
    }
    double *pl = arr(N / 2, 1.0), *pr = arr(N / 2, 0.5), *q = arr(nq, 1.0), *psi = arr(nq, 0), *phi = arr(np, 0);
    double *hist = arr(2000, 0), *qq = arr(nq, 0), *x = arr(nq, 0), *U = arr(nq, 0), *ph2 = arr(np, 0);
    or_moments(K, N, L, mu, w, q, phi);
    or_scatter_source(K, N, L, mu, ss, phi, q, qq);
    or_sweep(K, N, mu, h, st, qq, pl, pr, psi);
    or_sweep_adjoint(K, N, mu, h, st, psi, x);
    for (int method = 0; method < 2; ++method)
        for (int scheme = 0; scheme < 2; ++scheme) {
            int it = 0;
            memset(phi, 0, sizeof(double) * np);
            CHECK(or_solve(K, N, L, h, st, ss, pl, pr, q, method, scheme, 1e-10, 2000, phi, psi, &it, hist) == 0);
            CHECK(it > 0);
        }
    double f_s = -1, i_s = -1;
    or_last_timing(&f_s, &i_s);
    CHECK(f_s >= 0 && i_s >= 0);
    for (size_t i = 0; i < np; ++i) ph2[i] = phi[i] * (1.0 + 0.01 * urand(&s));
    CHECK(or_fpsa_correct(K, N, L, h, st, ss, 0, ph2, phi, x, U) == 0);
    double *sa = arr(K, 0.2), *str = arr(K, 0.3);
    CHECK(or_fp_solve(K, N, h, sa, str, 1, q, U) == 0);
    double *c = arr(nq, 0), *lam = arr(nq, 0), *gt = arr(K, 0), *gs = arr((size_t)K * (L + 1), 0);
    for (int n = N / 2; n < N; ++n) c[((size_t)(K - 1) * 2 + 1) * N + n] = w[n] * mu[n];
    int ia = 0;
    CHECK(or_adjoint_solve(K, N, L, h, st, ss, c, 1e-12, 5000, lam, &ia) == 0);
    or_response_gradient(K, N, L, psi, lam, gt, gs);
    free(mu); free(w); free(P); free(A); free(h); free(st); free(ss); free(pl); free(pr); free(q); free(psi);
    free(phi); free(hist); free(qq); free(x); free(U); free(ph2); free(sa); free(str); free(c); free(lam);
    free(gt); free(gs);
    return 0;
}

int main(void)
{
    or_set_threads(2);
    if (or_get_threads() < 1) return 1;
    /* K = 1 and N = 2 (the smallest slab), odd cell counts, L < N - 1 */
    const int cases[][3] = {{1, 2, 1}, {7, 4, 3}, {13, 8, 5}, {9, 16, 15}, {5, 6, 2}};
    for (size_t i = 0; i < sizeof(cases) / sizeof(cases[0]); ++i)
        if (one_slab(cases[i][0], cases[i][1], cases[i][2], 17u + (unsigned)i)) return 1;
    printf("oracle driver ok\n");
    return 0;
}
