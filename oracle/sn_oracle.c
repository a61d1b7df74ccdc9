/*
 * Plain FP64 CPU oracle for slab S_N source iteration and Fokker-Planck
 * synthetic acceleration (Patel, Warsa, Prinja, "Acceleration of the S_N
 * equations with highly anisotropic scattering using the Fokker-Planck
 * equation").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the HIP library is
 * checked against.  It shares no code with the library; only tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Everything is written for clarity, not speed: explicit 2x2 and dense block
 * solves, straight loops, no blocking or fusion beyond what the equations
 * state.
 *
 * Layouts (slab of K cells, LD nodes nu = 0 (left) / 1 (right), N angles in
 * ascending mu order, moments l = 0..L):
 *   psi, q, source : [K][2][N]       phi : [K][2][L+1]
 *   sigma_s        : [K][L+1]        h, sigma_t : [K]
 *   psi_left[N/2]  : inflow at z0 for the positive cosines (ascending)
 *   psi_right[N/2] : inflow at z1 for the negative cosines (ascending)
 *
 * Readings where the paper is silent (its spatial scheme is only named):
 *   - LD = nodal linear-discontinuous Galerkin in z, upwind face fluxes,
 *     consistent mass matrix (h/6)[[2,1],[1,2]]; the same scheme discretises
 *     both the transport operator and the Fokker-Planck operator, with the
 *     removal term sigma_t replaced by sigma_a I - (sigma_tr/2) A.
 *   - Gauss-Legendre S_N quadrature, weights summing to 2.
 *   - WFD recursion uses nu = -2 with gamma_{1/2} = 0.
 *   - The correction equation has zero inflow on both faces.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define IDX3(k, nu, n, N) (((size_t)(k) * 2 + (nu)) * (size_t)(N) + (n))

/* ------------------------------------------------------------------------ */
/* Quadrature and Legendre tables                                            */
/* ------------------------------------------------------------------------ */

/* Gauss-Legendre nodes/weights by Newton's method on P_N; ascending mu. */
int or_gauss_legendre(int N, double *mu, double *w)
{
    if (N < 1) return -1;
    for (int i = 0; i < N; ++i) {
        /* descending initial guesses, stored ascending */
        double x = cos(M_PI * (i + 0.75) / (N + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int l = 1; l < N; ++l) {
                double p2 = ((2.0 * l + 1.0) * x * p1 - l * p0) / (l + 1.0);
                p0 = p1;
                p1 = p2;
            }
            double pN = (N == 1) ? x : p1;
            double pNm1 = (N == 1) ? 1.0 : p0;
            dp = N * (x * pN - pNm1) / (x * x - 1.0);
            double dx = pN / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        /* re-evaluate derivative at the converged root */
        {
            double p0 = 1.0, p1 = x;
            for (int l = 1; l < N; ++l) {
                double p2 = ((2.0 * l + 1.0) * x * p1 - l * p0) / (l + 1.0);
                p0 = p1;
                p1 = p2;
            }
            double pN = (N == 1) ? x : p1;
            double pNm1 = (N == 1) ? 1.0 : p0;
            dp = N * (x * pN - pNm1) / (x * x - 1.0);
        }
        mu[N - 1 - i] = x;
        w[N - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return 0;
}

/* P[l*N + n] = P_l(mu_n), l = 0..L (Bonnet recurrence). */
void or_legendre(int N, int L, const double *mu, double *P)
{
    for (int n = 0; n < N; ++n) {
        double x = mu[n];
        P[0 * N + n] = 1.0;
        if (L >= 1) P[1 * N + n] = x;
        for (int l = 1; l < L; ++l)
            P[(l + 1) * N + n] = ((2.0 * l + 1.0) * x * P[l * N + n] - l * P[(l - 1) * N + n]) / (l + 1.0);
    }
}

/* ------------------------------------------------------------------------ */
/* Angular Laplacians (Sec. 2.2)                                             */
/* ------------------------------------------------------------------------ */

/* WFD three-point Laplacian, eq:fp-wdd / eq:sph-weights / eq:w_wfd.
 * gamma_{n+1/2} = gamma_{n-1/2} - 2 mu_n w_n, gamma_{1/2} = 0. */
void or_wfd_matrix(int N, const double *mu, const double *w, double *W)
{
    double *gam = (double *)calloc((size_t)N + 1, sizeof(double));
    gam[0] = 0.0; /* gamma_{1/2} */
    for (int n = 0; n < N; ++n) gam[n + 1] = gam[n] - 2.0 * mu[n] * w[n];
    gam[N] = 0.0; /* exact value; removes the O(eps) round-off of the sum */
    memset(W, 0, sizeof(double) * (size_t)N * N);
    for (int n = 0; n < N; ++n) {
        double lo = 0.0, hi = 0.0;
        if (n > 0) lo = gam[n] / (mu[n] - mu[n - 1]);         /* gamma_{n-1/2} / (mu_n - mu_{n-1}) */
        if (n < N - 1) hi = gam[n + 1] / (mu[n + 1] - mu[n]); /* gamma_{n+1/2} / (mu_{n+1} - mu_n) */
        if (n > 0) W[n * N + n - 1] = lo / w[n];
        if (n < N - 1) W[n * N + n + 1] = hi / w[n];
        W[n * N + n] = -(lo + hi) / w[n];
    }
    free(gam);
}

/* Dense Gaussian elimination with partial pivoting, in place.
 * A is n x n row-major; piv[n]. Returns 0 or -1 if singular. */
static int lu_factor(int n, double *A, int *piv)
{
    for (int c = 0; c < n; ++c) {
        int p = c;
        double best = fabs(A[(size_t)c * n + c]);
        for (int r = c + 1; r < n; ++r) {
            double v = fabs(A[(size_t)r * n + c]);
            if (v > best) { best = v; p = r; }
        }
        piv[c] = p;
        if (best == 0.0) return -1;
        if (p != c)
            for (int j = 0; j < n; ++j) {
                double t = A[(size_t)c * n + j];
                A[(size_t)c * n + j] = A[(size_t)p * n + j];
                A[(size_t)p * n + j] = t;
            }
        double inv = 1.0 / A[(size_t)c * n + c];
        for (int r = c + 1; r < n; ++r) {
            double f = A[(size_t)r * n + c] * inv;
            A[(size_t)r * n + c] = f;
            for (int j = c + 1; j < n; ++j) A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
        }
    }
    return 0;
}

static void lu_solve(int n, const double *LU, const int *piv, double *b)
{
    /* lu_factor swaps whole rows, so P b first, then L y = P b, U x = y */
    for (int c = 0; c < n; ++c) {
        int p = piv[c];
        if (p != c) { double t = b[c]; b[c] = b[p]; b[p] = t; }
    }
    for (int c = 0; c < n; ++c)
        for (int r = c + 1; r < n; ++r) b[r] -= LU[(size_t)r * n + c] * b[c];
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int j = r + 1; j < n; ++j) s -= LU[(size_t)r * n + j] * b[j];
        b[r] = s / LU[(size_t)r * n + r];
    }
}

/* MPD Laplacian, eq:fp-mpd: F = V^{-1} diag(-l(l+1)) V with
 * V_{l,n} = P_l(mu_n) w_n, l = 0..N-1.  V^{-1} by numerical LU. */
int or_mpd_matrix(int N, const double *mu, const double *w, double *F)
{
    double *P = (double *)malloc(sizeof(double) * (size_t)N * N);
    double *V = (double *)malloc(sizeof(double) * (size_t)N * N);
    double *LV = (double *)malloc(sizeof(double) * (size_t)N * N);
    double *col = (double *)malloc(sizeof(double) * (size_t)N);
    int *piv = (int *)malloc(sizeof(int) * (size_t)N);
    or_legendre(N, N - 1, mu, P);
    for (int l = 0; l < N; ++l)
        for (int n = 0; n < N; ++n) V[l * N + n] = P[l * N + n] * w[n];
    /* LV = diag(-l(l+1)) V */
    for (int l = 0; l < N; ++l)
        for (int n = 0; n < N; ++n) LV[l * N + n] = -(double)l * (l + 1) * V[l * N + n];
    double *LU = P; /* reuse */
    memcpy(LU, V, sizeof(double) * (size_t)N * N);
    int rc = lu_factor(N, LU, piv);
    if (rc == 0) {
        /* F = V^{-1} LV, column by column */
        for (int j = 0; j < N; ++j) {
            for (int i = 0; i < N; ++i) col[i] = LV[i * N + j];
            lu_solve(N, LU, piv, col);
            for (int i = 0; i < N; ++i) F[i * N + j] = col[i];
        }
    }
    free(P); free(V); free(LV); free(col); free(piv);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Moments and scattering source (eq:treq, eq:phi-mom)                      */
/* ------------------------------------------------------------------------ */

/* phi_l = sum_n w_n P_l(mu_n) psi_n at every cell and LD node. */
void or_moments(int K, int N, int L, const double *mu, const double *w,
                const double *psi, double *phi)
{
    double *P = (double *)malloc(sizeof(double) * (size_t)(L + 1) * N);
    or_legendre(N, L, mu, P);
    for (int k = 0; k < K; ++k)
        for (int nu = 0; nu < 2; ++nu)
            for (int l = 0; l <= L; ++l) {
                double s = 0.0;
                for (int n = 0; n < N; ++n) s += w[n] * P[l * N + n] * psi[IDX3(k, nu, n, N)];
                phi[((size_t)k * 2 + nu) * (L + 1) + l] = s;
            }
    free(P);
}

/* q_n = sum_l (2l+1)/2 sigma_{s,l} P_l(mu_n) phi_l (+ q_ext_n). */
void or_scatter_source(int K, int N, int L, const double *mu,
                       const double *sigma_s, const double *phi,
                       const double *q_ext, double *q)
{
    double *P = (double *)malloc(sizeof(double) * (size_t)(L + 1) * N);
    or_legendre(N, L, mu, P);
    for (int k = 0; k < K; ++k)
        for (int nu = 0; nu < 2; ++nu)
            for (int n = 0; n < N; ++n) {
                double s = 0.0;
                for (int l = 0; l <= L; ++l)
                    s += 0.5 * (2.0 * l + 1.0) * sigma_s[(size_t)k * (L + 1) + l] * P[l * N + n] *
                         phi[((size_t)k * 2 + nu) * (L + 1) + l];
                if (q_ext) s += q_ext[IDX3(k, nu, n, N)];
                q[IDX3(k, nu, n, N)] = s;
            }
    free(P);
}

/* ------------------------------------------------------------------------ */
/* LD transport sweep (eq:trsi with L = mu d/dz + sigma_t)                   */
/* ------------------------------------------------------------------------ */

/* Cell equations of the LD scheme for one angle (tests b_L, b_R):
 *  mu>0: mu(psiL+psiR)/2 - mu psi_in + (h/6) s(2 psiL + psiR) = (h/6)(2 qL + qR)
 *        mu(psiR-psiL)/2            + (h/6) s(psiL + 2 psiR) = (h/6)(qL + 2 qR)
 *  mu<0: mu(psiR-psiL)/2            + (h/6) s(2 psiL + psiR) = (h/6)(2 qL + qR)
 *        mu psi_in - mu(psiL+psiR)/2 + (h/6) s(psiL + 2 psiR) = (h/6)(qL + 2 qR)
 * solved by Cramer's rule. */
static void ld_cell(double m, double h, double s, double qL, double qR,
                    double psi_in, double *psiL, double *psiR)
{
    double a11, a12, a21, a22, b1, b2;
    if (m > 0) {
        a11 = m / 2 + s * h / 3; a12 = m / 2 + s * h / 6;
        a21 = -m / 2 + s * h / 6; a22 = m / 2 + s * h / 3;
        b1 = h / 6 * (2 * qL + qR) + m * psi_in;
        b2 = h / 6 * (qL + 2 * qR);
    } else {
        a11 = -m / 2 + s * h / 3; a12 = m / 2 + s * h / 6;
        a21 = -m / 2 + s * h / 6; a22 = -m / 2 + s * h / 3;
        b1 = h / 6 * (2 * qL + qR);
        b2 = h / 6 * (qL + 2 * qR) - m * psi_in;
    }
    double det = a11 * a22 - a12 * a21;
    *psiL = (b1 * a22 - a12 * b2) / det;
    *psiR = (a11 * b2 - a21 * b1) / det;
}

/* psi = L_h^{-1} q with inflow psi_left (mu>0 at z0) and psi_right (mu<0 at
 * z1); NULL inflow = vacuum. */
void or_sweep(int K, int N, const double *mu, const double *h,
              const double *sigma_t, const double *q, const double *psi_left,
              const double *psi_right, double *psi)
{
    int half = N / 2;
#pragma omp parallel for schedule(static)
    for (int n = 0; n < N; ++n) {
        double m = mu[n];
        if (m > 0) {
            double in = psi_left ? psi_left[n - half] : 0.0;
            for (int k = 0; k < K; ++k) {
                double pl, pr;
                ld_cell(m, h[k], sigma_t[k], q[IDX3(k, 0, n, N)], q[IDX3(k, 1, n, N)], in, &pl, &pr);
                psi[IDX3(k, 0, n, N)] = pl;
                psi[IDX3(k, 1, n, N)] = pr;
                in = pr;
            }
        } else {
            double in = psi_right ? psi_right[n] : 0.0;
            for (int k = K - 1; k >= 0; --k) {
                double pl, pr;
                ld_cell(m, h[k], sigma_t[k], q[IDX3(k, 0, n, N)], q[IDX3(k, 1, n, N)], in, &pl, &pr);
                psi[IDX3(k, 0, n, N)] = pl;
                psi[IDX3(k, 1, n, N)] = pr;
                in = pl;
            }
        }
    }
}

/* Transpose of the zero-inflow sweep operator q -> psi.  Per angle the sweep
 * is psi = B^{-1} M q with B the block-bidiagonal LD matrix and M the
 * symmetric mass blocks, so the transpose is M B^{-T}: a sweep in the
 * opposite direction with transposed 2x2 cell blocks, then the mass blocks. */
void or_sweep_adjoint(int K, int N, const double *mu, const double *h,
                      const double *sigma_t, const double *y, double *x)
{
#pragma omp parallel for schedule(static)
    for (int n = 0; n < N; ++n) {
        double m = mu[n];
        double carry = 0.0; /* coupling value entering the current cell */
        int k0 = (m > 0) ? K - 1 : 0, dk = (m > 0) ? -1 : 1;
        for (int k = k0; k >= 0 && k < K; k += dk) {
            double s = sigma_t[k], hh = h[k];
            double a11, a12, a21, a22;
            if (m > 0) {
                a11 = m / 2 + s * hh / 3; a12 = m / 2 + s * hh / 6;
                a21 = -m / 2 + s * hh / 6; a22 = m / 2 + s * hh / 3;
            } else {
                a11 = -m / 2 + s * hh / 3; a12 = m / 2 + s * hh / 6;
                a21 = -m / 2 + s * hh / 6; a22 = -m / 2 + s * hh / 3;
            }
            /* B^T block = [[a11, a21], [a12, a22]] */
            double r1 = y[IDX3(k, 0, n, N)], r2 = y[IDX3(k, 1, n, N)];
            /* off-diagonal of B: mu>0 couples row L of cell k to psiR of k-1
             * with -mu; its transpose feeds row R of cell k-1 from z_L of k.
             * mu<0 couples row R of cell k to psiL of k+1 with +mu; transpose
             * feeds row L of k+1 from z_R of k. */
            if (m > 0) r2 -= carry; else r1 -= carry;
            double det = a11 * a22 - a12 * a21;
            double zL = (r1 * a22 - a21 * r2) / det;
            double zR = (a11 * r2 - a12 * r1) / det;
            carry = (m > 0) ? (-m) * zL : m * zR;
            x[IDX3(k, 0, n, N)] = hh / 6 * (2 * zL + zR);
            x[IDX3(k, 1, n, N)] = hh / 6 * (zL + 2 * zR);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Fokker-Planck correction operator (eq:fpop, eq:fp-mpd-oper, eq:wd-eq-oper)*/
/* ------------------------------------------------------------------------ */

/* LD x S_N discretisation of H dU/dz + (sigma_a I - sigma_tr/2 A) U = r with
 * zero inflow; unknowns per cell [U_L(0..N-1), U_R(0..N-1)].  The global
 * matrix is block tridiagonal; it is factored once by block Gaussian
 * elimination (block Thomas) with dense LU of each pivot block. */
typedef struct {
    int K, N;
    double *mu;   /* [N] */
    double *h;    /* [K] */
    double *LU;   /* [K][2N][2N] LU of the pivot blocks */
    int *piv;     /* [K][2N] */
} or_fp;

/* Cell block D_k (2N x 2N) for T = sigma_a I - (sigma_tr/2) A. */
static void fp_cell_block(int N, const double *mu, const double *A, double h,
                          double sa, double str, double *D)
{
    int n2 = 2 * N;
    memset(D, 0, sizeof(double) * (size_t)n2 * n2);
    for (int n = 0; n < N; ++n) {
        double m = mu[n], am = fabs(m);
        for (int j = 0; j < N; ++j) {
            double T = (n == j ? sa : 0.0) - 0.5 * str * A[n * N + j];
            D[(size_t)n * n2 + j] += h / 3 * T;           /* row L, col L */
            D[(size_t)n * n2 + N + j] += h / 6 * T;       /* row L, col R */
            D[(size_t)(N + n) * n2 + j] += h / 6 * T;     /* row R, col L */
            D[(size_t)(N + n) * n2 + N + j] += h / 3 * T; /* row R, col R */
        }
        /* streaming terms from the LD cell equations (see ld_cell) */
        D[(size_t)n * n2 + n] += am / 2;
        D[(size_t)n * n2 + N + n] += m / 2;
        D[(size_t)(N + n) * n2 + n] += -m / 2;
        D[(size_t)(N + n) * n2 + N + n] += am / 2;
    }
}

or_fp *or_fp_factor(int K, int N, const double *mu, const double *w,
                    const double *h, const double *sigma_a,
                    const double *sigma_tr, int scheme /*0 WFD, 1 MPD*/)
{
    int n2 = 2 * N;
    double *A = (double *)malloc(sizeof(double) * (size_t)N * N);
    if (scheme == 0) or_wfd_matrix(N, mu, w, A);
    else if (or_mpd_matrix(N, mu, w, A) != 0) { free(A); return NULL; }
    or_fp *f = (or_fp *)calloc(1, sizeof(or_fp));
    f->K = K; f->N = N;
    f->mu = (double *)malloc(sizeof(double) * N);
    memcpy(f->mu, mu, sizeof(double) * N);
    f->h = (double *)malloc(sizeof(double) * K);
    memcpy(f->h, h, sizeof(double) * K);
    f->LU = (double *)malloc(sizeof(double) * (size_t)K * n2 * n2);
    f->piv = (int *)malloc(sizeof(int) * (size_t)K * n2);
    double *col = (double *)malloc(sizeof(double) * n2);
    double *Sinv = (double *)malloc(sizeof(double) * (size_t)N * N); /* S^{-1}[R_n, R_m] */
    for (int k = 0; k < K; ++k) {
        double *S = f->LU + (size_t)k * n2 * n2;
        fp_cell_block(N, mu, A, h[k], sigma_a[k], sigma_tr[k], S);
        if (k > 0) {
            /* S_k = D_k - A_k S_{k-1}^{-1} C_{k-1}.  A_k: row L_n (mu_n>0)
             * <- -mu_n * U_R,n of cell k-1.  C_{k-1}: row R_m of k-1 (mu_m<0)
             * <- +mu_m * U_L,m of cell k.  Product entry [L_n, L_m] is
             * (-mu_n) * Sinv[R_n, R_m] * mu_m. */
            const double *Sp = f->LU + (size_t)(k - 1) * n2 * n2;
            const int *pp = f->piv + (size_t)(k - 1) * n2;
            for (int m = 0; m < N; ++m) {
                if (mu[m] >= 0) continue;
                for (int i = 0; i < n2; ++i) col[i] = 0.0;
                col[N + m] = 1.0;
                lu_solve(n2, Sp, pp, col);
                for (int n = 0; n < N; ++n) Sinv[n * N + m] = col[N + n];
            }
            for (int n = 0; n < N; ++n) {
                if (mu[n] <= 0) continue;
                for (int m = 0; m < N; ++m) {
                    if (mu[m] >= 0) continue;
                    S[(size_t)n * n2 + m] -= (-mu[n]) * Sinv[n * N + m] * mu[m];
                }
            }
        }
        if (lu_factor(n2, S, f->piv + (size_t)k * n2) != 0) {
            free(col); free(Sinv); free(A);
            free(f->mu); free(f->h); free(f->LU); free(f->piv); free(f);
            return NULL;
        }
    }
    free(col); free(Sinv); free(A);
    return f;
}

/* U = F_h^{-1} r.  r is the nodal source [K][2][N]; the right-hand side of
 * each cell is the consistent-mass projection (h/6)[2 1; 1 2] r. */
void or_fp_apply(const or_fp *f, const double *r, double *U)
{
    int K = f->K, N = f->N, n2 = 2 * N;
    const double *mu = f->mu;
    double *y = (double *)malloc(sizeof(double) * (size_t)K * n2);
    double *z = (double *)malloc(sizeof(double) * n2);
    for (int k = 0; k < K; ++k) {
        double hh = f->h[k];
        double *yk = y + (size_t)k * n2;
        for (int n = 0; n < N; ++n) {
            double rl = r[IDX3(k, 0, n, N)], rr = r[IDX3(k, 1, n, N)];
            yk[n] = hh / 6 * (2 * rl + rr);
            yk[N + n] = hh / 6 * (rl + 2 * rr);
        }
        if (k > 0) {
            /* y_k -= A_k S_{k-1}^{-1} y_{k-1} */
            memcpy(z, y + (size_t)(k - 1) * n2, sizeof(double) * n2);
            lu_solve(n2, f->LU + (size_t)(k - 1) * n2 * n2, f->piv + (size_t)(k - 1) * n2, z);
            for (int n = 0; n < N; ++n)
                if (mu[n] > 0) yk[n] -= (-mu[n]) * z[N + n];
        }
    }
    for (int k = K - 1; k >= 0; --k) {
        double *yk = y + (size_t)k * n2;
        memcpy(z, yk, sizeof(double) * n2);
        if (k < K - 1) {
            const double *xn = U + (size_t)(k + 1) * n2; /* U stored as [K][2N] = [K][2][N] */
            for (int n = 0; n < N; ++n)
                if (mu[n] < 0) z[N + n] -= mu[n] * xn[n];
        }
        lu_solve(n2, f->LU + (size_t)k * n2 * n2, f->piv + (size_t)k * n2, z);
        memcpy(U + (size_t)k * n2, z, sizeof(double) * n2);
    }
    free(y); free(z);
}

void or_fp_free(or_fp *f)
{
    if (!f) return;
    free(f->mu); free(f->h); free(f->LU); free(f->piv); free(f);
}

/* ------------------------------------------------------------------------ */
/* Solver drivers (eq:trsi; eq:predict, eq:correct, eq:iterate)              */
/* ------------------------------------------------------------------------ */

/* Wall-clock split of the last or_solve call (for the CPU baseline, timed
 * like the paper's Sec. 4: the Fokker-Planck factorisation is setup, the
 * iterations are the solve), and the OpenMP thread count of the sweep. */
static double g_last_factor_s = 0.0, g_last_iterate_s = 0.0;

void or_last_timing(double *factor_s, double *iterate_s)
{
    if (factor_s) *factor_s = g_last_factor_s;
    if (iterate_s) *iterate_s = g_last_iterate_s;
}

void or_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}

int or_get_threads(void)
{
    return omp_get_max_threads();
}

/* method 0 = source iteration, 1 = FPSA.  phi holds phi^0 on entry (the
 * caller zeroes it for the default initial guess) and the last iterate on
 * exit.  psi (nullable) receives the last angular flux (for FPSA the
 * corrected psi^{m+1/2} + U).  Returns 0 if converged, 1 if max_iter hit,
 * negative on failure.  The stopping test is max |phi^{m+1}_l - phi^m_l|
 * over all cells, nodes and l <= L. */
int or_solve(int K, int N, int L, const double *h, const double *sigma_t,
             const double *sigma_s, const double *psi_left,
             const double *psi_right, const double *q_ext, int method,
             int scheme, double tol, int max_iter, double *phi, double *psi_out,
             int *iters, double *resid_hist)
{
    size_t nq = (size_t)K * 2 * N, np = (size_t)K * 2 * (L + 1);
    double *mu = (double *)malloc(sizeof(double) * N);
    double *w = (double *)malloc(sizeof(double) * N);
    or_gauss_legendre(N, mu, w);
    double *q = (double *)malloc(sizeof(double) * nq);
    double *psi = (double *)malloc(sizeof(double) * nq);
    double *U = (double *)malloc(sizeof(double) * nq);
    double *phi_half = (double *)malloc(sizeof(double) * np);
    double *dphi = (double *)malloc(sizeof(double) * np);
    double *phiU = (double *)malloc(sizeof(double) * np);
    or_fp *fp = NULL;
    double t_start = omp_get_wtime();
    if (method == 1) {
        double *sa = (double *)malloc(sizeof(double) * K);
        double *str = (double *)malloc(sizeof(double) * K);
        for (int k = 0; k < K; ++k) {
            double s0 = sigma_s[(size_t)k * (L + 1)];
            double s1 = L >= 1 ? sigma_s[(size_t)k * (L + 1) + 1] : 0.0;
            sa[k] = sigma_t[k] - s0;
            str[k] = s0 - s1;
        }
        fp = or_fp_factor(K, N, mu, w, h, sa, str, scheme);
        free(sa); free(str);
        if (!fp) { free(mu); free(w); free(q); free(psi); free(U); free(phi_half); free(dphi); free(phiU); return -2; }
    }
    double t_iter = omp_get_wtime();
    g_last_factor_s = t_iter - t_start;
    int status = 1, m;
    for (m = 1; m <= max_iter; ++m) {
        /* predict: L psi^{m+1/2} = S psi^m + q */
        or_scatter_source(K, N, L, mu, sigma_s, phi, q_ext, q);
        or_sweep(K, N, mu, h, sigma_t, q, psi_left, psi_right, psi);
        or_moments(K, N, L, mu, w, psi, phi_half);
        if (method == 1) {
            /* correct: psi^{m+1} = psi^{m+1/2} + F^{-1} S (psi^{m+1/2} - psi^m) */
            for (size_t i = 0; i < np; ++i) dphi[i] = phi_half[i] - phi[i];
            or_scatter_source(K, N, L, mu, sigma_s, dphi, NULL, q);
            or_fp_apply(fp, q, U);
            for (size_t i = 0; i < nq; ++i) psi[i] += U[i];
            or_moments(K, N, L, mu, w, U, phiU);
            for (size_t i = 0; i < np; ++i) phi_half[i] += phiU[i];
        }
        double diff = 0.0;
        for (size_t i = 0; i < np; ++i) {
            double d = fabs(phi_half[i] - phi[i]);
            if (d > diff || isnan(d)) diff = d;
        }
        memcpy(phi, phi_half, sizeof(double) * np);
        if (resid_hist) resid_hist[m - 1] = diff;
        if (diff <= tol) { status = 0; break; }
        if (isnan(diff)) { status = -3; break; }
    }
    g_last_iterate_s = omp_get_wtime() - t_iter;
    if (iters) *iters = (m > max_iter) ? max_iter : m;
    if (psi_out) memcpy(psi_out, psi, sizeof(double) * nq);
    or_fp_free(fp);
    free(mu); free(w); free(q); free(psi); free(U); free(phi_half); free(dphi); free(phiU);
    return status;
}

/* One FPSA correction as a standalone map:
 * phi_new = phi_half + D F_h^{-1} M Sigma_s (phi_half - phi_old). */
int or_fpsa_correct(int K, int N, int L, const double *h, const double *sigma_t,
                    const double *sigma_s, int scheme, const double *phi_half,
                    const double *phi_old, double *phi_new, double *U_out)
{
    size_t nq = (size_t)K * 2 * N, np = (size_t)K * 2 * (L + 1);
    double *mu = (double *)malloc(sizeof(double) * N);
    double *w = (double *)malloc(sizeof(double) * N);
    or_gauss_legendre(N, mu, w);
    double *sa = (double *)malloc(sizeof(double) * K);
    double *str = (double *)malloc(sizeof(double) * K);
    for (int k = 0; k < K; ++k) {
        double s0 = sigma_s[(size_t)k * (L + 1)];
        double s1 = L >= 1 ? sigma_s[(size_t)k * (L + 1) + 1] : 0.0;
        sa[k] = sigma_t[k] - s0;
        str[k] = s0 - s1;
    }
    or_fp *fp = or_fp_factor(K, N, mu, w, h, sa, str, scheme);
    free(sa); free(str);
    if (!fp) { free(mu); free(w); return -2; }
    double *dphi = (double *)malloc(sizeof(double) * np);
    double *r = (double *)malloc(sizeof(double) * nq);
    double *U = (double *)malloc(sizeof(double) * nq);
    for (size_t i = 0; i < np; ++i) dphi[i] = phi_half[i] - phi_old[i];
    or_scatter_source(K, N, L, mu, sigma_s, dphi, NULL, r);
    or_fp_apply(fp, r, U);
    or_moments(K, N, L, mu, w, U, phi_new);
    for (size_t i = 0; i < np; ++i) phi_new[i] += phi_half[i];
    if (U_out) memcpy(U_out, U, sizeof(double) * nq);
    or_fp_free(fp);
    free(mu); free(w); free(dphi); free(r); free(U);
    return 0;
}

/* Standalone F_h^{-1} r for tests. */
int or_fp_solve(int K, int N, const double *h, const double *sigma_a,
                const double *sigma_tr, int scheme, const double *r, double *U)
{
    double *mu = (double *)malloc(sizeof(double) * N);
    double *w = (double *)malloc(sizeof(double) * N);
    or_gauss_legendre(N, mu, w);
    or_fp *fp = or_fp_factor(K, N, mu, w, h, sigma_a, sigma_tr, scheme);
    if (!fp) { free(mu); free(w); return -2; }
    or_fp_apply(fp, r, U);
    or_fp_free(fp);
    free(mu); free(w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Adjoint and response gradient                                             */
/* ------------------------------------------------------------------------ */

/* The discrete transport solution is the fixed point psi = Linv(S psi + q)
 * of or_sweep (Linv, with the problem's inflow) and S = M Sigma D
 * (or_scatter_source of or_moments).  For a response J = <c, psi> (plain
 * dot product over [K][2][N]) the adjoint lambda is the fixed point of the
 * transposed map, lambda = Linv^T (S^T lambda + c) with Linv^T =
 * or_sweep_adjoint (zero inflow) and S^T = D^T Sigma M^T; then
 * J = <lambda, q + inflow response>, and a parameter p of the operator
 * moves J by dJ/dp = -<lambda, (d(Linv^-1 - S)/dp) psi>. */

/* x = S^T lambda: (M^T lambda)_l = sum_n (2l+1)/2 P_l(mu_n) lambda_n, times
 * sigma_{s,l}, then x_n = sum_l w_n P_l(mu_n) (.)_l. */
static void scatter_transposed(int K, int N, int L, const double *mu, const double *w,
                               const double *sigma_s, const double *lambda, double *x)
{
    double *P = (double *)malloc(sizeof(double) * (size_t)(L + 1) * N);
    double *t = (double *)malloc(sizeof(double) * (size_t)(L + 1));
    or_legendre(N, L, mu, P);
    for (int k = 0; k < K; ++k)
        for (int nu = 0; nu < 2; ++nu) {
            for (int l = 0; l <= L; ++l) {
                double s = 0.0;
                for (int n = 0; n < N; ++n)
                    s += 0.5 * (2.0 * l + 1.0) * P[l * N + n] * lambda[IDX3(k, nu, n, N)];
                t[l] = s * sigma_s[(size_t)k * (L + 1) + l];
            }
            for (int n = 0; n < N; ++n) {
                double s = 0.0;
                for (int l = 0; l <= L; ++l) s += w[n] * P[l * N + n] * t[l];
                x[IDX3(k, nu, n, N)] = s;
            }
        }
    free(P); free(t);
}

/* Adjoint source iteration from the lambda given on entry until
 * max |lambda^{m+1} - lambda^m| <= tol.  Returns 0 if converged, 1 at the
 * iteration limit. */
int or_adjoint_solve(int K, int N, int L, const double *h, const double *sigma_t,
                     const double *sigma_s, const double *c, double tol, int max_iter,
                     double *lambda, int *iters)
{
    size_t nq = (size_t)K * 2 * N;
    double *mu = (double *)malloc(sizeof(double) * N);
    double *w = (double *)malloc(sizeof(double) * N);
    double *x = (double *)malloc(sizeof(double) * nq);
    double *nxt = (double *)malloc(sizeof(double) * nq);
    or_gauss_legendre(N, mu, w);
    int status = 1, m;
    for (m = 1; m <= max_iter; ++m) {
        scatter_transposed(K, N, L, mu, w, sigma_s, lambda, x);
        for (size_t i = 0; i < nq; ++i) x[i] += c[i];
        or_sweep_adjoint(K, N, mu, h, sigma_t, x, nxt);
        double diff = 0.0;
        for (size_t i = 0; i < nq; ++i) {
            double d = fabs(nxt[i] - lambda[i]);
            if (d > diff) diff = d;
        }
        memcpy(lambda, nxt, sizeof(double) * nq);
        if (diff <= tol) { status = 0; break; }
    }
    if (iters) *iters = (m > max_iter) ? max_iter : m;
    free(mu); free(w); free(x); free(nxt);
    return status;
}

/* Gradient of J = <c, psi> from the converged psi and lambda.  Linv^-1 =
 * Mass^-1 B with B holding sigma_t(k) Mass_k for every angle of cell k, so
 * d(Linv^-1)/dsigma_t(k) is the identity on cell k and
 *   dJ/dsigma_t(k)     = - sum_{nu,n} lambda(k,nu,n) psi(k,nu,n);
 * S depends on sigma_{s,l}(k) through M e_l e_l^T D on cell k, so
 *   dJ/dsigma_{s,l}(k) = sum_nu (M^T lambda)(k,nu,l) (D psi)(k,nu,l). */
void or_response_gradient(int K, int N, int L, const double *psi, const double *lambda,
                          double *g_sigma_t, double *g_sigma_s)
{
    double *mu = (double *)malloc(sizeof(double) * N);
    double *w = (double *)malloc(sizeof(double) * N);
    double *P = (double *)malloc(sizeof(double) * (size_t)(L + 1) * N);
    or_gauss_legendre(N, mu, w);
    or_legendre(N, L, mu, P);
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int nu = 0; nu < 2; ++nu)
            for (int n = 0; n < N; ++n) s += lambda[IDX3(k, nu, n, N)] * psi[IDX3(k, nu, n, N)];
        g_sigma_t[k] = -s;
        for (int l = 0; l <= L; ++l) {
            double g = 0.0;
            for (int nu = 0; nu < 2; ++nu) {
                double ml = 0.0, dl = 0.0;
                for (int n = 0; n < N; ++n) {
                    ml += 0.5 * (2.0 * l + 1.0) * P[l * N + n] * lambda[IDX3(k, nu, n, N)];
                    dl += w[n] * P[l * N + n] * psi[IDX3(k, nu, n, N)];
                }
                g += ml * dl;
            }
            g_sigma_s[(size_t)k * (L + 1) + l] = g;
        }
    }
    free(mu); free(w); free(P);
}
