"""Angularly-discrete Fourier analysis of SI and FPSA (test tool).

Independent of both the oracle and the HIP library: NumPy's Gauss-Legendre
rule and Legendre evaluation, complex dense algebra.  Follows the paper's
Sec. 3.3 (eq:fpsa6, eq:fpsa7 for the predictor; eq:fper and eq:matdef3mpd for
the correction):

  predictor   A_hat = Y^{-1} Z,  Y_{ln} = P_l(mu_n) w_n (i lam sigma_t mu_n + sigma_t),
                                 Z_{ln} = sigma_{s,l} P_l(mu_n) w_n
  correction  B^{-1} C D with C_{ln} = sigma_{s,l} P_l(mu_n) w_n, D = I - A_hat,
              B = V (i lam sigma_t H + sigma_a I - (sigma_tr/2) A)
              (A = W for WFD, A = V^{-1} diag(-l(l+1)) V for MPD; the MPD
              form is the paper's B-tilde written out, the WFD form is the
              same expression with the three-point matrix, which is how the
              garbled B-hat of the WFD subsection is read)
  iteration   I_M = A_hat - B^{-1} C D,   rho = max_lam spectral radius.
"""
from __future__ import annotations

import numpy as np


def quadrature(N):
    mu, w = np.polynomial.legendre.leggauss(N)
    P = np.array([np.polynomial.legendre.legval(mu, np.eye(N)[l]) for l in range(N)])
    return mu, w, P


def wfd(mu, w):
    N = mu.size
    gam = np.concatenate([[0.0], -2.0 * np.cumsum(mu * w)])
    gam[-1] = 0.0
    W = np.zeros((N, N))
    for n in range(N):
        lo = gam[n] / (mu[n] - mu[n - 1]) if n > 0 else 0.0
        hi = gam[n + 1] / (mu[n + 1] - mu[n]) if n < N - 1 else 0.0
        if n > 0:
            W[n, n - 1] = lo / w[n]
        if n < N - 1:
            W[n, n + 1] = hi / w[n]
        W[n, n] = -(lo + hi) / w[n]
    return W


def mpd(V):
    N = V.shape[0]
    lam = -np.arange(N) * (np.arange(N) + 1.0)
    return np.linalg.solve(V, lam[:, None] * V)


def iteration_matrix(lam, sigma_s, sigma_t=1.0, scheme="wfd", N=None, accel=True):
    N = N or len(sigma_s)
    mu, w, P = quadrature(N)
    V = P * w[None, :]
    ss = np.zeros(N)
    ss[: min(N, len(sigma_s))] = sigma_s[:N]
    sa = sigma_t - ss[0]
    st = ss[0] - (ss[1] if N > 1 else 0.0)
    Y = V * (1j * lam * sigma_t * mu + sigma_t)[None, :]
    Z = ss[:, None] * V
    A_hat = np.linalg.solve(Y, Z)
    if not accel:
        return A_hat
    Aang = wfd(mu, w) if scheme == "wfd" else mpd(V)
    B = V @ (np.diag(1j * lam * sigma_t * mu + sa) - 0.5 * st * Aang)
    C = Z
    D = np.eye(N) - A_hat
    return A_hat - np.linalg.solve(B, C @ D)


def spectral_radius(sigma_s, sigma_t=1.0, scheme="wfd", N=None, accel=True,
                    lams=None):
    if lams is None:
        lams = np.concatenate([[0.0], np.logspace(-4, 3, 1401)])
    best = 0.0
    for lam in lams:
        ev = np.linalg.eigvals(iteration_matrix(lam, sigma_s, sigma_t, scheme, N, accel))
        best = max(best, np.abs(ev).max())
    return best
