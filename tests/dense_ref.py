"""Brute-force dense assembly of the LD x S_N slab operators (test tool).

Builds the full (2 K N) x (2 K N) matrix of the linear-discontinuous,
upwind S_N system with a per-cell nodal removal matrix T_k and solves it with
numpy.linalg.solve.  Independent of the oracle (which sweeps and uses block
elimination) and of the HIP library.

  transport:  T_k = sigma_t I - M diag(sigma_s) V      ->  L_h - S_h
  Fokker-Planck: T_k = sigma_a I - (sigma_tr / 2) A    ->  F_h
Unknown ordering: index(k, nu, n) = (k*2 + nu)*N + n.
"""
from __future__ import annotations

import numpy as np


def quadrature(N):
    mu, w = np.polynomial.legendre.leggauss(N)
    P = np.array([np.polynomial.legendre.legval(mu, np.eye(N)[l]) for l in range(N)])
    return mu, w, P


def assemble(mu, h, T, psi_left=None, psi_right=None, q=None):
    """Return (A, b) of the LD system sum_k cell equations.

    Cell equations (test functions b_L, b_R; mass (h/6)[[2,1],[1,2]]):
      mu>0: mu(uL+uR)/2 - mu u_in + (h/6)(2 TuL + TuR) = (h/6)(2 qL + qR)
            mu(uR-uL)/2 +            (h/6)(TuL + 2 TuR) = (h/6)(qL + 2 qR)
      mu<0: mu(uR-uL)/2 +            (h/6)(2 TuL + TuR) = (h/6)(2 qL + qR)
            mu u_in - mu(uL+uR)/2  + (h/6)(TuL + 2 TuR) = (h/6)(qL + 2 qR)
    """
    K = len(h)
    N = mu.size
    n_unk = 2 * K * N
    A = np.zeros((n_unk, n_unk))
    b = np.zeros(n_unk)

    def ix(k, nu, n):
        return (k * 2 + nu) * N + n

    for k in range(K):
        hk = h[k]
        Tk = T[k]
        for n in range(N):
            m = mu[n]
            rL, rR = ix(k, 0, n), ix(k, 1, n)
            # removal / mass terms
            for j in range(N):
                A[rL, ix(k, 0, j)] += hk / 6 * 2 * Tk[n, j]
                A[rL, ix(k, 1, j)] += hk / 6 * Tk[n, j]
                A[rR, ix(k, 0, j)] += hk / 6 * Tk[n, j]
                A[rR, ix(k, 1, j)] += hk / 6 * 2 * Tk[n, j]
            if m > 0:
                A[rL, ix(k, 0, n)] += m / 2
                A[rL, ix(k, 1, n)] += m / 2
                A[rR, ix(k, 0, n)] += -m / 2
                A[rR, ix(k, 1, n)] += m / 2
                if k > 0:
                    A[rL, ix(k - 1, 1, n)] += -m
                elif psi_left is not None:
                    b[rL] += m * psi_left[n - N // 2]
            else:
                A[rL, ix(k, 0, n)] += -m / 2
                A[rL, ix(k, 1, n)] += m / 2
                A[rR, ix(k, 0, n)] += -m / 2
                A[rR, ix(k, 1, n)] += -m / 2
                if k < K - 1:
                    A[rR, ix(k + 1, 0, n)] += m
                elif psi_right is not None:
                    b[rR] += -m * psi_right[n]
            if q is not None:
                b[rL] += hk / 6 * (2 * q[k, 0, n] + q[k, 1, n])
                b[rR] += hk / 6 * (q[k, 0, n] + 2 * q[k, 1, n])
    return A, b


def transport_solution(prob):
    """Direct solve of (L_h - S_h) psi = q + inflow; returns psi [K,2,N]."""
    N, L = prob.N, prob.L
    mu, w, P = quadrature(N)
    V = P[: L + 1] * w[None, :]                              # (L+1) x N
    M = (P[: L + 1].T * (2 * np.arange(L + 1) + 1) / 2.0)   # N x (L+1)
    T = [prob.sigma_t[k] * np.eye(N) - M @ np.diag(prob.sigma_s[k]) @ V for k in range(prob.K)]
    A, b = assemble(mu, prob.h, T, prob.psi_left, prob.psi_right, prob.q)
    return np.linalg.solve(A, b).reshape(prob.K, 2, N)


def fp_operator_solve(r, h, sigma_a, sigma_tr, A_ang):
    """Direct solve of F_h U = r with zero inflow; A_ang is W or F (N x N)."""
    K, _, N = r.shape
    mu, _, _ = quadrature(N)
    T = [sigma_a[k] * np.eye(N) - 0.5 * sigma_tr[k] * A_ang for k in range(K)]
    A, b = assemble(mu, h, T, None, None, r)
    return np.linalg.solve(A, b).reshape(K, 2, N)


def moments(psi, L):
    N = psi.shape[2]
    mu, w, P = quadrature(N)
    V = P[: L + 1] * w[None, :]
    return np.einsum("ln,kvn->kvl", V, psi)
