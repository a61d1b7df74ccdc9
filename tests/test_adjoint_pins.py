"""Pins of the adjoint and the response gradient (no GPU).

The oracle's adjoint is the transposed fixed point of the discrete transport
problem, iterated with its transposed sweep; its gradient formula is pinned
here against central finite differences of the oracle's own forward solves
and against a dense transposed solve.  The identity the HIP adjoint rests on
(A^T = X A X^{-1}, X = diag(w) R with R the angle reflection) is checked on
dense matrices for the transport and both Fokker-Planck operators, and the
reflected forward solve it implies is checked against the oracle's adjoint.
"""
import copy

import numpy as np
import pytest

import dense_ref
import oracle
import sn_workloads as sw


def _prob(seed=3, K=12, N=8, h=0.4, inflow=False):
    p = sw.cellwise_hg_slab(seed, K=K, N=N, h=h)
    if inflow:
        rng = np.random.Generator(np.random.PCG64(seed + 100))
        p.psi_left = rng.uniform(0.0, 1.0, N // 2)
        p.psi_right = rng.uniform(0.0, 1.0, N // 2)
    return p


def _J(p, sigma_t, sigma_s, c):
    q = copy.deepcopy(p)
    q.sigma_t, q.sigma_s = sigma_t, sigma_s
    r = oracle.solve(q, "si", tol=1e-15, max_iter=100000)
    return float((c * r["psi"]).sum())


def _grad(p, c):
    r = oracle.solve(p, "si", tol=1e-15, max_iter=100000)
    a = oracle.adjoint_solve(p, c, tol=1e-15)
    assert a["status"] == 0
    gt, gs = oracle.response_gradient(p, r["psi"], a["lam"])
    return r, a, gt, gs


@pytest.mark.parametrize("inflow", [False, True])
def test_oracle_gradient_matches_central_differences(inflow):
    """Every dJ/dsigma_t(k) and a spread of dJ/dsigma_{s,l}(k) against
    (J(p + d) - J(p - d)) / 2d with the oracle's forward solve."""
    p = _prob(inflow=inflow)
    c = oracle.exit_current_weights(p.K, p.N)
    _, _, gt, gs = _grad(p, c)
    for k in range(p.K):
        d = 1e-6 * p.sigma_t[k]
        st = p.sigma_t.copy()
        st[k] += d
        jp = _J(p, st, p.sigma_s, c)
        st[k] -= 2 * d
        jm = _J(p, st, p.sigma_s, c)
        fd = (jp - jm) / (2 * d)
        assert abs(fd - gt[k]) <= 1e-6 * abs(fd), (k, fd, gt[k])
    for k, l in [(0, 0), (3, 1), (6, 4), (11, 7), (5, 2)]:
        d = 1e-6 * max(abs(p.sigma_s[k, l]), 1e-3)
        ss = p.sigma_s.copy()
        ss[k, l] += d
        jp = _J(p, p.sigma_t, ss, c)
        ss[k, l] -= 2 * d
        jm = _J(p, p.sigma_t, ss, c)
        fd = (jp - jm) / (2 * d)
        assert abs(fd - gs[k, l]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gs).max()), (k, l, fd, gs[k, l])


def _dense_transport(p):
    mu, w, P = dense_ref.quadrature(p.N)
    L = p.L
    V = P[: L + 1] * w[None, :]
    M = P[: L + 1].T * (2 * np.arange(L + 1) + 1) / 2.0
    T = [p.sigma_t[k] * np.eye(p.N) - M @ np.diag(p.sigma_s[k]) @ V for k in range(p.K)]
    A, b = dense_ref.assemble(mu, p.h, T, p.psi_left, p.psi_right, p.q)
    return A, b, w


def _reflection(K, N, w):
    n = 2 * K * N
    X = np.zeros((n, n))
    for k in range(K):
        for nu in range(2):
            for j in range(N):
                X[(k * 2 + nu) * N + j, (k * 2 + nu) * N + N - 1 - j] = w[j]
    return X


def _mass(K, N, h):
    n = 2 * K * N
    Ms = np.zeros((n, n))
    for k in range(K):
        for j in range(N):
            i0, i1 = (k * 2) * N + j, (k * 2 + 1) * N + j
            Ms[i0, i0] = Ms[i1, i1] = h[k] / 3.0
            Ms[i0, i1] = Ms[i1, i0] = h[k] / 6.0
    return Ms


def test_oracle_adjoint_matches_dense_transposed_solve():
    """A psi = Mass q + b (dense, unnormalised) gives J = <c, psi>; the
    oracle's lambda (for the sweep-normalised operator) is Mass A^{-T} c,
    and J = <A^{-T} c, Mass q + b> (reciprocity)."""
    p = _prob(seed=5, K=6, N=8, inflow=True)
    c = oracle.exit_current_weights(p.K, p.N)
    A, b, _ = _dense_transport(p)
    lam_dense = np.linalg.solve(A.T, c.ravel())
    Ms = _mass(p.K, p.N, p.h)
    a = oracle.adjoint_solve(p, c, tol=1e-15)
    assert np.abs(a["lam"].ravel() - Ms @ lam_dense).max() <= 1e-12 * np.abs(Ms @ lam_dense).max()
    psi = np.linalg.solve(A, b)
    assert abs(c.ravel() @ psi - lam_dense @ b) <= 1e-13 * abs(c.ravel() @ psi)


@pytest.mark.parametrize("scheme", [None, "wfd", "mpd"])
def test_operator_transpose_is_a_reflection(scheme):
    """A^T = X A X^{-1} with X = diag(w_n) R (R: mu_n -> -mu_n) for the LD x
    S_N transport operator with Legendre scattering and for the
    Fokker-Planck operators with the WFD and MPD Laplacians."""
    p = _prob(seed=9, K=5, N=8)
    mu, w, _ = dense_ref.quadrature(p.N)
    if scheme is None:
        A, _, _ = _dense_transport(p)
    else:
        Aang = oracle.wfd_matrix(p.N) if scheme == "wfd" else oracle.mpd_matrix(p.N)
        sa = p.sigma_t - p.sigma_s[:, 0]
        st = p.sigma_s[:, 0] - p.sigma_s[:, 1]
        A, _ = dense_ref.assemble(mu, p.h, [sa[k] * np.eye(p.N) - 0.5 * st[k] * Aang for k in range(p.K)])
    X = _reflection(p.K, p.N, w)
    assert np.abs(A.T - X @ A @ np.linalg.inv(X)).max() <= 1e-14 * np.abs(A).max()


def test_reflected_forward_solve_is_the_adjoint():
    """The adjoint from a forward solve: y solves the forward problem with
    zero inflow and nodal source Mass^{-1} R W^{-1} c; then lambda' = W R y
    and lambda = Mass lambda' equals the oracle's transposed iteration."""
    p = _prob(seed=11, K=10, N=8, inflow=True)
    c = oracle.exit_current_weights(p.K, p.N)
    mu, w = oracle.gauss_legendre(p.N)
    ct = c[:, :, ::-1] / w[None, None, :]
    qy = np.empty_like(ct)
    for k in range(p.K):
        f = 2.0 / p.h[k]
        qy[k, 0] = f * (2 * ct[k, 0] - ct[k, 1])
        qy[k, 1] = f * (2 * ct[k, 1] - ct[k, 0])
    y = oracle.solve(p, "si", tol=1e-15, q_ext=qy, bc=False)["psi"]
    lam1 = w[None, None, :] * y[:, :, ::-1]
    lam = np.empty_like(lam1)
    for k in range(p.K):
        lam[k, 0] = p.h[k] / 6 * (2 * lam1[k, 0] + lam1[k, 1])
        lam[k, 1] = p.h[k] / 6 * (lam1[k, 0] + 2 * lam1[k, 1])
    a = oracle.adjoint_solve(p, c, tol=1e-15)
    assert np.abs(lam - a["lam"]).max() <= 1e-12 * np.abs(a["lam"]).max()


def test_hg_parameter_gradients_by_chain_rule():
    """dJ/dc and dJ/dg of a cell through sigma_{s,l} = c sigma_t g^l,
    against central differences of the oracle's forward solve."""
    p = _prob(seed=13, K=8, N=8)
    c = oracle.exit_current_weights(p.K, p.N)
    _, _, gt, gs = _grad(p, c)
    cc, gg = p.meta["c"], p.meta["g"]
    l = np.arange(p.L + 1)

    def moments(st, cv, gv):
        return (cv * st)[:, None] * gv[:, None] ** l[None, :]

    for k in (0, 4, 7):
        # chain rule
        dc = np.dot(gs[k], p.sigma_t[k] * gg[k] ** l)
        dg = np.dot(gs[k], cc[k] * p.sigma_t[k] * l * gg[k] ** np.maximum(l - 1, 0))
        dst = gt[k] + np.dot(gs[k], cc[k] * gg[k] ** l)
        for which, ana in (("c", dc), ("g", dg), ("st", dst)):
            vals = []
            for sgn in (1, -1):
                st, cv, gv = p.sigma_t.copy(), cc.copy(), gg.copy()
                arr = {"c": cv, "g": gv, "st": st}[which]
                d = 1e-6 * arr[k]
                arr[k] += sgn * d
                vals.append(_J(p, st, moments(st, cv, gv), c))
            fd = (vals[0] - vals[1]) / (2 * d)
            assert abs(fd - ana) <= 1e-6 * abs(fd), (k, which, fd, ana)
