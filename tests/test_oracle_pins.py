"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics (no GPU).  Each test names what it pins."""
import math
import os

import numpy as np
import pytest

import oracle
import sn_workloads as sw
import dense_ref
import fa_tool

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Quadrature, Legendre tables, angular Laplacians
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N", [2, 8, 16, 64, 256])
def test_gauss_legendre_matches_library_and_is_exact(N):
    mu, w = oracle.gauss_legendre(N)
    m2, w2 = np.polynomial.legendre.leggauss(N)
    assert np.all(np.diff(mu) > 0)
    assert np.abs(mu - m2).max() < 1e-14
    assert np.abs(w - w2).max() < 1e-14
    for k in range(0, 2 * N, max(1, (2 * N) // 16)):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, mu ** k) - exact) < 1e-13


@pytest.mark.parametrize("N", [8, 64])
def test_legendre_table_and_moment_orthogonality(N):
    mu, w = oracle.gauss_legendre(N)
    P = oracle.legendre(N, N - 1, mu)
    ref = np.array([np.polynomial.legendre.legval(mu, np.eye(N)[l]) for l in range(N)])
    assert np.abs(P - ref).max() < 1e-12
    D = P * w[None, :]
    M = (P.T * (2 * np.arange(N) + 1) / 2.0)
    assert np.abs(D @ M - np.eye(N)).max() < 1e-12      # discrete-to-moment o moment-to-discrete


@pytest.mark.parametrize("N", [4, 8, 16, 64])
def test_wfd_matrix_properties(N):
    """Sec. 2.2: WFD preserves the zeroth and first moments and gives an
    M-matrix (non-negative off-diagonals of W)."""
    mu, w = oracle.gauss_legendre(N)
    W = oracle.wfd_matrix(N)
    V = oracle.legendre(N, N - 1, mu) * w[None, :]
    lam = -np.arange(N) * (np.arange(N) + 1.0)
    assert np.abs(W.sum(axis=1)).max() < 1e-12 * N * N
    R = V @ W - lam[:, None] * V
    assert np.abs(R[:2]).max() < 1e-11 * N
    if N >= 4:
        assert np.abs(R[2]).max() > 1e-8                  # only two moments preserved
    off = W - np.diag(np.diag(W))
    assert off.min() >= 0.0
    assert np.count_nonzero(np.triu(W, 2)) == 0 and np.count_nonzero(np.tril(W, -2)) == 0
    T = 0.01 * np.eye(N) - 0.5 * 0.3 * W
    assert np.linalg.inv(T).min() > -1e-12              # inverse-positive
    assert np.abs(W - fa_tool.wfd(mu, w)).max() < 1e-10 * np.abs(W).max()


@pytest.mark.parametrize("N", [4, 8, 16, 32])
def test_mpd_matrix_properties(N):
    """Sec. 2.2, eq:legendre / eq:fp-mpd: V F = diag(-l(l+1)) V, and for
    Gauss-Legendre V^{-1} = M gives the closed form F = M diag V."""
    mu, w = oracle.gauss_legendre(N)
    F = oracle.mpd_matrix(N)
    P = oracle.legendre(N, N - 1, mu)
    V = P * w[None, :]
    lam = -np.arange(N) * (np.arange(N) + 1.0)
    scale = N * N
    assert np.abs(V @ F - lam[:, None] * V).max() < 1e-11 * scale
    M = P.T * (2 * np.arange(N) + 1) / 2.0
    assert np.abs(F - M @ (lam[:, None] * V)).max() < 1e-10 * scale
    # F applied to P_l sampled at the nodes returns -l(l+1) P_l (eq:legendre)
    for l in range(N):
        assert np.abs(F @ P[l] + l * (l + 1) * P[l]).max() < 1e-10 * scale


# --------------------------------------------------------------------------
# LD sweep closed forms
# --------------------------------------------------------------------------

def _absorber(K, width, N, sigma, inflow=1.0):
    return sw.homogeneous("abs", K=K, width=width, N=N, L=0, sigma_t=sigma,
                          moments=np.array([1.0]), c=0.0, psi_left=inflow,
                          psi_right=inflow)


def test_pure_absorber_exact_ld_attenuation():
    """Pure absorber: after k uniform cells the outgoing flux is
    r(tau)^k psi_in with r = (6 - 2 tau)/(6 + 4 tau + tau^2), tau = sigma h/|mu|."""
    N, K = 8, 37
    p = _absorber(K, 3.7, N, 1.3)
    mu, _ = oracle.gauss_legendre(N)
    psi = oracle.sweep(np.zeros((K, 2, N)), p.h, p.sigma_t, p.psi_left, p.psi_right)
    for n in range(N):
        tau = 1.3 * 0.1 / abs(mu[n])
        r = (6 - 2 * tau) / (6 + 4 * tau + tau * tau)
        for k in range(K):
            if mu[n] > 0:
                got = psi[k, 1, n]
            else:
                got = psi[K - 1 - k, 0, n]
            assert abs(got - r ** (k + 1)) < 1e-14


def test_pure_absorber_converges_to_exponential_third_order():
    """The LD edge flux converges to exp(-sigma z/mu) at O(h^3)."""
    N = 8
    mu, _ = oracle.gauss_legendre(N)
    errs = []
    for K in (8, 16, 32, 64):
        p = _absorber(K, 2.0, N, 1.0)
        psi = oracle.sweep(np.zeros((K, 2, N)), p.h, p.sigma_t, p.psi_left, None)
        errs.append(abs(psi[-1, 1, N // 2] - math.exp(-2.0 / mu[N // 2])))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(7.0 < r < 9.0 for r in ratios[1:]), ratios


def test_infinite_medium_closed_form():
    """Uniform medium, isotropic source q and inflow q/sigma_a on both faces:
    psi = q/sigma_a everywhere, phi_0 = 2 q/sigma_a, phi_{l>=1} = 0."""
    N, L, K = 8, 7, 40
    c, st, qv = 0.9, 2.0, 1.5
    p = sw.homogeneous("inf", K=K, width=4.0, N=N, L=L, sigma_t=st,
                       moments=sw.hg_moments(0.7, L), c=c, source=qv)
    sa = st * (1 - c)
    p.psi_left[:] = qv / sa
    p.psi_right[:] = qv / sa
    for method, scheme in [("si", "wfd"), ("fpsa", "wfd"), ("fpsa", "mpd")]:
        r = oracle.solve(p, method, scheme, tol=1e-13, max_iter=5000)
        assert r["status"] == 0
        assert np.abs(r["psi"] - qv / sa).max() < 1e-10
        assert np.abs(r["phi"][:, :, 0] - 2 * qv / sa).max() < 1e-10
        assert np.abs(r["phi"][:, :, 1:]).max() < 1e-10


def test_particle_balance_at_convergence():
    """LD is conservative per cell: leakage + absorption = source."""
    p = sw.random_slab(11, K=60, N=16, regions=4, kernel="srk", source="random")
    r = oracle.solve(p, "fpsa", "wfd", tol=1e-13, max_iter=2000)
    assert r["status"] == 0
    mu, w = oracle.gauss_legendre(p.N)
    psi, phi = r["psi"], r["phi"]
    half = p.N // 2
    z1 = np.where(mu > 0, psi[-1, 1, :], np.concatenate([p.psi_right, np.zeros(half)]))
    z0 = np.where(mu > 0, np.concatenate([np.zeros(half), p.psi_left]), psi[0, 0, :])
    leak = np.sum(w * mu * (z1 - z0))
    sa = p.sigma_t - p.sigma_s[:, 0]
    absorb = np.sum(p.h * sa * 0.5 * (phi[:, 0, 0] + phi[:, 1, 0]))
    src = np.sum(p.h * 0.5 * ((p.q[:, 0, :] + p.q[:, 1, :]) @ w))
    assert abs(leak + absorb - src) < 1e-10 * src


def test_straight_ahead_scattering_is_pure_absorber():
    """sigma_{s,l} = sigma_{s,0} for all l <= N-1 makes S = sigma_{s,0} I: the
    solution is the pure absorber with sigma_a, and FPSA (sigma_tr = 0) is
    exact after one iteration."""
    N, K = 8, 30
    p = sw.homogeneous("sa", K=K, width=3.0, N=N, L=N - 1, sigma_t=1.0,
                       moments=np.ones(N), c=0.95, source=1.0, psi_left=0.5)
    direct = oracle.sweep(p.q, p.h, p.sigma_t * 0.05, p.psi_left, p.psi_right)
    r = oracle.solve(p, "fpsa", "mpd", tol=1e-13)
    assert r["hist"][1] < 1e-12 * r["hist"][0]
    assert np.abs(r["psi"] - direct).max() < 1e-11
    r = oracle.solve(p, "si", tol=1e-13, max_iter=5000)
    assert np.abs(r["psi"] - direct).max() < 1e-10


def test_pl_equivalent_moments_converge_in_one_fpsa_iteration():
    """Sec. 3.2, eq:fsa_pl_eq: with P_L-equivalent moments and N = L+1,
    FPSA (MPD) is P_L acceleration and converges in one iteration."""
    for N in (4, 8, 16):
        L = N - 1
        ss = sw.pl_equivalent_moments(0.99, 0.985, L)
        p = sw.homogeneous("pl", K=40, width=4.0, N=N, L=L, sigma_t=1.0,
                           moments=np.ones(L + 1), c=1.0, source=1.0, psi_left=0.3)
        p.sigma_s = np.tile(ss, (40, 1))
        r = oracle.solve(p, "fpsa", "mpd", tol=1e-300, max_iter=3)
        assert r["hist"][1] < 1e-11 * r["hist"][0], r["hist"]
        w = oracle.solve(p, "fpsa", "wfd", tol=1e-300, max_iter=3)
        if N > 2:
            assert w["hist"][1] > 1e-6 * w["hist"][0]       # WFD is not exact


# --------------------------------------------------------------------------
# Brute force on tiny grids
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N,kernel,seed", [(4, "hg", 1), (8, "srk", 2), (8, "hg", 3), (2, "iso", 4)])
def test_si_and_fpsa_converge_to_dense_solution(N, kernel, seed):
    p = sw.random_slab(seed, K=7, N=N, regions=3, kernel=kernel, source="random")
    psi_ref = dense_ref.transport_solution(p)
    phi_ref = dense_ref.moments(psi_ref, p.L)
    scale = np.abs(psi_ref).max()
    for method, scheme in [("si", "wfd"), ("fpsa", "wfd"), ("fpsa", "mpd")]:
        r = oracle.solve(p, method, scheme, tol=1e-14, max_iter=20000)
        assert r["status"] == 0
        assert np.abs(r["psi"] - psi_ref).max() < 1e-11 * scale, (method, scheme)
        assert np.abs(r["phi"] - phi_ref).max() < 1e-11 * scale


@pytest.mark.parametrize("scheme,N", [("wfd", 4), ("mpd", 4), ("wfd", 8), ("mpd", 8)])
def test_fp_solve_matches_dense_operator(scheme, N):
    K = 9
    rng = np.random.default_rng(5)
    h = rng.uniform(0.02, 0.5, K)
    sa = rng.uniform(1e-3, 1.0, K)
    st = rng.uniform(1e-3, 2.0, K)
    r = rng.uniform(-1, 1, (K, 2, N))
    mu, w, P = dense_ref.quadrature(N)
    A = fa_tool.wfd(mu, w) if scheme == "wfd" else fa_tool.mpd(P * w[None, :])
    ref = dense_ref.fp_operator_solve(r, h, sa, st, A)
    got = oracle.fp_solve(r, h, sa, st, scheme)
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


def test_sweep_matches_dense_and_adjoint_is_transpose():
    p = sw.random_slab(9, K=8, N=6, regions=3, kernel="hg")
    mu, w, P = dense_ref.quadrature(p.N)
    T = [p.sigma_t[k] * np.eye(p.N) for k in range(p.K)]
    A, _ = dense_ref.assemble(mu, p.h, T)
    n = A.shape[0]
    # map q -> psi for zero inflow, column by column
    G = np.zeros((n, n))
    Gt = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        G[:, j] = oracle.sweep(e.reshape(p.K, 2, p.N), p.h, p.sigma_t).ravel()
        Gt[:, j] = oracle.sweep_adjoint(e.reshape(p.K, 2, p.N), p.h, p.sigma_t).ravel()
    for j in range(0, n, 7):
        e = np.zeros(n)
        e[j] = 1.0
        _, b = dense_ref.assemble(mu, p.h, T, None, None, e.reshape(p.K, 2, p.N))
        assert np.abs(np.linalg.solve(A, b) - G[:, j]).max() < 1e-12
    assert np.abs(Gt - G.T).max() < 1e-12


def test_adjoint_dot_product_identity():
    p = sw.random_slab(21, K=300, N=16, regions=5, kernel="srk")
    x = sw.random_vectors(1, p.K, 2, p.N)
    y = sw.random_vectors(2, p.K, 2, p.N)
    lhs = np.sum(y * oracle.sweep(x, p.h, p.sigma_t))
    rhs = np.sum(oracle.sweep_adjoint(y, p.h, p.sigma_t) * x)
    assert abs(lhs - rhs) < 1e-13 * max(abs(lhs), 1.0)


# --------------------------------------------------------------------------
# Convergence rates and the paper's Table 1
# --------------------------------------------------------------------------

def _table1():
    rows = {}
    with open(os.path.join(GOLDEN, "table1_spectral_radii.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, par, a, b, c, d = line.split()
            rows[k] = (float(par), float(a), float(b), float(c), float(d))
    return rows


def test_si_rate_tends_to_scattering_ratio():
    """Sec. 2.1 / eq:fpsa7: the SI spectral radius is sigma_{s,0}/sigma_t."""
    c = 0.99
    p = sw.homogeneous("thick", K=100, width=100.0, N=8, L=7, sigma_t=10.0,
                       moments=sw.hg_moments(0.9, 7), c=c)
    phi0 = sw.random_vectors(3, 100, 2, 8)
    r = oracle.solve(p, "si", tol=1e-300, max_iter=600, phi0=phi0)
    h = r["hist"]
    rho = (h[-1] / h[-201]) ** (1 / 200)
    assert rho < c and c - rho < 2e-3


def test_fourier_analysis_reproduces_table1():
    """Paper Table 1, FA columns (HG to 4 printed digits; SRK to 3)."""
    t = _table1()
    g, mpd_fa, _, wfd_fa, _ = t["hg"]
    ss = 0.9999 * sw.hg_moments(g, 15)
    assert abs(fa_tool.spectral_radius(ss, scheme="mpd", N=16) - mpd_fa) < 6e-5
    assert abs(fa_tool.spectral_radius(ss, scheme="wfd", N=16) - wfd_fa) < 6e-5
    eta, mpd_fa, _, wfd_fa, _ = t["srk"]
    ss = 0.9999 * sw.srk_moments(eta, 15)
    assert abs(fa_tool.spectral_radius(ss, scheme="mpd", N=16) - mpd_fa) < 1e-3
    assert abs(fa_tool.spectral_radius(ss, scheme="wfd", N=16) - wfd_fa) < 1e-3
    assert abs(fa_tool.spectral_radius(ss, N=16, accel=False) - 0.9999) < 1e-12


def test_oracle_measured_fpsa_rate_matches_table1_hg():
    """Paper Table 1, measured columns for HG g = 0.9 (100 cells, 100 cm,
    vacuum): power iteration of the oracle's FPSA on the homogeneous
    problem."""
    t = _table1()
    g, _, mpd_meas, _, wfd_meas = t["hg"]
    p = sw.homogeneous("t1", K=100, width=100.0, N=16, L=15, sigma_t=1000.0,
                       moments=sw.hg_moments(g, 15), c=0.9999)
    phi0 = sw.random_vectors(7, 100, 2, 16)
    for scheme, ref in [("mpd", mpd_meas), ("wfd", wfd_meas)]:
        h = oracle.solve(p, "fpsa", scheme, tol=1e-300, max_iter=200, phi0=phi0)["hist"]
        rho = (h[-1] / h[-51]) ** (1 / 50)
        assert abs(rho - ref) < 1.5e-3, (scheme, rho, ref)


# --------------------------------------------------------------------------
# Scattering-kernel moments used by the workloads
# --------------------------------------------------------------------------

@pytest.mark.parametrize("eta", [1e-7, 1e-5, 2.83e-5, 1e-3])
def test_srk_moments(eta):
    f = sw.srk_moments(eta, 255)
    assert f[0] == 1.0
    assert abs(f[1] - sw.srk_f1_closed_form(eta)) < 1e-13
    assert np.all(np.diff(f) < 0) and f[-1] > 0
    f2 = sw.srk_moments(eta, 255, panels=2 * int(math.ceil(math.log((1 + eta) / eta) * 255 / 3)))
    assert np.abs(f - f2).max() < 1e-12


def test_srk_moments_against_adaptive_quadrature():
    from scipy.integrate import quad
    from scipy.special import eval_legendre
    eta = 1e-3
    f = sw.srk_moments(eta, 12)
    for l in (2, 5, 12):
        v = quad(lambda m: eval_legendre(l, m) / (1 + 2 * eta - m) ** 2, -1, 1,
                 points=[0.9, 0.99, 0.999], limit=500)[0] * 2 * eta * (1 + eta)
        assert abs(v - f[l]) < 1e-10


# --------------------------------------------------------------------------
# The standalone correction map (eq:correct)
# --------------------------------------------------------------------------

def _dense_fpsa_correct(p, phi_half, phi_old, scheme):
    """eq:correct composed from dense pieces written here: the residual
    source r = M diag(sigma_s) (phi_half - phi_old) at every LD node, the
    dense LD x S_N Fokker-Planck solve with zero inflow (eq:fpop), and the
    moments D of the correction added to phi_half."""
    N, L = p.N, p.L
    mu, w, P = dense_ref.quadrature(N)
    M = P[: L + 1].T * (2 * np.arange(L + 1) + 1) / 2.0        # N x (L+1)
    V = P[: L + 1] * w[None, :]                                # (L+1) x N
    A = fa_tool.wfd(mu, w) if scheme == "wfd" else fa_tool.mpd(P * w[None, :])
    s0 = p.sigma_s[:, 0]
    s1 = p.sigma_s[:, 1] if L >= 1 else np.zeros(p.K)
    dphi = phi_half - phi_old
    r = np.einsum("nl,kl,kvl->kvn", M, p.sigma_s, dphi)
    U = dense_ref.fp_operator_solve(r, p.h, p.sigma_t - s0, s0 - s1, A)
    return phi_half + np.einsum("ln,kvn->kvl", V, U), U


@pytest.mark.parametrize("scheme", ["wfd", "mpd"])
@pytest.mark.parametrize("N,K,kernel,seed", [(4, 7, "hg", 11), (8, 9, "srk", 12), (8, 5, "hg", 13),
                                             (4, 9, "srk", 14)])
def test_fpsa_correct_matches_dense_composition(scheme, N, K, kernel, seed):
    """oracle.fpsa_correct (eq:correct in moment form) equals the dense
    composition above to 1e-12: a sign slip in phi_half - phi_old, a dropped
    phi_half, a wrong sigma_a / sigma_tr or a transposed moment map fails."""
    p = sw.random_slab(seed, K=K, N=N, regions=3, kernel=kernel, source="random")
    ph = sw.random_vectors(100 + seed, p.K, 2, p.L + 1)
    po = sw.random_vectors(200 + seed, p.K, 2, p.L + 1)
    got, U = oracle.fpsa_correct(p, ph, po, scheme)
    ref, Uref = _dense_fpsa_correct(p, ph, po, scheme)
    assert np.abs(U - Uref).max() < 1e-12 * np.abs(Uref).max()
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # the correction itself, not only phi_half, is what is compared
    assert np.abs((got - ph) - (ref - ph)).max() < 1e-11 * np.abs(ref - ph).max()


@pytest.mark.parametrize("scheme", ["wfd", "mpd"])
def test_fpsa_correct_is_the_correction_inside_one_fpsa_iteration(scheme):
    """One FPSA iteration of oracle.solve from phi0 is one source iteration
    (eq:predict) followed by oracle.fpsa_correct(phi_half, phi0) (eq:correct)."""
    p = sw.random_slab(15, K=23, N=8, regions=4, kernel="srk", source="random")
    phi0 = sw.random_vectors(16, p.K, 2, p.L + 1)
    half = oracle.solve(p, "si", scheme, tol=0.0, max_iter=1, phi0=phi0)["phi"]
    one = oracle.solve(p, "fpsa", scheme, tol=0.0, max_iter=1, phi0=phi0)["phi"]
    got, _ = oracle.fpsa_correct(p, half, phi0, scheme)
    assert np.abs(got - one).max() < 1e-13 * np.abs(one).max()
    ref, _ = _dense_fpsa_correct(p, half, phi0, scheme)
    assert np.abs(one - ref).max() < 1e-12 * np.abs(ref).max()
