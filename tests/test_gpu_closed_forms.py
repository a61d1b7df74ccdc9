"""The GPU solvers against closed forms of the discrete problem (no oracle).

- Pure absorber (sigma_s = 0): the outgoing face flux of every angle is
  r(tau)^K psi_in exactly, r = (6 - 2 tau)/(6 + 4 tau + tau^2), tau =
  sigma_t h / |mu| (the LD cell map composed K times).
- Infinite medium: uniform material, isotropic source q and inflow
  q / sigma_a on both faces give psi = q / sigma_a everywhere, so
  phi_0 = 2 q / sigma_a and phi_{l >= 1} = 0 at every node.
- Straight-ahead scattering (sigma_{s,l} = sigma_{s,0} for all l, L = N - 1):
  S = sigma_{s,0} I, the solution is the pure absorber with sigma_a, and FPSA
  (sigma_tr = 0) converges after one iteration.
- Particle balance: at convergence, leakage + absorption = source (LD is
  conservative cell by cell).

FP64 handles to 1e-12 (1e-10 where an iteration stops at 1e-13), the
batched FP32 path to its FP32 bounds (1e-5 relative; 5e-5 where K cell maps
are composed in FP32)."""
import sys

import numpy as np
import pytest

import oracle
import sn_workloads as sw

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def snfpsa(torch):
    import paper_1907_13013_amd as m
    m.load_library()
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _absorber(K, width, N, sigma, inflow):
    return sw.homogeneous("abs", K=K, width=width, N=N, L=0, sigma_t=sigma, moments=np.array([1.0]), c=0.0,
                          psi_left=inflow, psi_right=inflow)


def _absorber_exit(p, sigma):
    """Outgoing face fluxes r(tau)^K psi_in, in the exit layout (mu < 0 at
    z0, then mu > 0 at z1)."""
    mu, _ = oracle.gauss_legendre(p.N)
    h = p.h[0]
    tau = sigma * h / np.abs(mu)
    r = (6 - 2 * tau) / (6 + 4 * tau + tau * tau)
    inflow = np.concatenate([p.psi_right, p.psi_left])  # mu < 0 enter at z1, mu > 0 at z0
    return r ** p.K * inflow


@pytest.mark.parametrize("method", ["si", "fpsa"])
def test_pure_absorber_exit_flux_fp64(torch, snfpsa, method):
    p = _absorber(K=37, width=3.7, N=16, sigma=1.3, inflow=1.0)
    p.psi_left = np.linspace(0.5, 1.5, p.N // 2)
    p.psi_right = np.linspace(2.0, 0.2, p.N // 2)
    S = snfpsa.SlabSolver([p], fp_scheme="wfd" if method == "fpsa" else "none")
    ex = torch.zeros(S.exit_len, dtype=torch.float64, device="cuda")
    r = S.solve(method, tol=1e-14, max_iter=20, psi_exit=ex)
    assert r["status"] == 0 and r["iters"][0] <= 2
    ref = _absorber_exit(p, 1.3)
    e = np.abs(host(ex) - ref).max() / np.abs(ref).max()
    say("pure absorber", method, "exit rel err", e)
    assert e < 1e-13
    S.close()


def test_pure_absorber_exit_flux_batched_fp32(torch, snfpsa):
    probs = [_absorber(K=K, width=0.1 * K, N=N, sigma=s, inflow=1.0)
             for K, N, s in [(37, 16, 1.3), (200, 64, 0.7), (5, 128, 3.0)]]
    S = snfpsa.SlabSolver(probs, fp_scheme="none", precision="f32")
    ex = torch.zeros(S.exit_len, dtype=torch.float32, device="cuda")
    r = S.solve("si", tol=0.0, max_iter=3, psi_exit=ex)
    got = host(ex)
    off = 0
    for p, s in zip(probs, [1.3, 0.7, 3.0]):
        ref = _absorber_exit(p, s)
        e = np.abs(got[off:off + p.N] - ref).max() / np.abs(ref).max()
        say("batched pure absorber K", p.K, "N", p.N, "exit rel err", e)
        assert e < 5e-5  # K FP32 cell maps composed: up to ~K eps_32
        off += p.N
    S.close()


def _infinite_medium(N, L, K, c=0.9):
    st, qv = 2.0, 1.5
    p = sw.homogeneous("inf", K=K, width=0.05 * K, N=N, L=L, sigma_t=st, moments=sw.hg_moments(0.7, L), c=c,
                       source=qv)
    sa = st * (1 - c)
    p.psi_left[:] = qv / sa
    p.psi_right[:] = qv / sa
    return p, qv / sa


@pytest.mark.parametrize("method,scheme", [("si", "none"), ("fpsa", "wfd"), ("fpsa", "mpd")])
def test_infinite_medium_fp64(torch, snfpsa, method, scheme):
    p, psi0 = _infinite_medium(N=16, L=15, K=70)
    S = snfpsa.SlabSolver([p], fp_scheme=scheme)
    q = torch.from_numpy(p.q.ravel().copy()).cuda()
    r = S.solve(method, tol=1e-13, max_iter=5000, q_ext=q)
    assert r["status"] == 0
    phi = host(r["phi"]).reshape(p.K, 2, p.L + 1)
    say("infinite medium", method, scheme, "iterations", r["iters"][0])
    assert np.abs(phi[:, :, 0] - 2 * psi0).max() < 1e-10 * psi0
    assert np.abs(phi[:, :, 1:]).max() < 1e-10 * psi0
    S.close()


def test_infinite_medium_batched_fp32(torch, snfpsa):
    # c = 0.5: the stopping test (above the FP32 floor of ~16 eps_32 |phi|)
    # then bounds the error by about the same amount
    probs = [_infinite_medium(N=N, L=N - 1, K=K, c=0.5)[0] for K, N in [(70, 16), (33, 64), (129, 128)]]
    psi0 = _infinite_medium(N=16, L=15, K=1, c=0.5)[1]
    S = snfpsa.SlabSolver(probs, fp_scheme="none", precision="f32")
    q = torch.from_numpy(np.concatenate([p.q.ravel() for p in probs]).astype(np.float32)).cuda()
    r = S.solve("si", tol=1e-5 * psi0, max_iter=3000, q_ext=q)
    assert r["status"] == 0
    phi = host(r["phi"])
    off = 0
    for p in probs:
        f = phi[off:off + p.K * 2 * (p.L + 1)].reshape(p.K, 2, p.L + 1)
        assert np.abs(f[:, :, 0] - 2 * psi0).max() < 1e-5 * 2 * psi0, p.N
        assert np.abs(f[:, :, 1:]).max() < 1e-5 * 2 * psi0, p.N
        off += f.size
    S.close()


def test_straight_ahead_scattering(torch, snfpsa):
    """S = sigma_{s,0} I: FPSA-MPD converges after one iteration to the pure
    absorber with sigma_a, whose exit flux is the closed form."""
    N, K, st, c = 16, 30, 1.0, 0.95
    p = sw.homogeneous("sa", K=K, width=3.0, N=N, L=N - 1, sigma_t=st, moments=np.ones(N), c=c, psi_left=0.5)
    S = snfpsa.SlabSolver([p], fp_scheme="mpd")
    ex = torch.zeros(S.exit_len, dtype=torch.float64, device="cuda")
    r = S.solve("fpsa", tol=1e-300, max_iter=3, psi_exit=ex)
    h = r["hist"][0]
    say("straight ahead FPSA-MPD history", h)
    assert h[1] < 1e-12 * h[0]
    absorber = _absorber(K=K, width=3.0, N=N, sigma=st * (1 - c), inflow=0.0)
    absorber.psi_left[:] = 0.5
    ref = _absorber_exit(absorber, st * (1 - c))
    assert np.abs(host(ex) - ref).max() < 1e-12 * np.abs(ref).max()
    S.close()


def test_particle_balance_fp64(torch, snfpsa):
    """Leakage through both faces + absorption = source, from the GPU
    solution's exit fluxes and zeroth moments (FPSA-WFD, srk, 4 regions)."""
    p = sw.random_slab(11, K=60, N=16, regions=4, kernel="srk", source="random")
    S = snfpsa.SlabSolver([p], fp_scheme="wfd")
    ex = torch.zeros(S.exit_len, dtype=torch.float64, device="cuda")
    q = torch.from_numpy(p.q.ravel().copy()).cuda()
    r = S.solve("fpsa", tol=1e-13, max_iter=2000, q_ext=q, psi_exit=ex)
    assert r["status"] == 0
    mu, w = oracle.gauss_legendre(p.N)
    half = p.N // 2
    e = host(ex)
    z1 = np.concatenate([p.psi_right, e[half:]])       # mu < 0 enter at z1, mu > 0 leave
    z0 = np.concatenate([e[:half], p.psi_left])        # mu < 0 leave at z0, mu > 0 enter
    leak = np.sum(w * mu * (z1 - z0))
    phi = host(r["phi"]).reshape(p.K, 2, p.L + 1)
    sa = p.sigma_t - p.sigma_s[:, 0]
    absorb = np.sum(p.h * sa * 0.5 * (phi[:, 0, 0] + phi[:, 1, 0]))
    src = np.sum(p.h * 0.5 * ((p.q[:, 0, :] + p.q[:, 1, :]) @ w))
    say("balance: leak", leak, "absorb", absorb, "source", src)
    assert abs(leak + absorb - src) < 1e-10 * src
    S.close()
