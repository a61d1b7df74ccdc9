"""Parity of the HIP adjoint solve and response gradient (FP64 handles).

- Against the oracle, element by element: the oracle iterates the
  transposed fixed point with its transposed sweep; the HIP path solves the
  reflected forward problem with the FPSA kernels and regenerates both
  angular fluxes from converged moments.  Bound 1e-9 of the largest
  gradient entry (HIP solves stopped at 2e-13 absolute on moments of order
  one to ten, the oracle's at 1e-14).
- Against FP64 central differences of the HIP forward solve on 32 sampled
  per-cell parameters (sigma_t, c, g of the Henyey-Greenstein moments),
  through the torch.autograd.Function; bound 1e-6 relative, with a floor at
  1e-3 of the largest sampled derivative for parameters deep in a slab.
- At the full differentiation batch (256 slabs x 4096 cells, S_64):
  the same finite-difference check on 32 sampled parameters of two slabs,
  each re-solved alone.
"""
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


def _q_ext(torch, probs):
    return torch.from_numpy(np.concatenate([p.q_or_zero().ravel() for p in probs])).cuda()


@pytest.mark.parametrize("scheme,coef", [("wfd", "cell"), ("mpd", "mean")])
def test_gradient_matches_oracle(torch, snfpsa, scheme, coef):
    probs = [sw.cellwise_hg_slab(21, K=150, N=16, h=0.1), sw.cellwise_hg_slab(22, K=90, N=8, h=0.2),
             sw.random_slab(23, K=100, N=8, regions=3, kernel="hg", source="random", inflow="random",
                            c_range=(0.5, 0.95))]
    say("gradient vs oracle", scheme, coef)
    S = snfpsa.SlabSolver(probs, fp_scheme=scheme, fp_coefficients=coef)
    qe = _q_ext(torch, probs)
    r = S.solve("fpsa", tol=2e-13, max_iter=500, q_ext=qe)
    assert r["status"] == 0
    c = S.exit_current_weights()
    a = S.solve_adjoint(c, "fpsa", tol=2e-13, max_iter=500)
    assert a["status"] == 0
    say("forward iterations", r["iters"], "adjoint iterations", a["iters"])
    J, gt, gs = S.response_gradient(r["phi"], c, a["phi_y"], q_ext=qe)
    torch.cuda.synchronize()
    J, gt, gs = host(J), host(gt), host(gs)
    co, so = 0, 0
    for b, p in enumerate(probs):
        ref = oracle.solve(p, "si", tol=1e-14, max_iter=200000)
        cw = oracle.exit_current_weights(p.K, p.N)
        lam = oracle.adjoint_solve(p, cw, tol=1e-16, max_iter=20000)["lam"]
        rgt, rgs = oracle.response_gradient(p, ref["psi"], lam)
        Jref = float((cw * ref["psi"]).sum())
        g1 = gt[co:co + p.K]
        g2 = gs[so:so + p.K * (p.L + 1)].reshape(p.K, p.L + 1)
        e1 = np.abs(g1 - rgt).max() / np.abs(rgt).max()
        e2 = np.abs(g2 - rgs).max() / np.abs(rgs).max()
        say("slab", b, "J", J[b], Jref, "grad sigma_t err", e1, "grad sigma_s err", e2)
        assert abs(J[b] - Jref) <= 1e-12 * abs(Jref)
        assert e1 < 1e-9 and e2 < 1e-9
        co += p.K
        so += p.K * (p.L + 1)
    S.close()


def _params(torch, probs):
    st = torch.from_numpy(np.concatenate([p.sigma_t for p in probs])).cuda()
    cc = torch.from_numpy(np.concatenate([p.meta["c"] for p in probs])).cuda()
    gg = torch.from_numpy(np.concatenate([p.meta["g"] for p in probs])).cuda()
    return st, cc, gg


def _sigma_s(snfpsa, st, cc, gg, L):
    return snfpsa.hg_moments(st, cc, gg, L).reshape(-1)


def _fd_check(torch, snfpsa, S, probs, qe, samples, tol, step=1e-5):
    """Central differences of the exit current of slab b with respect to
    parameter (which, cell) against the autograd gradient; returns the
    errors."""
    L = probs[0].L
    st, cc, gg = _params(torch, probs)
    for t in (st, cc, gg):
        t.requires_grad_(True)
    J = snfpsa.exit_current(st, _sigma_s(snfpsa, st, cc, gg, L), S, q_ext=qe, tol=tol)
    J.sum().backward()
    grads = {"sigma_t": host(st.grad), "c": host(cc.grad), "g": host(gg.grad)}
    base = {"sigma_t": host(st), "c": host(cc), "g": host(gg)}
    offs = np.cumsum([0] + [p.K for p in probs])
    fds, anas = [], []
    for b, which, k in samples:
        cell = offs[b] + k
        vals = []
        for sgn in (1, -1):
            v = {n: a.copy() for n, a in base.items()}
            d = step * v[which][cell]
            v[which][cell] += sgn * d
            ss = (v["c"] * v["sigma_t"])[:, None] * v["g"][:, None] ** np.arange(L + 1)[None, :]
            S.update_cross_sections(v["sigma_t"], ss)
            pe = torch.zeros(S.exit_len, dtype=torch.float64, device="cuda")
            r = S.solve("fpsa", tol=tol, max_iter=2000, q_ext=qe, psi_exit=pe, history=False)
            assert r["status"] == 0
            vals.append(float(S.exit_current(pe)[b]))
        fds.append((vals[0] - vals[1]) / (2 * d))
        anas.append(grads[which][cell])
    fds, anas = np.array(fds), np.array(anas)
    floor = 1e-3 * np.abs(fds).max()
    return np.abs(fds - anas) / np.maximum(np.abs(fds), floor), fds, anas


def test_exit_current_autograd_matches_central_differences(torch, snfpsa):
    probs = [sw.cellwise_hg_slab(31 + b, K=300, N=16, h=0.05) for b in range(3)]
    say("autograd vs central differences, 3 slabs x 300 cells, S_16")
    S = snfpsa.SlabSolver(probs, fp_scheme="wfd", fp_coefficients="mean")
    qe = _q_ext(torch, probs)
    rng = np.random.Generator(np.random.PCG64(5))
    samples = [(int(rng.integers(0, 3)), ["sigma_t", "c", "g"][i % 3], int(rng.integers(0, 300)))
               for i in range(32)]
    err, fds, anas = _fd_check(torch, snfpsa, S, probs, qe, samples, tol=2e-13)
    say("max rel err", err.max(), "median |dJ|", np.median(np.abs(fds)))
    assert err.max() < 1e-6
    S.close()


def test_differentiation_batch_full_size(torch, snfpsa):
    """256 slabs x 4096 cells, S_64, L = 63, HG g = 0.95, per-cell sigma_t
    and c: gradients through the autograd function on the whole batch;
    32 sampled parameters of two slabs checked by central differences of
    those slabs re-solved alone (same shared-coefficient preconditioner)."""
    probs = sw.differentiation_batch(256, with_source=False)
    K, N, L = probs[0].K, probs[0].N, probs[0].L
    say("differentiation batch", len(probs), "x", K, "cells, S_%d" % N)
    S = snfpsa.SlabSolver(probs, fp_scheme="wfd", fp_coefficients="mean")
    qe = torch.ones(S.psi_len, dtype=torch.float64, device="cuda")
    st, cc, gg = _params(torch, probs)
    for t in (st, cc, gg):
        t.requires_grad_(True)
    opts = {}
    J = snfpsa.exit_current(st, _sigma_s(snfpsa, st, cc, gg, L), S, q_ext=qe, tol=1e-11, opts=opts)
    J.sum().backward()
    say("forward iterations (first slabs)", opts["state"]["iters"][:4],
        "adjoint", opts["state"]["iters_adjoint"][:4])
    assert opts["state"]["status"] == 0 and opts["state"]["status_adjoint"] == 0
    assert bool(torch.isfinite(st.grad).all()) and bool(torch.isfinite(gg.grad).all())
    g_all = {"sigma_t": host(st.grad), "c": host(cc.grad), "g": host(gg.grad)}
    J_all = host(J)
    S.close()
    del S, qe
    torch.cuda.empty_cache()
    rng = np.random.Generator(np.random.PCG64(6))
    for b in (17, 200):
        p = probs[b]
        p.q = np.ones((K, 2, N))
        S1 = snfpsa.SlabSolver([p], fp_scheme="wfd", fp_coefficients="mean")
        qe1 = _q_ext(torch, [p])
        samples = [(0, ["sigma_t", "c", "g"][i % 3], int(K - 1 - rng.integers(0, 400))) for i in range(16)]
        err, fds, anas = _fd_check(torch, snfpsa, S1, [p], qe1, samples, tol=1e-11)
        # the single-slab gradients agree with the batch's
        floor = 1e-3 * np.abs(anas).max()
        for (_, which, k), a in zip(samples, anas):
            gb = g_all[which][b * K + k]
            assert abs(gb - a) <= 1e-8 * max(abs(a), floor), (b, which, k, gb, a)
        say("slab", b, "J", J_all[b], "max rel err vs central differences", err.max())
        assert err.max() < 1e-6
        S1.close()


def test_adjoint_entry_points_reject_wrong_handles(torch, snfpsa):
    p = sw.cellwise_hg_slab(41, K=20, N=8)
    S = snfpsa.SlabSolver([p], fp_scheme="none", precision="f32")
    c = torch.zeros(S.psi_len, dtype=torch.float64, device="cuda")
    with pytest.raises(snfpsa.SnError) as e:
        S.solve_adjoint(c, "si", tol=1e-8, max_iter=5)
    assert e.value.status == snfpsa.SN_E_STATE
    with pytest.raises(snfpsa.SnError):
        S.update_cross_sections(p.sigma_t, p.sigma_s)
    S.close()
    S = snfpsa.SlabSolver([p], fp_scheme="none")
    c = S.exit_current_weights()
    with pytest.raises(snfpsa.SnError) as e:
        S.solve_adjoint(c, "fpsa", tol=1e-8, max_iter=5)     # no Fokker-Planck factors
    assert e.value.status == snfpsa.SN_E_STATE
    bad = p.sigma_s.copy()
    bad[3, 0] = 2 * p.sigma_t[3]                             # sigma_a < 0
    with pytest.raises(snfpsa.SnError) as e:
        S.update_cross_sections(p.sigma_t, bad)
    assert e.value.status == snfpsa.SN_E_INVALID
    # source iteration adjoint without factors works and matches the oracle's J
    q = torch.from_numpy(p.q.ravel()).cuda()
    r = S.solve("si", tol=1e-13, max_iter=5000, q_ext=q)
    a = S.solve_adjoint(c, "si", tol=1e-13, max_iter=5000)
    J, gt, gs = S.response_gradient(r["phi"], c, a["phi_y"], q_ext=q)
    ref = oracle.solve(p, "si", tol=1e-14)
    Jref = float((oracle.exit_current_weights(p.K, p.N) * ref["psi"]).sum())
    assert abs(float(J[0]) - Jref) <= 1e-11 * abs(Jref)
    S.close()


def test_exit_current_calls(torch, snfpsa):
    """sn_exit_current_weights gives the oracle's response weights, and
    sn_exit_current on the solve's exit fluxes gives the oracle's exit
    current, for FP64 handles (several slabs, mixed N) and a batched FP32
    handle (float exit fluxes, FP64 sums)."""
    probs = [sw.random_slab(51, K=40, N=8, regions=2, kernel="hg", source="random", inflow="random",
                            c_range=(0.3, 0.8)),
             sw.random_slab(52, K=33, N=16, regions=3, kernel="srk", source="random", inflow="random",
                            c_range=(0.3, 0.8))]
    say("exit current calls")
    qe = _q_ext(torch, probs)
    refs = [oracle.solve(p, "si", tol=1e-14, max_iter=20000) for p in probs]
    Jref = np.array([float((oracle.exit_current_weights(p.K, p.N) * r["psi"]).sum()) for p, r in zip(probs, refs)])
    S = snfpsa.SlabSolver(probs, fp_scheme="wfd")
    c = host(S.exit_current_weights())
    off = 0
    for p in probs:
        n = p.K * 2 * p.N
        assert np.abs(c[off:off + n] - oracle.exit_current_weights(p.K, p.N).ravel()).max() < 1e-15
        off += n
    pe = torch.zeros(S.exit_len, dtype=torch.float64, device="cuda")
    r = S.solve("fpsa", tol=1e-13, max_iter=500, q_ext=qe, psi_exit=pe)
    assert r["status"] == 0
    J = host(S.exit_current(pe))
    say("FP64 J", J, "oracle", Jref)
    assert np.abs(J - Jref).max() <= 1e-11 * np.abs(Jref).max()
    S.close()
    B = snfpsa.SlabSolver(probs, fp_scheme="none", precision="f32")
    pe = torch.zeros(B.exit_len, dtype=torch.float32, device="cuda")
    r = B.solve("si", tol=2e-6, max_iter=2000, q_ext=qe.float(), psi_exit=pe)
    assert r["status"] == 0
    J = host(B.exit_current(pe))
    # the same reduction in FP64 on the host, with the oracle's quadrature
    pe_h, off, Jh = host(pe).astype(np.float64), 0, []
    for p in probs:
        mu, w = oracle.gauss_legendre(p.N)
        Jh.append(float(np.sum(np.where(mu > 0, w * mu, 0.0) * pe_h[off:off + p.N])))
        off += p.N
    say("FP32 J", J, "host sum", Jh)
    assert np.abs(J - np.array(Jh)).max() <= 1e-13 * np.abs(Jref).max()
    assert np.abs(J - Jref).max() <= 5e-5 * np.abs(Jref).max()
    B.close()
