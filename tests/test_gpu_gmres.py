"""Parity of the restarted GMRES outer solvers (SN_FPSA_GMRES, SN_GMRES).

GMRES solves the same discrete problem as SI and FPSA, so its solution is
checked against the oracle's converged FPSA solution (1e-10 of the largest
moment at the workloads' tolerances, which the GMRES residual bounds).  The
residual history is checked for what GMRES guarantees: within a restart
cycle the minimised residual never grows.  FPSA-preconditioned GMRES needs
no more sweeps than FPSA (the paper's FPSA_GMRES columns need fewer).
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


def _check_history(hist, tol, restart=30):
    """Non-increasing residual inside every restart cycle.  A cycle starts
    with the residual sweep (the true residual of the current iterate) and
    has up to `restart` Arnoldi sweeps (the minimised residual estimates); it
    ends early at the first estimate <= tol, after which the next entry is the
    true residual of the updated iterate, which starts the next cycle and may
    differ from that estimate by rounding."""
    i = 0
    while i < len(hist):
        end = i + 1
        if hist[i] > tol:
            while end < len(hist) and end - i <= restart:
                end += 1
                if hist[end - 1] <= tol:
                    break
        cyc = hist[i:end]
        assert np.all(np.diff(cyc) <= 1e-12 * cyc[0] + 1e-300), cyc
        i = end


@pytest.mark.parametrize("method,scheme", [("fpsa_gmres", "wfd"), ("fpsa_gmres", "mpd"), ("gmres", "wfd")])
def test_gmres_hg_slab_200(torch, snfpsa, method, scheme):
    p = sw.hg_slab_200()
    say("gmres hg_slab_200", method, scheme)
    S = snfpsa.SlabSolver([p], fp_scheme=scheme)
    ex = torch.zeros(S.exit_len, dtype=torch.float64, device="cuda")
    res = S.solve(method, tol=p.tol, max_iter=2000, psi_exit=ex)
    assert res["status"] == 0
    ref = oracle.solve(p, "fpsa", scheme, tol=1e-14, max_iter=2000)
    phi = host(res["phi"]).reshape(ref["phi"].shape)
    err = np.abs(phi - ref["phi"]).max()
    fp = S.solve("fpsa", tol=p.tol, max_iter=2000)
    say("sweeps", res["iters"][0], "FPSA iterations", fp["iters"][0], "max err", err)
    assert err < 1e-10 * np.abs(ref["phi"]).max()
    if method == "fpsa_gmres":
        assert res["iters"][0] <= fp["iters"][0]
    _check_history(res["hist"][0], p.tol)
    mu, _ = oracle.gauss_legendre(p.N)
    exit_ref = np.where(mu > 0, ref["psi"][-1, 1, :], ref["psi"][0, 0, :])
    assert np.abs(host(ex) - exit_ref).max() < 1e-9
    S.close()


def test_fpsa_gmres_srk_slab_2000(torch, snfpsa):
    p = sw.srk_slab_2000()
    say("fpsa_gmres srk_slab_2000")
    S = snfpsa.SlabSolver([p], fp_scheme="wfd")
    q = torch.from_numpy(p.q.ravel().copy()).cuda()
    res = S.solve("fpsa_gmres", tol=p.tol, max_iter=500, q_ext=q)
    assert res["status"] == 0
    fp = S.solve("fpsa", tol=p.tol, max_iter=500, q_ext=q)
    ref = oracle.solve(p, "fpsa", "wfd", tol=1e-12, max_iter=200)
    phi = host(res["phi"]).reshape(ref["phi"].shape)
    err = np.abs(phi - ref["phi"]).max() / np.abs(ref["phi"]).max()
    say("sweeps", res["iters"][0], "FPSA iterations", fp["iters"][0], "rel err", err)
    assert err < 1e-10
    assert res["iters"][0] <= fp["iters"][0]
    _check_history(res["hist"][0], p.tol)
    S.close()


def test_gmres_multi_slab_and_limits(torch, snfpsa):
    probs = [sw.random_slab(61 + i, K=K, N=N, regions=3, kernel="srk", source="uniform", inflow="random")
             for i, (K, N) in enumerate([(120, 8), (300, 16), (45, 32)])]
    S = snfpsa.SlabSolver(probs, fp_scheme="mpd")
    q = torch.from_numpy(np.concatenate([p.q.ravel() for p in probs])).cuda()
    res = S.solve("fpsa_gmres", tol=1e-11, max_iter=400, q_ext=q)
    assert res["status"] == 0
    off = 0
    for p, it in zip(probs, res["iters"]):
        ref = oracle.solve(p, "fpsa", "mpd", tol=1e-13, max_iter=400)
        n = p.K * 2 * (p.L + 1)
        phi = host(res["phi"][off:off + n]).reshape(ref["phi"].shape)
        assert np.abs(phi - ref["phi"]).max() < 1e-9 * np.abs(ref["phi"]).max(), (p.K, p.N, it)
        off += n
    # the iteration limit: NOT_CONVERGED, never more sweeps than allowed
    lim = S.solve("gmres", tol=1e-14, max_iter=7, q_ext=q)
    assert lim["status"] == snfpsa.SN_NOT_CONVERGED
    assert all(1 <= i <= 7 for i in lim["iters"])
    S.close()
    # GMRES needs an FP64 handle
    B = snfpsa.SlabSolver(probs[:1], fp_scheme="none", precision="f32")
    with pytest.raises(snfpsa.SnError):
        B.solve("gmres", tol=1e-8, max_iter=5)
    B.close()
