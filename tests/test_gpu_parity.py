"""Parity of the HIP library (through its C ABI) with the FP64 CPU oracle."""
import os
import sys

import numpy as np
import pytest

import oracle
import sn_workloads as sw

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


SLABS = [
    # (seed, K, N, regions, kernel): ragged tiles (K not a multiple of 64),
    # single-cell slab, N from 2 to 256
    (1, 1, 2, 1, "iso"),
    (2, 37, 8, 3, "hg"),
    (3, 200, 16, 4, "srk"),
    (4, 129, 64, 2, "srk"),
    (5, 515, 32, 5, "hg"),
    (6, 70, 256, 3, "srk"),
    (7, 64, 6, 2, "hg"),
]


# long slabs: more than 128 tiles of 32 cells, so the tile carries go
# through the two-level scan over 64-tile groups (ragged last group; 193,
# 2188 and 6251 tiles)
LONG_SLABS = [
    (8, 6161, 16, 4, "srk"),
    (9, 70001, 8, 3, "hg"),
    (10, 200003, 32, 6, "hg"),
]


def _prob(seed, K, N, regions, kernel):
    return sw.random_slab(seed, K=K, N=N, regions=regions, kernel=kernel, source="random")


@pytest.mark.parametrize("case", SLABS + LONG_SLABS, ids=lambda c: f"K{c[1]}N{c[2]}")
def test_sweep_and_moments(torch, snfpsa, case):
    p = _prob(*case)
    say("sweep", case)
    S = snfpsa.SlabSolver([p])
    q = dev(torch, p.q)
    for bc in ("problem", "zero"):
        psi = S.psi_tensor()
        phi = S.phi_tensor()
        S.sweep(q, psi, phi, bc=bc)
        torch.cuda.synchronize()
        ref = oracle.sweep(p.q, p.h, p.sigma_t, p.psi_left if bc == "problem" else None,
                           p.psi_right if bc == "problem" else None)
        got = host(psi).reshape(p.K, 2, p.N)
        assert rel(got, ref) < 1e-12, bc
        phiref = oracle.moments(ref, p.L)
        assert rel(host(phi).reshape(p.K, 2, p.L + 1), phiref) < 1e-12
    S.close()


@pytest.mark.parametrize("case", SLABS, ids=lambda c: f"K{c[1]}N{c[2]}")
def test_scatter_source(torch, snfpsa, case):
    p = _prob(*case)
    say("scatter", case)
    S = snfpsa.SlabSolver([p])
    phi = sw.random_vectors(case[0], p.K, 2, p.L + 1)
    for qe in (None, p.q):
        q = S.scatter_source(dev(torch, phi), None if qe is None else dev(torch, qe))
        torch.cuda.synchronize()
        ref = oracle.scatter_source(phi, p.sigma_s, p.N, qe)
        assert rel(host(q).reshape(p.K, 2, p.N), ref) < 1e-12
    S.close()


# angle counts that reach every dispatched form of the Fokker-Planck chain:
# N/2 = 1 and 2 (staged, padded to 2), N/2 = 6, 12, 24, 48 (staged, padded
# to 8, 16, 32, 64), N/2 = 64 (the LDS-ring chain at its widest)
FP_EXTRA = [
    (71, 9, 4, 2, "hg"),
    (72, 53, 12, 3, "srk"),
    (73, 101, 24, 2, "hg"),
    (74, 77, 48, 3, "srk"),
    (75, 45, 96, 2, "hg"),
    (76, 150, 128, 3, "srk"),
]


@pytest.mark.parametrize("scheme", ["wfd", "mpd"])
@pytest.mark.parametrize("case", SLABS + FP_EXTRA, ids=lambda c: f"K{c[1]}N{c[2]}")
def test_fpsa_correct(torch, snfpsa, case, scheme):
    p = _prob(*case)
    say("fpsa_correct", case, scheme)
    S = snfpsa.SlabSolver([p], fp_scheme=scheme)
    ph = sw.random_vectors(10 + case[0], p.K, 2, p.L + 1)
    po = sw.random_vectors(20 + case[0], p.K, 2, p.L + 1)
    out = S.fpsa_correct(dev(torch, ph), dev(torch, po))
    torch.cuda.synchronize()
    ref, _ = oracle.fpsa_correct(p, ph, po, scheme)
    got = host(out).reshape(p.K, 2, p.L + 1)
    assert np.abs((got - ph) - (ref - ph)).max() < 1e-10 * max(np.abs(ref - ph).max(), 1e-30)
    S.close()


# slabs of one cell type, whose correction forms its Fokker-Planck source
# inside the additive-term kernel: every padded row length 8..64, K below,
# at and around a block's cell count (256 / padded NH), and moment rows
# 2 (L+1) that are not a multiple of 4
FP_ONE_TYPE = [
    (81, 1, 16, None), (82, 7, 16, None), (83, 31, 16, 8), (84, 33, 24, None), (85, 8, 64, None),
    (86, 9, 48, 4), (87, 515, 64, None), (88, 70, 96, None), (89, 131, 128, None), (90, 300, 32, None),
]


@pytest.mark.parametrize("scheme", ["wfd", "mpd"])
@pytest.mark.parametrize("case", FP_ONE_TYPE, ids=lambda c: f"K{c[1]}N{c[2]}L{c[3]}")
def test_fpsa_correct_one_type(torch, snfpsa, case, scheme):
    seed, K, N, L = case
    p = sw.random_slab(seed, K=K, N=N, L=L, regions=1, kernel="srk", source="random")
    say("fpsa_correct one type", case, scheme)
    S = snfpsa.SlabSolver([p], fp_scheme=scheme)
    ph = sw.random_vectors(10 + seed, p.K, 2, p.L + 1)
    po = sw.random_vectors(20 + seed, p.K, 2, p.L + 1)
    out = S.fpsa_correct(dev(torch, ph), dev(torch, po))
    torch.cuda.synchronize()
    ref, _ = oracle.fpsa_correct(p, ph, po, scheme)
    got = host(out).reshape(p.K, 2, p.L + 1)
    err = np.abs((got - ph) - (ref - ph)).max() / max(np.abs(ref - ph).max(), 1e-30)
    say("rel err of the correction %.2e" % err)
    assert err < 1e-10
    S.close()


@pytest.mark.parametrize("scheme", ["wfd", "mpd"])
def test_wide_update_gemm(torch, snfpsa, scheme):
    """A one-type slab of 4100 cells (at least 4096 rows) with 2 (L+1) = 68
    moment columns, where the correction's update GEMM takes its wide form
    (one block over all 68 columns, two accumulators per wave): the
    standalone correction against the oracle's at 1e-10, and an FPSA solve
    (the update carrying the fused stopping test) against the oracle's
    iteration count and moments."""
    p = sw.random_slab(95, K=4100, N=34, regions=1, kernel="srk", source="random", inflow="random",
                       c_range=(0.9, 0.99))
    say("wide update GEMM", p.K, p.N, scheme)
    S = snfpsa.SlabSolver([p], fp_scheme=scheme)
    ph = sw.random_vectors(96, p.K, 2, p.L + 1)
    po = sw.random_vectors(97, p.K, 2, p.L + 1)
    out = S.fpsa_correct(dev(torch, ph), dev(torch, po))
    torch.cuda.synchronize()
    ref, _ = oracle.fpsa_correct(p, ph, po, scheme)
    got = host(out).reshape(p.K, 2, p.L + 1)
    err = np.abs((got - ph) - (ref - ph)).max() / np.abs(ref - ph).max()
    say("correction rel err %.2e" % err)
    assert err < 1e-10
    r = S.solve("fpsa", tol=1e-11, max_iter=500, q_ext=dev(torch, p.q))
    torch.cuda.synchronize()
    ro = oracle.solve(p, "fpsa", scheme, tol=1e-11, max_iter=500)
    err = np.abs(host(r["phi"]).reshape(ro["phi"].shape) - ro["phi"]).max() / np.abs(ro["phi"]).max()
    say("FPSA iterations", r["iters"][0], "oracle", ro["iters"], "rel err %.2e" % err)
    assert r["status"] == 0 and r["iters"][0] == ro["iters"] and err < 1e-10
    S.close()


@pytest.mark.parametrize("coef", ["cell", "mean"])
def test_one_type_fused_correction_vs_batched(torch, snfpsa, coef):
    """FPSA solves of single-type slabs slab by slab (the correction's
    Fokker-Planck source formed inside the additive-term kernel; with
    slab-mean coefficients the moment difference is scaled by sigma_s there)
    against the batched solve of the same handle, which runs the separate
    source GEMM: the same iteration counts and moments within 1e-10; and
    against the oracle's converged solution."""
    probs = [sw.random_slab(91 + b, K=K, N=N, regions=1, kernel=k, source="random", inflow="random",
                            c_range=(0.9, 0.99))
             for b, (K, N, k) in enumerate([(400, 16, "hg"), (257, 32, "srk"), (130, 64, "srk"), (64, 128, "hg")])]
    S = snfpsa.SlabSolver(probs, fp_scheme="wfd", fp_coefficients=coef)
    qe = torch.from_numpy(np.concatenate([p.q.ravel() for p in probs])).cuda()
    res = {}
    for batched in (True, False):
        S.set_batched_solve(batched)
        r = S.solve("fpsa", tol=1e-12, max_iter=3000, q_ext=qe)
        torch.cuda.synchronize()
        assert r["status"] == 0
        res[batched] = (r["iters"], host(r["phi"]))
    say("iterations", coef, res[True][0], res[False][0])
    assert res[True][0] == res[False][0]
    scale = np.abs(res[False][1]).max()
    assert np.abs(res[True][1] - res[False][1]).max() <= 1e-10 * scale
    off = 0
    for p in probs:
        n = p.K * 2 * (p.L + 1)
        ref = oracle.solve(p, "fpsa", "wfd", tol=1e-13, max_iter=5000)["phi"].ravel()
        got = res[False][1][off:off + n]
        off += n
        assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max(), (p.K, p.N)
    S.close()


@pytest.mark.parametrize("case", SLABS + LONG_SLABS, ids=lambda c: f"K{c[1]}N{c[2]}")
def test_sweep_adjoint(torch, snfpsa, case):
    p = _prob(*case)
    say("adjoint", case)
    S = snfpsa.SlabSolver([p])
    y = sw.random_vectors(30 + case[0], p.K, 2, p.N)
    x = sw.random_vectors(40 + case[0], p.K, 2, p.N)
    ya = S.psi_tensor()
    S.sweep_adjoint(dev(torch, y), ya)
    sx = S.psi_tensor()
    S.sweep(dev(torch, x), sx, bc="zero")
    torch.cuda.synchronize()
    ref = oracle.sweep_adjoint(y, p.h, p.sigma_t)
    got = host(ya).reshape(p.K, 2, p.N)
    assert rel(got, ref) < 1e-12
    lhs = float(np.sum(y.ravel() * host(sx)))
    rhs = float(np.sum(got.ravel() * x.ravel()))
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0)
    S.close()


def test_multi_slab_handle(torch, snfpsa):
    probs = [_prob(*SLABS[1]), _prob(*SLABS[3]), _prob(*SLABS[4])]
    say("multi-slab")
    S = snfpsa.SlabSolver(probs, fp_scheme="wfd")
    q = dev(torch, np.concatenate([p.q.ravel() for p in probs]))
    psi = S.psi_tensor()
    phi = S.phi_tensor()
    S.sweep(q, psi, phi)
    torch.cuda.synchronize()
    gp, gf = host(psi), host(phi)
    o1 = o2 = 0
    for p in probs:
        ref = oracle.sweep(p.q, p.h, p.sigma_t, p.psi_left, p.psi_right)
        n1, n2 = ref.size, p.K * 2 * (p.L + 1)
        assert rel(gp[o1:o1 + n1].reshape(ref.shape), ref) < 1e-12
        assert rel(gf[o2:o2 + n2].reshape(p.K, 2, p.L + 1), oracle.moments(ref, p.L)) < 1e-12
        o1 += n1
        o2 += n2
    res = S.solve("fpsa", tol=1e-11, max_iter=500, q_ext=q)
    phi = host(res["phi"])
    o2 = 0
    for b, p in enumerate(probs):
        r = oracle.solve(p, "fpsa", "wfd", tol=1e-11, max_iter=500)
        n2 = p.K * 2 * (p.L + 1)
        assert res["iters"][b] == r["iters"]
        assert rel(phi[o2:o2 + n2].reshape(r["phi"].shape), r["phi"]) < 1e-10
        o2 += n2
    S.close()


@pytest.mark.parametrize("method,scheme", [("si", "wfd"), ("fpsa", "wfd"), ("fpsa", "mpd")])
def test_solve_hg_slab_200(torch, snfpsa, method, scheme):
    """200 cells, S_8, HG g=0.9, c=0.99, incident flux on the left, 1e-10."""
    p = sw.hg_slab_200()
    say("solve hg_slab_200", method, scheme)
    S = snfpsa.SlabSolver([p], fp_scheme=scheme)
    ex = torch.zeros(S.exit_len, dtype=torch.float64, device="cuda")
    res = S.solve(method, tol=p.tol, max_iter=2000, psi_exit=ex)
    ref = oracle.solve(p, method, scheme, max_iter=2000)
    assert res["status"] == 0
    assert res["iters"][0] == ref["iters"]
    phi = host(res["phi"]).reshape(ref["phi"].shape)
    assert np.abs(phi - ref["phi"]).max() < 1e-10
    hist = res["hist"][0]
    assert np.abs(hist - ref["hist"]).max() < 1e-10 * max(ref["hist"].max(), 1.0)
    mu, _ = oracle.gauss_legendre(p.N)
    exit_ref = np.where(mu > 0, ref["psi"][-1, 1, :], ref["psi"][0, 0, :])
    assert np.abs(host(ex) - exit_ref).max() < 1e-10
    S.close()


def _golden():
    rec, smp = {}, {}
    with open(os.path.join(GOLDEN, "oracle_reference.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "record":
                rec[(t[1], t[2], t[3])] = (int(t[4]), float(t[5]), float(t[6]))
            else:
                smp.setdefault((t[1], t[2], t[3]), []).append((int(t[4]), int(t[5]), int(t[6]), float(t[7])))
    return rec, smp


@pytest.mark.parametrize("method,scheme", [("fpsa", "wfd"), ("fpsa", "mpd"), ("si", "wfd")])
def test_solve_srk_slab_2000(torch, snfpsa, method, scheme):
    """2000 cells, S_64, SRK eta=1e-5, L=63, c=0.999, q=1: the benchmark
    workload, against the stored oracle solves (iterations and sampled
    moments) and, for FPSA, against a fresh oracle FPSA solve."""
    rec, smp = _golden()
    p = sw.srk_slab_2000()
    say("solve srk_slab_2000", method, scheme)
    S = snfpsa.SlabSolver([p], fp_scheme=scheme)
    res = S.solve(method, tol=p.tol, max_iter=20000, q_ext=dev(torch, p.q))
    it, h0, hl = rec[(p.name, method, scheme)]
    assert res["status"] == 0
    assert res["iters"][0] == it
    hist = res["hist"][0]
    phi = host(res["phi"]).reshape(p.K, 2, p.L + 1)
    # the stopping-test value is a difference of moments of size |phi|, so
    # its FP64 noise floor is a few ulps of |phi|
    scale = np.abs(phi).max()
    assert abs(hist[0] - h0) < 1e-12 * scale and abs(hist[-1] - hl) < 1e-11 * scale
    for k, nu, l, v in smp[(p.name, method, scheme)]:
        assert abs(phi[k, nu, l] - v) < 1e-10 * max(abs(phi[:, :, 0]).max(), 1.0), (k, nu, l)
    if method == "fpsa":
        r = oracle.solve(p, method, scheme, max_iter=200)
        assert np.abs(phi - r["phi"]).max() < 1e-10 * np.abs(r["phi"]).max()
    S.close()


def test_not_converged_status(torch, snfpsa):
    p = sw.hg_slab_200()
    S = snfpsa.SlabSolver([p])
    res = S.solve("si", tol=1e-12, max_iter=5)
    assert res["status"] == snfpsa.SN_NOT_CONVERGED and res["iters"] == [5]
    ref = oracle.solve(p, "si", tol=1e-12, max_iter=5)
    assert np.abs(host(res["phi"]).reshape(ref["phi"].shape) - ref["phi"]).max() < 1e-12
    S.close()


def test_pl_equivalent_one_iteration_on_gpu(torch, snfpsa):
    """Sec. 3.2: P_L-equivalent moments make MPD-FPSA exact in one step."""
    N = 16
    p = sw.homogeneous("pl", K=100, width=5.0, N=N, L=N - 1, sigma_t=1.0,
                       moments=np.ones(N), c=1.0, source=1.0, psi_left=0.3)
    p.sigma_s = np.tile(sw.pl_equivalent_moments(0.99, 0.985, N - 1), (p.K, 1))
    S = snfpsa.SlabSolver([p], fp_scheme="mpd")
    res = S.solve("fpsa", tol=0.0, max_iter=2, q_ext=dev(torch, p.q))
    h = res["hist"][0]
    assert h[1] < 1e-11 * h[0]
    S.close()


@pytest.mark.parametrize("K,L", [(2100, 255), (2049, 200)])
def test_tall_gemm_large_slab(torch, snfpsa, K, L):
    """Slabs of >= 4096 LD-node rows with N = 256 take the tall FP64 GEMM
    (64 x 256 block tiles, K in chunks of 16): ragged row tiles and, for
    L = 200, a ragged K chunk in the source GEMM (the moments GEMM then has
    201 columns and stays on the general kernel)."""
    p = sw.random_slab(80 + K, K=K, N=256, L=L, regions=3, kernel="srk", source="random", c_range=(0.2, 0.4))
    say("tall gemm", K, L)
    S = snfpsa.SlabSolver([p], fp_scheme="none")
    phi = sw.random_vectors(K, p.K, 2, p.L + 1)
    for qe in (None, p.q):
        q = S.scatter_source(dev(torch, phi), None if qe is None else dev(torch, qe))
        torch.cuda.synchronize()
        ref = oracle.scatter_source(phi, p.sigma_s, p.N, qe)
        assert rel(host(q).reshape(p.K, 2, p.N), ref) < 1e-12
    psi = S.psi_tensor()
    ph = S.phi_tensor()
    S.sweep(dev(torch, p.q), psi, ph, bc="problem")
    torch.cuda.synchronize()
    ref = oracle.sweep(p.q, p.h, p.sigma_t, p.psi_left, p.psi_right)
    assert rel(host(psi).reshape(p.K, 2, p.N), ref) < 1e-12
    assert rel(host(ph).reshape(p.K, 2, p.L + 1), oracle.moments(ref, p.L)) < 1e-12
    if L < 255:
        S.close()
        return
    # source iteration with the stopping test fused into the tall moments GEMM
    r = S.solve("si", tol=1e-10, max_iter=200, q_ext=dev(torch, p.q))
    o = oracle.solve(p, "si", tol=1e-10, max_iter=200)
    assert r["iters"][0] == o["iters"]
    assert rel(host(r["phi"]).reshape(o["phi"].shape), o["phi"]) < 1e-10
    S.close()


@pytest.mark.parametrize("scheme", ["wfd", "mpd"])
def test_solve_fpsa_s128(torch, snfpsa, scheme):
    """FP64 FPSA at N = 128 (the LDS-ring chain with 64-wide steps, the
    unfused sweep and separate GEMMs) against the oracle: same iteration
    count, moments within 1e-10."""
    p = sw.random_slab(77, K=300, N=128, regions=3, kernel="srk", source="uniform", inflow="random",
                       c_range=(0.9, 0.99))
    say("solve fpsa S_128", scheme)
    S = snfpsa.SlabSolver([p], fp_scheme=scheme)
    res = S.solve("fpsa", tol=1e-10, max_iter=500, q_ext=dev(torch, p.q))
    ref = oracle.solve(p, "fpsa", scheme, tol=1e-10, max_iter=500)
    say("iterations", res["iters"][0], "oracle", ref["iters"])
    assert res["status"] == 0 and res["iters"][0] == ref["iters"]
    phi = host(res["phi"]).reshape(ref["phi"].shape)
    assert np.abs(phi - ref["phi"]).max() < 1e-10 * np.abs(ref["phi"]).max()
    S.close()
