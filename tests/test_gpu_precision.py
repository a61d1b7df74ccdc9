"""The precision ladder on the single large slab: 2^20 cells, S_256, L = 255,
screened-Rutherford eta = 1e-6, c = 0.9999, 16 random regions.

At this size the oracle cannot run the GEMMs of a solve in seconds, so the
checks are:
- the FP64 path's sweep over every cell and angle against the oracle's sweep;
- every precision's scattering source against the oracle on sampled cells:
  both boundary layers, both sides of every region interface, random
  interior cells;
- the FP32 and split-BF16 sweeps against the oracle's sweep of the same
  FP32-rounded source;
- ten source iterations in FP32 and split-BF16 against the same iterations
  in FP64, whose every step was checked above.

FP64 bounds are the rounding of a 2^20-cell recurrence and of a 256-term
dot product (1e-12); FP32 and split-BF16 bounds are those of the batched
path (5e-5 sweep, 2e-5 / 1e-4 scattering source) and 2e-5 for the moments
after ten iterations (the FP32 target is 1e-5 relative)."""
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


@pytest.fixture(scope="module")
def slab():
    return sw.large_slab()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def sample_cells(p, n=48, seed=7):
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = np.flatnonzero(np.diff(p.sigma_t))
    return np.unique(np.concatenate([np.arange(8), p.K - 1 - np.arange(8), edges, edges + 1,
                                     rng.choice(p.K, size=n, replace=False)]))


def test_large_slab_shape(slab):
    p = slab
    assert (p.K, p.N, p.L) == (1 << 20, 256, 255)
    assert len(np.unique(p.sigma_t)) == 16
    # screened Rutherford with c = 0.9999: sigma_{s,0} = c sigma_t, moments
    # decreasing in l
    assert np.allclose(p.sigma_s[:, 0], 0.9999 * p.sigma_t, rtol=1e-14)
    assert np.all(np.diff(p.sigma_s[0]) < 0)


@pytest.mark.parametrize("precision,tol_sweep,tol_src", [("f64", 1e-12, 1e-12), ("f32", 5e-5, 2e-5),
                                                         ("bf16x3", 5e-5, 1e-4)])
def test_large_slab_sweep_and_scatter(torch, snfpsa, slab, precision, tol_sweep, tol_src):
    p = slab
    K, N, L1 = p.K, p.N, p.L + 1
    cells = sample_cells(p)
    say("large slab", precision, "K", K, "N", N, "L1", L1, "sampled cells", len(cells))
    S = snfpsa.SlabSolver([p], fp_scheme="none", precision=precision)
    qn = sw.random_vectors(61, K, 2, N)
    if precision != "f64":
        qn = qn.astype(np.float32).astype(np.float64)
    q = torch.from_numpy(qn).to(device="cuda", dtype=S.qdtype)
    psi = S.psi_tensor()
    S.sweep(q, psi, None, bc="problem")
    torch.cuda.synchronize()
    del q
    got = host(psi).reshape(K, 2, N)
    del psi
    ref = oracle.sweep(qn, p.h, p.sigma_t)
    del qn
    e = rel(got, ref)
    say("sweep rel err", e)
    assert e < tol_sweep
    del got, ref
    phin = sw.random_vectors(62, K, 2, L1)
    phi = torch.from_numpy(phin).cuda()
    qo = S.scatter_source(phi, None)
    torch.cuda.synchronize()
    del phi
    got = host(qo).reshape(K, 2, N)[cells]
    del qo
    ref = oracle.scatter_source(phin[cells], p.sigma_s[cells], N)
    e = rel(got, ref)
    say("scatter rel err (sampled)", e)
    assert e < tol_src
    S.close()
    torch.cuda.empty_cache()


def test_large_slab_si_ladder(torch, snfpsa, slab):
    """Ten source iterations from zero with q = 1 in every precision; the
    FP32 and split-BF16 moments stay within 2e-5 of the FP64 ones."""
    p = slab
    res = {}
    for prec in ("f64", "f32", "bf16x3"):
        say("large slab SI x10", prec)
        S = snfpsa.SlabSolver([p], fp_scheme="none", precision=prec)
        q = torch.ones(S.psi_len, dtype=S.qdtype, device="cuda")
        phi = S.phi_tensor()
        phi.zero_()
        r = S.solve("si", tol=0.0, max_iter=10, q_ext=q, phi=phi)
        assert r["iters"][0] == 10
        torch.cuda.synchronize()
        res[prec] = host(phi)
        del q, phi
        S.close()
        torch.cuda.empty_cache()
    for prec in ("f32", "bf16x3"):
        e = rel(res[prec], res["f64"])
        say(prec, "phi rel err vs f64", e)
        assert e < 2e-5


def test_reduced_slab_ladder_against_oracle(torch, snfpsa):
    """The large slab's recipe at 2048 cells (4096 LD-node rows, so the FP64
    path takes its tall GEMM; S_256, L = 255, eta = 1e-6, c = 0.9999, 16
    regions, q = 1, vacuum): ten source iterations from zero in FP64, FP32
    and split-BF16 against ten iterations of the oracle.  FP64 within 1e-12
    of the largest moment; FP32 and split-BF16 within 2e-5, each error
    printed."""
    p = sw.large_slab(K=2048, with_source=True)
    say("reduced large slab: oracle, 10 source iterations")
    ref = oracle.solve(p, "si", tol=0.0, max_iter=10)["phi"]
    for prec, bound in (("f64", 1e-12), ("f32", 2e-5), ("bf16x3", 2e-5)):
        S = snfpsa.SlabSolver([p], fp_scheme="none", precision=prec)
        q = torch.ones(S.psi_len, dtype=S.qdtype, device="cuda")
        r = S.solve("si", tol=0.0, max_iter=10, q_ext=q)
        assert r["iters"][0] == 10
        e = rel(host(r["phi"]).reshape(ref.shape), ref)
        say("reduced large slab", prec, "phi rel err vs oracle %.3e" % e)
        assert e < bound, prec
        S.close()
