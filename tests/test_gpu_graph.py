"""Graph replay of the batched source iteration against its eager launches.

A batched handle captures the kernels of one source iteration into a HIP
graph (they find the current iteration through a device counter) and
replays it once per iteration.  The replayed solve must reproduce the eager
solve bit for bit: the same moments, the same per-slab iteration counts and
stopping-test history, the same exit fluxes.  Each graph is replayed many
times within a solve and reused across solves from the cache, with eager
work of the program in between; changing a baked-in argument (tolerance,
sweep decomposition) must give a new graph with the eager result again."""
import sys

import numpy as np
import pytest

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
    return t.detach().cpu().numpy()


# uneven batch: short and long slabs (the 30000-cell one is swept in
# segments with a carry scan), N from 8 to 128
CASES = [(81, 30000, 32, 3, "hg"), (82, 1, 8, 1, "srk"), (83, 200, 16, 3, "hg"), (84, 513, 64, 2, "srk"),
         (85, 65, 128, 2, "hg"), (86, 37, 8, 2, "hg"), (87, 900, 16, 4, "srk")]


def _probs():
    return [sw.random_slab(s, K=K, N=N, regions=r, kernel=k, source="uniform", inflow="random",
                           c_range=(0.3, 0.9)) for s, K, N, r, k in CASES]


def _solve(torch, S, qe, tol, max_iter=400):
    ex = torch.zeros(S.exit_len, dtype=torch.float32, device="cuda")
    r = S.solve("si", tol=tol, max_iter=max_iter, q_ext=qe, psi_exit=ex)
    torch.cuda.synchronize()
    return host(r["phi"]).copy(), list(r["iters"]), [np.array(h) for h in r["hist"]], host(ex).copy(), r["status"]


def _same(a, b):
    assert a[4] == b[4]
    assert a[1] == b[1], (a[1], b[1])
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[3], b[3])
    for x, y in zip(a[2], b[2]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("precision", ["f32", "bf16x3"])
def test_graph_replay_matches_eager(torch, snfpsa, precision):
    probs = _probs()
    say("graph replay vs eager", precision)
    S = snfpsa.SlabSolver(probs, fp_scheme="none", precision=precision)
    qe = torch.from_numpy(np.concatenate([p.q.ravel() for p in probs]).astype(np.float32)).cuda()
    for choice in (S.sweep_tuning()["choice"], 0, 2):
        S.set_sweep_choice(choice)
        for tol in (1e-5, 3e-7):
            S.set_graph_replay(False)
            eager = _solve(torch, S, qe, tol)
            S.set_graph_replay(True)
            first = _solve(torch, S, qe, tol)          # captured here
            # eager work of the program between graph solves
            psi = S.psi_tensor()
            S.sweep(qe, psi, None, bc="problem")
            torch.cuda.synchronize()
            again = _solve(torch, S, qe, tol)          # cached graph
            say("choice", choice, "tol", tol, "iterations", eager[1])
            assert len(set(eager[1])) > 1              # slabs stop at different iterations
            _same(first, eager)
            _same(again, eager)
    # an iteration limit below convergence: NOT_CONVERGED in both modes
    S.set_graph_replay(False)
    eager = _solve(torch, S, qe, 1e-9, max_iter=7)
    S.set_graph_replay(True)
    graph = _solve(torch, S, qe, 1e-9, max_iter=7)
    assert eager[4] == snfpsa.SN_NOT_CONVERGED
    _same(graph, eager)
    S.close()


def test_graph_replay_rejects_f64_handles(torch, snfpsa):
    p = sw.random_slab(88, K=20, N=8, regions=1, kernel="hg")
    S = snfpsa.SlabSolver([p], fp_scheme="none")
    with pytest.raises(snfpsa.SnError) as e:
        S.set_graph_replay(True)
    assert e.value.status == snfpsa.SN_E_STATE
    S.close()
