"""The allocation-free correction (fpsa_correct_noalloc) against fpsa_correct
through the C ABI: the same kernels on the same inputs, with the work vectors
in the library's fixed per-device scratch instead of the handle's workspace.
Two calls in a row on different handles, the second with a smaller input,
so the scratch carries the first call's contents into the second; a slab too
large for the scratch is rejected."""
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


def _case(torch, snfpsa, probs, scheme, seed):
    S = snfpsa.SlabSolver(probs, fp_scheme=scheme)
    ph = torch.from_numpy(np.concatenate([sw.random_vectors(seed + b, p.K, 2, p.L + 1).ravel()
                                          for b, p in enumerate(probs)])).cuda()
    po = torch.from_numpy(np.concatenate([sw.random_vectors(seed + 50 + b, p.K, 2, p.L + 1).ravel()
                                          for b, p in enumerate(probs)])).cuda()
    ref = S.fpsa_correct(ph, po)
    got = torch.full_like(ref, float("nan"))
    S.fpsa_correct_noalloc(ph, po, got)
    torch.cuda.synchronize()
    d = ref - ph
    err = float((got - ref).abs().max()) / max(float(d.abs().max()), 1e-300)
    return S, err


def test_noalloc_correction_matches_fpsa_correct(torch, snfpsa):
    big = [sw.random_slab(501, K=2000, N=64, regions=3, kernel="srk", source="random"),
           sw.random_slab(502, K=300, N=16, regions=2, kernel="hg", source="random"),
           sw.random_slab(504, K=515, N=32, regions=1, kernel="srk", source="random")]
    small = [sw.random_slab(503, K=37, N=8, regions=2, kernel="hg", source="random")]
    say("noalloc: first call, 3 slabs (2000 x S_64, 300 x S_16, 515 x S_32 of one cell type), WFD")
    S1, e1 = _case(torch, snfpsa, big, "wfd", 10)
    say("noalloc: first call rel diff", e1)
    say("noalloc: second call, 1 slab (37 x S_8), MPD")
    S2, e2 = _case(torch, snfpsa, small, "mpd", 20)
    say("noalloc: second call rel diff", e2)
    # the same kernels in the same order: identical up to FP64 rounding
    assert e1 < 1e-13 and e2 < 1e-13
    S1.close()
    S2.close()


def test_noalloc_correction_rejects_oversized_slab(torch, snfpsa):
    # 1.5e6 cells x S_2: about 96 MB of work vectors (> 64 MiB); rejected
    # before any kernel runs
    p = sw.homogeneous("big", K=1500000, width=15000.0, N=2, L=1, sigma_t=1.0,
                       moments=np.array([1.0, 0.9]), c=0.9, source=1.0, psi_left=0.0)
    say("noalloc: oversized slab", p.K, p.N)
    S = snfpsa.SlabSolver([p], fp_scheme="wfd")
    ph = S.phi_tensor().zero_()
    po = S.phi_tensor().zero_()
    out = S.phi_tensor()
    with pytest.raises(snfpsa.SnError) as e:
        S.fpsa_correct_noalloc(ph, po, out)
    assert e.value.status == snfpsa.SN_E_INVALID and "scratch" in str(e.value)
    S.close()
