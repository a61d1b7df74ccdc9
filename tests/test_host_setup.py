"""CPU checks of the HIP library's host side: exported symbols and the FP64
setup math (no device work)."""
import os
import re

import numpy as np
import pytest

import oracle
import sn_workloads as sw

snfpsa = pytest.importorskip("paper_1907_13013_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for hdr in ("snfpsa.h", "snfpsa_diag.h"):
        txt = open(os.path.join(ROOT, "include", hdr)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(?:sn_status|const char\s*\*)\s*([a-z_0-9]+)\s*\(", txt):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = snfpsa.load_library()
    declared = _declared_functions()
    assert {"sn_setup", "sn_sweep", "sn_scatter_source", "fpsa_correct", "sn_solve",
            "sn_sweep_adjoint", "sn_destroy", "sn_last_error"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert declared <= set(snfpsa.EXPORTS)


@pytest.mark.parametrize("N", [2, 8, 16, 64, 256])
def test_library_quadrature(N):
    mu, w = snfpsa.diag_quadrature(N)
    m2, w2 = np.polynomial.legendre.leggauss(N)
    assert np.abs(mu - m2).max() < 2e-15 and np.abs((w - w2) / w2).max() < 1e-10
    for k in range(0, 2 * N, max(1, (2 * N) // 16)):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, mu ** k) - exact) < 1e-13


@pytest.mark.parametrize("N", [8, 64, 256])
def test_library_quadrature_against_extended_precision(N):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    mu, w = snfpsa.diag_quadrature(N)
    for i in (0, 1, N // 3):
        x = mpmath.findroot(lambda t: mpmath.legendre(N, t), mpmath.mpf(mu[i]))
        dp = mpmath.diff(lambda t: mpmath.legendre(N, t), x)
        wx = 2 / ((1 - x * x) * dp * dp)
        assert abs(float(mu[i] - x)) < 1e-16
        assert abs(float((w[i] - wx) / wx)) < 1e-12


@pytest.mark.parametrize("N", [4, 16, 64])
@pytest.mark.parametrize("scheme", ["wfd", "mpd"])
def test_library_laplacians_match_oracle(N, scheme):
    A = snfpsa.diag_laplacian(N, scheme)
    R = oracle.wfd_matrix(N) if scheme == "wfd" else oracle.mpd_matrix(N)
    assert np.abs(A - R).max() < 1e-11 * max(1.0, np.abs(R).max())


def apply_factors(F, prob, dphi, chunked):
    """NumPy model of the library's FP correction: phi_new - phi_half, the
    correction's outflow b_0 at the left face and a_K at the right face.

    Two Riccati eliminations (from the left: a = rho b + p, from the right:
    b = sig a + q) combined at each interface, in one of three orders:
    plain sequential recursions (False), chunked with sequential carries
    (True) or the kernels' scheme ("parallel": local chains from zero, carries
    through the transfer products, fix-up through the prefix products)."""
    K, N, L = prob.K, prob.N, prob.L
    NH = N // 2
    L2 = 2 * (L + 1)
    d = dphi.reshape(K, L2)
    s = np.zeros((K, N))
    sb, stp = F["seg_begin"], F["seg_type"]
    for g in range(len(stp)):
        s[sb[g]:sb[g + 1]] = d[sb[g]:sb[g + 1]] @ F["EsrcT"][stp[g]]
    cm = F["cellmats"]
    G, Hm, Gb, Hb, W, Wr, Sg = (cm[:, i] for i in range(7))
    sp, sm = s[:, :NH], s[:, NH:]
    fv = np.einsum("kij,kj->ki", Hm, sm) + sp
    gv = np.einsum("kij,kj->ki", Hb, sp) + sm
    p = np.zeros((K + 1, NH))
    q = np.zeros((K + 1, NH))
    ch, nc = F["chunk"], F["nchunks"]
    lo = lambda c: c * ch
    hi = lambda c: min(K, c * ch + ch)
    if not chunked:
        for j in range(K):
            p[j + 1] = G[j] @ p[j] + fv[j]
        for j in range(K - 1, -1, -1):
            q[j] = Gb[j] @ q[j + 1] + gv[j]
    elif chunked == "parallel":
        tri = lambda a: (a - 1) * (a - 2) // 2
        ploc = np.zeros((K + 1, NH))
        e = np.zeros((nc, NH))
        for c in range(nc):
            v = np.zeros(NH)
            for j in range(lo(c), hi(c)):
                ploc[j] = v
                v = G[j] @ v + fv[j]
            e[c] = v
        carry = np.zeros((nc + 1, NH))
        for c in range(1, nc + 1):
            carry[c] = e[c - 1] + sum(F["theta_fwd"][tri(c) + cp] @ e[cp] for cp in range(c - 1))
        for j in range(K):
            p[j] = ploc[j] + F["psi_fwd"][j] @ carry[j // ch]
        p[K] = carry[nc]
        qloc = np.zeros((K + 1, NH))
        e2 = np.zeros((nc, NH))
        for c in range(nc):
            v = np.zeros(NH)
            for j in range(hi(c) - 1, lo(c) - 1, -1):
                v = Gb[j] @ v + gv[j]
                qloc[j] = v
            e2[c] = v
        carry2 = np.zeros((nc, NH))
        for c in range(nc - 1):
            a = nc - 1 - c
            carry2[c] = e2[c + 1] + sum(F["theta_bwd"][tri(a) + (nc - 1 - cp)] @ e2[cp]
                                        for cp in range(c + 2, nc))
        for j in range(K):
            q[j] = qloc[j] + F["psi_bwd"][j] @ carry2[j // ch]
    else:
        e = np.zeros((nc, NH))
        for c in range(nc):
            v = np.zeros(NH)
            for j in range(lo(c), hi(c)):
                v = G[j] @ v + fv[j]
            e[c] = v
        for c in range(nc):
            v = np.zeros(NH)
            for cc in range(c):
                v = F["chunk_fwd"][cc] @ v + e[cc]
            for j in range(lo(c), hi(c)):
                p[j] = v
                v = G[j] @ v + fv[j]
            if hi(c) == K:
                p[K] = v
        e2 = np.zeros((nc, NH))
        for c in range(nc):
            v = np.zeros(NH)
            for j in range(hi(c) - 1, lo(c) - 1, -1):
                v = Gb[j] @ v + gv[j]
            e2[c] = v
        for c in range(nc):
            v = np.zeros(NH)
            for cc in range(nc - 1, c, -1):
                v = F["chunk_bwd"][cc] @ v + e2[cc]
            for j in range(hi(c) - 1, lo(c) - 1, -1):
                v = Gb[j] @ v + gv[j]
                q[j] = v
    a = np.einsum("kij,kj->ki", W, p[:K]) + np.einsum("kij,kj->ki", Wr, q[:K])
    b = np.zeros((K + 1, NH))
    b[:K] = np.einsum("kij,kj->ki", Sg, a) + q[:K]
    inflow = np.concatenate([a, b[1:K + 1]], axis=1)
    out = np.zeros((K, L2))
    for g in range(len(stp)):
        r = slice(sb[g], sb[g + 1])
        out[r] = d[r] @ F["PhisrcT"][stp[g]] + inflow[r] @ F["PhiinfT"][stp[g]]
    return out.reshape(K, 2, L + 1), b[0], p[K]


@pytest.mark.parametrize("scheme", ["wfd", "mpd"])
@pytest.mark.parametrize("kernel,N,K,regions,chunk", [("hg", 8, 23, 3, 5), ("srk", 16, 40, 4, 0),
                                                      ("hg", 4, 7, 1, 3), ("srk", 32, 64, 2, 0)])
def test_fp_factorisation_reproduces_oracle_correction(scheme, kernel, N, K, regions, chunk):
    prob = sw.random_slab(100 + N + K, K=K, N=N, regions=regions, kernel=kernel, source="random")
    L = prob.L
    phi_half = sw.random_vectors(1, K, 2, L + 1)
    phi_old = sw.random_vectors(2, K, 2, L + 1)
    ref, U = oracle.fpsa_correct(prob, phi_half, phi_old, scheme)
    F = snfpsa.diag_fp_factors(K, N, L, prob.h, prob.sigma_t, prob.sigma_s, scheme, chunk)
    assert F["ntypes"] == regions or regions > K
    for chunked in (False, True, "parallel"):
        corr, b0, pK = apply_factors(F, prob, phi_half - phi_old, chunked)
        got = phi_half + corr
        scale = np.abs(ref - phi_half).max()
        assert np.abs(got - ref).max() < 1e-11 * max(scale, 1.0), chunked
        # correction outflow at the faces equals the oracle's U there
        assert np.abs(b0 - U[0, 0, : N // 2]).max() < 1e-11 * max(np.abs(U).max(), 1.0)
        assert np.abs(pK - U[-1, 1, N // 2:]).max() < 1e-11 * max(np.abs(U).max(), 1.0)
