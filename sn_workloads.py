"""Seeded synthetic slab problems for the S_N / FPSA solvers.

This module only builds problem *inputs*: cell widths, total cross sections,
Legendre scattering moments sigma_{s,l}, boundary inflows and nodal sources.
It holds none of the solver arithmetic (no quadrature set, no sweep, no
Fokker-Planck operator); both the HIP library and the CPU oracle consume the
arrays produced here, and nothing here imports either of them.

Problem statement (paper, Sec. 2, eq:trans / eq:trans-equation-bc / eq:treq):
  mu dpsi/dz + sigma_t psi = sum_l (2l+1)/2 sigma_{s,l} P_l(mu) phi_l + q,
  psi(z0, mu>0) = psi_L(mu), psi(z1, mu<0) = psi_R(mu),
with sigma_{s,l} = int_{-1}^{1} sigma_s(mu0) P_l(mu0) dmu0 truncated at l = L.

Scattering kernels (paper, Sec. 3.4 and Sec. 4):
  Henyey-Greenstein:      sigma_{s,l} = c sigma_t g^l
  screened Rutherford:    sigma_s(mu0) proportional to (1 + 2 eta - mu0)^-2,
                          sigma_{s,l} = c sigma_t f_l(eta), f_0 = 1.
  P_L-equivalent moments: sigma_{s,l} = sigma_{s,0} - (sigma_tr/2) l (l+1)
                          (paper, Sec. 3.2, eq:fsa_pl_eq).

Array layouts (per slab, cells k = 0..K-1, LD nodes nu in {left, right},
angles n = 0..N-1 in ascending mu order):
  h[K], sigma_t[K], sigma_s[K, L+1], q[K, 2, N] (or None = zero source),
  psi_left[N/2]  inflow at z0 for the N/2 positive cosines (ascending),
  psi_right[N/2] inflow at z1 for the N/2 negative cosines (ascending).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED = 1907130130


@dataclasses.dataclass
class SlabProblem:
    name: str
    K: int
    N: int
    L: int
    h: np.ndarray
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    psi_left: np.ndarray
    psi_right: np.ndarray
    q: Optional[np.ndarray] = None
    tol: float = 1e-10
    meta: dict = dataclasses.field(default_factory=dict)

    def q_or_zero(self) -> np.ndarray:
        if self.q is None:
            return np.zeros((self.K, 2, self.N))
        return self.q

    def validate(self) -> None:
        assert self.N % 2 == 0 and self.N >= 2
        assert 0 <= self.L <= self.N - 1
        assert self.h.shape == (self.K,) and self.sigma_t.shape == (self.K,)
        assert self.sigma_s.shape == (self.K, self.L + 1)
        assert self.psi_left.shape == (self.N // 2,)
        assert self.psi_right.shape == (self.N // 2,)
        if self.q is not None:
            assert self.q.shape == (self.K, 2, self.N)


# ---------------------------------------------------------------------------
# Scattering-kernel moments
# ---------------------------------------------------------------------------

def hg_moments(g: float, L: int) -> np.ndarray:
    """Normalised Henyey-Greenstein Legendre moments f_l = g^l, l = 0..L."""
    return np.power(float(g), np.arange(L + 1, dtype=np.float64))


def _legendre_upto(L: int, x: np.ndarray) -> np.ndarray:
    """P_0..P_L at points x (Bonnet recurrence); shape (L+1, len(x))."""
    P = np.empty((L + 1, x.size))
    P[0] = 1.0
    if L >= 1:
        P[1] = x
    for l in range(1, L):
        P[l + 1] = ((2 * l + 1) * x * P[l] - l * P[l - 1]) / (l + 1)
    return P


def srk_moments(eta: float, L: int, panels: Optional[int] = None,
                points: int = 32) -> np.ndarray:
    """Normalised screened-Rutherford moments f_l(eta), l = 0..L, in FP64.

    With a = 1 + 2 eta the kernel k(mu0) = (a - mu0)^-2 integrates to
    1 / (2 eta (1 + eta)).  We evaluate g_l = 1 - f_l =
    int (1 - P_l(mu0)) k dmu0 / int k dmu0 after the substitution
    u = ln(a - mu0), which turns the near-singular peak at mu0 = 1 into a
    smooth integrand (1 - P_l(a - e^u)) e^-u on [ln 2 eta, ln(2 + 2 eta)].
    Composite Gauss-Legendre with `points` nodes per panel; the panel count
    scales with L so each panel spans a fraction of a P_L oscillation.
    """
    if eta <= 0:
        raise ValueError("eta must be positive")
    a = 1.0 + 2.0 * eta
    u0, u1 = math.log(2.0 * eta), math.log(2.0 + 2.0 * eta)
    if panels is None:
        panels = max(64, int(math.ceil((u1 - u0) * max(L, 1) / 3.0)))
    x, w = np.polynomial.legendre.leggauss(points)
    edges = np.linspace(u0, u1, panels + 1)
    mid = 0.5 * (edges[1:] + edges[:-1])
    half = 0.5 * (edges[1:] - edges[:-1])
    u = (mid[:, None] + half[:, None] * x[None, :]).ravel()
    wu = (half[:, None] * w[None, :]).ravel()
    mu0 = a - np.exp(u)
    mu0 = np.clip(mu0, -1.0, 1.0)
    P = _legendre_upto(L, mu0)
    weight = wu * np.exp(-u)
    g = (1.0 - P) @ weight
    norm = 2.0 * eta * (1.0 + eta)
    f = 1.0 - norm * g
    f[0] = 1.0
    return f


def srk_f1_closed_form(eta: float) -> float:
    """f_1(eta) = 1 + 2 eta - 2 eta (1 + eta) ln(1 + 1/eta) (exact integral)."""
    return 1.0 + 2.0 * eta - 2.0 * eta * (1.0 + eta) * math.log1p(1.0 / eta)


def pl_equivalent_moments(sigma_s0: float, sigma_s1: float, L: int) -> np.ndarray:
    """P_L-equivalent moments sigma_{s,0} - (sigma_tr/2) l (l+1) (eq:fsa_pl_eq)."""
    l = np.arange(L + 1, dtype=np.float64)
    return sigma_s0 - 0.5 * (sigma_s0 - sigma_s1) * l * (l + 1)


# ---------------------------------------------------------------------------
# Problem builders
# ---------------------------------------------------------------------------

def homogeneous(name: str, K: int, width: float, N: int, L: int,
                sigma_t: float, moments: np.ndarray, c: float,
                source: float = 0.0, psi_left: float = 0.0,
                psi_right: float = 0.0, tol: float = 1e-10) -> SlabProblem:
    """Uniform slab with sigma_{s,l} = c sigma_t f_l on every cell."""
    f = np.asarray(moments, dtype=np.float64)[: L + 1]
    h = np.full(K, width / K)
    st = np.full(K, float(sigma_t))
    ss = np.tile(c * sigma_t * f, (K, 1))
    q = None if source == 0.0 else np.full((K, 2, N), float(source))
    return SlabProblem(name, K, N, L, h, st, ss,
                       np.full(N // 2, float(psi_left)),
                       np.full(N // 2, float(psi_right)), q, tol)


def hg_slab_200() -> SlabProblem:
    """10 mfp slab, 200 cells, S_8, HG g=0.9 to L=7, c=0.99, incident flux 1
    on the left, vacuum right, no interior source; 1e-10 stopping test."""
    return homogeneous("hg_slab_200", K=200, width=10.0, N=8, L=7, sigma_t=1.0,
                       moments=hg_moments(0.9, 7), c=0.99, psi_left=1.0,
                       tol=1e-10)


def srk_slab_2000() -> SlabProblem:
    """100 mfp slab, 2000 cells, S_64, screened Rutherford eta=1e-5 to L=63,
    c=0.999, uniform source q_n = 1, vacuum boundaries; 1e-8 stopping test."""
    return homogeneous("srk_slab_2000", K=2000, width=100.0, N=64, L=63,
                       sigma_t=1.0, moments=srk_moments(1e-5, 63), c=0.999,
                       source=1.0, tol=1e-8)


def random_regions(rng: np.random.Generator, K: int, R: int) -> np.ndarray:
    """Region index per cell: R contiguous regions split at sorted distinct
    random cell indices."""
    R = max(1, min(R, K))
    cuts = np.sort(rng.choice(np.arange(1, K), size=R - 1, replace=False)) if R > 1 else np.array([], dtype=int)
    reg = np.zeros(K, dtype=np.int64)
    for r, c0 in enumerate(cuts):
        reg[c0:] = r + 1
    return reg


def random_slab(seed: int, K: int, N: int, L: Optional[int] = None,
                regions: int = 3, kernel: str = "hg", h: float = 0.05,
                source: str = "uniform", inflow: str = "random",
                c_range=(0.9, 0.999), sigma_range=(0.5, 5.0),
                name: Optional[str] = None) -> SlabProblem:
    """Heterogeneous test slab: piecewise-constant sigma_t and c over random
    regions, HG or SRK moments, random or uniform source and inflows."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = N - 1 if L is None else L
    reg = random_regions(rng, K, regions)
    R = int(reg.max()) + 1
    st_r = rng.uniform(*sigma_range, size=R)
    c_r = rng.uniform(*c_range, size=R)
    if kernel == "hg":
        g = rng.uniform(0.8, 0.99)
        f = hg_moments(g, L)
        meta = {"kernel": "hg", "g": g}
    elif kernel == "srk":
        eta = 10.0 ** rng.uniform(-5, -3)
        f = srk_moments(eta, L)
        meta = {"kernel": "srk", "eta": eta}
    elif kernel == "iso":
        f = np.zeros(L + 1)
        f[0] = 1.0
        meta = {"kernel": "iso"}
    else:
        raise ValueError(kernel)
    st = st_r[reg]
    ss = (c_r[reg] * st_r[reg])[:, None] * f[None, :]
    hh = np.full(K, float(h))
    if source == "uniform":
        q = np.ones((K, 2, N))
    elif source == "random":
        q = rng.uniform(0.0, 2.0, size=(K, 2, N))
    elif source == "none":
        q = None
    else:
        raise ValueError(source)
    if inflow == "random":
        pl = rng.uniform(0.0, 1.0, size=N // 2)
        pr = rng.uniform(0.0, 1.0, size=N // 2)
    else:
        pl = np.zeros(N // 2)
        pr = np.zeros(N // 2)
    meta.update({"regions": R, "seed": seed})
    return SlabProblem(name or f"random_{kernel}_{K}x{N}_s{seed}", K, N, L, hh,
                       st, ss, pl, pr, q, 1e-10, meta)


def batched_slabs(count: int = 4096, seed: int = SEED, k_range=(256, 8192),
                  n_choices=(16, 32, 64, 128), with_source: bool = True) -> List[SlabProblem]:
    """Batch of independent uneven slabs: K uniform in k_range, N from
    n_choices (L = N-1), HG (g in [0.8,0.99]) on even slabs and screened
    Rutherford (eta log-uniform in [1e-7,1e-3]) on odd slabs, c in
    [0.9,0.9999], 1-8 random regions with sigma_t in [0.5,5], h = 0.05,
    q = 1, vacuum.  with_source=False leaves q empty (a caller that builds
    the uniform source on the device saves the host arrays)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(count):
        K = int(rng.integers(k_range[0], k_range[1] + 1))
        N = int(rng.choice(n_choices))
        L = N - 1
        c = rng.uniform(0.9, 0.9999)
        if b % 2 == 0:
            g = rng.uniform(0.8, 0.99)
            f = hg_moments(g, L)
            meta = {"kernel": "hg", "g": g}
        else:
            eta = 10.0 ** rng.uniform(-7, -3)
            f = srk_moments(eta, L)
            meta = {"kernel": "srk", "eta": eta}
        reg = random_regions(rng, K, int(rng.integers(1, 9)))
        st_r = rng.uniform(0.5, 5.0, size=int(reg.max()) + 1)
        st = st_r[reg]
        ss = (c * st)[:, None] * f[None, :]
        meta["c"] = c
        out.append(SlabProblem(f"batch{b}", K, N, L, np.full(K, 0.05), st, ss,
                               np.zeros(N // 2), np.zeros(N // 2),
                               np.ones((K, 2, N)) if with_source else np.zeros(0), 1e-8, meta))
    return out


def large_slab(K: int = 1 << 20, N: int = 256, L: int = 255, eta: float = 1e-6, c: float = 0.9999,
               regions: int = 16, seed: int = SEED, with_source: bool = False) -> SlabProblem:
    """Single large slab: K cells of width 0.05, S_N, screened Rutherford
    (eta) expanded to L, scattering ratio c, sigma_t uniform in [0.5, 5] over
    `regions` random regions, q = 1, vacuum.  with_source=False leaves q empty
    (the caller builds the uniform source on the device)."""
    rng = np.random.Generator(np.random.PCG64(seed + 4))
    reg = random_regions(rng, K, regions)
    st_r = rng.uniform(0.5, 5.0, size=int(reg.max()) + 1)
    st = st_r[reg]
    f = srk_moments(eta, L)
    ss = (c * st)[:, None] * f[None, :]
    return SlabProblem(f"large{K}", K, N, L, np.full(K, 0.05), st, ss, np.zeros(N // 2), np.zeros(N // 2),
                       np.ones((K, 2, N)) if with_source else np.zeros(0), 1e-8,
                       {"kernel": "srk", "eta": eta, "c": c, "regions": regions})


def random_vectors(seed: int, *shape) -> np.ndarray:
    """Seeded uniform(-1, 1) FP64 array (adjoint tests, power iteration)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=shape)


def cellwise_hg_slab(seed: int, K: int = 4096, N: int = 64, L: Optional[int] = None, g: float = 0.95,
                     sigma_range=(0.5, 2.0), c_range=(0.95, 0.999), h: float = 0.05,
                     source: str = "uniform", with_source: bool = True) -> SlabProblem:
    """Slab heterogeneous from cell to cell: sigma_t and c drawn per cell
    (uniform in the given ranges), Henyey-Greenstein moments
    sigma_{s,l} = c sigma_t g^l with the same g in every cell, q = 1 (or
    none), vacuum.  meta holds the per-cell parameters "c" and "g" (arrays),
    from which sigma_t and sigma_s are rebuilt when they are differentiated."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = N - 1 if L is None else L
    st = rng.uniform(*sigma_range, size=K)
    c = rng.uniform(*c_range, size=K)
    gc = np.full(K, float(g))
    ss = (c * st)[:, None] * gc[:, None] ** np.arange(L + 1)[None, :]
    q = None
    if source == "uniform":
        q = np.ones((K, 2, N)) if with_source else np.zeros(0)
    return SlabProblem(f"cellwise_hg_{K}x{N}_s{seed}", K, N, L, np.full(K, float(h)), st, ss,
                       np.zeros(N // 2), np.zeros(N // 2), q, 1e-12,
                       {"kernel": "hg", "c": c, "g": gc, "seed": seed})


def differentiation_batch(count: int = 256, K: int = 4096, N: int = 64, g: float = 0.95, seed: int = SEED,
                          with_source: bool = False) -> List[SlabProblem]:
    """Batch for gradients: `count` slabs of K cells, S_N with L = N-1,
    Henyey-Greenstein g in every cell, per-cell sigma_t ~ U[0.5, 2] and
    c ~ U[0.95, 0.999], h = 0.05, q = 1, vacuum.  with_source=False leaves q
    empty (the caller builds the uniform source on the device)."""
    return [cellwise_hg_slab(seed + 7 + b, K=K, N=N, g=g, with_source=with_source) for b in range(count)]
