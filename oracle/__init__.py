"""FP64 CPU oracle for slab S_N source iteration and FPSA (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the reference the HIP library is checked against.
Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
it.  It shares no code with the HIP library (``sn_oracle.c`` is compiled on
its own with gcc) and never imports the library package.

Every function takes and returns NumPy FP64 arrays in the layouts documented
in ``sn_oracle.c``: psi/q ``[K, 2, N]``, phi ``[K, 2, L+1]``,
sigma_s ``[K, L+1]``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sn_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over angles in the sweep)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = C.CDLL(_LIB)
    i, d, vp = C.c_int, C.c_double, C.c_void_p
    lib.or_gauss_legendre.argtypes = [i, _dp, _dp]
    lib.or_legendre.argtypes = [i, i, _dp, _dp]
    lib.or_wfd_matrix.argtypes = [i, _dp, _dp, _dp]
    lib.or_mpd_matrix.argtypes = [i, _dp, _dp, _dp]
    lib.or_mpd_matrix.restype = i
    lib.or_moments.argtypes = [i, i, i, _dp, _dp, _dp, _dp]
    lib.or_scatter_source.argtypes = [i, i, i, _dp, _dp, _dp, vp, _dp]
    lib.or_sweep.argtypes = [i, i, _dp, _dp, _dp, _dp, vp, vp, _dp]
    lib.or_sweep_adjoint.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp]
    lib.or_solve.argtypes = [i, i, i, _dp, _dp, _dp, vp, vp, vp, i, i, d, i, _dp,
                             vp, C.POINTER(C.c_int), vp]
    lib.or_solve.restype = i
    lib.or_fpsa_correct.argtypes = [i, i, i, _dp, _dp, _dp, i, _dp, _dp, _dp, vp]
    lib.or_fpsa_correct.restype = i
    lib.or_fp_solve.argtypes = [i, i, _dp, _dp, _dp, i, _dp, _dp]
    lib.or_fp_solve.restype = i
    lib.or_adjoint_solve.argtypes = [i, i, i, _dp, _dp, _dp, _dp, d, i, _dp, C.POINTER(C.c_int)]
    lib.or_adjoint_solve.restype = i
    lib.or_response_gradient.argtypes = [i, i, i, _dp, _dp, _dp, _dp]
    lib.or_last_timing.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.or_set_threads.argtypes = [i]
    lib.or_get_threads.restype = i
    _lib = lib
    return lib


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


SCHEMES = {"wfd": 0, "mpd": 1}


def gauss_legendre(N: int):
    mu, w = np.zeros(N), np.zeros(N)
    _load().or_gauss_legendre(N, mu, w)
    return mu, w


def legendre(N: int, L: int, mu) -> np.ndarray:
    P = np.zeros((L + 1) * N)
    _load().or_legendre(N, L, _c(mu), P)
    return P.reshape(L + 1, N)


def wfd_matrix(N: int) -> np.ndarray:
    mu, w = gauss_legendre(N)
    W = np.zeros(N * N)
    _load().or_wfd_matrix(N, mu, w, W)
    return W.reshape(N, N)


def mpd_matrix(N: int) -> np.ndarray:
    mu, w = gauss_legendre(N)
    F = np.zeros(N * N)
    if _load().or_mpd_matrix(N, mu, w, F) != 0:
        raise RuntimeError("singular V")
    return F.reshape(N, N)


def moments(psi: np.ndarray, L: int) -> np.ndarray:
    K, _, N = psi.shape
    mu, w = gauss_legendre(N)
    phi = np.zeros(K * 2 * (L + 1))
    _load().or_moments(K, N, L, mu, w, _c(psi), phi)
    return phi.reshape(K, 2, L + 1)


def scatter_source(phi: np.ndarray, sigma_s: np.ndarray, N: int,
                   q_ext: Optional[np.ndarray] = None) -> np.ndarray:
    K, _, L1 = phi.shape
    mu, _ = gauss_legendre(N)
    q = np.zeros(K * 2 * N)
    qe = None if q_ext is None else _c(q_ext)
    _load().or_scatter_source(K, N, L1 - 1, mu, _c(sigma_s), _c(phi), _ptr(qe), q)
    return q.reshape(K, 2, N)


def sweep(q: np.ndarray, h, sigma_t, psi_left=None, psi_right=None) -> np.ndarray:
    K, _, N = q.shape
    mu, _ = gauss_legendre(N)
    psi = np.zeros(K * 2 * N)
    pl = None if psi_left is None else _c(psi_left)
    pr = None if psi_right is None else _c(psi_right)
    _load().or_sweep(K, N, mu, _c(h), _c(sigma_t), _c(q), _ptr(pl), _ptr(pr), psi)
    return psi.reshape(K, 2, N)


def sweep_adjoint(y: np.ndarray, h, sigma_t) -> np.ndarray:
    K, _, N = y.shape
    mu, _ = gauss_legendre(N)
    x = np.zeros(K * 2 * N)
    _load().or_sweep_adjoint(K, N, mu, _c(h), _c(sigma_t), _c(y), x)
    return x.reshape(K, 2, N)


def fp_solve(r: np.ndarray, h, sigma_a, sigma_tr, scheme: str = "wfd") -> np.ndarray:
    K, _, N = r.shape
    U = np.zeros(K * 2 * N)
    rc = _load().or_fp_solve(K, N, _c(h), _c(sigma_a), _c(sigma_tr), SCHEMES[scheme], _c(r), U)
    if rc != 0:
        raise RuntimeError("FP factorisation failed")
    return U.reshape(K, 2, N)


def fpsa_correct(prob, phi_half: np.ndarray, phi_old: np.ndarray, scheme: str = "wfd"):
    """phi_new = phi_half + D F_h^{-1} M Sigma (phi_half - phi_old); returns
    (phi_new, U) with U the angular correction."""
    K, N, L = prob.K, prob.N, prob.L
    phi_new = np.zeros(K * 2 * (L + 1))
    U = np.zeros(K * 2 * N)
    rc = _load().or_fpsa_correct(K, N, L, _c(prob.h), _c(prob.sigma_t), _c(prob.sigma_s),
                                 SCHEMES[scheme], _c(phi_half), _c(phi_old), phi_new,
                                 _ptr(U))
    if rc != 0:
        raise RuntimeError("FP factorisation failed")
    return phi_new.reshape(K, 2, L + 1), U.reshape(K, 2, N)


def solve(prob, method: str = "si", scheme: str = "wfd", tol: Optional[float] = None,
          max_iter: int = 100000, phi0: Optional[np.ndarray] = None,
          q_ext: Optional[np.ndarray] = "problem", bc: bool = True):
    """Source iteration ("si") or FPSA ("fpsa") to max|phi^{m+1}-phi^m| <= tol.

    Returns dict(phi, psi, iters, status, hist)."""
    K, N, L = prob.K, prob.N, prob.L
    tol = prob.tol if tol is None else tol
    phi = np.zeros(K * 2 * (L + 1)) if phi0 is None else _c(phi0).ravel().copy()
    psi = np.zeros(K * 2 * N)
    hist = np.zeros(max_iter)
    it = C.c_int(0)
    if isinstance(q_ext, str):
        q_ext = prob.q
    qe = None if q_ext is None else _c(q_ext)
    pl = _c(prob.psi_left) if bc else None
    pr = _c(prob.psi_right) if bc else None
    st = _load().or_solve(K, N, L, _c(prob.h), _c(prob.sigma_t), _c(prob.sigma_s),
                          _ptr(pl), _ptr(pr), _ptr(qe), 1 if method == "fpsa" else 0,
                          SCHEMES[scheme], float(tol), int(max_iter), phi, _ptr(psi),
                          C.byref(it), _ptr(hist))
    if st < 0:
        raise RuntimeError(f"oracle solve failed ({st})")
    n = it.value
    return {"phi": phi.reshape(K, 2, L + 1), "psi": psi.reshape(K, 2, N), "iters": n,
            "status": st, "hist": hist[:n].copy()}


def adjoint_solve(prob, c: np.ndarray, tol: float = 1e-14, max_iter: int = 200000,
                  lam0: Optional[np.ndarray] = None):
    """Adjoint lambda of the response <c, psi>: fixed point of
    lambda = Linv^T (S^T lambda + c) by adjoint source iteration.
    Returns dict(lam [K,2,N], iters, status)."""
    K, N, L = prob.K, prob.N, prob.L
    lam = np.zeros(K * 2 * N) if lam0 is None else _c(lam0).ravel().copy()
    it = C.c_int(0)
    st = _load().or_adjoint_solve(K, N, L, _c(prob.h), _c(prob.sigma_t), _c(prob.sigma_s), _c(c).ravel(),
                                  float(tol), int(max_iter), lam, C.byref(it))
    return {"lam": lam.reshape(K, 2, N), "iters": it.value, "status": st}


def response_gradient(prob, psi: np.ndarray, lam: np.ndarray):
    """(dJ/dsigma_t [K], dJ/dsigma_s [K, L+1]) of J = <c, psi> from the
    converged psi and its adjoint lambda."""
    K, N, L = prob.K, prob.N, prob.L
    gt = np.zeros(K)
    gs = np.zeros(K * (L + 1))
    _load().or_response_gradient(K, N, L, _c(psi).ravel(), _c(lam).ravel(), gt, gs)
    return gt, gs.reshape(K, L + 1)


def exit_current_weights(K: int, N: int) -> np.ndarray:
    """c of the partial current through z1: w_n mu_n at the right node of the
    last cell for mu_n > 0."""
    mu, w = gauss_legendre(N)
    c = np.zeros((K, 2, N))
    c[K - 1, 1, N // 2:] = (w * mu)[N // 2:]
    return c


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's sweep (the CPU baseline's core count)."""
    _load().or_set_threads(int(n))


def get_threads() -> int:
    return int(_load().or_get_threads())


def last_timing():
    """(factorisation seconds, iteration seconds) of the last solve() call:
    the Fokker-Planck factorisation is setup, excluded from solve timings
    as in the paper's Sec. 4."""
    f, i = C.c_double(), C.c_double()
    _load().or_last_timing(C.byref(f), C.byref(i))
    return f.value, i.value
