"""MI355X slab S_N / Fokker-Planck synthetic acceleration (Python binding).

Thin ctypes binding over ``libsnfpsa.so`` (C ABI in ``include/snfpsa.h``).
It only marshals arguments: torch tensors supply device memory and
``torch.cuda`` streams supply the HIP stream; every step of the solver runs in
the library's HIP kernels.  The binding fails loudly if the library has not
been built (``python -m paper_1907_13013_amd.build``).

Layouts (per slab, concatenated over slabs): psi/q ``[K, 2, N]`` (LD node,
angle ascending in mu), phi ``[K, 2, L+1]``; all FP64.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsnfpsa.so")

SN_OK, SN_NOT_CONVERGED = 0, 1
SN_E_INVALID, SN_E_NOMEM, SN_E_HIP, SN_E_NONFINITE, SN_E_STATE = -1, -2, -3, -4, -5
SN_F64, SN_F32, SN_BF16X3 = 0, 1, 2
SN_FP_WFD, SN_FP_MPD, SN_FP_NONE = 0, 1, 2
SN_FP_CELL, SN_FP_MEAN = 0, 1
SN_SI, SN_FPSA, SN_FPSA_GMRES, SN_GMRES = 0, 1, 2, 3
SN_BC_PROBLEM, SN_BC_ZERO = 0, 1
SN_KERNEL_COUNT = 20

SCHEMES = {"wfd": SN_FP_WFD, "mpd": SN_FP_MPD, "none": SN_FP_NONE}
PRECISIONS = {"f64": SN_F64, "f32": SN_F32, "bf16x3": SN_BF16X3}
METHODS = {"si": SN_SI, "fpsa": SN_FPSA, "fpsa_gmres": SN_FPSA_GMRES, "gmres": SN_GMRES}
FP_COEFFICIENTS = {"cell": SN_FP_CELL, "mean": SN_FP_MEAN}

# every symbol declared in include/snfpsa.h and include/snfpsa_diag.h
EXPORTS = ["sn_setup", "sn_destroy", "sn_last_error", "sn_sweep", "sn_scatter_source",
           "fpsa_correct", "fpsa_correct_noalloc", "sn_solve", "sn_sweep_adjoint", "sn_update_cross_sections",
           "sn_solve_adjoint", "sn_response_gradient", "sn_exit_current_weights", "sn_exit_current",
           "sn_sweep_tuning", "sn_set_sweep_choice", "sn_scan_tuning", "sn_set_scan_choice", "sn_fused_iteration", "sn_set_fused_iteration", "sn_set_graph_replay", "sn_set_batched_solve",
           "sn_solve_refined", "sn_sizes", "sn_slab_info",
           "sn_set_kernel_timing",
           "sn_get_kernel_timing",
           "sn_diag_quadrature", "sn_diag_laplacian", "sn_diag_fp_factor", "sn_diag_fp_info",
           "sn_diag_fp_get", "sn_diag_fp_free"]


class SnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"snfpsa status {status}: {msg}")
        self.status = status


class ProblemDesc(C.Structure):
    _fields_ = [("num_slabs", C.c_int32),
                ("K", C.POINTER(C.c_int32)), ("N", C.POINTER(C.c_int32)),
                ("L", C.POINTER(C.c_int32)),
                ("h", C.POINTER(C.c_double)), ("sigma_t", C.POINTER(C.c_double)),
                ("sigma_s", C.POINTER(C.c_double)),
                ("psi_left", C.POINTER(C.c_double)), ("psi_right", C.POINTER(C.c_double)),
                ("fp_scheme", C.c_int32), ("precision", C.c_int32),
                ("fp_coefficients", C.c_int32)]


_lib = None


def load_library():
    """Load libsnfpsa.so; raises if it is missing (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1907_13013_amd.build")
    lib = C.CDLL(LIB_PATH)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    lib.sn_setup.argtypes = [C.POINTER(ProblemDesc), vp, C.POINTER(vp)]
    lib.sn_destroy.argtypes = [vp]
    lib.sn_last_error.restype = C.c_char_p
    lib.sn_sweep.argtypes = [vp, vp, vp, vp, i32, vp]
    lib.sn_scatter_source.argtypes = [vp, vp, vp, vp, vp]
    lib.fpsa_correct.argtypes = [vp, vp, vp, vp, vp]
    lib.fpsa_correct_noalloc.argtypes = [vp, vp, vp, vp, vp]
    lib.sn_solve.argtypes = [vp, i32, dbl, i32, vp, vp, vp, C.POINTER(i32), vp, vp]
    lib.sn_sweep_adjoint.argtypes = [vp, vp, vp, vp, vp]
    lib.sn_update_cross_sections.argtypes = [vp, vp, vp, vp]
    lib.sn_sweep_tuning.argtypes = [vp, C.POINTER(i32), vp]
    lib.sn_set_sweep_choice.argtypes = [vp, i32]
    lib.sn_scan_tuning.argtypes = [vp, C.POINTER(i32), vp]
    lib.sn_set_scan_choice.argtypes = [vp, i32]
    lib.sn_fused_iteration.argtypes = [vp, vp, vp]
    lib.sn_set_fused_iteration.argtypes = [vp, i32]
    lib.sn_set_graph_replay.argtypes = [vp, i32]
    lib.sn_set_batched_solve.argtypes = [vp, i32]
    lib.sn_solve_refined.argtypes = [vp, vp, dbl, dbl, dbl, i32, i32, vp, vp, C.POINTER(i32), vp, vp, vp]
    lib.sn_solve_adjoint.argtypes = [vp, i32, dbl, i32, vp, vp, C.POINTER(i32), vp, vp]
    lib.sn_response_gradient.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.sn_exit_current_weights.argtypes = [vp, vp, vp]
    lib.sn_exit_current.argtypes = [vp, vp, vp, vp]
    lib.sn_sizes.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.sn_slab_info.argtypes = [vp, i32, vp]
    lib.sn_set_kernel_timing.argtypes = [vp, i32]
    lib.sn_get_kernel_timing.argtypes = [vp, i32, C.POINTER(C.c_char_p), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_double)]
    lib.sn_diag_quadrature.argtypes = [i32, vp, vp]
    lib.sn_diag_laplacian.argtypes = [i32, i32, vp]
    lib.sn_diag_fp_factor.argtypes = [i32, i32, i32, vp, vp, vp, i32, i32, C.POINTER(vp)]
    lib.sn_diag_fp_info.argtypes = [vp, vp]
    lib.sn_diag_fp_get.argtypes = [vp, i32, vp]
    lib.sn_diag_fp_free.argtypes = [vp]
    for name in EXPORTS:
        if name not in ("sn_last_error",):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status: int, allow=(SN_OK,)) -> int:
    if status in allow:
        return status
    msg = load_library().sn_last_error().decode(errors="replace")
    raise SnError(status, msg)


def _np_ptr(a: Optional[np.ndarray], ctype=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(ctype))


def _dptr(t, dtype=None) -> Optional[int]:
    """Device pointer of a contiguous GPU tensor of the given dtype (default
    float64)."""
    if t is None:
        return None
    import torch
    dtype = torch.float64 if dtype is None else dtype
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous {dtype} tensor on the GPU")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class SlabSolver:
    """One library handle over one or more slabs.

    ``slabs`` is a sequence of objects with attributes K, N, L, h, sigma_t,
    sigma_s, psi_left, psi_right (NumPy FP64), e.g. ``sn_workloads.SlabProblem``.
    ``precision``: "f64", or "f32" / "bf16x3" (batched source iteration with
    float32 q / psi tensors; phi stays float64).
    ``fp_coefficients``: "cell" (each cell's sigma_a, sigma_tr in the
    Fokker-Planck operator) or "mean" (each slab's width-weighted mean
    sigma_a, sigma_tr rounded to two significant digits; slabs with equal
    rounded means share one factorisation).
    """

    def __init__(self, slabs: Sequence, fp_scheme: str = "wfd", stream=None, precision: str = "f64",
                 fp_coefficients: str = "cell"):
        lib = load_library()
        self._lib = lib
        self.slabs = list(slabs)
        self.fp_scheme = fp_scheme
        self.precision = precision
        K = np.array([s.K for s in self.slabs], dtype=np.int32)
        N = np.array([s.N for s in self.slabs], dtype=np.int32)
        L = np.array([s.L for s in self.slabs], dtype=np.int32)
        h = np.ascontiguousarray(np.concatenate([s.h for s in self.slabs]), dtype=np.float64)
        st = np.ascontiguousarray(np.concatenate([s.sigma_t for s in self.slabs]), dtype=np.float64)
        ss = np.ascontiguousarray(np.concatenate([np.ravel(s.sigma_s) for s in self.slabs]), dtype=np.float64)
        pl = np.ascontiguousarray(np.concatenate([s.psi_left for s in self.slabs]), dtype=np.float64)
        pr = np.ascontiguousarray(np.concatenate([s.psi_right for s in self.slabs]), dtype=np.float64)
        self._keep = (K, N, L, h, st, ss, pl, pr)
        d = ProblemDesc(len(self.slabs), _np_ptr(K, C.c_int32), _np_ptr(N, C.c_int32),
                        _np_ptr(L, C.c_int32), _np_ptr(h), _np_ptr(st), _np_ptr(ss),
                        _np_ptr(pl), _np_ptr(pr), SCHEMES[fp_scheme], PRECISIONS[precision],
                        FP_COEFFICIENTS[fp_coefficients])
        handle = C.c_void_p()
        _check(lib.sn_setup(C.byref(d), _stream(stream), C.byref(handle)))
        self.handle = handle
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib.sn_sizes(handle, C.byref(a), C.byref(b), C.byref(c)))
        self.psi_len, self.phi_len, self.exit_len = a.value, b.value, c.value
        self._xs_version = 0

    def close(self):
        if getattr(self, "handle", None):
            self._lib.sn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def slab_info(self, b: int = 0) -> dict:
        info = np.zeros(8, dtype=np.int32)
        _check(self._lib.sn_slab_info(self.handle, b, info.ctypes.data))
        return {"K": int(info[0]), "N": int(info[1]), "L": int(info[2]), "chunk": int(info[3]),
                "nchunks": int(info[4]), "sweep_tiles": int(info[5]),
                "tile_cells": int(info[6])}

    def sweep_tuning(self) -> dict:
        """The autotuned sweep decomposition (sn_sweep_tuning).  Batched
        handles: {"pair", "segment_small_n", "choice", "candidates_ms"[4]};
        FP64 handles: {"tile_policy": "default" | "half" | "double",
        "choice", "candidates_ms"[3]}."""
        ch = C.c_int32()
        ms = np.zeros(4)
        _check(self._lib.sn_sweep_tuning(self.handle, C.byref(ch), ms.ctypes.data))
        if self.precision == "f64":
            return {"tile_policy": ("default", "half", "double")[ch.value],
                    "choice": ch.value, "candidates_ms": ms[:3].tolist()}
        return {"pair": (ch.value & 1) == 0, "segment_small_n": (ch.value & 2) == 0,
                "choice": ch.value, "candidates_ms": ms.tolist()}

    def set_sweep_choice(self, choice: int):
        _check(self._lib.sn_set_sweep_choice(self.handle, int(choice)))

    def scan_tuning(self) -> dict:
        """Batched handles: the autotuned segment length of the long-slab
        scan (sn_scan_tuning): {"seg_cells", "candidates_ms"[3]}."""
        cells = C.c_int32()
        ms = np.zeros(3)
        _check(self._lib.sn_scan_tuning(self.handle, C.byref(cells), ms.ctypes.data))
        return {"seg_cells": cells.value, "candidates_ms": ms.tolist()}

    def set_scan_choice(self, choice: int):
        _check(self._lib.sn_set_scan_choice(self.handle, int(choice)))

    def fused_iteration(self) -> dict:
        """Batched handles: state of the fused source iteration
        (sn_fused_iteration): {"enabled", "available"}."""
        en, av = C.c_int32(), C.c_int32()
        _check(self._lib.sn_fused_iteration(self.handle, C.byref(en), C.byref(av)))
        return {"enabled": bool(en.value), "available": bool(av.value)}

    def set_fused_iteration(self, enable: bool):
        _check(self._lib.sn_set_fused_iteration(self.handle, int(bool(enable))))

    def set_graph_replay(self, enable: bool):
        """Batched handles: replay one captured iteration per source
        iteration (default) or launch every kernel from the host."""
        _check(self._lib.sn_set_graph_replay(self.handle, int(bool(enable))))

    def set_batched_solve(self, enable: bool):
        """FP64 handles with several slabs: solve them together in batched
        launches (default) or slab by slab (sn_set_batched_solve)."""
        _check(self._lib.sn_set_batched_solve(self.handle, int(bool(enable))))

    # -- kernel timing ---------------------------------------------------------
    def set_kernel_timing(self, enable: bool):
        _check(self._lib.sn_set_kernel_timing(self.handle, 1 if enable else 0))

    def kernel_timing(self) -> dict:
        """{kernel name: (launches, total ms)} recorded since timing was enabled."""
        out = {}
        for k in range(SN_KERNEL_COUNT):
            nm, n, ms = C.c_char_p(), C.c_int64(), C.c_double()
            _check(self._lib.sn_get_kernel_timing(self.handle, k, C.byref(nm), C.byref(n), C.byref(ms)))
            out[nm.value.decode()] = (n.value, ms.value)
        return out

    # -- tensors -----------------------------------------------------------
    @property
    def qdtype(self):
        """dtype of q / psi / q_ext / psi_exit tensors of this handle."""
        import torch
        return torch.float64 if self.precision == "f64" else torch.float32

    def _new(self, n, dtype=None):
        import torch
        return torch.empty(n, dtype=torch.float64 if dtype is None else dtype, device="cuda")

    def psi_tensor(self):
        return self._new(self.psi_len, self.qdtype)

    def phi_tensor(self):
        return self._new(self.phi_len)

    # -- C-ABI calls ---------------------------------------------------------
    def sweep(self, q, psi=None, phi=None, bc: str = "problem", stream=None):
        qd = self.qdtype
        _check(self._lib.sn_sweep(self.handle, _dptr(q, qd), _dptr(psi, qd), _dptr(phi),
                                  SN_BC_PROBLEM if bc == "problem" else SN_BC_ZERO,
                                  _stream(stream)))
        return psi, phi

    def sweep_adjoint(self, q_adj, psi_adj=None, phi_adj=None, stream=None):
        _check(self._lib.sn_sweep_adjoint(self.handle, _dptr(q_adj), _dptr(psi_adj),
                                          _dptr(phi_adj), _stream(stream)))
        return psi_adj, phi_adj

    def scatter_source(self, phi, q_ext=None, q_out=None, stream=None):
        if q_out is None:
            q_out = self.psi_tensor()
        qd = self.qdtype
        _check(self._lib.sn_scatter_source(self.handle, _dptr(phi), _dptr(q_ext, qd), _dptr(q_out, qd),
                                           _stream(stream)))
        return q_out

    def fpsa_correct(self, phi_half, phi_old, phi_new=None, stream=None):
        if phi_new is None:
            phi_new = self.phi_tensor()
        _check(self._lib.fpsa_correct(self.handle, _dptr(phi_half), _dptr(phi_old), _dptr(phi_new),
                                      _stream(stream)))
        return phi_new

    def fpsa_correct_noalloc(self, phi_half, phi_old, phi_new, stream=None):
        """fpsa_correct with its work vectors in the library's fixed per-device
        scratch (fpsa_correct_noalloc): allocates nothing, so phi_new is
        required."""
        _check(self._lib.fpsa_correct_noalloc(self.handle, _dptr(phi_half), _dptr(phi_old), _dptr(phi_new),
                                              _stream(stream)))
        return phi_new

    def solve(self, method: str = "fpsa", tol: float = 1e-8, max_iter: int = 100000,
              q_ext=None, phi=None, psi_exit=None, history: Optional[bool] = None, stream=None):
        """Returns dict(phi, iters, status, hist, psi_exit).  ``history``
        (the stopping-test value of every iteration, a host array of
        slabs x max_iter doubles): None keeps it when that array is at most
        256 MB."""
        if phi is None:
            phi = self.phi_tensor()
            phi.zero_()
        n = len(self.slabs)
        if history is None:
            history = n * max_iter <= (1 << 25)
        iters = (C.c_int32 * n)()
        hist = np.full(n * max_iter, np.nan) if history else None
        qd = self.qdtype
        st = _check(self._lib.sn_solve(self.handle, METHODS[method], float(tol), int(max_iter),
                                       _dptr(q_ext, qd), _dptr(phi), _dptr(psi_exit, qd), iters,
                                       None if hist is None else hist.ctypes.data_as(C.c_void_p),
                                       _stream(stream)),
                    allow=(SN_OK, SN_NOT_CONVERGED))
        its = list(iters)
        hs = None
        if hist is not None:
            hs = [hist[b * max_iter: b * max_iter + its[b]].copy() for b in range(n)]
        return {"phi": phi, "iters": its, "status": st, "hist": hs, "psi_exit": psi_exit}

    # -- adjoint and gradients (FP64 handles) -----------------------------------
    def update_cross_sections(self, sigma_t: np.ndarray, sigma_s: np.ndarray, stream=None):
        """New sigma_t [sum K] / sigma_s [sum K (L+1)] (host FP64) for the sweep
        and scattering source; the Fokker-Planck factors are kept."""
        st = np.ascontiguousarray(np.ravel(sigma_t), dtype=np.float64)
        ss = np.ascontiguousarray(np.ravel(sigma_s), dtype=np.float64)
        _check(self._lib.sn_update_cross_sections(self.handle, st.ctypes.data, ss.ctypes.data, _stream(stream)))
        self._xs_version += 1

    def exit_current(self, psi_exit, J=None, stream=None):
        """J [num_slabs] (FP64) = sum_{mu_n > 0} w_n mu_n psi_exit[b][n]: the
        partial current leaving each slab through z1 (sn_exit_current)."""
        import torch
        if J is None:
            J = torch.empty(len(self.slabs), dtype=torch.float64, device="cuda")
        _check(self._lib.sn_exit_current(self.handle, _dptr(psi_exit, self.qdtype), _dptr(J), _stream(stream)))
        return J

    def exit_current_weights(self, c=None, stream=None):
        """c with <c, psi> = sum_{mu_n > 0} w_n mu_n psi_n at the right node of
        each slab's last cell: the partial current leaving through z1
        (sn_exit_current_weights; FP64 handles)."""
        if c is None:
            c = self.psi_tensor()
        _check(self._lib.sn_exit_current_weights(self.handle, _dptr(c), _stream(stream)))
        return c

    def solve_adjoint(self, c, method: str = "fpsa", tol: float = 1e-8, max_iter: int = 100000,
                      phi_y=None, history: bool = False, stream=None):
        """Adjoint for the response <c, psi>; returns dict(phi_y, iters,
        status, hist) with phi_y the moments of the transformed adjoint."""
        if phi_y is None:
            phi_y = self.phi_tensor()
            phi_y.zero_()
        n = len(self.slabs)
        iters = (C.c_int32 * n)()
        hist = np.full(n * max_iter, np.nan) if history else None
        st = _check(self._lib.sn_solve_adjoint(self.handle, METHODS[method], float(tol), int(max_iter),
                                               _dptr(c), _dptr(phi_y), iters,
                                               None if hist is None else hist.ctypes.data_as(C.c_void_p),
                                               _stream(stream)),
                    allow=(SN_OK, SN_NOT_CONVERGED))
        its = list(iters)
        hs = None
        if hist is not None:
            hs = [hist[b * max_iter: b * max_iter + its[b]].copy() for b in range(n)]
        return {"phi_y": phi_y, "iters": its, "status": st, "hist": hs}

    def response_gradient(self, phi, c, phi_y, q_ext=None, stream=None):
        """(J [slabs], dJ/dsigma_t [sum K], dJ/dsigma_s [sum K (L+1)]) from the
        converged forward and adjoint moments."""
        import torch
        n = len(self.slabs)
        J = torch.empty(n, dtype=torch.float64, device="cuda")
        gt = torch.empty(sum(p.K for p in self.slabs), dtype=torch.float64, device="cuda")
        gs = torch.empty(sum(p.K * (p.L + 1) for p in self.slabs), dtype=torch.float64, device="cuda")
        _check(self._lib.sn_response_gradient(self.handle, _dptr(q_ext), _dptr(phi), _dptr(c), _dptr(phi_y),
                                              _dptr(J), _dptr(gt), _dptr(gs), _stream(stream)))
        return J, gt, gs


def solve_refined(lo: "SlabSolver", hi: "SlabSolver", q_ext=None, phi=None, tol: float = 1e-10,
                  tol_lo: float = 1e-5, inner_rel: float = 1e-4, max_steps: int = 10, max_iter: int = 100000,
                  stream=None) -> dict:
    """Mixed-precision iterative refinement (sn_solve_refined): low-precision
    batched source iterations on ``lo`` corrected by FP64 residuals of ``hi``
    (same slabs).  q_ext: FP64 device tensor or None.  Returns dict(phi,
    status, steps, inner_iters, resid)."""
    if phi is None:
        phi = hi.phi_tensor()
        phi.zero_()
    n = len(hi.slabs)
    steps = C.c_int32()
    inner = np.zeros(n, dtype=np.int32)
    resid = np.zeros(max_steps)
    st = _check(lo._lib.sn_solve_refined(lo.handle, hi.handle, float(tol), float(tol_lo), float(inner_rel),
                                         int(max_steps), int(max_iter), _dptr(q_ext), _dptr(phi), C.byref(steps),
                                         inner.ctypes.data, resid.ctypes.data, _stream(stream)),
                allow=(SN_OK, SN_NOT_CONVERGED))
    return {"phi": phi, "status": st, "steps": steps.value, "inner_iters": inner.tolist(),
            "resid": resid[:steps.value].tolist()}


def hg_moments(sigma_t, c, g, L: int):
    """Henyey-Greenstein moments sigma_{s,l} = c sigma_t g^l, l = 0..L, per cell
    (torch, differentiable): [cells] x3 -> [cells, L+1]."""
    import torch
    l = torch.arange(L + 1, dtype=sigma_t.dtype, device=sigma_t.device)
    return (c * sigma_t)[:, None] * g[:, None] ** l[None, :]


class _ExitCurrentFn:
    """Lazily built torch.autograd.Function (torch is imported on first use)."""
    fn = None

    @classmethod
    def get(cls):
        if cls.fn is not None:
            return cls.fn
        import torch

        class ExitCurrent(torch.autograd.Function):
            @staticmethod
            def forward(ctx, sigma_t, sigma_s, solver, q_ext, opts):
                solver.update_cross_sections(sigma_t.detach().cpu().numpy(), sigma_s.detach().cpu().numpy())
                pe = torch.zeros(solver.exit_len, dtype=torch.float64, device="cuda")
                r = solver.solve(opts["method"], tol=opts["tol"], max_iter=opts["max_iter"], q_ext=q_ext,
                                 psi_exit=pe, history=False)
                opts["state"] = {"phi": r["phi"], "iters": r["iters"], "status": r["status"]}
                if r["status"] != SN_OK:
                    # the adjoint gradient holds only at the converged forward
                    # fixed point (eq:iterate)
                    raise SnError(r["status"], f"forward solve not converged in {opts['max_iter']} "
                                               f"iterations (iters {r['iters']})")
                J = solver.exit_current(pe)
                # converged-state checkpoint: the moments only; backward
                # regenerates the angular flux from them with one sweep
                ctx.solver, ctx.q_ext, ctx.opts = solver, q_ext, opts
                ctx.version = solver._xs_version
                ctx.save_for_backward(sigma_t, sigma_s, r["phi"])
                return J

            @staticmethod
            def backward(ctx, gJ):
                sigma_t, sigma_s, phi = ctx.saved_tensors
                S, o = ctx.solver, ctx.opts
                if S._xs_version != ctx.version:  # the handle was reused since
                    S.update_cross_sections(sigma_t.detach().cpu().numpy(), sigma_s.detach().cpu().numpy())
                c = S.exit_current_weights()
                y = S.solve_adjoint(c, o["method"], tol=o["tol"], max_iter=o["max_iter"], phi_y=o.get("phi_y"))
                o.setdefault("state", {}).update({"phi_y": y["phi_y"], "iters_adjoint": y["iters"],
                                                  "status_adjoint": y["status"]})
                if y["status"] != SN_OK:
                    raise SnError(y["status"], f"adjoint solve not converged in {o['max_iter']} "
                                               f"iterations (iters {y['iters']})")
                _, gt, gs = S.response_gradient(phi, c, y["phi_y"], q_ext=ctx.q_ext)
                K = torch.tensor([p.K for p in S.slabs], device=gt.device)
                KL = torch.tensor([p.K * (p.L + 1) for p in S.slabs], device=gt.device)
                g = gJ.to(gt.device, torch.float64)
                return (gt * torch.repeat_interleave(g, K), gs * torch.repeat_interleave(g, KL),
                        None, None, None)

        cls.fn = ExitCurrent
        return cls.fn


def exit_current(sigma_t, sigma_s, solver: "SlabSolver", q_ext=None, method: str = "fpsa",
                 tol: float = 1e-12, max_iter: int = 100000, opts: Optional[dict] = None):
    """Partial current leaving each slab through z1 (torch [num_slabs]) as a
    differentiable function of every cell's sigma_t [sum K] and sigma_s
    [sum K (L+1)] (FP64 device tensors).  Forward: the cross sections of
    ``solver`` (an FP64 handle) are replaced by these and the transport
    problem is solved; only the converged moments are kept.  Backward: the
    adjoint solve and the gradient kernels, which regenerate both angular
    fluxes by one sweep each.  ``opts`` (optional dict) receives the
    converged moments and iteration counts under "state"; an entry "phi_y"
    (a previous adjoint's moments) warm-starts the adjoint solve."""
    o = opts if opts is not None else {}
    o.update({"method": method, "tol": tol, "max_iter": max_iter})
    return _ExitCurrentFn.get().apply(sigma_t, sigma_s, solver, q_ext, o)


# ---------------------------------------------------------------------------
# Host diagnostics of the setup math (no device work)
# ---------------------------------------------------------------------------

def diag_quadrature(N: int):
    lib = load_library()
    mu, w = np.zeros(N), np.zeros(N)
    _check(lib.sn_diag_quadrature(N, mu.ctypes.data, w.ctypes.data))
    return mu, w


def diag_laplacian(N: int, scheme: str):
    lib = load_library()
    A = np.zeros((N, N))
    _check(lib.sn_diag_laplacian(N, SCHEMES[scheme], A.ctypes.data))
    return A


def diag_fp_factors(K, N, L, h, sigma_t, sigma_s, scheme: str = "wfd", chunk: int = 0) -> dict:
    lib = load_library()
    h = np.ascontiguousarray(h, dtype=np.float64)
    st = np.ascontiguousarray(sigma_t, dtype=np.float64)
    ss = np.ascontiguousarray(sigma_s, dtype=np.float64)
    p = C.c_void_p()
    _check(lib.sn_diag_fp_factor(K, N, L, h.ctypes.data, st.ctypes.data, ss.ctypes.data,
                                 SCHEMES[scheme], chunk, C.byref(p)))
    try:
        info = np.zeros(4, dtype=np.int32)
        _check(lib.sn_diag_fp_info(p, info.ctypes.data))
        chunk, nchunks, ntypes, nseg = (int(x) for x in info)
        NH, L2 = N // 2, 2 * (L + 1)
        ntri = nchunks * (nchunks - 1) // 2
        shapes = {0: (K, 7, NH, NH), 1: (nchunks, NH, NH), 2: (nchunks, NH, NH),
                  3: (ntypes, L2, N), 4: (ntypes, L2, L2), 5: (ntypes, N, L2),
                  8: (K, NH, NH), 9: (K, NH, NH), 10: (ntri, NH, NH), 11: (ntri, NH, NH)}
        out = {"chunk": chunk, "nchunks": nchunks, "ntypes": ntypes}
        names = {0: "cellmats", 1: "chunk_fwd", 2: "chunk_bwd", 3: "EsrcT", 4: "PhisrcT",
                 5: "PhiinfT", 8: "psi_fwd", 9: "psi_bwd", 10: "theta_fwd", 11: "theta_bwd"}
        for k, shp in shapes.items():
            a = np.zeros(shp)
            _check(lib.sn_diag_fp_get(p, k, a.ctypes.data))
            out[names[k]] = a
        sb = np.zeros(nseg + 1, dtype=np.int32)
        stp = np.zeros(nseg, dtype=np.int32)
        _check(lib.sn_diag_fp_get(p, 6, sb.ctypes.data))
        _check(lib.sn_diag_fp_get(p, 7, stp.ctypes.data))
        out["seg_begin"], out["seg_type"] = sb, stp
        return out
    finally:
        lib.sn_diag_fp_free(p)
