"""C-ABI argument validation, forced from the host (no GPU needed: sn_setup
validates the descriptor before any HIP call)."""
import ctypes as C

import numpy as np
import pytest

snfpsa = pytest.importorskip("paper_1907_13013_amd")


def _setup(K=4, N=4, L=3, h=0.1, st=1.0, ss0=0.5, ss1=0.2, scheme=0, prec=0, nan_field=None, coef=0):
    lib = snfpsa.load_library()
    Ka = np.array([K], dtype=np.int32)
    Na = np.array([N], dtype=np.int32)
    La = np.array([L], dtype=np.int32)
    hh = np.full(max(K, 1), h)
    sts = np.full(max(K, 1), st)
    ss = np.zeros((max(K, 1), L + 1 if L >= 0 else 1))
    ss[:, 0] = ss0
    if ss.shape[1] > 1:
        ss[:, 1] = ss1
    pl = np.zeros(max(N // 2, 1))
    pr = np.zeros(max(N // 2, 1))
    if nan_field == "sigma_t":
        sts[0] = np.nan
    if nan_field == "psi_left":
        pl[0] = np.inf
    keep = (Ka, Na, La, hh, sts, ss, pl, pr)
    P = lambda a, t=C.c_double: a.ctypes.data_as(C.POINTER(t))
    d = snfpsa.ProblemDesc(1, P(Ka, C.c_int32), P(Na, C.c_int32), P(La, C.c_int32), P(hh), P(sts),
                           P(ss), P(pl), P(pr), scheme, prec, coef)
    h = C.c_void_p()
    st = lib.sn_setup(C.byref(d), None, C.byref(h))
    del keep
    return st, lib.sn_last_error().decode()


@pytest.mark.parametrize("kw,expect", [
    (dict(N=5, L=3), snfpsa.SN_E_INVALID),       # odd N
    (dict(N=4, L=4), snfpsa.SN_E_INVALID),       # L >= N
    (dict(N=258, L=3), snfpsa.SN_E_INVALID),     # N above the kernel limit
    (dict(K=0), snfpsa.SN_E_INVALID),            # no cells
    (dict(h=0.0), snfpsa.SN_E_INVALID),          # degenerate cell
    (dict(st=-1.0), snfpsa.SN_E_INVALID),        # negative sigma_t
    (dict(ss0=1.5), snfpsa.SN_E_INVALID),        # sigma_a < 0
    (dict(ss0=0.2, ss1=0.5), snfpsa.SN_E_INVALID),  # sigma_tr < 0
    (dict(scheme=7), snfpsa.SN_E_INVALID),
    (dict(prec=7), snfpsa.SN_E_INVALID),         # unknown precision
    (dict(scheme=3), snfpsa.SN_E_INVALID),       # unknown Fokker-Planck scheme
    (dict(coef=2), snfpsa.SN_E_INVALID),         # unknown Fokker-Planck coefficient mode
    (dict(nan_field="sigma_t"), snfpsa.SN_E_NONFINITE),
    (dict(nan_field="psi_left"), snfpsa.SN_E_NONFINITE),
])
def test_setup_rejects_bad_descriptors(kw, expect):
    st, msg = _setup(**kw)
    assert st == expect, msg
    assert msg


def test_null_arguments():
    lib = snfpsa.load_library()
    h = C.c_void_p()
    assert lib.sn_setup(None, None, C.byref(h)) == snfpsa.SN_E_INVALID
    assert lib.sn_destroy(None) == snfpsa.SN_E_STATE
    assert lib.sn_sweep(None, None, None, None, 0, None) == snfpsa.SN_E_STATE
    assert lib.sn_update_cross_sections(None, None, None, None) == snfpsa.SN_E_STATE
    assert lib.sn_solve_adjoint(None, 1, 1e-8, 10, None, None, None, None, None) == snfpsa.SN_E_STATE
    assert lib.sn_response_gradient(None, None, None, None, None, None, None, None, None) == snfpsa.SN_E_STATE
    assert lib.sn_sweep_tuning(None, None, None) == snfpsa.SN_E_STATE
    assert lib.sn_set_sweep_choice(None, 0) == snfpsa.SN_E_STATE
    assert lib.sn_set_graph_replay(None, 1) == snfpsa.SN_E_STATE
    assert lib.sn_set_kernel_timing(None, 1) == snfpsa.SN_E_STATE
