"""ctypes view of the C ABI in include/jfnk.h (argument marshalling only).

The shared library is loaded from this package directory; there is no fallback: importing
the binding without a built ``libjfnk.so`` raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjfnk.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "jfnk.h")

OK = 0
E_INVALID = -1
E_DEVICE = -2
E_NONFINITE = -3
E_GMRES_NOCONV = -4
E_NEWTON_NOCONV = -5
E_INADMISSIBLE = -6

BC_PERIODIC, BC_WALL = 0, 1
CHI_NONE, CHI_CONST, CHI_POWER = 0, 1, 2
JV_FD, JV_EXACT = 0, 1
PC_NONE, PC_SOUND, PC_SOUND_THERMAL = 0, 1, 2
FP64, FP32 = 0, 1


class Problem(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32),
        ("n", C.c_int32 * 3),
        ("dx", C.c_double * 3),
        ("bc", C.c_int32 * 3),
        ("gamma", C.c_double),
        ("g", C.c_double * 3),
        ("chi_model", C.c_int32),
        ("chi0", C.c_double),
        ("chi_tref", C.c_double),
        ("chi_exp", C.c_double),
        ("qwall", (C.c_double * 2) * 3),
        ("theta", C.c_double),
        ("a_rad", C.c_double),
    ]


class Opts(C.Structure):
    _fields_ = [
        ("newton_tol", C.c_double),
        ("newton_max", C.c_int32),
        ("newton_min", C.c_int32),
        ("gmres_m", C.c_int32),
        ("gmres_maxit", C.c_int32),
        ("gmres_eta", C.c_double),
        ("jv_mode", C.c_int32),
        ("fd_lambda", C.c_double),
        ("alpha1", C.c_double),
        ("alpha2", C.c_double),
        ("precond", C.c_int32),
        ("ell_precision", C.c_int32),
        ("cg_eta", C.c_double),
        ("cg_maxit", C.c_int32),
        ("pc_schur", C.c_int32),
        ("phase_timing", C.c_int32),
        ("mg_levels", C.c_int32),
        ("mg_smooth", C.c_int32),
    ]


class StepStats(C.Structure):
    _fields_ = [
        ("newton_its", C.c_int32),
        ("gmres_its", C.c_int32),
        ("cg_its", C.c_int32),
        ("converged", C.c_int32),
        ("f0_norm", C.c_double),
        ("f_norm", C.c_double),
        ("last_dx_norm", C.c_double),
        ("dt", C.c_double),
        ("t_resid", C.c_double),
        ("t_jv", C.c_double),
        ("t_prec", C.c_double),
        ("t_orth", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_D = C.c_double
SIGNATURES = {
    "jfnk_default_opts": (None, [C.POINTER(Opts)]),
    "jfnk_create": (C.c_int, [C.POINTER(Problem), C.POINTER(Opts), _P, C.POINTER(_P)]),
    "jfnk_destroy": (C.c_int, [_P]),
    "jfnk_set_opts": (C.c_int, [_P, C.POINTER(Opts)]),
    "jfnk_workspace_bytes": (C.c_size_t, [_P]),
    "jfnk_last_error": (C.c_char_p, [_P]),
    "jfnk_set_state_n": (C.c_int, [_P, _P, _D]),
    "jfnk_residual": (C.c_int, [_P, _P, _P]),
    "jfnk_jvp": (C.c_int, [_P, _P, _P, _P, C.c_int32]),
    "jfnk_vjp": (C.c_int, [_P, _P, _P, _P]),
    "jfnk_vjp_prev": (C.c_int, [_P, _P, _P, _P]),
    "jfnk_precond_apply": (C.c_int, [_P, _P, _P, _P]),
    "jfnk_precond_apply_transpose": (C.c_int, [_P, _P, _P, _P]),
    "jfnk_implicit_step": (C.c_int, [_P, _P, _D, C.POINTER(StepStats)]),
    "jfnk_si_step": (C.c_int, [_P, _P, _D, C.POINTER(StepStats)]),
    "jfnk_adjoint_step": (C.c_int, [_P, _P, _P, _D, _P, _P, C.POINTER(StepStats)]),
    "jfnk_cfl_dt": (C.c_double, [_P, _P, _D]),
    "jfnk_cfl_dt_noalloc": (C.c_int, [C.POINTER(Problem), _P, _D, _P, _P]),
    "jfnk_probe_enable": (C.c_int, [C.c_int32]),
    "jfnk_probe_count": (C.c_int, []),
    "jfnk_probe_name": (C.c_char_p, [C.c_int32]),
    "jfnk_probe_read": (C.c_int, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_double)]),
}


def probe_enable(on=True):
    lib().jfnk_probe_enable(1 if on else 0)


def probe_results():
    """{kernel family: (ms, launches, algorithmic bytes)} of the instrumented kernels."""
    L = lib()
    out = {}
    for k in range(L.jfnk_probe_count()):
        ms, n, b = C.c_double(), C.c_int64(), C.c_double()
        L.jfnk_probe_read(k, C.byref(ms), C.byref(n), C.byref(b))
        if n.value:
            out[L.jfnk_probe_name(k).decode()] = (ms.value, n.value, b.value)
    return out


def header_functions(path=HEADER):
    """Names of the functions declared in include/jfnk.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(jfnk_[a-z_0-9]+)\s*\(", txt)))


_lib = None


def lib():
    """Load libjfnk.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python -m paper_1512_03662_amd.build)")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L
