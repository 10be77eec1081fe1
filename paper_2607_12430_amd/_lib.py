"""ctypes binding of libmsqrt.so (argument marshalling only).

The library is loaded from this package directory; if it is missing the import
of any entry point raises, there is no fallback implementation.
"""

from __future__ import annotations

import atexit
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsqrt.so")

# status codes (include/msqrt.h)
OK, INVALID_ARG, NONFINITE, NO_PRINCIPAL, NOT_CONVERGED, DIVERGED, DEVICE, OUT_OF_MEMORY, UNSUPPORTED = range(9)
STATUS_NAMES = {
    OK: "ok", INVALID_ARG: "invalid_arg", NONFINITE: "nonfinite", NO_PRINCIPAL: "no_principal",
    NOT_CONVERGED: "not_converged", DIVERGED: "diverged", DEVICE: "device",
    OUT_OF_MEMORY: "out_of_memory", UNSUPPORTED: "unsupported",
}
REAL64, COMPLEX128 = 0, 1
PREC_AUTO, PREC_BF16SPLIT, PREC_FP32, PREC_FP64 = 0, 1, 2, 3
PREC_NAMES = {"auto": PREC_AUTO, "bf16split": PREC_BF16SPLIT, "fp32": PREC_FP32, "fp64": PREC_FP64}
STRUCT_AUTO, STRUCT_GENERAL, STRUCT_HPD = 0, 1, 2
STRUCT_NAMES = {"auto": STRUCT_AUTO, "general": STRUCT_GENERAL, "hpd": STRUCT_HPD, "spd": STRUCT_HPD}
PHASES = ["validate", "select", "reduce", "eig", "back", "x0", "residual", "transform", "solve",
          "update", "total", "spare"]

EXPORTED = [
    "msqrt_default_options", "msqrt_factor", "msqrt_refine", "msqrt_refine_noalloc", "msqrt_sqrtm",
    "msqrt_sqrtm_backward", "msqrt_factor_destroy", "msqrt_status_string", "msqrt_last_error",
    "msqrt_release_cached",
    "msqrt_factor_wrap", "msqrt_factor_export", "msqrt_test_sytrd", "msqrt_test_sy2tr",
    "msqrt_test_stedc",
    "msqrt_test_gehrd", "msqrt_test_schur", "msqrt_test_trsqrt", "msqrt_test_trsyl",
    "msqrt_test_trcbrt", "msqrt_rootm",
    "msqrt_test_gemm_f32", "msqrt_test_syrk", "msqrt_features", "msqrt_mlp_forward", "msqrt_mlp_grad",
    "msqrt_mlp_adam", "msqrt_selector_set", "msqrt_selector_load", "msqrt_selector_clear",
    "msqrt_selector_installed",
    "msqrt_profile_enable", "msqrt_profile_query", "msqrt_profile_list",
]


class Options(ctypes.Structure):
    _fields_ = [
        ("prec", ctypes.c_int),
        ("structure", ctypes.c_int),
        ("maxit", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("blks", ctypes.c_int),
        ("fallback", ctypes.c_int),
        ("batch", ctypes.c_int64),
        ("real_schur", ctypes.c_int),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int),
        ("relres", ctypes.c_double),
        ("relres_hist", ctypes.c_double * 64),
        ("nhist", ctypes.c_int),
        ("prec_used", ctypes.c_int),
        ("struct_used", ctypes.c_int),
        ("fallbacks", ctypes.c_int),
        ("scale_exp", ctypes.c_int),
        ("predicted_steps", ctypes.c_float * 3),
        ("t_ms", ctypes.c_float * 12),
    ]

    def to_dict(self):
        inv_prec = {v: k for k, v in PREC_NAMES.items()}
        return {
            "steps": self.steps,
            "relres": self.relres,
            "relres_hist": [self.relres_hist[i] for i in range(self.nhist)],
            "prec_used": inv_prec.get(self.prec_used, self.prec_used),
            "struct_used": {STRUCT_HPD: "hpd", STRUCT_GENERAL: "general"}.get(self.struct_used, "auto"),
            "fallbacks": self.fallbacks,
            "scale_exp": self.scale_exp,
            "predicted_steps": list(self.predicted_steps),
            "t_ms": {PHASES[i]: self.t_ms[i] for i in range(12) if self.t_ms[i] != 0.0},
        }


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, ci, cd = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.msqrt_release_cached.argtypes = []
    L.msqrt_release_cached.restype = None
    # ordered shutdown: cached device memory and events are released while
    # the HIP runtime is still up
    atexit.register(L.msqrt_release_cached)
    L.msqrt_default_options.argtypes = [ctypes.POINTER(Options)]
    L.msqrt_default_options.restype = None
    L.msqrt_factor.argtypes = [ctypes.POINTER(Options), ci, i64, vp, i64, i64, vp, ctypes.POINTER(vp)]
    L.msqrt_refine.argtypes = [vp, vp, i64, i64, vp, i64, i64, ci, ci, cd, vp, ctypes.POINTER(Info)]
    L.msqrt_refine_noalloc.argtypes = [vp, vp, i64, i64, vp, i64, i64, ci, ci, cd, vp,
                                       ctypes.POINTER(Info)]
    L.msqrt_sqrtm.argtypes = [ctypes.POINTER(Options), ci, i64, vp, i64, i64, vp, i64, i64, vp,
                              ctypes.POINTER(Info), ctypes.POINTER(vp)]
    L.msqrt_sqrtm_backward.argtypes = [vp, vp, i64, vp, i64, vp, i64, i64, ci, cd, vp,
                                       ctypes.POINTER(Info)]
    L.msqrt_factor_destroy.argtypes = [vp]
    L.msqrt_factor_destroy.restype = None
    L.msqrt_status_string.argtypes = [ci]
    L.msqrt_status_string.restype = ctypes.c_char_p
    L.msqrt_last_error.argtypes = []
    L.msqrt_last_error.restype = ctypes.c_char_p
    L.msqrt_factor_wrap.argtypes = [ci, ci, ci, i64, vp, vp, ci, ctypes.POINTER(vp)]
    L.msqrt_factor_export.argtypes = [vp, vp, vp, ctypes.POINTER(ci)]
    L.msqrt_profile_enable.argtypes = [ci]
    L.msqrt_profile_enable.restype = None
    L.msqrt_profile_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(i64), ctypes.POINTER(cd),
                                      ctypes.POINTER(cd), ctypes.POINTER(cd)]
    L.msqrt_profile_query.restype = ci
    L.msqrt_profile_list.argtypes = [ctypes.c_char_p, ci]
    L.msqrt_profile_list.restype = ci
    L.msqrt_test_sytrd.argtypes = [ci, i64, vp, vp, vp, vp]
    L.msqrt_test_sy2tr.argtypes = [ci, i64, vp, vp, vp, vp]
    L.msqrt_test_stedc.argtypes = [ci, i64, vp, vp, vp, vp]
    dp = ctypes.POINTER(ctypes.c_double)
    L.msqrt_test_gehrd.argtypes = [ci, i64, dp, dp, dp]
    L.msqrt_test_schur.argtypes = [ci, i64, dp, dp, dp]
    L.msqrt_test_trsqrt.argtypes = [ci, i64, dp, dp]
    L.msqrt_test_trcbrt.argtypes = [ci, i64, dp, dp]
    L.msqrt_rootm.argtypes = [ctypes.POINTER(Options), ci, ci, i64, vp, i64, vp, i64, vp,
                              ctypes.POINTER(Info)]
    L.msqrt_test_trsyl.argtypes = [ci, i64, i64, dp, dp, dp, dp]
    L.msqrt_test_gemm_f32.argtypes = [ci, ci, ci, i64, i64, i64, vp, vp, vp]
    L.msqrt_test_syrk.argtypes = [ci, i64, i64, vp, vp]
    L.msqrt_features.argtypes = [ci, i64, vp, i64, vp, vp]
    L.msqrt_mlp_forward.argtypes = [i64, vp, vp, vp, vp]
    L.msqrt_mlp_grad.argtypes = [i64, vp, vp, vp, vp, vp, vp]
    L.msqrt_mlp_adam.argtypes = [vp, vp, vp, vp, ci, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, vp]
    L.msqrt_selector_set.argtypes = [vp, vp, vp, vp, ci]
    L.msqrt_selector_load.argtypes = [ctypes.c_char_p]
    L.msqrt_selector_clear.argtypes = []
    L.msqrt_selector_clear.restype = None
    L.msqrt_selector_installed.argtypes = []
    L.msqrt_selector_installed.restype = ci
    for name in ("msqrt_factor", "msqrt_refine", "msqrt_refine_noalloc", "msqrt_sqrtm",
                 "msqrt_sqrtm_backward",
                 "msqrt_factor_wrap", "msqrt_factor_export", "msqrt_test_sytrd",
                 "msqrt_test_stedc", "msqrt_test_gehrd", "msqrt_test_schur", "msqrt_test_trsqrt",
                 "msqrt_test_trcbrt", "msqrt_rootm",
                 "msqrt_test_trsyl", "msqrt_test_gemm_f32", "msqrt_test_syrk", "msqrt_features",
                 "msqrt_mlp_forward", "msqrt_mlp_grad", "msqrt_mlp_adam", "msqrt_selector_set",
                 "msqrt_selector_load"):
        getattr(L, name).restype = ci
    _lib = L
    return L


class MsqrtError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        msg = lib().msqrt_last_error().decode(errors="replace")
        super().__init__(f"{where}: {self.name} ({msg})")


def check(status, where, allow=()):
    if status != OK and status not in allow:
        raise MsqrtError(status, where)
    return status


def profile_enable(on: bool):
    lib().msqrt_profile_enable(1 if on else 0)


def profile_stats():
    """{kernel_class: dict(launches, ms, flops, bytes)} recorded since enable."""
    L = lib()
    buf = ctypes.create_string_buffer(4096)
    L.msqrt_profile_list(buf, 4096)
    out = {}
    for cls in filter(None, buf.value.decode().split(",")):
        n = ctypes.c_int64(0)
        ms, fl, by = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        if L.msqrt_profile_query(cls.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl),
                                 ctypes.byref(by)) == 0:
            out[cls] = {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}
    return out
