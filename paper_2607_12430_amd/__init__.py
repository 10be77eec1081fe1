"""Mixed-precision principal matrix square root on MI355X (gfx950).

Thin Python layer over the C-ABI in include/msqrt.h: torch supplies device
memory and the current stream; every step of the computation runs in the HIP
kernels of libmsqrt.so.

    X, info = sqrtm(A)                 # A: cuda float64 (n, n) or (b, n, n)
    X = sqrtm_autograd(A)              # differentiable (torch.autograd.Function)
"""

from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import MsqrtError, check, lib

__all__ = ["sqrtm", "sqrtm_autograd", "Factor", "factor", "refine", "factor_wrap", "MsqrtError",
           "default_options"]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_matrix(a: torch.Tensor, name: str):
    if not a.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if a.dtype not in (torch.float64, torch.complex128):
        raise ValueError(f"{name} must be float64 or complex128, got {a.dtype}")
    if a.dim() not in (2, 3) or a.shape[-1] != a.shape[-2]:
        raise ValueError(f"{name} must be (n, n) or (b, n, n)")
    if not a.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _dims(a: torch.Tensor):
    n = a.shape[-1]
    batch = a.shape[0] if a.dim() == 3 else 1
    return n, batch, n * n


_selector_tried = False


def _ensure_selector():
    """Installs the packaged selector file once (AUTO falls back to FP32
    inside the library when none is installed)."""
    global _selector_tried
    if _selector_tried:
        return
    _selector_tried = True
    if not lib().msqrt_selector_installed():
        from . import selector
        selector.install()


def default_options(prec="fp32", structure="auto", maxit=30, tol=1e-13, blks=32, fallback=True,
                    batch=1, real_schur=True):
    o = _lib.Options()
    lib().msqrt_default_options(ctypes.byref(o))
    o.prec = _lib.PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
    o.structure = _lib.STRUCT_NAMES[structure] if isinstance(structure, str) else int(structure)
    o.maxit = int(maxit)
    o.tol = float(tol)
    o.blks = int(blks)
    o.fallback = 1 if fallback else 0
    o.batch = int(batch)
    o.real_schur = 1 if real_schur else 0
    return o


class Factor:
    """Owns a msqrt_factor_t handle."""

    def __init__(self, handle: int, n: int, batch: int):
        self.handle = ctypes.c_void_p(handle)
        self.n = n
        self.batch = batch

    def close(self):
        if self.handle and self.handle.value:
            lib().msqrt_factor_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def export(self, single: bool, structure: str = "hpd"):
        """Host copies (Q, S, k) of the factor (test hook)."""
        import numpy as np
        n, b = self.n, self.batch
        dt = np.float32 if single else np.float64
        q = np.zeros((b, n, n), dtype=dt)
        s = np.zeros((b, n) if structure == "hpd" else (b, n, n), dtype=dt)
        k = ctypes.c_int(0)
        check(lib().msqrt_factor_export(self.handle, q.ctypes.data_as(ctypes.c_void_p),
                                        s.ctypes.data_as(ctypes.c_void_p), ctypes.byref(k)),
              "msqrt_factor_export")
        # buffers are column-major per batch entry
        return np.ascontiguousarray(np.swapaxes(q, 1, 2)), s, k.value


def factor(a: torch.Tensor, prec="fp32", structure="auto", blks=32, real_schur=True) -> Factor:
    _check_matrix(a, "A")
    n, batch, nn = _dims(a)
    o = default_options(prec=prec, structure=structure, blks=blks, batch=batch,
                        real_schur=real_schur)
    h = ctypes.c_void_p(0)
    dt = _lib.COMPLEX128 if a.is_complex() else _lib.REAL64
    check(lib().msqrt_factor(ctypes.byref(o), dt, n, ctypes.c_void_p(a.data_ptr()), n, nn,
                             _stream(), ctypes.byref(h)), "msqrt_factor")
    return Factor(h.value, n, batch)


def factor_wrap(q, s, prec="fp32", structure="hpd") -> Factor:
    """Builds a factor from host NumPy arrays Q (n x n) and S (test hook)."""
    import numpy as np
    single = prec == "fp32"
    dt = np.float32 if single else np.float64
    n = q.shape[0]
    qf = np.asfortranarray(q, dtype=dt)
    sf = np.asfortranarray(s, dtype=dt)
    h = ctypes.c_void_p(0)
    check(lib().msqrt_factor_wrap(_lib.PREC_NAMES[prec], _lib.STRUCT_NAMES[structure], _lib.REAL64, n,
                                  qf.ctypes.data_as(ctypes.c_void_p), sf.ctypes.data_as(ctypes.c_void_p),
                                  0, ctypes.byref(h)), "msqrt_factor_wrap")
    return Factor(h.value, n, 1)


def refine(f: Factor, a: torch.Tensor, x: torch.Tensor, init_from_factor=True, maxit=30, tol=1e-13,
           allow_fail=False):
    """Runs the refinement loop in place on x.  Returns the info dict."""
    _check_matrix(a, "A")
    _check_matrix(x, "X")
    n, batch, nn = _dims(a)
    info = _lib.Info()
    st = lib().msqrt_refine(f.handle, ctypes.c_void_p(a.data_ptr()), n, nn,
                            ctypes.c_void_p(x.data_ptr()), n, nn, 1 if init_from_factor else 0,
                            int(maxit), float(tol), _stream(), ctypes.byref(info))
    d = info.to_dict()
    d["status"] = _lib.STATUS_NAMES.get(st, st)
    if not allow_fail:
        check(st, "msqrt_refine")
    return d


def refine_noalloc(f: Factor, a: torch.Tensor, x: torch.Tensor, init_from_factor=True, maxit=30,
                   tol=1e-13, allow_fail=False):
    """refine() through msqrt_refine_noalloc: no device allocation, static
    scratch (HPD factors, bounded size).  Returns the info dict."""
    _check_matrix(a, "A")
    _check_matrix(x, "X")
    n, batch, nn = _dims(a)
    info = _lib.Info()
    st = lib().msqrt_refine_noalloc(f.handle, ctypes.c_void_p(a.data_ptr()), n, nn,
                                    ctypes.c_void_p(x.data_ptr()), n, nn,
                                    1 if init_from_factor else 0, int(maxit), float(tol),
                                    _stream(), ctypes.byref(info))
    d = info.to_dict()
    d["status"] = _lib.STATUS_NAMES.get(st, st)
    if not allow_fail:
        check(st, "msqrt_refine_noalloc")
    return d


def sqrtm(a: torch.Tensor, prec="fp32", structure="auto", maxit=30, tol=1e-13, blks=32,
          fallback=True, keep_factor=False, allow_fail=False, out=None, real_schur=True):
    """Principal square root of a (batch of) matrices.  Returns (X, info) or
    (X, info, factor) when keep_factor is set.  real_schur selects the real
    Schur form (default) or the complex one for real nonsymmetric input."""
    if isinstance(a, torch.Tensor) and not a.is_contiguous():
        a = a.contiguous()
    _check_matrix(a, "A")
    if prec == "auto":
        _ensure_selector()
    n, batch, nn = _dims(a)
    x = torch.empty_like(a) if out is None else out
    o = default_options(prec=prec, structure=structure, maxit=maxit, tol=tol, blks=blks,
                        fallback=fallback, batch=batch, real_schur=real_schur)
    info = _lib.Info()
    h = ctypes.c_void_p(0)
    dt = _lib.COMPLEX128 if a.is_complex() else _lib.REAL64
    st = lib().msqrt_sqrtm(ctypes.byref(o), dt, n, ctypes.c_void_p(a.data_ptr()), n, nn,
                           ctypes.c_void_p(x.data_ptr()), n, nn, _stream(), ctypes.byref(info),
                           ctypes.byref(h) if keep_factor else None)
    d = info.to_dict()
    d["status"] = _lib.STATUS_NAMES.get(st, st)
    if not allow_fail:
        check(st, "msqrt_sqrtm")
    if keep_factor:
        return x, d, (Factor(h.value, n, batch) if h.value else None)
    return x, d


def rootm(a: torch.Tensor, p=3, prec="fp32", maxit=30, tol=1e-13, blks=32, fallback=True,
          allow_fail=False, out=None):
    """Principal p-th root (p = 2 or 3) of one matrix through msqrt_rootm.
    Returns (X, info)."""
    if isinstance(a, torch.Tensor) and not a.is_contiguous():
        a = a.contiguous()
    _check_matrix(a, "A")
    if a.dim() != 2:
        raise ValueError("rootm takes one matrix")
    n = a.shape[-1]
    x = torch.empty_like(a) if out is None else out
    o = default_options(prec=prec, structure="general" if p == 3 else "auto", maxit=maxit, tol=tol,
                        blks=blks, fallback=fallback, batch=1)
    info = _lib.Info()
    dt = _lib.COMPLEX128 if a.is_complex() else _lib.REAL64
    st = lib().msqrt_rootm(ctypes.byref(o), int(p), dt, n, ctypes.c_void_p(a.data_ptr()), n,
                           ctypes.c_void_p(x.data_ptr()), n, _stream(), ctypes.byref(info))
    d = info.to_dict()
    d["status"] = _lib.STATUS_NAMES.get(st, st)
    if not allow_fail:
        check(st, "msqrt_rootm")
    return x, d


def sqrtm_backward(f: Factor, x: torch.Tensor, gbar: torch.Tensor, maxit=30, tol=1e-13):
    _check_matrix(x, "X")
    gbar = gbar.contiguous()
    _check_matrix(gbar, "Gbar")
    n, batch, nn = _dims(x)
    g = torch.empty_like(gbar)
    info = _lib.Info()
    st = lib().msqrt_sqrtm_backward(f.handle, ctypes.c_void_p(x.data_ptr()), n,
                                    ctypes.c_void_p(gbar.data_ptr()), n,
                                    ctypes.c_void_p(g.data_ptr()), n, nn, int(maxit), float(tol),
                                    _stream(), ctypes.byref(info))
    check(st, "msqrt_sqrtm_backward")
    return g, info.to_dict()


def test_sytrd(a, prec="fp32"):
    """Test hook: (d, e, tau) of the on-device tridiagonalisation of host A."""
    import numpy as np
    dt = np.float32 if prec == "fp32" else np.float64
    a = np.asfortranarray(a, dtype=dt)
    n = a.shape[0]
    d = np.zeros(n, dt)
    e = np.zeros(max(n - 1, 1), dt)
    tau = np.zeros(max(n - 1, 1), dt)
    vp = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    check(lib().msqrt_test_sytrd(_lib.PREC_NAMES[prec], n, vp(a), vp(d), vp(e), vp(tau)),
          "msqrt_test_sytrd")
    return d, e[: n - 1], tau[: n - 1]


def test_sy2tr(a, prec="fp32"):
    """Test hook: (d, e, Q) of the on-device two-stage tridiagonalisation of
    host A (A = Q T Q^T)."""
    import numpy as np
    dt = np.float32 if prec == "fp32" else np.float64
    a = np.asfortranarray(a, dtype=dt)
    n = a.shape[0]
    d = np.zeros(n, dt)
    e = np.zeros(max(n - 1, 1), dt)
    q = np.zeros((n, n), dt, order="F")
    vp = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    check(lib().msqrt_test_sy2tr(_lib.PREC_NAMES[prec], n, vp(a), vp(d), vp(e), vp(q)),
          "msqrt_test_sy2tr")
    return d, e[: n - 1], q


def test_stedc(d, e, prec="fp32"):
    """Test hook: (lam, Z) of the on-device divide-and-conquer eigensolver."""
    import numpy as np
    dt = np.float32 if prec == "fp32" else np.float64
    n = len(d)
    d = np.ascontiguousarray(d, dtype=dt)
    e = np.ascontiguousarray(np.concatenate([np.asarray(e, dt), np.zeros(1, dt)]))
    lam = np.zeros(n, np.float64)
    z = np.zeros((n, n), dt, order="F")
    vp = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    check(lib().msqrt_test_stedc(_lib.PREC_NAMES[prec], n, vp(d), vp(e), vp(lam), vp(z)),
          "msqrt_test_stedc")
    return lam, z


def _cplx_f(a):
    import numpy as np
    return np.asfortranarray(a, dtype=np.complex128)


def _dp(x):
    return ctypes.cast(x.ctypes.data, ctypes.POINTER(ctypes.c_double))


def test_gehrd(a, prec="fp32"):
    """Test hook: (H, Q) of the on-device Hessenberg reduction, A = Q H Q^*."""
    import numpy as np
    a = _cplx_f(a)
    n = a.shape[0]
    h = np.zeros((n, n), np.complex128, order="F")
    q = np.zeros((n, n), np.complex128, order="F")
    check(lib().msqrt_test_gehrd(_lib.PREC_NAMES[prec], n, _dp(a), _dp(h), _dp(q)),
          "msqrt_test_gehrd")
    return h, q


def test_schur(a, prec="fp32"):
    """Test hook: (T, Q) of the on-device complex Schur decomposition."""
    import numpy as np
    a = _cplx_f(a)
    n = a.shape[0]
    t = np.zeros((n, n), np.complex128, order="F")
    q = np.zeros((n, n), np.complex128, order="F")
    check(lib().msqrt_test_schur(_lib.PREC_NAMES[prec], n, _dp(a), _dp(t), _dp(q)),
          "msqrt_test_schur")
    return t, q


def test_trsqrt(t, prec="fp32"):
    """Test hook: principal square root of an upper triangular matrix."""
    import numpy as np
    t = _cplx_f(t)
    n = t.shape[0]
    s = np.zeros((n, n), np.complex128, order="F")
    check(lib().msqrt_test_trsqrt(_lib.PREC_NAMES[prec], n, _dp(t), _dp(s)), "msqrt_test_trsqrt")
    return s


def test_trcbrt(t, prec="fp32"):
    """Test hook: principal cube root of an upper triangular matrix."""
    import numpy as np
    t = _cplx_f(t)
    n = t.shape[0]
    u = np.zeros((n, n), np.complex128, order="F")
    check(lib().msqrt_test_trcbrt(_lib.PREC_NAMES[prec], n, _dp(t), _dp(u)), "msqrt_test_trcbrt")
    return u


def test_trsyl(s, s2, c, prec="fp32"):
    """Test hook: Y with S Y + Y S2 = C (S, S2 upper triangular)."""
    import numpy as np
    s, s2, c = _cplx_f(s), _cplx_f(s2), _cplx_f(c)
    m, p = c.shape
    y = np.zeros((m, p), np.complex128, order="F")
    check(lib().msqrt_test_trsyl(_lib.PREC_NAMES[prec], m, p, _dp(s), _dp(s2), _dp(c), _dp(y)),
          "msqrt_test_trsyl")
    return y


def test_gemm_f32(a, b, split=False, ta=False, tb=False):
    """Test hook: C = op(A) op(B) with the float or the BF16-split MFMA GEMM."""
    import numpy as np
    a = np.asfortranarray(a, dtype=np.float32)
    b = np.asfortranarray(b, dtype=np.float32)
    m = a.shape[1] if ta else a.shape[0]
    k = a.shape[0] if ta else a.shape[1]
    n = b.shape[0] if tb else b.shape[1]
    c = np.zeros((m, n), np.float32, order="F")
    vp = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    check(lib().msqrt_test_gemm_f32(1 if split else 0, 1 if ta else 0, 1 if tb else 0, m, n, k,
                                    vp(a), vp(b), vp(c)), "msqrt_test_gemm_f32")
    return c


def test_syrk(a, prec="fp32"):
    """Test hook: C = A A^T through the symmetric-output (mirroring) GEMM."""
    import numpy as np
    dt = np.float32 if prec == "fp32" else np.float64
    a = np.asfortranarray(a, dtype=dt)
    n, k = a.shape
    c = np.zeros((n, n), dt, order="F")
    vp = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    check(lib().msqrt_test_syrk(_lib.PREC_NAMES[prec], n, k, vp(a), vp(c)), "msqrt_test_syrk")
    return c


class _SqrtmFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, prec, tol, maxit):
        x, info, f = sqrtm(a.contiguous(), prec=prec, tol=tol, maxit=maxit, keep_factor=True)
        ctx.factor = f
        ctx.tol = tol
        ctx.maxit = maxit
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        g, _ = sqrtm_backward(ctx.factor, x, gx.contiguous(), maxit=ctx.maxit, tol=ctx.tol)
        return g, None, None, None


def sqrtm_autograd(a: torch.Tensor, prec="fp32", tol=1e-13, maxit=30) -> torch.Tensor:
    """Differentiable principal square root (gradient: X G + G X = dL/dX for
    symmetric positive definite A; X^H G + G X^H = dL/dX in general)."""
    return _SqrtmFn.apply(a, prec, tol, maxit)
