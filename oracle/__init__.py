"""Oracle for banded solves: TEST INFRASTRUCTURE ONLY.

A thin ctypes wrapper over ``band_oracle.c``: plain FP64 banded Gaussian
elimination (with and without partial pivoting) for ``A X = F`` and
``A^T X = F``, in real and in complex arithmetic (``A^H`` too), banded
products, residual metrics and a 1-norm condition estimate.  Only ``tests/``, the smoke check and the CPU-baseline leg of the
benchmark use it.  The solver library never imports it, and it imports
nothing from the solver library.

Band arrays are numpy arrays of shape ``(n, ldab)`` in C order, i.e. LAPACK
column-major band storage with ``ab[j, ku + i - j] = A(i, j)``.  Right-hand
sides are ``(nrhs, n)`` C-order arrays (column-major ``n x nrhs``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "band_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double
_p = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            lib.orc_gbsv.restype = _i64
            lib.orc_gbsv.argtypes = [_i64, _int, _int, _p, _i64, _int, _int, _int, _p, _i64]
            lib.orc_gbsv_nt.restype = _i64
            lib.orc_gbsv_nt.argtypes = [_i64, _int, _int, _p, _i64, _int, _int, _p, _p, _i64]
            lib.orc_gbtrf.restype = _i64
            lib.orc_gbtrf.argtypes = [_i64, _int, _int, _p, _i64, _int, _p, _p]
            lib.orc_gbtrs.restype = None
            lib.orc_gbtrs.argtypes = [_i64, _int, _int, _p, _p, _int, _int, _int, _p, _i64]
            lib.orc_zgbsv.restype = _i64
            lib.orc_zgbsv.argtypes = [_i64, _int, _int, _p, _i64, _int, _int, _int, _p, _i64]
            lib.orc_zgbmv.restype = None
            lib.orc_zgbmv.argtypes = [_i64, _int, _int, _p, _i64, _int, _int, _p, _i64, _p, _i64]
            lib.orc_zrelres.restype = _dbl
            lib.orc_zrelres.argtypes = [_i64, _int, _int, _p, _i64, _int, _int, _p, _i64, _p, _i64]
            lib.orc_gbmv.restype = None
            lib.orc_gbmv.argtypes = [_i64, _int, _int, _p, _i64, _int, _int, _p, _i64, _p, _i64]
            lib.orc_gbnorm.restype = _dbl
            lib.orc_gbnorm.argtypes = [_i64, _int, _int, _p, _i64, _int]
            lib.orc_relres.restype = _dbl
            lib.orc_relres.argtypes = [_i64, _int, _int, _p, _i64, _int, _int, _p, _i64, _p, _i64]
            lib.orc_gbcond1.restype = _dbl
            lib.orc_gbcond1.argtypes = [_i64, _int, _int, _p, _i64]
            lib.orc_r13.restype = _dbl
            lib.orc_r13.argtypes = [_dbl, _dbl]
            _lib = lib
    return _lib


def _band(ab, kl, ku):
    ab = np.ascontiguousarray(ab, dtype=np.float64)
    n, ldab = ab.shape
    if ldab < kl + ku + 1:
        raise ValueError("ldab too small")
    return ab, n, ldab


def _rhs(F, n):
    F = np.array(F, dtype=np.float64, order="C", copy=True)
    if F.ndim == 1:
        F = F[None, :]
    if F.shape[1] != n:
        raise ValueError("rhs must have shape (nrhs, n)")
    return F


def gbsv(ab, kl, ku, F, pivot=True, trans=False):
    """Return X with op(A) X = F (F given as (nrhs, n) or (n,)).  Raises on a
    zero pivot."""
    ab, n, ldab = _band(ab, kl, ku)
    squeeze = np.ndim(F) == 1
    X = _rhs(F, n)
    info = _load().orc_gbsv(n, kl, ku, ab.ctypes.data, ldab, int(bool(pivot)), int(bool(trans)),
                            X.shape[0], X.ctypes.data, max(n, 1))
    if info != 0:
        raise ZeroDivisionError("oracle factorisation info=%d" % info)
    return X[0] if squeeze else X


def gbsv_nt(ab, kl, ku, F, pivot=True):
    """One factorisation, then (A^{-1} F, A^{-T} F)."""
    ab, n, ldab = _band(ab, kl, ku)
    X = _rhs(F, n)
    Xt = X.copy()
    info = _load().orc_gbsv_nt(n, kl, ku, ab.ctypes.data, ldab, int(bool(pivot)), X.shape[0],
                               X.ctypes.data, Xt.ctypes.data, max(n, 1))
    if info != 0:
        raise ZeroDivisionError("oracle factorisation info=%d" % info)
    return X, Xt


def gbtrf(ab, kl, ku, pivot=True):
    """Factor only.  Returns (info, w, ipiv) with the working band w of shape
    (n, 2kl+ku+1) (pivot) or (n, kl+ku+1) and 0-based pivots."""
    ab, n, ldab = _band(ab, kl, ku)
    ldw = kl + (kl + ku if pivot else ku) + 1
    w = np.zeros((n, ldw), dtype=np.float64)
    ipiv = np.zeros(n, dtype=np.int64)
    info = _load().orc_gbtrf(n, kl, ku, ab.ctypes.data, ldab, int(bool(pivot)),
                             w.ctypes.data, ipiv.ctypes.data)
    return int(info), w, ipiv


def gbtrs(w, ipiv, kl, ku, F, pivot=True, trans=False):
    """Solve op(A) X = F with the factors (w, ipiv) of gbtrf (same pivot
    flag); F as (nrhs, n) or (n,)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int64)
    n = w.shape[0]
    squeeze = np.ndim(F) == 1
    X = _rhs(F, n)
    _load().orc_gbtrs(n, kl, ku, w.ctypes.data, ipiv.ctypes.data, int(bool(pivot)), int(bool(trans)),
                      X.shape[0], X.ctypes.data, max(n, 1))
    return X[0] if squeeze else X


def gbmv(ab, kl, ku, X, trans=False):
    """Return op(A) X for X of shape (nrhs, n) or (n,)."""
    ab, n, ldab = _band(ab, kl, ku)
    squeeze = np.ndim(X) == 1
    Xc = _rhs(X, n)
    Y = np.zeros_like(Xc)
    _load().orc_gbmv(n, kl, ku, ab.ctypes.data, ldab, int(bool(trans)), Xc.shape[0],
                     Xc.ctypes.data, max(n, 1), Y.ctypes.data, max(n, 1))
    return Y[0] if squeeze else Y


def gbnorm(ab, kl, ku, which="inf"):
    ab, n, ldab = _band(ab, kl, ku)
    return _load().orc_gbnorm(n, kl, ku, ab.ctypes.data, ldab, 0 if which == "inf" else 1)


def relres(ab, kl, ku, X, F, trans=False):
    """max over columns of ||F - op(A) X||_inf / (||op(A)||_inf ||X||_inf)."""
    ab, n, ldab = _band(ab, kl, ku)
    Xc = _rhs(X, n)
    Fc = _rhs(F, n)
    return _load().orc_relres(n, kl, ku, ab.ctypes.data, ldab, int(bool(trans)), Xc.shape[0],
                              Xc.ctypes.data, max(n, 1), Fc.ctypes.data, max(n, 1))


def cond1(ab, kl, ku):
    """Hager/Higham estimate of the 1-norm condition number."""
    ab, n, ldab = _band(ab, kl, ku)
    return _load().orc_gbcond1(n, kl, ku, ab.ctypes.data, ldab)


def r13(K, nrhs_over_k):
    """Load-balancing ratio R13 = n1/n3 of the paper's load-balancing section."""
    return _load().orc_r13(float(K), float(nrhs_over_k))


_ZTRANS = {False: 0, True: 1, "N": 0, "T": 1, "C": 2, 0: 0, 1: 1, 2: 2}


def _zband(ab, kl, ku):
    ab = np.ascontiguousarray(ab, dtype=np.complex128)
    n, ldab = ab.shape
    if ldab < kl + ku + 1:
        raise ValueError("ldab too small")
    return ab, n, ldab


def _zrhs(F, n):
    F = np.array(F, dtype=np.complex128, order="C", copy=True)
    if F.ndim == 1:
        F = F[None, :]
    if F.shape[1] != n:
        raise ValueError("rhs must have shape (nrhs, n)")
    return F


def zgbsv(ab, kl, ku, F, pivot=True, trans="N"):
    """Complex band solve: op(A) Z = F with trans "N", "T" (A^T) or "C"
    (A^H); ab complex (n, ldab) in the real band's layout, F (nrhs, n)."""
    ab, n, ldab = _zband(ab, kl, ku)
    squeeze = np.ndim(F) == 1
    X = _zrhs(F, n)
    info = _load().orc_zgbsv(n, kl, ku, ab.ctypes.data, ldab, int(bool(pivot)), _ZTRANS[trans],
                             X.shape[0], X.ctypes.data, max(n, 1))
    if info != 0:
        raise ZeroDivisionError("oracle factorisation info=%d" % info)
    return X[0] if squeeze else X


def zgbmv(ab, kl, ku, X, trans="N"):
    ab, n, ldab = _zband(ab, kl, ku)
    squeeze = np.ndim(X) == 1
    Xc = _zrhs(X, n)
    Y = np.zeros_like(Xc)
    _load().orc_zgbmv(n, kl, ku, ab.ctypes.data, ldab, _ZTRANS[trans], Xc.shape[0], Xc.ctypes.data,
                      max(n, 1), Y.ctypes.data, max(n, 1))
    return Y[0] if squeeze else Y


def zrelres(ab, kl, ku, X, F, trans="N"):
    ab, n, ldab = _zband(ab, kl, ku)
    Xc = _zrhs(X, n)
    Fc = _zrhs(F, n)
    return _load().orc_zrelres(n, kl, ku, ab.ctypes.data, ldab, _ZTRANS[trans], Xc.shape[0], Xc.ctypes.data,
                               max(n, 1), Fc.ctypes.data, max(n, 1))


def fwd_err(X, Xref):
    """max over columns of ||X - Xref||_inf / ||Xref||_inf."""
    X = np.atleast_2d(X)
    Xref = np.atleast_2d(Xref)
    num = np.abs(X - Xref).max(axis=1)
    den = np.abs(Xref).max(axis=1)
    return float(np.max(num / np.where(den > 0, den, 1.0)))
