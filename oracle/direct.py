"""ctypes wrapper over the oracle's C direct summation (``direct.c``).

Test infrastructure only.  Computes the plain definitions:
kernel (Sec. 3, eq. extended_Gaussian_ANOVA_kernel, weighted as in Sec. 5),
product K alpha (Sec. 2, eq. mult_with_K), the shifted product
(K + beta I) alpha of the normal equation (Sec. 2), and the sum over training
points at new points, s(z_i) = sum_j alpha_j kappa(z_i, x_j) (Sec. 4.2,
eq. kernelsum; used for prediction in Sec. 4.3).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from . import _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        P = ctypes.POINTER
        lib.oracle_anova_matvec.restype = ctypes.c_int
        lib.oracle_anova_matvec.argtypes = [
            P(ctypes.c_double), ctypes.c_int64, ctypes.c_int64,
            P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_double), ctypes.c_int32,
            ctypes.c_double, ctypes.c_double,
            P(ctypes.c_double), ctypes.c_int32, ctypes.c_int64,
            P(ctypes.c_int64), ctypes.c_int64, P(ctypes.c_double)]
        lib.oracle_anova_predict.restype = ctypes.c_int
        lib.oracle_anova_predict.argtypes = [
            P(ctypes.c_double), ctypes.c_int64, ctypes.c_int64,
            P(ctypes.c_double), ctypes.c_int64, ctypes.c_int64,
            P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_double), ctypes.c_int32,
            ctypes.c_double, P(ctypes.c_double), ctypes.c_int32, ctypes.c_int64,
            P(ctypes.c_int64), ctypes.c_int64, P(ctypes.c_double)]
        lib.oracle_kernel_block.restype = None
        lib.oracle_kernel_block.argtypes = [
            P(ctypes.c_double), ctypes.c_int64,
            P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_double), ctypes.c_int32,
            ctypes.c_double, P(ctypes.c_int64), ctypes.c_int64, P(ctypes.c_int64),
            ctypes.c_int64, P(ctypes.c_double)]
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _windows(windows):
    P = len(windows)
    feat = np.zeros(3 * P, dtype=np.int32)
    dA = np.zeros(P, dtype=np.int32)
    eta = np.zeros(P, dtype=np.float64)
    for l, w in enumerate(windows):
        f = tuple(w.feat) if hasattr(w, "feat") else tuple(w[0])
        e = w.eta if hasattr(w, "eta") else w[1]
        if not 1 <= len(f) <= 3:
            raise ValueError("a window holds 1, 2 or 3 features")
        dA[l] = len(f)
        feat[3 * l:3 * l + len(f)] = f
        eta[l] = e
    return feat, dA, eta


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def set_threads(n: int) -> None:
    """Threads of later oracle calls (n >= 1)."""
    _load().oracle_set_threads(int(n))


def anova_matvec(X: np.ndarray, windows, ell: float, beta: float, alpha: np.ndarray,
                 rows: Optional[Sequence[int]] = None, return_threads: bool = False):
    """((K + beta I) alpha)[rows] in float64.  X: (N, d); alpha: (N,) or
    (N, nrhs).  Returns (len(rows), nrhs) or (N,) for a vector alpha."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    N, d = X.shape
    vec = alpha.ndim == 1
    A = np.asfortranarray(alpha.reshape(N, -1), dtype=np.float64)
    nrhs = A.shape[1]
    feat, dA, eta = _windows(windows)
    if rows is None:
        rows_arr = None
        nrows = N
    else:
        rows_arr = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        nrows = rows_arr.size
        if nrows and (rows_arr.min() < 0 or rows_arr.max() >= N):
            raise IndexError("row index out of range")
    out = np.zeros((nrhs, nrows), dtype=np.float64)
    nt = lib.oracle_anova_matvec(
        _ptr(X, ctypes.c_double), N, d, _ptr(feat, ctypes.c_int32), _ptr(dA, ctypes.c_int32),
        _ptr(eta, ctypes.c_double), len(windows), float(ell), float(beta),
        _ptr(A, ctypes.c_double), nrhs, N,
        None if rows_arr is None else _ptr(rows_arr, ctypes.c_int64), nrows,
        _ptr(out, ctypes.c_double))
    res = out.T
    if vec:
        res = res[:, 0]
    return (res, nt) if return_threads else res


def anova_predict(Z: np.ndarray, X: np.ndarray, windows, ell: float, alpha: np.ndarray,
                  rows: Optional[Sequence[int]] = None, return_threads: bool = False):
    """s(z_i) = sum_j alpha_j kappa(z_i, x_j) for i in rows (all of Z by
    default), in float64.  Z: (Nz, d) new points; X: (N, d) training points;
    alpha: (N,) or (N, nrhs).  Returns (len(rows), nrhs), or a vector for a
    vector alpha."""
    lib = _load()
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    N, d = X.shape
    Nz, dz = Z.shape
    if dz != d:
        raise ValueError("Z and X must have the same number of features")
    vec = alpha.ndim == 1
    A = np.asfortranarray(alpha.reshape(N, -1), dtype=np.float64)
    nrhs = A.shape[1]
    feat, dA, eta = _windows(windows)
    if rows is None:
        rows_arr = None
        nrows = Nz
    else:
        rows_arr = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        nrows = rows_arr.size
        if nrows and (rows_arr.min() < 0 or rows_arr.max() >= Nz):
            raise IndexError("row index out of range")
    out = np.zeros((nrhs, nrows), dtype=np.float64)
    nt = lib.oracle_anova_predict(
        _ptr(Z, ctypes.c_double), Nz, d, _ptr(X, ctypes.c_double), N, d,
        _ptr(feat, ctypes.c_int32), _ptr(dA, ctypes.c_int32), _ptr(eta, ctypes.c_double),
        len(windows), float(ell), _ptr(A, ctypes.c_double), nrhs, N,
        None if rows_arr is None else _ptr(rows_arr, ctypes.c_int64), nrows,
        _ptr(out, ctypes.c_double))
    res = out.T
    if vec:
        res = res[:, 0]
    return (res, nt) if return_threads else res


def kernel_block(X: np.ndarray, windows, ell: float, rows: Sequence[int],
                 cols: Sequence[int]) -> np.ndarray:
    """Dense block K[rows][:, cols] of the ANOVA kernel matrix (no shift)."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    N, d = X.shape
    feat, dA, eta = _windows(windows)
    ri = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    cj = np.ascontiguousarray(np.asarray(cols, dtype=np.int64))
    out = np.zeros((ri.size, cj.size), dtype=np.float64)
    lib.oracle_kernel_block(_ptr(X, ctypes.c_double), d, _ptr(feat, ctypes.c_int32),
                            _ptr(dA, ctypes.c_int32), _ptr(eta, ctypes.c_double),
                            len(windows), float(ell), _ptr(ri, ctypes.c_int64), ri.size,
                            _ptr(cj, ctypes.c_int64), cj.size, _ptr(out, ctypes.c_double))
    return out


def kernel_matrix(X: np.ndarray, windows, ell: float) -> np.ndarray:
    """The full N x N kernel matrix K (small N only)."""
    idx = np.arange(X.shape[0])
    return kernel_block(X, windows, ell, idx, idx)
