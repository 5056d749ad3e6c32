"""FP64 CPU oracle of the CF-completion hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of the
benchmark use it to produce expected values.  The GPU product path never imports it.

The arithmetic lives in ``oracle.c`` (ridge row solve, ALS-WR fit, objective, Alg. 2,
residual) and ``mlp.py`` (surrogate network).  This module only marshals numpy arrays into
the C library, converting every floating-point input to float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.oracle_ridge_rows.argtypes = [i64, i32, P, P, P, P, f64, i32, P, P]
        lib.oracle_ridge_rows.restype = i64
        lib.oracle_ridge_subset.argtypes = [i64, P, i32, P, P, P, P, f64, i32, P, P]
        lib.oracle_ridge_subset.restype = i64
        lib.oracle_csr_to_csc.argtypes = [i64, i32, P, P, P, P, P, P]
        lib.oracle_csr_to_csc.restype = None
        lib.oracle_objective.argtypes = [i64, i32, i32, P, P, P, P, P, f64, i32]
        lib.oracle_objective.restype = f64
        lib.oracle_fit.argtypes = [i64, i32, i32, P, P, P, f64, i32, i32, P, P, P]
        lib.oracle_fit.restype = i32
        lib.oracle_predict_select.argtypes = [i64, i32, i32, P, P, P, P, i32, f64, P, P, P, P]
        lib.oracle_predict_select.restype = None
        lib.oracle_residual.argtypes = [i64, i32, P, P, P, P, P, P]
        lib.oracle_residual.restype = None
        lib.oracle_set_threads.argtypes = [i32]
        lib.oracle_set_threads.restype = None
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = i32
        _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else ctypes.c_void_p(0)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def ridge_rows(row_ptr, col, val, F, lam, weighted=True):
    """Fold-in / half-sweep: one ridge solve per CSR row against fixed factors F.
    Returns (X f64[m,k], status int32[m])."""
    lib = _load()
    row_ptr, col, val, F = _i64(row_ptr), _i32(col), _f64(val), _f64(F)
    m, k = len(row_ptr) - 1, F.shape[1]
    X = np.zeros((m, k))
    st = np.zeros(m, dtype=np.int32)
    lib.oracle_ridge_rows(m, k, _p(row_ptr), _p(col), _p(val), _p(F), float(lam), int(bool(weighted)), _p(X), _p(st))
    return X, st


def ridge_subset(rows, row_ptr, col, val, F, lam, weighted=True):
    """Ridge solve of the listed rows only.  Returns (X f64[len(rows),k], status)."""
    lib = _load()
    rows, row_ptr, col, val, F = _i64(rows), _i64(row_ptr), _i32(col), _f64(val), _f64(F)
    k = F.shape[1]
    X = np.zeros((len(rows), k))
    st = np.zeros(len(rows), dtype=np.int32)
    lib.oracle_ridge_subset(len(rows), _p(rows), k, _p(row_ptr), _p(col), _p(val), _p(F), float(lam),
                            int(bool(weighted)), _p(X), _p(st))
    return X, st


def csr_to_csc(row_ptr, col, val, n):
    lib = _load()
    row_ptr, col, val = _i64(row_ptr), _i32(col), _f64(val)
    m = len(row_ptr) - 1
    nnz = int(row_ptr[-1])
    col_ptr = np.zeros(n + 1, dtype=np.int64)
    ridx = np.zeros(max(nnz, 1), dtype=np.int32)
    cval = np.zeros(max(nnz, 1))
    lib.oracle_csr_to_csc(m, n, _p(row_ptr), _p(col), _p(val), _p(col_ptr), _p(ridx), _p(cval))
    return col_ptr, ridx[:nnz], cval[:nnz]


def objective(row_ptr, col, val, U, V, lam, weighted=True) -> float:
    lib = _load()
    row_ptr, col, val, U, V = _i64(row_ptr), _i32(col), _f64(val), _f64(U), _f64(V)
    return float(lib.oracle_objective(len(row_ptr) - 1, V.shape[0], U.shape[1], _p(row_ptr), _p(col), _p(val),
                                      _p(U), _p(V), float(lam), int(bool(weighted))))


def fit(row_ptr, col, val, U0, V0, lam, sweeps, weighted=True):
    """ALS-WR from (U0, V0).  Returns (U, V, obj f64[2*sweeps])."""
    lib = _load()
    row_ptr, col, val = _i64(row_ptr), _i32(col), _f64(val)
    U, V = _f64(U0).copy(), _f64(V0).copy()
    obj = np.zeros(2 * sweeps)
    lib.oracle_fit(len(row_ptr) - 1, V.shape[0], U.shape[1], _p(row_ptr), _p(col), _p(val), float(lam),
                   int(bool(weighted)), int(sweeps), _p(U), _p(V), _p(obj))
    return U, V, obj


def predict_select(U, V, cap_c, cap_g, base, gamma, want_p=False):
    """Alg. 2 per row on p = U V^T.  Returns (best int32[m], saving f64[m], status int32[m], P or None)."""
    lib = _load()
    U, V, cap_c, cap_g = _f64(U), _f64(V), _f64(cap_c), _f64(cap_g)
    m, k, n = U.shape[0], U.shape[1], V.shape[0]
    P = np.zeros((m, n)) if want_p else None
    best = np.zeros(m, dtype=np.int32)
    saving = np.zeros(m)
    st = np.zeros(m, dtype=np.int32)
    lib.oracle_predict_select(m, n, k, _p(U), _p(V), _p(cap_c), _p(cap_g), int(base), float(gamma), _p(P),
                              _p(best), _p(saving), _p(st))
    return best, saving, st, P


def residual(row_ptr, col, val, U, V):
    lib = _load()
    row_ptr, col, val, U, V = _i64(row_ptr), _i32(col), _f64(val), _f64(U), _f64(V)
    m = len(row_ptr) - 1
    rho = np.zeros(m)
    lib.oracle_residual(m, U.shape[1], _p(row_ptr), _p(col), _p(val), _p(U), _p(V), _p(rho))
    return rho
