"""Oracle O1 from Python: the plain product over Z/pZ (test infrastructure only).

Thin ctypes wrapper around ``matmul_ref.c``.  Only tests/, the smoke check and
the benchmark's CPU-baseline leg may call it.

Value computed (Section 3.2's operation over Z/pZ):
    C_out = (alpha * (A @ B) + beta * C_in) mod p,  canonical in [0, p).
Inputs may be int64 or float64 arrays holding integers; float64 is converted
exactly (every canonical residue below 2**31 is an exact double).
"""
import ctypes
import os

import numpy as np

from .build import build_oracle

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = build_oracle()
        lib = ctypes.CDLL(path)
        i64 = ctypes.c_int64
        p64 = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_matmul_mod_p.argtypes = [i64, i64, i64, i64, p64, i64, p64, i64,
                                            p64, i64, i64, i64, ctypes.c_int]
        lib.oracle_matmul_mod_p.restype = ctypes.c_int
        lib.oracle_matmul_entries.argtypes = [i64, i64, i64, i64, p64, i64, p64, i64,
                                              p64, i64, i64, i64, i64, p64, p64, p64,
                                              ctypes.c_int]
        lib.oracle_matmul_entries.restype = ctypes.c_int
        _lib = lib
    return _lib


def _as_i64(x):
    x = np.asarray(x)
    if x.dtype == np.int64:
        return np.ascontiguousarray(x)
    if x.dtype.kind == "f":
        y = x.astype(np.int64)
        if not np.array_equal(y.astype(x.dtype), x):
            raise ValueError("float input holds a non-integer value")
        return np.ascontiguousarray(y)
    return np.ascontiguousarray(x.astype(np.int64))


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def matmul_mod_p(A, B, C=None, alpha=1, beta=0, p=2, threads=0):
    """Return (alpha*A@B + beta*C) mod p as a new int64 array."""
    lib = _load()
    A = _as_i64(A)
    B = _as_i64(B)
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    if C is None:
        out = np.zeros((m, n), dtype=np.int64)
        beta = 0
    else:
        out = _as_i64(C).copy()
        if out.shape != (m, n):
            raise ValueError("C has the wrong shape")
    dummy = np.zeros(1, dtype=np.int64)
    rc = lib.oracle_matmul_mod_p(m, k, n, int(p),
                                 _ptr(A if A.size else dummy), max(k, 1),
                                 _ptr(B if B.size else dummy), max(n, 1),
                                 _ptr(out if out.size else dummy), max(n, 1),
                                 int(alpha), int(beta), int(threads))
    if rc == -2:
        raise ValueError("an entry is outside [0, p)")
    if rc != 0:
        raise ValueError("bad arguments")
    return out


def matmul_entries(A, B, C, alpha, beta, p, rows, cols, threads=0):
    """Return the entries (rows[t], cols[t]) of (alpha*A@B + beta*C) mod p."""
    lib = _load()
    A = _as_i64(A)
    B = _as_i64(B)
    m, k = A.shape
    n = B.shape[1]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros(rows.shape[0], dtype=np.int64)
    if C is None or beta % p == 0:
        Cin = np.zeros(1, dtype=np.int64)
        beta = 0
        ldc = 1
    else:
        Cin = _as_i64(C)
        ldc = n
    dummy = np.zeros(1, dtype=np.int64)
    rc = lib.oracle_matmul_entries(m, k, n, int(p),
                                   _ptr(A if A.size else dummy), max(k, 1),
                                   _ptr(B if B.size else dummy), max(n, 1),
                                   _ptr(Cin), ldc, int(alpha), int(beta),
                                   rows.shape[0], _ptr(rows), _ptr(cols), _ptr(out),
                                   int(threads))
    if rc != 0:
        raise ValueError("bad arguments")
    return out


def threads_available() -> int:
    """Number of host threads the oracle uses by default."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1
