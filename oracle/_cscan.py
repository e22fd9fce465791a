"""ctypes binding of the oracle's plain-C scans (``oracle/scan.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "scan.c"), os.path.join(_HERE, "ldl.c")]
_LIB = os.path.join(_HERE, "_oracle_scan.so")

_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile the scan library with gcc (plain -O2, no FP contraction)."""
    stale = not os.path.exists(_LIB) or \
        any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in _SRCS)
    if force or stale:
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                               "-fPIC", "-shared", "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_price.restype = _i64
        _ci = ctypes.c_int
        L.orc_price.argtypes = [_i64, _i64, _p, _p, _p, _p, _p, _i64, _i64, _p, _p, _p, _ci,
                                _i64]
        L.orc_rmin.restype = ctypes.c_double
        L.orc_rmin.argtypes = [_i64, _i64, _p, _p, _p, _p, _p, _ci]
        L.orc_cost_hist.restype = None
        L.orc_cost_hist.argtypes = [_i64, _i64, _p, _p, _i64, _p, _ci]
        L.orc_collect_le.restype = _i64
        L.orc_collect_le.argtypes = [_i64, _i64, _p, _p, _i64, _p, _i64, _ci]
        L.orc_row_col_argmin.restype = None
        L.orc_row_col_argmin.argtypes = [_i64, _i64, _p, _p, _p, _p, _ci]
        _i32 = ctypes.c_int32
        L.orc_ldl_factor.restype = _p
        L.orc_ldl_factor.argtypes = [_i32, _p, _p, _p, ctypes.c_double]
        L.orc_ldl_free.restype = None
        L.orc_ldl_free.argtypes = [_p]
        L.orc_ldl_nnz.restype = _i64
        L.orc_ldl_nnz.argtypes = [_p]
        L.orc_ldl_ninf.restype = _i32
        L.orc_ldl_ninf.argtypes = [_p]
        L.orc_ldl_solve.restype = None
        L.orc_ldl_solve.argtypes = [_p, _p]
        L.orc_ldl_export.restype = None
        L.orc_ldl_export.argtypes = [_p, _p, _p, _p, _p]
        _lib = L
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def price(xs, xt, y, z, support_idx, kmax, kind=0, key_limit=0):
    """(idx, r, n_negative): the <= kmax most negative reduced costs outside the support
    (cost kind as in scan.c); key_limit > 0 scans only the variables whose cost
    key is below it (the heuristic subset of Section 3.4)."""
    xs = _c(xs, np.int32); xt = _c(xt, np.int32)
    y = _c(y, np.float64); z = _c(z, np.float64)
    sup = _c(support_idx, np.int64)
    m, n = xs.shape[0], xt.shape[0]
    kmax = int(max(kmax, 0))
    out_idx = np.empty(max(kmax, 1), np.int64)
    out_r = np.empty(max(kmax, 1), np.float64)
    nneg = np.zeros(1, np.int64)
    k = lib().orc_price(m, n, _ptr(xs), _ptr(xt), _ptr(y), _ptr(z), _ptr(sup), sup.shape[0],
                        kmax, _ptr(out_idx), _ptr(out_r), _ptr(nneg), int(kind),
                        int(key_limit))
    if k < 0:
        raise MemoryError("orc_price")
    return out_idx[:k].copy(), out_r[:k].copy(), int(nneg[0])


def rmin(xs, xt, y, z, kind=0):
    xs = _c(xs, np.int32); xt = _c(xt, np.int32)
    y = _c(y, np.float64); z = _c(z, np.float64)
    arg = np.zeros(1, np.int64)
    v = lib().orc_rmin(xs.shape[0], xt.shape[0], _ptr(xs), _ptr(xt), _ptr(y), _ptr(z), _ptr(arg),
                       int(kind))
    return float(v), int(arg[0])


def cost_hist(xs, xt, cmax, kind=0):
    xs = _c(xs, np.int32); xt = _c(xt, np.int32)
    h = np.zeros(int(cmax) + 1, np.int64)
    lib().orc_cost_hist(xs.shape[0], xt.shape[0], _ptr(xs), _ptr(xt), int(cmax), _ptr(h), int(kind))
    return h


def collect_le(xs, xt, T, cap, kind=0):
    xs = _c(xs, np.int32); xt = _c(xt, np.int32)
    out = np.empty(max(int(cap), 1), np.int64)
    k = lib().orc_collect_le(xs.shape[0], xt.shape[0], _ptr(xs), _ptr(xt), int(T), _ptr(out), int(cap),
                             int(kind))
    if k > cap:
        raise RuntimeError("collect_le: capacity too small")
    return out[:k].copy()


def row_col_argmin(xs, xt, kind=0):
    xs = _c(xs, np.int32); xt = _c(xt, np.int32)
    ra = np.empty(xs.shape[0], np.int64)
    ca = np.empty(xt.shape[0], np.int64)
    lib().orc_row_col_argmin(xs.shape[0], xt.shape[0], _ptr(xs), _ptr(xt), _ptr(ra), _ptr(ca), int(kind))
    return ra, ca


class LDL:
    """L D L^T of a symmetric sparse matrix (lower triangle used) under a given
    symmetric permutation, with small or negative pivots replaced by +inf
    (``ldl.c``: column by column from the definition of the factorisation)."""

    def __init__(self, S, perm, pivtol):
        import scipy.sparse as sp
        n = S.shape[0]
        self.n = n
        self.perm = np.asarray(perm, np.int64)
        Sp = S.tocsr()[self.perm][:, self.perm]
        Lo = sp.tril(Sp, format="csc")
        Lo.sort_indices()
        Ap = _c(Lo.indptr, np.int32)
        Ai = _c(Lo.indices, np.int32)
        Ax = _c(Lo.data, np.float64)
        self._h = lib().orc_ldl_factor(n, _ptr(Ap), _ptr(Ai), _ptr(Ax), float(pivtol))
        if not self._h:
            raise MemoryError("orc_ldl_factor")
        self.n_inf = int(lib().orc_ldl_ninf(self._h))
        self.nnz_L = int(lib().orc_ldl_nnz(self._h)) + n  # strictly lower part + unit diagonal

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_ldl_free(h)
            self._h = None

    def factors(self):
        """(L as a scipy CSC unit lower triangular matrix, D) in the permuted order."""
        import scipy.sparse as sp
        nnz = self.nnz_L - self.n
        colp = np.empty(self.n + 1, np.int64)
        row = np.empty(max(nnz, 1), np.int32)
        val = np.empty(max(nnz, 1), np.float64)
        d = np.empty(self.n, np.float64)
        lib().orc_ldl_export(self._h, _ptr(colp), _ptr(row), _ptr(val), _ptr(d))
        L = sp.csc_matrix((val[:nnz], row[:nnz], colp), shape=(self.n, self.n))
        return (L + sp.identity(self.n, format="csc")).tocsc(), d

    def solve(self, b):
        x = _c(np.asarray(b, np.float64)[self.perm], np.float64)
        lib().orc_ldl_solve(self._h, _ptr(x))
        out = np.empty_like(x)
        out[self.perm] = x
        return out
