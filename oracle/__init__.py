"""FP64 CPU oracle for core-elements ALS (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is the independent reference the HIP library is
checked against: plain C in double precision (``coreals_oracle.c``) plus the
NumPy pieces in ``foldin.py``.  It shares no code with the HIP library; the
two only see the same seeded inputs.

Functions cite the passage of Xue, Li, Zhang and Meng, "Core-elements
Subsampling for Alternating Least Squares", that they follow.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "coreals_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

I64P = ctypes.POINTER(ctypes.c_int64)
I32P = ctypes.POINTER(ctypes.c_int32)
F32P = ctypes.POINTER(ctypes.c_float)
F64P = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.ora_num_threads.restype = ctypes.c_int
        L.ora_set_threads.argtypes = [ctypes.c_int]
        L.ora_validate.restype = ctypes.c_int
        L.ora_validate.argtypes = [ctypes.c_int64, ctypes.c_int64, I64P, I32P, F32P]
        L.ora_transpose.argtypes = [ctypes.c_int64, ctypes.c_int64, I64P, I32P, F32P,
                                    I64P, I32P, F32P]
        L.ora_budget.restype = ctypes.c_int64
        L.ora_budget.argtypes = [ctypes.c_int64] * 4
        L.ora_select.argtypes = [ctypes.c_int64, ctypes.c_int32, F64P, ctypes.c_int64, I32P]
        L.ora_core_row.restype = ctypes.c_int
        L.ora_core_row.argtypes = [ctypes.c_int64, ctypes.c_int32, F64P, F64P, ctypes.c_double,
                                   ctypes.c_int64, F64P]
        L.ora_half_sweep.argtypes = [ctypes.c_int64, ctypes.c_int32, I64P, I32P, F32P, F64P,
                                     ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_int64, F64P, I64P]
        L.ora_half_sweep_rows.argtypes = [ctypes.c_int64, I64P, ctypes.c_int32, I64P, I32P, F32P,
                                          F64P, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int64, F64P, I64P]
        L.ora_core_select_rows.argtypes = [ctypes.c_int64, I64P, ctypes.c_int32, I64P, I32P, F64P,
                                           ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, I64P,
                                           I32P]
        L.ora_objective.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, I64P, I32P,
                                    F32P, F64P, F64P, ctypes.c_double, F64P]
        U8P = ctypes.POINTER(ctypes.c_uint8)
        L.ora_global_select.argtypes = [ctypes.c_int64, ctypes.c_int32, F64P, ctypes.c_int64, U8P]
        L.ora_masked_row.restype = ctypes.c_int
        L.ora_masked_row.argtypes = [ctypes.c_int64, ctypes.c_int32, F64P, U8P, F64P, ctypes.c_double, F64P]
        L.ora_fast_half_sweep.argtypes = [ctypes.c_int64, ctypes.c_int32, I64P, I32P, F32P, ctypes.c_int64,
                                          F64P, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int64, F64P, I64P]
        L.ora_splitmix64.restype = ctypes.c_uint64
        L.ora_splitmix64.argtypes = [ctypes.c_uint64]
        L.ora_unif_key.restype = ctypes.c_uint32
        L.ora_unif_key.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.ora_unif_select.argtypes = [ctypes.c_int64, I32P, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                      ctypes.c_int64, U8P]
        L.ora_unif_row.restype = ctypes.c_int
        L.ora_unif_row.argtypes = [ctypes.c_int64, ctypes.c_int32, F64P, U8P, F64P, ctypes.c_double,
                                   ctypes.c_int64, F64P]
        L.ora_unif_half_sweep.argtypes = [ctypes.c_int64, ctypes.c_int32, I64P, I32P, F32P, ctypes.c_int64,
                                          F64P, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_uint64, F64P, I64P]
        L.ora_global_gram.argtypes = [ctypes.c_int64, ctypes.c_int32, F64P, F64P]
        L.ora_implicit_row.restype = ctypes.c_int
        L.ora_implicit_row.argtypes = [ctypes.c_int64, ctypes.c_int32, F64P, F64P, F64P, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int64, F64P]
        L.ora_implicit_half_sweep.argtypes = [ctypes.c_int64, ctypes.c_int32, I64P, I32P, F32P, ctypes.c_int64,
                                              F64P, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                              ctypes.c_int64, ctypes.c_int64, F64P, I64P]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def num_threads() -> int:
    return lib().ora_num_threads()


def set_threads(n: int) -> None:
    lib().ora_set_threads(int(n))


def validate(n_rows, n_cols, row_ptr, col_idx, val) -> int:
    """0 ok, 2 index error, 3 value error (problem statement, Section 2.1)."""
    rp, ci, v = _c(row_ptr, np.int64), _c(col_idx, np.int32), _c(val, np.float32)
    return lib().ora_validate(n_rows, n_cols, _p(rp, I64P), _p(ci, I32P), _p(v, F32P))


def transpose(n_rows, n_cols, row_ptr, col_idx, val):
    """CSR -> CSC (the item half-sweep regresses over I_j^M, Section 2.1)."""
    rp, ci, v = _c(row_ptr, np.int64), _c(col_idx, np.int32), _c(val, np.float32)
    cp = np.zeros(n_cols + 1, np.int64)
    ri = np.zeros(len(ci), np.int32)
    vt = np.zeros(len(ci), np.float32)
    lib().ora_transpose(n_rows, n_cols, _p(rp, I64P), _p(ci, I32P), _p(v, F32P),
                        _p(cp, I64P), _p(ri, I32P), _p(vt, F32P))
    return cp, ri, vt


def budget(n, num, den, min_keep) -> int:
    """s = min(n, max(min_keep, floor(n num/den)))  (selection rule, Section 3)."""
    return int(lib().ora_budget(int(n), int(num), int(den), int(min_keep)))


def select(X, s):
    """CES, Algorithm 1: per column the s positions of largest |x| (ascending)."""
    X = _c(X, np.float64)
    n, nf = X.shape
    pos = np.zeros((nf, max(s, 0)), np.int32)
    if s > 0:
        lib().ora_select(n, nf, _p(X, F64P), int(s), _p(pos, I32P))
    return pos


def core_row(X, y, lam, s):
    """Core estimator for one row, eq. core_ui.  Returns (u, status)."""
    X = _c(X, np.float64)
    y = _c(y, np.float64)
    n, nf = X.shape
    u = np.zeros(nf, np.float64)
    st = lib().ora_core_row(n, nf, _p(X, F64P), _p(y, F64P), float(lam), int(s), _p(u, F64P))
    return u, st


def half_sweep(row_ptr, col_idx, val, other, lam, num, den, min_keep):
    """One half-sweep of Algorithm 2 over the rows of a CSR.  Returns (out, stats)."""
    rp, ci, v = _c(row_ptr, np.int64), _c(col_idx, np.int32), _c(val, np.float32)
    O = _c(other, np.float64)
    n_rows = len(rp) - 1
    nf = O.shape[1]
    out = np.zeros((n_rows, nf), np.float64)
    st = np.zeros(2, np.int64)
    lib().ora_half_sweep(n_rows, nf, _p(rp, I64P), _p(ci, I32P), _p(v, F32P), _p(O, F64P),
                         float(lam), int(num), int(den), int(min_keep), _p(out, F64P),
                         _p(st, I64P))
    return out, st


def half_sweep_rows(rows, row_ptr, col_idx, val, other, lam, num, den, min_keep):
    """half_sweep restricted to the listed rows (sampled checks at full size)."""
    rows = _c(rows, np.int64)
    rp, ci, v = _c(row_ptr, np.int64), _c(col_idx, np.int32), _c(val, np.float32)
    O = _c(other, np.float64)
    nf = O.shape[1]
    out = np.zeros((len(rows), nf), np.float64)
    st = np.zeros(2, np.int64)
    lib().ora_half_sweep_rows(len(rows), _p(rows, I64P), nf, _p(rp, I64P), _p(ci, I32P),
                              _p(v, F32P), _p(O, F64P), float(lam), int(num), int(den),
                              int(min_keep), _p(out, F64P), _p(st, I64P))
    return out, st


def core_select_rows(rows, row_ptr, col_idx, other, num, den, min_keep):
    """CES positions for the listed rows; returns (sel_ptr, sel) where row t's
    column a occupies sel[sel_ptr[t] + a*s : sel_ptr[t] + (a+1)*s]."""
    rows = _c(rows, np.int64)
    rp, ci = _c(row_ptr, np.int64), _c(col_idx, np.int32)
    O = _c(other, np.float64)
    nf = O.shape[1]
    deg = rp[rows + 1] - rp[rows]
    s = np.array([budget(d, num, den, min_keep) for d in deg], np.int64)
    sel_ptr = np.zeros(len(rows) + 1, np.int64)
    np.cumsum(s * nf, out=sel_ptr[1:])
    sel = np.zeros(int(sel_ptr[-1]), np.int32)
    lib().ora_core_select_rows(len(rows), _p(rows, I64P), nf, _p(rp, I64P), _p(ci, I32P),
                               _p(O, F64P), int(num), int(den), int(min_keep),
                               _p(sel_ptr, I64P), _p(sel, I32P))
    return sel_ptr, sel


def global_select(other, num, den, min_keep):
    """Fast variant of Core-ALS (Section 3): CES applied once to the whole factor
    matrix `other` at budget(n_other).  Returns the kept mask (n_other x nf, uint8)."""
    O = _c(other, np.float64)
    n, nf = O.shape
    keep = np.zeros((n, nf), np.uint8)
    lib().ora_global_select(n, nf, _p(O, F64P), budget(n, num, den, min_keep),
                            keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return keep


def masked_row(X, K, y, lam):
    """One regression on the sketch X* = K * X (eq. core_ui).  Returns (u, status)."""
    X = _c(X, np.float64)
    K = _c(K, np.uint8)
    y = _c(y, np.float64)
    n, nf = X.shape
    u = np.zeros(nf, np.float64)
    st = lib().ora_masked_row(n, nf, _p(X, F64P), K.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                              _p(y, F64P), float(lam), _p(u, F64P))
    return u, st


def fast_half_sweep(row_ptr, col_idx, val, other, lam, num, den, min_keep):
    """One half-sweep of the fast variant (Section 3): the global sketch of
    `other`, then every row's regression on it.  Returns (out, stats)."""
    rp, ci, v = _c(row_ptr, np.int64), _c(col_idx, np.int32), _c(val, np.float32)
    O = _c(other, np.float64)
    n_rows = len(rp) - 1
    nf = O.shape[1]
    out = np.zeros((n_rows, nf), np.float64)
    st = np.zeros(2, np.int64)
    lib().ora_fast_half_sweep(n_rows, nf, _p(rp, I64P), _p(ci, I32P), _p(v, F32P), O.shape[0], _p(O, F64P),
                              float(lam), int(num), int(den), int(min_keep), _p(out, F64P), _p(st, I64P))
    return out, st


def splitmix64(x: int) -> int:
    """splitmix64 (Steele, Lea and Flood, 2014): the output for state x."""
    return int(lib().ora_splitmix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def unif_select(cols, row, n_cols, seed, s):
    """UNIF draw of one row (Section 5 comparator): the s entries with the
    smallest keys h(seed, row, col).  Returns the kept mask (uint8 [n])."""
    c = _c(cols, np.int32)
    keep = np.zeros(len(c), np.uint8)
    lib().ora_unif_select(len(c), _p(c, I32P), int(row), int(n_cols), ctypes.c_uint64(seed), int(s),
                          keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return keep


def unif_row(X, keep, y, lam, s):
    """Ridge regression of a UNIF subsample: (X_S^T X_S + lambda s E) u = X_S^T y_S."""
    X = _c(X, np.float64)
    keep = _c(keep, np.uint8)
    y = _c(y, np.float64)
    n, nf = X.shape
    u = np.zeros(nf, np.float64)
    st = lib().ora_unif_row(n, nf, _p(X, F64P), keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                            _p(y, F64P), float(lam), int(s), _p(u, F64P))
    return u, st


def unif_half_sweep(row_ptr, col_idx, val, other, lam, num, den, min_keep, seed):
    """One half-sweep of UNIF (Section 5).  Returns (out, stats)."""
    rp, ci, v = _c(row_ptr, np.int64), _c(col_idx, np.int32), _c(val, np.float32)
    O = _c(other, np.float64)
    n_rows = len(rp) - 1
    nf = O.shape[1]
    out = np.zeros((n_rows, nf), np.float64)
    st = np.zeros(2, np.int64)
    lib().ora_unif_half_sweep(n_rows, nf, _p(rp, I64P), _p(ci, I32P), _p(v, F32P), O.shape[0], _p(O, F64P),
                              float(lam), int(num), int(den), int(min_keep), ctypes.c_uint64(seed),
                              _p(out, F64P), _p(st, I64P))
    return out, st


def implicit_row(X, r, G, lam, alpha, s):
    """Implicit-feedback core regression (reading of Section 3's last
    paragraph): (G + X*^T W X + lambda E) u = X*^T (1 + alpha r), W = diag(alpha r),
    G = Y^T Y.  Returns (u, status)."""
    X = _c(X, np.float64)
    r = _c(r, np.float64)
    G = _c(G, np.float64)
    n, nf = X.shape
    u = np.zeros(nf, np.float64)
    st = lib().ora_implicit_row(n, nf, _p(X, F64P), _p(r, F64P), _p(G, F64P), float(lam), float(alpha), int(s),
                                _p(u, F64P))
    return u, st


def implicit_half_sweep(row_ptr, col_idx, val, other, lam, alpha, num, den, min_keep):
    """One implicit-feedback Core-ALS half-sweep.  Returns (out, stats)."""
    rp, ci, v = _c(row_ptr, np.int64), _c(col_idx, np.int32), _c(val, np.float32)
    O = _c(other, np.float64)
    n_rows = len(rp) - 1
    nf = O.shape[1]
    out = np.zeros((n_rows, nf), np.float64)
    st = np.zeros(2, np.int64)
    lib().ora_implicit_half_sweep(n_rows, nf, _p(rp, I64P), _p(ci, I32P), _p(v, F32P), O.shape[0], _p(O, F64P),
                                  float(lam), float(alpha), int(num), int(den), int(min_keep), _p(out, F64P),
                                  _p(st, I64P))
    return out, st


def objective(row_ptr, col_idx, val, U, M, lam):
    """(f, SSE, RMSE, ReMSE) of eq. for f (Section 2.1) and ReMSE (Section 5.1)."""
    rp, ci, v = _c(row_ptr, np.int64), _c(col_idx, np.int32), _c(val, np.float32)
    U = _c(U, np.float64)
    M = _c(M, np.float64)
    out = np.zeros(4, np.float64)
    lib().ora_objective(U.shape[0], M.shape[0], U.shape[1], _p(rp, I64P), _p(ci, I32P),
                        _p(v, F32P), _p(U, F64P), _p(M, F64P), float(lam), _p(out, F64P))
    return tuple(float(x) for x in out)


def als(problem, iters=None, M0=None, num=None, den=None, record=True):
    """Core-ALS driver, Algorithm 2 (full ALS when r = 1): users from M, then
    items from the new U, for a fixed number of iterations.  Returns
    (U, M, history) with the objective after every half-sweep."""
    p = problem
    iters = p.iters if iters is None else iters
    num = p.budget_num if num is None else num
    den = p.budget_den if den is None else den
    M = np.asarray(p.M0 if M0 is None else M0, np.float64)
    cp, ri, vt = transpose(p.n_u, p.n_m, p.row_ptr, p.col_idx, p.val)
    hist = []
    U = np.zeros((p.n_u, p.n_f))
    for _ in range(iters):
        U, _ = half_sweep(p.row_ptr, p.col_idx, p.val, M, p.lam, num, den, p.min_keep)
        if record:
            hist.append(objective(p.row_ptr, p.col_idx, p.val, U, M, p.lam))
        M, _ = half_sweep(cp, ri, vt, U, p.lam, num, den, p.min_keep)
        if record:
            hist.append(objective(p.row_ptr, p.col_idx, p.val, U, M, p.lam))
    return U, M, hist
