"""Python face of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  It loads ``liboracle.so`` built from ``stmf_oracle.cpp`` (plain
C++ loops restating the paper's definitions; see that file's header) and
marshals numpy arrays.  Nothing here is on the GPU library's path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class Opts(C.Structure):
    _fields_ = [
        ("init_mode", C.c_int),
        ("init_lo", C.c_float),
        ("init_hi", C.c_float),
        ("acol_p", C.c_int),
        ("U0", C.c_void_p),
        ("perm", C.c_void_p),
        ("eps", C.c_double),
        ("count_scope", C.c_int),
        ("noop_rule", C.c_int),
        ("integer_exact", C.c_int),
        ("selection", C.c_int),
        ("perm_mode", C.c_int),
        ("strategy", C.c_int),
    ]


class LogRec(C.Structure):
    _fields_ = [
        ("iter", C.c_int32), ("row", C.c_int32), ("trials", C.c_int32),
        ("noops", C.c_int32), ("j", C.c_int32), ("k", C.c_int32),
        ("op", C.c_int32), ("pad", C.c_int32), ("e", C.c_double),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("trials", C.c_int64), ("noops", C.c_int64), ("accepted", C.c_int64),
        ("row_visits", C.c_int64), ("iters_done", C.c_int32),
        ("transposed", C.c_int32), ("evaluated_cells", C.c_int64),
    ]


class LockReport(C.Structure):
    _fields_ = [
        ("row_visits", C.c_int64), ("trials", C.c_int64), ("agree", C.c_int64),
        ("flips", C.c_int64), ("flips_f32_accepts", C.c_int64), ("mismatches", C.c_int64),
        ("order_pairs", C.c_int64),
        ("order_flips", C.c_int64), ("order_mismatches", C.c_int64), ("k_checked", C.c_int64),
        ("k_flips", C.c_int64), ("k_mismatches", C.c_int64), ("iters_done", C.c_int32),
        ("first_bad_iter", C.c_int32), ("first_bad_row", C.c_int32), ("pad", C.c_int32),
        ("max_rel_traj", C.c_double), ("max_flip_margin", C.c_double),
    ]


LOG_DTYPE = np.dtype([("iter", "<i4"), ("row", "<i4"), ("trials", "<i4"),
                      ("noops", "<i4"), ("j", "<i4"), ("k", "<i4"),
                      ("op", "<i4"), ("pad", "<i4"), ("e", "<f8")])


def build(force: bool = False) -> str:
    import importlib
    return importlib.import_module(__name__ + ".build").build(force=force)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        for suf in ("f64", "f32"):
            getattr(L, f"oracle_maxplus_{suf}").argtypes = [P, P, C.c_int, C.c_int, C.c_int, P, P]
            f = getattr(L, f"oracle_masked_error_{suf}")
            f.argtypes = [P, P, P, P, C.c_int, C.c_int, C.c_int, P, P]
            f.restype = C.c_double
            for nm in ("col_res", "row_res"):
                getattr(L, f"oracle_{nm}_{suf}").argtypes = [P, P, C.c_int, C.c_int, C.c_int, C.c_int, P, P]
            for nm in ("update_U", "update_V"):
                f = getattr(L, f"oracle_{nm}_{suf}")
                f.argtypes = [P, P, P, P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P, P, P]
                f.restype = C.c_double
            f = getattr(L, f"oracle_fit_{suf}")
            f.argtypes = [P, P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint64, P, P, P, P, P,
                          C.c_int, P, P, C.c_int]
            f.restype = C.c_int
        L.oracle_lockstep.argtypes = [P, P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint64, P,
                                      C.c_double, P, P, P, C.c_int, P, P]
        L.oracle_lockstep.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_get_threads.restype = C.c_int
        L.oracle_splitmix64.argtypes = [C.c_uint64, C.c_int, P]
        L.oracle_draw_init.argtypes = [P, P, C.c_int, C.c_int, C.c_int, C.c_uint64, P, P, P]
        L.oracle_draw_init.restype = C.c_int
        _lib = L
    return _lib


def _dt(prec: str):
    if prec not in ("f64", "f32"):
        raise ValueError(prec)
    return np.float64 if prec == "f64" else np.float32


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def maxplus(U, V, prec="f64"):
    T = _dt(prec)
    U = _c(U, T); V = _c(V, T)
    m, r = U.shape; n = V.shape[1]
    P = np.empty((m, n), T); A = np.empty((m, n), np.int32)
    getattr(lib(), f"oracle_maxplus_{prec}")(_p(U), _p(V), m, r, n, _p(P), _p(A))
    return P, A


def masked_error(R, M, U, V, prec="f64"):
    T = _dt(prec)
    R = _c(R, T); M = _c(M, np.uint8); U = _c(U, T); V = _c(V, T)
    m, n = R.shape; r = U.shape[1]
    td = np.empty(n, np.float64); A = np.empty((m, n), np.int32)
    e = getattr(lib(), f"oracle_masked_error_{prec}")(_p(R), _p(M), _p(U), _p(V), m, n, r, _p(td), _p(A))
    return e, td, A


def col_res(R, M, U, V, k, prec="f64"):
    """Returns a copy of V with row k replaced by the column residual of U[:, k]."""
    T = _dt(prec)
    R = _c(R, T); M = _c(M, np.uint8); U = _c(U, T); V = _c(V, T).copy()
    m, n = R.shape; r = U.shape[1]
    getattr(lib(), f"oracle_col_res_{prec}")(_p(R), _p(M), m, n, r, k, _p(U), _p(V))
    return V


def row_res(R, M, U, V, k, prec="f64"):
    """Returns a copy of U with column k replaced by the row residual of V[k, :]."""
    T = _dt(prec)
    R = _c(R, T); M = _c(M, np.uint8); U = _c(U, T).copy(); V = _c(V, T)
    m, n = R.shape; r = U.shape[1]
    getattr(lib(), f"oracle_row_res_{prec}")(_p(R), _p(M), m, n, r, k, _p(V), _p(U))
    return U


def update(op, R, M, U, V, i, j, k, prec="f64"):
    """One F-ULF (op='U') or F-URF (op='V') trial on copies of U, V.

    Returns (U', V', e', U_col_prev, V_row_prev, td_col').
    """
    T = _dt(prec)
    R = _c(R, T); M = _c(M, np.uint8); U = _c(U, T).copy(); V = _c(V, T).copy()
    m, n = R.shape; r = U.shape[1]
    Ub = np.empty(m, T); Vb = np.empty(n, T); td = np.empty(n, np.float64)
    fn = getattr(lib(), f"oracle_update_{'U' if op == 'U' else 'V'}_{prec}")
    e = fn(_p(R), _p(M), _p(U), _p(V), m, n, r, i, j, k, _p(Ub), _p(Vb), _p(td))
    return U, V, e, Ub, Vb, td


@dataclass
class FitResult:
    status: int
    U: np.ndarray
    V: np.ndarray
    traj: np.ndarray
    log: np.ndarray
    stats: dict


def make_opts(init_mode=0, init_lo=0.0, init_hi=100.0, acol_p=5, U0=None, perm=None,
              eps=0.0, count_scope=0, noop_rule=1, integer_exact=0, selection=0, perm_mode=0,
              strategy=0):
    o = Opts()
    o.init_mode = init_mode; o.init_lo = init_lo; o.init_hi = init_hi; o.acol_p = acol_p
    keep = []
    if U0 is not None:
        U0 = _c(U0, np.float32); keep.append(U0); o.U0 = U0.ctypes.data
    if perm is not None:
        perm = _c(perm, np.int32); keep.append(perm); o.perm = perm.ctypes.data
    o.eps = eps; o.count_scope = count_scope; o.noop_rule = noop_rule
    o.integer_exact = integer_exact
    o.selection = selection; o.perm_mode = perm_mode; o.strategy = strategy
    return o, keep


def fit(R, M, rank, iters, seed=0, prec="f32", log_cap=None, row_limit=0, no_traj=False,
        **opts) -> FitResult:
    """Algorithm 3 on the oracle.  prec='f64' is the FP64 oracle.  no_traj:
    pass no trajectory buffer (the returned traj stays zero)."""
    R = _c(R, np.float32); M = _c(M, np.uint8)
    m, n = R.shape
    o, keep = make_opts(**opts)
    U = np.zeros((m, rank), np.float32); V = np.zeros((rank, n), np.float32)
    traj = np.zeros(iters + 1, np.float64)
    mw = min(m, n)
    cap = log_cap if log_cap is not None else mw * max(iters, 1)
    log = np.zeros(max(cap, 1), LOG_DTYPE)
    nlog = C.c_int(0)
    st = Stats()
    fn = getattr(lib(), f"oracle_fit_{prec}")
    s = fn(_p(R), _p(M), m, n, rank, iters, C.c_uint64(seed), C.byref(o), _p(U), _p(V),
           None if no_traj else _p(traj), _p(log), cap, C.byref(nlog), C.byref(st), row_limit)
    del keep
    stats = {f: getattr(st, f) for f, _ in Stats._fields_}
    return FitResult(s, U, V, traj, log[: min(nlog.value, cap)], stats)


@dataclass
class LockResult:
    status: int
    traj_f32: np.ndarray
    traj_f64: np.ndarray
    log: np.ndarray
    report: dict


def lockstep(R, M, rank, iters, seed=0, band=1e-6, log_cap=None, **opts) -> LockResult:
    """The FP32-value fit (FastSTMF: ByRow, TD_A) with every decision replayed
    in FP64 from the same state (see oracle_lockstep in stmf_oracle.cpp)."""
    R = _c(R, np.float32); M = _c(M, np.uint8)
    m, n = R.shape
    o, keep = make_opts(**opts)
    tf = np.zeros(iters + 1, np.float64); td = np.zeros(iters + 1, np.float64)
    mw = min(m, n)
    cap = log_cap if log_cap is not None else mw * max(iters, 1)
    log = np.zeros(max(cap, 1), LOG_DTYPE)
    nlog = C.c_int(0)
    rep = LockReport()
    s = lib().oracle_lockstep(_p(R), _p(M), m, n, rank, iters, C.c_uint64(seed), C.byref(o),
                              band, _p(tf), _p(td), _p(log), cap, C.byref(nlog), C.byref(rep))
    del keep
    report = {f: getattr(rep, f) for f, _ in LockReport._fields_ if f != "pad"}
    return LockResult(s, tf, td, log[: min(nlog.value, cap)], report)


def set_threads(n: int) -> None:
    """Threads of the oracle's row loops (OpenMP); results do not depend on it."""
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, np.uint64)
    lib().oracle_splitmix64(C.c_uint64(seed), count, _p(out))
    return out


def draw_init(R, M, rank, seed, **opts):
    R = _c(R, np.float32); M = _c(M, np.uint8)
    m, n = R.shape
    mw = min(m, n)
    o, keep = make_opts(**opts)
    perm = np.zeros(mw, np.int32); U0 = np.zeros((mw, rank), np.float32)
    s = lib().oracle_draw_init(_p(R), _p(M), m, n, rank, C.c_uint64(seed), C.byref(o), _p(perm), _p(U0))
    del keep
    return s, perm, U0
