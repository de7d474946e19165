"""Python binding of the C ABI in include/stmf.h (argument marshalling only).

Every function here forwards to ``libstmf.so``; all computation runs in the
library's HIP kernels on the GPU.  Tensors are torch CUDA tensors (device
memory and streams only); host-side arguments are numpy arrays.  If the
library is missing or does not load, importing this module raises: there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstmf.so")

STMF_OK, STMF_EINVAL, STMF_EEMPTY_LINE, STMF_ERANGE, STMF_ENOMEM, STMF_EHIP, STMF_EBUSY, STMF_ETIMEOUT = range(8)

# every exported entry point declared in include/stmf.h
EXPORTS = (
    "stmf_status_str", "stmf_version", "stmf_maxplus_product", "stmf_masked_error_workspace",
    "stmf_masked_error", "stmf_update_workspace", "stmf_update_U", "stmf_update_V",
    "stmf_options_default", "stmf_fit_workspace", "stmf_fit", "stmf_draw_init",
    "stmf_fit_batched_workspace", "stmf_fit_batched", "stmf_engine_create", "stmf_engine_destroy",
    "stmf_job_footprint", "stmf_engine_admit", "stmf_batch_tick", "stmf_engine_poll",
    "stmf_engine_retire", "stmf_engine_set_graph", "stmf_dcor_workspace", "stmf_distance_correlation",
    "stmf_completion_metrics_workspace", "stmf_completion_metrics", "stmf_engine_job_footprint",
    "stmf_masked_error_noalloc",
)


class StmfError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} (status {status})")


class Options(C.Structure):
    _fields_ = [
        ("init_mode", C.c_int), ("init_lo", C.c_float), ("init_hi", C.c_float),
        ("acol_p", C.c_int), ("U0", C.c_void_p), ("perm", C.c_void_p), ("eps", C.c_double),
        ("count_scope", C.c_int), ("noop_rule", C.c_int), ("integer_exact", C.c_int),
        ("decision_log", C.c_void_p), ("log_cap", C.c_int), ("batch_first", C.c_int),
        ("batch_max", C.c_int), ("group_size", C.c_int), ("max_row_visits", C.c_int),
        ("selection", C.c_int), ("perm_mode", C.c_int), ("strategy", C.c_int),
        ("barrier_wait_us", C.c_int),
    ]


class FitInfo(C.Structure):
    _fields_ = [
        ("trials", C.c_longlong), ("spec_trials", C.c_longlong), ("noops", C.c_longlong),
        ("accepted", C.c_longlong), ("row_visits", C.c_longlong), ("cells", C.c_longlong),
        ("iters_done", C.c_int), ("transposed", C.c_int), ("m_work", C.c_int),
        ("n_work", C.c_int), ("group_size", C.c_int), ("nlog", C.c_int),
        ("batches", C.c_longlong), ("phase_ms", C.c_double * 8), ("kernel_ms", C.c_double),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["phase_ms"] = list(self.phase_ms)
        return d


class Problem(C.Structure):
    _fields_ = [
        ("R", C.c_void_p), ("M", C.c_void_p), ("m", C.c_int), ("n", C.c_int),
        ("rank", C.c_int), ("iters", C.c_int), ("seed", C.c_uint64), ("U_out", C.c_void_p),
        ("V_out", C.c_void_p), ("err_traj", C.c_void_p), ("status", C.c_int), ("pad", C.c_int),
    ]


LOG_DTYPE = np.dtype([("iter", "<i4"), ("row", "<i4"), ("trials", "<i4"), ("noops", "<i4"),
                      ("j", "<i4"), ("k", "<i4"), ("op", "<i4"), ("pad", "<i4"), ("e", "<f8")])


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2205_06619_amd.build")
    # torch first: its wheel carries its own HIP runtime under the same
    # soname, and the library must bind to that one.  Loaded the other way
    # round, a process holds two HIP runtimes, torch's streams and memory are
    # foreign to the library's, and the library's first device query fails.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, I, Z = C.c_void_p, C.c_int, C.c_size_t
    sig = {
        "stmf_status_str": ([I], C.c_char_p),
        "stmf_version": ([], C.c_char_p),
        "stmf_maxplus_product": ([P, P, I, I, I, P, P, P], I),
        "stmf_masked_error_workspace": ([I, I, I], Z),
        "stmf_masked_error": ([P, P, P, P, I, I, I, P, P, P, Z, P], I),
        "stmf_masked_error_noalloc": ([P, P, P, P, I, I, I, P, P, P], I),
        "stmf_update_workspace": ([I, I, I], Z),
        "stmf_update_U": ([P, P, P, P, I, I, I, I, I, I, P, P, P, P, Z, P], I),
        "stmf_update_V": ([P, P, P, P, I, I, I, I, I, I, P, P, P, P, Z, P], I),
        "stmf_options_default": ([P], None),
        "stmf_fit_workspace": ([I, I, I, I, P], Z),
        "stmf_fit": ([P, P, I, I, I, I, C.c_uint64, P, P, P, P, P, P, Z, P], I),
        "stmf_draw_init": ([I, I, I, C.c_uint64, P, P, P], I),
        "stmf_fit_batched_workspace": ([P, I, I, P], Z),
        "stmf_fit_batched": ([P, I, I, P, P, P, Z, P], I),
        "stmf_engine_create": ([P, Z, I, P, P], I),
        "stmf_engine_destroy": ([P], None),
        "stmf_job_footprint": ([I, I, I, I], Z),
        "stmf_engine_job_footprint": ([P, I, I, I, I], Z),
        "stmf_engine_admit": ([P, P, P, I, I, I, I, C.c_uint64, P, P], I),
        "stmf_batch_tick": ([P, I, P], I),
        "stmf_engine_poll": ([P, I, P, P], I),
        "stmf_engine_retire": ([P, I, P, P, P, P, P], I),
        "stmf_engine_set_graph": ([P, I], I),
        "stmf_dcor_workspace": ([I], Z),
        "stmf_distance_correlation": ([P, P, I, P, P, P, Z, P], I),
        "stmf_completion_metrics_workspace": ([I, I, I], Z),
        "stmf_completion_metrics": ([P, P, P, P, P, I, I, I, P, P, Z, P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


lib = _load()


def status_str(s: int) -> str:
    return lib.stmf_status_str(int(s)).decode()


def _chk(s: int, where: str):
    if s != STMF_OK:
        raise StmfError(s, where)


# ------------------------------------------------------------------ torch glue
def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a CUDA (device) tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _check(t, dtype, shape, name):
    torch = _torch()
    if t.dtype != dtype or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected {dtype} {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")


def workspace(nbytes: int, device=None):
    """Device workspace of at least nbytes (256-byte aligned)."""
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")


def options(**kw) -> Options:
    o = Options()
    lib.stmf_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


# ------------------------------------------------------------------ primitives
def stmf_maxplus_product(U, V, P=None, argmax=None, stream=None):
    """P = U (x) V and the lowest argmax; allocates outputs that are None."""
    torch = _torch()
    m, r = U.shape
    n = V.shape[1]
    _check(U, torch.float32, (m, r), "U"); _check(V, torch.float32, (r, n), "V")
    if P is None:
        P = torch.empty((m, n), dtype=torch.float32, device=U.device)
    if argmax is None:
        argmax = torch.empty((m, n), dtype=torch.int32, device=U.device)
    _chk(lib.stmf_maxplus_product(_ptr(U), _ptr(V), m, r, n, _ptr(P), _ptr(argmax), _stream(stream)),
         "stmf_maxplus_product")
    return P, argmax


def stmf_masked_error(R, M, U, V, td_col=None, ws=None, stream=None):
    """Masked b-norm; returns (err tensor (1,) float64, td_col (n,) float64)."""
    torch = _torch()
    m, n = R.shape
    r = U.shape[1]
    _check(R, torch.float32, (m, n), "R"); _check(M, torch.uint8, (m, n), "M")
    _check(U, torch.float32, (m, r), "U"); _check(V, torch.float32, (r, n), "V")
    need = lib.stmf_masked_error_workspace(m, n, r)
    if ws is None:
        ws = workspace(need, R.device)
    err = torch.empty(1, dtype=torch.float64, device=R.device)
    if td_col is None:
        td_col = torch.empty(n, dtype=torch.float64, device=R.device)
    _chk(lib.stmf_masked_error(_ptr(R), _ptr(M), _ptr(U), _ptr(V), m, n, r, _ptr(err), _ptr(td_col),
                               _ptr(ws), ws.numel(), _stream(stream)), "stmf_masked_error")
    return err, td_col


def stmf_masked_error_noalloc(R, M, U, V, err=None, td_col=None, stream=None):
    """Masked b-norm through the entry point that allocates nothing (its
    scratch is the library's static device array); err and td_col are
    allocated here when None.  Returns (err tensor (1,), td_col (n,))."""
    torch = _torch()
    m, n = R.shape
    r = U.shape[1]
    _check(R, torch.float32, (m, n), "R"); _check(M, torch.uint8, (m, n), "M")
    _check(U, torch.float32, (m, r), "U"); _check(V, torch.float32, (r, n), "V")
    if err is None:
        err = torch.empty(1, dtype=torch.float64, device=R.device)
    if td_col is None:
        td_col = torch.empty(n, dtype=torch.float64, device=R.device)
    _chk(lib.stmf_masked_error_noalloc(_ptr(R), _ptr(M), _ptr(U), _ptr(V), m, n, r, _ptr(err),
                                       _ptr(td_col), _stream(stream)), "stmf_masked_error_noalloc")
    return err, td_col


def _update(fn, name, R, M, U, V, i, j, k, ws, stream):
    torch = _torch()
    m, n = R.shape
    r = U.shape[1]
    _check(R, torch.float32, (m, n), "R"); _check(M, torch.uint8, (m, n), "M")
    _check(U, torch.float32, (m, r), "U"); _check(V, torch.float32, (r, n), "V")
    if ws is None:
        ws = workspace(lib.stmf_update_workspace(m, n, r), R.device)
    Ub = torch.empty(m, dtype=torch.float32, device=R.device)
    Vb = torch.empty(n, dtype=torch.float32, device=R.device)
    err = torch.empty(1, dtype=torch.float64, device=R.device)
    _chk(fn(_ptr(R), _ptr(M), _ptr(U), _ptr(V), m, n, r, int(i), int(j), int(k), _ptr(Ub), _ptr(Vb),
            _ptr(err), _ptr(ws), ws.numel(), _stream(stream)), name)
    return err, Ub, Vb


def stmf_update_U(R, M, U, V, i, j, k, ws=None, stream=None):
    """F-ULF in place on U, V; returns (err, U_col_prev, V_row_prev)."""
    return _update(lib.stmf_update_U, "stmf_update_U", R, M, U, V, i, j, k, ws, stream)


def stmf_update_V(R, M, U, V, i, j, k, ws=None, stream=None):
    """F-URF in place on U, V; returns (err, U_col_prev, V_row_prev)."""
    return _update(lib.stmf_update_V, "stmf_update_V", R, M, U, V, i, j, k, ws, stream)


# ------------------------------------------------------------------ fitting
@dataclass
class FitResult:
    U: object
    V: object
    traj: np.ndarray
    info: dict
    log: Optional[np.ndarray] = None


def _opts(opt: Optional[Options], kw) -> Options:
    if opt is None:
        opt = options()
    for k, v in kw.items():
        setattr(opt, k, v)
    return opt


def stmf_fit_workspace(m, n, rank, iters, opt=None) -> int:
    return int(lib.stmf_fit_workspace(m, n, rank, iters, C.byref(opt) if opt is not None else None))


def stmf_fit(R, M, rank, iters, seed=0, opt: Optional[Options] = None, ws=None, log_cap=0,
             U0=None, perm=None, stream=None, **kw) -> FitResult:
    """FastSTMF (Algorithm 3) on the GPU.  U0 / perm: host numpy arrays
    (working orientation) for init_mode=2 / an explicit permutation."""
    torch = _torch()
    m, n = R.shape
    _check(R, torch.float32, (m, n), "R"); _check(M, torch.uint8, (m, n), "M")
    opt = _opts(opt, kw)
    keep = []
    if U0 is not None:
        U0 = np.ascontiguousarray(U0, dtype=np.float32); keep.append(U0)
        opt.U0 = U0.ctypes.data; opt.init_mode = 2
    if perm is not None:
        perm = np.ascontiguousarray(perm, dtype=np.int32); keep.append(perm)
        opt.perm = perm.ctypes.data
    log = None
    if log_cap:
        log = torch.zeros(log_cap * LOG_DTYPE.itemsize, dtype=torch.uint8, device=R.device)
        opt.decision_log = log.data_ptr(); opt.log_cap = log_cap
    need = lib.stmf_fit_workspace(m, n, rank, iters, C.byref(opt))
    if need == 0:
        raise StmfError(STMF_EINVAL, "stmf_fit_workspace")
    if ws is None or ws.numel() < need:
        ws = workspace(need, R.device)
    U = torch.empty((m, rank), dtype=torch.float32, device=R.device)
    V = torch.empty((rank, n), dtype=torch.float32, device=R.device)
    traj = np.zeros(iters + 1, np.float64)
    info = FitInfo()
    s = lib.stmf_fit(_ptr(R), _ptr(M), m, n, rank, iters, C.c_uint64(seed), _ptr(U), _ptr(V),
                     traj.ctypes.data_as(C.c_void_p), C.byref(opt), C.byref(info), _ptr(ws),
                     ws.numel(), _stream(stream))
    del keep
    _chk(s, "stmf_fit")
    logarr = None
    if log is not None:
        raw = log.cpu().numpy().view(LOG_DTYPE)
        logarr = raw[: min(info.nlog, log_cap)]
    return FitResult(U, V, traj, info.as_dict(), logarr)


def stmf_draw_init(m, n, rank, seed, opt: Optional[Options] = None, **kw):
    opt = _opts(opt, kw)
    mw = min(m, n)
    perm = np.zeros(mw, np.int32)
    cnt = rank * opt.acol_p if opt.init_mode == 1 else mw * rank
    U0 = np.zeros(cnt, np.float32)
    _chk(lib.stmf_draw_init(m, n, rank, C.c_uint64(seed), C.byref(opt),
                            perm.ctypes.data_as(C.c_void_p), U0.ctypes.data_as(C.c_void_p)),
         "stmf_draw_init")
    return perm, U0


def stmf_fit_batched(problems: Sequence[dict], restarts=1, opt: Optional[Options] = None, ws=None,
                     stream=None, **kw):
    """Batched fits.  problems: dicts with R, M (device tensors), rank, iters,
    seed.  Returns (list of (U, V, traj) per problem with a leading restart
    axis, statuses, info)."""
    torch = _torch()
    opt = _opts(opt, kw)
    arr = (Problem * len(problems))()
    outs = []
    for p, pr in enumerate(problems):
        R, M = pr["R"], pr["M"]
        m, n = R.shape
        rank, iters = int(pr["rank"]), int(pr["iters"])
        U = torch.empty((restarts, m, rank), dtype=torch.float32, device=R.device)
        V = torch.empty((restarts, rank, n), dtype=torch.float32, device=R.device)
        T = torch.zeros((restarts, iters + 1), dtype=torch.float64, device=R.device)
        arr[p] = Problem(R.data_ptr(), M.data_ptr(), m, n, rank, iters, int(pr.get("seed", 0)),
                         U.data_ptr(), V.data_ptr(), T.data_ptr(), 0, 0)
        outs.append((U, V, T))
    need = lib.stmf_fit_batched_workspace(arr, len(problems), restarts, C.byref(opt))
    if need == 0:
        raise StmfError(STMF_EINVAL, "stmf_fit_batched_workspace")
    if ws is None or ws.numel() < need:
        ws = workspace(need)
    info = FitInfo()
    _chk(lib.stmf_fit_batched(arr, len(problems), restarts, C.byref(opt), C.byref(info), _ptr(ws),
                              ws.numel(), _stream(stream)), "stmf_fit_batched")
    statuses = [arr[p].status for p in range(len(problems))]
    return outs, statuses, info.as_dict()


# ------------------------------------------------------------------ serving
def stmf_job_footprint(m, n, rank, iters) -> int:
    """Arena bytes one job of this shape holds from admission to retirement."""
    return int(lib.stmf_job_footprint(m, n, rank, iters))


def stmf_engine_job_footprint(eng: "Engine", m, n, rank, iters) -> int:
    """The same for a job of this engine (its options and group size)."""
    return int(lib.stmf_engine_job_footprint(eng.handle, m, n, rank, iters))


class Engine:
    """Handle of a continuous-batching engine (stmf_engine_create) and the
    arena tensor it lives in."""

    def __init__(self, handle, arena, max_slots, opt):
        self.handle = handle
        self.arena = arena
        self.max_slots = max_slots
        self.opt = opt
        self.shapes = {}  # slot -> (m, n, rank, iters)


def stmf_engine_create(arena_bytes: int, max_slots: int, opt: Optional[Options] = None,
                       device=None, **kw) -> Engine:
    """An engine over a fresh device arena of arena_bytes."""
    opt = _opts(opt, kw)
    arena = workspace(arena_bytes, device)
    h = C.c_void_p()
    _chk(lib.stmf_engine_create(_ptr(arena), arena.numel(), max_slots, C.byref(opt), C.byref(h)),
         "stmf_engine_create")
    return Engine(h, arena, max_slots, opt)


def stmf_engine_destroy(eng: Engine):
    if eng.handle:
        lib.stmf_engine_destroy(eng.handle)
        eng.handle = None


def stmf_engine_admit(eng: Engine, R, M, rank, iters, seed=0, stream=None) -> Optional[int]:
    """Admit a job; returns its slot, or None when no slot or arena room is
    free (STMF_EBUSY).  Other errors raise."""
    torch = _torch()
    m, n = R.shape
    _check(R, torch.float32, (m, n), "R"); _check(M, torch.uint8, (m, n), "M")
    slot = C.c_int(-1)
    s = lib.stmf_engine_admit(eng.handle, _ptr(R), _ptr(M), m, n, rank, iters, C.c_uint64(seed),
                              C.byref(slot), _stream(stream))
    if s == STMF_EBUSY:
        return None
    _chk(s, "stmf_engine_admit")
    eng.shapes[slot.value] = (m, n, rank, iters)
    return slot.value


def stmf_batch_tick(eng: Engine, max_rows: int, stream=None):
    """Advance every resident job by at most max_rows row visits."""
    _chk(lib.stmf_batch_tick(eng.handle, max_rows, _stream(stream)), "stmf_batch_tick")


def stmf_engine_set_graph(eng: Engine, on: bool):
    """Ticks as a captured HIP graph (default) or as eager launches."""
    _chk(lib.stmf_engine_set_graph(eng.handle, 1 if on else 0), "stmf_engine_set_graph")


def stmf_engine_poll(eng: Engine, slot: int, stream=None) -> bool:
    done = C.c_int(0)
    _chk(lib.stmf_engine_poll(eng.handle, slot, C.byref(done), _stream(stream)), "stmf_engine_poll")
    return bool(done.value)


def stmf_engine_retire(eng: Engine, slot: int, stream=None) -> FitResult:
    """Results of a finished job (U, V on the device, host trajectory); frees
    its slot and arena memory."""
    torch = _torch()
    m, n, rank, iters = eng.shapes[slot]
    U = torch.empty((m, rank), dtype=torch.float32, device=eng.arena.device)
    V = torch.empty((rank, n), dtype=torch.float32, device=eng.arena.device)
    traj = np.zeros(iters + 1, np.float64)
    info = FitInfo()
    _chk(lib.stmf_engine_retire(eng.handle, slot, _ptr(U), _ptr(V), traj.ctypes.data_as(C.c_void_p),
                                C.byref(info), _stream(stream)), "stmf_engine_retire")
    del eng.shapes[slot]
    return FitResult(U, V, traj, info.as_dict())


# ------------------------------------------------------------------ quality
def stmf_distance_correlation(x, y, row_terms=False, ws=None, stream=None):
    """Distance correlation of two device float32 vectors: dict with dcor,
    dcov2, dvarx2, dvary2 (and row_terms, an (N, 5) float64 tensor, if asked)."""
    torch = _torch()
    N = x.numel()
    _check(x, torch.float32, (N,), "x"); _check(y, torch.float32, (N,), "y")
    need = lib.stmf_dcor_workspace(N)
    if ws is None or ws.numel() < need:
        ws = workspace(need, x.device)
    terms = torch.empty((N, 5), dtype=torch.float64, device=x.device) if row_terms else None
    out = np.zeros(4, np.float64)
    _chk(lib.stmf_distance_correlation(_ptr(x), _ptr(y), N, out.ctypes.data_as(C.c_void_p),
                                       _ptr(terms), _ptr(ws), ws.numel(), _stream(stream)),
         "stmf_distance_correlation")
    res = dict(dcor=float(out[0]), dcov2=float(out[1]), dvarx2=float(out[2]), dvary2=float(out[3]))
    if row_terms:
        res["row_terms"] = terms
    return res


def stmf_completion_metrics(R, M_train, M_test, U, V, ws=None, stream=None):
    """RMSE-A, RMSE-P and DC of a factorization on a held-out split (device
    tensors); returns a dict with rmse_a, rmse_p, dc, n_train, n_test."""
    torch = _torch()
    m, n = R.shape
    r = U.shape[1]
    _check(R, torch.float32, (m, n), "R")
    _check(M_train, torch.uint8, (m, n), "M_train"); _check(M_test, torch.uint8, (m, n), "M_test")
    _check(U, torch.float32, (m, r), "U"); _check(V, torch.float32, (r, n), "V")
    need = lib.stmf_completion_metrics_workspace(m, n, r)
    if need == 0:
        raise StmfError(STMF_EINVAL, "stmf_completion_metrics_workspace")
    if ws is None or ws.numel() < need:
        ws = workspace(need, R.device)
    out = np.zeros(5, np.float64)
    _chk(lib.stmf_completion_metrics(_ptr(R), _ptr(M_train), _ptr(M_test), _ptr(U), _ptr(V), m, n, r,
                                     out.ctypes.data_as(C.c_void_p), _ptr(ws), ws.numel(),
                                     _stream(stream)), "stmf_completion_metrics")
    return dict(rmse_a=float(out[0]), rmse_p=float(out[1]), dc=float(out[2]),
                n_train=int(out[3]), n_test=int(out[4]))

