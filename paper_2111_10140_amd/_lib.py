"""Thin ctypes binding over ``libanova.so`` (the C ABI in ``include/anova.h``).

Argument marshalling only: every step of the fast summation and of CG runs
in the library's HIP kernels.  Device arrays are torch CUDA tensors (used for
device memory and streams only).  There is no CPU fallback: if the library is
missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libanova.so")

ANOVA_OK = 0
ANOVA_E_INVALID = 1
ANOVA_E_NOMEM = 2
ANOVA_E_HIP = 3
ANOVA_E_NOT_CONVERGED = 4
ANOVA_E_BREAKDOWN = 5
ANOVA_E_ACCURACY = 6
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_NOMEM", 3: "E_HIP", 4: "E_NOT_CONVERGED",
                5: "E_BREAKDOWN", 6: "E_ACCURACY"}

ANOVA_FP64 = 0
ANOVA_FP32_NFFT = 1

ANOVA_RESIDUAL_FP64 = 0
ANOVA_RESIDUAL_SAME = 1


class anova_window(ctypes.Structure):
    _fields_ = [("d_A", ctypes.c_int32), ("feat", ctypes.c_int32 * 3), ("eta", ctypes.c_double)]


class anova_params(ctypes.Structure):
    _fields_ = [("ell", ctypes.c_double), ("precision", ctypes.c_int32), ("M", ctypes.c_int32),
                ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("h", ctypes.c_double),
                ("target_err", ctypes.c_double), ("center", ctypes.c_int32),
                ("residual", ctypes.c_int32), ("tune", ctypes.c_int32),
                ("reg_q", ctypes.c_int32)]


class anova_window_info(ctypes.Structure):
    _fields_ = [("d_A", ctypes.c_int32), ("M", ctypes.c_int32), ("n", ctypes.c_int32),
                ("m", ctypes.c_int32), ("h", ctypes.c_double), ("center", ctypes.c_double * 3),
                ("extent", ctypes.c_double), ("err_images", ctypes.c_double),
                ("err_trunc", ctypes.c_double), ("err_window", ctypes.c_double),
                ("err_round", ctypes.c_double), ("err_total", ctypes.c_double),
                ("n_tiles", ctypes.c_int64), ("n_subproblems", ctypes.c_int64),
                ("per_cell", ctypes.c_int32), ("tile", ctypes.c_int32)]


class krr_cg_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("relres", ctypes.c_double), ("true_relres", ctypes.c_double)]


class AnovaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
VP = ctypes.c_void_p


def load():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2111_10140_amd/build.py "
                          "(there is no CPU fallback)")
    # torch ships its own HIP runtime; it has to be the one loaded first, so
    # that the library's HIP calls and torch's tensors and streams share one
    # runtime (loading the library first pulls in the system runtime, and
    # the two then disagree about the devices)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sigs = {
        "anova_fastsum_plan": [ctypes.POINTER(VP), VP, i64, i32, i64, ctypes.POINTER(anova_window),
                               i32, ctypes.POINTER(anova_params), VP],
        "anova_matvec": [VP, VP, VP, i32, i64, dbl, VP],
        "anova_matvec_noalloc": [VP, VP, VP, i32, i64, dbl, VP],
        "krr_cg_solve": [VP, VP, VP, i32, i64, dbl, dbl, i32, ctypes.POINTER(krr_cg_info), VP],
        "anova_plan_destroy": [VP],
        "anova_plan_query": [VP, i32, ctypes.POINTER(anova_window_info)],
        "anova_plan_shape": [VP, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "anova_stage_spread": [VP, i32, VP, VP, VP],
        "anova_stage_convolve": [VP, i32, VP, VP],
        "anova_stage_gather": [VP, i32, VP, VP, VP],
        "anova_plan_set_timing": [VP, i32],
        "krr_cg_start": [ctypes.POINTER(VP), VP, VP, VP, i32, i64, dbl, dbl, i32, VP],
        "krr_cg_iterate": [ctypes.POINTER(VP), i32, i32, VP],
        "krr_cg_poll": [VP, ctypes.POINTER(i32), ctypes.POINTER(krr_cg_info), VP],
        "krr_cg_finish": [VP, ctypes.POINTER(krr_cg_info), VP],
        "krr_cg_destroy": [VP],
        "krr_cg_solve_batched": [i32, ctypes.POINTER(VP), ctypes.POINTER(VP), ctypes.POINTER(VP),
                                 ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(dbl),
                                 dbl, i32, ctypes.POINTER(krr_cg_info), VP],
        "anova_plan_stage_times": [VP, ctypes.POINTER(dbl), ctypes.POINTER(i64)],
        "anova_plan_footprint": [VP, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "krr_cg_active": [ctypes.POINTER(VP), i32, VP, VP, VP],
        "anova_fastsum_plan_host": [ctypes.POINTER(VP), VP, i64, i32, i64,
                                    ctypes.POINTER(anova_window), i32, ctypes.POINTER(anova_params)],
        "anova_predict_plan": [ctypes.POINTER(VP), VP, i64, VP, i64, i32, i64, i64,
                               ctypes.POINTER(anova_window), i32, ctypes.POINTER(anova_params), VP],
        "anova_predict_plan_host": [ctypes.POINTER(VP), VP, i64, VP, i64, i32, i64, i64,
                                    ctypes.POINTER(anova_window), i32,
                                    ctypes.POINTER(anova_params)],
        "anova_predict": [VP, VP, VP, i32, i64, i64, VP],
        "krr_cg_solve_shifts": [VP, VP, VP, i32, ctypes.POINTER(dbl), i64, dbl, i32,
                                ctypes.POINTER(krr_cg_info), VP],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.anova_last_error.argtypes = []
    lib.anova_last_error.restype = ctypes.c_char_p
    lib.anova_matvec_noalloc_max_bytes.argtypes = []
    lib.anova_matvec_noalloc_max_bytes.restype = ctypes.c_int64
    _lib = lib
    return lib


def anova_last_error() -> str:
    return load().anova_last_error().decode()


def _check(st: int, allow=(ANOVA_OK,)) -> int:
    if st not in allow:
        raise AnovaError(st, anova_last_error())
    return st


def _stream(stream) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _dev_f64(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a CUDA float64 tensor")
    return t


def _colmajor(t, name, N):
    """(N,) or (N, nrhs) tensor stored column-major: returns (ptr, nrhs, ld)."""
    _dev_f64(t, name)
    if t.dim() == 1:
        if t.stride(0) != 1 or t.shape[0] != N:
            raise ValueError(f"{name} must be a contiguous vector of N entries")
        return t.data_ptr(), 1, N
    if t.dim() != 2 or t.shape[0] != N or t.stride(0) != 1:
        raise ValueError(f"{name} must be (N, nrhs) column-major (stride(0) == 1)")
    return t.data_ptr(), t.shape[1], max(t.stride(1), N)


def make_windows(windows) -> "ctypes.Array":
    P = len(windows)
    arr = (anova_window * P)()
    for l, w in enumerate(windows):
        feat = tuple(w.feat) if hasattr(w, "feat") else tuple(w[0])
        eta = w.eta if hasattr(w, "eta") else w[1]
        arr[l].d_A = len(feat)
        for t, f in enumerate(feat):
            arr[l].feat[t] = int(f)
        arr[l].eta = float(eta)
    return arr


def make_params(ell: float, precision: int = ANOVA_FP32_NFFT, M: int = 0, m: int = 0, n: int = 0,
                h: float = 0.0, target_err: float = 0.0, center: int = 0,
                residual: int = 0, tune: int = 0, reg_q: int = 0) -> anova_params:
    p = anova_params()
    p.ell, p.precision, p.M, p.m, p.n = float(ell), int(precision), int(M), int(m), int(n)
    p.h, p.target_err, p.center, p.residual = float(h), float(target_err), int(center), int(residual)
    p.tune, p.reg_q = int(tune), int(reg_q)
    return p


@dataclass
class WindowInfo:
    d_A: int
    M: int
    n: int
    m: int
    h: float
    center: tuple
    extent: float
    err_images: float
    err_trunc: float
    err_window: float
    err_round: float
    err_total: float
    n_tiles: int
    n_subproblems: int
    per_cell: int
    tile: int


STAGE_KINDS = ("permute", "spread", "tile_sum", "fold", "convolve", "gather", "combine")


class Plan:
    """Owning wrapper over an anova_plan_t."""

    def __init__(self, handle: int, N: int, P: int, precision: int, Nz: int = 0):
        self.handle = handle
        self.N, self.P, self.precision = N, P, precision
        self.Nz = Nz  # prediction plans: number of targets

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def destroy(self):
        if self.handle:
            _check(load().anova_plan_destroy(self.handle))
            self.handle = None

    def info(self, l: int) -> WindowInfo:
        r = anova_window_info()
        _check(load().anova_plan_query(self.handle, l, ctypes.byref(r)))
        return WindowInfo(r.d_A, r.M, r.n, r.m, r.h, tuple(r.center), r.extent, r.err_images,
                          r.err_trunc, r.err_window, r.err_round, r.err_total, r.n_tiles,
                          r.n_subproblems, r.per_cell, r.tile)

    def set_timing(self, enable: bool) -> None:
        _check(load().anova_plan_set_timing(self.handle, 1 if enable else 0))

    def stage_times(self):
        """{kind: (total_ms, launches)} per stage kind, in execution order; resets."""
        ms = (ctypes.c_double * len(STAGE_KINDS))()
        cnt = (ctypes.c_int64 * len(STAGE_KINDS))()
        _check(load().anova_plan_stage_times(self.handle, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(STAGE_KINDS)}

    def footprint(self, nrhs: int = 1):
        """(plan_bytes, solve_bytes): device bytes the plan holds and that a
        CG solve with nrhs columns allocates."""
        pb, sb = ctypes.c_int64(), ctypes.c_int64()
        _check(load().anova_plan_footprint(self.handle, nrhs, ctypes.byref(pb), ctypes.byref(sb)))
        return pb.value, sb.value

    def err_estimate(self) -> float:
        return sum(self.info(l).err_total for l in range(self.P))


def anova_fastsum_plan(X, windows, params: anova_params, stream=None) -> Plan:
    """Plan for device points X ((N, d) row-major CUDA float64)."""
    _dev_f64(X, "X")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be (N, d) row-major")
    N, d = X.shape
    wins = make_windows(windows)
    h = VP()
    st = load().anova_fastsum_plan(ctypes.byref(h), X.data_ptr(), N, d, X.stride(0), wins,
                                   len(windows), ctypes.byref(params), _stream(stream))
    _check(st)
    return Plan(h.value, N, len(windows), params.precision)


def anova_fastsum_plan_host(X, windows, params: anova_params) -> Plan:
    """Plan for host points X ((N, d) float64 numpy array); no device copy of
    X is made, and it may run on any host thread."""
    import numpy as np
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim != 2:
        raise ValueError("X must be (N, d)")
    N, d = X.shape
    wins = make_windows(windows)
    h = VP()
    st = load().anova_fastsum_plan_host(ctypes.byref(h), X.ctypes.data, N, d, d, wins,
                                        len(windows), ctypes.byref(params))
    _check(st)
    return Plan(h.value, N, len(windows), params.precision)


def anova_predict_plan(X, Z, windows, params: anova_params, stream=None) -> Plan:
    """Prediction plan for device training points X ((N, d)) and targets Z
    ((Nz, d)), both row-major CUDA float64."""
    for t, name in ((X, "X"), (Z, "Z")):
        _dev_f64(t, name)
        if t.dim() != 2 or t.stride(1) != 1:
            raise ValueError(f"{name} must be (rows, d) row-major")
    N, d = X.shape
    Nz, dz = Z.shape
    if dz != d:
        raise ValueError("X and Z must have the same number of features")
    wins = make_windows(windows)
    h = VP()
    st = load().anova_predict_plan(ctypes.byref(h), X.data_ptr(), N, Z.data_ptr(), Nz, d,
                                   X.stride(0), Z.stride(0), wins, len(windows),
                                   ctypes.byref(params), _stream(stream))
    _check(st)
    return Plan(h.value, N, len(windows), params.precision, Nz)


def anova_predict_plan_host(X, Z, windows, params: anova_params) -> Plan:
    """Prediction plan for host arrays X ((N, d)) and Z ((Nz, d))."""
    import numpy as np
    X = np.ascontiguousarray(X, dtype=np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    if X.ndim != 2 or Z.ndim != 2 or X.shape[1] != Z.shape[1]:
        raise ValueError("X and Z must be (rows, d) with the same d")
    N, d = X.shape
    Nz = Z.shape[0]
    wins = make_windows(windows)
    h = VP()
    st = load().anova_predict_plan_host(ctypes.byref(h), X.ctypes.data, N, Z.ctypes.data, Nz, d,
                                        d, d, wins, len(windows), ctypes.byref(params))
    _check(st)
    return Plan(h.value, N, len(windows), params.precision, Nz)


def anova_predict(plan: Plan, alpha, out, stream=None) -> None:
    """out = K~(Z, X) alpha at the plan's targets (asynchronous on the stream).
    alpha: (N,) or (N, nrhs); out: (Nz,) or (Nz, nrhs), column-major."""
    pa, nrhs, lda = _colmajor(alpha, "alpha", plan.N)
    po, nrhs2, ldo = _colmajor(out, "out", plan.Nz)
    if nrhs != nrhs2:
        raise ValueError("alpha and out must have the same number of columns")
    _check(load().anova_predict(plan.handle, pa, po, nrhs, lda, ldo, _stream(stream)))


def anova_matvec(plan: Plan, alpha, out, beta: float, stream=None) -> None:
    """out = (K~ + beta I) alpha (asynchronous on the stream)."""
    pa, nrhs, lda = _colmajor(alpha, "alpha", plan.N)
    po, nrhs2, ldo = _colmajor(out, "out", plan.N)
    if nrhs != nrhs2 or lda != ldo:
        raise ValueError("alpha and out must have the same shape and leading dimension")
    _check(load().anova_matvec(plan.handle, pa, po, nrhs, lda, float(beta), _stream(stream)))


def anova_matvec_noalloc(plan: Plan, alpha, out, beta: float, stream=None) -> None:
    """anova_matvec with its work space in the library's static device array
    (no device allocation; synchronises the stream first)."""
    pa, nrhs, lda = _colmajor(alpha, "alpha", plan.N)
    po, nrhs2, ldo = _colmajor(out, "out", plan.N)
    if nrhs != nrhs2 or lda != ldo:
        raise ValueError("alpha and out must have the same shape and leading dimension")
    _check(load().anova_matvec_noalloc(plan.handle, pa, po, nrhs, lda, float(beta),
                                       _stream(stream)))


def anova_matvec_noalloc_max_bytes() -> int:
    """Size of the static work space of anova_matvec_noalloc."""
    return int(load().anova_matvec_noalloc_max_bytes())


def krr_cg_solve(plan: Plan, y, alpha, beta: float, tol: float, maxit: int, stream=None,
                 allow_not_converged: bool = False):
    """Solve (K~ + beta I) alpha = y; returns a list of krr_cg_info per column."""
    py, nrhs, ldy = _colmajor(y, "y", plan.N)
    pa, nrhs2, lda = _colmajor(alpha, "alpha", plan.N)
    if nrhs != nrhs2 or ldy != lda:
        raise ValueError("y and alpha must have the same shape and leading dimension")
    info = (krr_cg_info * nrhs)()
    st = load().krr_cg_solve(plan.handle, py, pa, nrhs, lda, float(beta), float(tol), int(maxit),
                             info, _stream(stream))
    allow = (ANOVA_OK, ANOVA_E_NOT_CONVERGED) if allow_not_converged else (ANOVA_OK,)
    _check(st, allow)
    return [dict(iters=i.iters, converged=bool(i.converged), relres=i.relres,
                 true_relres=i.true_relres, status=STATUS_NAMES[st]) for i in info]


def krr_cg_solve_shifts(plan: Plan, y, alpha, shifts, tol: float, maxit: int, stream=None,
                        allow_not_converged: bool = False):
    """Solve (K~ + shifts[s] I) alpha[:, s] = y for every shift at once;
    y: (N,), alpha: (N, len(shifts)) column-major.  Returns a list of info
    dicts, one per shift."""
    py, ny, _ = _colmajor(y, "y", plan.N)
    if ny != 1:
        raise ValueError("y must be one column")
    S = len(shifts)
    pa, na, lda = _colmajor(alpha, "alpha", plan.N)
    if na != S:
        raise ValueError("alpha must have one column per shift")
    sh = (ctypes.c_double * S)(*[float(v) for v in shifts])
    info = (krr_cg_info * S)()
    st = load().krr_cg_solve_shifts(plan.handle, py, pa, S, sh, lda, float(tol), int(maxit), info,
                                    _stream(stream))
    allow = (ANOVA_OK, ANOVA_E_NOT_CONVERGED) if allow_not_converged else (ANOVA_OK,)
    _check(st, allow)
    return [dict(iters=i.iters, converged=bool(i.converged), relres=i.relres,
                 true_relres=i.true_relres, status=STATUS_NAMES[st]) for i in info]


def anova_plan_destroy(plan: Plan) -> None:
    plan.destroy()


def grid_tensor(plan: Plan, l: int):
    """A zeroed device tensor with the grid shape of window l (x fastest)."""
    import torch
    inf = plan.info(l)
    dt = torch.float64 if plan.precision == ANOVA_FP64 else torch.float32
    return torch.zeros((inf.n,) * inf.d_A, dtype=dt, device="cuda")


def anova_stage_spread(plan: Plan, l: int, alpha, grid, stream=None) -> None:
    pa, _, _ = _colmajor(alpha, "alpha", plan.N)
    _check(load().anova_stage_spread(plan.handle, l, pa, grid.data_ptr(), _stream(stream)))


def anova_stage_convolve(plan: Plan, l: int, grid, stream=None) -> None:
    _check(load().anova_stage_convolve(plan.handle, l, grid.data_ptr(), _stream(stream)))


def anova_stage_gather(plan: Plan, l: int, grid, out, stream=None) -> None:
    po, _, _ = _colmajor(out, "out", plan.N)
    _check(load().anova_stage_gather(plan.handle, l, grid.data_ptr(), po, _stream(stream)))


def _info_dicts(info, st):
    return [dict(iters=i.iters, converged=bool(i.converged), relres=i.relres,
                 true_relres=i.true_relres, status=STATUS_NAMES[st]) for i in info]


class Solve:
    """One problem's CG state (krr_cg_start ... krr_cg_destroy).  y and alpha
    must stay alive until destroy(); several solves advance together with
    krr_cg_iterate."""

    def __init__(self, plan: Plan, y, alpha, beta: float, tol: float, maxit: int, stream=None):
        py, nrhs, ldy = _colmajor(y, "y", plan.N)
        pa, nrhs2, lda = _colmajor(alpha, "alpha", plan.N)
        if nrhs != nrhs2 or ldy != lda:
            raise ValueError("y and alpha must have the same shape and leading dimension")
        h = VP()
        _check(load().krr_cg_start(ctypes.byref(h), plan.handle, py, pa, nrhs, lda, float(beta),
                                   float(tol), int(maxit), _stream(stream)))
        self.handle = h.value
        self.plan, self.y, self.alpha, self.nrhs = plan, y, alpha, nrhs

    def poll(self, stream=None):
        """(number of iterating columns, per-column info)"""
        a = ctypes.c_int32()
        info = (krr_cg_info * self.nrhs)()
        _check(load().krr_cg_poll(self.handle, ctypes.byref(a), info, _stream(stream)))
        return a.value, _info_dicts(info, ANOVA_OK)

    def finish(self, stream=None, allow_not_converged: bool = True):
        info = (krr_cg_info * self.nrhs)()
        st = load().krr_cg_finish(self.handle, info, _stream(stream))
        allow = (ANOVA_OK, ANOVA_E_NOT_CONVERGED) if allow_not_converged else (ANOVA_OK,)
        _check(st, allow)
        return _info_dicts(info, st)

    def destroy(self):
        if self.handle:
            _check(load().krr_cg_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def krr_cg_iterate(solves: Sequence["Solve"], iters: int, stream=None) -> None:
    arr = (VP * len(solves))(*[s.handle for s in solves])
    _check(load().krr_cg_iterate(arr, len(solves), int(iters), _stream(stream)))


def krr_cg_active(solves: Sequence["Solve"], dev_counts, host_counts, stream=None) -> None:
    """Enqueue the still-iterating column count of each solve into
    dev_counts (CUDA int32) and copy it to host_counts (pinned CPU int32);
    read host_counts after synchronising on an event recorded afterwards."""
    import torch
    if dev_counts.dtype != torch.int32 or host_counts.dtype != torch.int32:
        raise TypeError("count arrays must be int32")
    n = len(solves)
    if dev_counts.numel() < n or host_counts.numel() < n or not dev_counts.is_cuda:
        raise ValueError("count arrays too small or not on the device/host")
    arr = (VP * n)(*[s.handle for s in solves])
    _check(load().krr_cg_active(arr, n, dev_counts.data_ptr(), host_counts.data_ptr(),
                                _stream(stream)))


def krr_cg_solve_batched(plans, ys, alphas, betas, tol: float, maxit: int, stream=None,
                         allow_not_converged: bool = False):
    """Solve several problems together; returns one info list per problem."""
    n = len(plans)
    P = (VP * n)(*[p.handle for p in plans])
    Y = (VP * n)()
    A = (VP * n)()
    R = (ctypes.c_int32 * n)()
    L = (ctypes.c_int64 * n)()
    B = (ctypes.c_double * n)(*[float(b) for b in betas])
    for i, (p, y, a) in enumerate(zip(plans, ys, alphas)):
        py, nrhs, ldy = _colmajor(y, "y", p.N)
        pa, nrhs2, lda = _colmajor(a, "alpha", p.N)
        if nrhs != nrhs2 or ldy != lda:
            raise ValueError("y and alpha must have the same shape and leading dimension")
        Y[i], A[i], R[i], L[i] = py, pa, nrhs, lda
    info = (krr_cg_info * sum(R))()
    st = load().krr_cg_solve_batched(n, P, Y, A, R, L, B, float(tol), int(maxit), info,
                                     _stream(stream))
    allow = (ANOVA_OK, ANOVA_E_NOT_CONVERGED) if allow_not_converged else (ANOVA_OK,)
    _check(st, allow)
    out, k = [], 0
    for i in range(n):
        out.append(_info_dicts(info[k:k + R[i]], st))
        k += R[i]
    return out
