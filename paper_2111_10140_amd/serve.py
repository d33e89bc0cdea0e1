"""Request loop for kernel ridge regression solves with continuous batching.

A request is one KRR problem of the paper's form (Sec. 2 and Sec. 5): points
X (N x d), feature windows with weights, kernel width ell, shift beta and
1..nrhs right-hand sides y; the answer is alpha = (K~ + beta I)^-1 y, found
by CG around the fast ANOVA product.

The loop keeps every admitted request's plan (sorted nodes, permutations,
multipliers) and CG state on the device and advances all of them together:
each scheduling round runs a few CG iterations of the whole live list in
one batched product per iteration (krr_cg_iterate), then retires the
requests whose columns have all stopped and admits waiting ones.  Requests
that arrive while others iterate join the list as memory frees up, so their
work overlaps on the device.  Because every column iterates independently
and each product is deterministic, a request's alpha is bitwise the same
alone and in any mix.

Admission is by device-memory footprint, first come first served: a request
is planned when a pre-plan estimate fits the free budget; once planned its
exact footprint (plan, CG vectors, product work space, y and alpha) is
reserved, or, if that exact figure does not fit yet, the plan is dropped and
the request waits at the head of the queue until it does.  A request whose
exact footprint exceeds the whole budget is rejected.

The device work is done by an executor; ``HipExecutor`` drives the C ABI.
Tests of the scheduling logic use an executor of their own on the CPU.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Deque, Dict, List, Optional, Sequence

import numpy as np

DONE_STATES = ("OK", "E_NOT_CONVERGED", "E_BREAKDOWN", "ERROR", "REJECTED", "CANCELLED")


@dataclass
class Request:
    """One KRR solve: X (N, d) float64, windows [(features, eta)], y (N,) or (N, nrhs)."""
    X: np.ndarray
    windows: Sequence[Any]
    ell: float
    beta: float
    y: np.ndarray
    tol: float
    maxit: int
    arrival: float
    handle: int = -1
    # filled by the server
    est_bytes: int = 0
    exact_bytes: Optional[int] = None
    admitted: float = math.nan
    state: Any = None

    @property
    def N(self) -> int:
        return int(self.X.shape[0])

    @property
    def nrhs(self) -> int:
        return 1 if self.y.ndim == 1 else int(self.y.shape[1])


@dataclass
class Result:
    handle: int
    status: str                      # one of DONE_STATES
    alpha: Optional[np.ndarray]      # (N,) or (N, nrhs) float64, None unless solved
    info: List[Dict[str, Any]]       # per column: iters, converged, relres, true_relres
    arrival: float
    admitted: float
    finished: float
    error: str = ""

    @property
    def latency(self) -> float:
        """Seconds from arrival to result (queueing, planning, iterations)."""
        return self.finished - self.arrival


def _feat(w) -> tuple:
    return tuple(w.feat) if hasattr(w, "feat") else tuple(w[0])


def validate(req: Request) -> None:
    """Checks made at submission; raises ValueError."""
    X, y = req.X, req.y
    if X.ndim != 2 or X.shape[0] < 1 or X.shape[1] < 1:
        raise ValueError("X must be (N, d) with N, d >= 1")
    if y.ndim not in (1, 2) or y.shape[0] != X.shape[0] or (y.ndim == 2 and y.shape[1] < 1):
        raise ValueError("y must be (N,) or (N, nrhs)")
    if not (np.isfinite(X).all() and np.isfinite(y).all()):
        raise ValueError("X and y must be finite")
    if not (math.isfinite(req.ell) and req.ell > 0):
        raise ValueError("ell must be finite and > 0")
    if not (math.isfinite(req.beta) and req.beta > 0):
        raise ValueError("beta must be finite and > 0")
    if not (math.isfinite(req.tol) and req.tol >= 0) or req.maxit < 1:
        raise ValueError("tol must be >= 0 and maxit >= 1")
    if not req.windows:
        raise ValueError("at least one feature window")
    seen = set()
    for w in req.windows:
        f = _feat(w)
        if not 1 <= len(f) <= 3:
            raise ValueError("feature windows hold 1 to 3 features")
        for t in f:
            if not 0 <= t < X.shape[1] or t in seen:
                raise ValueError("feature index out of range or repeated")
            seen.add(t)


def estimate_bytes(N: int, P: int, nrhs: int, precision_bytes: int = 4) -> int:
    """Pre-plan estimate of a request's device bytes, used only to decide
    whether planning may start (the exact figure is known after planning):
    per window the sorted node records (4 * (1 + 3) or 8 * 4 bytes), the two
    permutations, and per (window, column) the sorted values and about as
    much again for grids and spread regions; per column three float64 CG
    vectors plus y and alpha."""
    node = 16 if precision_bytes == 4 else 32
    per_point = P * (node + 8) + P * nrhs * 2 * precision_bytes + nrhs * 5 * 8
    return int(N) * per_point + (1 << 20) * P * nrhs


class Server:
    """Continuous-batching KRR solver.

    submit() enqueues a request and returns a handle; step() runs one
    scheduling round (iterate the live list, admit, retire); result(handle)
    returns the Result once the request is done.  ``budget`` is the device
    memory (bytes) the live requests may hold together; ``max_live`` caps the
    number of requests iterating at once; ``iters_per_round`` CG iterations
    are run between polls of the live requests.
    """

    def __init__(self, executor, budget: int, max_live: int = 64, iters_per_round: int = 4,
                 clock: Callable[[], float] = time.perf_counter):
        if budget <= 0 or max_live < 1 or iters_per_round < 1:
            raise ValueError("budget, max_live and iters_per_round must be positive")
        self.ex = executor
        self.budget = int(budget)
        self.max_live = int(max_live)
        self.iters_per_round = int(iters_per_round)
        self.clock = clock
        self.queue: Deque[Request] = collections.deque()
        self.live: List[Request] = []
        self.results: Dict[int, Result] = {}
        self.reserved = 0
        self.peak_reserved = 0
        self.peak_live = 0
        self.rounds = 0
        self._next = 0

    # ------------------------------------------------------------ client side
    def submit(self, X, windows, ell: float, beta: float, y, tol: float = 1e-6,
               maxit: int = 2000, arrival: Optional[float] = None) -> int:
        """Enqueue a solve; invalid input is rejected at once (ValueError)."""
        req = Request(np.ascontiguousarray(X, dtype=np.float64), list(windows), float(ell),
                      float(beta), np.asarray(y, dtype=np.float64), float(tol), int(maxit),
                      self.clock() if arrival is None else float(arrival))
        validate(req)
        req.handle = self._next
        self._next += 1
        req.est_bytes = self.ex.estimate(req)
        self.queue.append(req)
        return req.handle

    def result(self, handle: int) -> Optional[Result]:
        return self.results.get(handle)

    def cancel(self, handle: int) -> bool:
        """Drop a queued or live request (its result says CANCELLED)."""
        for q in list(self.queue):
            if q.handle == handle:
                self.queue.remove(q)
                self._done(q, "CANCELLED", None, [], "")
                return True
        for r in self.live:
            if r.handle == handle:
                self.live.remove(r)
                self._release(r)
                self._done(r, "CANCELLED", None, [], "")
                return True
        return False

    def busy(self) -> bool:
        return bool(self.queue or self.live)

    # ------------------------------------------------------------ scheduling
    def _done(self, req: Request, status: str, alpha, info, err: str) -> None:
        self.results[req.handle] = Result(req.handle, status, alpha, info, req.arrival,
                                          req.admitted, self.clock(), err)

    def _release(self, req: Request) -> None:
        if req.state is not None:
            self.ex.release(req.state)
            req.state = None
        if req.exact_bytes is not None and not math.isnan(req.admitted):
            self.reserved -= req.exact_bytes

    def _admit(self) -> None:
        while self.queue and len(self.live) < self.max_live:
            req = self.queue[0]
            free = self.budget - self.reserved
            need = req.exact_bytes if req.exact_bytes is not None else req.est_bytes
            if need > free and self.live:
                return  # wait for memory; first come, first served
            try:
                state, exact = self.ex.plan(req)
            except Exception as e:  # invalid problem for the library, accuracy, memory
                self.queue.popleft()
                self._done(req, "ERROR", None, [], str(e))
                continue
            req.exact_bytes = int(exact)
            if req.exact_bytes > self.budget:
                self.ex.release(state)
                self.queue.popleft()
                self._done(req, "REJECTED", None, [],
                           f"needs {req.exact_bytes} bytes, budget {self.budget}")
                continue
            if req.exact_bytes > free:
                self.ex.release(state)  # plan again once memory frees up
                return
            try:
                self.ex.start(state)
            except Exception as e:
                self.ex.release(state)
                self.queue.popleft()
                self._done(req, "ERROR", None, [], str(e))
                continue
            self.queue.popleft()
            req.state = state
            req.admitted = self.clock()
            self.reserved += req.exact_bytes
            self.peak_reserved = max(self.peak_reserved, self.reserved)
            self.live.append(req)
            self.peak_live = max(self.peak_live, len(self.live))

    def step(self) -> None:
        """One round: launch iterations of the live list, admit waiting
        requests while the device works, then retire finished ones."""
        self.rounds += 1
        if self.live:
            self.ex.iterate([r.state for r in self.live], self.iters_per_round)
        self._admit()
        still = []
        for r in self.live:
            if self.ex.active(r.state) > 0:
                still.append(r)
                continue
            try:
                alpha, info, status = self.ex.finish(r.state)
                self._done(r, status, alpha, info, "")
            except Exception as e:
                self._done(r, "ERROR", None, [], str(e))
            self._release(r)
        self.live = still

    def run_until_idle(self, max_rounds: int = 1_000_000) -> None:
        for _ in range(max_rounds):
            if not self.busy():
                return
            self.step()
        raise RuntimeError("requests still pending after max_rounds")

    # ------------------------------------------------------------ reporting
    def stats(self, warmup_fraction: float = 0.1) -> Dict[str, Any]:
        """Latency percentiles over solved requests in arrival order after
        the first warmup_fraction of them, and solves per second."""
        done = sorted((r for r in self.results.values()
                       if r.status in ("OK", "E_NOT_CONVERGED")), key=lambda r: r.arrival)
        if not done:
            return dict(completed=0)
        skip = int(len(done) * warmup_fraction)
        kept = done[skip:] or done
        lat = np.array([r.latency for r in kept])
        span = max(r.finished for r in done) - min(r.arrival for r in done)
        return dict(completed=len(done), measured=len(kept),
                    p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    mean_s=float(lat.mean()), solves_per_s=len(done) / span if span > 0 else 0.0,
                    rejected=sum(r.status == "REJECTED" for r in self.results.values()),
                    errors=sum(r.status == "ERROR" for r in self.results.values()),
                    peak_live=self.peak_live, peak_reserved_bytes=self.peak_reserved,
                    rounds=self.rounds)


class HipExecutor:
    """Device work of the server through the C ABI: plan, CG state, batched
    iterations.  All work runs on one stream; planning uploads the points on
    a second stream so that it overlaps the iterations already launched."""

    def __init__(self, precision: Optional[int] = None, target_err: float = 1e-4,
                 params: Optional[Dict[str, Any]] = None):
        import torch

        from . import _lib
        self.torch, self.A = torch, _lib
        _lib.load()
        self.precision = _lib.ANOVA_FP32_NFFT if precision is None else precision
        self.target_err = target_err
        self.params = dict(params or {})
        self.stream = torch.cuda.Stream()
        self.plan_stream = torch.cuda.Stream()

    def estimate(self, req: Request) -> int:
        return estimate_bytes(req.N, len(req.windows), req.nrhs,
                              4 if self.precision == self.A.ANOVA_FP32_NFFT else 8)

    def estimate_problem(self, p) -> int:
        """estimate() for an object with X, windows and y."""
        y = np.asarray(p.y)
        return estimate_bytes(p.X.shape[0], len(p.windows), 1 if y.ndim == 1 else y.shape[1],
                              4 if self.precision == self.A.ANOVA_FP32_NFFT else 8)

    def plan(self, req: Request):
        torch, A = self.torch, self.A
        with torch.cuda.stream(self.plan_stream):
            Xd = torch.from_numpy(req.X).to("cuda", non_blocking=False)
            prm = A.make_params(req.ell, self.precision, target_err=self.target_err,
                                **self.params)
            plan = A.anova_fastsum_plan(Xd, req.windows, prm, stream=self.plan_stream)
            del Xd
        pb, sb = plan.footprint(req.nrhs)
        io = 2 * req.N * req.nrhs * 8  # y and alpha
        return {"plan": plan, "req": req, "solve": None}, pb + sb + io

    def start(self, st) -> None:
        torch, A = self.torch, self.A
        req = st["req"]
        with torch.cuda.stream(self.stream):
            y = torch.from_numpy(np.asfortranarray(req.y)).to("cuda")
            if y.dim() == 2:
                y = y.t().contiguous().t()  # column-major
            alpha = torch.zeros_like(y)
        st["solve"] = A.Solve(st["plan"], y, alpha, req.beta, req.tol, req.maxit,
                              stream=self.stream)

    def iterate(self, states, iters: int) -> None:
        self.A.krr_cg_iterate([s["solve"] for s in states], iters, stream=self.stream)

    def active(self, st) -> int:
        return st["solve"].poll(stream=self.stream)[0]

    def finish(self, st):
        sv = st["solve"]
        try:
            info = sv.finish(stream=self.stream, allow_not_converged=True)
            status = info[0]["status"]
        except self.A.AnovaError as e:
            if e.status != self.A.ANOVA_E_BREAKDOWN:
                raise
            info = sv.poll(stream=self.stream)[1]
            status = "E_BREAKDOWN"
        self.stream.synchronize()
        alpha = sv.alpha.cpu().numpy()
        return alpha, info, status

    def release(self, st) -> None:
        if st.get("solve") is not None:
            st["solve"].destroy()
            st["solve"] = None
        if st.get("plan") is not None:
            st["plan"].destroy()
            st["plan"] = None
