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
import threading
import time
from dataclasses import dataclass
from typing import Any, Callable, Deque, Dict, List, Optional, Sequence

import numpy as np

DONE_STATES = ("OK", "E_NOT_CONVERGED", "E_BREAKDOWN", "ERROR", "REJECTED", "CANCELLED")


@dataclass(eq=False)  # compared by identity
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
    hold: int = 0                    # bytes reserved for it now
    admitted: float = math.nan
    state: Any = None
    future: Any = None

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
    number of requests planning or iterating at once; ``iters_per_round`` CG
    iterations are run between polls of the live requests.  With
    ``planners`` > 0, plans are built by that many host threads while the
    device iterates (the library releases the interpreter lock during a
    call); with 0 they are built in step().
    """

    def __init__(self, executor, budget: int, max_live: int = 64, iters_per_round: int = 4,
                 planners: int = 0, clock: Callable[[], float] = time.perf_counter):
        if budget <= 0 or max_live < 1 or iters_per_round < 1 or planners < 0:
            raise ValueError("budget, max_live and iters_per_round must be positive")
        self.ex = executor
        self.budget = int(budget)
        self.max_live = int(max_live)
        self.iters_per_round = int(iters_per_round)
        self.clock = clock
        self.queue: Deque[Request] = collections.deque()
        self.planning: List[Request] = []
        self.live: List[Request] = []
        self.results: Dict[int, Result] = {}
        self.reserved = 0
        self.peak_reserved = 0
        self.peak_live = 0
        self.rounds = 0
        self._next = 0
        self._inflight = None  # (requests, poll handle) of the last launched round
        self._pool = None
        if planners > 0:
            import concurrent.futures
            self._pool = concurrent.futures.ThreadPoolExecutor(max_workers=planners)

    def close(self) -> None:
        """Cancel everything still pending and stop the planner threads."""
        for q in list(self.queue) + list(self.planning) + list(self.live):
            self.cancel(q.handle)
        if self._pool is not None:
            self._pool.shutdown(wait=True)
            self._pool = None

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
        """Drop a queued, planning or live request (its result says CANCELLED)."""
        for q in list(self.queue):
            if q.handle == handle:
                self.queue.remove(q)
                self._done(q, "CANCELLED", None, [], "")
                return True
        for r in list(self.planning):
            if r.handle == handle:
                self.planning.remove(r)
                try:
                    state, _ = r.future.result()
                    self.ex.release(state)
                except Exception:
                    pass
                self._unhold(r)
                self._done(r, "CANCELLED", None, [], "")
                return True
        for r in self.live:
            if r.handle == handle:
                self.live.remove(r)
                self._release(r)
                self._done(r, "CANCELLED", None, [], "")
                return True
        return False

    def busy(self) -> bool:
        return bool(self.queue or self.planning or self.live)

    # ------------------------------------------------------------ scheduling
    def _done(self, req: Request, status: str, alpha, info, err: str) -> None:
        self.results[req.handle] = Result(req.handle, status, alpha, info, req.arrival,
                                          req.admitted, self.clock(), err)

    def _hold(self, req: Request, nbytes: int) -> None:
        self.reserved += nbytes - req.hold
        req.hold = nbytes
        self.peak_reserved = max(self.peak_reserved, self.reserved)

    def _unhold(self, req: Request) -> None:
        self.reserved -= req.hold
        req.hold = 0

    def _release(self, req: Request) -> None:
        if req.state is not None:
            self.ex.release(req.state)
            req.state = None
        self._unhold(req)

    def _place(self, req: Request, state, exact: int) -> None:
        """A plan is built: reserve its exact footprint and start it, or put
        the request back at the head of the queue until memory frees up."""
        req.exact_bytes = int(exact)
        if req.exact_bytes > self.budget:
            self.ex.release(state)
            self._unhold(req)
            self._done(req, "REJECTED", None, [],
                       f"needs {req.exact_bytes} bytes, budget {self.budget}")
            return
        if req.exact_bytes - req.hold > self.budget - self.reserved:
            self.ex.release(state)  # plan again once memory frees up
            self._unhold(req)
            self.queue.appendleft(req)
            return
        self._hold(req, req.exact_bytes)
        try:
            self.ex.start(state)
        except Exception as e:
            self.ex.release(state)
            self._unhold(req)
            self._done(req, "ERROR", None, [], str(e))
            return
        req.state = state
        req.admitted = self.clock()
        self.live.append(req)
        self.peak_live = max(self.peak_live, len(self.live))

    def _admit(self) -> None:
        # plans finished by the planner threads, in submission order
        for req in sorted(self.planning, key=lambda r: r.handle):
            if not req.future.done():
                continue
            self.planning.remove(req)
            try:
                state, exact = req.future.result()
            except Exception as e:  # invalid for the library, accuracy, memory
                self._unhold(req)
                self._done(req, "ERROR", None, [], str(e))
                continue
            self._place(req, state, exact)
        # start plans for waiting requests while the estimate fits
        while self.queue and len(self.live) + len(self.planning) < self.max_live:
            req = self.queue[0]
            need = req.exact_bytes if req.exact_bytes is not None else req.est_bytes
            if need > self.budget - self.reserved and (self.live or self.planning):
                return  # wait for memory; first come, first served
            self.queue.popleft()
            self._hold(req, need)
            if self._pool is not None:
                req.future = self._pool.submit(self.ex.plan, req)
                self.planning.append(req)
                continue
            try:
                state, exact = self.ex.plan(req)
            except Exception as e:
                self._unhold(req)
                self._done(req, "ERROR", None, [], str(e))
                continue
            self._place(req, state, exact)

    def _retire(self, finished) -> None:
        for r in finished:
            try:
                alpha, info, status = self.ex.finish(r.state)
                self._done(r, status, alpha, info, "")
            except Exception as e:
                self._done(r, "ERROR", None, [], str(e))
            self._release(r)
        gone = set(id(r) for r in finished)
        self.live = [r for r in self.live if id(r) not in gone]

    def step(self) -> None:
        """One round: launch iterations of the live list, admit waiting
        requests while the device works, then retire finished ones.

        With an executor that polls asynchronously (active_async), the
        still-iterating counts are enqueued behind each round's iterations
        and read one round later, after the next round has been launched, so
        the device does not wait for the host between rounds; a request that
        has just finished may take part in one more round (its columns are
        frozen, the round changes nothing of it)."""
        self.rounds += 1
        asynchronous = hasattr(self.ex, "active_async")
        launched = None
        if self.live:
            states = [r.state for r in self.live]
            self.ex.iterate(states, self.iters_per_round)
            if asynchronous:
                launched = (list(self.live), self.ex.active_async(states))
        self._admit()
        if asynchronous:
            prev, self._inflight = self._inflight, launched
            if prev is None:
                return
            reqs, handle = prev
            counts = self.ex.active_wait(handle)
            live_ids = set(id(r) for r in self.live)
            finished = [r for r, a in zip(reqs, counts)
                        if id(r) in live_ids and r.state is not None and a == 0]
        else:
            finished = [r for r in self.live if r.state is not None and self.ex.active(r.state) == 0]
        self._retire(finished)
        if not self.live and self.planning:
            # nothing to iterate: wait for the oldest plan instead of spinning
            import concurrent.futures
            concurrent.futures.wait([r.future for r in self.planning],
                                    return_when=concurrent.futures.FIRST_COMPLETED)

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
    iterations.  Iterations run on one stream; plans are built on the device
    from an upload of the request's points, each planner thread on a stream
    of its own (overlapping the iterations already launched)."""

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
        self._planner = threading.local()  # per planner thread: its stream

    def estimate(self, req: Request) -> int:
        return estimate_bytes(req.N, len(req.windows), req.nrhs,
                              4 if self.precision == self.A.ANOVA_FP32_NFFT else 8)

    def estimate_problem(self, p) -> int:
        """estimate() for an object with X, windows and y."""
        y = np.asarray(p.y)
        return estimate_bytes(p.X.shape[0], len(p.windows), 1 if y.ndim == 1 else y.shape[1],
                              4 if self.precision == self.A.ANOVA_FP32_NFFT else 8)

    def plan(self, req: Request):
        """Build the plan (any thread): the points go to the device and are
        binned and sorted there; returns (state, exact device bytes)."""
        torch, A = self.torch, self.A
        prm = A.make_params(req.ell, self.precision, target_err=self.target_err, **self.params)
        s = getattr(self._planner, "stream", None)
        if s is None:
            s = self._planner.stream = torch.cuda.Stream()
        with torch.cuda.stream(s):
            X = torch.from_numpy(np.ascontiguousarray(req.X, dtype=np.float64)).to("cuda")
        plan = A.anova_fastsum_plan(X, req.windows, prm, stream=s)  # synchronises s
        del X
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

    def active_async(self, states):
        """Enqueue the still-iterating column counts of the listed solves
        behind the launched iterations (two alternating buffer pairs, so a
        round's counts are not overwritten before they are read)."""
        torch = self.torch
        n = len(states)
        self._ring = getattr(self, "_ring", [None, None])
        self._slot = 1 - getattr(self, "_slot", 1)
        buf = self._ring[self._slot]
        if buf is None or buf[0].numel() < n:
            cap = max(64, 2 * n)
            buf = (torch.empty(cap, dtype=torch.int32, device="cuda"),
                   torch.empty(cap, dtype=torch.int32, pin_memory=True),
                   torch.cuda.Event())
            self._ring[self._slot] = buf
        dev, host, ev = buf
        self.A.krr_cg_active([s["solve"] for s in states], dev, host, stream=self.stream)
        ev.record(self.stream)
        return (host, ev, n)

    def active_wait(self, handle):
        host, ev, n = handle
        ev.synchronize()
        return host[:n].tolist()

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
