"""Scheduling logic of the serving loop, on the CPU with a stand-in executor.

The executor below does no arithmetic: each request needs a fixed number of
iterations (from its seed) and holds a fixed number of bytes.  The tests check
admission by footprint (the reserved bytes never exceed the budget, first
come first served), rejection, cancellation, errors, non-convergence and the
latency statistics.
"""
import math

import numpy as np
import pytest

from paper_2111_10140_amd.serve import Server, estimate_bytes, validate, Request


class FakeExecutor:
    def __init__(self, bytes_per_point=100, exact_factor=1.0, fail_plan=()):
        self.bpp = bytes_per_point
        self.exact_factor = exact_factor
        self.fail_plan = set(fail_plan)
        self.plans = 0
        self.released = []
        self.iterated = []  # lists of handles per iterate call
        self.live_states = set()

    def estimate(self, req):
        return req.N * self.bpp

    def plan(self, req):
        self.plans += 1
        if req.handle in self.fail_plan:
            raise RuntimeError("E_INVALID: planted failure")
        st = {"h": req.handle, "it": 0, "need": int(req.y.ravel()[0]), "maxit": req.maxit,
              "req": req}
        self.live_states.add(req.handle)
        return st, int(req.N * self.bpp * self.exact_factor)

    def start(self, st):
        pass

    def iterate(self, states, iters):
        self.iterated.append([s["h"] for s in states])
        for s in states:
            s["it"] = min(s["it"] + iters, s["need"], s["maxit"])

    def active(self, st):
        return 0 if st["it"] >= min(st["need"], st["maxit"]) else 1

    def finish(self, st):
        conv = st["need"] <= st["maxit"]
        info = [dict(iters=st["it"], converged=conv)]
        return st["req"].y.copy(), info, "OK" if conv else "E_NOT_CONVERGED"

    def release(self, st):
        assert st["h"] in self.live_states, "released twice"
        self.live_states.remove(st["h"])
        self.released.append(st["h"])


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3
        return self.t


def submit(srv, N, need, maxit=100, arrival=None, X=None):
    X = np.zeros((N, 3)) if X is None else X
    y = np.full(N, float(need))
    return srv.submit(X, [((0, 1, 2), 1.0)], 0.2, 1.0, y, 1e-6, maxit, arrival=arrival)


def test_admission_respects_budget_and_order():
    ex = FakeExecutor()
    srv = Server(ex, budget=10_000, max_live=8, iters_per_round=2, clock=Clock())
    sizes = [30, 50, 20, 40, 10, 60, 25, 35]
    hs = [submit(srv, N, need=3 + k) for k, N in enumerate(sizes)]
    while srv.busy():
        srv.step()
        assert srv.reserved <= srv.budget
        assert sum(ex.bpp * r.N for r in srv.live) == srv.reserved
    assert srv.reserved == 0 and not ex.live_states
    assert sorted(ex.released) == sorted(hs)
    res = [srv.result(h) for h in hs]
    assert all(r.status == "OK" for r in res)
    # first come first served: admission times follow submission order
    adm = [r.admitted for r in res]
    assert adm == sorted(adm)
    # the budget held at most 100 points at once
    assert srv.peak_reserved <= 10_000 and srv.peak_live < len(sizes)
    # iterations were batched across requests
    assert max(len(it) for it in ex.iterated) >= 2


def test_oversized_request_rejected_others_served():
    ex = FakeExecutor()
    srv = Server(ex, budget=5_000, clock=Clock())
    a = submit(srv, 20, 2)
    big = submit(srv, 100, 2)  # 10_000 bytes > budget
    c = submit(srv, 30, 2)
    srv.run_until_idle()
    assert srv.result(big).status == "REJECTED"
    assert srv.result(a).status == "OK" and srv.result(c).status == "OK"
    assert srv.reserved == 0 and not ex.live_states


def test_exact_footprint_above_estimate_replans_when_memory_frees():
    ex = FakeExecutor(exact_factor=1.5)  # estimate too low by a third
    srv = Server(ex, budget=10_000, clock=Clock())
    a = submit(srv, 40, 8)   # estimate 4000, exact 6000
    b = submit(srv, 30, 2)   # estimate 3000 fits beside a, exact 4500 does not
    while srv.busy():
        srv.step()
        assert srv.reserved <= srv.budget
    assert srv.result(a).status == "OK" and srv.result(b).status == "OK"
    assert srv.result(b).admitted > srv.result(a).admitted
    assert ex.plans >= 3  # b was planned, dropped, and planned again
    assert not ex.live_states


def test_not_converged_error_and_invalid():
    ex = FakeExecutor(fail_plan={1})
    srv = Server(ex, budget=100_000, clock=Clock())
    h0 = submit(srv, 10, need=50, maxit=1)
    h1 = submit(srv, 10, need=2)
    srv.run_until_idle()
    r0 = srv.result(h0)
    assert r0.status == "E_NOT_CONVERGED" and r0.info[0]["iters"] == 1
    assert srv.result(h1).status == "ERROR" and "planted" in srv.result(h1).error
    bad = np.zeros((10, 3))
    bad[3, 1] = np.nan
    with pytest.raises(ValueError):
        submit(srv, 10, 2, X=bad)
    with pytest.raises(ValueError):
        srv.submit(np.zeros((10, 3)), [((0, 1, 1), 1.0)], 0.2, 1.0, np.zeros(10))
    with pytest.raises(ValueError):
        srv.submit(np.zeros((10, 3)), [((0, 1, 2), 1.0)], -0.2, 1.0, np.zeros(10))
    with pytest.raises(ValueError):
        srv.submit(np.zeros((10, 3)), [((0, 1, 2), 1.0)], 0.2, 0.0, np.zeros(10))
    with pytest.raises(ValueError):
        srv.submit(np.zeros((10, 3)), [((0, 1, 2, 3), 1.0)], 0.2, 1.0, np.zeros(10))
    assert srv.reserved == 0 and not ex.live_states


def test_cancel_queued_and_live():
    ex = FakeExecutor()
    srv = Server(ex, budget=3_000, clock=Clock())
    a = submit(srv, 20, need=100)
    b = submit(srv, 20, need=100)  # waits for memory
    srv.step()
    assert [r.handle for r in srv.live] == [a] and srv.queue[0].handle == b
    assert srv.cancel(b) and srv.result(b).status == "CANCELLED"
    assert srv.cancel(a) and srv.result(a).status == "CANCELLED"
    assert not srv.cancel(12345)
    assert not srv.busy() and srv.reserved == 0 and not ex.live_states


def test_latency_statistics_follow_the_clock():
    ex = FakeExecutor()
    clk = Clock()
    srv = Server(ex, budget=10**9, clock=clk, iters_per_round=1)
    hs = [submit(srv, 5, need=k + 1, arrival=0.0) for k in range(20)]
    srv.run_until_idle()
    lat = [srv.result(h).latency for h in hs]
    # a request needing more iterations finishes later
    assert lat == sorted(lat)
    st = srv.stats(warmup_fraction=0.1)
    assert st["completed"] == 20 and st["measured"] == 18
    assert math.isclose(st["p50_s"], float(np.percentile(lat[2:], 50)))
    assert st["p99_s"] >= st["p50_s"] > 0 and st["solves_per_s"] > 0


def test_estimate_grows_with_size():
    assert estimate_bytes(2000, 3, 2) > estimate_bytes(1000, 3, 2)
    assert estimate_bytes(1000, 3, 4) > estimate_bytes(1000, 3, 2)
    assert estimate_bytes(1000, 3, 1, 8) > estimate_bytes(1000, 3, 1, 4)
    r = Request(np.zeros((4, 3)), [((0, 1, 2), 1.0)], 0.1, 1.0, np.zeros((4, 2)), 1e-6, 10, 0.0)
    validate(r)
    assert r.nrhs == 2 and r.N == 4


class SlowPlanExecutor(FakeExecutor):
    def plan(self, req):
        import time
        time.sleep(0.002 * (1 + req.handle % 3))  # finish out of order
        return super().plan(req)


def test_planner_threads_keep_order_and_budget():
    ex = SlowPlanExecutor()
    srv = Server(ex, budget=8_000, max_live=6, iters_per_round=1, planners=3, clock=Clock())
    hs = [submit(srv, 10 + 7 * (k % 5), need=2 + k % 4) for k in range(15)]
    while srv.busy():
        srv.step()
        assert srv.reserved <= srv.budget
    assert srv.reserved == 0 and not ex.live_states
    assert all(srv.result(h).status == "OK" for h in hs)
    srv.close()


def test_close_cancels_pending():
    ex = SlowPlanExecutor()
    srv = Server(ex, budget=100_000, planners=2, clock=Clock())
    hs = [submit(srv, 10, need=50) for _ in range(5)]
    srv.step()
    srv.close()
    assert all(srv.result(h).status == "CANCELLED" for h in hs)
    assert srv.reserved == 0 and not ex.live_states


class AsyncPollExecutor(FakeExecutor):
    """Polls one round late, like the device executor's asynchronous poll."""

    def active_async(self, states):
        return [self.active(s) for s in states]

    def active_wait(self, handle):
        return handle


def test_asynchronous_poll_retires_one_round_late():
    ex = AsyncPollExecutor()
    srv = Server(ex, budget=10_000, max_live=4, iters_per_round=2, clock=Clock())
    hs = [submit(srv, 10 + k, need=2 + 3 * k) for k in range(6)]
    while srv.busy():
        srv.step()
        assert srv.reserved <= srv.budget
    assert all(srv.result(h).status == "OK" for h in hs)
    assert srv.reserved == 0 and not ex.live_states
    # a cancelled live request is not retired again from a stale poll
    h = submit(srv, 10, need=50)
    srv.step()
    srv.step()
    assert srv.cancel(h)
    srv.step()
    assert srv.result(h).status == "CANCELLED" and not ex.live_states
