"""The serving loop's scheduler on the CPU, with a fake backend that sleeps
for a request-dependent service time (no device): continuous admission under
the slot and HBM-budget limits, skip-ahead without starvation, failure
isolation and the latency bookkeeping."""
import threading
import time

import pytest

from paper_1809_05334_amd.serve import Server, summarize


class FakeBackend:
    def __init__(self, service_s=0.02, fail_rids=()):
        self.service_s = service_s
        self.fail_rids = set(fail_rids)
        self.lock = threading.Lock()
        self.live_bytes = 0
        self.max_live_bytes = 0
        self.live = 0
        self.max_live = 0
        self.released = []

    def prepare(self, req):
        return {"req": req}, req["bytes"]

    def make_worker(self, wid):
        return wid

    def run(self, prep, state):
        req = prep["req"]
        with self.lock:
            self.live += 1
            self.live_bytes += req["bytes"]
            self.max_live = max(self.max_live, self.live)
            self.max_live_bytes = max(self.max_live_bytes, self.live_bytes)
        time.sleep(req.get("service", self.service_s))
        with self.lock:
            self.live -= 1
            self.live_bytes -= req["bytes"]
        if req["rid"] in self.fail_rids:
            raise RuntimeError("injected failure")
        n = req["bytes"] // 100
        return {"N": n, "A": [req["rid"] * 1e-3], "R": 0.1, "T": 0.2, "iters": 7}

    def release(self, prep):
        with self.lock:
            self.released.append(prep["req"]["rid"])


def reqs(spec):
    return [{"rid": i, "arrival": a, "bytes": b, **extra} for i, (a, b, extra) in enumerate(spec)]


def test_all_requests_complete_within_slots_and_budget():
    be = FakeBackend()
    trace = reqs([(0.002 * i, 100 * (1 + i % 5), {}) for i in range(40)])
    srv = Server(be, slots=3, hbm_budget=900)
    res = srv.run_trace(trace)
    assert [r.rid for r in res] == list(range(40))
    assert all(r.ok for r in res)
    assert be.max_live <= 3 and srv.peak_running <= 3
    assert be.max_live_bytes <= 900 and srv.peak_used <= 900
    assert sorted(be.released) == list(range(40))
    for r in res:
        assert r.t_arrival <= r.t_admit <= r.t_done
        assert r.latency >= 0.018
        assert r.A == [r.rid * 1e-3]


def test_requests_overlap_when_resources_allow():
    be = FakeBackend(service_s=0.1)
    trace = reqs([(0.0, 100, {}) for _ in range(4)])
    srv = Server(be, slots=4, hbm_budget=1000)
    t0 = time.perf_counter()
    srv.run_trace(trace)
    assert be.max_live == 4
    assert time.perf_counter() - t0 < 0.35    # four 0.1 s requests ran together


def test_skip_ahead_admits_small_requests_behind_a_large_one():
    be = FakeBackend()
    # a long request holds 600 of 1000 bytes; a large one (700) must wait,
    # small ones (100) arriving after it are admitted meanwhile
    trace = reqs([(0.0, 600, {"service": 0.3}), (0.01, 700, {}), (0.02, 100, {}), (0.03, 100, {})])
    srv = Server(be, slots=4, hbm_budget=1000, max_skip_s=5.0)
    res = srv.run_trace(trace)
    assert all(r.ok for r in res)
    order = srv.admit_order
    assert order.index(2) < order.index(1) and order.index(3) < order.index(1)
    assert res[2].t_done < res[1].t_admit


def test_no_skip_ahead_once_the_head_waited_too_long():
    be = FakeBackend()
    trace = reqs([(0.0, 600, {"service": 0.3}), (0.01, 700, {}), (0.2, 100, {})])
    srv = Server(be, slots=4, hbm_budget=1000, max_skip_s=0.05)
    srv.run_trace(trace)
    order = srv.admit_order
    assert order.index(1) < order.index(2)     # the large request is not starved


def test_failures_are_isolated_and_oversized_requests_rejected():
    be = FakeBackend(fail_rids={1})
    trace = reqs([(0.0, 100, {}), (0.0, 100, {}), (0.0, 5000, {}), (0.01, 100, {})])
    srv = Server(be, slots=2, hbm_budget=1000)
    res = srv.run_trace(trace)
    assert res[0].ok and res[3].ok
    assert not res[1].ok and "injected" in res[1].error
    assert not res[2].ok and "budget" in res[2].error
    s = summarize(res, srv.t_end - srv.t_start)
    assert s["ok"] == 2 and s["requests"] == 4


def test_bad_configuration():
    with pytest.raises(ValueError):
        Server(FakeBackend(), slots=0)
