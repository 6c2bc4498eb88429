"""Scheduling of the serving loop with a stand-in executor (no device):
first-come-first-served admission, the device-memory cap, several groups in
service at once, grouping by grid side, per-request failure isolation and the
latency statistics."""
import threading
import time

import numpy as np

from paper_1312_4587_amd.serving import Outcome, Server, footprint_bytes


class FakeExecutor:
    """Sleeps a per-design time per group; fails the request ids in `bad`
    (per request) or raises for groups containing an id in `boom`."""

    def __init__(self, seconds, bad=(), boom=()):
        self.seconds = seconds
        self.bad = set(bad)
        self.boom = set(boom)
        self.lock = threading.Lock()
        self.order = []
        self.groups = []

    def __call__(self, slot, reqs):
        with self.lock:
            self.order.extend(r.rid for r in reqs)
            self.groups.append([r.rid for r in reqs])
        time.sleep(max(self.seconds[r.design] for r in reqs))
        if any(r.rid in self.boom for r in reqs):
            raise RuntimeError("executor failure")
        return [Outcome(False, error="bad request") if r.rid in self.bad else
                Outcome(True, np.array([r.design, r.variant, 0, 0], float))
                for r in reqs]


def test_all_served_in_arrival_order_with_one_slot():
    ex = FakeExecutor([0.002] * 3)
    srv = Server(ex, lambda d: 100, slots=1, capacity_bytes=1e9)
    st = srv.run(np.arange(20) * 0.001, np.arange(20) % 3, variants=np.arange(20) % 4)
    assert st["requests"] == 20 and st["served"] == 20 and st["errors"] == 0
    assert ex.order == list(range(20)) and st["max_in_service"] == 1
    assert all(srv.results[r].out4[0] == r % 3 and srv.results[r].out4[1] == r % 4
               for r in range(20))
    assert st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]


def test_slots_overlap_and_memory_cap_binds():
    # a burst of 40 requests: with four slots and room for everything, four
    # run at once; with room for two footprints, at most two do
    arrivals = np.zeros(40)
    designs = np.zeros(40, int)
    srv = Server(FakeExecutor([0.01]), lambda d: 100, slots=4, capacity_bytes=1e9)
    st = srv.run(arrivals, designs)
    assert st["max_in_service"] == 4 and st["peak_admitted_bytes"] == 400
    srv = Server(FakeExecutor([0.01]), lambda d: 100, slots=4, capacity_bytes=250)
    st = srv.run(arrivals, designs)
    assert st["max_in_service"] == 2 and st["peak_admitted_bytes"] <= 250


def test_request_larger_than_capacity_runs_alone():
    srv = Server(FakeExecutor([0.005, 0.005]), lambda d: [100, 1000][d], slots=4,
                 capacity_bytes=300)
    st = srv.run(np.zeros(6), np.array([0, 1, 0, 0, 1, 0]))
    assert st["requests"] == 6
    for r in srv.results.values():
        if r.design == 1:
            others = [q for q in srv.results.values() if q.rid != r.rid and
                      q.start < r.done and r.start < q.done]
            assert not others


def test_latency_counts_queueing():
    # one slot, 10 requests at once, 10 ms each: the last waits ~90 ms
    srv = Server(FakeExecutor([0.01]), lambda d: 1, slots=1)
    st = srv.run(np.zeros(10), np.zeros(10, int))
    assert st["max_ms"] >= 90.0 and st["p50_ms"] >= 40.0


def test_groups_share_a_grid_side_and_respect_batch_and_memory():
    # designs 0, 1 on grid 64, design 2 on grid 128: a burst is served in
    # groups of one grid side, at most max_batch each, within the memory cap
    grid = {0: 64, 1: 64, 2: 128}
    ex = FakeExecutor([0.01, 0.01, 0.01])
    srv = Server(ex, lambda d: 100, slots=1, capacity_bytes=350, grid=grid.get,
                 max_batch=4)
    designs = np.array([0, 2, 1, 0, 2, 1, 1, 0, 2, 2])
    st = srv.run(np.zeros(10), designs)
    assert st["served"] == 10 and sorted(ex.order) == list(range(10))
    for g in ex.groups:
        assert len({grid[designs[r]] for r in g}) == 1
        assert len(g) <= 3                      # 350 bytes hold three requests
    assert st["max_batch_seen"] == 3 and st["groups"] < 10
    # the head of the queue is always served first (no starvation)
    assert ex.groups[0][0] == 0 and ex.groups[1][0] == 1
    # one request at a time without batching
    ex = FakeExecutor([0.001] * 3)
    st = Server(ex, lambda d: 1, slots=1, grid=grid.get).run(np.zeros(10), designs)
    assert st["max_batch_seen"] == 1 and st["groups"] == 10


def test_failed_requests_fail_alone_and_release_their_share():
    # requests 3 and 7 fail inside the executor; the others are served, every
    # slot share and admitted byte is released, the statistics cover the
    # successes and list the failures
    ex = FakeExecutor([0.003], bad=(3, 7))
    srv = Server(ex, lambda d: 100, slots=2, capacity_bytes=1e9)
    st = srv.run(np.arange(12) * 0.001, np.zeros(12, int))
    assert st["requests"] == 12 and st["served"] == 10 and st["errors"] == 2
    assert st["failed_ids"] == [3, 7]
    assert not srv.results[3].ok and srv.results[3].error == "bad request"
    assert all(srv.results[r].ok for r in range(12) if r not in (3, 7))
    assert srv.admitted_bytes == 0 and srv.in_service == 0


def test_executor_exception_fails_only_its_group():
    # the executor raises for the group holding request 4: that group fails,
    # later requests are served, nothing stays admitted
    ex = FakeExecutor([0.002], boom=(4,))
    srv = Server(ex, lambda d: 10, slots=1, capacity_bytes=1e9)
    st = srv.run(np.arange(10) * 0.004, np.zeros(10, int))
    assert st["errors"] >= 1 and 4 in st["failed_ids"]
    assert srv.results[4].error.startswith("RuntimeError")
    assert srv.results[9].ok and st["served"] == 10 - st["errors"]
    assert srv.admitted_bytes == 0 and srv.in_service == 0


def test_footprint_formula():
    assert footprint_bytes(10, 5, 20, 8) == 16 * 10 + 8 * 10 + 12 * 20 + 4 * 6 + 8 * 64
    assert footprint_bytes(10, 5, 20, 8, 7, 3) == footprint_bytes(10, 5, 20, 8) + 10


def test_waiting_requests_time_out_without_running():
    # one slot, 20 ms per request, 10 at once, 50 ms deadline: the requests
    # that would start after it fail with "timeout" and never reach the
    # executor; everything admitted is released
    ex = FakeExecutor([0.02])
    srv = Server(ex, lambda d: 100, slots=1, capacity_bytes=1e9, timeout_s=0.05)
    st = srv.run(np.zeros(10), np.zeros(10, int))
    late = [r for r in range(10) if srv.results[r].error == "timeout"]
    assert st["requests"] == 10 and st["timeouts"] == len(late) >= 5
    assert st["served"] + st["timeouts"] == 10
    assert not set(late) & set(ex.order)
    assert all(srv.results[r].ok for r in ex.order)
    assert srv.admitted_bytes == 0 and srv.in_service == 0
    assert st["max_queue_depth"] >= 8 and st["mean_queue_depth"] > 0


def test_cancel_withdraws_a_waiting_request_only():
    # the executor, while running request 0 on the only slot, cancels
    # request 5 (waiting: withdrawn) and request 0 (in service: refused)
    answers = {}

    class Canceller(FakeExecutor):
        def __call__(self, slot, reqs):
            if reqs[0].rid == 0:
                time.sleep(0.01)               # let the burst queue up
                answers[5] = srv.cancel(5)
                answers[0] = srv.cancel(0)
                answers[99] = srv.cancel(99)
            return super().__call__(slot, reqs)

    ex = Canceller([0.002])
    srv = Server(ex, lambda d: 10, slots=1, capacity_bytes=1e9)
    st = srv.run(np.zeros(8), np.zeros(8, int))
    assert answers == {5: True, 0: False, 99: False}
    assert srv.results[5].error == "cancelled" and 5 not in ex.order
    assert st["cancelled"] == 1 and st["served"] == 7 and srv.results[0].ok
    assert srv.admitted_bytes == 0 and srv.in_service == 0
