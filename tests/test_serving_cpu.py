"""Scheduling of the serving loop with a stand-in executor (no device):
first-come-first-served admission, the device-memory cap, several requests
in service at once, and the latency statistics."""
import threading
import time

import numpy as np

from paper_1312_4587_amd.serving import Server, footprint_bytes


class FakeExecutor:
    def __init__(self, seconds):
        self.seconds = seconds
        self.lock = threading.Lock()
        self.order = []

    def __call__(self, slot, rid, design):
        with self.lock:
            self.order.append(rid)
        time.sleep(self.seconds[design])
        return np.array([design, 0, 0, 0], float), None, None


def test_all_served_in_arrival_order_with_one_slot():
    ex = FakeExecutor([0.002] * 3)
    srv = Server(ex, lambda d: 100, slots=1, capacity_bytes=1e9)
    st = srv.run(np.arange(20) * 0.001, np.arange(20) % 3)
    assert st["requests"] == 20 and ex.order == list(range(20))
    assert st["max_in_service"] == 1
    assert all(srv.results[r].out4[0] == r % 3 for r in range(20))
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


def test_footprint_formula():
    assert footprint_bytes(10, 5, 20, 8) == 16 * 10 + 8 * 10 + 12 * 20 + 4 * 6 + 8 * 64
    assert footprint_bytes(10, 5, 20, 8, 7, 3) == footprint_bytes(10, 5, 20, 8) + 10
