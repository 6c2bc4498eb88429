"""Serving loop: evaluation requests of different designs and grid sizes
arriving over time, served with continuous batching on one device.

A request carries a whole design (cells, nets, sizes) in pinned host memory
and asks for one evaluation (the density, the solve and both gradients, as in
Algorithm 1's density / solve / gradient steps).  The server keeps ``slots``
worker threads, each with its own HIP stream (default priority) and its own
plans (one per grid side).  A waiting request is admitted, first come first
served, as soon as a slot is free and its device footprint fits under
``capacity_bytes`` together with the requests already on the device; its
upload, index build, evaluation and download then run on the slot's stream,
overlapping the other slots' work on the device.  Latency is the time from the
request's arrival to its results being in host memory.

The executor is the part that touches the device; ``Server`` only schedules,
so the scheduling logic can be exercised with any callable of the same
signature.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Result:
    rid: int
    design: int
    arrival: float
    start: float = 0.0
    done: float = 0.0
    slot: int = -1
    out4: Optional[np.ndarray] = None
    gx: Optional[np.ndarray] = None
    gy: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def footprint_bytes(m: int, num_nets: int, num_pins: int, n: int, index_bytes: int = 0,
                    work_bytes: int = 0) -> int:
    """Device bytes one request holds while admitted: cells (x, y, w, h) and
    gradients, pins (cell, dx, dy), net pointers, the fixed maps, plus the
    index and evaluation workspace when known."""
    return (16 * m + 8 * m + 12 * num_pins + 4 * (num_nets + 1) + 8 * n * n
            + index_bytes + work_bytes)


class Server:
    """Continuous-batching scheduler over ``slots`` workers.

    executor(slot, request_id, design_index) -> (out4, gx, gy) runs one request
    to completion (results in host memory); footprint(design_index) -> bytes.
    """

    def __init__(self, executor: Callable, footprint: Callable[[int], int], slots: int = 8,
                 capacity_bytes: float = 200e9, keep: Sequence[int] = ()):
        self.executor = executor
        self.footprint = footprint
        self.slots = slots
        self.capacity = capacity_bytes
        self.keep = set(keep)
        self.cv = threading.Condition()
        self.waiting: collections.deque = collections.deque()
        self.admitted_bytes = 0
        self.peak_bytes = 0
        self.in_service = 0
        self.max_in_service = 0
        self.closed = False
        self.results: Dict[int, Result] = {}
        self.errors: List[BaseException] = []
        self.busy_intervals: List[tuple] = []

    def _worker(self, slot: int):
        while True:
            with self.cv:
                while True:
                    if self.waiting:
                        res, need = self.waiting[0]
                        if self.admitted_bytes + need <= self.capacity or self.in_service == 0:
                            self.waiting.popleft()
                            break
                    elif self.closed:
                        return
                    self.cv.wait()
                self.admitted_bytes += need
                self.peak_bytes = max(self.peak_bytes, self.admitted_bytes)
                self.in_service += 1
                self.max_in_service = max(self.max_in_service, self.in_service)
                res.start = time.perf_counter() - self.t0
                res.slot = slot
            try:
                out4, gx, gy = self.executor(slot, res.rid, res.design)
                res.out4 = out4
                if res.rid in self.keep:
                    res.gx, res.gy = gx, gy
            except BaseException as e:   # reported by run()
                with self.cv:
                    self.errors.append(e)
            res.done = time.perf_counter() - self.t0
            with self.cv:
                self.admitted_bytes -= need
                self.in_service -= 1
                self.busy_intervals.append((res.start, res.done))
                self.results[res.rid] = res
                self.cv.notify_all()

    def run(self, arrivals: Sequence[float], designs: Sequence[int]) -> Dict[str, float]:
        """Serve requests r = 0.. arriving at arrivals[r] seconds (from the
        start of the run) for designs[r]; returns the latency statistics."""
        self.t0 = time.perf_counter()
        workers = [threading.Thread(target=self._worker, args=(s,), daemon=True)
                   for s in range(self.slots)]
        for w in workers:
            w.start()
        for rid, (t, d) in enumerate(zip(arrivals, designs)):
            now = time.perf_counter() - self.t0
            if t > now:
                time.sleep(t - now)
            res = Result(rid=rid, design=int(d), arrival=float(t))
            with self.cv:
                self.waiting.append((res, self.footprint(int(d))))
                self.cv.notify_all()
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for w in workers:
            w.join()
        wall = time.perf_counter() - self.t0
        if self.errors:
            raise self.errors[0]
        return self.stats(wall)

    def stats(self, wall: float) -> Dict[str, float]:
        lat = np.array([r.latency for r in self.results.values()])
        # time with at least one request in service
        iv = sorted(self.busy_intervals)
        busy, cur_s, cur_e = 0.0, None, None
        for s, e in iv:
            if cur_e is None or s > cur_e:
                if cur_e is not None:
                    busy += cur_e - cur_s
                cur_s, cur_e = s, e
            else:
                cur_e = max(cur_e, e)
        if cur_e is not None:
            busy += cur_e - cur_s
        return dict(requests=int(lat.size), wall_s=wall,
                    evals_per_s=lat.size / wall if wall > 0 else 0.0,
                    p50_ms=float(np.percentile(lat, 50) * 1e3),
                    p99_ms=float(np.percentile(lat, 99) * 1e3),
                    mean_ms=float(lat.mean() * 1e3), max_ms=float(lat.max() * 1e3),
                    in_service_fraction=busy / wall if wall > 0 else 0.0,
                    max_in_service=self.max_in_service, peak_admitted_bytes=self.peak_bytes)


class DeviceExecutor:
    """Runs a request on the GPU: pinned host copies of each design are
    uploaded on the slot's stream, the exchange index and fixed maps are built,
    one fftpl_eval runs, and the gradients and scalars come back to pinned
    host buffers."""

    def __init__(self, pool, slots: int, dct: str = "fft", grad_mode: str = "field",
                 lam: float = 1.0):
        import torch

        from . import fftpl
        self.torch, self.fftpl = torch, fftpl
        self.pool = pool
        self.dct, self.grad_mode, self.lam = dct, grad_mode, lam
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.plans = [dict() for _ in range(slots)]
        self.host = []
        for inst in pool:
            def pin(a, dt):
                return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).pin_memory()
            f, i = torch.float32, torch.int32
            self.host.append(dict(
                x=pin(inst.x, f), y=pin(inst.y, f), w=pin(inst.w, f), h=pin(inst.h, f),
                net_ptr=pin(inst.net_ptr, i), pin_cell=pin(inst.pin_cell, i),
                pin_dx=pin(inst.pin_dx, f), pin_dy=pin(inst.pin_dy, f),
                max_degree=int(np.diff(inst.net_ptr).max()) if inst.num_nets else 0))
        self.out = [dict() for _ in range(slots)]

    def footprint(self, d: int) -> int:
        inst = self.pool[d]
        ib, _ = self.fftpl.xindex_bytes(inst.num_cells, inst.num_nets, inst.num_pins,
                                        self.host[d]["max_degree"])
        wb = self.fftpl.problem_work_bytes(inst.n, inst.num_cells, inst.num_nets,
                                           inst.num_pins)
        return footprint_bytes(inst.num_cells, inst.num_nets, inst.num_pins, inst.n, ib, wb)

    def warm(self) -> None:
        """Create every slot's plans for the pool's grid sides up front."""
        for s in range(len(self.streams)):
            for n in sorted({inst.n for inst in self.pool}):
                self._plan(s, n)
        self.torch.cuda.synchronize()

    def _plan(self, slot: int, n: int):
        p = self.plans[slot].get(n)
        if p is None:
            p = self.fftpl.Plan(n, self.dct, stream=self.streams[slot])
            self.plans[slot][n] = p
        return p

    def __call__(self, slot: int, rid: int, d: int):
        torch, fftpl = self.torch, self.fftpl
        inst, h = self.pool[d], self.host[d]
        st = self.streams[slot]
        m = inst.num_cells
        with torch.cuda.stream(st):
            dv = {k: v.to("cuda", non_blocking=True) for k, v in h.items()
                  if isinstance(v, torch.Tensor)}
            grid = fftpl.Grid.of(inst)
            n2 = grid.n * grid.n
            base = torch.empty(n2, dtype=torch.float32, device="cuda")
            cap = torch.empty(n2, dtype=torch.float32, device="cuda")
            fftpl.fixed_map(grid, None, None, None, None, base, cap, stream=st)
            prob = fftpl.Problem(grid, dv["w"], dv["h"], dv["net_ptr"], dv["pin_cell"],
                                 dv["pin_dx"], dv["pin_dy"], base=base, cap=cap, stream=st,
                                 max_degree=h["max_degree"])
            gx = torch.empty(m, dtype=torch.float32, device="cuda")
            gy = torch.empty(m, dtype=torch.float32, device="cuda")
            out4 = torch.empty(4, dtype=torch.float64, device="cuda")
            fftpl.eval(self._plan(slot, inst.n), prob, dv["x"], dv["y"], self.lam, inst.gamma,
                       self.grad_mode, gx, gy, out4, stream=st)
            o = self.out[slot]
            if o.get("m", 0) < m:
                o["gx"] = torch.empty(m, dtype=torch.float32).pin_memory()
                o["gy"] = torch.empty(m, dtype=torch.float32).pin_memory()
                o["m"] = m
            if "out4" not in o:
                o["out4"] = torch.empty(4, dtype=torch.float64).pin_memory()
            o["gx"][:m].copy_(gx, non_blocking=True)
            o["gy"][:m].copy_(gy, non_blocking=True)
            o["out4"].copy_(out4, non_blocking=True)
            st.synchronize()
            res = (o["out4"].numpy().copy(), o["gx"][:m].numpy().copy(),
                   o["gy"][:m].numpy().copy())
        return res

    def close(self) -> None:
        for d in self.plans:
            for p in d.values():
                p.close()
