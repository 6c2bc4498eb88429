"""Serving loop: evaluation requests for placements of different designs and
grid sizes arriving over time, served with continuous batching on one device.

A request names a registered design and carries one placement of its cells
(positions in pinned host memory); it asks for one evaluation (the density,
the solve and both gradients, as in Algorithm 1's density / solve / gradient
steps).  A design's static state (cell sizes, netlist, fixed maps, exchange
index) is uploaded and indexed once, by the first request that needs it, and
then stays resident in device memory (least recently used designs are evicted
when the resident bytes would pass the executor's budget).

The server keeps ``slots`` worker threads, each with its own HIP stream
(default priority).  When a slot is free it takes the waiting request at the
head of the queue, first come first served, provided its device footprint
fits under ``capacity_bytes`` together with the requests already in service,
and with it every other waiting request of the same grid side that also fits,
up to ``max_batch``: the group is evaluated by one batched call, every stage
one launch over all of its designs.  Groups on different slots overlap on the
device.  Latency is the time from a request's arrival to its results being in
host memory.

Failures stay with their request: an executor reports a status per request,
a request that fails releases its slot share and its admitted bytes like any
other, and the statistics cover the requests that succeeded, with the failed
ones counted and listed.  A request still waiting ``timeout_s`` after its
arrival is failed with "timeout" without running, and ``cancel(rid)``
withdraws a waiting request ("cancelled"); neither touches a request already
in service.

The executor is the part that touches the device; ``Server`` only schedules,
so the scheduling logic can be exercised with any callable of the same
signature.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    design: int
    variant: int = 0


@dataclasses.dataclass
class Result:
    rid: int
    design: int
    arrival: float
    variant: int = 0
    start: float = 0.0
    done: float = 0.0
    slot: int = -1
    batch: int = 0
    ok: bool = False
    error: Optional[str] = None
    out4: Optional[np.ndarray] = None
    gx: Optional[np.ndarray] = None
    gy: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclasses.dataclass
class Outcome:
    """One request's result from an executor: ok with (out4, gx, gy), or an
    error message."""
    ok: bool
    out4: Optional[np.ndarray] = None
    gx: Optional[np.ndarray] = None
    gy: Optional[np.ndarray] = None
    error: Optional[str] = None


def footprint_bytes(m: int, num_nets: int, num_pins: int, n: int, index_bytes: int = 0,
                    work_bytes: int = 0) -> int:
    """Device bytes one request holds while admitted: cells (x, y, w, h) and
    gradients, pins (cell, dx, dy), net pointers, the fixed maps, plus the
    index and evaluation workspace when known."""
    return (16 * m + 8 * m + 12 * num_pins + 4 * (num_nets + 1) + 8 * n * n
            + index_bytes + work_bytes)


class Server:
    """Continuous-batching scheduler over ``slots`` workers.

    executor(slot, [Request, ...]) -> [Outcome, ...] runs a group of requests
    (one grid side) to completion, results in host memory, one outcome per
    request (it may also raise: then every request of the group fails with
    that error); footprint(design) -> bytes; grid(design) -> grid side.
    """

    def __init__(self, executor: Callable, footprint: Callable[[int], int], slots: int = 8,
                 capacity_bytes: float = 200e9, keep: Sequence[int] = (),
                 grid: Optional[Callable[[int], int]] = None, max_batch: int = 1,
                 timeout_s: Optional[float] = None):
        self.executor = executor
        self.footprint = footprint
        self.grid = grid or (lambda d: 0)
        self.slots = slots
        self.max_batch = max(1, int(max_batch))
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
        self.busy_intervals: List[tuple] = []
        self.batch_sizes: List[int] = []
        self.timeout_s = timeout_s
        self.queue_seen: List[int] = []   # queue length each arrival found
        self.max_queue = 0

    def _fail_waiting(self, res: Result, why: str) -> None:
        """Under the lock: a request that leaves the queue without running."""
        res.done = time.perf_counter() - self.t0
        res.start = res.done
        res.ok = False
        res.error = why
        self.results[res.rid] = res

    def _expire(self) -> None:
        """Under the lock: fail the waiting requests past their deadline."""
        if self.timeout_s is None or not self.waiting:
            return
        now = time.perf_counter() - self.t0
        keep = collections.deque()
        for item in self.waiting:
            if now - item[0].arrival > self.timeout_s:
                self._fail_waiting(item[0], "timeout")
            else:
                keep.append(item)
        self.waiting = keep

    def cancel(self, rid: int) -> bool:
        """Withdraw request rid if it is still waiting (it fails with
        "cancelled"); False if it is in service, done or unknown."""
        with self.cv:
            for i, item in enumerate(self.waiting):
                if item[0].rid == rid:
                    del self.waiting[i]
                    self._fail_waiting(item[0], "cancelled")
                    self.cv.notify_all()
                    return True
        return False

    def _take(self) -> Optional[List[Tuple[Result, int]]]:
        """Under the lock: the head request and the other waiting requests of
        its grid side that fit, or None when nothing can start yet."""
        res, need = self.waiting[0]
        if not (self.admitted_bytes + need <= self.capacity or self.in_service == 0):
            return None
        group = [self.waiting.popleft()]
        room = self.admitted_bytes + need
        if self.max_batch > 1:
            n = self.grid(res.design)
            keep_q = collections.deque()
            while self.waiting and len(group) < self.max_batch:
                item = self.waiting.popleft()
                if self.grid(item[0].design) == n and room + item[1] <= self.capacity:
                    group.append(item)
                    room += item[1]
                else:
                    keep_q.append(item)
            keep_q.extend(self.waiting)
            self.waiting = keep_q
        return group

    def _worker(self, slot: int):
        while True:
            with self.cv:
                while True:
                    self._expire()
                    group = self._take() if self.waiting else None
                    if group is not None:
                        break
                    if self.closed and not self.waiting:
                        return
                    # with a deadline, wake up to expire waiting requests
                    self.cv.wait(self.timeout_s if self.timeout_s else None)
                need = sum(g[1] for g in group)
                self.admitted_bytes += need
                self.peak_bytes = max(self.peak_bytes, self.admitted_bytes)
                self.in_service += len(group)
                self.max_in_service = max(self.max_in_service, self.in_service)
                start = time.perf_counter() - self.t0
                for res, _ in group:
                    res.start = start
                    res.slot = slot
                    res.batch = len(group)
                self.batch_sizes.append(len(group))
            reqs = [Request(r.rid, r.design, r.variant) for r, _ in group]
            try:
                outs = list(self.executor(slot, reqs))
                if len(outs) != len(reqs):
                    raise RuntimeError("executor returned a wrong number of outcomes")
            except Exception as e:   # the whole group failed
                outs = [Outcome(False, error=f"{type(e).__name__}: {e}") for _ in reqs]
            done = time.perf_counter() - self.t0
            # whatever happened, the group's slot share and bytes are released
            with self.cv:
                for (res, _), o in zip(group, outs):
                    res.done = done
                    res.ok = bool(o.ok)
                    res.error = o.error
                    res.out4 = o.out4
                    if res.rid in self.keep:
                        res.gx, res.gy = o.gx, o.gy
                    self.results[res.rid] = res
                self.admitted_bytes -= need
                self.in_service -= len(group)
                self.busy_intervals.append((start, done))
                self.cv.notify_all()

    def run(self, arrivals: Sequence[float], designs: Sequence[int],
            variants: Optional[Sequence[int]] = None) -> Dict[str, float]:
        """Serve requests r = 0.. arriving at arrivals[r] seconds (from the
        start of the run) for designs[r] (placement variants[r]); returns the
        latency statistics of the requests that succeeded."""
        self.t0 = time.perf_counter()
        workers = [threading.Thread(target=self._worker, args=(s,), daemon=True)
                   for s in range(self.slots)]
        for w in workers:
            w.start()
        for rid, (t, d) in enumerate(zip(arrivals, designs)):
            now = time.perf_counter() - self.t0
            if t > now:
                time.sleep(t - now)
            v = int(variants[rid]) if variants is not None else 0
            res = Result(rid=rid, design=int(d), arrival=float(t), variant=v)
            with self.cv:
                self.queue_seen.append(len(self.waiting))
                self.waiting.append((res, self.footprint(int(d))))
                self.max_queue = max(self.max_queue, len(self.waiting))
                self.cv.notify_all()
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for w in workers:
            w.join()
        return self.stats(time.perf_counter() - self.t0)

    def stats(self, wall: float) -> Dict[str, float]:
        good = [r for r in self.results.values() if r.ok]
        failed = sorted(r.rid for r in self.results.values() if not r.ok)
        lat = np.array([r.latency for r in good]) if good else np.zeros(1)
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
        bs = np.array(self.batch_sizes) if self.batch_sizes else np.zeros(1)
        why = collections.Counter(r.error for r in self.results.values() if not r.ok)
        return dict(requests=len(self.results), served=len(good), errors=len(failed),
                    failed_ids=failed[:20], timeouts=why.get("timeout", 0),
                    cancelled=why.get("cancelled", 0), wall_s=wall,
                    max_queue_depth=self.max_queue,
                    mean_queue_depth=float(np.mean(self.queue_seen)) if self.queue_seen else 0.0,
                    evals_per_s=len(good) / wall if wall > 0 else 0.0,
                    p50_ms=float(np.percentile(lat, 50) * 1e3),
                    p99_ms=float(np.percentile(lat, 99) * 1e3),
                    mean_ms=float(lat.mean() * 1e3), max_ms=float(lat.max() * 1e3),
                    in_service_fraction=busy / wall if wall > 0 else 0.0,
                    max_in_service=self.max_in_service, peak_admitted_bytes=self.peak_bytes,
                    groups=len(self.batch_sizes), mean_batch=float(bs.mean()),
                    max_batch_seen=int(bs.max()))


class DeviceExecutor:
    """Runs groups of requests on the GPU.  Each design's static state is
    uploaded, its fixed maps rasterised and its exchange index built once, on
    first use, and kept resident (least recently used designs evicted past
    ``resident_bytes``); each slot owns max_batch evaluation workspaces and
    position / gradient buffers sized for the largest design, so a request
    only moves its positions in and its gradients and scalars out.  A group
    is one fftpl_eval_batch call; if the call refuses the group (an argument
    error: nothing ran) its requests are retried one at a time, so only the
    faulty one fails."""

    def __init__(self, pool, slots: int, dct: str = "fft", grad_mode: str = "field",
                 lam: float = 1.0, max_batch: int = 1, variants: int = 4, seed: int = 5,
                 resident_bytes: float = 100e9):
        import torch

        from . import fftpl
        self.torch, self.fftpl = torch, fftpl
        self.pool = pool
        self.dct, self.grad_mode, self.lam = dct, grad_mode, lam
        self.max_batch = max(1, int(max_batch))
        self.resident_bytes = resident_bytes
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.plans = [dict() for _ in range(slots)]
        self.lock = threading.Lock()
        self.design_locks = [threading.Lock() for _ in pool]
        self.resident: "collections.OrderedDict[int, dict]" = collections.OrderedDict()
        self.in_use = collections.Counter()
        self.resident_total = 0
        self.loads = 0
        self.load_s = 0.0
        # host side, pinned: static arrays and `variants` placements per design
        # (request r of design d evaluates placement r mod variants: the
        # design's positions moved by a seeded sub-bin jitter)
        self.host = []
        rng = np.random.default_rng(np.random.SeedSequence([seed, 7]))
        f, i = torch.float32, torch.int32

        def pin(a, dt):
            return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).pin_memory()
        for inst in pool:
            pos = []
            for v in range(max(1, variants)):
                jx = 0 if v == 0 else rng.uniform(-0.5, 0.5, inst.num_cells) * inst.bin_w
                jy = 0 if v == 0 else rng.uniform(-0.5, 0.5, inst.num_cells) * inst.bin_h
                pos.append((pin(np.clip(inst.x + jx, 0, inst.side), f),
                            pin(np.clip(inst.y + jy, 0, inst.side), f)))
            self.host.append(dict(
                w=pin(inst.w, f), h=pin(inst.h, f), net_ptr=pin(inst.net_ptr, i),
                pin_cell=pin(inst.pin_cell, i), pin_dx=pin(inst.pin_dx, f),
                pin_dy=pin(inst.pin_dy, f), pos=pos,
                max_degree=int(np.diff(inst.net_ptr).max()) if inst.num_nets else 0))
        self.m_max = max(inst.num_cells for inst in pool)
        self.work_max = max(fftpl.problem_work_bytes(inst.n, inst.num_cells, inst.num_nets,
                                                     inst.num_pins) for inst in pool)
        self.slot_bufs = [None] * slots

    def positions(self, d: int, variant: int):
        """Host copies (x, y) of placement `variant` of design d."""
        x, y = self.host[d]["pos"][variant % len(self.host[d]["pos"])]
        return x.numpy(), y.numpy()

    def footprint(self, d: int) -> int:
        inst = self.pool[d]
        ib, _ = self.fftpl.xindex_bytes(inst.num_cells, inst.num_nets, inst.num_pins,
                                        self.host[d]["max_degree"])
        wb = self.fftpl.problem_work_bytes(inst.n, inst.num_cells, inst.num_nets,
                                           inst.num_pins)
        return footprint_bytes(inst.num_cells, inst.num_nets, inst.num_pins, inst.n, ib, wb)

    def grid(self, d: int) -> int:
        return int(self.pool[d].n)

    def warm(self, load_designs: bool = False) -> None:
        """Every slot's plans and buffers up front; with load_designs, every
        design of the pool made resident too."""
        for s in range(len(self.streams)):
            for n in sorted({inst.n for inst in self.pool}):
                self._plan(s, n)
            self._bufs(s)
        if load_designs:
            for d in range(len(self.pool)):
                self._acquire(d, self.streams[0])
                self._release(d)
        self.torch.cuda.synchronize()

    def _plan(self, slot: int, n: int):
        p = self.plans[slot].get(n)
        if p is None:
            p = self.fftpl.Plan(n, self.dct, stream=self.streams[slot],
                                max_batch=self.max_batch)
            self.plans[slot][n] = p
        return p

    def _bufs(self, slot: int):
        b = self.slot_bufs[slot]
        if b is None:
            torch = self.torch
            B, m = self.max_batch, self.m_max
            b = dict(work=[torch.empty(self.work_max, dtype=torch.uint8, device="cuda")
                           for _ in range(B)],
                     x=torch.empty((B, m), device="cuda"), y=torch.empty((B, m), device="cuda"),
                     gx=torch.empty((B, m), device="cuda"), gy=torch.empty((B, m), device="cuda"),
                     out4=torch.empty((B, 4), dtype=torch.float64, device="cuda"),
                     hgx=torch.empty((B, m)).pin_memory(), hgy=torch.empty((B, m)).pin_memory(),
                     hout=torch.empty((B, 4), dtype=torch.float64).pin_memory())
            self.slot_bufs[slot] = b
        return b

    def _load(self, d: int, stream) -> dict:
        """Upload design d, rasterise its (empty) fixed map and build its
        exchange index on `stream` (the index build waits for it)."""
        torch, fftpl = self.torch, self.fftpl
        inst, h = self.pool[d], self.host[d]
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            dv = {k: h[k].to("cuda", non_blocking=True)
                  for k in ("w", "h", "net_ptr", "pin_cell", "pin_dx", "pin_dy")}
            grid = fftpl.Grid.of(inst)
            n2 = grid.n * grid.n
            base = torch.empty(n2, dtype=torch.float32, device="cuda")
            cap = torch.empty(n2, dtype=torch.float32, device="cuda")
            fftpl.fixed_map(grid, None, None, None, None, base, cap, stream=stream)
            prob = fftpl.Problem(grid, dv["w"], dv["h"], dv["net_ptr"], dv["pin_cell"],
                                 dv["pin_dx"], dv["pin_dy"], base=base, cap=cap,
                                 stream=stream, max_degree=h["max_degree"], own_work=False)
        stream.synchronize()
        self.loads += 1
        self.load_s += time.perf_counter() - t0
        return dict(prob=prob, bytes=self.footprint(d))

    def _acquire(self, d: int, stream) -> dict:
        with self.design_locks[d]:
            with self.lock:
                ent = self.resident.get(d)
                if ent is not None:
                    self.resident.move_to_end(d)
                    self.in_use[d] += 1
                    return ent
            ent = self._load(d, stream)
            with self.lock:
                # evict idle designs, least recently used first, past the budget
                for od in list(self.resident):
                    if self.resident_total + ent["bytes"] <= self.resident_bytes:
                        break
                    if self.in_use[od] == 0:
                        self.resident_total -= self.resident.pop(od)["bytes"]
                self.resident[d] = ent
                self.resident_total += ent["bytes"]
                self.in_use[d] += 1
                return ent

    def _release(self, d: int) -> None:
        with self.lock:
            self.in_use[d] -= 1

    def __call__(self, slot: int, reqs: Sequence[Request]) -> List[Outcome]:
        torch, fftpl = self.torch, self.fftpl
        st = self.streams[slot]
        b = self._bufs(slot)
        ok = [True] * len(reqs)
        err: List[Optional[str]] = [None] * len(reqs)
        ents: List[Optional[dict]] = [None] * len(reqs)
        try:
            # a design that cannot be made resident (a malformed netlist the
            # index build refuses) fails its own requests only
            for k, r in enumerate(reqs):
                try:
                    ents[k] = self._acquire(r.design, st)
                except (fftpl.FFTPLError, ValueError, TypeError) as e:
                    ok[k] = False
                    err[k] = f"{type(e).__name__}: {e}"
            good = [k for k in range(len(reqs)) if ok[k]]
            with torch.cuda.stream(st):
                probs, xs, ys, gxs, gys = [], [], [], [], []
                for j, k in enumerate(good):
                    r = reqs[k]
                    m = self.pool[r.design].num_cells
                    hx, hy = self.host[r.design]["pos"][r.variant % len(
                        self.host[r.design]["pos"])]
                    b["x"][j, :m].copy_(hx, non_blocking=True)
                    b["y"][j, :m].copy_(hy, non_blocking=True)
                    probs.append(ents[k]["prob"].with_work(b["work"][j]))
                    xs.append(b["x"][j, :m])
                    ys.append(b["y"][j, :m])
                    gxs.append(b["gx"][j, :m])
                    gys.append(b["gy"][j, :m])
                if good:
                    n = self.pool[reqs[good[0]].design].n
                    plan = self._plan(slot, n)
                    lams = [self.lam] * len(good)
                    gams = [self.pool[reqs[k].design].gamma for k in good]
                    try:
                        fftpl.eval_batch(plan, probs, xs, ys, lams, gams, self.grad_mode, gxs,
                                         gys, b["out4"][:len(good)], stream=st)
                    except (fftpl.FFTPLError, ValueError, TypeError):
                        # the group was refused before anything ran: one at a time
                        for j, k in enumerate(good):
                            try:
                                fftpl.eval(plan, probs[j], xs[j], ys[j], lams[j], gams[j],
                                           self.grad_mode, gxs[j], gys[j], b["out4"][j],
                                           stream=st)
                            except (fftpl.FFTPLError, ValueError, TypeError) as e:
                                ok[k] = False
                                err[k] = f"{type(e).__name__}: {e}"
                    b["hout"][:len(good)].copy_(b["out4"][:len(good)], non_blocking=True)
                    for j, k in enumerate(good):
                        m = self.pool[reqs[k].design].num_cells
                        if ok[k]:
                            b["hgx"][j, :m].copy_(gxs[j], non_blocking=True)
                            b["hgy"][j, :m].copy_(gys[j], non_blocking=True)
                st.synchronize()
                outs = [Outcome(False, error=err[k]) for k in range(len(reqs))]
                for j, k in enumerate(good):
                    if ok[k]:
                        m = self.pool[reqs[k].design].num_cells
                        outs[k] = Outcome(True, b["hout"][j].numpy().copy(),
                                          b["hgx"][j, :m].numpy().copy(),
                                          b["hgy"][j, :m].numpy().copy())
                    else:
                        outs[k] = Outcome(False, error=err[k])
                return outs
        finally:
            for k, r in enumerate(reqs):
                if ents[k] is not None:
                    self._release(r.design)

    def close(self) -> None:
        self.torch.cuda.synchronize()
        for d in self.plans:
            for p in d.values():
                p.close()
        self.resident.clear()
        self.slot_bufs = [None] * len(self.slot_bufs)
