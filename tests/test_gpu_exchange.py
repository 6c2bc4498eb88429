"""Exchange-index wirelength path of fftpl_eval against the FP64 oracle:
many cell and net blocks, ragged last blocks, empty / one-pin / very large
nets, repeated evaluations with new positions on one index, the index
build's refusal of malformed netlists, and the two-stream schedule against
the one-stream one (bit-identical)."""
import dataclasses

import numpy as np
import pytest

import gen
import oracle
from _helpers import rel_l2
from tests.gpu_common import RTOL, dev, host, lib_or_build, say
from tests.test_gpu_parity import _check_eval, _run_eval

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_or_build()
    from paper_1312_4587_amd import fftpl
    return fftpl


def _with_nets(inst, degs, seed):
    """Replace the netlist by nets of the given degrees on random distinct cells."""
    rng = np.random.default_rng(seed)
    m = inst.num_cells
    cells = [rng.choice(m, size=d, replace=False) for d in degs]
    pin_cell = np.concatenate(cells).astype(np.int32) if len(cells) else np.zeros(0, np.int32)
    net_ptr = np.concatenate([[0], np.cumsum(degs)]).astype(np.int32)
    w = inst.w[pin_cell]
    h = inst.h[pin_cell]
    dx = ((rng.random(len(pin_cell)) - 0.5) * w).astype(np.float32)
    dy = ((rng.random(len(pin_cell)) - 0.5) * h).astype(np.float32)
    return dataclasses.replace(inst, net_ptr=net_ptr, pin_cell=pin_cell, pin_dx=dx, pin_dy=dy)


@pytest.mark.parametrize("mode", ["field", "exact"])
def test_exchange_many_blocks_and_new_positions(F, mode):
    # 60k cells = 59 cell blocks (the last one ragged), nets up to degree 3000
    # so the net blocks shrink below their default target
    inst = gen.make_instance(7, num_cells=60_000, util=0.8, n=256, num_nets=70_000,
                             hi_frac=0.01, hi_range=(20, 3000), num_macros=5,
                             macro_area_frac=0.1)
    say("exchange many blocks", mode, inst.num_cells, inst.num_pins)
    got = _run_eval(F, inst, 2.0, mode)
    _check_eval(inst, got, oracle.evaluate(inst, lam=2.0, grad_mode=mode), 2.0, mode)
    # one index, another placement
    rng = np.random.default_rng(70)
    x = np.clip(inst.x + rng.normal(0, 3.0, inst.num_cells), 0, inst.side)
    y = np.clip(inst.y + rng.normal(0, 3.0, inst.num_cells), 0, inst.side)
    inst2 = inst.with_positions(x, y)
    got2 = _run_eval(F, inst2, 2.0, mode)
    _check_eval(inst2, got2, oracle.evaluate(inst2, lam=2.0, grad_mode=mode), 2.0, mode)


def test_exchange_odd_nets(F):
    # empty nets, one-pin nets (zero gradient), a net at the largest degree the
    # index takes (8705), a net of 5000, and ordinary nets, over 20 cell blocks
    base = gen.make_instance(8, num_cells=20000, util=0.7, n=64, num_nets=10)
    rng = np.random.default_rng(80)
    degs = np.concatenate([rng.integers(2, 9, 3000), [8705, 5000, 1, 1, 0, 0],
                           rng.integers(9, 60, 40)])
    rng.shuffle(degs)
    degs = np.concatenate([[0, 1], degs, [0]])
    inst = _with_nets(base, degs, 81)
    say("exchange odd nets", inst.num_cells, inst.num_pins, int(degs.max()))
    for mode in ("field", "exact"):
        got = _run_eval(F, inst, 1.5, mode)
        _check_eval(inst, got, oracle.evaluate(inst, lam=1.5, grad_mode=mode), 1.5, mode)


def test_exchange_matches_other_paths_at_200k(F):
    inst = gen.make_config("mid_200k")
    say("exchange vs slots vs atomic, mid_200k")
    ref = oracle.evaluate(inst, lam=1.0, grad_mode="field")
    for path in ("xch", "slots", "atomic"):
        got = _run_eval(F, inst, 1.0, "field", path=path)
        _check_eval(inst, got, ref, 1.0, "field")


def _build(F, m, net_ptr, pin_cell, max_degree):
    import torch
    ib, _ = F.xindex_bytes(m, len(net_ptr) - 1, len(pin_cell), max_degree)
    index = torch.empty(ib, dtype=torch.uint8, device="cuda")
    F.xindex_build(m, dev(np.asarray(net_ptr, np.int32)), dev(np.asarray(pin_cell, np.int32)),
                   max_degree, index)


def test_exchange_build_rejects_malformed_netlists(F):
    m = 100
    net_ptr = [0, 3, 5, 9]
    pin_cell = [1, 2, 3, 4, 5, 6, 7, 8, 9]
    _build(F, m, net_ptr, pin_cell, 4)                      # valid
    cases = {
        "degree above max_degree": (net_ptr, pin_cell, 3),
        "pin cell out of range": (net_ptr, [1, 2, 3, 4, 5, 6, 7, 8, 100], 4),
        "negative pin cell": (net_ptr, [1, 2, 3, -1, 5, 6, 7, 8, 9], 4),
        "last pointer short": ([0, 3, 5, 8], pin_cell, 4),
        "decreasing pointers": ([0, 5, 3, 9], pin_cell, 6),
        "first pointer nonzero": ([1, 3, 5, 9], pin_cell, 4),
    }
    for name, (ptr, pc, md) in cases.items():
        say("malformed:", name)
        with pytest.raises(F.FFTPLError) as ei:
            _build(F, m, ptr, pc, md)
        assert ei.value.status == F.E_INVAL, name


@pytest.mark.parametrize("path", ["xch", "slots"])
def test_two_stream_schedule_matches_one_stream(F, path):
    # The evaluation normally forks its wirelength branch to the plan's side
    # stream and joins it before the cell sums; with per-kernel timing on,
    # everything runs in order on the caller's stream.  Every sum in the
    # evaluation is order-independent (fixed-point LDS adds, fixed-order
    # block partials), so both schedules must give the same bits, also for
    # evaluations enqueued back to back with new positions and no host wait
    # between them (the next fork must wait for the previous cell sums).
    import torch
    from tests.gpu_common import DeviceCells
    inst = gen.make_instance(31, num_cells=120_000, util=0.8, n=512, num_nets=130_000,
                             hi_frac=0.01, hi_range=(20, 500))
    m = inst.num_cells
    rng = np.random.default_rng(31)
    insts = [inst]
    for _ in range(2):
        x = np.clip(insts[-1].x + rng.normal(0, 2.0, m), 0, inst.side)
        y = np.clip(insts[-1].y + rng.normal(0, 2.0, m), 0, inst.side)
        insts.append(insts[-1].with_positions(x, y))
    say("two-stream schedule", path, m, inst.num_pins)
    prob = F.Problem.from_instance(inst, path=path)
    assert prob.path == path
    plan = F.Plan(inst.n, "fft")
    cells = [DeviceCells(i) for i in insts]
    outs = {}
    for timing in (True, False):
        plan.timing(timing)
        bufs = [(torch.empty(m, device="cuda"), torch.empty(m, device="cuda"),
                 torch.empty(4, dtype=torch.float64, device="cuda")) for _ in insts]
        for c, (gx, gy, o4) in zip(cells, bufs):
            F.eval(plan, prob, c.x, c.y, 1.5, inst.gamma, "field", gx, gy, o4)
        torch.cuda.synchronize()
        outs[timing] = [[host(t) for t in b] for b in bufs]
    plan.timing(False)
    plan.close()
    for one, two in zip(outs[True], outs[False]):
        for a, b in zip(one, two):
            assert np.array_equal(a, b)
    # and the last of them against the oracle
    gx, gy, out = outs[False][-1]
    ref = oracle.evaluate(insts[-1], lam=1.5, grad_mode="field")
    assert rel_l2(gx, ref["gx"]) < RTOL and rel_l2(gy, ref["gy"]) < RTOL
    assert abs(out[1] - ref["wa"]) < RTOL * abs(ref["wa"])
