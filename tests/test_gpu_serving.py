"""Serving form on the GPU: a burst-heavy Poisson stream of placements of
mixed-size designs served by several slots at once, grouped by grid side
into batched evaluations; 50 sampled requests give the same results alone as
in the mix, three are checked against the FP64 oracle, and a malformed
request fails alone."""
import numpy as np
import pytest

import gen
import oracle
from _helpers import rel_l2
from tests.gpu_common import RTOL, lib_or_build, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_or_build()
    from paper_1312_4587_amd import serving
    return serving


@pytest.mark.parametrize("max_batch", [1, 4])
def test_alone_equals_mix(S, max_batch):
    pool = gen.serving_pool(12, m_range=(1e4, 2e5), seed=11)
    arrivals, designs = gen.serving_stream(300, rate_hz=3000.0, pool_size=len(pool), seed=11)
    variants = np.arange(300) % 3
    keep = sorted(np.random.default_rng(12).choice(300, 50, replace=False).tolist())
    ex = S.DeviceExecutor(pool, slots=4, max_batch=max_batch, variants=3)
    ex.warm()
    srv = S.Server(ex, ex.footprint, slots=4, capacity_bytes=200e9, keep=keep, grid=ex.grid,
                   max_batch=max_batch)
    st = srv.run(arrivals, designs, variants)
    say("mix", max_batch, st)
    assert st["requests"] == 300 and st["served"] == 300 and st["errors"] == 0
    assert st["max_in_service"] >= 2          # requests really overlapped
    if max_batch > 1:
        assert st["max_batch_seen"] >= 2      # and were evaluated in groups
    for rid in keep:
        mix = srv.results[rid]
        one = ex(0, [S.Request(rid, mix.design, mix.variant)])[0]   # the same request alone
        assert one.ok
        # the grouped and the single evaluation run the same kernels on the
        # same inputs: the same bits
        assert np.array_equal(mix.gx, one.gx) and np.array_equal(mix.gy, one.gy), rid
        assert np.all(np.abs(mix.out4 - one.out4) <= 1e-12 * np.abs(one.out4)), rid
    # and a few designs against the oracle
    for d in sorted({srv.results[r].design for r in keep})[:3]:
        rid = next(r for r in keep if srv.results[r].design == d)
        mix = srv.results[rid]
        x, y = ex.positions(d, mix.variant)
        ref = oracle.evaluate(pool[d].with_positions(x, y), lam=1.0, grad_mode="field")
        e = rel_l2(np.concatenate([mix.gx, mix.gy]), np.concatenate([ref["gx"], ref["gy"]]))
        say("design", d, pool[d].num_cells, "vs oracle", e)
        assert e < RTOL
        assert abs(mix.out4[1] - ref["wa"]) <= RTOL * abs(ref["wa"])
    ex.close()


def test_malformed_request_fails_alone(S):
    # a group holding a request whose design carries a malformed netlist (a
    # pin on a cell that does not exist): the index build refuses it, that
    # request fails, the rest of the stream is served
    pool = gen.serving_pool(4, m_range=(1e4, 3e4), seed=13)
    bad = pool[2]
    bad.pin_cell[5] = bad.num_cells + 3
    ex = S.DeviceExecutor(pool, slots=2, max_batch=4, variants=1)
    ex.warm()
    srv = S.Server(ex, ex.footprint, slots=2, capacity_bytes=200e9, grid=ex.grid, max_batch=4)
    designs = np.array([0, 1, 2, 3] * 10)
    st = srv.run(np.zeros(40), designs)
    say("with a malformed design", st)
    assert st["errors"] == 10 and st["served"] == 30
    assert all(not srv.results[r].ok for r in range(40) if designs[r] == 2)
    assert all(srv.results[r].ok for r in range(40) if designs[r] != 2)
    assert srv.admitted_bytes == 0 and srv.in_service == 0
    ex.close()
