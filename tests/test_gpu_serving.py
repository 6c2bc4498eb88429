"""Serving form on the GPU: a burst-heavy Poisson stream of mixed-size
designs served by several slots at once; 50 sampled requests give the same
results alone as in the mix, and three are checked against the FP64 oracle."""
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


def test_alone_equals_mix(S):
    pool = gen.serving_pool(12, m_range=(1e4, 2e5), seed=11)
    arrivals, designs = gen.serving_stream(300, rate_hz=3000.0, pool_size=len(pool), seed=11)
    keep = sorted(np.random.default_rng(12).choice(300, 50, replace=False).tolist())
    ex = S.DeviceExecutor(pool, slots=4)
    ex.warm()
    srv = S.Server(ex, ex.footprint, slots=4, capacity_bytes=200e9, keep=keep)
    st = srv.run(arrivals, designs)
    say("mix", st)
    assert st["requests"] == 300
    assert st["max_in_service"] >= 2          # requests really overlapped
    for rid in keep:
        mix = srv.results[rid]
        out4, gx, gy = ex(0, rid, mix.design)  # the same request alone
        e = rel_l2(np.concatenate([mix.gx, mix.gy]), np.concatenate([gx, gy]))
        assert e <= RTOL, (rid, e)
        assert np.all(np.abs(mix.out4 - out4) <= RTOL * np.abs(out4) + 1e-12), rid
    # and a few designs against the oracle
    for d in sorted({srv.results[r].design for r in keep})[:3]:
        rid = next(r for r in keep if srv.results[r].design == d)
        ref = oracle.evaluate(pool[d], lam=1.0, grad_mode="field")
        mix = srv.results[rid]
        e = rel_l2(np.concatenate([mix.gx, mix.gy]), np.concatenate([ref["gx"], ref["gy"]]))
        say("design", d, pool[d].num_cells, "vs oracle", e)
        assert e < RTOL
        assert abs(mix.out4[1] - ref["wa"]) <= RTOL * abs(ref["wa"])
    ex.close()
