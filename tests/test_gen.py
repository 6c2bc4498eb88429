"""The seeded instance recipe: determinism and the stated distributions."""
import numpy as np
import pytest

import gen


def test_deterministic_per_seed():
    a = gen.make_config("small_2k")
    b = gen.make_config("small_2k")
    for f in ("x", "y", "w", "net_ptr", "pin_cell", "pin_dx"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = gen.make_config("small_2k", seed=99)
    assert not np.array_equal(a.x, c.x)


def test_small_config_shape():
    inst = gen.make_config("small_2k")
    assert inst.num_cells == 2000 and inst.n == 64 and inst.num_nets == 2200
    assert set(np.unique(inst.w)) <= {1.0, 2.0, 3.0, 4.0} and np.all(inst.h == 1)
    util = float(np.sum(inst.w * inst.h)) / inst.side ** 2
    assert util == pytest.approx(0.70, rel=1e-9)
    assert np.all(inst.x - inst.w / 2 >= 0) and np.all(inst.x + inst.w / 2 <= inst.side * (1 + 1e-6))
    assert inst.gamma == pytest.approx(0.5 * inst.bin_w)


def test_degree_mix_and_distinct_pins():
    inst = gen.make_instance(7, num_cells=50_000, util=0.8, n=256, num_nets=60_000,
                             hi_frac=0.01, hi_range=(20, 200),
                             num_macros=20, macro_area_frac=0.15)
    deg = np.diff(inst.net_ptr)
    hi = deg >= 20
    assert abs(hi.mean() - 0.01) < 1e-3
    base = deg[~hi]
    assert abs((base == 2).mean() - 0.6) < 0.01 and abs((base == 3).mean() - 0.2) < 0.01
    assert base.max() == 8 and base.min() == 2
    for e in np.nonzero(hi)[0][:50]:
        cells = inst.pin_cell[inst.net_ptr[e]:inst.net_ptr[e + 1]]
        assert np.unique(cells).size == cells.size
    key = np.repeat(np.arange(inst.num_nets), deg).astype(np.int64) * inst.num_cells + inst.pin_cell
    assert np.unique(key).size == key.size
    # pin offsets lie within their cell
    assert np.all(np.abs(inst.pin_dx) <= inst.w[inst.pin_cell] / 2)
    assert np.all(np.abs(inst.pin_dy) <= inst.h[inst.pin_cell] / 2)
    # macros cover the stated fraction of the region and stay inside it
    area = float(np.sum(inst.fw.astype(float) * inst.fh))
    assert area == pytest.approx(0.15 * inst.side ** 2, rel=1e-5)
    assert np.all(inst.fx - inst.fw / 2 >= -1e-3) and np.all(inst.fx + inst.fw / 2 <= inst.side + 1e-3)


def test_serving_stream():
    reqs = list(gen.serving_requests(count=200, materialize=False))
    t = np.array([r[1] for r in reqs])
    assert t[0] == 0 and np.all(np.diff(t) >= 0)
    assert 0.6 < (t[-1] / 199) / 0.005 < 1.4
    for (_, _, _, m, n) in reqs:
        assert 1e4 <= m <= 1e6 and n in (128, 256, 512, 1024)
        assert n * n >= m or n == 1024
