"""Pins of the oracle's cell-to-bin rule and density map (Section II,
Eq. (2); Section III-B) against brute force, closed forms and a hand-computed
fixture."""
import numpy as np
import pytest

import oracle
from _helpers import hand_instance, load_golden_density, tiny_instance, with_macros


def _step_by_step_f32(origin, bin_size, centre, size):
    # Each float32 operation done in float64 (exact for these operands) and
    # rounded once to float32: an independent statement of IEEE single ops.
    inv = np.float32(1.0 / bin_size)
    o = np.float32(origin)
    out_lo, out_hi = [], []
    for c, s in zip(np.asarray(centre, np.float32), np.asarray(size, np.float32)):
        d = np.float32(float(c) - float(o))
        cc = np.float32(float(d) * float(inv))
        ws = np.float32(float(s) * float(inv))
        half = np.float32(0.5 * float(ws))
        out_lo.append(np.float32(float(cc) - float(half)))
        out_hi.append(np.float32(float(cc) + float(half)))
    return np.array(out_lo, np.float32), np.array(out_hi, np.float32)


def test_rect_rule_is_ieee_single_step_by_step():
    rng = np.random.default_rng(7)
    for origin, bsz in [(0.0, 1.3314690044538884), (-3.25, 2.558), (10.0, 0.7)]:
        c = (origin + rng.random(500) * 1000).astype(np.float32)
        s = rng.integers(1, 5, 500).astype(np.float32)
        lo, hi = oracle.cell_rect_f32(origin, bsz, c, s)
        lo2, hi2 = _step_by_step_f32(origin, bsz, c, s)
        assert np.array_equal(lo.view(np.uint32), lo2.view(np.uint32))
        assert np.array_equal(hi.view(np.uint32), hi2.view(np.uint32))


def _brute_range(lo, hi, n):
    # every bin with positive overlap, scanned one by one
    js = [j for j in range(n)
          if min(min(float(hi), n), j + 1) - max(max(float(lo), 0.0), j) > 0.0]
    return (js[0], js[-1]) if js else None


@pytest.mark.parametrize("n", [1, 4, 16, 64])
def test_bin_range_matches_brute_force(n):
    rng = np.random.default_rng(n)
    lo = (rng.random(2000) * (n + 4) - 2).astype(np.float32)
    hi = (lo + rng.random(2000) * 4).astype(np.float32)
    i0, i1 = oracle.bin_range(lo, hi, n)
    for k in range(lo.size):
        b = _brute_range(lo[k], hi[k], n)
        if b is None:
            assert i0[k] > i1[k]
        else:
            assert (i0[k], i1[k]) == b


def test_bin_range_on_lines_and_neighbours():
    n = 8
    vals = []
    for j in range(0, n + 1):
        f = np.float32(j)
        vals += [f, np.nextafter(f, np.float32(-1)), np.nextafter(f, np.float32(100))]
    vals = np.array(vals, np.float32)
    lo, hi = np.meshgrid(vals, vals)
    lo, hi = lo.ravel(), hi.ravel()
    keep = hi > lo
    lo, hi = lo[keep], hi[keep]
    i0, i1 = oracle.bin_range(lo, hi, n)
    for k in range(lo.size):
        b = _brute_range(lo[k], hi[k], n)
        if b is None:
            assert i0[k] > i1[k]
        else:
            assert (i0[k], i1[k]) == b
    # a left edge exactly on line j starts in bin j; a right edge exactly on
    # line j+1 ends in bin j (half-open bins)
    i0, i1 = oracle.bin_range(np.float32([2.0]), np.float32([5.0]), n)
    assert (i0[0], i1[0]) == (2, 4)


def test_golden_tiny_density():
    cells, expect = load_golden_density()
    inst = hand_instance(cells, n=4)
    rho = oracle.density_map(inst)
    assert np.array_equal(rho, expect)


def test_area_conservation_and_clipping():
    inst = tiny_instance(seed=3, m=300, n=32)
    rho = oracle.density_map(inst)
    xlo, xhi = oracle.cell_rect_f32(inst.xl, inst.bin_w, inst.x, inst.w)
    ylo, yhi = oracle.cell_rect_f32(inst.yl, inst.bin_h, inst.y, inst.h)
    n = inst.n
    area = np.sum((np.clip(xhi.astype(float), 0, n) - np.clip(xlo.astype(float), 0, n))
                  * (np.clip(yhi.astype(float), 0, n) - np.clip(ylo.astype(float), 0, n)))
    assert abs(rho.sum() - area) < 1e-9 * area
    # a cell sticking out of the region keeps only its in-region area
    inst2 = hand_instance([[0.25, 2.0, 1.5, 1.0]], n=4)
    r2 = oracle.density_map(inst2)
    assert r2.sum() == pytest.approx(1.0)          # [-0.5,1.0)x[1.5,2.5) -> 1.0 x 1.0
    assert r2[1, 0] == 0.5 and r2[2, 0] == 0.5


def test_aligned_unit_cell_and_full_cover():
    n = 8
    for (j, k) in [(0, 0), (3, 5), (7, 7)]:
        inst = hand_instance([[j + 0.5, k + 0.5, 1.0, 1.0]], n=n)
        rho = oracle.density_map(inst)
        e = np.zeros((n, n))
        e[k, j] = 1.0
        assert np.array_equal(rho, e)
    inst = hand_instance([[4.0, 4.0, 8.0, 8.0]], n=n)
    assert np.array_equal(oracle.density_map(inst), np.ones((n, n)))


def test_fixed_maps_scaled_and_capacity():
    n = 8
    base_inst = hand_instance([[1.0, 1.0, 1.0, 1.0]], n=n)
    # two overlapping macros over bins; second overlaps the first by a bin
    inst = with_macros(base_inst, [[2.0, 2.0, 2.0, 2.0], [3.0, 2.0, 2.0, 2.0]])
    inst.target_density = 0.8
    base, cap = oracle.fixed_maps(inst)
    f = np.zeros((n, n))
    f[1:3, 1:3] += 1.0
    f[1:3, 2:4] += 1.0
    assert np.allclose(base, 0.8 * f)
    assert np.allclose(cap, 0.8 * np.maximum(0, 1 - np.minimum(1, f)))
    assert cap[1, 1] == 0.0 and cap[1, 2] == 0.0 and cap[0, 0] == pytest.approx(0.8)
    assert base[1, 2] == pytest.approx(1.6)
