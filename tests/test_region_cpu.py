"""Dark nodes of an irregular region (Section III-B): the host-only
fftpl_dark_nodes decomposition against exact brute force on compressed
coordinates (no GPU needed)."""
import ctypes

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def F():
    from paper_1312_4587_amd import fftpl, _lib
    _lib.load()
    return fftpl


def _inside_any(px, py, rects):
    return np.any((rects[:, 0] <= px) & (px < rects[:, 2]) & (rects[:, 1] <= py)
                  & (py < rects[:, 3]))


def _brute(bbox, placeable, dark):
    """On the grid of every x and y edge: each elementary cell must be
    covered exactly once by placeable-or-dark, and never by both."""
    xl, yl, xh, yh = bbox
    xs = np.unique(np.concatenate([[xl, xh], np.clip(placeable[:, [0, 2]].ravel(), xl, xh),
                                   dark[:, [0, 2]].ravel()]))
    ys = np.unique(np.concatenate([[yl, yh], np.clip(placeable[:, [1, 3]].ravel(), yl, yh),
                                   dark[:, [1, 3]].ravel()]))
    for i in range(len(xs) - 1):
        for j in range(len(ys) - 1):
            cx, cy = 0.5 * (xs[i] + xs[i + 1]), 0.5 * (ys[j] + ys[j + 1])
            p = _inside_any(cx, cy, placeable) if len(placeable) else False
            nd = int(np.sum((dark[:, 0] <= cx) & (cx < dark[:, 2]) & (dark[:, 1] <= cy)
                            & (cy < dark[:, 3]))) if len(dark) else 0
            assert nd == (0 if p else 1), (cx, cy, p, nd)


def test_l_shape_is_one_rectangle(F):
    d = F.dark_nodes(0, 0, 10, 10, [[0, 0, 10, 5], [0, 5, 5, 10]])
    assert d.tolist() == [[5.0, 5.0, 10.0, 10.0]]


def test_empty_and_full_regions(F):
    assert F.dark_nodes(0, 0, 4, 3, np.zeros((0, 4))).tolist() == [[0, 0, 4, 3]]
    assert len(F.dark_nodes(0, 0, 4, 3, [[-1, -1, 5, 5]])) == 0
    # a rectangle entirely outside R changes nothing
    assert F.dark_nodes(0, 0, 4, 3, [[10, 10, 12, 12]]).tolist() == [[0, 0, 4, 3]]


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_random_overlapping_rectangles_brute_force(F, seed):
    rng = np.random.default_rng(seed)
    k = 12
    x0 = rng.integers(-2, 18, k) * 0.5
    y0 = rng.integers(-2, 18, k) * 0.5
    r = np.stack([x0, y0, x0 + rng.integers(1, 8, k) * 0.5,
                  y0 + rng.integers(1, 8, k) * 0.5], axis=1)
    bbox = (0.0, 0.0, 8.0, 8.0)
    d = F.dark_nodes(*bbox, r)
    assert np.all(d[:, 2] > d[:, 0]) and np.all(d[:, 3] > d[:, 1])
    assert np.all(d[:, [0, 2]] >= 0) and np.all(d[:, [0, 2]] <= 8)
    _brute(bbox, r, d)


def test_rasterised_dark_plus_placeable_fills_every_bin(F):
    # disjoint placeable rectangles on a bin grid: the dark nodes' overlap
    # plus the placeable overlap is exactly one bin in every bin
    n, side = 16, 16.0
    placeable = np.array([[0, 0, 16, 4], [0, 4, 6.5, 11], [9.25, 4, 16, 16], [0, 11, 3, 16]])
    d = F.dark_nodes(0, 0, side, side, placeable)

    def cover(r):
        return oracle.rasterise(n, ((r[:, 0]).astype(np.float64), r[:, 2].astype(np.float64),
                                    r[:, 1].astype(np.float64), r[:, 3].astype(np.float64)))
    tot = cover(d) + cover(placeable)
    assert np.max(np.abs(tot - 1.0)) < 1e-12


def test_output_too_small_and_bad_arguments(F):
    from paper_1312_4587_amd import _lib
    lib = _lib.load()
    r = np.array([[0, 0, 1, 10], [2, 0, 3, 10], [4, 0, 5, 10]], np.float64)
    out = np.zeros((2, 4))
    cnt = ctypes.c_int32(0)
    st = lib.fftpl_dark_nodes(0.0, 0.0, 10.0, 10.0, 3, r.ctypes.data, 2, out.ctypes.data,
                              ctypes.byref(cnt))
    assert st == F.E_INVAL and cnt.value == 3
    assert len(F.dark_nodes(0, 0, 10, 10, r)) == 3
    bad = np.array([[1, 1, 0, 2]], np.float64)      # inverted
    assert lib.fftpl_dark_nodes(0.0, 0.0, 10.0, 10.0, 1, bad.ctypes.data, 4, out.ctypes.data,
                                ctypes.byref(cnt)) == F.E_INVAL
    assert lib.fftpl_dark_nodes(0.0, 0.0, 0.0, 10.0, 0, None, 4, out.ctypes.data,
                                ctypes.byref(cnt)) == F.E_INVAL
    nanr = np.array([[0, 0, np.nan, 1]], np.float64)
    assert lib.fftpl_dark_nodes(0.0, 0.0, 10.0, 10.0, 1, nanr.ctypes.data, 4,
                                out.ctypes.data, ctypes.byref(cnt)) == F.E_INVAL
