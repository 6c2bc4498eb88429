"""Seeded synthetic instances shaped like the paper's ISPD 2005 workloads.

The benchmark circuits the paper evaluates on (Section V, Table I) are not
available, so every instance here is drawn from a fixed recipe:

* site width = row height = 1; movable cells are one row high with an integer
  width drawn uniformly from 1..4 sites;
* the region is a square of side L = sqrt(A_mov / (util * (1 - f_mac))) with
  f_mac the fraction of the region covered by fixed macros;
* macro sides are drawn uniformly in [2%, 8%] of L per axis and then all
  scaled by one common factor so that the macros cover exactly f_mac of the
  region (they may overlap each other); macro centres are uniform such that
  each macro lies inside the region;
* movable cell centres are uniform in [w/2, L - w/2] x [h/2, L - h/2], drawn
  in float64 and stored as float32;
* a net of degree d connects d distinct movable cells drawn uniformly; each
  pin sits at the cell centre plus an offset uniform within the cell;
* the base degree mix is 2 (60%), 3 (20%) or uniform 4..8 (20%); a stated
  share of nets is replaced by "high-degree" nets of uniform degree in a
  stated range, interleaved at random positions in net order.

Nothing here computes densities, transforms or wirelengths.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, Optional, Tuple

import numpy as np


@dataclasses.dataclass
class Instance:
    """One placement instance in structure-of-arrays form.

    Grid: ``n`` x ``n`` bins over [xl, xl + n*bin_w] x [yl, yl + n*bin_h].
    Movable cells: centres ``x``, ``y`` and sizes ``w``, ``h`` (float32).
    Fixed macros: centres ``fx``, ``fy`` and sizes ``fw``, ``fh`` (float32).
    Nets: CSR ``net_ptr`` (int32, E+1) over pins ``pin_cell`` (int32) with
    offsets ``pin_dx``, ``pin_dy`` (float32) from the cell centre.
    ``gamma`` is the wirelength smoothing parameter in physical units.
    """

    n: int
    xl: float
    yl: float
    bin_w: float
    bin_h: float
    target_density: float
    x: np.ndarray
    y: np.ndarray
    w: np.ndarray
    h: np.ndarray
    fx: np.ndarray
    fy: np.ndarray
    fw: np.ndarray
    fh: np.ndarray
    net_ptr: np.ndarray
    pin_cell: np.ndarray
    pin_dx: np.ndarray
    pin_dy: np.ndarray
    gamma: float
    side: float
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def num_cells(self) -> int:
        return int(self.x.shape[0])

    @property
    def num_nets(self) -> int:
        return int(self.net_ptr.shape[0] - 1)

    @property
    def num_pins(self) -> int:
        return int(self.pin_cell.shape[0])

    @property
    def num_fixed(self) -> int:
        return int(self.fx.shape[0])

    def with_positions(self, x: np.ndarray, y: np.ndarray) -> "Instance":
        return dataclasses.replace(self, x=np.asarray(x, np.float32),
                                   y=np.asarray(y, np.float32))


def _degrees(rng: np.random.Generator, num_nets: int, hi_frac: float,
             hi_range: Tuple[int, int]) -> np.ndarray:
    n_hi = int(round(hi_frac * num_nets))
    n_base = num_nets - n_hi
    u = rng.random(n_base)
    deg = np.where(u < 0.6, 2, 3).astype(np.int64)
    tail = u >= 0.8
    deg[tail] = rng.integers(4, 9, size=int(tail.sum()))
    if n_hi:
        hi = rng.integers(hi_range[0], hi_range[1] + 1, size=n_hi)
        deg = np.concatenate([deg, hi])
    return deg[rng.permutation(num_nets)]


def _distinct_cells(rng: np.random.Generator, deg: np.ndarray, m: int) -> np.ndarray:
    """Uniform cells per net, redrawn until the cells of each net are distinct."""
    if deg.size and int(deg.max()) > m:
        raise ValueError("net degree exceeds the number of cells")
    num_pins = int(deg.sum())
    net_of_pin = np.repeat(np.arange(deg.size, dtype=np.int64), deg)
    cells = rng.integers(0, m, size=num_pins, dtype=np.int64)
    while num_pins:
        key = net_of_pin * m + cells
        order = np.argsort(key, kind="stable")
        sk = key[order]
        dup_sorted = np.zeros(num_pins, dtype=bool)
        dup_sorted[1:] = sk[1:] == sk[:-1]
        dup = np.zeros(num_pins, dtype=bool)
        dup[order[dup_sorted]] = True
        nd = int(dup.sum())
        if nd == 0:
            break
        cells[dup] = rng.integers(0, m, size=nd, dtype=np.int64)
    return cells.astype(np.int32)


def _macros(rng: np.random.Generator, num_macros: int, area_frac: float,
            side: float):
    if num_macros == 0 or area_frac <= 0.0:
        z = np.zeros(0, np.float32)
        return z, z.copy(), z.copy(), z.copy()
    sx = rng.uniform(0.02, 0.08, size=num_macros) * side
    sy = rng.uniform(0.02, 0.08, size=num_macros) * side
    scale = math.sqrt(area_frac * side * side / float(np.sum(sx * sy)))
    sx *= scale
    sy *= scale
    cx = sx / 2 + rng.random(num_macros) * (side - sx)
    cy = sy / 2 + rng.random(num_macros) * (side - sy)
    return (cx.astype(np.float32), cy.astype(np.float32),
            sx.astype(np.float32), sy.astype(np.float32))


def make_instance(seed, num_cells: int, util: float, n: int, num_nets: int,
                  hi_frac: float = 0.0, hi_range: Tuple[int, int] = (20, 200),
                  num_macros: int = 0, macro_area_frac: float = 0.0,
                  gamma_bins: float = 0.5, target_density: float = 1.0,
                  max_width: int = 4) -> Instance:
    """Draw one instance; ``seed`` may be an int or a sequence of ints."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    m = int(num_cells)
    w64 = rng.integers(1, max_width + 1, size=m).astype(np.float64)
    h64 = np.ones(m, np.float64)
    area = float(np.sum(w64 * h64))
    f_mac = macro_area_frac if num_macros > 0 else 0.0
    side = math.sqrt(area / (util * (1.0 - f_mac)))
    fx, fy, fw, fh = _macros(rng, num_macros, f_mac, side)
    x64 = w64 / 2 + rng.random(m) * (side - w64)
    y64 = h64 / 2 + rng.random(m) * (side - h64)
    deg = _degrees(rng, num_nets, hi_frac, hi_range)
    net_ptr = np.zeros(num_nets + 1, np.int64)
    np.cumsum(deg, out=net_ptr[1:])
    if net_ptr[-1] >= 2**31:
        raise ValueError("pin count exceeds int32")
    pin_cell = _distinct_cells(rng, deg, m)
    dx = (rng.random(pin_cell.size) - 0.5) * w64[pin_cell]
    dy = (rng.random(pin_cell.size) - 0.5) * h64[pin_cell]
    bin_w = side / n
    return Instance(
        n=int(n), xl=0.0, yl=0.0, bin_w=bin_w, bin_h=bin_w,
        target_density=float(target_density),
        x=x64.astype(np.float32), y=y64.astype(np.float32),
        w=w64.astype(np.float32), h=h64.astype(np.float32),
        fx=fx, fy=fy, fw=fw, fh=fh,
        net_ptr=net_ptr.astype(np.int32), pin_cell=pin_cell,
        pin_dx=dx.astype(np.float32), pin_dy=dy.astype(np.float32),
        gamma=float(gamma_bins * bin_w), side=side,
        meta=dict(seed=seed, util=util, hi_frac=hi_frac, hi_range=hi_range,
                  macro_area_frac=f_mac),
    )


# The five workloads.  Keys are short names; values are make_instance kwargs.
CONFIGS = {
    # one FP64 evaluation, seconds on a CPU
    "small_2k": dict(seed=1, num_cells=2_000, util=0.70, n=64, num_nets=2_200),
    # Nesterov driver workload
    "mid_200k": dict(seed=2, num_cells=200_000, util=0.80, n=512,
                     num_nets=210_000, hi_frac=0.01, hi_range=(20, 200),
                     num_macros=20, macro_area_frac=0.15),
    # precision / headline workload
    "large_2m": dict(seed=3, num_cells=2_100_000, util=0.90, n=1024,
                     num_nets=2_200_000, hi_frac=0.005, hi_range=(50, 1000),
                     num_macros=50, macro_area_frac=0.15),
    # differentiation workload
    "diff_500k": dict(seed=4, num_cells=500_000, util=0.80, n=512,
                      num_nets=525_000, hi_frac=0.01, hi_range=(20, 200),
                      num_macros=20, macro_area_frac=0.15),
}


def make_config(name: str, **overrides) -> Instance:
    kw = dict(CONFIGS[name])
    kw.update(overrides)
    return make_instance(**kw)


def serving_grid_size(m: int) -> int:
    """Grid side for a serving request: the smallest power of two not below
    sqrt(m), capped at 1024 (the recipe the serving workload is defined by)."""
    k = max(3, math.ceil(math.log2(math.sqrt(max(m, 1)))))
    return int(min(1024, 2 ** k))


def serving_requests(count: int = 5000, rate_hz: float = 200.0,
                     m_range: Tuple[float, float] = (1e4, 1e6),
                     seed: int = 5, materialize: bool = True
                     ) -> Iterator[Tuple[int, float, Optional[Instance], int, int]]:
    """Poisson stream of evaluation requests.

    Yields ``(r, arrival_s, instance_or_None, m, n)``; request ``r`` is drawn
    from seed ``(seed, r)``.  Cell counts are log-uniform over ``m_range``,
    nets number 1.1*m with the base degree mix, utilisation 0.7, no macros.
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed]))
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    logm = rng.uniform(math.log(m_range[0]), math.log(m_range[1]), size=count)
    for r in range(count):
        m = int(round(math.exp(logm[r])))
        n = serving_grid_size(m)
        inst = None
        if materialize:
            inst = make_instance((seed, r), num_cells=m, util=0.70, n=n,
                                 num_nets=int(round(1.1 * m)))
        yield r, float(arrivals[r]), inst, m, n


def serving_pool(size: int = 64, m_range: Tuple[float, float] = (1e4, 1e6),
                 seed: int = 5) -> list:
    """``size`` designs for the serving stream, cell counts log-uniform over
    ``m_range`` (design ``i`` drawn from seed ``(seed, 1, i)``), each with nets
    1.1*m of the base degree mix, utilisation 0.7, no macros and the grid side
    of ``serving_grid_size``."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0]))
    logm = rng.uniform(math.log(m_range[0]), math.log(m_range[1]), size=size)
    pool = []
    for i in range(size):
        m = int(round(math.exp(logm[i])))
        pool.append(make_instance((seed, 1, i), num_cells=m, util=0.70,
                                  n=serving_grid_size(m), num_nets=int(round(1.1 * m))))
    return pool


def serving_stream(count: int = 5000, rate_hz: float = 200.0, pool_size: int = 64,
                   seed: int = 5) -> Tuple[np.ndarray, np.ndarray]:
    """Poisson arrivals (exponential gaps of mean 1/rate_hz, first at 0) and,
    per request, the index of its design in a pool of ``pool_size``."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 2]))
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    design = rng.integers(0, pool_size, size=count)
    return arrivals, design
