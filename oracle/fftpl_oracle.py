"""Plain, slow FP64 reference of one FFTPL evaluation (objective + gradient).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Paper: J. Lu et al., "FFTPL: An Analytic Placement Algorithm Using Fast
Fourier Transform for Density Equalization".  Each function names the
passage it follows.  Everything is float64 except the cell-to-bin rectangle
rule, which the paper leaves unspecified and which decides integers (the bin
index sets); it is evaluated in float32, step by step, exactly as stated in
``cell_rect_f32``.

Readings of points the paper leaves open or prints ambiguously:

* Eq. (10) prints a 1/(2n) factor; that factor does not invert Eq. (9).  The
  coefficients here are the exact inverse of Eq. (9):
  a_uv = (c_u c_v / n^2) sum rho cos cos with c_0 = 1 and c_{k>0} = 2.
* The mirrored, periodically extended domain of Section III-E is sampled at
  bin centres x = i + 1/2 (the half-sample even extension), u, v in [0, n).
* Work is in bin units: a bin is the unit square [j, j+1) x [k, k+1), w_u =
  pi*u/n, densities are cell area per bin area, gradients are converted to
  physical units by 1/bin_w and 1/bin_h.
* The DC term is removed (Section III-A): a_00 := 0.
* The field-form density gradient of Section III-C is dN/dx ~ -q E with the
  per-cell field taken as the overlap-weighted sum of E over the bins the
  cell covers; E = -grad(psi) is exactly what Eq. (12) gives from Eq. (11).
  The exact derivative of N (Eq. (6)) is provided too; it carries the factor
  2 of a quadratic form.
* The weighted-average wirelength of Eq. (3) is evaluated with max/min
  shifted exponentials (identical in exact arithmetic).
* The screened (Helmholtz) equation that Section II cites as Eq. (4) is
  taken with the sign convention of Eq. (8), -laplace(psi) + eps psi =
  rho - mean, so each cosine mode divides by w_u^2 + w_v^2 + eps; eps = 0
  is Eq. (8) itself.
* The log-sum-exp wirelength that Section II names beside Eq. (3) is not
  printed; it is taken in its usual form gamma ln sum exp(X/gamma) + gamma
  ln sum exp(-X/gamma) per net and axis.
* Overflow (the stopping criterion of Section IV-A, defined only by
  reference to NTUplace3): tau = sum_b max(0, rho_mov,b - cap_b) /
  sum_b rho_mov,b with cap_b = rho_t * max(0, 1 - min(1, f_b)) and f_b the
  summed fixed-macro overlap of bin b.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

__all__ = [
    "cell_rect_f32", "bin_range", "overlaps_1d", "rasterise",
    "fixed_maps", "density_map", "cos_table", "sin_table",
    "dct_coefficients", "dct_coefficients_literal", "remove_dc",
    "spectral_potential", "potential_field", "poisson_solve", "energy",
    "field_gradient", "exact_gradient", "wa_wirelength", "lse_wirelength",
    "hpwl", "net_values",
    "overflow", "evaluate", "local_fd_gradient", "potential_differences",
]


# ---------------------------------------------------------------------------
# Cells on the bin grid (Section II: the region is cut into n x n bins and
# the bin density is cell area over bin area; Eq. (2)).
# ---------------------------------------------------------------------------

def cell_rect_f32(origin: float, bin_size: float, centre, size
                  ) -> Tuple[np.ndarray, np.ndarray]:
    """Cell edges in bin units, in float32 with one rounding per operation.

        c    = (centre - fl32(origin)) * fl32(1 / bin_size)
        half = 0.5 * (size * fl32(1 / bin_size))
        lo, hi = c - half, c + half

    The grid maps positions to bins without saying in which precision; this
    float32 rule is the definition both sides share, so that the index sets
    it decides are unique.
    """
    inv = np.float32(1.0 / float(bin_size))
    o = np.float32(origin)
    c = (np.asarray(centre, dtype=np.float32) - o) * inv
    half = np.float32(0.5) * (np.asarray(size, dtype=np.float32) * inv)
    return (c - half).astype(np.float32), (c + half).astype(np.float32)


def bin_range(lo: np.ndarray, hi: np.ndarray, n: int
              ) -> Tuple[np.ndarray, np.ndarray]:
    """Half-open bins [j, j+1): the first and last bin a rectangle [lo, hi)
    touches, clipped to [0, n-1]; empty when first > last."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    i0 = np.floor(np.clip(lo, 0.0, n)).astype(np.int64)
    i1 = np.ceil(np.clip(hi, -1.0, n)).astype(np.int64) - 1
    return i0, i1


def overlaps_1d(lo: np.ndarray, hi: np.ndarray, n: int):
    """Per-cell 1-D overlaps with the bins of its range (Eq. (2) density).

    Returns (i0, span, ov) with ov[i, k] = length of [lo, hi) intersected
    with the bin i0+k and with [0, n], zero for k >= span.
    """
    i0, i1 = bin_range(lo, hi, n)
    span = np.maximum(i1 - i0 + 1, 0)
    kmax = int(span.max()) if span.size else 0
    lo64 = np.clip(np.asarray(lo, np.float64), 0.0, n)
    hi64 = np.clip(np.asarray(hi, np.float64), 0.0, n)
    ov = np.zeros((lo64.size, max(kmax, 1)))
    for k in range(kmax):
        j = (i0 + k).astype(np.float64)
        o = np.minimum(hi64, j + 1.0) - np.maximum(lo64, j)
        ov[:, k] = np.where(k < span, np.maximum(o, 0.0), 0.0)
    return i0, span, ov


def rasterise(n: int, rects, weight=None) -> np.ndarray:
    """Sum over cells of weight * (x-overlap) * (y-overlap) per bin."""
    (xlo, xhi, ylo, yhi) = rects
    rho = np.zeros((n, n))
    if len(xlo) == 0:
        return rho
    ix0, sx, ox = overlaps_1d(xlo, xhi, n)
    iy0, sy, oy = overlaps_1d(ylo, yhi, n)
    wgt = np.ones(len(xlo)) if weight is None else np.asarray(weight, np.float64)
    for ky in range(oy.shape[1]):
        for kx in range(ox.shape[1]):
            sel = (kx < sx) & (ky < sy)
            if not np.any(sel):
                continue
            np.add.at(rho, (iy0[sel] + ky, ix0[sel] + kx),
                      (wgt * ox[:, kx] * oy[:, ky])[sel])
    return rho


def _rects(inst, fixed: bool = False):
    if fixed:
        cx, cy, sw, sh = inst.fx, inst.fy, inst.fw, inst.fh
    else:
        cx, cy, sw, sh = inst.x, inst.y, inst.w, inst.h
    xlo, xhi = cell_rect_f32(inst.xl, inst.bin_w, cx, sw)
    ylo, yhi = cell_rect_f32(inst.yl, inst.bin_h, cy, sh)
    return xlo, xhi, ylo, yhi


def fixed_maps(inst) -> Tuple[np.ndarray, np.ndarray]:
    """Fixed charge and the capacity left for movable cells.

    Fixed (and dark) node areas are scaled by the target density
    (Section III-B): base = rho_t * f_b with f_b the summed macro overlap.
    cap_b = rho_t * max(0, 1 - min(1, f_b)) is what movable cells may fill.
    """
    f = rasterise(inst.n, _rects(inst, fixed=True))
    rt = float(inst.target_density)
    return rt * f, rt * np.maximum(0.0, 1.0 - np.minimum(1.0, f))


def density_map(inst, base=None) -> np.ndarray:
    """rho = base + movable cell area per bin (Eq. (2); Section III-B)."""
    rho = rasterise(inst.n, _rects(inst))
    if base is not None:
        rho = rho + base
    return rho


# ---------------------------------------------------------------------------
# Spectral Poisson solve (Section III-D, III-E; Eqs. (8)-(12)).
# ---------------------------------------------------------------------------

def cos_table(n: int) -> np.ndarray:
    """K[u, i] = cos(w_u (i + 1/2)), w_u = pi u / n, argument reduced exactly
    as pi * ((u (2i+1)) mod 4n) / (2n)."""
    u = np.arange(n, dtype=np.int64)[:, None]
    i = np.arange(n, dtype=np.int64)[None, :]
    return np.cos(np.pi * ((u * (2 * i + 1)) % (4 * n)) / (2.0 * n))


def sin_table(n: int) -> np.ndarray:
    """S[u, i] = sin(w_u (i + 1/2)), reduced like ``cos_table``."""
    u = np.arange(n, dtype=np.int64)[:, None]
    i = np.arange(n, dtype=np.int64)[None, :]
    return np.sin(np.pi * ((u * (2 * i + 1)) % (4 * n)) / (2.0 * n))


def _cweights(n: int) -> np.ndarray:
    c = np.full(n, 2.0)
    c[0] = 1.0
    return c


def dct_coefficients(rho: np.ndarray) -> np.ndarray:
    """Eq. (10) with the normalisation that inverts Eq. (9):

        a[v, u] = c_u c_v / n^2 * sum_{iy, ix} rho[iy, ix]
                  cos(w_v (iy + 1/2)) cos(w_u (ix + 1/2))

    as two direct matrix products with exact cosine tables (no FFT).
    ``rho`` is indexed [iy, ix]; ``a`` is indexed [v, u].
    """
    n = rho.shape[0]
    K = cos_table(n)
    c = _cweights(n)
    return (np.outer(c, c) / (n * n)) * (K @ np.asarray(rho, np.float64) @ K.T)


def dct_coefficients_literal(rho: np.ndarray) -> np.ndarray:
    """The same coefficients as a literal quadruple sum with direct cosine
    calls; O(n^4), for tiny grids only."""
    n = rho.shape[0]
    a = np.zeros((n, n))
    for v in range(n):
        for u in range(n):
            s = 0.0
            for iy in range(n):
                cy = math.cos(math.pi * v * (iy + 0.5) / n)
                for ix in range(n):
                    s += rho[iy, ix] * math.cos(math.pi * u * (ix + 0.5) / n) * cy
            cu = 1.0 if u == 0 else 2.0
            cv = 1.0 if v == 0 else 2.0
            a[v, u] = cu * cv / (n * n) * s
    return a


def remove_dc(a: np.ndarray) -> np.ndarray:
    """Section III-A: the DC component is removed so that under-filled
    regions carry negative charge; also the zero-integral condition of
    Eq. (8)."""
    a = np.array(a, dtype=np.float64, copy=True)
    a[0, 0] = 0.0
    return a


def spectral_potential(a: np.ndarray, eps: float = 0.0):
    """G = a / (w_u^2 + w_v^2 + eps) and its frequency-weighted copies
    Gx = w_u G, Gy = w_v G (the coefficients of Eqs. (11) and (12)), with
    the (0, 0) entry zero.

    eps = 0 is the paper's Poisson equation (8).  eps > 0 is the screened
    (Helmholtz) form of Eq. (4), taken with the sign convention of Eq. (8):
    -laplace(psi) + eps psi = rho - mean, whose cosine modes divide by
    w_u^2 + w_v^2 + eps (eps in bin^-2, like w_u^2).  The DC is still
    removed first, so the (0, 0) mode stays zero."""
    n = a.shape[0]
    wfreq = np.pi * np.arange(n) / n
    denom = wfreq[:, None] ** 2 + wfreq[None, :] ** 2 + float(eps)   # [v, u]
    denom[0, 0] = 1.0
    G = np.asarray(a, np.float64) / denom
    G[0, 0] = 0.0
    return G, G * wfreq[None, :], G * wfreq[:, None]


def potential_field(a: np.ndarray, eps: float = 0.0):
    """Eqs. (11) and (12) at the bin centres, by direct sums:

        psi[iy, ix] = sum_{v,u} G[v,u]   cos(w_v y) cos(w_u x)
        Ex [iy, ix] = sum_{v,u} Gx[v,u]  cos(w_v y) sin(w_u x)
        Ey [iy, ix] = sum_{v,u} Gy[v,u]  sin(w_v y) cos(w_u x)
    """
    n = a.shape[0]
    K = cos_table(n)
    S = sin_table(n)
    G, Gx, Gy = spectral_potential(a, eps)
    psi = K.T @ G @ K
    ex = K.T @ Gx @ S
    ey = S.T @ Gy @ K
    return psi, ex, ey


def poisson_solve(rho: np.ndarray, eps: float = 0.0):
    """Neumann Poisson solve of Eq. (8) through Eqs. (9)-(12) (or, with
    eps > 0, the screened form of Eq. (4), see ``spectral_potential``):
    returns (psi, Ex, Ey, a) with a the DC-free coefficients."""
    a = remove_dc(dct_coefficients(rho))
    psi, ex, ey = potential_field(a, eps)
    return psi, ex, ey, a


def potential_differences(psi: np.ndarray):
    """Differences of psi to the next bin centre, Dx[iy, ix] = psi[iy, ix+1]
    - psi[iy, ix] and Dy[iy, ix] = psi[iy+1, ix] - psi[iy, ix] (the terms the
    exact gradient of Section III-C sums).  The mirror of Section III-E makes
    the potential at the next centre past the border equal to the last one,
    so the last column of Dx and the last row of Dy are zero."""
    psi = np.asarray(psi, np.float64)
    dx = np.zeros_like(psi)
    dy = np.zeros_like(psi)
    dx[:, :-1] = psi[:, 1:] - psi[:, :-1]
    dy[:-1, :] = psi[1:, :] - psi[:-1, :]
    return dx, dy


def energy(rho: np.ndarray, psi: np.ndarray) -> float:
    """Eq. (6) on the bin grid: N = sum_b rho_b psi_b (all charges,
    fixed ones included, each bin's charge times its potential)."""
    return float(np.sum(np.asarray(rho, np.float64) * psi))


# ---------------------------------------------------------------------------
# Density gradients (Section III-C).
# ---------------------------------------------------------------------------

def field_gradient(inst, ex: np.ndarray, ey: np.ndarray):
    """Field form of the density gradient, dN/dx_i ~ -q_i E_i:

        gx_i = -(1 / bin_w) sum_b ov(i, b) Ex_b,  gy_i likewise with Ey, bin_h

    with ov the overlap area (bin units) of cell i with bin b."""
    n = inst.n
    xlo, xhi, ylo, yhi = _rects(inst)
    ix0, sx, ox = overlaps_1d(xlo, xhi, n)
    iy0, sy, oy = overlaps_1d(ylo, yhi, n)
    gx = np.zeros(len(xlo))
    gy = np.zeros(len(xlo))
    for ky in range(oy.shape[1]):
        for kx in range(ox.shape[1]):
            sel = (kx < sx) & (ky < sy)
            iy = np.where(sel, iy0 + ky, 0)
            ix = np.where(sel, ix0 + kx, 0)
            wgt = np.where(sel, ox[:, kx] * oy[:, ky], 0.0)
            gx += wgt * ex[iy, ix]
            gy += wgt * ey[iy, ix]
    return -gx / inst.bin_w, -gy / inst.bin_h


def exact_gradient(inst, psi: np.ndarray):
    """Exact derivative of N = rho^T M rho (Eq. (6), M symmetric) with
    respect to the movable cell centres.

    Moving a cell right by dx in bin units adds dx of overlap in the bin
    holding its right edge and removes dx in the bin holding its left edge
    (edges strictly inside (0, n) only), so

        dN/dx_i = (2 / bin_w) sum_iy oy(i, iy)
                  [psi(iy, floor(hi)) - psi(iy, floor(lo))]
    """
    n = inst.n
    xlo, xhi, ylo, yhi = _rects(inst)
    iy0, sy, oy = overlaps_1d(ylo, yhi, n)
    ix0, sx, ox = overlaps_1d(xlo, xhi, n)

    def edge_terms(lo, hi, o0, so, oo, p):
        # p is psi arranged so that p[k, j] is (row k of the other axis, col j)
        g = np.zeros(len(lo))
        lo64 = np.asarray(lo, np.float64)
        hi64 = np.asarray(hi, np.float64)
        in_r = (hi64 > 0) & (hi64 < n)
        in_l = (lo64 > 0) & (lo64 < n)
        cr = np.where(in_r, np.floor(hi64), 0).astype(np.int64)
        cl = np.where(in_l, np.floor(lo64), 0).astype(np.int64)
        for k in range(oo.shape[1]):
            sel = k < so
            row = np.where(sel, o0 + k, 0)
            wgt = np.where(sel, oo[:, k], 0.0)
            g += wgt * (np.where(in_r, p[row, cr], 0.0) - np.where(in_l, p[row, cl], 0.0))
        return g

    gx = edge_terms(xlo, xhi, iy0, sy, oy, psi)        # rows iy, cols ix
    gy = edge_terms(ylo, yhi, ix0, sx, ox, psi.T)      # rows ix, cols iy
    return 2.0 * gx / inst.bin_w, 2.0 * gy / inst.bin_h


# ---------------------------------------------------------------------------
# Wirelength (Eqs. (1) and (3)).
# ---------------------------------------------------------------------------

def _segments(net_ptr):
    net_ptr = np.asarray(net_ptr, np.int64)
    deg = np.diff(net_ptr)
    nonempty = np.nonzero(deg > 0)[0]
    return net_ptr, deg, nonempty


def _wa_axis(pos: np.ndarray, net_ptr, gamma: float):
    """One axis of Eq. (3) for every net: returns (W~ per net, gradient per
    pin, max per net, min per net) over non-empty nets."""
    net_ptr, deg, ne = _segments(net_ptr)
    starts = net_ptr[:-1][ne]
    if starts.size == 0:
        return (np.zeros(0), np.zeros(pos.size), np.zeros(0), np.zeros(0))
    M = np.maximum.reduceat(pos, starts)
    L = np.minimum.reduceat(pos, starts)
    seg = np.repeat(np.arange(starts.size), deg[ne])
    ep = np.exp((pos - M[seg]) / gamma)
    em = np.exp((L[seg] - pos) / gamma)
    sp = np.add.reduceat(ep, starts)
    sm = np.add.reduceat(em, starts)
    wp = M + np.add.reduceat((pos - M[seg]) * ep, starts) / sp
    wm = L + np.add.reduceat((pos - L[seg]) * em, starts) / sm
    # dW+/dX_p = e+_p/S+ (1 + (X_p - W+)/gamma); dW-/dX_p = e-_p/S- (1 - (X_p - W-)/gamma)
    grad = (ep / sp[seg]) * (1.0 + (pos - wp[seg]) / gamma) \
        - (em / sm[seg]) * (1.0 - (pos - wm[seg]) / gamma)
    return wp - wm, grad, M, L


def wa_wirelength(inst, x=None, y=None, gamma=None):
    """Weighted-average wirelength (Eq. (3)) over both axes, FP64.

    Pins sit at cell centre + offset.  Returns (W~, gx, gy) with gx, gy the
    gradient summed over each cell's pins (physical units)."""
    x = inst.x if x is None else x
    y = inst.y if y is None else y
    gamma = inst.gamma if gamma is None else gamma
    pc = np.asarray(inst.pin_cell, np.int64)
    px = np.asarray(x, np.float64)[pc] + np.asarray(inst.pin_dx, np.float64)
    py = np.asarray(y, np.float64)[pc] + np.asarray(inst.pin_dy, np.float64)
    m = len(x)
    wx, gpx, _, _ = _wa_axis(px, inst.net_ptr, float(gamma))
    wy, gpy, _, _ = _wa_axis(py, inst.net_ptr, float(gamma))
    gx = np.bincount(pc, weights=gpx, minlength=m) if pc.size else np.zeros(m)
    gy = np.bincount(pc, weights=gpy, minlength=m) if pc.size else np.zeros(m)
    return float(np.sum(wx) + np.sum(wy)), gx, gy


def _lse_axis(pos: np.ndarray, net_ptr, gamma: float):
    """One axis of the log-sum-exp model (Section II) for every net:
    LSE = gamma ln sum exp(X/gamma) + gamma ln sum exp(-X/gamma), evaluated
    as (M - L) + gamma (ln S+ + ln S-) with S+ = sum exp((X - M)/gamma) and
    S- = sum exp((L - X)/gamma) (the same value: the shifts cancel); the
    gradient is the difference of the two softmax weights, e+/S+ - e-/S-.
    Returns (LSE per net, gradient per pin) over non-empty nets."""
    net_ptr, deg, ne = _segments(net_ptr)
    starts = net_ptr[:-1][ne]
    if starts.size == 0:
        return np.zeros(0), np.zeros(pos.size)
    M = np.maximum.reduceat(pos, starts)
    L = np.minimum.reduceat(pos, starts)
    seg = np.repeat(np.arange(starts.size), deg[ne])
    ep = np.exp((pos - M[seg]) / gamma)
    em = np.exp((L[seg] - pos) / gamma)
    sp = np.add.reduceat(ep, starts)
    sm = np.add.reduceat(em, starts)
    val = (M - L) + gamma * (np.log(sp) + np.log(sm))
    return val, ep / sp[seg] - em / sm[seg]


def lse_wirelength(inst, x=None, y=None, gamma=None):
    """Log-sum-exp wirelength (the smooth model Section II sets beside
    Eq. (3)) over both axes, FP64: returns (LSE, gx, gy) like
    ``wa_wirelength``."""
    x = inst.x if x is None else x
    y = inst.y if y is None else y
    gamma = inst.gamma if gamma is None else gamma
    pc = np.asarray(inst.pin_cell, np.int64)
    px = np.asarray(x, np.float64)[pc] + np.asarray(inst.pin_dx, np.float64)
    py = np.asarray(y, np.float64)[pc] + np.asarray(inst.pin_dy, np.float64)
    m = len(x)
    vx, gpx = _lse_axis(px, inst.net_ptr, float(gamma))
    vy, gpy = _lse_axis(py, inst.net_ptr, float(gamma))
    gx = np.bincount(pc, weights=gpx, minlength=m) if pc.size else np.zeros(m)
    gy = np.bincount(pc, weights=gpy, minlength=m) if pc.size else np.zeros(m)
    return float(np.sum(vx) + np.sum(vy)), gx, gy


def hpwl(inst, x=None, y=None) -> float:
    """Eq. (1): sum over nets of (max - min) of pin x plus the same in y."""
    x = inst.x if x is None else x
    y = inst.y if y is None else y
    pc = np.asarray(inst.pin_cell, np.int64)
    net_ptr, deg, ne = _segments(inst.net_ptr)
    starts = net_ptr[:-1][ne]
    if starts.size == 0:
        return 0.0
    tot = 0.0
    for pos in (np.asarray(x, np.float64)[pc] + np.asarray(inst.pin_dx, np.float64),
                np.asarray(y, np.float64)[pc] + np.asarray(inst.pin_dy, np.float64)):
        tot += float(np.sum(np.maximum.reduceat(pos, starts)
                            - np.minimum.reduceat(pos, starts)))
    return tot


def net_values(inst, x=None, y=None, gamma=None, model: str = "wa"):
    """Per net, over both axes: its wirelength term (Eq. (3), or the
    log-sum-exp model with model="lse") and its half-perimeter (Eq. (1)).
    Returns two float64 arrays [num_nets], zero for nets without pins."""
    x = inst.x if x is None else x
    y = inst.y if y is None else y
    gamma = inst.gamma if gamma is None else gamma
    pc = np.asarray(inst.pin_cell, np.int64)
    net_ptr, deg, ne = _segments(inst.net_ptr)
    E = net_ptr.size - 1
    wl = np.zeros(E)
    hp = np.zeros(E)
    starts = net_ptr[:-1][ne]
    if starts.size == 0:
        return wl, hp
    for pos in (np.asarray(x, np.float64)[pc] + np.asarray(inst.pin_dx, np.float64),
                np.asarray(y, np.float64)[pc] + np.asarray(inst.pin_dy, np.float64)):
        if model == "lse":
            v = _lse_axis(pos, inst.net_ptr, float(gamma))[0]
        else:
            v = _wa_axis(pos, inst.net_ptr, float(gamma))[0]
        wl[ne] += v
        hp[ne] += np.maximum.reduceat(pos, starts) - np.minimum.reduceat(pos, starts)
    return wl, hp


def overflow(rho: np.ndarray, base: np.ndarray, cap: np.ndarray) -> float:
    """Density overflow ratio tau (Section IV-A): movable area above the
    capacity each bin has left, over the total movable area in the region."""
    mov = np.asarray(rho, np.float64) - base
    tot = float(np.sum(mov))
    if tot <= 0.0:
        return 0.0
    return float(np.sum(np.maximum(0.0, mov - cap))) / tot


# ---------------------------------------------------------------------------
# One evaluation (Algorithm 1, the density / solve / gradient steps).
# ---------------------------------------------------------------------------

def evaluate(inst, lam: float = 1.0, gamma=None, grad_mode: str = "field",
             wl_model: str = "wa", eps: float = 0.0) -> Dict[str, object]:
    """f = W~ + lambda N (Eq. (7)) and its gradient for the movable cells.

    grad_mode "field": g = grad W~ + lambda * (-q E) (Section III-C);
    grad_mode "exact": g = grad W~ + lambda * dN/dx.
    wl_model "wa" (Eq. (3)) or "lse" (Section II) for W~; eps > 0 solves
    the screened equation (Eq. (4)) instead of Eq. (8).
    """
    base, cap = fixed_maps(inst)
    rho = density_map(inst, base)
    psi, ex, ey, a = poisson_solve(rho, eps)
    N = energy(rho, psi)
    if wl_model == "wa":
        wa, gwx, gwy = wa_wirelength(inst, gamma=gamma)
    elif wl_model == "lse":
        wa, gwx, gwy = lse_wirelength(inst, gamma=gamma)
    else:
        raise ValueError(wl_model)
    if grad_mode == "field":
        gnx, gny = field_gradient(inst, ex, ey)
    elif grad_mode == "exact":
        gnx, gny = exact_gradient(inst, psi)
    else:
        raise ValueError(grad_mode)
    return dict(
        base=base, cap=cap, rho=rho, a=a, psi=psi, ex=ex, ey=ey,
        energy=N, wa=wa, hpwl=hpwl(inst), overflow=overflow(rho, base, cap),
        gnx=gnx, gny=gny, gwx=gwx, gwy=gwy,
        gx=gwx + lam * gnx, gy=gwy + lam * gny,
        loss=wa + lam * N,
    )


# ---------------------------------------------------------------------------
# Finite differences of the objective (Eq. (7)) for a subset of cells.
# ---------------------------------------------------------------------------

def _axis_overlap(lo: float, hi: float, j0: int, j1: int, n: int) -> np.ndarray:
    """Overlap of [lo, hi) (clipped to [0, n]) with bins j0..j1, float64."""
    j = np.arange(j0, j1 + 1, dtype=np.float64)
    a = min(max(lo, 0.0), float(n))
    b = min(max(hi, 0.0), float(n))
    return np.maximum(0.0, np.minimum(b, j + 1.0) - np.maximum(a, j))


def local_fd_gradient(inst, cells, h: float = 1e-3, lam: float = 1.0, gamma=None,
                      psi=None):
    """Central differences of f = W~ + lam * N (Eq. (7)) for the given cells,
    each moved by +-h bin widths along x and along y, in FP64.

    N is evaluated locally: with d the density change of the moved cell,
    N(rho + d) = N + 2 d.psi + d.G d (Eq. (6) is a quadratic form in rho with
    the symmetric Green's operator G of the solve).  When no edge of the cell
    crosses a bin line within +-h, d(-h) = -d(+h), the quadratic terms cancel
    exactly and the central difference of N is (d(+h) - d(-h)).psi / h.
    Cells with an edge that close to a line (or to the region border) are
    flagged in ``kink`` and get NaN.  W~ changes only on the cell's nets.

    Returns (gx, gy, kink) for the cells, gradients in physical units."""
    n = inst.n
    gamma = inst.gamma if gamma is None else float(gamma)
    if psi is None:
        base, _ = fixed_maps(inst)
        psi = poisson_solve(density_map(inst, base))[0]
    xlo, xhi, ylo, yhi = (np.asarray(a, np.float64) for a in _rects(inst))
    pc = np.asarray(inst.pin_cell, np.int64)
    net_ptr = np.asarray(inst.net_ptr, np.int64)
    deg = np.diff(net_ptr)
    net_of_pin = np.repeat(np.arange(len(deg)), deg)
    order = np.argsort(pc, kind="stable")
    first = np.searchsorted(pc[order], np.arange(len(inst.x) + 1))
    X = np.asarray(inst.x, np.float64)
    Y = np.asarray(inst.y, np.float64)
    dxp = np.asarray(inst.pin_dx, np.float64)
    dyp = np.asarray(inst.pin_dy, np.float64)

    def net_wa(e, px, py):
        tot = 0.0
        for pos in (px, py):
            M, L = pos.max(), pos.min()
            ep = np.exp((pos - M) / gamma)
            em = np.exp((L - pos) / gamma)
            tot += (M + np.sum((pos - M) * ep) / np.sum(ep)) \
                - (L + np.sum((pos - L) * em) / np.sum(em))
        return tot

    def wa_nets(i, sx, sy):
        tot = 0.0
        for e in np.unique(net_of_pin[order[first[i]:first[i + 1]]]):
            p = np.arange(net_ptr[e], net_ptr[e + 1])
            px = X[pc[p]] + dxp[p]
            py = Y[pc[p]] + dyp[p]
            px[pc[p] == i] += sx
            py[pc[p] == i] += sy
            tot += net_wa(e, px, py)
        return tot

    cells = np.asarray(cells, np.int64)
    gx = np.full(cells.size, np.nan)
    gy = np.full(cells.size, np.nan)
    kink = np.zeros(cells.size, bool)
    for t, i in enumerate(cells):
        for axis in (0, 1):
            lo, hi = (xlo[i], xhi[i]) if axis == 0 else (ylo[i], yhi[i])
            olo, ohi = (ylo[i], yhi[i]) if axis == 0 else (xlo[i], xhi[i])
            if any(math.floor(e - h) != math.floor(e + h) for e in (lo, hi)):
                kink[t] = True
                continue
            j0 = max(int(math.floor(lo)) - 1, 0)
            j1 = min(int(math.floor(hi)) + 1, n - 1)
            k0 = max(int(math.floor(olo)), 0)
            k1 = min(int(math.ceil(ohi)) - 1, n - 1)
            if j1 < j0 or k1 < k0:
                dn = 0.0
            else:
                base1 = _axis_overlap(lo, hi, j0, j1, n)
                dp = _axis_overlap(lo + h, hi + h, j0, j1, n) - base1
                dm = _axis_overlap(lo - h, hi - h, j0, j1, n) - base1
                if np.max(np.abs(dp + dm)) > 1e-12:
                    kink[t] = True
                    continue
                oo = _axis_overlap(olo, ohi, k0, k1, n)
                sub = psi[k0:k1 + 1, j0:j1 + 1] if axis == 0 else psi[j0:j1 + 1, k0:k1 + 1].T
                # 2 (d+ - d-).psi / (2h), d = outer(other-axis overlap, change)
                dn = float(oo @ sub @ (dp - dm)) / h
            bw = inst.bin_w if axis == 0 else inst.bin_h
            hp = h * bw
            sx, sy = (hp, 0.0) if axis == 0 else (0.0, hp)
            dw = (wa_nets(i, sx, sy) - wa_nets(i, -sx, -sy)) / (2.0 * hp)
            g = dw + lam * dn / bw
            if axis == 0:
                gx[t] = g
            else:
                gy[t] = g
    gx[kink] = np.nan
    gy[kink] = np.nan
    return gx, gy, kink
