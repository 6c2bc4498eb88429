"""Pins of the oracle's spectral Poisson solve (Section III-D/E, Eqs.
(8)-(12)) against closed forms, the PDE itself, Parseval, symmetry and a
library DCT."""
import math

import numpy as np
import pytest
import scipy.fft

import oracle


def _cw(n):
    c = np.full(n, 2.0)
    c[0] = 1.0
    return c


@pytest.mark.parametrize("n", [4, 8])
def test_literal_quadruple_sum_equals_separable(n):
    rho = np.random.default_rng(n).random((n, n))
    a1 = oracle.dct_coefficients_literal(rho)
    a2 = oracle.dct_coefficients(rho)
    assert np.max(np.abs(a1 - a2)) < 1e-13


@pytest.mark.parametrize("n", [8, 64, 256])
def test_coefficients_are_scaled_library_dct2(n):
    # scipy's unnormalised DCT-II is 2 * sum x_i cos(pi k (2i+1) / 2n)
    rho = np.random.default_rng(n + 1).random((n, n))
    a = oracle.dct_coefficients(rho)
    ref = np.outer(_cw(n), _cw(n)) / (4.0 * n * n) * scipy.fft.dctn(rho, type=2)
    assert np.max(np.abs(a - ref)) < 1e-13


@pytest.mark.parametrize("n", [8, 32])
def test_coefficients_reconstruct_density(n):
    # Eq. (9) with these coefficients gives rho back at the bin centres
    rng = np.random.default_rng(2 * n)
    rho = rng.random((n, n))
    a = oracle.dct_coefficients(rho)
    x = np.arange(n) + 0.5
    w = np.pi * np.arange(n) / n
    rec = np.cos(np.outer(x, w)) @ a @ np.cos(np.outer(w, x))   # [iy, v] a[v, u] [u, ix]
    assert np.max(np.abs(rec - rho)) < 1e-12


@pytest.mark.parametrize("n,u,v", [(16, 3, 5), (16, 1, 0), (16, 0, 7), (64, 17, 40)])
def test_single_mode_closed_form(n, u, v):
    x = np.arange(n) + 0.5
    wu, wv = np.pi * u / n, np.pi * v / n
    rho = np.outer(np.cos(wv * x), np.cos(wu * x))          # [iy, ix]
    psi, ex, ey, a = oracle.poisson_solve(rho)
    d = wu * wu + wv * wv
    assert np.max(np.abs(psi - rho / d)) < 1e-12 * max(1.0, 1.0 / d)
    ex_ref = wu / d * np.outer(np.cos(wv * x), np.sin(wu * x))
    ey_ref = wv / d * np.outer(np.sin(wv * x), np.cos(wu * x))
    assert np.max(np.abs(ex - ex_ref)) < 1e-12 * max(1.0, 1.0 / d)
    assert np.max(np.abs(ey - ey_ref)) < 1e-12 * max(1.0, 1.0 / d)


@pytest.mark.parametrize("n,u,v", [(16, 3, 5), (16, 1, 0), (16, 0, 7), (64, 17, 40)])
def test_single_mode_potential_differences(n, u, v):
    # psi = mode / d; its difference to the next bin centre in closed form,
    # cos(w (i + 3/2)) - cos(w (i + 1/2)) = -2 sin(w / 2) sin(w (i + 1)), which
    # is zero at the last centre (the mirror of the Neumann extension)
    x = np.arange(n) + 0.5
    wu, wv = np.pi * u / n, np.pi * v / n
    rho = np.outer(np.cos(wv * x), np.cos(wu * x))
    psi = oracle.poisson_solve(rho)[0]
    dx, dy = oracle.potential_differences(psi)
    d = wu * wu + wv * wv
    i1 = np.arange(n) + 1.0
    dx_ref = -2.0 * np.sin(wu / 2) / d * np.outer(np.cos(wv * x), np.sin(wu * i1))
    dy_ref = -2.0 * np.sin(wv / 2) / d * np.outer(np.sin(wv * i1), np.cos(wu * x))
    tol = 1e-12 * max(1.0, 1.0 / d)
    assert np.max(np.abs(dx - dx_ref)) < tol and np.max(np.abs(dy - dy_ref)) < tol


def test_constant_density_gives_nothing():
    rho = np.full((16, 16), 0.9)
    psi, ex, ey, a = oracle.poisson_solve(rho)
    assert np.max(np.abs(psi)) < 1e-14 and np.max(np.abs(ex)) < 1e-14
    assert np.max(np.abs(ey)) < 1e-14
    assert abs(oracle.energy(rho, psi)) < 1e-12


def test_dc_removed_and_psi_zero_mean():
    rho = np.random.default_rng(1).random((32, 32)) + 5.0
    psi, ex, ey, a = oracle.poisson_solve(rho)
    assert a[0, 0] == 0.0
    assert abs(psi.sum()) < 1e-10 * np.abs(psi).sum()      # zero integral, Eq. (8)
    rho2 = rho + 3.0                                        # shifting rho changes nothing
    psi2, ex2, ey2, _ = oracle.poisson_solve(rho2)
    assert np.max(np.abs(psi2 - psi)) < 1e-11


@pytest.mark.parametrize("n", [16, 64])
def test_parseval_energy(n):
    rho = np.random.default_rng(n).random((n, n))
    psi, ex, ey, a = oracle.poisson_solve(rho)
    w = np.pi * np.arange(n) / n
    d = w[:, None] ** 2 + w[None, :] ** 2
    d[0, 0] = 1.0
    c = _cw(n)
    N_spec = n * n * np.sum(a * a / (np.outer(c, c) * d))
    N = oracle.energy(rho, psi)
    assert N > 0
    assert abs(N - N_spec) < 1e-12 * N


def _series(G, Gx, Gy, xs, ys):
    # continuous Fourier series of Eqs. (11)/(12) at arbitrary points
    n = G.shape[0]
    w = np.pi * np.arange(n) / n
    cy, sy = np.cos(np.outer(ys, w)), np.sin(np.outer(ys, w))
    cx, sx = np.cos(np.outer(w, xs)), np.sin(np.outer(w, xs))
    return cy @ G @ cx, cy @ Gx @ sx, sy @ Gy @ cx


def test_poisson_pde_neumann_and_field_is_minus_gradient():
    n = 16
    rng = np.random.default_rng(11)
    rho = rng.random((n, n))
    psi, ex, ey, a = oracle.poisson_solve(rho)
    G, Gx, Gy = oracle.spectral_potential(a)
    xc = np.arange(n) + 0.5
    h = 1e-3
    P = lambda xs, ys: _series(G, Gx, Gy, xs, ys)[0]
    # series at the bin centres is what the oracle returned
    assert np.max(np.abs(P(xc, xc) - psi)) < 1e-12
    # -Laplacian(psi) = rho - mean(rho) at the bin centres (Eq. (8))
    lap = (P(xc + h, xc) + P(xc - h, xc) + P(xc, xc + h) + P(xc, xc - h)
           - 4 * P(xc, xc)) / (h * h)
    assert np.max(np.abs(-lap - (rho - rho.mean()))) < 2e-5
    # E = -grad psi (Eq. (12) from Eq. (11)), by central differences
    dpx = (P(xc + h, xc) - P(xc - h, xc)) / (2 * h)
    dpy = (P(xc, xc + h) - P(xc, xc - h)) / (2 * h)
    assert np.max(np.abs(ex + dpx)) < 1e-6 * np.max(np.abs(ex))
    assert np.max(np.abs(ey + dpy)) < 1e-6 * np.max(np.abs(ey))
    # Neumann: zero normal derivative on the region boundary x = 0, n
    ys = np.linspace(0, n, 7)
    for xb in (0.0, float(n)):
        _, exb, _ = _series(G, Gx, Gy, np.array([xb]), ys)
        assert np.max(np.abs(exb)) < 1e-12
        _, _, eyb = _series(G, Gx, Gy, ys, np.array([xb]))
        assert np.max(np.abs(eyb)) < 1e-12


def test_mirror_and_transpose_symmetry():
    n = 32
    rho = np.random.default_rng(5).random((n, n))
    psi, ex, ey, _ = oracle.poisson_solve(rho)
    psf, exf, eyf, _ = oracle.poisson_solve(rho[:, ::-1])        # flip in x
    assert np.max(np.abs(psf - psi[:, ::-1])) < 1e-12
    assert np.max(np.abs(exf + ex[:, ::-1])) < 1e-12
    assert np.max(np.abs(eyf - ey[:, ::-1])) < 1e-12
    pst, ext, eyt, _ = oracle.poisson_solve(rho.T)               # transpose
    assert np.max(np.abs(pst - psi.T)) < 1e-12
    assert np.max(np.abs(ext - ey.T)) < 1e-12
    assert np.max(np.abs(eyt - ex.T)) < 1e-12


def test_dst_as_reversed_cosine_identity():
    # sum_{u>=1} b_u sin(w_u (i+1/2)) = (-1)^i sum_{k>=1} b_{n-k} cos(w_k (i+1/2))
    n = 32
    b = np.random.default_rng(3).random(n)
    b[0] = 0.0
    i = np.arange(n)
    S = oracle.sin_table(n)
    K = oracle.cos_table(n)
    lhs = b @ S
    br = np.zeros(n)
    br[1:] = b[n - np.arange(1, n)]
    rhs = ((-1.0) ** i) * (br @ K)
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_tables_against_direct_trig():
    n = 1024
    u = np.array([0, 1, 511, 512, 1023])
    i = np.array([0, 5, 1023])
    K = oracle.cos_table(n)
    S = oracle.sin_table(n)
    for uu in u:
        for ii in i:
            ang = math.pi * uu * (2 * ii + 1) / (2 * n)
            assert abs(K[uu, ii] - math.cos(ang)) < 1e-12
            assert abs(S[uu, ii] - math.sin(ang)) < 1e-12


# ---- the screened (Helmholtz) form of Eq. (4), Eq. (8)'s sign convention ----

@pytest.mark.parametrize("n,u,v,eps", [(16, 3, 5, 0.05), (16, 0, 1, 2.0), (64, 17, 40, 0.3)])
def test_screened_single_mode_closed_form(n, u, v, eps):
    x = np.arange(n) + 0.5
    wu, wv = np.pi * u / n, np.pi * v / n
    rho = np.outer(np.cos(wv * x), np.cos(wu * x))
    psi, ex, ey, _ = oracle.poisson_solve(rho, eps)
    d = wu * wu + wv * wv + eps
    assert np.max(np.abs(psi - rho / d)) < 1e-12 / d
    assert np.max(np.abs(ex - wu / d * np.outer(np.cos(wv * x), np.sin(wu * x)))) < 1e-12 / d
    assert np.max(np.abs(ey - wv / d * np.outer(np.sin(wv * x), np.cos(wu * x)))) < 1e-12 / d


def test_screened_pde_and_neumann_boundary():
    n, eps = 16, 0.4
    rho = np.random.default_rng(12).random((n, n))
    psi, ex, ey, a = oracle.poisson_solve(rho, eps)
    G, Gx, Gy = oracle.spectral_potential(a, eps)
    xc = np.arange(n) + 0.5
    h = 1e-3
    P = lambda xs, ys: _series(G, Gx, Gy, xs, ys)[0]
    assert np.max(np.abs(P(xc, xc) - psi)) < 1e-12
    lap = (P(xc + h, xc) + P(xc - h, xc) + P(xc, xc + h) + P(xc, xc - h)
           - 4 * P(xc, xc)) / (h * h)
    # -laplace(psi) + eps psi = rho - mean at the bin centres
    assert np.max(np.abs(-lap + eps * psi - (rho - rho.mean()))) < 2e-5
    dpx = (P(xc + h, xc) - P(xc - h, xc)) / (2 * h)
    assert np.max(np.abs(ex + dpx)) < 1e-6 * np.max(np.abs(ex))
    ys = np.linspace(0, n, 7)
    for xb in (0.0, float(n)):
        assert np.max(np.abs(_series(G, Gx, Gy, np.array([xb]), ys)[1])) < 1e-12


def test_screened_parseval_monotone_and_limits():
    n = 32
    rho = np.random.default_rng(13).random((n, n))
    w = np.pi * np.arange(n) / n
    c = _cw(n)
    last = None
    for eps in (0.0, 1e-3, 0.1, 1.0, 10.0):
        psi, _, _, a = oracle.poisson_solve(rho, eps)
        d = w[:, None] ** 2 + w[None, :] ** 2 + eps
        d[0, 0] = 1.0
        N_spec = n * n * np.sum(a * a / (np.outer(c, c) * d))
        N = oracle.energy(rho, psi)
        assert abs(N - N_spec) < 1e-12 * N
        if last is not None:
            assert N < last          # screening only lowers every mode's weight
        last = N
    # eps -> 0 is Eq. (8); eps -> infinity makes the potential local: eps psi -> rho - mean
    p0 = oracle.poisson_solve(rho)[0]
    p1 = oracle.poisson_solve(rho, 1e-9)[0]
    assert np.max(np.abs(p1 - p0)) < 1e-7 * np.max(np.abs(p0))
    big = 1e6
    pb = oracle.poisson_solve(rho, big)[0]
    dev = rho - rho.mean()
    assert np.max(np.abs(big * pb - dev)) < 3e-5 * np.max(np.abs(dev))
