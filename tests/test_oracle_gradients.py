"""Pins of the oracle's wirelength (Eqs. (1), (3)), density gradients
(Section III-C, Eq. (6)) and overflow (Section IV-A)."""
import math

import numpy as np
import pytest

import gen
import oracle
from _helpers import hand_instance, tiny_instance, with_macros


def _net_inst(coords, gamma):
    # cells of zero size at given centres; one net over all of them
    k = len(coords)
    cells = [[cx, cy, 0.5, 0.5] for (cx, cy) in coords]
    inst = hand_instance(cells, n=8, nets=[[(i, 0.0, 0.0) for i in range(k)]])
    inst.gamma = gamma
    return inst


@pytest.mark.parametrize("d,gamma", [(0.375, 0.5), (2.0, 0.5), (7.0, 0.25), (40.0, 3.0)])
def test_wa_two_pin_closed_form(d, gamma):
    # two pins distance d apart: W~ = d tanh(d / 2 gamma) per axis
    inst = _net_inst([(1.0, 2.0), (1.0 + d, 2.0 + d)], gamma)
    W, gx, gy = oracle.wa_wirelength(inst)
    assert W == pytest.approx(2 * d * math.tanh(d / (2 * gamma)), rel=1e-12)
    # and its derivative: d/dd [d tanh(d/2g)] = tanh + d/(2g) sech^2
    t = math.tanh(d / (2 * gamma))
    dd = t + d / (2 * gamma) * (1 - t * t)
    assert gx[1] == pytest.approx(dd, rel=1e-10) and gx[0] == pytest.approx(-dd, rel=1e-10)


def test_wa_gradient_by_finite_differences():
    inst = tiny_instance(seed=4, m=40, n=8, num_nets=30)
    inst.gamma = 0.8
    W, gx, gy = oracle.wa_wirelength(inst)
    x = inst.x.astype(np.float64)
    y = inst.y.astype(np.float64)
    h = 1e-5
    for i in range(0, 40, 3):
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (oracle.wa_wirelength(inst, x=xp, y=y)[0]
              - oracle.wa_wirelength(inst, x=xm, y=y)[0]) / (2 * h)
        assert abs(fd - gx[i]) < 1e-6 * max(1.0, abs(gx[i]))
        yp, ym = y.copy(), y.copy()
        yp[i] += h
        ym[i] -= h
        fd = (oracle.wa_wirelength(inst, x=x, y=yp)[0]
              - oracle.wa_wirelength(inst, x=x, y=ym)[0]) / (2 * h)
        assert abs(fd - gy[i]) < 1e-6 * max(1.0, abs(gy[i]))


def test_wa_translation_invariance_bounds_and_limit():
    inst = tiny_instance(seed=5, m=80, n=8, num_nets=60)
    W, gx, gy = oracle.wa_wirelength(inst)
    # gradient of a translation-invariant function sums to zero
    assert abs(gx.sum()) < 1e-9 and abs(gy.sum()) < 1e-9
    H = oracle.hpwl(inst)
    assert W <= H + 1e-9                                   # WA underestimates HPWL
    Ws = [oracle.wa_wirelength(inst, gamma=g)[0] for g in (1.0, 0.1, 0.01, 0.001)]
    assert all(a <= b + 1e-9 for a, b in zip(Ws, Ws[1:]))  # grows as gamma shrinks
    assert abs(Ws[-1] - H) < 1e-6 * H                      # converges to HPWL
    W2, gx2, _ = oracle.wa_wirelength(inst, x=inst.x.astype(np.float64) + 1234.5)
    assert W2 == pytest.approx(W, rel=1e-12) and np.allclose(gx2, gx, atol=1e-12)


def test_wa_matches_unshifted_textbook_form():
    # Eq. (3) as printed, without max/min shifting, where exp does not overflow
    inst = tiny_instance(seed=6, m=50, n=8, num_nets=40)
    g = 2.0
    px = inst.x.astype(np.float64)[inst.pin_cell] + inst.pin_dx
    tot = 0.0
    for e in range(inst.num_nets):
        s = px[inst.net_ptr[e]:inst.net_ptr[e + 1]]
        ep, em = np.exp(s / g), np.exp(-s / g)
        tot += np.sum(s * ep) / np.sum(ep) - np.sum(s * em) / np.sum(em)
    py = inst.y.astype(np.float64)[inst.pin_cell] + inst.pin_dy
    for e in range(inst.num_nets):
        s = py[inst.net_ptr[e]:inst.net_ptr[e + 1]]
        ep, em = np.exp(s / g), np.exp(-s / g)
        tot += np.sum(s * ep) / np.sum(ep) - np.sum(s * em) / np.sum(em)
    assert oracle.wa_wirelength(inst, gamma=g)[0] == pytest.approx(tot, rel=1e-11)


def test_hpwl_brute_force_and_degenerate_nets():
    inst = tiny_instance(seed=7, m=30, n=8, num_nets=25)
    px = [float(inst.x[c]) + float(d) for c, d in zip(inst.pin_cell, inst.pin_dx)]
    py = [float(inst.y[c]) + float(d) for c, d in zip(inst.pin_cell, inst.pin_dy)]
    tot = 0.0
    for e in range(inst.num_nets):
        a, b = inst.net_ptr[e], inst.net_ptr[e + 1]
        tot += max(abs(p - q) for p in px[a:b] for q in px[a:b])
        tot += max(abs(p - q) for p in py[a:b] for q in py[a:b])
    assert oracle.hpwl(inst) == pytest.approx(tot, rel=1e-12)
    # an empty net and a single-pin net contribute nothing
    one = hand_instance([[1, 1, 1, 1], [3, 3, 1, 1]], n=4,
                        nets=[[], [(0, 0.1, 0.2)], [(0, 0, 0), (1, 0, 0)]])
    W, gx, gy = oracle.wa_wirelength(one)
    assert oracle.hpwl(one) == pytest.approx(4.0)
    assert W == pytest.approx(2 * 2 * math.tanh(2 / (2 * one.gamma)))
    assert gx[0] == pytest.approx(-gx[1])


def _energy_of_rects(n, rects, base):
    rho = oracle.rasterise(n, rects) + base
    psi, _, _, _ = oracle.poisson_solve(rho)
    return oracle.energy(rho, psi)


def test_exact_gradient_by_finite_differences():
    # N is piecewise quadratic in each edge position: central differences of
    # N over the cell's float64 rectangle are exact up to rounding unless an
    # edge crosses a bin line within +-h
    inst = tiny_instance(seed=8, m=40, n=16, num_nets=10, util=0.5)
    inst = with_macros(inst, [[10.0, 10.0, 4.0, 3.0]])
    base, _ = oracle.fixed_maps(inst)
    rho = oracle.density_map(inst, base)
    psi, _, _, _ = oracle.poisson_solve(rho)
    gx, gy = oracle.exact_gradient(inst, psi)
    xlo, xhi = oracle.cell_rect_f32(inst.xl, inst.bin_w, inst.x, inst.w)
    ylo, yhi = oracle.cell_rect_f32(inst.yl, inst.bin_h, inst.y, inst.h)
    rects = [a.astype(np.float64) for a in (xlo, xhi, ylo, yhi)]
    h = 1e-3                                             # in bins
    checked = 0
    for i in range(40):
        for axis in (0, 1):
            lo, hi = (0, 1) if axis == 0 else (2, 3)
            if (np.floor(rects[lo][i] - h) != np.floor(rects[lo][i] + h)
                    or np.floor(rects[hi][i] - h) != np.floor(rects[hi][i] + h)):
                continue
            vals = []
            for s in (+h, -h):
                rr = [r.copy() for r in rects]
                rr[lo][i] += s
                rr[hi][i] += s
                vals.append(_energy_of_rects(inst.n, rr, base))
            bsz = inst.bin_w if axis == 0 else inst.bin_h
            fd = (vals[0] - vals[1]) / (2 * h) / bsz
            g = (gx if axis == 0 else gy)[i]
            assert abs(fd - g) < 1e-8 * max(1.0, abs(g)), (i, axis, fd, g)
            checked += 1
    assert checked > 60


def test_field_gradient_is_adjoint_of_density_scatter():
    # <lam, gather(E)> = <scatter(lam), E> for any weights lam and any map E
    inst = tiny_instance(seed=9, m=70, n=16)
    rng = np.random.default_rng(9)
    E = rng.standard_normal((16, 16))
    lam = rng.standard_normal(70)
    gx, gy = oracle.field_gradient(inst, E, E)
    xlo, xhi = oracle.cell_rect_f32(inst.xl, inst.bin_w, inst.x, inst.w)
    ylo, yhi = oracle.cell_rect_f32(inst.yl, inst.bin_h, inst.y, inst.h)
    rho_l = oracle.rasterise(16, (xlo, xhi, ylo, yhi), weight=lam)
    assert np.dot(lam, -gx * inst.bin_w) == pytest.approx(np.sum(rho_l * E), rel=1e-11)
    assert np.dot(lam, -gy * inst.bin_h) == pytest.approx(np.sum(rho_l * E), rel=1e-11)


def test_field_gradient_aligned_cell_and_agreement_with_exact():
    n = 16
    cells = [[j + 0.5, k + 0.5, 1.0, 1.0] for (j, k) in [(2, 3), (9, 9), (14, 1)]]
    inst = hand_instance(cells, n=n)
    rng = np.random.default_rng(2)
    ex, ey = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    gx, gy = oracle.field_gradient(inst, ex, ey)
    for c, (j, k) in enumerate([(2, 3), (9, 9), (14, 1)]):
        assert gx[c] == -ex[k, j] and gy[c] == -ey[k, j]
    # the field form approximates half the exact derivative of N on a
    # smooth-ish density (Section III-C surrogate; informational bound)
    inst = tiny_instance(seed=10, m=120, n=32, util=0.3)
    r = oracle.evaluate(inst, grad_mode="field")
    gxe, gye = oracle.exact_gradient(inst, r["psi"])
    a = np.concatenate([r["gnx"], r["gny"]])
    b = 0.5 * np.concatenate([gxe, gye])
    cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
    assert cos > 0.8


def test_overflow_hand_cases():
    n = 4
    inst = hand_instance([[0.5, 0.5, 1.0, 1.0], [0.5, 0.5, 1.0, 1.0],
                          [2.5, 2.5, 1.0, 1.0]], n=n)
    base, cap = oracle.fixed_maps(inst)
    rho = oracle.density_map(inst, base)
    # bin (0,0) holds 2 with capacity 1: overflow 1 of total movable 3
    assert oracle.overflow(rho, base, cap) == pytest.approx(1.0 / 3.0)
    inst2 = hand_instance([[0.5, 0.5, 1.0, 1.0], [2.5, 2.5, 1.0, 1.0]], n=n)
    base, cap = oracle.fixed_maps(inst2)
    assert oracle.overflow(oracle.density_map(inst2, base), base, cap) == 0.0
    # a macro removes capacity: a cell on a fully covered bin overflows fully
    inst3 = with_macros(inst2, [[0.5, 0.5, 1.0, 1.0]])
    base, cap = oracle.fixed_maps(inst3)
    assert oracle.overflow(oracle.density_map(inst3, base), base, cap) == pytest.approx(0.5)


def test_evaluate_composition():
    inst = tiny_instance(seed=12, m=100, n=16, num_nets=80, macros=2, macro_frac=0.1)
    r = oracle.evaluate(inst, lam=0.37)
    assert r["loss"] == pytest.approx(r["wa"] + 0.37 * r["energy"])
    assert np.allclose(r["gx"], r["gwx"] + 0.37 * r["gnx"])
    assert r["energy"] > 0 and 0 <= r["overflow"] <= 1


def test_local_finite_differences_match_the_exact_gradient():
    # the local central differences of W~ + lam N (moving one cell at a time,
    # N updated through its quadratic form) against the closed-form exact
    # gradient, on cells whose edges stay inside their bins
    inst = with_macros(gen.make_config("small_2k"), [[30.0, 30.0, 10.0, 8.0]])
    ref = oracle.evaluate(inst, lam=2.0, grad_mode="exact")
    cells = np.random.default_rng(40).choice(inst.num_cells, 300, replace=False)
    gx, gy, kink = oracle.local_fd_gradient(inst, cells, 1e-3, 2.0, psi=ref["psi"])
    assert kink.sum() < 0.05 * cells.size
    ok = ~kink
    ex = np.concatenate([ref["gx"][cells][ok], ref["gy"][cells][ok]])
    fd = np.concatenate([gx[ok], gy[ok]])
    assert np.linalg.norm(ex - fd) / np.linalg.norm(ex) < 1e-6


# ---- log-sum-exp wirelength (the model Section II sets beside Eq. (3)) ----

@pytest.mark.parametrize("d,gamma", [(0.375, 0.5), (2.0, 0.5), (7.0, 0.25), (40.0, 3.0)])
def test_lse_two_pin_closed_form(d, gamma):
    # per axis: gamma ln(e^{a/g} + e^{b/g}) + gamma ln(e^{-a/g} + e^{-b/g})
    #         = d + 2 gamma ln(1 + e^{-d/gamma}); derivative tanh(d / 2 gamma)
    inst = _net_inst([(1.0, 2.0), (1.0 + d, 2.0 + d)], gamma)
    W, gx, gy = oracle.lse_wirelength(inst)
    per_axis = d + 2 * gamma * math.log1p(math.exp(-d / gamma))
    assert W == pytest.approx(2 * per_axis, rel=1e-12)
    t = math.tanh(d / (2 * gamma))
    assert gx[1] == pytest.approx(t, rel=1e-10) and gx[0] == pytest.approx(-t, rel=1e-10)
    assert gy[1] == pytest.approx(t, rel=1e-10)


def test_lse_unshifted_form_at_moderate_gamma():
    # the textbook form with unshifted exponentials, where they do not overflow
    inst = tiny_instance(seed=6, m=30, n=8, num_nets=20)
    inst.gamma = 4.0
    W, _, _ = oracle.lse_wirelength(inst)
    pc = np.asarray(inst.pin_cell)
    ref = 0.0
    for pos in (inst.x.astype(np.float64)[pc] + inst.pin_dx, inst.y.astype(np.float64)[pc] + inst.pin_dy):
        for e in range(len(inst.net_ptr) - 1):
            q = pos[inst.net_ptr[e]:inst.net_ptr[e + 1]]
            if q.size:
                g = inst.gamma
                ref += g * math.log(math.fsum(math.exp(v / g) for v in q))
                ref += g * math.log(math.fsum(math.exp(-v / g) for v in q))
    assert W == pytest.approx(ref, rel=1e-12)


def test_lse_gradient_by_finite_differences():
    inst = tiny_instance(seed=7, m=40, n=8, num_nets=30)
    inst.gamma = 0.6
    W, gx, gy = oracle.lse_wirelength(inst)
    x = inst.x.astype(np.float64)
    y = inst.y.astype(np.float64)
    h = 1e-5
    for i in range(0, 40, 3):
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (oracle.lse_wirelength(inst, x=xp, y=y)[0]
              - oracle.lse_wirelength(inst, x=xm, y=y)[0]) / (2 * h)
        assert abs(fd - gx[i]) < 1e-6 * max(1.0, abs(gx[i]))
        yp, ym = y.copy(), y.copy()
        yp[i] += h
        ym[i] -= h
        fd = (oracle.lse_wirelength(inst, x=x, y=yp)[0]
              - oracle.lse_wirelength(inst, x=x, y=ym)[0]) / (2 * h)
        assert abs(fd - gy[i]) < 1e-6 * max(1.0, abs(gy[i]))


def test_lse_bounds_translation_invariance_and_limit():
    inst = tiny_instance(seed=8, m=80, n=8, num_nets=60)
    W, gx, gy = oracle.lse_wirelength(inst)
    assert abs(gx.sum()) < 1e-9 and abs(gy.sum()) < 1e-9
    # per net and axis HPWL <= LSE <= HPWL + 2 gamma ln(degree)
    hp = oracle.hpwl(inst)
    deg = np.diff(inst.net_ptr)
    slack = 2.0 * 2.0 * inst.gamma * np.sum(np.log(deg[deg > 0]))
    assert hp <= W <= hp + slack
    # LSE -> HPWL as gamma -> 0 (WA approaches from below, LSE from above)
    Wa, _, _ = oracle.wa_wirelength(inst, gamma=1e-4)
    Ws, _, _ = oracle.lse_wirelength(inst, gamma=1e-4)
    assert Wa <= hp <= Ws and Ws - hp < 1e-2


@pytest.mark.parametrize("model", ["wa", "lse"])
def test_net_values_by_brute_force_per_net(model):
    # per-net values against each net's definition written out pin by pin
    # (unshifted exponentials at a moderate gamma; max - min by pairwise
    # distances), including empty and one-pin nets
    base = tiny_instance(seed=8, m=40, n=8, num_nets=30)
    rng = np.random.default_rng(8)
    nets = [[], [(3, 0.1, -0.2)]]
    for d in (2, 3, 5, 9, 17):
        nets.append([(int(c), float(rng.random() - 0.5), float(rng.random() - 0.5))
                     for c in rng.choice(40, d, replace=False)])
    nets.append([])
    cells = np.stack([base.x, base.y, base.w, base.h], axis=1)
    inst = hand_instance(cells, n=8, bin_size=base.bin_w, nets=nets)
    g = 2.5
    wl, hp = oracle.net_values(inst, gamma=g, model=model)
    assert wl.shape == hp.shape == (inst.num_nets,)
    for e in range(inst.num_nets):
        a, b = inst.net_ptr[e], inst.net_ptr[e + 1]
        if b - a == 0:
            assert wl[e] == 0.0 and hp[e] == 0.0
            continue
        w_ref = h_ref = 0.0
        for pos, off in ((inst.x, inst.pin_dx), (inst.y, inst.pin_dy)):
            s = [float(pos[inst.pin_cell[p]]) + float(off[p]) for p in range(a, b)]
            h_ref += max(abs(u - v) for u in s for v in s)
            ep = [math.exp(v / g) for v in s]
            em = [math.exp(-v / g) for v in s]
            if model == "lse":
                w_ref += g * math.log(sum(ep)) + g * math.log(sum(em))
            else:
                w_ref += (sum(v * q for v, q in zip(s, ep)) / sum(ep)
                          - sum(v * q for v, q in zip(s, em)) / sum(em))
        assert wl[e] == pytest.approx(w_ref, rel=1e-11, abs=1e-12)
        assert hp[e] == pytest.approx(h_ref, rel=1e-12, abs=1e-12)
    # a one-pin net: zero spread; its LSE value is 2 gamma ln 1 = 0 too
    assert hp[1] == 0.0 and abs(wl[1]) < 1e-12
