"""GPU parity: every entry point of the C ABI against the FP64 oracle on the
same seeded inputs.  Index sets are compared bit for bit; floating-point
outputs to a relative L2 error of 1e-5 (float32 kernels vs float64 oracle)."""
import dataclasses

import numpy as np
import pytest

import gen
import oracle
from _helpers import hand_instance, rel_l2, tiny_instance, with_macros
from gpu_common import RTOL, DeviceCells, dev, host, lib_or_build, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_or_build()
    from paper_1312_4587_amd import fftpl
    return fftpl


def _grid(F, inst):
    return F.Grid.of(inst)


# ---------------------------------------------------------------------------
# index sets (bit-exact)
# ---------------------------------------------------------------------------

def _adversarial_cells():
    # bin size 0.5 (1/bin exact in float32): edges land exactly on bin lines,
    # and the float32 neighbours of those positions on both sides
    cells = []
    for j in range(0, 40):
        for w in (0.5, 1.0, 1.5, 2.0):
            c = np.float32(j * 0.25)
            for cc in (c, np.nextafter(c, np.float32(-10)), np.nextafter(c, np.float32(100))):
                cells.append([cc, cc, w, w])
    cells += [[-3.0, 2.0, 1.0, 1.0], [9.0, 9.0, 2.0, 2.0], [7.9, -0.1, 0.5, 0.5],
              [4.0, 4.0, 20.0, 20.0]]
    return hand_instance(cells, n=16, bin_size=0.5)


@pytest.mark.parametrize("case", ["adversarial", "random_large_bins", "small_2k"])
def test_cell_bins_bit_exact(F, case):
    import torch
    if case == "adversarial":
        inst = _adversarial_cells()
    elif case == "random_large_bins":
        rng = np.random.default_rng(17)
        m = 20000
        inst = gen.make_config("small_2k")
        inst = dataclasses.replace(
            inst, n=1024, bin_w=2.558117, bin_h=2.558117, xl=-1.5, yl=3.25,
            x=(rng.random(m) * 2700 - 50).astype(np.float32),
            y=(rng.random(m) * 2700 - 50).astype(np.float32),
            w=rng.integers(1, 5, m).astype(np.float32), h=np.ones(m, np.float32))
    else:
        inst = gen.make_config("small_2k")
    say("cell_bins", case, inst.num_cells, inst.n)
    c = DeviceCells(inst)
    rng_d = torch.empty(4 * inst.num_cells, dtype=torch.int32, device="cuda")
    F.debug_cell_bins(_grid(F, inst), c.x, c.y, c.w, c.h, rng_d)
    got = host(rng_d).reshape(-1, 4)
    xlo, xhi = oracle.cell_rect_f32(inst.xl, inst.bin_w, inst.x, inst.w)
    ylo, yhi = oracle.cell_rect_f32(inst.yl, inst.bin_h, inst.y, inst.h)
    ix0, ix1 = oracle.bin_range(xlo, xhi, inst.n)
    iy0, iy1 = oracle.bin_range(ylo, yhi, inst.n)
    exp = np.stack([ix0, ix1, iy0, iy1], axis=1)
    empty_g = (got[:, 0] > got[:, 1]) | (got[:, 2] > got[:, 3])
    empty_o = (exp[:, 0] > exp[:, 1]) | (exp[:, 2] > exp[:, 3])
    assert np.array_equal(empty_g, empty_o)
    assert np.array_equal(got[~empty_g], exp[~empty_o])


# ---------------------------------------------------------------------------
# density
# ---------------------------------------------------------------------------

def test_fixed_map(F):
    import torch
    inst = gen.make_instance(21, num_cells=1000, util=0.6, n=256, num_nets=10,
                             num_macros=20, macro_area_frac=0.15, target_density=0.9)
    say("fixed_map", inst.num_fixed)
    n2 = inst.n ** 2
    base = torch.empty(n2, device="cuda")
    cap = torch.empty(n2, device="cuda")
    F.fixed_map(_grid(F, inst), dev(inst.fx), dev(inst.fy), dev(inst.fw), dev(inst.fh),
                base, cap)
    b0, c0 = oracle.fixed_maps(inst)
    assert rel_l2(host(base).reshape(inst.n, inst.n), b0) < RTOL
    assert rel_l2(host(cap).reshape(inst.n, inst.n), c0) < RTOL
    F.fixed_map(_grid(F, inst), None, None, None, None, base, cap)
    assert float(base.abs().max()) == 0.0 and np.allclose(host(cap), 0.9)


@pytest.mark.parametrize("which", ["tiny_outside", "small_2k", "mid_macros", "n1024",
                                   "n2048_atomic"])
def test_density_map(F, which):
    import torch
    if which == "tiny_outside":
        inst = hand_instance([[0.25, 2.0, 1.5, 1.0], [7.9, 7.9, 1.0, 3.0],
                              [-5, -5, 1, 1], [4, 4, 0.25, 0.25]], n=8)
    elif which == "small_2k":
        inst = gen.make_config("small_2k")
    elif which == "mid_macros":
        inst = gen.make_instance(22, num_cells=100_000, util=0.8, n=512, num_nets=10,
                                 num_macros=20, macro_area_frac=0.15)
    elif which == "n1024":
        inst = gen.make_instance(23, num_cells=300_000, util=0.9, n=1024, num_nets=10)
    else:
        # past the band kernels' rows: float atomics
        inst = gen.make_instance(26, num_cells=400_000, util=0.9, n=2048, num_nets=10)
    say("density", which, inst.num_cells, inst.n)
    n2 = inst.n ** 2
    base = torch.empty(n2, device="cuda")
    grid = _grid(F, inst)
    if inst.num_fixed:
        F.fixed_map(grid, dev(inst.fx), dev(inst.fy), dev(inst.fw), dev(inst.fh), base)
    else:
        base.zero_()
    rho = torch.empty(n2, device="cuda")
    c = DeviceCells(inst)
    F.density_map(grid, c.x, c.y, c.w, c.h, base, rho)
    rho2 = torch.full((n2,), -1.0, device="cuda")
    F.density_map(grid, c.x, c.y, c.w, c.h, base, rho2)
    torch.cuda.synchronize()
    if inst.n <= 1024:
        assert torch.equal(rho, rho2)      # banded scatter: the same bits every run
    else:
        assert rel_l2(host(rho2), host(rho)) < 1e-6
    b0, _ = oracle.fixed_maps(inst)
    r0 = oracle.density_map(inst, b0)
    assert rel_l2(host(rho).reshape(inst.n, inst.n), r0) < RTOL
    F.density_map(grid, c.x, c.y, c.w, c.h, None, rho)
    assert rel_l2(host(rho).reshape(inst.n, inst.n), oracle.density_map(inst)) < RTOL


# ---------------------------------------------------------------------------
# spectral solve
# ---------------------------------------------------------------------------

def _solve(F, n, rho, mode="fft"):
    import torch
    grid = F.Grid(n, 0.0, 0.0, 1.0, 1.0)
    plan = F.Plan(n, mode)
    r = dev(rho.astype(np.float32).ravel())
    psi = torch.empty(n * n, device="cuda")
    ex = torch.empty(n * n, device="cuda")
    ey = torch.empty(n * n, device="cuda")
    en = torch.empty(1, dtype=torch.float64, device="cuda")
    F.poisson_solve(plan, grid, r, psi, ex, ey, en)
    out = [host(t).reshape(n, n) for t in (psi, ex, ey)] + [float(host(en)[0])]
    plan.close()
    return out


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 512, 1024])
def test_poisson_solve_random_density(F, n):
    rng = np.random.default_rng(100 + n)
    rho = (0.9 + 0.4 * rng.standard_normal((n, n))).astype(np.float32)
    say("poisson random", n)
    psi, ex, ey, en = _solve(F, n, rho)
    psi0, ex0, ey0, _ = oracle.poisson_solve(rho.astype(np.float64))
    e0 = oracle.energy(rho.astype(np.float64), psi0)
    say("errors psi/ex/ey/N", rel_l2(psi, psi0), rel_l2(ex, ex0), rel_l2(ey, ey0),
        abs(en - e0) / abs(e0))
    assert rel_l2(psi, psi0) < RTOL
    assert rel_l2(ex, ex0) < RTOL
    assert rel_l2(ey, ey0) < RTOL
    assert abs(en - e0) < RTOL * abs(e0)


@pytest.mark.parametrize("n,u,v", [(64, 3, 0), (256, 0, 1), (256, 17, 200), (1024, 1, 1)])
def test_poisson_single_mode_closed_form(F, n, u, v):
    x = np.arange(n) + 0.5
    wu, wv = np.pi * u / n, np.pi * v / n
    rho = np.outer(np.cos(wv * x), np.cos(wu * x))
    say("poisson mode", n, u, v)
    psi, ex, ey, _ = _solve(F, n, rho.astype(np.float32) + np.float32(0.75))
    d = wu * wu + wv * wv
    rho32 = rho.astype(np.float32).astype(np.float64)
    assert rel_l2(psi, rho32 / d) < RTOL
    ref_ex = wu / d * np.outer(np.cos(wv * x), np.sin(wu * x))
    ref_ey = wv / d * np.outer(np.sin(wv * x), np.cos(wu * x))
    if u:
        assert rel_l2(ex, ref_ex) < RTOL
    else:
        assert np.max(np.abs(ex)) < 1e-5 * np.max(np.abs(psi))
    if v:
        assert rel_l2(ey, ref_ey) < RTOL


@pytest.mark.parametrize("cfg", ["small_2k", "n1024_macros"])
def test_poisson_solve_instance_density(F, cfg):
    if cfg == "small_2k":
        inst = gen.make_config("small_2k")
    else:
        inst = gen.make_instance(24, num_cells=400_000, util=0.9, n=1024, num_nets=10,
                                 num_macros=50, macro_area_frac=0.15)
    b0, _ = oracle.fixed_maps(inst)
    rho = oracle.density_map(inst, b0)
    say("poisson instance", cfg)
    psi, ex, ey, en = _solve(F, inst.n, rho.astype(np.float32))
    r32 = rho.astype(np.float32).astype(np.float64)
    psi0, ex0, ey0, _ = oracle.poisson_solve(r32)
    assert rel_l2(psi, psi0) < RTOL
    assert rel_l2(ex, ex0) < RTOL and rel_l2(ey, ey0) < RTOL
    e0 = oracle.energy(r32, psi0)
    assert abs(en - e0) < RTOL * abs(e0)


# ---------------------------------------------------------------------------
# gathers and wirelength
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["field", "exact"])
def test_field_gather(F, mode):
    import torch
    inst = gen.make_config("small_2k")
    inst = with_macros(inst, [[20.0, 20.0, 6.0, 6.0]])
    b0, _ = oracle.fixed_maps(inst)
    rho = oracle.density_map(inst, b0)
    psi, ex, ey, _ = oracle.poisson_solve(rho)
    # both sides read the same float32 maps
    psi32, ex32, ey32 = (a.astype(np.float32) for a in (psi, ex, ey))
    c = DeviceCells(inst)
    m = inst.num_cells
    gx = torch.full((m,), 7.0, device="cuda")
    gy = torch.full((m,), -3.0, device="cuda")
    say("gather", mode)
    F.field_gather(_grid(F, inst), c.x, c.y, c.w, c.h, dev(ex32.ravel()), dev(ey32.ravel()),
                   dev(psi32.ravel()), mode, 0.5, 0, gx, gy)
    if mode == "field":
        rx, ry = oracle.field_gradient(inst, ex32.astype(np.float64), ey32.astype(np.float64))
    else:
        rx, ry = oracle.exact_gradient(inst, psi32.astype(np.float64))
    assert rel_l2(host(gx), 0.5 * rx) < RTOL and rel_l2(host(gy), 0.5 * ry) < RTOL
    F.field_gather(_grid(F, inst), c.x, c.y, c.w, c.h, dev(ex32.ravel()), dev(ey32.ravel()),
                   dev(psi32.ravel()), mode, 0.5, 1, gx, gy)
    assert rel_l2(host(gx), rx) < RTOL and rel_l2(host(gy), ry) < RTOL


def _wa_case(which):
    if which == "small_2k":
        return gen.make_config("small_2k")
    if which == "hi_degree":
        return gen.make_instance(31, num_cells=20_000, util=0.8, n=128, num_nets=20_000,
                                 hi_frac=0.02, hi_range=(9, 700))
    # empty, single-pin and boundary-degree nets mixed with ordinary ones
    base = tiny_instance(seed=32, m=200, n=16, num_nets=10)
    rng = np.random.default_rng(32)
    nets = [[], [(5, 0.1, 0.1)], []]
    for d in (2, 8, 9, 64, 65, 130):
        cells = rng.choice(200, d, replace=False)
        nets.append([(int(c), float(rng.random() - 0.5), float(rng.random() - 0.5))
                     for c in cells])
    nets.append([])
    cells = np.stack([base.x, base.y, base.w, base.h], axis=1)
    return hand_instance(cells, n=16, bin_size=base.bin_w, nets=nets)


@pytest.mark.parametrize("which", ["small_2k", "hi_degree", "degenerate"])
def test_wa_grad(F, which):
    import torch
    inst = _wa_case(which)
    say("wa", which, inst.num_nets, inst.num_pins)
    c = DeviceCells(inst)
    m = inst.num_cells
    gx = torch.full((m,), 11.0, device="cuda")
    gy = torch.full((m,), 11.0, device="cuda")
    wa = torch.zeros(1, dtype=torch.float64, device="cuda")
    hp = torch.zeros(1, dtype=torch.float64, device="cuda")
    gamma = inst.gamma
    F.wa_grad(dev(inst.net_ptr), dev(inst.pin_cell), dev(inst.pin_dx), dev(inst.pin_dy),
              c.x, c.y, gamma, 0, gx, gy, wa, hp)
    W0, rx, ry = oracle.wa_wirelength(inst)
    H0 = oracle.hpwl(inst)
    assert rel_l2(host(gx), rx) < RTOL and rel_l2(host(gy), ry) < RTOL
    assert abs(float(host(wa)[0]) - W0) <= RTOL * W0
    assert abs(float(host(hp)[0]) - H0) <= RTOL * H0
    # fixed-point per-cell sums and fixed-order totals: the same bits again
    gx2, gy2 = torch.empty_like(gx), torch.empty_like(gy)
    wa2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    hp2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    F.wa_grad(dev(inst.net_ptr), dev(inst.pin_cell), dev(inst.pin_dx), dev(inst.pin_dy),
              c.x, c.y, gamma, 0, gx2, gy2, wa2, hp2)
    torch.cuda.synchronize()
    assert torch.equal(gx, gx2) and torch.equal(gy, gy2)
    assert torch.equal(wa, wa2) and torch.equal(hp, hp2)
    F.wa_grad(dev(inst.net_ptr), dev(inst.pin_cell), dev(inst.pin_dx), dev(inst.pin_dy),
              c.x, c.y, gamma, 1, gx, gy, None, None)
    assert rel_l2(host(gx), 2 * rx) < RTOL


# ---------------------------------------------------------------------------
# full evaluation
# ---------------------------------------------------------------------------

def _run_eval(F, inst, lam, mode, dct="fft", plan=None, path="xch", wl_model="wa",
              screening=0.0):
    import torch
    prob = F.Problem.from_instance(inst, path=path, wl_model=wl_model, screening=screening)
    assert prob.path == path
    own = plan is None
    plan = plan or F.Plan(inst.n, dct)
    c = DeviceCells(inst)
    m = inst.num_cells
    gx = torch.empty(m, device="cuda")
    gy = torch.empty(m, device="cuda")
    out4 = torch.empty(4, dtype=torch.float64, device="cuda")
    F.eval(plan, prob, c.x, c.y, lam, inst.gamma, mode, gx, gy, out4)
    torch.cuda.synchronize()
    rho, psi, exy = (host(t) for t in plan.maps())
    res = dict(gx=host(gx), gy=host(gy), out=host(out4), rho=rho, psi=psi, exy=exy)
    if own:
        plan.close()
    return res


def _check_eval(inst, got, ref, lam, mode):
    say("errors rho/gx/gy", rel_l2(got["rho"], ref["rho"]), rel_l2(got["gx"], ref["gx"]),
        rel_l2(got["gy"], ref["gy"]), "scalars", got["out"], ref["energy"], ref["wa"],
        ref["hpwl"], ref["overflow"])
    assert rel_l2(got["rho"], ref["rho"]) < RTOL
    N, W, H, tau = got["out"]
    assert abs(N - ref["energy"]) < RTOL * abs(ref["energy"])
    assert abs(W - ref["wa"]) < RTOL * abs(ref["wa"])
    assert abs(H - ref["hpwl"]) < RTOL * abs(ref["hpwl"])
    assert abs(tau - ref["overflow"]) < RTOL
    if mode == "field":
        assert rel_l2(got["exy"][..., 0], ref["ex"]) < RTOL
        assert rel_l2(got["exy"][..., 1], ref["ey"]) < RTOL
    else:
        assert rel_l2(got["psi"], ref["psi"]) < RTOL
        # the exact gradient's inputs: differences of psi to the next bin centre
        dx, dy = oracle.potential_differences(ref["psi"])
        say("difference maps", rel_l2(got["exy"][..., 0], dx), rel_l2(got["exy"][..., 1], dy))
        assert rel_l2(got["exy"][..., 0], dx) < RTOL
        assert rel_l2(got["exy"][..., 1], dy) < RTOL
    assert rel_l2(got["gx"], ref["gx"]) < RTOL and rel_l2(got["gy"], ref["gy"]) < RTOL
    # per element: no cell or bin may be far off while the aggregate passes
    # (a cell without a band entry, a block edge); the bound is MAX_ABS_FRAC of
    # the largest magnitude, where float32 rounding of the largest terms sits
    for key, g in (("gx", got["gx"]), ("gy", got["gy"]), ("rho", got["rho"])):
        r = ref[key]
        err = np.abs(np.asarray(g, np.float64) - r).max() / np.abs(r).max()
        say("max abs err /", key, err)
        assert err < MAX_ABS_FRAC, key


# per-element bound of the evaluation outputs, relative to their largest
# magnitude: float32 rounding of the sums feeding one element (a few tens of
# terms of that magnitude) stays well inside 1e-5 of it
MAX_ABS_FRAC = 2e-5


@pytest.mark.parametrize("path", ["xch", "slots", "atomic"])
@pytest.mark.parametrize("mode", ["field", "exact"])
def test_eval_small(F, mode, path):
    inst = gen.make_config("small_2k")
    inst = with_macros(inst, [[30.0, 30.0, 10.0, 8.0], [60.0, 20.0, 5.0, 12.0]])
    lam = 3.0
    say("eval small", mode, path)
    got = _run_eval(F, inst, lam, mode, path=path)
    ref = oracle.evaluate(inst, lam=lam, grad_mode=mode)
    _check_eval(inst, got, ref, lam, mode)


@pytest.fixture(scope="module")
def large_2m_ref():
    inst = gen.make_config("large_2m")
    say("oracle large_2m")
    return inst, oracle.evaluate(inst, lam=1.0, grad_mode="field")


@pytest.mark.parametrize("dct", ["fft", "gemm_f32", "gemm_bf16x3"])
def test_eval_large_2m_full_workload(F, large_2m_ref, dct):
    # the 2.1M-cell, n = 1024 workload the benchmark times, every output, with
    # each spectral variant (split-BF16 against its sanity bound only)
    inst, ref = large_2m_ref
    say("eval large_2m", dct, inst.num_cells, inst.num_pins)
    got = _run_eval(F, inst, 1.0, "field", dct=dct)
    if dct != "gemm_bf16x3":
        _check_eval(inst, got, ref, 1.0, "field")
    else:
        e = rel_l2(np.concatenate([got["gx"], got["gy"]]), np.concatenate([ref["gx"], ref["gy"]]))
        say("bf16x3 large_2m grad err", e)
        assert e < BF16X3_SANITY and rel_l2(got["rho"], ref["rho"]) < RTOL


@pytest.mark.parametrize("dct", ["fft", "gemm_f32"])
def test_eval_exact_mode_mid_200k(F, dct):
    # the exact gradient sums the solve's difference maps: float32 differences
    # of psi itself would miss 1e-5 at this size (psi is ~10^3, its bin-to-bin
    # differences ~1)
    inst = gen.make_config("mid_200k")
    say("eval exact mid_200k", dct)
    got = _run_eval(F, inst, 2.0, "exact", dct=dct)
    ref = oracle.evaluate(inst, lam=2.0, grad_mode="exact")
    _check_eval(inst, got, ref, 2.0, "exact")


def test_eval_exact_mode_large_2m(F):
    inst = gen.make_config("large_2m")
    say("eval exact large_2m")
    got = _run_eval(F, inst, 1.0, "exact")
    ref = oracle.evaluate(inst, lam=1.0, grad_mode="exact")
    _check_eval(inst, got, ref, 1.0, "exact")


def test_eval_edge_cases(F):
    import torch
    # no cells and no nets at the smallest grid
    inst = hand_instance(np.zeros((0, 4)), n=8)
    for path in ("xch", "slots", "atomic"):
        got = _run_eval(F, inst, 1.0, "field", path=path)
        assert np.all(got["out"] == 0.0) and np.all(got["rho"] == 0.0)
    # cells partly and fully outside the region, exact mode, n = 8
    inst = hand_instance([[0.25, 2.0, 1.5, 1.0], [7.9, 7.9, 1.0, 3.0], [-5, -5, 1, 1],
                          [4, 4, 0.25, 0.25], [3.3, 5.1, 2.0, 1.0]], n=8,
                         nets=[[(0, 0, 0), (1, 0.1, 0)], [(2, 0, 0), (3, 0, 0), (4, 0, 0)]])
    for mode in ("field", "exact"):
        for path in ("xch", "slots", "atomic"):
            got = _run_eval(F, inst, 2.0, mode, path=path)
            ref = oracle.evaluate(inst, lam=2.0, grad_mode=mode)
            _check_eval(inst, got, ref, 2.0, mode)
    # a plan of another size is refused
    plan = F.Plan(16)
    with pytest.raises(F.FFTPLError) as ei:
        _run_eval(F, inst, 1.0, "field", plan=plan)
    assert ei.value.status == F.E_STATE
    plan.close()


@pytest.mark.parametrize("mode", ["field", "exact"])
def test_eval_repeatable(F, mode):
    # the exchange path has no float atomics: the same inputs give the same
    # bits (gradients, maps and all four scalars), on a fresh plan and problem
    # as on the same ones
    inst = gen.make_instance(81, num_cells=150_000, util=0.85, n=512, num_nets=160_000,
                             hi_frac=0.01, hi_range=(20, 400), num_macros=10,
                             macro_area_frac=0.1)
    a = _run_eval(F, inst, 1.0, mode)
    b = _run_eval(F, inst, 1.0, mode)
    for k in ("gx", "gy", "rho", "exy", "out"):
        assert np.array_equal(a[k], b[k]), k
    if mode == "exact":
        assert np.array_equal(a["psi"], b["psi"])


def test_netlist_index_is_a_cell_major_permutation(F):
    import torch
    inst = gen.make_instance(41, num_cells=50_000, util=0.8, n=256, num_nets=60_000,
                             hi_frac=0.01, hi_range=(20, 300))
    m, P = inst.num_cells, inst.num_pins
    say("netlist index", m, P)
    cp = torch.empty(m + 1, dtype=torch.int32, device="cuda")
    ps = torch.empty(P, dtype=torch.int32, device="cuda")
    F.netlist_index(m, dev(inst.pin_cell), cp, ps)
    cp, ps = host(cp), host(ps)
    cnt = np.bincount(inst.pin_cell, minlength=m)
    assert np.array_equal(cp, np.concatenate([[0], np.cumsum(cnt)]))
    assert np.array_equal(np.sort(ps), np.arange(P))
    c = inst.pin_cell
    assert np.all(ps >= cp[c]) and np.all(ps < cp[c + 1])


@pytest.mark.parametrize("mode", ["field", "exact"])
@pytest.mark.parametrize("n", [16, 64, 512, 1024])
def test_banded_scatter_with_tall_and_outside_cells(F, n, mode):
    # cells spanning many bands take the short list every band block walks
    # (and have no band entry, so their density gradient is taken from the
    # maps directly); cells outside the region and ragged sizes mixed in
    rng = np.random.default_rng(n)
    m = 3000
    side = 100.0
    x = rng.random(m) * 110 - 5
    y = rng.random(m) * 110 - 5
    w = rng.integers(1, 5, m).astype(float)
    h = np.ones(m)
    tall = rng.random(m) < 0.02
    h[tall] = rng.random(tall.sum()) * 60 + 5
    w[rng.random(m) < 0.01] = 40.0
    cells = np.stack([x, y, w, h], axis=1)
    nets = [[(int(a), 0.0, 0.0), (int(b), 0.1, -0.1)] for a, b in rng.integers(0, m, (500, 2)) if a != b]
    inst = hand_instance(cells, n=n, bin_size=side / n, nets=nets)
    inst = with_macros(inst, [[50.0, 50.0, 10.0, 30.0]])
    say("band scatter", n, mode)
    got = _run_eval(F, inst, 1.0, mode)
    ref = oracle.evaluate(inst, lam=1.0, grad_mode=mode)
    _check_eval(inst, got, ref, 1.0, mode)


@pytest.mark.parametrize("mode", ["field", "exact"])
def test_eval_clustered_cells(F, mode):
    # every cell near the centre: long slices per band and cell block, filled
    # into the walks' owner maps by whole wavefronts, several windows per band
    rng = np.random.default_rng(31)
    inst = gen.make_instance(31, num_cells=120_000, util=0.8, n=256, num_nets=100_000)
    c = 0.5 * inst.n * inst.bin_w
    x = (c + rng.normal(0.0, 5.0 * inst.bin_w, inst.num_cells)).astype(np.float32)
    y = (c + rng.normal(0.0, 5.0 * inst.bin_h, inst.num_cells)).astype(np.float32)
    inst = inst.with_positions(x, y)
    say("clustered", inst.num_cells, inst.n, mode)
    got = _run_eval(F, inst, 1.0, mode)
    ref = oracle.evaluate(inst, lam=1.0, grad_mode=mode)
    _check_eval(inst, got, ref, 1.0, mode)


# ---------------------------------------------------------------------------
# GEMM (matrix-core) variants of the spectral solve
# ---------------------------------------------------------------------------

# split-bf16 errors are reported, not gated at 1e-5; this bound only catches
# a broken product (a wrong operand layout gives errors of order 1)
BF16X3_SANITY = 1e-4


@pytest.mark.parametrize("mode", ["gemm_f32", "gemm_bf16x3"])
@pytest.mark.parametrize("n", [64, 128, 192, 256, 1024, 2048])
def test_poisson_solve_gemm_random_density(F, mode, n):
    rng = np.random.default_rng(200 + n)
    rho = (0.9 + 0.4 * rng.standard_normal((n, n))).astype(np.float32)
    psi, ex, ey, en = _solve(F, n, rho, mode)
    psi0, ex0, ey0, _ = oracle.poisson_solve(rho.astype(np.float64))
    e0 = oracle.energy(rho.astype(np.float64), psi0)
    errs = (rel_l2(psi, psi0), rel_l2(ex, ex0), rel_l2(ey, ey0), abs(en - e0) / abs(e0))
    say("gemm", mode, n, "errors psi/ex/ey/N", *errs)
    tol = RTOL if mode == "gemm_f32" else BF16X3_SANITY
    assert max(errs) < tol


@pytest.mark.parametrize("mode", ["gemm_f32", "gemm_bf16x3"])
def test_poisson_single_mode_gemm(F, mode):
    n, u, v = 256, 3, 5
    x = np.arange(n) + 0.5
    wu, wv = np.pi * u / n, np.pi * v / n
    rho = np.outer(np.cos(wv * x), np.cos(wu * x))
    psi, ex, ey, _ = _solve(F, n, rho.astype(np.float32) + np.float32(0.75), mode)
    d = wu * wu + wv * wv
    err = rel_l2(psi, rho.astype(np.float32).astype(np.float64) / d)
    say("gemm single mode", mode, err)
    assert err < (RTOL if mode == "gemm_f32" else BF16X3_SANITY)


@pytest.mark.parametrize("mode", ["gemm_f32", "gemm_bf16x3"])
def test_eval_gemm_field_and_exact_share_a_plan(F, mode):
    # n = 128: the field mode takes the even/odd split products and the exact
    # mode the dense ones; the two alternate on one plan (one GEMM workspace)
    inst = gen.make_config("small_2k", n=128)
    refs = {g: oracle.evaluate(inst, lam=2.0, grad_mode=g) for g in ("field", "exact")}
    plan = F.Plan(inst.n, mode)
    try:
        for grad in ("field", "exact", "field"):
            got = _run_eval(F, inst, 2.0, grad, dct=mode, plan=plan)
            if mode == "gemm_f32":
                _check_eval(inst, got, refs[grad], 2.0, grad)
            else:
                e = rel_l2(got["gx"], refs[grad]["gx"])
                say("bf16x3 n=128", grad, "grad err", e)
                assert e < BF16X3_SANITY
    finally:
        plan.close()


@pytest.mark.parametrize("mode", ["gemm_f32", "gemm_bf16x3"])
@pytest.mark.parametrize("grad", ["field", "exact"])
def test_eval_small_gemm(F, mode, grad):
    inst = gen.make_config("small_2k")
    inst = with_macros(inst, [[30.0, 30.0, 10.0, 8.0]])
    got = _run_eval(F, inst, 2.0, grad, dct=mode)
    ref = oracle.evaluate(inst, lam=2.0, grad_mode=grad)
    if mode == "gemm_f32":
        _check_eval(inst, got, ref, 2.0, grad)
    else:
        e = rel_l2(got["gx"], ref["gx"])
        say("bf16x3 eval small", grad, "grad err", e)
        assert e < BF16X3_SANITY
