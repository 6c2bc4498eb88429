"""GPU tests of the workspace-backed standalone calls (density map and
wirelength through the atomic-free kernels), the per-net test export, the
host-side refusal of unusable workspaces and indexes, and batched
evaluations (several designs per launch) against single evaluations and the
FP64 oracle."""
import dataclasses

import numpy as np
import pytest

import gen
import oracle
from _helpers import hand_instance, rel_l2, with_macros
from gpu_common import RTOL, DeviceCells, dev, host, lib_or_build, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_or_build()
    from paper_1312_4587_amd import fftpl
    return fftpl


def _tall_outside(n, seed):
    rng = np.random.default_rng(seed)
    m = 3000
    x = rng.random(m) * 110 - 5
    y = rng.random(m) * 110 - 5
    w = rng.integers(1, 5, m).astype(float)
    h = np.ones(m)
    tall = rng.random(m) < 0.02
    h[tall] = rng.random(tall.sum()) * 60 + 5
    cells = np.stack([x, y, w, h], axis=1)
    nets = [[(int(a), 0.0, 0.0), (int(b), 0.1, -0.1)]
            for a, b in rng.integers(0, m, (500, 2)) if a != b]
    return with_macros(hand_instance(cells, n=n, bin_size=100.0 / n, nets=nets),
                       [[50.0, 50.0, 10.0, 30.0]])


def clustered(inst, sigma_bins, seed):
    """The instance with every cell drawn around the region's centre (normal,
    sigma in bins): most bands hold long slices from every cell block."""
    rng = np.random.default_rng(seed)
    c = 0.5 * inst.n * inst.bin_w
    x = (c + rng.normal(0.0, sigma_bins * inst.bin_w, inst.num_cells)).astype(np.float32)
    y = (c + rng.normal(0.0, sigma_bins * inst.bin_h, inst.num_cells)).astype(np.float32)
    return inst.with_positions(x, y)


@pytest.mark.parametrize("case", ["small_2k", "tall_outside_64", "n1024_300k", "empty",
                                  "clustered_256", "n1024_4_3m"])
def test_problem_density_matches_oracle_and_repeats_bit_for_bit(F, case):
    import torch
    if case == "small_2k":
        inst = with_macros(gen.make_config("small_2k"), [[30.0, 30.0, 10.0, 8.0]])
    elif case == "tall_outside_64":
        inst = _tall_outside(64, 5)
    elif case == "n1024_300k":
        inst = gen.make_instance(23, num_cells=300_000, util=0.9, n=1024, num_nets=10,
                                 num_macros=30, macro_area_frac=0.15)
    elif case == "clustered_256":
        # slices of hundreds of entries per cell block and band, several
        # windows per band
        inst = clustered(gen.make_instance(24, num_cells=200_000, util=0.8, n=256,
                                           num_nets=10), 6.0, 24)
    elif case == "n1024_4_3m":
        # more than 1024 cell blocks: the band walks take their slices in
        # two chunks
        inst = gen.make_instance(25, num_cells=4_300_000, util=0.9, n=1024, num_nets=10)
    else:
        inst = hand_instance(np.zeros((0, 4)), n=16)
    say("problem_density", case, inst.num_cells, inst.n)
    prob = F.Problem.from_instance(inst)
    assert F.problem_path(prob) == "xch"
    c = DeviceCells(inst)
    n2 = inst.n ** 2
    rho = torch.empty(n2, device="cuda")
    F.problem_density(prob, c.x, c.y, rho)
    rho2 = torch.full((n2,), -1.0, device="cuda")
    F.problem_density(prob, c.x, c.y, rho2)
    torch.cuda.synchronize()
    assert torch.equal(rho, rho2)   # no atomics: the same bits on every run
    b0, _ = oracle.fixed_maps(inst)
    r0 = oracle.density_map(inst, b0)
    got = host(rho).reshape(inst.n, inst.n)
    if inst.num_cells == 0 and not inst.num_fixed:
        assert np.all(got == 0.0)
        return
    say("rho err", rel_l2(got, r0), "max abs", np.abs(got - r0).max())
    assert rel_l2(got, r0) < RTOL
    assert np.abs(got - r0).max() < 1e-5 * max(1.0, np.abs(r0).max())
    # the stateless call runs the same kernels in a temporary workspace: the
    # same bits
    rho3 = torch.empty(n2, device="cuda")
    F.density_map(prob.grid, c.x, c.y, prob.arrays["w"], prob.arrays["h"],
                  prob.arrays["base"], rho3)
    torch.cuda.synchronize()
    assert torch.equal(rho3, rho)


def _wl_case(which):
    if which == "small_2k":
        return gen.make_config("small_2k")
    if which == "hi_degree":
        return gen.make_instance(31, num_cells=20_000, util=0.8, n=128, num_nets=20_000,
                                 hi_frac=0.02, hi_range=(9, 3000))
    base = gen.make_instance(32, num_cells=200, util=0.6, n=16, num_nets=10)
    rng = np.random.default_rng(32)
    nets = [[], [(5, 0.1, 0.1)], []]
    for d in (2, 8, 9, 64, 65, 130):
        nets.append([(int(c), float(rng.random() - 0.5), float(rng.random() - 0.5))
                     for c in rng.choice(200, d, replace=False)])
    nets.append([])
    cells = np.stack([base.x, base.y, base.w, base.h], axis=1)
    return hand_instance(cells, n=16, bin_size=base.bin_w, nets=nets)


@pytest.mark.parametrize("model", ["wa", "lse"])
@pytest.mark.parametrize("which", ["small_2k", "hi_degree", "degenerate"])
def test_problem_wl_grad_matches_oracle(F, which, model):
    import torch
    inst = _wl_case(which)
    say("problem_wl_grad", which, model, inst.num_nets, inst.num_pins)
    prob = F.Problem.from_instance(inst, wl_model=model)
    c = DeviceCells(inst)
    m = inst.num_cells
    gx = torch.full((m,), 11.0, device="cuda")
    gy = torch.full((m,), 11.0, device="cuda")
    wl = torch.zeros(1, dtype=torch.float64, device="cuda")
    hp = torch.zeros(1, dtype=torch.float64, device="cuda")
    F.problem_wl_grad(prob, c.x, c.y, inst.gamma, 0, gx, gy, wl, hp)
    torch.cuda.synchronize()
    if model == "wa":
        W0, rx, ry = oracle.wa_wirelength(inst)
    else:
        W0, rx, ry = oracle.lse_wirelength(inst)
    H0 = oracle.hpwl(inst)
    ex, ey = rel_l2(host(gx), rx), rel_l2(host(gy), ry)
    say("grad err", ex, ey, "W", float(host(wl)[0]), W0)
    assert ex < RTOL and ey < RTOL
    assert abs(float(host(wl)[0]) - W0) <= RTOL * abs(W0)
    assert abs(float(host(hp)[0]) - H0) <= RTOL * H0
    # repeatable bit for bit; accumulate adds the same sums again
    gx2 = torch.empty_like(gx)
    gy2 = torch.empty_like(gy)
    F.problem_wl_grad(prob, c.x, c.y, inst.gamma, 0, gx2, gy2)
    torch.cuda.synchronize()
    assert torch.equal(gx, gx2) and torch.equal(gy, gy2)
    F.problem_wl_grad(prob, c.x, c.y, inst.gamma, 1, gx2, gy2)
    torch.cuda.synchronize()
    assert rel_l2(host(gx2), 2 * rx) < RTOL and rel_l2(host(gy2), 2 * ry) < RTOL


@pytest.mark.parametrize("model", ["wa", "lse"])
@pytest.mark.parametrize("which", ["small_2k", "hi_degree", "degenerate"])
def test_per_net_values_match_oracle_net_by_net(F, which, model):
    # every net's wirelength term and half-perimeter as the net blocks
    # compute them: each net was read with exactly its own pins
    import torch
    inst = _wl_case(which)
    prob = F.Problem.from_instance(inst, wl_model=model)
    c = DeviceCells(inst)
    P = inst.num_pins
    wl = torch.full((P,), -1.0, dtype=torch.float64, device="cuda")
    hp = torch.full((P,), -1.0, dtype=torch.float64, device="cuda")
    F.debug_net_values(prob, c.x, c.y, inst.gamma, wl, hp)
    torch.cuda.synchronize()
    w0, h0 = oracle.net_values(inst, model=model)
    deg = np.diff(inst.net_ptr)
    first = inst.net_ptr[:-1][deg > 0]
    gw, gh = host(wl)[first], host(hp)[first]
    rw, rh = w0[deg > 0], h0[deg > 0]
    # float32 pin coordinates relative to each net's first cell: a per-net
    # bound of 1e-5 of the net's size (or of gamma for a net of tiny extent)
    scale = np.maximum(np.abs(rh), inst.gamma)
    say("per-net max rel err W~ / HPWL", np.max(np.abs(gw - rw) / scale),
        np.max(np.abs(gh - rh) / scale))
    assert np.all(np.abs(gw - rw) <= 1e-5 * scale)
    assert np.all(np.abs(gh - rh) <= 1e-5 * scale)
    # entries at pins that are not a net's first pin are left alone
    other = np.ones(P, bool)
    other[first] = False
    assert np.all(host(wl)[other] == -1.0)


def test_unusable_index_or_workspace_is_refused(F):
    import torch
    a = gen.make_instance(51, num_cells=5000, util=0.7, n=128, num_nets=5500)
    b = gen.make_instance(52, num_cells=5000, util=0.7, n=128, num_nets=5500)
    pa, pb = F.Problem.from_instance(a), F.Problem.from_instance(b)
    plan = F.Plan(128)
    c = DeviceCells(a)
    gx = torch.empty(a.num_cells, device="cuda")
    gy = torch.empty(a.num_cells, device="cuda")
    out4 = torch.empty(4, dtype=torch.float64, device="cuda")
    # b's index in a's problem: same sizes, another netlist
    saved = (pa.c.xindex, pa.c.xindex_bytes, pa.c.xindex_key)
    pa.c.xindex, pa.c.xindex_bytes, pa.c.xindex_key = (pb.c.xindex, pb.c.xindex_bytes,
                                                        pb.c.xindex_key)
    for call in (lambda: F.eval(plan, pa, c.x, c.y, 1.0, a.gamma, "field", gx, gy, out4),
                 lambda: F.problem_wl_grad(pa, c.x, c.y, a.gamma, 0, gx, gy)):
        with pytest.raises(F.FFTPLError) as ei:
            call()
        assert ei.value.status == F.E_STATE
    pa.c.xindex, pa.c.xindex_bytes, pa.c.xindex_key = saved
    # a workspace one byte short: an error, not a silent change of path
    pa.c.work_bytes -= 1
    with pytest.raises(F.FFTPLError) as ei:
        F.eval(plan, pa, c.x, c.y, 1.0, a.gamma, "field", gx, gy, out4)
    assert ei.value.status == F.E_INVAL
    pa.c.work_bytes += 1
    F.eval(plan, pa, c.x, c.y, 1.0, a.gamma, "field", gx, gy, out4)
    torch.cuda.synchronize()
    ref = oracle.evaluate(a, lam=1.0, grad_mode="field")
    assert rel_l2(host(gx), ref["gx"]) < RTOL
    plan.close()


def _designs(n, count, seed):
    out = []
    for k in range(count):
        m = int(n * n * (0.3 + 0.6 * k / max(1, count - 1)))
        out.append(gen.make_instance((seed, k), num_cells=m, util=0.7, n=n,
                                     num_nets=int(1.1 * m), hi_frac=0.01,
                                     hi_range=(9, 100), num_macros=3 * (k % 2),
                                     macro_area_frac=0.1 if k % 2 else 0.0))
    return out


@pytest.mark.parametrize("dct,grad", [("fft", "field"), ("fft", "exact"),
                                      ("gemm_f32", "field"), ("gemm_f32", "exact"),
                                      ("gemm_bf16x3", "field")])
def test_batched_groups_equal_single_evaluations_bit_for_bit(F, dct, grad):
    # designs of one grid side evaluated in groups of up to max_batch per
    # launch give the same bits as one evaluation each (every sum is
    # order-independent), including a design that cannot join a group
    # (log-sum-exp model) and one on the slot path
    import torch
    n = 128
    insts = _designs(n, 6, 61)
    probs = [F.Problem.from_instance(i) for i in insts]
    probs[3] = F.Problem.from_instance(insts[3], wl_model="lse")
    probs[5] = F.Problem.from_instance(insts[5], path="slots")
    cells = [DeviceCells(i) for i in insts]
    lams = [0.5 + 0.25 * k for k in range(6)]
    gammas = [i.gamma for i in insts]
    plan = F.Plan(n, dct, max_batch=4)
    gxs = [torch.empty(i.num_cells, device="cuda") for i in insts]
    gys = [torch.empty(i.num_cells, device="cuda") for i in insts]
    out = torch.empty((6, 4), dtype=torch.float64, device="cuda")
    say("batch", dct, grad, [i.num_cells for i in insts])
    F.eval_batch(plan, probs, [c.x for c in cells], [c.y for c in cells], lams, gammas, grad,
                 gxs, gys, out)
    torch.cuda.synchronize()
    single = F.Plan(n, dct)
    for k, inst in enumerate(insts):
        gx = torch.empty(inst.num_cells, device="cuda")
        gy = torch.empty(inst.num_cells, device="cuda")
        o4 = torch.empty(4, dtype=torch.float64, device="cuda")
        F.eval(single, probs[k], cells[k].x, cells[k].y, lams[k], gammas[k], grad, gx, gy, o4)
        torch.cuda.synchronize()
        # gradients (fixed-point sums) and N, HPWL, tau (fixed-order partials of
        # float-exact terms) bit for bit; W~ to the last bits (the log-sum-exp
        # value is summed in double in an order set by the net blocks' work
        # counters)
        same = torch.equal(gx, gxs[k]) and torch.equal(gy, gys[k])
        idx = torch.tensor([0, 2, 3], device="cuda")
        same = same and torch.equal(o4[idx], out[k][idx])
        say("design", k, "bit-identical", same)
        assert same
        assert abs(float(o4[1]) - float(out[k][1])) <= 1e-12 * abs(float(o4[1]))
    # and one of the grouped designs against the oracle
    ref = oracle.evaluate(insts[1], lam=lams[1], grad_mode=grad)
    tol = 1e-4 if dct == "gemm_bf16x3" else RTOL   # split-bf16: reported, not gated at 1e-5
    assert rel_l2(host(gxs[1]), ref["gx"]) < tol and rel_l2(host(gys[1]), ref["gy"]) < tol
    assert abs(float(host(out[1])[0]) - ref["energy"]) < tol * abs(ref["energy"])
    single.close()
    plan.close()


def test_batched_scalars_only_and_full_groups(F):
    # eight designs in one group (the largest batch), scalars only
    import torch
    n = 64
    insts = _designs(n, 8, 71)
    probs = [F.Problem.from_instance(i) for i in insts]
    cells = [DeviceCells(i) for i in insts]
    plan = F.Plan(n, "fft", max_batch=8)
    out = torch.empty((8, 4), dtype=torch.float64, device="cuda")
    F.eval_batch(plan, probs, [c.x for c in cells], [c.y for c in cells], [1.0] * 8,
                 [i.gamma for i in insts], "field", None, None, out)
    torch.cuda.synchronize()
    o = host(out)
    for k, inst in enumerate(insts):
        ref = oracle.evaluate(inst, lam=1.0, grad_mode="field")
        assert abs(o[k][0] - ref["energy"]) < RTOL * abs(ref["energy"])
        assert abs(o[k][1] - ref["wa"]) < RTOL * abs(ref["wa"])
        assert abs(o[k][2] - ref["hpwl"]) < RTOL * abs(ref["hpwl"])
        assert abs(o[k][3] - ref["overflow"]) < RTOL
        # the group's maps: design k in batch slot k
        rho = host(plan.maps(k)[0])
        assert rel_l2(rho, ref["rho"]) < RTOL
    plan.close()
