"""Global placement loop: the device update and statistics kernels against
numpy, per-evaluation parity with the FP64 oracle at sampled iterations of a
1000-iteration Nesterov run on the 200k-cell workload, and checkpoint /
resume."""
import ctypes

import numpy as np
import pytest

import gen
import oracle
from _helpers import rel_l2
from tests.gpu_common import RTOL, dev, host, lib_or_build, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_or_build()
    from paper_1312_4587_amd import _lib, driver, fftpl
    return fftpl, driver, _lib


def test_update_and_statistics_kernels(F):
    import torch
    fftpl, driver, L = F
    lib = L.load()
    rng = np.random.default_rng(9)
    m = 50_001
    inst = gen.make_instance(9, num_cells=m, util=0.7, n=64, num_nets=10)
    grid = fftpl.Grid.of(inst)
    side = grid.n * grid.bin_w
    w = rng.integers(1, 5, m).astype(np.float32)
    h = np.ones(m, np.float32)
    w[0] = 2.0 * side                                   # wider than the region
    arr = {k: rng.uniform(-5, side + 5, m).astype(np.float32) for k in ("x", "y", "ux", "uy")}
    g = {k: rng.normal(0, 3, m).astype(np.float32) for k in ("gx", "gy", "gpx", "gpy")}
    up = {k: rng.uniform(0, side, m).astype(np.float32) for k in ("upx", "upy")}
    d = {k: dev(v) for k, v in {**arr, **g, **up, "w": w, "h": h}.items()}
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    work = torch.empty(1024, dtype=torch.float64, device="cuda")
    p = fftpl._ptr
    assert lib.fftpl_step_stats(m, p(d["ux"]), p(d["uy"]), p(d["upx"]), p(d["upy"]), p(d["gx"]),
                                p(d["gy"]), p(d["gpx"]), p(d["gpy"]), p(out), p(work), 1024,
                                None) == 0
    o = host(out)
    f64 = {k: v.astype(np.float64) for k, v in {**arr, **g, **up}.items()}
    assert o[0] == pytest.approx(np.sum((f64["ux"] - f64["upx"]) ** 2 + (f64["uy"] - f64["upy"]) ** 2), rel=1e-12)
    assert o[1] == pytest.approx(np.sum((f64["gx"] - f64["gpx"]) ** 2 + (f64["gy"] - f64["gpy"]) ** 2), rel=1e-12)
    assert o[2] == max(np.abs(g["gx"]).max(), np.abs(g["gy"]).max())
    assert o[3] == pytest.approx(np.sum(np.abs(f64["gx"]) + np.abs(f64["gy"])), rel=1e-12)
    step, beta = 0.37, 0.6
    assert lib.fftpl_nesterov_update(ctypes.byref(grid.c()), m, p(d["w"]), p(d["h"]), p(d["x"]),
                                     p(d["y"]), p(d["ux"]), p(d["uy"]), p(d["upx"]), p(d["upy"]),
                                     p(d["gpx"]), p(d["gpy"]), p(d["gx"]), p(d["gy"]), step, beta,
                                     None) == 0
    lo_x, hi_x = grid.xl + 0.5 * w, grid.xl + side - 0.5 * w
    lo_y, hi_y = grid.yl + 0.5 * h, grid.yl + side - 0.5 * h

    def clamp(v, lo, hi):
        return np.where(lo <= hi, np.minimum(np.maximum(v, lo), hi), 0.5 * (lo + hi))
    nx = clamp(f64["ux"] - step * f64["gx"], lo_x, hi_x)
    ny = clamp(f64["uy"] - step * f64["gy"], lo_y, hi_y)
    vx = clamp(nx + beta * (nx - f64["x"]), lo_x, hi_x)
    vy = clamp(ny + beta * (ny - f64["y"]), lo_y, hi_y)
    for name, ref in (("x", nx), ("y", ny), ("ux", vx), ("uy", vy)):
        assert np.max(np.abs(host(d[name]) - ref)) < 1e-4, name
    assert np.array_equal(host(d["upx"]), arr["ux"]) and np.array_equal(host(d["gpy"]), g["gy"])
    assert host(d["x"])[0] == pytest.approx(grid.xl + 0.5 * side)


def test_placement_run_mid_200k_parity_at_sampled_iterations(F):
    # 1000 Nesterov iterations with lambda doubling every 50; at k = 0, 1, 10,
    # 100, 999 the evaluation at the look-ahead point is checked against the
    # oracle on the same positions, and the overflow must fall
    import torch
    fftpl, driver, _ = F
    inst = gen.make_config("mid_200k")
    pl = driver.Placer(inst)
    snaps = {}

    def grab(p):
        if p.k in (0, 1, 10, 100, 999):
            snaps[p.k] = dict(x=host(p.ux), y=host(p.uy), gx=host(p.gx), gy=host(p.gy),
                              s=host(p.scal)[:4].copy(), lam=p.lam, gamma=p.gamma)
    import time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = pl.run(1000, on_eval=grab)
    torch.cuda.synchronize()
    say("1000 iterations", time.perf_counter() - t0, "s; tau", hist[0]["tau"], "->",
        hist[-1]["tau"], "hpwl", hist[0]["hpwl"], "->", hist[-1]["hpwl"])
    assert len(hist) == 1000
    assert hist[-1]["tau"] < 0.5 * hist[0]["tau"]
    assert hist[-1]["hpwl"] < 0.6 * hist[0]["hpwl"]
    assert all(np.isfinite(h["hpwl"]) and h["hpwl"] > 0 for h in hist)
    for k, sn in sorted(snaps.items()):
        ik = inst.with_positions(sn["x"], sn["y"])
        ref = oracle.evaluate(ik, lam=sn["lam"], gamma=sn["gamma"], grad_mode="field")
        N, W, H, tau = sn["s"]
        e = rel_l2(np.concatenate([sn["gx"], sn["gy"]]), np.concatenate([ref["gx"], ref["gy"]]))
        say("k", k, "grad rel-L2", e, "tau", tau, ref["overflow"])
        assert e < RTOL
        assert abs(N - ref["energy"]) <= RTOL * abs(ref["energy"])
        assert abs(W - ref["wa"]) <= RTOL * abs(ref["wa"])
        assert abs(H - ref["hpwl"]) <= RTOL * abs(ref["hpwl"])
        assert abs(tau - ref["overflow"]) <= RTOL
    pl.close()


def test_checkpoint_and_resume(F, tmp_path):
    # a saved state reloads bit for bit, and the step taken from it is the
    # step the original run takes, bit for bit: every sum of the evaluation
    # and of the step statistics is order-independent (fixed-point LDS adds,
    # fixed-order block partials)
    fftpl, driver, _ = F
    inst = gen.make_config("mid_200k")
    b = driver.Placer(inst)
    b.run(20)
    path = str(tmp_path / "ckpt.npz")
    b.save(path)
    s20 = b.state()
    b.step()
    s21 = b.state()
    b.close()
    c = driver.Placer(inst)
    c.load(path)
    r20 = c.state()
    for name in ("x", "y", "ux", "uy", "upx", "upy", "gpx", "gpy", "scalars", "history"):
        assert np.array_equal(r20[name], s20[name]), name
    assert c.k == 20 and len(c.history) == 20
    c.step()
    r21 = c.state()
    c.close()
    for name in ("x", "y", "ux", "uy", "gpx", "gpy", "scalars"):
        say("one step after resume", name, rel_l2(r21[name], s21[name]))
        assert np.array_equal(r21[name], s21[name]), name
    assert np.allclose(r21["history"], s21["history"], rtol=1e-6, atol=0.0)


def test_fillers_and_irregular_region(F):
    # an L-shaped region: the box's top-right quadrant is not placeable (one
    # dark node, charged like a fixed node); fillers fill the capacity left.
    # Cells start uniformly over the whole box.  Checked: the dark node's
    # fixed map, per-evaluation parity of the full (real + filler) evaluation
    # and of the real cells' overflow against the oracle, and that the density
    # force empties the dark quadrant.
    import dataclasses
    fftpl, driver, _ = F
    inst = gen.make_instance(21, num_cells=30_000, util=0.5, n=128, num_nets=32_000)
    side = inst.n * inst.bin_w
    xl, yl = inst.xl, inst.yl
    half = 0.5 * side
    d = fftpl.dark_nodes(xl, yl, xl + side, yl + side,
                         [[xl, yl, xl + side, yl + half], [xl, yl + half, xl + half, yl + side]])
    assert d.shape == (1, 4)
    mac = np.stack([(d[:, 0] + d[:, 2]) / 2, (d[:, 1] + d[:, 3]) / 2, d[:, 2] - d[:, 0],
                    d[:, 3] - d[:, 1]], axis=1).astype(np.float32)
    inst = dataclasses.replace(inst, fx=mac[:, 0], fy=mac[:, 1], fw=mac[:, 2], fh=mac[:, 3])
    pl = driver.Placer(inst, fillers=True, filler_seed=5)
    m, nf = pl.num_real, pl.num_fillers
    cap_area = float(host(pl.prob_real.arrays["cap"]).astype(np.float64).sum()) * inst.bin_w ** 2
    filler_area = nf * float(np.mean(inst.w)) * float(np.mean(inst.h))
    say("fillers", nf, "cap area", cap_area, "movable", float(np.sum(inst.w * inst.h)))
    assert nf > 0
    assert 0 <= cap_area - float(np.sum(inst.w * inst.h)) - filler_area < np.mean(inst.w)
    # the dark quadrant carries rho_t and leaves no capacity
    base = host(pl.prob.arrays["base"]).reshape(inst.n, inst.n)
    h2 = inst.n // 2
    assert np.max(np.abs(base[h2:, h2:] - 1.0)) < 1e-4
    assert np.max(np.abs(base[:h2])) < 1e-4 and np.max(np.abs(base[:, :h2])) < 1e-4

    def dark_area(x, y):
        sel = (x > xl + half) & (y > yl + half)
        return float(np.sum(inst.w[sel] * inst.h[sel]))
    a0 = dark_area(inst.x, inst.y)
    snaps = {}

    def grab(p):
        if p.k in (0, 150):
            snaps[p.k] = dict(x=host(p.ux), y=host(p.uy), gx=host(p.gx), gy=host(p.gy),
                              s=host(p.scal).copy(), lam=p.lam, gamma=p.gamma)
    hist = pl.run(400, on_eval=grab)
    x, y = pl.positions()
    a1 = dark_area(x, y)
    say("dark-quadrant cell area", a0, "->", a1, "tau", hist[0]["tau"], "->", hist[-1]["tau"])
    assert a1 < 0.5 * a0
    assert hist[-1]["tau"] < hist[0]["tau"]
    whole = pl.inst
    for k, sn in sorted(snaps.items()):
        ik = whole.with_positions(sn["x"], sn["y"])
        ref = oracle.evaluate(ik, lam=sn["lam"], gamma=sn["gamma"], grad_mode="field")
        e = rel_l2(np.concatenate([sn["gx"], sn["gy"]]), np.concatenate([ref["gx"], ref["gy"]]))
        real = dataclasses.replace(inst.with_positions(sn["x"][:m], sn["y"][:m]),
                                   net_ptr=np.zeros(1, np.int32), pin_cell=np.zeros(0, np.int32),
                                   pin_dx=np.zeros(0, np.float32), pin_dy=np.zeros(0, np.float32))
        rref = oracle.evaluate(real, lam=sn["lam"], gamma=sn["gamma"], grad_mode="field")
        say("k", k, "grad rel-L2", e, "tau all / real", sn["s"][3], ref["overflow"], sn["s"][11],
            rref["overflow"])
        assert e < RTOL
        assert abs(sn["s"][0] - ref["energy"]) <= RTOL * abs(ref["energy"])
        assert abs(sn["s"][3] - ref["overflow"]) <= RTOL
        assert abs(sn["s"][8] - rref["energy"]) <= RTOL * abs(rref["energy"])
        assert abs(sn["s"][11] - rref["overflow"]) <= RTOL
        assert sn["s"][9] == 0.0 and sn["s"][10] == 0.0      # no nets among the real-only cells
    pl.close()


@pytest.mark.parametrize("wl,eps", [("lse", 0.0), ("wa", 0.1)])
def test_placement_with_objective_variants(F, wl, eps):
    # the loop with the log-sum-exp model or the screened solve: parity of
    # the evaluation at a sampled iteration, and a falling wirelength (the
    # random start is already spread out: a screened, short-range density
    # force lets the overflow rise while the wirelength shrinks)
    fftpl, driver, _ = F
    inst = gen.make_instance(22, num_cells=20_000, util=0.7, n=128, num_nets=21_000)
    pl = driver.Placer(inst, schedule=driver.Schedule(wl_model=wl, screening=eps))
    snap = {}

    def grab(p):
        if p.k == 60:
            snap.update(x=host(p.ux), y=host(p.uy), gx=host(p.gx), gy=host(p.gy),
                        s=host(p.scal)[:4].copy(), lam=p.lam, gamma=p.gamma)
    hist = pl.run(200, on_eval=grab)
    say(wl, eps, "tau", hist[0]["tau"], "->", hist[-1]["tau"], "hpwl", hist[0]["hpwl"], "->",
        hist[-1]["hpwl"])
    ik = inst.with_positions(snap["x"], snap["y"])
    ref = oracle.evaluate(ik, lam=snap["lam"], gamma=snap["gamma"], grad_mode="field",
                          wl_model=wl, eps=eps)
    e = rel_l2(np.concatenate([snap["gx"], snap["gy"]]), np.concatenate([ref["gx"], ref["gy"]]))
    say("grad rel-L2", e)
    assert e < RTOL
    assert abs(snap["s"][0] - ref["energy"]) <= RTOL * abs(ref["energy"])
    assert abs(snap["s"][1] - ref["wa"]) <= RTOL * abs(ref["wa"])
    # (a screened solve spreads cells less: with eps = 0.1 bin^-2 the
    # wirelength falls by only ~10% over these iterations)
    assert all(np.isfinite(h["hpwl"]) for h in hist)
    assert hist[-1]["hpwl"] < hist[0]["hpwl"] and hist[-1]["tau"] < 0.5
    pl.close()


def test_cg_kernels_against_numpy(F):
    # the vector steps of the CG inner solver: dots, direction, clamped move
    import torch
    fftpl, driver, L = F
    lib = L.load()
    rng = np.random.default_rng(19)
    m = 40_001
    inst = gen.make_instance(19, num_cells=m, util=0.7, n=64, num_nets=10)
    grid = fftpl.Grid.of(inst)
    side = grid.n * grid.bin_w
    v = {k: rng.normal(0, 3, m).astype(np.float32)
         for k in ("gx", "gy", "gpx", "gpy", "dx", "dy")}
    x = rng.uniform(0, side, m).astype(np.float32)
    y = rng.uniform(0, side, m).astype(np.float32)
    w = rng.integers(1, 5, m).astype(np.float32)
    h = np.ones(m, np.float32)
    d = {k: dev(a) for k, a in {**v, "x": x, "y": y, "w": w, "h": h}.items()}
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    work = torch.empty(1024, dtype=torch.float64, device="cuda")
    p = fftpl._ptr
    assert lib.fftpl_cg_dots(m, p(d["gx"]), p(d["gy"]), p(d["gpx"]), p(d["gpy"]), p(d["dx"]),
                             p(d["dy"]), p(out), p(work), 1024, None) == 0
    f = {k: a.astype(np.float64) for k, a in v.items()}
    o = host(out)
    assert o[0] == pytest.approx(np.sum(f["gx"] ** 2 + f["gy"] ** 2), rel=1e-12)
    assert o[1] == pytest.approx(np.sum(f["gx"] * f["gpx"] + f["gy"] * f["gpy"]), rel=1e-12)
    assert o[2] == pytest.approx(np.sum(f["gpx"] ** 2 + f["gpy"] ** 2), rel=1e-12)
    assert o[3] == pytest.approx(np.sum(f["gx"] * f["dx"] + f["gy"] * f["dy"]), rel=1e-12)
    assert lib.fftpl_cg_dots(m, p(d["gx"]), p(d["gy"]), None, None, None, None, p(out),
                             p(work), 1024, None) == 0
    o = host(out)
    assert o[1] == 0.0 and o[2] == 0.0 and o[3] == 0.0
    beta = 0.625
    dmax = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert lib.fftpl_cg_direction(m, p(d["gx"]), p(d["gy"]), beta, p(d["dx"]), p(d["dy"]),
                                  p(dmax), p(work), 1024, None) == 0
    # (the device may fuse beta * d - g into one rounding)
    rx = (beta * f["dx"] - f["gx"]).astype(np.float32)
    ry = (beta * f["dy"] - f["gy"]).astype(np.float32)
    gdx, gdy = host(d["dx"]), host(d["dy"])
    assert np.max(np.abs(gdx - rx)) <= 1e-6 * np.abs(rx).max()
    assert np.max(np.abs(gdy - ry)) <= 1e-6 * np.abs(ry).max()
    assert float(host(dmax)[0]) == max(np.abs(gdx).max(), np.abs(gdy).max())
    t = 0.75
    assert lib.fftpl_cg_move(ctypes.byref(grid.c()), m, p(d["w"]), p(d["h"]), p(d["x"]),
                             p(d["y"]), p(d["dx"]), p(d["dy"]), t, p(d["x"]), p(d["y"]),
                             None) == 0
    lo, hi = grid.xl + 0.5 * w, grid.xl + side - 0.5 * w
    ex = np.minimum(np.maximum(x + np.float32(t) * gdx, lo), hi)
    assert np.max(np.abs(host(d["x"]) - ex)) < 1e-4
    assert lib.fftpl_cg_direction(m, p(d["gx"]), p(d["gy"]), -1.0, p(d["dx"]), p(d["dy"]),
                                  p(dmax), p(work), 1024, None) == -1


def test_cg_paper_schedule_mid_200k(F):
    # Algorithm 1 as printed on the 200k-cell workload: nonlinear CG with the
    # line search inside [alpha_min, alpha_max], lambda_k = mu_k lambda_(k-1)
    # from the HPWL change, gamma(tau), stop once tau <= 10%.  The evaluation
    # at sampled iterations matches the oracle on the same positions, and the
    # energy N falls together with tau (the paper's Fig. 3(a))
    import json
    import os
    import time
    import torch
    fftpl, driver, _ = F
    inst = gen.make_config("mid_200k")
    pl = driver.Placer(inst, schedule=driver.paper_schedule())
    snaps = {}
    pick = {0, 1, 10, 50, 100, 200}

    def grab(p):
        if p.k in pick:
            snaps[p.k] = dict(x=host(p.ux), y=host(p.uy), gx=host(p.gx), gy=host(p.gy),
                              s=host(p.scal)[:4].copy(), lam=p.lam, gamma=p.gamma)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = pl.run(1000, on_eval=grab)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    say("CG, paper schedule:", len(hist), "iterations in", dt, "s; tau", hist[0]["tau"], "->",
        hist[-1]["tau"], "hpwl", hist[0]["hpwl"], "->", hist[-1]["hpwl"], "trials",
        sum(h["trials"] for h in hist))
    out = os.environ.get("FFTPL_TRACE_OUT")
    if out:
        with open(out, "w") as f:
            for h in hist:
                f.write(json.dumps({k: h[k] for k in ("k", "energy", "tau", "hpwl", "wa", "lam",
                                                      "gamma", "alpha", "trials")}) + "\n")
    assert hist[-1]["tau"] <= 0.1 and len(hist) < 1000       # stopped by the criterion
    assert all(h["alpha"] >= 0 and np.isfinite(h["hpwl"]) for h in hist)
    taus = np.array([h["tau"] for h in hist])
    ens = np.array([h["energy"] for h in hist])
    assert ens[-1] < ens[0] and taus[-1] < taus[0]
    # N tracks tau: rank correlation over the run
    rt = np.argsort(np.argsort(taus))
    re = np.argsort(np.argsort(ens))
    rho_s = np.corrcoef(rt, re)[0, 1]
    say("rank correlation of N and tau", rho_s)
    assert rho_s > 0.8
    last = hist[-1]["k"]
    for k, sn in sorted(snaps.items()):
        ik = inst.with_positions(sn["x"], sn["y"])
        ref = oracle.evaluate(ik, lam=sn["lam"], gamma=sn["gamma"], grad_mode="field")
        N, W, H, tau = sn["s"]
        e = rel_l2(np.concatenate([sn["gx"], sn["gy"]]), np.concatenate([ref["gx"], ref["gy"]]))
        say("k", k, "of", last, "grad rel-L2", e, "tau", tau, ref["overflow"])
        assert e < RTOL
        assert abs(N - ref["energy"]) <= RTOL * abs(ref["energy"])
        assert abs(W - ref["wa"]) <= RTOL * abs(ref["wa"])
        assert abs(tau - ref["overflow"]) <= RTOL
    pl.close()


@pytest.mark.parametrize("lam_mode", ["double", "paper"])
def test_device_loop_matches_host_loop(F, lam_mode):
    # The schedule on the device (fftpl_nesterov_schedule, eval with lambda
    # and gamma read on the device, update with step and beta read there)
    # follows the host loop: same histories and positions.  Enqueued and
    # graph-replayed device loops run the same kernels on the same inputs:
    # the same bits.  The lambda rule crosses a doubling (with the momentum
    # restart) or applies mu_k every iteration.
    import torch
    fftpl, driver, _ = F
    inst = gen.make_instance(61, num_cells=40_000, util=0.8, n=256, num_nets=42_000,
                             hi_frac=0.01, hi_range=(20, 200), num_macros=5,
                             macro_area_frac=0.1)
    iters = 16
    sched = driver.Schedule(lam_mode=lam_mode, lam_every=6)
    runs = {}
    for how in ("host", "device", "graph"):
        pl = driver.Placer(inst, schedule=sched)
        if how == "host":
            pl.run(iters)
        else:
            pl.run_device(iters, graph=(how == "graph"))
        torch.cuda.synchronize()
        runs[how] = (pl.history, host(pl.x), host(pl.y), pl.k, pl.lam, pl.gamma, pl.a)
        say(how, pl.k, pl.lam, pl.gamma, pl.history[-1])
        pl.close()
    hh, dh, gh = runs["host"][0], runs["device"][0], runs["graph"][0]
    assert len(hh) == len(dh) == len(gh) == iters
    assert [r["k"] for r in dh] == list(range(iters))
    for a, b in zip(dh, gh):
        assert a == b
    assert np.array_equal(runs["device"][1], runs["graph"][1])
    assert np.array_equal(runs["device"][2], runs["graph"][2])
    # host vs device: the same rule in double; pow may round differently in
    # the last bit, which float32 gamma almost always absorbs
    for a, b in zip(hh, dh):
        for key in ("energy", "wa", "hpwl", "tau", "lam", "gamma", "alpha"):
            assert b[key] == pytest.approx(a[key], rel=1e-5, abs=1e-12), (a["k"], key)
    if lam_mode == "double":
        lams = [r["lam"] for r in dh]
        assert lams[6] == 2.0 * lams[5] and lams[12] == 2.0 * lams[11]
    assert runs["device"][3] == runs["host"][3] == iters
    side = inst.n * inst.bin_w
    for i in (1, 2):
        assert np.max(np.abs(runs["device"][i] - runs["host"][i])) < 1e-4 * side
    # the loop state handed back to the host continues like a host-only run
    assert runs["device"][4] == pytest.approx(runs["host"][4], rel=1e-6)
    assert runs["device"][5] == pytest.approx(runs["host"][5], rel=1e-5)
    assert runs["device"][6] == pytest.approx(runs["host"][6], rel=1e-12)


def test_eval_params_matches_eval(F):
    # lambda and gamma read on the device give the bits of the host-argument
    # evaluation; paths other than the exchange are refused
    import torch
    fftpl, driver, _ = F
    inst = gen.make_instance(62, num_cells=30_000, util=0.8, n=128, num_nets=33_000,
                             hi_frac=0.01, hi_range=(20, 200))
    prob = fftpl.Problem.from_instance(inst)
    plan = fftpl.Plan(inst.n)
    x, y = dev(inst.x), dev(inst.y)
    m = inst.num_cells
    lam, gamma = 0.731, float(inst.gamma) * 1.37
    for wl in ("wa", "lse"):
        prob.set_objective(wl_model=wl)
        g1 = [torch.empty(m, device="cuda") for _ in range(2)]
        g2 = [torch.empty(m, device="cuda") for _ in range(2)]
        o1 = torch.zeros(4, dtype=torch.float64, device="cuda")
        o2 = torch.zeros(4, dtype=torch.float64, device="cuda")
        fftpl.eval(plan, prob, x, y, lam, gamma, "field", g1[0], g1[1], o1)
        params = torch.tensor([lam, gamma], dtype=torch.float32, device="cuda")
        fftpl.eval_params(plan, prob, x, y, params, "field", g2[0], g2[1], o2)
        torch.cuda.synchronize()
        assert torch.equal(g1[0], g2[0]) and torch.equal(g1[1], g2[1]), wl
        assert torch.equal(o1, o2), wl
    slots = fftpl.Problem.from_instance(inst, path="slots")
    with pytest.raises(fftpl.FFTPLError) as ei:
        fftpl.eval_params(plan, slots, x, y, params, "field", g2[0], g2[1], o2)
    assert ei.value.status == fftpl.E_UNSUPPORTED
    plan.close()


def test_device_loop_graph_replays_match_eager_each_time(F):
    # every replay of the captured iteration, with the program's own eager
    # work and synchronisations between replays, gives the bits of the same
    # iteration enqueued directly
    import torch
    fftpl, driver, _ = F
    inst = gen.make_instance(63, num_cells=25_000, util=0.8, n=128, num_nets=27_000,
                             hi_frac=0.01, hi_range=(20, 200))
    snaps = {}
    for graph in (False, True):
        pl = driver.Placer(inst, schedule=driver.Schedule(lam_every=3))
        seen = []

        def between(i):
            torch.cuda.synchronize()
            junk = torch.randn(4096, device="cuda")
            junk.mul_(2.0).sum().item()          # eager device work between replays
            seen.append((host(pl.x), host(pl.y), host(pl.gx), host(pl.scal)))
        pl.run_device(8, graph=graph, between=between)
        snaps[graph] = seen
        pl.close()
    assert len(snaps[False]) == len(snaps[True]) == 7
    for i, (a, b) in enumerate(zip(snaps[False], snaps[True])):
        for u, v in zip(a, b):
            assert np.array_equal(u, v), i


def test_periodic_checkpoint_and_trace(F, tmp_path):
    # run() with a JSON-lines trace and a checkpoint every 5 iterations: the
    # trace holds every iteration's record as the history does; the last
    # checkpoint (after iteration 12) resumes into the same next step; the
    # device loop appends its records to a trace the same way
    import json
    fftpl, driver, _ = F
    inst = gen.make_instance(64, num_cells=20_000, util=0.8, n=128, num_nets=22_000)
    trace = str(tmp_path / "trace.jsonl")
    ckpt = str(tmp_path / "ckpt.npz")
    a = driver.Placer(inst)
    a.run(12, trace=trace, checkpoint=ckpt, checkpoint_every=5)
    recs = [json.loads(line) for line in open(trace)]
    assert [r["k"] for r in recs] == list(range(12))
    for r, h in zip(recs, a.history):
        for key in ("energy", "wa", "hpwl", "tau", "lam", "gamma", "alpha"):
            assert r[key] == h[key], key
    a.step()
    nxt = a.history[-1]
    a.close()
    b = driver.Placer(inst)
    b.load(ckpt)
    assert b.k == 12
    b.step()
    for key in ("energy", "wa", "hpwl", "tau", "alpha"):
        assert b.history[-1][key] == pytest.approx(nxt[key], rel=1e-6), key
    dtrace = str(tmp_path / "device.jsonl")
    b.run_device(4, trace=dtrace)
    drecs = [json.loads(line) for line in open(dtrace)]
    assert [r["k"] for r in drecs] == [13, 14, 15, 16]
    b.close()
