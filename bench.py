"""Benchmark of one FFTPL evaluation (density -> spectral solve -> gradients).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large_2m]
                [--dct fft|gemm_f32|gemm_bf16x3] [--no-cpu-baseline]

A step is one full fftpl_eval over the workload's positions, inputs resident
in HBM: scatter, the FFT Poisson solve, field gather, WA wirelength, and the
FP64 energy / wirelength / HPWL / overflow reductions.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("cell-gradient evals/s at 2M cells n=1024 (plain vs split-BF16); "
          "served p50/p99")
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0

# HBM traffic per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (KiB per
# dispatch) on the 2.1M-cell workload, scaled by what the same counters read
# for a plain 256 MiB device copy in the same run (FETCH_SIZE x2.0, WRITE_SIZE
# x1.0).  Each entry records the SHA-1 of the kernel's source files when the
# counters were taken; once they change the figure is stale and the report
# gives null.
PMC_FETCH_SCALE, PMC_WRITE_SCALE = 2.0, 1.0
PMC_TRAFFIC = {
    # kernel: (source files, sha1, FETCH_SIZE KiB, WRITE_SIZE KiB)
    "k_band_place": (("band_scatter.hip", "fftpl_internal.hpp"),
        "363d6c18c810a50f8ba1358a41d225290199574c", 16523.6, 64791.1),
    "k_xch_spread": (("exchange.hip", "fftpl_internal.hpp"),
        "aa1810760312d0fe8d4d95a86c95e7764cd01c4a", 28609.1, 96907.1),
    "k_band_accum": (("band_scatter.hip", "fftpl_internal.hpp"),
        "363d6c18c810a50f8ba1358a41d225290199574c", 27911.0, 4096.0),
    "k_xch_wa": (("exchange.hip", "fftpl_internal.hpp"),
        "aa1810760312d0fe8d4d95a86c95e7764cd01c4a", 178984.5, 112289.7),
    "k_rows_dct2": (("spectral_fft.hip", "fftpl_internal.hpp"),
        "63506664793af2e33294635574c5e783f13c917a", 6235.8, 4112.0),
    "k_cols_solve": (("spectral_fft.hip", "fftpl_internal.hpp"),
        "63506664793af2e33294635574c5e783f13c917a", 2180.6, 8192.0),
    "k_rows_inverse": (("spectral_fft.hip", "fftpl_internal.hpp"),
        "63506664793af2e33294635574c5e783f13c917a", 6264.1, 8196.0),
    "k_band_gather": (("band_scatter.hip", "fftpl_internal.hpp"),
        "363d6c18c810a50f8ba1358a41d225290199574c", 30994.6, 21000.0),
    "k_xch_cellsum": (("exchange.hip", "fftpl_internal.hpp"),
        "aa1810760312d0fe8d4d95a86c95e7764cd01c4a", 80868.2, 16406.5),
}


def pmc_traffic(kernel):
    """Scaled HBM bytes per launch of `kernel`, or None if not measured or stale."""
    import hashlib
    rec = PMC_TRAFFIC.get(kernel)
    if rec is None:
        return None
    srcs, sha, fetch_kib, write_kib = rec
    h = hashlib.sha1()
    for src in srcs:
        with open(os.path.join(ROOT, "paper_1312_4587_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != sha:
        return None
    return (PMC_FETCH_SCALE * fetch_kib + PMC_WRITE_SCALE * write_kib) * 1024.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="large_2m")
    ap.add_argument("--dct", default="fft")
    ap.add_argument("--variants", default="fft,gemm_f32,gemm_bf16x3",
                    help="spectral variants to time besides --dct")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-evals", type=int, default=3)
    ap.add_argument("--kernel-reps", type=int, default=0,
                    help="evaluations timed kernel by kernel (default max(10, steps/4))")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the per-variant error report against the FP64 oracle")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--no-standalone", action="store_true",
                    help="skip timing the standalone entry points")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the serving, placement-loop and differentiation runs")
    ap.add_argument("--serve-requests", type=int, default=5000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-pool", type=int, default=32)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-batch", type=int, default=8,
                    help="most requests of one grid side evaluated in one group")
    ap.add_argument("--serve-variants", type=int, default=4,
                    help="placements per design (request r uses placement r mod this)")
    ap.add_argument("--serve-saturate", type=int, default=2000,
                    help="requests of the saturated run (arrivals far above the "
                         "service rate), with and without grouping; 0 skips it")
    ap.add_argument("--driver-iters", type=int, default=1000)
    return ap.parse_args()


def serving_run(args, dct, count, rate=None, max_batch=None):
    """The serving workload: Poisson arrivals at `rate` (default --serve-rate)
    of placements of designs with 10^4..10^6 cells (log-uniform, a pool of
    --serve-pool designs made resident before the stream starts, --serve-variants
    placements each); requests of one grid side waiting together are
    evaluated in groups of up to `max_batch` (one launch per stage); latency
    from arrival to results in host memory."""
    import numpy as np

    import gen
    from paper_1312_4587_amd import serving
    rate = args.serve_rate if rate is None else rate
    mb = args.serve_batch if max_batch is None else max_batch
    pool = gen.serving_pool(args.serve_pool, seed=5)
    arrivals, designs = gen.serving_stream(count, rate_hz=rate, pool_size=len(pool), seed=5)
    variants = np.arange(count) % args.serve_variants
    ex = serving.DeviceExecutor(pool, slots=args.serve_slots, dct=dct, max_batch=mb,
                                variants=args.serve_variants)
    t0 = time.perf_counter()
    ex.warm(load_designs=True)
    load_s = time.perf_counter() - t0
    srv = serving.Server(ex, ex.footprint, slots=args.serve_slots, capacity_bytes=200e9,
                         grid=ex.grid, max_batch=mb)
    st = srv.run(arrivals, designs, variants)
    ex.close()
    cells = [p.num_cells for p in pool]
    st.update(dct=dct, rate_hz=rate, slots=args.serve_slots, max_batch=mb,
              pool=len(pool), pool_cells_min=int(min(cells)), pool_cells_max=int(max(cells)),
              capacity_bytes=200e9, designs_loaded=ex.loads,
              design_load_s=load_s, design_load_ms_mean=1e3 * ex.load_s / max(1, ex.loads))
    return st


def driver_run(args):
    """The placement loop on the 200k-cell workload: Nesterov iterations with
    lambda doubling every 50, each one full evaluation plus the update; once
    with the schedule on the host (one read of the scalars per iteration) and
    once with the schedule on the device, replayed from a HIP graph."""
    import gen
    import torch
    from paper_1312_4587_amd import driver
    inst = gen.make_config("mid_200k")
    out = {"workload": "mid_200k", "cells": inst.num_cells, "grid_n": inst.n}
    for how in ("host", "device_graph"):
        pl = driver.Placer(inst)
        pl.step()                  # lambda_0 and the first step outside the timing
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if how == "host":
            hist = pl.run(args.driver_iters - 1)
        else:
            hist = pl.run_device(args.driver_iters - 1, graph=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        pl.close()
        pick = [h for h in hist if h["k"] in (0, 1, 10, 100, 200, 500, args.driver_iters - 1)]
        leg = {"iterations": len(hist), "ms_per_iteration": 1e3 * dt / max(1, len(hist) - 1),
               "iterations_per_s": (len(hist) - 1) / dt,
               "trajectory": [{k: h[k] for k in ("k", "tau", "hpwl", "lam", "gamma")}
                              for h in pick]}
        if how == "host":
            out.update(leg)        # the host-scheduled loop keeps the top-level keys
        else:
            leg["note"] = "schedule on the device, one iteration captured in a HIP graph " \
                          "and replayed (the capture is inside the timing)"
            out["device_schedule"] = leg
    return out


def autograd_run():
    """The differentiation workload: W~ + lambda N through the autograd
    function on 500k cells, n = 512 (backward recomputes the solve)."""
    import gen
    import torch
    from paper_1312_4587_amd import autograd, fftpl
    inst = gen.make_config("diff_500k")
    prob = fftpl.Problem.from_instance(inst)
    plan = fftpl.Plan(inst.n, "fft")
    x = torch.as_tensor(inst.x).cuda().requires_grad_(True)
    y = torch.as_tensor(inst.y).cuda().requires_grad_(True)
    for _ in range(3):
        loss, _ = autograd.objective(x, y, plan, prob, 1.0, inst.gamma)
        loss.backward()
    reps = 20
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tf = tb = 0.0
    for _ in range(reps):
        x.grad = None
        y.grad = None
        ev[0].record()
        loss, _ = autograd.objective(x, y, plan, prob, 1.0, inst.gamma)
        ev[1].record()
        loss.backward()
        ev[2].record()
        torch.cuda.synchronize()
        tf += ev[0].elapsed_time(ev[1])
        tb += ev[1].elapsed_time(ev[2])
    plan.close()
    return {"workload": "diff_500k", "cells": inst.num_cells, "grid_n": inst.n,
            "forward_ms": tf / reps, "backward_ms": tb / reps,
            "saved_tensors": "positions only (backward recomputes density and solve)"}


def band_entries(inst):
    """Number of (cell, band) entries the banded scatter lists: bookkeeping
    for the byte counts only (float32 edges, bands of ceil(n/256) rows)."""
    import numpy as np
    inv = np.float32(1.0 / inst.bin_h)
    c = (inst.y.astype(np.float32) - np.float32(inst.yl)) * inv
    half = np.float32(0.5) * (inst.h.astype(np.float32) * inv)
    lo = np.clip(c - half, 0, inst.n)
    hi = np.clip(c + half, -1, inst.n)
    i0 = np.floor(lo).astype(np.int64)
    i1 = np.ceil(hi).astype(np.int64) - 1
    rows = (inst.n + 255) // 256
    ok = i1 >= i0
    return int(np.sum(np.where(ok, i1 // rows - i0 // rows + 1, 0)))


def kernel_bytes(inst, nent):
    """Design bytes per launch of every kernel of the atomic-free evaluation:
    each array the kernel's own layout reads or writes, once (index arrays,
    the exchange buffer and the 16-byte band records included).  These are
    not the compulsory bytes of stage_bytes."""
    import numpy as np
    m, E, P, n2 = inst.num_cells, inst.num_nets, inst.num_pins, inst.n ** 2
    deg = np.diff(inst.net_ptr.astype(np.int64))
    p_big = int(deg[deg > 8].sum())
    p_small = P - p_big
    return {
        "k_init_eval": 0,
        # pins (cell, dx, dy) in, per-pin gradient out, net_ptr; positions once
        "k_wa_slots_small": 12 * p_small + 8 * p_small + 4 * (E + 1) + 8 * m,
        "k_wa_slots_big": 12 * p_big + 8 * p_big + 4 * (E + 1),
        "k_interleave": 8 * m + 8 * m,
        # cells in; entries, each cell's first entry and the per-(band, block)
        # slice offsets and counts out (4096 cells per block)
        "k_band_place": 16 * m + 16 * nent + 4 * m
        + 8 * (-(-inst.n // (-(-inst.n // 256))) + 1) * (-(-m // 4096)),
        "k_band_accum": 16 * nent + 4 * n2 + 4 * n2,
        "k_rows_dct2": 4 * n2 + 4 * n2 + 8 * n2,        # rho, base+cap in; bT out
        "k_cols_solve": 4 * n2 + 8 * n2,                # bT in; P, Q out
        "k_rows_inverse": 8 * n2 + 4 * n2 + 8 * n2,     # P, Q, rho in; (Ex, Ey) out
        "k_gather_pins": 16 * m + 8 * n2 + 4 * (m + 1) + 8 * P + 8 * m,
        # exchange path: u16 cell offsets and float2 pin records in A order,
        # int32 A positions and u16 CSR offsets in B order
        "k_xch_spread": 8 * m + 2 * P + 8 * P,
        "k_xch_wa": 4 * P + 2 * P + 8 * P + 8 * P + 8 * P + 4 * (E + 1) + 2 * E,
        "k_gather_xch": 16 * m + 8 * n2 + 4 * (m + 1) + 4 * P + 8 * P + 8 * m,
        # cell-block windows of T with their u16 cell-local indices; each
        # cell's entry position and density gradient in, its gradient out
        "k_xch_cellsum": 2 * P + 8 * P + 4 * m + 8 * m + 8 * m,
        # band entries in, the field rows of each band once, one gradient per
        # first-band entry out
        "k_band_gather": 16 * nent + 8 * n2 + 8 * m,
        "k_eval_finalize": 0,
    }


def gemm_flops(n):
    """Multiply-add flops (2 per MAC) each step of the matrix-core solve
    executes (field mode).  With n a multiple of 128 the products are split
    into even and odd frequencies: [Sx Ke^T | Dx Ko^T] and [Ke Sy ; Ko Dy]
    (2 x n (n/2)^2 MACs each), U and V (4 x n (n/2)^2), psi, Ey and Ex (6 x n
    (n/2)^2), 3.5 n^3 MACs in all; otherwise the five dense products, 7 n^3."""
    if n % 128 == 0:
        return {"k_gemm_w": n ** 3, "k_gemm_g": n ** 3, "k_gemm_uv": 2 * n ** 3,
                "k_gemm_psi_ey": 3 * n ** 3}
    return {"k_gemm_w": 2 * n ** 3, "k_gemm_g": 2 * n ** 3, "k_gemm_uv": 4 * n ** 3,
            "k_gemm_psi_ey": 4 * n ** 3, "k_gemm_ex": 2 * n ** 3}


def stage_bytes(inst):
    """Compulsory (algorithmic) bytes per step of one evaluation, whatever the
    implementation: each input read once and each output written once in the
    float32 structure-of-arrays layout (cells x, y, w, h; maps n*n; pins
    (cell, dx, dy); net_ptr)."""
    m, E, P, n2 = inst.num_cells, inst.num_nets, inst.num_pins, inst.n ** 2
    return {
        # a2: cells in; base in; rho out
        "a2_scatter": 16 * m + 4 * n2 + 4 * n2,
        # a3-a5: rho in; psi, Ex, Ey out
        "a3_a5_spectral": 4 * n2 * 4,
        # a6: cells and the field maps in; g out
        "a6_gather": 16 * m + 8 * n2 + 8 * m,
        # a8: pins and net_ptr in; x, y in; g read-modify-write counted once
        "a8_wirelength": 12 * P + 4 * E + 8 * m + 8 * m,
    }


# The kernels that carry each step (whichever path or spectral variant ran).
# k_xch_cellsum sums each cell's pin gradients (a8) and adds lambda times the
# density gradient (a9); its time is booked to a8.
STAGE_KERNELS = {
    "a2_scatter": ("k_band_place", "k_band_accum", "k_fill", "k_scatter"),
    "a3_a5_spectral": ("k_rows_dct2", "k_cols_solve", "k_rows_inverse", "k_gemm_rowsum",
                       "k_gemm_prep", "k_gemm_w", "k_gemm_bfly", "k_gemm_g", "k_gemm_uv",
                       "k_gemm_psi_ey", "k_gemm_ex"),
    "a6_gather": ("k_band_gather", "k_gather", "k_gather_pins"),
    "a8_wirelength": ("k_xch_spread", "k_xch_wa", "k_xch_cellsum", "k_interleave",
                      "k_wa_slots_small", "k_wa_slots_big", "k_wa_atomic"),
}


def stage_table(kernels, sb, eval_ms):
    """Per step: its kernels' summed event time (kernels timed one at a time),
    the compulsory bytes over that time against the HBM peak, and the counter
    traffic of its kernels over the compulsory bytes."""
    out = {}
    for st, names in STAGE_KERNELS.items():
        ks = [k for k in names if k in kernels]
        if not ks:
            continue
        t = sum(kernels[k]["ms"] for k in ks)
        row = {"kernels": ks, "ms": t, "algorithmic_bytes": sb[st],
               "GBps": sb[st] / (t / 1e3) / 1e9}
        row["frac"] = row["GBps"] / HBM_PEAK_GBS
        pmc = [kernels[k].get("pmc_hbm_bytes") for k in ks]
        if all(v is not None for v in pmc):
            row["pmc_hbm_bytes"] = sum(pmc)
            row["traffic_over_algorithmic"] = sum(pmc) / sb[st]
        out[st] = row
    tot = sum(sb.values())
    out["evaluation"] = {"ms": eval_ms, "algorithmic_bytes": tot,
                         "GBps": tot / (eval_ms / 1e3) / 1e9,
                         "frac": tot / (eval_ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    return out


def time_loop(fn, steps, stream):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def per_step_times(fn, steps, stream):
    import torch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for i in range(steps):
        fn()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    return [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]


def standalone_calls(fftpl, inst, prob, x, y, gx, gy, plan, stream, reps):
    """Milliseconds per call of each standalone entry point at the benchmark
    workload (inputs resident), and whether repeated calls give the same
    bits."""
    import ctypes

    import torch
    from paper_1312_4587_amd import _lib
    n2 = inst.n ** 2
    rho = torch.empty(n2, device="cuda")
    rho2 = torch.empty(n2, device="cuda")
    a = prob.arrays
    out = {}

    def run(name, f, check=None):
        f()
        ms = time_loop(f, reps, stream)
        out[name] = {"ms": ms}
        if check is not None:
            out[name]["repeatable"] = bool(check())

    def same_rho(f):
        def chk():
            f()
            torch.cuda.synchronize()
            r1 = rho.clone()
            f()
            torch.cuda.synchronize()
            return torch.equal(r1, rho)
        return chk
    fd = lambda: fftpl.density_map(prob.grid, x, y, a["w"], a["h"], a["base"], rho)  # noqa
    run("fftpl_density_map (temporary stream-ordered workspace)", fd, same_rho(fd))
    fp = lambda: fftpl.problem_density(prob, x, y, rho)  # noqa
    run("fftpl_problem_density", fp, same_rho(fp))
    # the allocation-free form holds at most 921,600 cells: its first ones
    mm = min(inst.num_cells, 921_600)
    lib = _lib.load()
    P = fftpl._ptr

    def fna():
        st = lib.fftpl_density_map_noalloc(ctypes.byref(prob.grid.c()), mm, P(x), P(y),
                                           P(a["w"]), P(a["h"]), P(a["base"]), P(rho),
                                           fftpl._stream(None))
        fftpl._check(st, "fftpl_density_map_noalloc")
    run(f"fftpl_density_map_noalloc ({mm} cells)", fna, same_rho(fna))
    exy = plan.maps()[2].reshape(-1, 2)
    ex, ey = exy[:, 0].contiguous(), exy[:, 1].contiguous()
    psi = plan.maps()[1].reshape(-1)
    fg = lambda: fftpl.field_gather(prob.grid, x, y, a["w"], a["h"], ex, ey, psi,  # noqa
                                    "field", 1.0, 0, gx, gy)
    run("fftpl_field_gather", fg)
    fw = lambda: fftpl.wa_grad(a["net_ptr"], a["pin_cell"], a["pin_dx"], a["pin_dy"],  # noqa
                               x, y, inst.gamma, 0, gx, gy)

    def same_g(f):
        def chk():
            f()
            torch.cuda.synchronize()
            a1, b1 = gx.clone(), gy.clone()
            f()
            torch.cuda.synchronize()
            return torch.equal(a1, gx) and torch.equal(b1, gy)
        return chk
    run("fftpl_wa_grad (fixed-point global atomics, temporary workspace)", fw, same_g(fw))
    fx = lambda: fftpl.problem_wl_grad(prob, x, y, inst.gamma, 0, gx, gy)  # noqa
    run("fftpl_problem_wl_grad", fx, same_g(fx))
    del rho2
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inst, name, evals, other_configs=("small_2k", "mid_200k")):
    """The FP64 oracle as it stands, timed on this machine's host cores: one
    leg with a single BLAS thread and one with every core, on the benchmark
    workload and on the smaller workloads.  The headline figure is the
    benchmark workload on every core.  Returns (record, oracle result of the
    benchmark workload)."""
    import gen
    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    nproc = os.cpu_count() or 1
    legs = []
    ref = None

    def leg(name, ins, threads, reps):
        nonlocal ref
        with threadpool_limits(threads):
            used = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
            t0 = time.perf_counter()
            for _ in range(reps):
                r = oracle.evaluate(ins, lam=1.0, grad_mode="field")
            dt = (time.perf_counter() - t0) / reps
        if ins is inst:
            ref = r
        legs.append({"workload": name, "cells": ins.num_cells, "grid_n": ins.n,
                     "threads": int(used), "evals": reps, "s_per_eval": dt,
                     "value": ins.num_cells / dt})

    leg(name, inst, nproc, evals)
    leg(name, inst, 1, 1)
    for name in other_configs:
        ins = gen.make_config(name)
        reps = 20 if ins.num_cells <= 10_000 else 2
        leg(name, ins, nproc, reps)
        leg(name, ins, 1, reps)
    head = legs[0]
    rec = {"value": head["value"], "unit": "cell-gradient evals/s",
           "cores": head["threads"], "kind": "oracle",
           "sample": (f"{evals} full FP64 oracle evaluation(s) of the same "
                      f"{inst.num_cells}-cell n={inst.n} workload, "
                      f"{head['s_per_eval']:.2f} s each, numpy with "
                      f"{head['threads']} BLAS threads (the dense cosine sums; the "
                      "rest is single-threaded); further legs: one thread, and the "
                      "2k- and 200k-cell workloads"),
           "nproc": nproc, "cpu_model": cpu_model(), "legs": legs}
    return rec, ref


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library "
              "evaluates one design on one GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import gen
    from paper_1312_4587_amd import _lib, fftpl

    from paper_1312_4587_amd import build
    build.ensure_built()   # rebuilt when the sources differ from the built ones
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    inst = gen.make_config(args.workload)
    prob = fftpl.Problem.from_instance(inst)
    x = torch.as_tensor(inst.x).cuda()
    y = torch.as_tensor(inst.y).cuda()
    m = inst.num_cells
    gx = torch.empty(m, device="cuda")
    gy = torch.empty(m, device="cuda")
    out4 = torch.empty(4, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    plans = {}

    def plan_for(mode):
        if mode not in plans:
            plans[mode] = fftpl.Plan(inst.n, mode)
        return plans[mode]

    def eval_fn(mode):
        plan = plan_for(mode)
        return lambda: fftpl.eval(plan, prob, x, y, 1.0, inst.gamma, "field", gx, gy, out4)

    # ---- headline: whole evaluation
    f = eval_fn(args.dct)
    for _ in range(args.warmup):
        f()
    ms = time_loop(f, args.steps, stream)
    steps_ms = per_step_times(f, min(args.steps, 200), stream)
    value = m / (ms / 1e3)

    variants = {}
    for mode in [v for v in args.variants.split(",") if v and v != args.dct]:
        try:
            fv = eval_fn(mode)
            for _ in range(3):
                fv()
            msv = time_loop(fv, max(10, args.steps // 2), stream)
            variants[mode] = {"ms_per_eval": msv, "value": m / (msv / 1e3)}
        except fftpl.FFTPLError as e:
            variants[mode] = {"unavailable": str(e)}
    variants[args.dct] = {"ms_per_eval": ms, "value": value}

    # ---- the other wirelength paths, for comparison: cell-major slots and
    # float atomics
    for path, key in (("slots", "fft_slots"), ("atomic", "fft_float_atomics")):
        try:
            prob_o = fftpl.Problem.from_instance(inst, path=path)
            plan_o = plan_for(args.dct)
            fo = lambda: fftpl.eval(plan_o, prob_o, x, y, 1.0, inst.gamma, "field",  # noqa
                                    gx, gy, out4)
            for _ in range(2):
                fo()
            mso = time_loop(fo, max(5, args.steps // 5), stream)
            variants[key] = {"ms_per_eval": mso, "value": m / (mso / 1e3)}
            del prob_o
        except fftpl.FFTPLError as e:
            variants[key] = {"unavailable": str(e)}

    # ---- the standalone calls of the boundary, one at a time on this stream:
    # the stateless ones (float atomics) beside their workspace-backed forms
    standalone = None
    if not args.no_standalone:
        standalone = standalone_calls(fftpl, inst, prob, x, y, gx, gy, plan_for(args.dct),
                                      stream, max(10, args.steps // 4))

    # ---- per-kernel durations: HIP events the library records on this
    # stream after every kernel (timing on the plan; no stream overlap then)
    nbytes = kernel_bytes(inst, band_entries(inst))
    gflop = gemm_flops(inst.n)

    def kernel_table(mode):
        plan = plan_for(mode)
        fk = eval_fn(mode)
        plan.timing(True)
        acc = {}
        for _ in range(args.kernel_reps or max(10, args.steps // 4)):
            fk()
            for name, t in plan.kernel_times():
                acc.setdefault(name, []).append(t)
        plan.timing(False)
        table = {}
        for name, ts in acc.items():
            t = float(np.mean(ts))
            row = {"ms": t}
            b = nbytes.get(name)
            if b:
                row.update(algorithmic_bytes=b, GBps=b / (t / 1e3) / 1e9)
            if name in gflop:
                mult = 3 if mode == "gemm_bf16x3" else 1
                peak = BF16_PEAK_TFLOPS if mode == "gemm_bf16x3" else FP32_PEAK_TFLOPS
                tf = mult * gflop[name] / (t / 1e3) / 1e12
                row.update(mfma_flops=mult * gflop[name], TFLOPs=tf, mfma_util=tf / peak)
            table[name] = row
        return table

    kernels = kernel_table(args.dct)
    variant_kernels = {}
    for mode in variants:
        if mode != args.dct and "ms_per_eval" in variants[mode] and mode in ("gemm_f32",
                                                                            "gemm_bf16x3"):
            variant_kernels[mode] = kernel_table(mode)
    for k, v in kernels.items():
        t = pmc_traffic(k)
        if t is not None:
            v["pmc_hbm_bytes"] = t
    sb = stage_bytes(inst)
    stages = stage_table(kernels, sb, ms)
    # The dominant kernel: the longest one of the HBM-bound steps.  `achieved`
    # books its whole step's compulsory bytes to it (the other kernels of the
    # step get none); the step's own fraction over all its kernels is the
    # stages entry.  `design_bytes` are what the kernel's own layout reads and
    # writes once (index arrays, the exchange buffer).
    hbm_steps = ("a2_scatter", "a6_gather", "a8_wirelength")
    cands = [(kernels[k]["ms"], k, st) for st in hbm_steps if st in stages
             for k in stages[st]["kernels"]]
    _, dom, dom_st = max(cands)
    ach = sb[dom_st] / (kernels[dom]["ms"] / 1e3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": pmc_traffic(dom),
                "algorithmic_bytes": sb[dom_st], "step": dom_st,
                "kernel_ms": kernels[dom]["ms"],
                "design_bytes": kernels[dom].get("algorithmic_bytes"),
                "step_frac": stages[dom_st]["frac"],
                "evaluation_frac": stages["evaluation"]["frac"]}
    for k, v in kernels.items():
        if "algorithmic_bytes" in v:
            # per kernel: bytes of its own layout (not the step's compulsory bytes)
            v["design_bytes"] = v.pop("algorithmic_bytes")
            v["design_GBps"] = v.pop("GBps")

    res = {
        "metric": METRIC, "value": value, "unit": "cell-gradient evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "cells": m, "nets": inst.num_nets,
                   "pins": inst.num_pins, "grid_n": inst.n, "macros": inst.num_fixed,
                   "dct": args.dct, "grad_mode": "field", "seed": inst.meta["seed"]},
        "p50_ms": float(np.percentile(steps_ms, 50)),
        "p90_ms": float(np.percentile(steps_ms, 90)),
        "variants": variants, "kernels": kernels, "variant_kernels": variant_kernels,
        "stages": stages, "roofline": roofline, "standalone": standalone,
    }
    ref = None
    if not args.no_cpu_baseline:
        res["cpu_baseline"], ref = cpu_baseline(inst, args.workload, args.cpu_evals)
    if not args.no_precision:
        if ref is None:
            import oracle
            ref = oracle.evaluate(inst, lam=1.0, grad_mode="field")
        res["precision"] = precision_report(fftpl, plans, plan_for, eval_fn, variants, ref,
                                            inst, prob, gx, gy)
    for p in plans.values():
        p.close()
    if not args.no_forms:
        del prob
        torch.cuda.empty_cache()
        res["driver"] = driver_run(args)
        res["differentiation"] = autograd_run()
        torch.cuda.empty_cache()
        sv = serving_run(args, "fft", args.serve_requests)
        res["serving"] = {"fft": sv,
                          "gemm_bf16x3": serving_run(args, "gemm_bf16x3",
                                                     max(1, args.serve_requests // 5))}
        if args.serve_saturate > 0:
            # arrivals far above the service rate: throughput with grouping by
            # grid side against one request per launch
            res["serving"]["saturated"] = {
                f"max_batch_{mb}": serving_run(args, "fft", args.serve_saturate,
                                               rate=50_000.0, max_batch=mb)
                for mb in (1, args.serve_batch)}
        res["served_p50_ms"] = sv["p50_ms"]
        res["served_p99_ms"] = sv["p99_ms"]
    print(json.dumps(res), flush=True)


def precision_report(fftpl, plans, plan_for, eval_fn, variants, ref, inst, prob, gx, gy):
    """Relative L2 error of psi, Ex, Ey and of the gradient against the FP64
    oracle, per spectral variant, at the benchmark workload."""
    import numpy as np
    import torch

    def rel(a, b):
        a = np.asarray(a, np.float64)
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))

    n2 = inst.n ** 2
    out = {}
    g0 = np.concatenate([ref["gx"], ref["gy"]])
    for mode, v in variants.items():
        if "ms_per_eval" not in v or mode not in ("fft", "gemm_f32", "gemm_bf16x3"):
            continue
        plan = plan_for(mode)
        eval_fn(mode)()
        g = np.concatenate([gx.cpu().numpy(), gy.cpu().numpy()])
        rho = plan.maps()[0].reshape(-1).clone()
        psi = torch.empty(n2, device="cuda")
        ex = torch.empty(n2, device="cuda")
        ey = torch.empty(n2, device="cuda")
        fftpl.poisson_solve(plan, prob.grid, rho, psi, ex, ey)
        torch.cuda.synchronize()
        shape = (inst.n, inst.n)
        out[mode] = {"psi": rel(psi.cpu().numpy().reshape(shape), ref["psi"]),
                     "ex": rel(ex.cpu().numpy().reshape(shape), ref["ex"]),
                     "ey": rel(ey.cpu().numpy().reshape(shape), ref["ey"]),
                     "grad": rel(g, g0)}
    return out


if __name__ == "__main__":
    main()
