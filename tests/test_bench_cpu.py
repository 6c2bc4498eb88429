"""Host-side arithmetic of bench.py: the compulsory bytes per step, the
per-step roofline fractions built from them, and the single-GPU guard."""
import os
import subprocess
import sys

import pytest

import bench
import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_stage_bytes_follow_the_step_definitions():
    # each input read once and each output written once, float32 SoA
    # layouts: cells (x, y, w, h), pins (cell, dx, dy), net_ptr, n x n maps
    inst = gen.make_config("small_2k")
    m, E, P, n2 = inst.num_cells, inst.num_nets, inst.num_pins, inst.n ** 2
    sb = bench.stage_bytes(inst)
    assert set(sb) == {"a2_scatter", "a3_a5_spectral", "a6_gather", "a8_wirelength"}
    # a2: cells and the fixed map in, rho out
    assert sb["a2_scatter"] == 4 * 4 * m + 4 * n2 + 4 * n2
    # a3-a5: rho in; psi, Ex, Ey out
    assert sb["a3_a5_spectral"] == 4 * n2 + 3 * 4 * n2
    # a6: cells and the two field maps in, one gradient pair per cell out
    assert sb["a6_gather"] == 4 * 4 * m + 2 * 4 * n2 + 2 * 4 * m
    # a8: pins and net_ptr in, positions in, the gradient pair once
    assert sb["a8_wirelength"] == 3 * 4 * P + 4 * E + 2 * 4 * m + 2 * 4 * m


def test_stage_table_fractions():
    inst = gen.make_config("small_2k")
    sb = bench.stage_bytes(inst)
    kernels = {"k_band_place": {"ms": 0.01}, "k_band_accum": {"ms": 0.03},
               "k_xch_spread": {"ms": 0.02, "pmc_hbm_bytes": 1000.0},
               "k_xch_wa": {"ms": 0.05, "pmc_hbm_bytes": 3000.0},
               "k_xch_cellsum": {"ms": 0.03, "pmc_hbm_bytes": 2000.0}}
    tab = bench.stage_table(kernels, sb, 0.2)
    a2 = tab["a2_scatter"]
    assert a2["kernels"] == ["k_band_place", "k_band_accum"]
    assert a2["ms"] == pytest.approx(0.04)
    assert a2["frac"] == pytest.approx(sb["a2_scatter"] / 0.04e-3 / 1e9 / bench.HBM_PEAK_GBS)
    # counter traffic only where every kernel of the step has it
    assert "pmc_hbm_bytes" not in a2
    a8 = tab["a8_wirelength"]
    assert a8["pmc_hbm_bytes"] == pytest.approx(6000.0)
    assert a8["traffic_over_algorithmic"] == pytest.approx(6000.0 / sb["a8_wirelength"])
    # steps with no timed kernel are left out; the whole evaluation counts
    # every step's compulsory bytes over the evaluation's time
    assert "a6_gather" not in tab and "a3_a5_spectral" not in tab
    ev = tab["evaluation"]
    assert ev["algorithmic_bytes"] == sum(sb.values())
    assert ev["frac"] == pytest.approx(sum(sb.values()) / 0.2e-3 / 1e9 / bench.HBM_PEAK_GBS)


def test_pmc_traffic_is_null_for_unrecorded_kernels():
    assert bench.pmc_traffic("k_no_such_kernel") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
