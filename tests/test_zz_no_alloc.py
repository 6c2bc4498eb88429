"""The allocation-free density map (fftpl_density_map_noalloc: band lists in
the library's static device array) against the workspace-backed entry point
it shares its kernels with, bit for bit, and against the FP64 oracle; two
calls in a row, the second with fewer cells and another grid side, and the
size limit refused on the host."""
import ctypes

import numpy as np
import pytest

import gen
import oracle
from _helpers import rel_l2, with_macros
from gpu_common import RTOL, DeviceCells, host, lib_or_build, say

pytestmark = pytest.mark.gpu


def test_noalloc_density_matches_workspace_entry_point():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_or_build()
    from paper_1312_4587_amd import _lib, fftpl
    lib = _lib.load()
    p = fftpl._ptr
    cases = [gen.make_instance(91, num_cells=600_000, util=0.9, n=1024, num_nets=10,
                               num_macros=20, macro_area_frac=0.12),
             with_macros(gen.make_config("small_2k"), [[30.0, 30.0, 10.0, 8.0]])]
    for inst in cases:
        say("noalloc density", inst.num_cells, inst.n)
        prob = fftpl.Problem.from_instance(inst)
        c = DeviceCells(inst)
        n2 = inst.n ** 2
        ref = torch.empty(n2, device="cuda")
        fftpl.problem_density(prob, c.x, c.y, ref)
        got = torch.full((n2,), -3.0, device="cuda")
        st = lib.fftpl_density_map_noalloc(
            ctypes.byref(prob.grid.c()), inst.num_cells, p(c.x), p(c.y), p(c.w), p(c.h),
            p(prob.arrays["base"]), p(got), fftpl._stream(None))
        assert st == 0
        torch.cuda.synchronize()
        # the same kernels on the same inputs: the same bits
        assert torch.equal(got, ref)
        b0, _ = oracle.fixed_maps(inst)
        r0 = oracle.density_map(inst, b0)
        assert rel_l2(host(got).reshape(inst.n, inst.n), r0) < RTOL
    # beyond the static array's capacity, or above n = 1024: refused, nothing runs
    g = fftpl.Grid(1024, 0.0, 0.0, 1.0, 1.0).c()
    one = torch.zeros(4, device="cuda")
    assert lib.fftpl_density_map_noalloc(ctypes.byref(g), 921_601, p(one), p(one), p(one),
                                         p(one), None, p(one), None) == fftpl.E_UNSUPPORTED
    g2 = fftpl.Grid(2048, 0.0, 0.0, 1.0, 1.0).c()
    assert lib.fftpl_density_map_noalloc(ctypes.byref(g2), 4, p(one), p(one), p(one),
                                         p(one), None, p(one), None) == fftpl.E_UNSUPPORTED
