"""The C-ABI library builds, loads and exports every declared entry point, and
its host-side argument checks return the documented status codes.  No GPU
work is enqueued by anything here (every call fails validation first)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fftpl.h")


def _lib():
    from paper_1312_4587_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1312_4587_amd import build
        build.build()
    return L.load()


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fftpl_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = _lib()
    from paper_1312_4587_amd import _lib as L
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, f"{name} has no binding"


def test_version_and_status_strings():
    lib = _lib()
    assert lib.fftpl_version() == 20100
    for st in (0, -1, -2, -3, -4, -5):
        assert lib.fftpl_status_string(st).startswith(b"FFTPL_")
    assert b"unknown" in lib.fftpl_status_string(17)


def test_struct_layouts_match_header():
    from paper_1312_4587_amd import _lib as L
    assert ctypes.sizeof(L.fftpl_grid) == 48
    assert L.fftpl_problem.w.offset == 64
    assert ctypes.sizeof(L.fftpl_problem) == 64 + 8 * 8 + 4 * 8 + 24 + 8
    assert L.fftpl_problem.work_bytes.offset == 152
    assert L.fftpl_problem.xindex.offset == 160
    assert L.fftpl_problem.max_degree.offset == 176
    assert L.fftpl_problem.xindex_key.offset == 184


def test_argument_errors_are_reported_before_any_device_work():
    lib = _lib()
    from paper_1312_4587_amd import _lib as L
    h = ctypes.c_void_p()
    assert lib.fftpl_plan_create(None, 64, 0, 1, None) == -1
    assert lib.fftpl_plan_create(ctypes.byref(h), 64, 7, 1, None) == -1
    for mb in (0, -1, 9):
        assert lib.fftpl_plan_create(ctypes.byref(h), 64, 0, mb, None) == -1
    for n in (0, 4, 100, 2048):
        assert lib.fftpl_plan_create(ctypes.byref(h), n, 0, 1, None) == -4
    for n in (32, 100, 8192):
        assert lib.fftpl_plan_create(ctypes.byref(h), n, 1, 1, None) == -4
    g = L.fftpl_grid(64, 0, 0.0, 0.0, 1.0, 1.0, 1.0)
    bad = [L.fftpl_grid(0, 0, 0.0, 0.0, 1.0, 1.0, 1.0),
           L.fftpl_grid(64, 1, 0.0, 0.0, 1.0, 1.0, 1.0),
           L.fftpl_grid(64, 0, 0.0, 0.0, 0.0, 1.0, 1.0),
           L.fftpl_grid(64, 0, float("nan"), 0.0, 1.0, 1.0, 1.0)]
    for b in bad:
        assert lib.fftpl_density_map(ctypes.byref(b), 0, None, None, None, None, None,
                                     ctypes.c_void_p(256), None) == -1
    assert lib.fftpl_density_map(ctypes.byref(g), 10, None, None, None, None, None,
                                 ctypes.c_void_p(256), None) == -1
    assert lib.fftpl_density_map(ctypes.byref(g), -1, None, None, None, None, None,
                                 ctypes.c_void_p(256), None) == -1
    assert lib.fftpl_fixed_map(ctypes.byref(g), 3, None, None, None, None,
                               ctypes.c_void_p(256), None, None) == -1
    p = ctypes.c_void_p(256)
    assert lib.fftpl_field_gather(ctypes.byref(g), 5, p, p, p, p, p, p, p, 9, 1.0, 0,
                                  p, p, None) == -1
    assert lib.fftpl_field_gather(ctypes.byref(g), 5, p, p, p, p, None, None, p, 0, 1.0,
                                  0, p, p, None) == -1
    assert lib.fftpl_field_gather(ctypes.byref(g), 5, p, p, p, p, p, p, None, 1, 1.0,
                                  0, p, p, None) == -1
    assert lib.fftpl_field_gather(ctypes.byref(g), 5, p, p, p, p, p, p, p, 0, 1.0,
                                  2, p, p, None) == -1
    assert lib.fftpl_wa_grad(3, p, 6, p, p, p, 4, p, p, 0.0, 0, p, p, None, None,
                             None) == -1
    assert lib.fftpl_wa_grad(3, p, 6, p, p, p, 4, p, p, float("inf"), 0, p, p, None,
                             None, None) == -1
    assert lib.fftpl_wa_grad(3, None, 6, p, p, p, 4, p, p, 1.0, 0, p, p, None, None,
                             None) == -1
    assert lib.fftpl_wa_grad(3, p, 6, p, p, p, 0, None, None, 1.0, 0, None, None, None,
                             None, None) == -1
    for gam in (0.0, -1.0, float("inf"), float("nan")):
        assert lib.fftpl_lse_grad(3, p, 6, p, p, p, 4, p, p, gam, 0, p, p, None, None,
                                  None) == -1
    assert lib.fftpl_lse_grad(3, p, 6, p, p, p, 4, p, p, 1.0, 3, p, p, None, None,
                              None) == -1
    assert lib.fftpl_helmholtz_solve(None, ctypes.byref(g), 0.5, p, p, None, None, None,
                                     None) == -1
    assert lib.fftpl_eval(None, None, p, p, 1.0, 1.0, 0, p, p, p, None) == -1
    assert lib.fftpl_eval_params(None, None, p, p, p, 0, p, p, p, None) == -1
    # the device loop's schedule and update: missing device arrays
    assert lib.fftpl_nesterov_schedule(None, p, p, p, None, 0, None) == -1
    assert lib.fftpl_nesterov_schedule(p, p, p, None, None, 0, None) == -1
    assert lib.fftpl_nesterov_schedule(p, p, p, p, None, 4, None) == -1
    assert lib.fftpl_nesterov_schedule(p, p, p, p, p, -1, None) == -1
    assert lib.fftpl_nesterov_update_dev(ctypes.byref(g), 5, p, p, p, p, p, p, p, p, p, p,
                                         p, p, None, None) == -1
    assert lib.fftpl_nesterov_update_dev(ctypes.byref(g), 5, None, p, p, p, p, p, p, p, p,
                                         p, p, p, p, None) == -1
    assert lib.fftpl_eval_batch(None, 0, None, None, None, None, None, 0, None, None, None,
                                None) == 0
    assert lib.fftpl_eval_batch(None, -1, None, None, None, None, None, 0, None, None, None,
                                None) == -1
    assert lib.fftpl_eval_batch(None, 2, None, None, None, None, None, 0, None, None, p,
                                None) == -1
    assert lib.fftpl_poisson_solve(None, ctypes.byref(g), p, p, None, None, None,
                                   None) == -1
    assert lib.fftpl_debug_cell_bins(ctypes.byref(g), 4, p, p, p, p, None, None) == -1
    u64 = ctypes.c_uint64
    ib, wb = u64(), u64()
    assert lib.fftpl_xindex_bytes(10, 3, 6, 2, None, ctypes.byref(wb)) == -1
    assert lib.fftpl_xindex_bytes(-1, 3, 6, 2, ctypes.byref(ib), ctypes.byref(wb)) == -1
    assert lib.fftpl_xindex_bytes(10, 3, 6, 8706, ctypes.byref(ib), ctypes.byref(wb)) == -4
    assert lib.fftpl_xindex_bytes(10, 3, 6, 2, ctypes.byref(ib), ctypes.byref(wb)) == 0
    assert ib.value > 0 and wb.value > 0
    # too small buffers, missing arrays, pins without cells: rejected on the host
    assert lib.fftpl_xindex_build(10, 3, 6, p, p, 2, p, ib.value - 1, p, wb.value,
                                  None, None) == -1
    assert lib.fftpl_xindex_build(10, 3, 6, p, p, 2, p, ib.value, p, wb.value - 1,
                                  None, None) == -1
    assert lib.fftpl_xindex_build(10, 3, 6, None, p, 2, p, ib.value, p, wb.value,
                                  None, None) == -1
    assert lib.fftpl_xindex_build(0, 3, 6, p, p, 2, p, ib.value, p, wb.value, None,
                                  None) == -1
    assert lib.fftpl_xindex_build(10, 3, 6, p, p, 8706, p, ib.value, p, wb.value,
                                  None, None) == -4
    assert lib.fftpl_plan_destroy(None) == 0
    assert lib.fftpl_plan_info(None, None, None, None) == -1


def _problem(L, n=64, m=10, E=3, P=6, **kw):
    """An fftpl_problem over fake (never dereferenced) device addresses."""
    p = ctypes.c_void_p(1 << 20)
    pr = L.fftpl_problem(L.fftpl_grid(n, 0, 0.0, 0.0, 1.0, 1.0, 1.0), m, E, P, 0,
                         p, p, None, None, p, p, p, p, None, None, None, 0, None, 0, 8, 0.0, 0)
    for k, v in kw.items():
        setattr(pr, k, v)
    return pr


def test_problem_paths_are_decided_on_the_host():
    # which evaluation path a problem takes, and the errors for a workspace or
    # an index that is given but cannot be used (never a silent fallback)
    lib = _lib()
    from paper_1312_4587_amd import _lib as L
    path = ctypes.c_int32(-7)
    pr = _problem(L)
    assert lib.fftpl_problem_path(ctypes.byref(pr), ctypes.byref(path)) == 0
    assert path.value == 2   # nothing given: float atomics
    need = ctypes.c_uint64()
    assert lib.fftpl_problem_work_bytes(64, 10, 3, 6, ctypes.byref(need)) == 0
    work = 1 << 30
    # a workspace without a pin index
    pr = _problem(L, work=work, work_bytes=need.value)
    assert lib.fftpl_problem_path(ctypes.byref(pr), ctypes.byref(path)) == -1
    # the cell-major slots
    pr = _problem(L, work=work, work_bytes=need.value, cell_ptr=work * 2, pin_slot=work * 3)
    assert lib.fftpl_problem_path(ctypes.byref(pr), ctypes.byref(path)) == 0
    assert path.value == 1
    # too small a workspace, an unaligned one, n above the banded limit
    pr = _problem(L, work=work, work_bytes=need.value - 1, cell_ptr=work * 2,
                  pin_slot=work * 3)
    assert lib.fftpl_problem_path(ctypes.byref(pr), ctypes.byref(path)) == -1
    pr = _problem(L, work=work + 16, work_bytes=need.value, cell_ptr=work * 2,
                  pin_slot=work * 3)
    assert lib.fftpl_problem_path(ctypes.byref(pr), ctypes.byref(path)) == -1
    pr = _problem(L, n=2048, work=work, work_bytes=1 << 40, cell_ptr=work * 2,
                  pin_slot=work * 3)
    assert lib.fftpl_problem_path(ctypes.byref(pr), ctypes.byref(path)) == -4
    # the exchange index: needs its size and the key of its build; an index of
    # another netlist (another key) is refused with FFTPL_E_STATE
    ib, wb = ctypes.c_uint64(), ctypes.c_uint64()
    assert lib.fftpl_xindex_bytes(10, 3, 6, 8, ctypes.byref(ib), ctypes.byref(wb)) == 0
    pr = _problem(L, work=work, work_bytes=need.value, xindex=work * 4, xindex_bytes=ib.value,
                  xindex_key=12345)
    assert lib.fftpl_problem_path(ctypes.byref(pr), ctypes.byref(path)) == -5
    pr.xindex_bytes = ib.value - 1
    assert lib.fftpl_problem_path(ctypes.byref(pr), ctypes.byref(path)) == -1
    # the same checks guard the evaluation and the standalone problem calls
    # (the key mismatch is found before anything is enqueued)
    pr.xindex_bytes = ib.value
    h = ctypes.c_void_p(1 << 20)
    assert lib.fftpl_problem_wl_grad(ctypes.byref(pr), h, h, 1.0, 0, h, h, None, None,
                                     None) == -5
    assert lib.fftpl_debug_net_values(ctypes.byref(pr), h, h, 1.0, h, h, None) == -5
    assert lib.fftpl_problem_wl_grad(ctypes.byref(pr), h, h, 0.0, 0, h, h, None, None,
                                     None) == -1
    assert lib.fftpl_problem_density(ctypes.byref(_problem(L)), h, h, h, None) == -1
    assert lib.fftpl_problem_density(ctypes.byref(_problem(L, n=2048)), h, h, h, None) == -4
    assert lib.fftpl_problem_path(None, ctypes.byref(path)) == -1


def test_roctx_ranges_only_in_the_flagged_build(tmp_path):
    # the entry points' profiler ranges compile in with FFTPL_ROCTX and out
    # without it (compiled here, host and gfx950 device code)
    import shutil
    import subprocess
    from paper_1312_4587_amd import build
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    src = os.path.join(build.CSRC, "abi.hip")
    refs = {}
    for flag in ([], ["-DFFTPL_ROCTX"]):
        obj = str(tmp_path / ("abi%s.o" % ("_roctx" if flag else "")))
        r = subprocess.run([hipcc, "-O1", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                            "-w", *flag, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        nm = subprocess.run(["nm", obj], capture_output=True, text=True).stdout
        refs[bool(flag)] = ("roctxRangePush" in nm, "roctxRangePop" in nm)
    assert refs[False] == (False, False) and refs[True] == (True, True)
