"""Thin Python binding of the libfftpl C ABI.

Same names as the C entry points (without the ``fftpl_`` prefix); arguments
are torch tensors on the GPU (device memory only) and an optional
``torch.cuda.Stream`` (default: the current stream).  Every step of the
computation runs in the HIP kernels of libfftpl; this module only marshals
pointers and sizes, and raises ``FFTPLError`` on a non-zero status.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib

OK, E_INVAL, E_NOMEM, E_DEVICE, E_UNSUPPORTED, E_STATE = 0, -1, -2, -3, -4, -5
DCT_MODES = {"fft": 0, "gemm_f32": 1, "gemm_bf16x3": 2}
GRAD_MODES = {"field": 0, "exact": 1}
WL_MODELS = {"wa": 0, "lse": 1}


class FFTPLError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = _lib.load()
        msg = lib.fftpl_status_string(status).decode()
        super().__init__(f"{where}: {msg}")
        self.status = status


def _check(status: int, where: str) -> None:
    if status != OK:
        raise FFTPLError(status, where)


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t, dtype=None, numel=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (None passes NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements (got {t.numel()})")
    return t.data_ptr()


@dataclasses.dataclass
class Grid:
    n: int
    xl: float
    yl: float
    bin_w: float
    bin_h: float
    target_density: float = 1.0

    @classmethod
    def of(cls, inst) -> "Grid":
        return cls(int(inst.n), float(inst.xl), float(inst.yl), float(inst.bin_w),
                   float(inst.bin_h), float(inst.target_density))

    def c(self) -> _lib.fftpl_grid:
        return _lib.fftpl_grid(self.n, 0, self.xl, self.yl, self.bin_w, self.bin_h,
                               self.target_density)


def version() -> int:
    return _lib.load().fftpl_version()


def status_string(status: int) -> str:
    return _lib.load().fftpl_status_string(status).decode()


class Plan:
    """fftpl_plan_create / fftpl_plan_destroy."""

    def __init__(self, n: int, dct_mode: str = "fft", stream=None, max_batch: int = 1):
        lib = _lib.load()
        h = ctypes.c_void_p()
        _check(lib.fftpl_plan_create(ctypes.byref(h), int(n), DCT_MODES[dct_mode],
                                     int(max_batch), _stream(stream)), "fftpl_plan_create")
        self._h = h
        self.n = int(n)
        self.dct_mode = dct_mode
        self.max_batch = int(max_batch)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("plan is destroyed")
        return self._h

    def info(self):
        n, mode, mb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.load().fftpl_plan_info(self.handle, ctypes.byref(n), ctypes.byref(mode),
                                           ctypes.byref(mb)), "fftpl_plan_info")
        return n.value, mode.value, mb.value

    def maps(self, slot: int = 0):
        """Views (no copy) of the plan's rho [n,n], psi [n,n] and exy [n,n,2]
        (batch slot ``slot``: request ``slot`` of the last batched group)."""
        if not 0 <= slot < self.max_batch:
            raise ValueError("slot outside the plan's batch")
        r, p, e = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(_lib.load().fftpl_plan_maps(self.handle, ctypes.byref(r), ctypes.byref(p),
                                           ctypes.byref(e)), "fftpl_plan_maps")
        n = self.n
        o = 4 * n * n * slot
        return (_wrap(r.value + o, (n, n)), _wrap(p.value + o, (n, n)),
                _wrap(e.value + 2 * o, (n, n, 2)))

    def timing(self, enable: bool = True):
        """fftpl_plan_timing: per-kernel HIP events on later calls."""
        _check(_lib.load().fftpl_plan_timing(self.handle, 1 if enable else 0),
               "fftpl_plan_timing")

    def kernel_times(self):
        """[(kernel name, ms)] of the last timed call (waits for it)."""
        mx = 32
        ms = (ctypes.c_float * mx)()
        names = (ctypes.c_char_p * mx)()
        cnt = ctypes.c_int32()
        _check(_lib.load().fftpl_plan_kernel_times(self.handle, mx, ms, names,
                                                   ctypes.byref(cnt)),
               "fftpl_plan_kernel_times")
        return [(names[i].decode(), float(ms[i])) for i in range(cnt.value)]

    def close(self):
        if self._h is not None:
            _check(_lib.load().fftpl_plan_destroy(self._h), "fftpl_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DevArray:
    """Minimal __cuda_array_interface__ holder to view plan-owned memory."""

    def __init__(self, ptr, shape):
        self.__cuda_array_interface__ = {
            "shape": tuple(shape), "typestr": "<f4", "data": (ptr, False),
            "version": 2, "strides": None}


def _wrap(ptr, shape):
    return torch.as_tensor(_DevArray(ptr, shape), device="cuda")


def fixed_map(grid: Grid, fx, fy, fw, fh, base, cap=None, stream=None):
    n2 = grid.n * grid.n
    nf = 0 if fx is None else int(fx.numel())
    _check(_lib.load().fftpl_fixed_map(
        ctypes.byref(grid.c()), nf, _ptr(fx, torch.float32, nf, "fx"),
        _ptr(fy, torch.float32, nf, "fy"), _ptr(fw, torch.float32, nf, "fw"),
        _ptr(fh, torch.float32, nf, "fh"), _ptr(base, torch.float32, n2, "base"),
        _ptr(cap, torch.float32, n2, "cap"), _stream(stream)), "fftpl_fixed_map")


def dark_nodes(xl: float, yl: float, xh: float, yh: float, rects) -> np.ndarray:
    """fftpl_dark_nodes on host arrays: the bounding box minus the union of
    the placeable rectangles ``rects`` [k, 4] (x0, y0, x1, y1), returned as
    disjoint rectangles [j, 4] in the same layout."""
    r = np.ascontiguousarray(np.asarray(rects, np.float64).reshape(-1, 4))
    lib = _lib.load()
    cap = 2 * len(r) + 2
    while True:
        out = np.zeros((cap, 4), np.float64)
        cnt = ctypes.c_int32(0)
        st = lib.fftpl_dark_nodes(float(xl), float(yl), float(xh), float(yh), len(r),
                                  r.ctypes.data if len(r) else None, cap, out.ctypes.data,
                                  ctypes.byref(cnt))
        if st == E_INVAL and cnt.value > cap:
            cap = cnt.value
            continue
        _check(st, "fftpl_dark_nodes")
        return out[:cnt.value].copy()


def density_map(grid: Grid, x, y, w, h, base, rho, stream=None):
    m = int(x.numel())
    n2 = grid.n * grid.n
    _check(_lib.load().fftpl_density_map(
        ctypes.byref(grid.c()), m, _ptr(x, torch.float32, m, "x"),
        _ptr(y, torch.float32, m, "y"), _ptr(w, torch.float32, m, "w"),
        _ptr(h, torch.float32, m, "h"), _ptr(base, torch.float32, n2, "base"),
        _ptr(rho, torch.float32, n2, "rho"), _stream(stream)), "fftpl_density_map")


def poisson_solve(plan: Plan, grid: Grid, rho, psi, ex=None, ey=None, energy=None,
                  stream=None):
    n2 = grid.n * grid.n
    _check(_lib.load().fftpl_poisson_solve(
        plan.handle, ctypes.byref(grid.c()), _ptr(rho, torch.float32, n2, "rho"),
        _ptr(psi, torch.float32, n2, "psi"), _ptr(ex, torch.float32, n2, "ex"),
        _ptr(ey, torch.float32, n2, "ey"), _ptr(energy, torch.float64, 1, "energy"),
        _stream(stream)), "fftpl_poisson_solve")


def helmholtz_solve(plan: Plan, grid: Grid, eps, rho, psi, ex=None, ey=None, energy=None,
                    stream=None):
    n2 = grid.n * grid.n
    _check(_lib.load().fftpl_helmholtz_solve(
        plan.handle, ctypes.byref(grid.c()), float(eps), _ptr(rho, torch.float32, n2, "rho"),
        _ptr(psi, torch.float32, n2, "psi"), _ptr(ex, torch.float32, n2, "ex"),
        _ptr(ey, torch.float32, n2, "ey"), _ptr(energy, torch.float64, 1, "energy"),
        _stream(stream)), "fftpl_helmholtz_solve")


def field_gather(grid: Grid, x, y, w, h, ex, ey, psi, grad_mode, scale, accumulate,
                 gx, gy, stream=None):
    m = int(x.numel())
    n2 = grid.n * grid.n
    _check(_lib.load().fftpl_field_gather(
        ctypes.byref(grid.c()), m, _ptr(x, torch.float32, m, "x"),
        _ptr(y, torch.float32, m, "y"), _ptr(w, torch.float32, m, "w"),
        _ptr(h, torch.float32, m, "h"), _ptr(ex, torch.float32, n2, "ex"),
        _ptr(ey, torch.float32, n2, "ey"), _ptr(psi, torch.float32, n2, "psi"),
        GRAD_MODES.get(grad_mode, grad_mode), float(scale), int(accumulate),
        _ptr(gx, torch.float32, m, "gx"), _ptr(gy, torch.float32, m, "gy"),
        _stream(stream)), "fftpl_field_gather")


def _wl_grad(name, net_ptr, pin_cell, pin_dx, pin_dy, x, y, gamma, accumulate, gx, gy,
             wa, hpwl, stream):
    E = int(net_ptr.numel()) - 1
    P = int(pin_cell.numel())
    m = int(x.numel())
    _check(getattr(_lib.load(), name)(
        E, _ptr(net_ptr, torch.int32, E + 1, "net_ptr"), P,
        _ptr(pin_cell, torch.int32, P, "pin_cell"), _ptr(pin_dx, torch.float32, P, "pin_dx"),
        _ptr(pin_dy, torch.float32, P, "pin_dy"), m, _ptr(x, torch.float32, m, "x"),
        _ptr(y, torch.float32, m, "y"), float(gamma), int(accumulate),
        _ptr(gx, torch.float32, m, "gx"), _ptr(gy, torch.float32, m, "gy"),
        _ptr(wa, torch.float64, 1, "wa"), _ptr(hpwl, torch.float64, 1, "hpwl"),
        _stream(stream)), name)


def wa_grad(net_ptr, pin_cell, pin_dx, pin_dy, x, y, gamma, accumulate, gx, gy,
            wa=None, hpwl=None, stream=None):
    _wl_grad("fftpl_wa_grad", net_ptr, pin_cell, pin_dx, pin_dy, x, y, gamma, accumulate,
             gx, gy, wa, hpwl, stream)


def lse_grad(net_ptr, pin_cell, pin_dx, pin_dy, x, y, gamma, accumulate, gx, gy,
             lse=None, hpwl=None, stream=None):
    _wl_grad("fftpl_lse_grad", net_ptr, pin_cell, pin_dx, pin_dy, x, y, gamma, accumulate,
             gx, gy, lse, hpwl, stream)


def problem_work_bytes(n: int, num_cells: int, num_nets: int, num_pins: int) -> int:
    b = ctypes.c_uint64()
    _check(_lib.load().fftpl_problem_work_bytes(int(n), int(num_cells), int(num_nets),
                                                int(num_pins), ctypes.byref(b)),
           "fftpl_problem_work_bytes")
    return int(b.value)


def netlist_index(num_cells: int, pin_cell, cell_ptr, pin_slot, stream=None):
    """fftpl_netlist_index with its int32 scratch allocated here."""
    m = int(num_cells)
    P = int(pin_cell.numel())
    work = torch.empty(m + (m + 1023) // 1024 + 1, dtype=torch.int32, device="cuda")
    _check(_lib.load().fftpl_netlist_index(
        m, P, _ptr(pin_cell, torch.int32, P, "pin_cell"),
        _ptr(cell_ptr, torch.int32, m + 1, "cell_ptr"),
        _ptr(pin_slot, torch.int32, P, "pin_slot"), _ptr(work, torch.int32, None, "work"),
        _stream(stream)), "fftpl_netlist_index")
    return work


def xindex_bytes(num_cells: int, num_nets: int, num_pins: int, max_degree: int):
    """(index bytes, build scratch bytes) of fftpl_xindex_build."""
    ib, wb = ctypes.c_uint64(), ctypes.c_uint64()
    _check(_lib.load().fftpl_xindex_bytes(int(num_cells), int(num_nets), int(num_pins),
                                          int(max_degree), ctypes.byref(ib), ctypes.byref(wb)),
           "fftpl_xindex_bytes")
    return int(ib.value), int(wb.value)


def xindex_build(num_cells: int, net_ptr, pin_cell, max_degree: int, index, stream=None):
    """fftpl_xindex_build into the uint8 device tensor `index` (scratch
    allocated here and released on return; the call synchronises).  Returns
    the index's key for fftpl_problem.xindex_key."""
    m = int(num_cells)
    E = int(net_ptr.numel()) - 1
    P = int(pin_cell.numel())
    ib, wb = xindex_bytes(m, E, P, max_degree)
    if index.numel() < ib:
        raise FFTPLError(E_INVAL, "fftpl_xindex_build (index tensor too small)")
    work = torch.empty(max(wb, 1), dtype=torch.uint8, device="cuda")
    key = ctypes.c_uint64(0)
    _check(_lib.load().fftpl_xindex_build(
        m, E, P, _ptr(net_ptr, torch.int32, E + 1, "net_ptr"),
        _ptr(pin_cell, torch.int32, P, "pin_cell"), int(max_degree),
        _ptr(index, torch.uint8, None, "index"), int(index.numel()),
        _ptr(work, torch.uint8, None, "work"), int(work.numel()), ctypes.byref(key),
        _stream(stream)), "fftpl_xindex_build")
    del work
    return int(key.value)


PATHS = ("xch", "slots", "atomic")


class Problem:
    """Device-resident static instance (sizes, netlist, fixed maps) and its
    fftpl_problem struct.  ``arrays`` holds the tensors the struct points to.

    ``path`` selects the evaluation path by what is built here:
    "xch" (default): the exchange index and the evaluation workspace;
    "slots": the cell-major pin slots and the workspace;
    "atomic": nothing (float atomics for the scatter and the wirelength).

    ``wl_model`` ("wa" or "lse") and ``screening`` (eps >= 0 of the
    screened solve) choose the objective; ``set_objective`` changes them
    later without rebuilding anything."""

    def __init__(self, grid: Grid, w, h, net_ptr, pin_cell, pin_dx, pin_dy,
                 base=None, cap=None, path="xch", stream=None, max_degree=None,
                 wl_model="wa", screening=0.0, own_work=True):
        if path not in PATHS:
            raise ValueError(f"path must be one of {PATHS}")
        if path != "atomic" and grid.n > 1024:
            raise ValueError("the atomic-free paths need n <= 1024; use path='atomic'")
        self.grid = grid
        self.path = path
        m = int(w.numel())
        E = int(net_ptr.numel()) - 1
        P = int(pin_cell.numel())
        n2 = grid.n * grid.n
        self.num_cells, self.num_nets, self.num_pins = m, E, P
        cell_ptr = pin_slot = work = xindex = None
        work_bytes = xbytes = xkey = 0
        if max_degree is None:
            max_degree = int((net_ptr[1:] - net_ptr[:-1]).max().item()) if E > 0 else 0
        self.max_degree = int(max_degree)
        self.work_bytes_needed = 0
        if path != "atomic":
            self.work_bytes_needed = problem_work_bytes(grid.n, m, E, P)
            if own_work:
                work_bytes = self.work_bytes_needed
                work = torch.empty(max(work_bytes, 1), dtype=torch.uint8, device="cuda")
        if path == "slots":
            cell_ptr = torch.empty(m + 1, dtype=torch.int32, device="cuda")
            pin_slot = torch.empty(max(P, 1), dtype=torch.int32, device="cuda")
            scratch = netlist_index(m, pin_cell, cell_ptr, pin_slot, stream=stream)
            torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
            del scratch
        elif path == "xch":
            xbytes, _ = xindex_bytes(m, E, P, self.max_degree)
            xindex = torch.empty(max(xbytes, 1), dtype=torch.uint8, device="cuda")
            xkey = xindex_build(m, net_ptr, pin_cell, self.max_degree, xindex, stream=stream)
        self.arrays = dict(w=w, h=h, net_ptr=net_ptr, pin_cell=pin_cell,
                           pin_dx=pin_dx, pin_dy=pin_dy, base=base, cap=cap,
                           cell_ptr=cell_ptr, pin_slot=pin_slot, work=work, xindex=xindex)
        self.c = _lib.fftpl_problem(
            grid.c(), m, E, P, WL_MODELS.get(wl_model, wl_model),
            _ptr(w, torch.float32, m, "w"), _ptr(h, torch.float32, m, "h"),
            _ptr(base, torch.float32, n2, "base"), _ptr(cap, torch.float32, n2, "cap"),
            _ptr(net_ptr, torch.int32, E + 1, "net_ptr"),
            _ptr(pin_cell, torch.int32, P, "pin_cell"),
            _ptr(pin_dx, torch.float32, P, "pin_dx"), _ptr(pin_dy, torch.float32, P, "pin_dy"),
            _ptr(cell_ptr, torch.int32, None, "cell_ptr"),
            _ptr(pin_slot, torch.int32, None, "pin_slot"),
            _ptr(work, torch.uint8, None, "work"), work_bytes,
            _ptr(xindex, torch.uint8, None, "xindex"), xbytes, self.max_degree,
            float(screening), xkey)

    def with_work(self, work) -> "Problem":
        """The same problem with the caller's workspace `work` (a uint8 device
        tensor of at least work_bytes_needed bytes) in place of its own; the
        static arrays and the index are shared, so views with distinct
        workspaces can be evaluated at the same time."""
        import copy
        if self.path == "atomic":
            raise ValueError("the float-atomic path has no workspace")
        if work.numel() < self.work_bytes_needed:
            raise ValueError(f"work needs {self.work_bytes_needed} bytes")
        v = copy.copy(self)
        v.c = _lib.fftpl_problem()
        ctypes.pointer(v.c)[0] = self.c
        v.c.work = _ptr(work, torch.uint8, None, "work")
        v.c.work_bytes = int(work.numel())
        v.arrays = dict(self.arrays, work=work)
        return v

    def set_objective(self, wl_model=None, screening=None) -> None:
        if wl_model is not None:
            self.c.wl_model = WL_MODELS.get(wl_model, wl_model)
        if screening is not None:
            self.c.screening = float(screening)

    @property
    def fast(self) -> bool:
        return self.path != "atomic"

    @classmethod
    def from_instance(cls, inst, device="cuda", stream=None, path="xch", wl_model="wa",
                      screening=0.0) -> "Problem":
        """Upload an instance's static arrays and rasterise its fixed maps."""
        def t(a, dt):
            return torch.as_tensor(a, dtype=dt).to(device).contiguous()
        grid = Grid.of(inst)
        n2 = grid.n * grid.n
        base = torch.empty(n2, dtype=torch.float32, device=device)
        cap = torch.empty(n2, dtype=torch.float32, device=device)
        fx = t(inst.fx, torch.float32) if inst.fx.size else None
        fixed_map(grid, fx, t(inst.fy, torch.float32) if fx is not None else None,
                  t(inst.fw, torch.float32) if fx is not None else None,
                  t(inst.fh, torch.float32) if fx is not None else None,
                  base, cap, stream=stream)
        return cls(grid, t(inst.w, torch.float32), t(inst.h, torch.float32),
                   t(inst.net_ptr, torch.int32), t(inst.pin_cell, torch.int32),
                   t(inst.pin_dx, torch.float32), t(inst.pin_dy, torch.float32),
                   base=base, cap=cap, path=path, stream=stream,
                   max_degree=int(np.diff(inst.net_ptr).max()) if inst.num_nets else 0,
                   wl_model=wl_model, screening=screening)


def problem_path(prob: Problem) -> str:
    """fftpl_problem_path: the path an evaluation of prob takes."""
    v = ctypes.c_int32()
    _check(_lib.load().fftpl_problem_path(ctypes.byref(prob.c), ctypes.byref(v)),
           "fftpl_problem_path")
    return PATHS[v.value]


def problem_density(prob: Problem, x, y, rho, stream=None):
    """fftpl_problem_density: rho = base + cells through the problem's workspace."""
    m = prob.num_cells
    n2 = prob.grid.n ** 2
    _check(_lib.load().fftpl_problem_density(
        ctypes.byref(prob.c), _ptr(x, torch.float32, m, "x"), _ptr(y, torch.float32, m, "y"),
        _ptr(rho, torch.float32, n2, "rho"), _stream(stream)), "fftpl_problem_density")


def problem_wl_grad(prob: Problem, x, y, gamma, accumulate, gx, gy, wl=None, hpwl=None,
                    stream=None):
    """fftpl_problem_wl_grad: the problem's wirelength model through its
    exchange index."""
    m = prob.num_cells
    _check(_lib.load().fftpl_problem_wl_grad(
        ctypes.byref(prob.c), _ptr(x, torch.float32, m, "x"), _ptr(y, torch.float32, m, "y"),
        float(gamma), int(accumulate), _ptr(gx, torch.float32, m, "gx"),
        _ptr(gy, torch.float32, m, "gy"), _ptr(wl, torch.float64, 1, "wl"),
        _ptr(hpwl, torch.float64, 1, "hpwl"), _stream(stream)), "fftpl_problem_wl_grad")


def debug_net_values(prob: Problem, x, y, gamma, wl_first, hpwl_first, stream=None):
    """fftpl_debug_net_values: per-net wirelength and HPWL at each net's first pin."""
    m, P = prob.num_cells, prob.num_pins
    _check(_lib.load().fftpl_debug_net_values(
        ctypes.byref(prob.c), _ptr(x, torch.float32, m, "x"), _ptr(y, torch.float32, m, "y"),
        float(gamma), _ptr(wl_first, torch.float64, P, "wl_first"),
        _ptr(hpwl_first, torch.float64, P, "hpwl_first"), _stream(stream)),
        "fftpl_debug_net_values")


def eval(plan: Plan, prob: Problem, x, y, lam, gamma, grad_mode, gx, gy, out4,
         stream=None):  # noqa: A001 - the C name
    m = prob.num_cells
    _check(_lib.load().fftpl_eval(
        plan.handle, ctypes.byref(prob.c), _ptr(x, torch.float32, m, "x"),
        _ptr(y, torch.float32, m, "y"), float(lam), float(gamma),
        GRAD_MODES.get(grad_mode, grad_mode),
        _ptr(gx, torch.float32, m, "gx") if gx is not None else None,
        _ptr(gy, torch.float32, m, "gy") if gy is not None else None,
        _ptr(out4, torch.float64, 4, "out4"),
        _stream(stream)), "fftpl_eval")


def eval_params(plan: Plan, prob: Problem, x, y, params, grad_mode, gx, gy, out4,
                stream=None):
    """fftpl_eval_params: fftpl_eval with (lambda, gamma) read on the device
    from params (a float32 device tensor of 2 entries)."""
    m = prob.num_cells
    _check(_lib.load().fftpl_eval_params(
        plan.handle, ctypes.byref(prob.c), _ptr(x, torch.float32, m, "x"),
        _ptr(y, torch.float32, m, "y"), _ptr(params, torch.float32, 2, "params"),
        GRAD_MODES.get(grad_mode, grad_mode), _ptr(gx, torch.float32, m, "gx"),
        _ptr(gy, torch.float32, m, "gy"), _ptr(out4, torch.float64, 4, "out4"),
        _stream(stream)), "fftpl_eval_params")


def eval_batch(plan: Plan, probs, xs, ys, lams, gammas, grad_mode, gxs, gys, out4s,
               stream=None):
    """fftpl_eval_batch: requests i = 0..len(probs)-1 in order on one stream.
    gxs and gys are lists of tensors, or None for the scalars only; out4s is
    a float64 device tensor [len(probs), 4]."""
    k = len(probs)
    if not (len(xs) == len(ys) == len(lams) == len(gammas) == k):
        raise ValueError("one x, y, lambda and gamma per problem")
    P = _lib.fftpl_problem
    pa = (P * max(k, 1))(*[pr.c for pr in probs])
    pp = (ctypes.POINTER(P) * max(k, 1))(*[ctypes.pointer(pa[i]) for i in range(k)])
    vp = lambda ts, name: (ctypes.c_void_p * max(k, 1))(
        *[_ptr(t, torch.float32, probs[i].num_cells, name) for i, t in enumerate(ts)])
    xa, ya = vp(xs, "x"), vp(ys, "y")
    la = (ctypes.c_float * max(k, 1))(*[float(v) for v in lams])
    ga = (ctypes.c_float * max(k, 1))(*[float(v) for v in gammas])
    gxa = vp(gxs, "gx") if gxs is not None else None
    gya = vp(gys, "gy") if gys is not None else None
    _check(_lib.load().fftpl_eval_batch(
        plan.handle, k, ctypes.cast(pp, ctypes.POINTER(ctypes.POINTER(P))),
        ctypes.cast(xa, ctypes.POINTER(ctypes.c_void_p)),
        ctypes.cast(ya, ctypes.POINTER(ctypes.c_void_p)),
        ctypes.cast(la, ctypes.POINTER(ctypes.c_float)),
        ctypes.cast(ga, ctypes.POINTER(ctypes.c_float)),
        GRAD_MODES.get(grad_mode, grad_mode),
        ctypes.cast(gxa, ctypes.POINTER(ctypes.c_void_p)) if gxa is not None else None,
        ctypes.cast(gya, ctypes.POINTER(ctypes.c_void_p)) if gya is not None else None,
        _ptr(out4s, torch.float64, 4 * k, "out4s"), _stream(stream)), "fftpl_eval_batch")


def debug_cell_bins(grid: Grid, x, y, w, h, ranges, stream=None):
    m = int(x.numel())
    _check(_lib.load().fftpl_debug_cell_bins(
        ctypes.byref(grid.c()), m, _ptr(x, torch.float32, m, "x"),
        _ptr(y, torch.float32, m, "y"), _ptr(w, torch.float32, m, "w"),
        _ptr(h, torch.float32, m, "h"), _ptr(ranges, torch.int32, 4 * m, "ranges"),
        _stream(stream)), "fftpl_debug_cell_bins")
