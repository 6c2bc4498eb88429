"""Global placement loop around the evaluation (Algorithm 1).

Each iteration evaluates f = W~ + lambda N and its gradient at the look-ahead
point (fftpl_eval), reduces the step statistics on the device
(fftpl_step_stats) and moves every cell (fftpl_nesterov_update).  The host
only reads eight doubles per iteration (the scalars and the statistics) to
set the next step length, lambda and gamma; ``Placer.run_device`` runs the
same rule on the device (fftpl_nesterov_schedule), so that iterations are
enqueued, or replayed from a HIP graph, without that read.

Schedules (Section IV-A):
* step length: a Barzilai-Borwein estimate |du| / |dg| of the inverse
  Lipschitz constant, expressed as the largest cell displacement and kept in
  [alpha_min, alpha_max] with alpha_max_0 = 0.044 bin widths,
  alpha_max_k = max(alpha_max_0, 2 alpha_k), alpha_min = 0.01 alpha_max;
* gamma = 8 w_b 10^(20/9 (tau - 0.1) - 1) from the current overflow tau;
* lambda_0 = sum |grad W~| / sum |grad N| at the start; then either doubled
  every ``lam_every`` iterations, or the paper's mu_k = 1.1^(1 - dW / 3.5e5)
  bounded to [0.75, 1.1] from the HPWL change;
* optional stop when tau <= 0.1;
* the momentum restarts (a = 1) whenever lambda doubles: the penalty term
  then changes the landscape, and momentum built on the old one makes the
  late, density-dominated iterations wander (overflow and wirelength grow
  again after a few hundred iterations without the restart).
Two inner solvers (``Schedule.solver``):
* "cg", the paper's (Algorithm 1, "CGsolver"): nonlinear conjugate gradients,
  Polak-Ribiere with restarts (beta = max(0, g.(g - g_prev) / |g_prev|^2);
  d = -g when that is not a descent direction), and per outer iteration one
  backtracking line search inside the step interval [alpha_min, alpha_max],
  expressed as the largest cell displacement: it starts at alpha_max, halves
  until f = W~ + lambda N has fallen by the Armijo amount, and stops at
  alpha_min.  Each trial costs a scalars-only evaluation.
* "nesterov": Nesterov's method with a Barzilai-Borwein step in the same
  interval (no line search: one evaluation per iteration).

Fillers (Section III-B): with ``fillers=True`` disconnected movable cells
are appended after the real ones so that movable plus filler area equals the
capacity the fixed and dark nodes leave (rho_t times the whitespace).  They
take part in the density and the update like any cell and have no pins; the
overflow tau that drives gamma and the stop is that of the real cells alone
(a second, scalars-only evaluation of the real cells per iteration).
Irregular regions enter through their dark nodes (``fftpl.dark_nodes``)
added to the instance's fixed rectangles.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Callable, Dict, Iterable, List, Optional

import numpy as np
import torch

from . import _lib, fftpl


def gamma_of_tau(tau: float, bin_w: float) -> float:
    """Section IV-A: gamma = 8 w_b 10^(20/9 (tau - 0.1) - 1)."""
    return 8.0 * bin_w * 10.0 ** (20.0 / 9.0 * (tau - 0.1) - 1.0)


def mu_of_hpwl_change(dw: float, dw_ref: float = 3.5e5) -> float:
    """Section IV-A: mu_k = 1.1^(1 - dW/dW_ref), bounded to [0.75, 1.1]."""
    return min(1.1, max(0.75, 1.1 ** (1.0 - dw / dw_ref)))


def nesterov_beta(a: float):
    """a_{k+1} = (1 + sqrt(4 a_k^2 + 1)) / 2 and beta_k = (a_k - 1) / a_{k+1}."""
    a1 = 0.5 * (1.0 + math.sqrt(4.0 * a * a + 1.0))
    return a1, (a - 1.0) / a1


def step_length(du2: float, dg2: float, gmax: float, alpha_min: float, alpha_max: float,
                first: bool) -> float:
    """Largest cell displacement of this step: alpha_max on the first step,
    else the BB estimate sqrt(du2/dg2) * gmax kept in [alpha_min, alpha_max]."""
    if first or dg2 <= 0.0 or du2 <= 0.0:
        return alpha_max
    return min(alpha_max, max(alpha_min, math.sqrt(du2 / dg2) * gmax))


def pr_beta(gg: float, ggp: float, gpgp: float) -> float:
    """Polak-Ribiere with restart: max(0, g.(g - g_prev) / |g_prev|^2)."""
    if gpgp <= 0.0:
        return 0.0
    return max(0.0, (gg - ggp) / gpgp)


def backtrack(phi: Callable[[float], float], f0: float, slope: float, alpha_max: float,
              alpha_min: float, dmax: float, c1: float = 1e-4, shrink: float = 0.5):
    """Backtracking line search inside [alpha_min, alpha_max] (step lengths as
    the largest cell displacement; the move along the direction is t =
    alpha / dmax).  phi(alpha) evaluates the objective after that move.
    Starts at alpha_max and shrinks by `shrink` until the Armijo condition
    f <= f0 + c1 t slope holds (slope = g.d < 0); at alpha_min the step is
    taken as it is.  Returns (alpha, f(alpha), trials)."""
    alpha = alpha_max
    trials = 0
    while True:
        f = phi(alpha)
        trials += 1
        t = alpha / dmax if dmax > 0 else 0.0
        if f <= f0 + c1 * t * slope or alpha <= alpha_min:
            return alpha, f, trials
        alpha = max(alpha_min, alpha * shrink)


def filler_cells(inst, cap_area: float, seed: int = 0):
    """Fillers of Section III-B: total filler area = cap_area - the movable
    cells' area, with cap_area the movable capacity of the region (bin area
    times the sum of the capacity map, i.e. rho_t times the area the fixed
    and dark nodes leave).  The paper does not size them; here each filler
    has the mean width and the mean height of the movable cells, and they
    start uniformly at random inside the region.  Returns float32 arrays
    (x, y, w, h), empty when the movable cells already fill the capacity."""
    w = np.asarray(inst.w, np.float64)
    h = np.asarray(inst.h, np.float64)
    empty = tuple(np.zeros(0, np.float32) for _ in range(4))
    if w.size == 0:
        return empty
    need = float(cap_area) - float(np.sum(w * h))
    fw, fh = float(np.mean(w)), float(np.mean(h))
    count = int(math.floor(need / (fw * fh))) if need > 0 else 0
    if count <= 0:
        return empty
    rng = np.random.default_rng(seed)
    xl, yl = float(inst.xl), float(inst.yl)
    sx, sy = inst.n * float(inst.bin_w), inst.n * float(inst.bin_h)
    x = xl + 0.5 * fw + rng.random(count) * max(sx - fw, 0.0)
    y = yl + 0.5 * fh + rng.random(count) * max(sy - fh, 0.0)
    return (x.astype(np.float32), y.astype(np.float32),
            np.full(count, fw, np.float32), np.full(count, fh, np.float32))


@dataclasses.dataclass
class Schedule:
    lam_mode: str = "double"         # "double" (every lam_every iterations) or "paper"
    lam_every: int = 50
    alpha_max0_bins: float = 0.044
    stop_tau: Optional[float] = None  # stop when tau <= stop_tau (the paper: 0.1)
    grad_mode: str = "field"
    restart_on_lambda: bool = True   # restart the momentum when lambda changes
    wl_model: str = "wa"             # "wa" (Eq. (3)) or "lse"
    screening: float = 0.0           # eps of the screened solve (0: Poisson)
    solver: str = "nesterov"         # "nesterov" or "cg" (the paper's)


def paper_schedule(**kw) -> Schedule:
    """Algorithm 1 as printed: nonlinear CG, lambda_k = mu_k lambda_(k-1),
    stop when tau <= 10%."""
    kw.setdefault("solver", "cg")
    kw.setdefault("lam_mode", "paper")
    kw.setdefault("stop_tau", 0.1)
    return Schedule(**kw)


class Placer:
    """Nesterov global placement on one device.  ``inst`` gives the netlist,
    sizes, fixed maps and starting positions.  With ``fillers`` the cells
    past ``num_real`` are fillers (``positions()`` returns the real ones)."""

    def __init__(self, inst, dct: str = "fft", schedule: Schedule = Schedule(),
                 stream=None, fillers: bool = False, filler_seed: int = 0):
        self.sched = schedule
        obj = dict(wl_model=schedule.wl_model, screening=schedule.screening)
        self.num_real = inst.num_cells
        self.prob_real = None
        if fillers:
            # the real cells alone (no nets): their capacity map sizes the
            # fillers, and their scalars-only evaluation gives tau
            bare = dataclasses.replace(
                inst, net_ptr=np.zeros(1, np.int32), pin_cell=np.zeros(0, np.int32),
                pin_dx=np.zeros(0, np.float32), pin_dy=np.zeros(0, np.float32))
            self.prob_real = fftpl.Problem.from_instance(bare, stream=stream, **obj)
            cap = self.prob_real.arrays["cap"]
            cap_area = float(cap.double().sum()) * float(inst.bin_w) * float(inst.bin_h)
            fx, fy, fw, fh = filler_cells(inst, cap_area, filler_seed)
            inst = dataclasses.replace(
                inst, x=np.concatenate([inst.x, fx]), y=np.concatenate([inst.y, fy]),
                w=np.concatenate([inst.w, fw]), h=np.concatenate([inst.h, fh]))
        self.inst = inst
        self.num_fillers = inst.num_cells - self.num_real
        self.prob = fftpl.Problem.from_instance(inst, stream=stream, **obj)
        self.plan = fftpl.Plan(inst.n, dct)
        self.region = fftpl.Grid.of(inst)
        m = inst.num_cells
        dev = "cuda"
        f32 = dict(dtype=torch.float32, device=dev)
        self.x = torch.as_tensor(inst.x, dtype=torch.float32).to(dev).contiguous()
        self.y = torch.as_tensor(inst.y, dtype=torch.float32).to(dev).contiguous()
        self.ux, self.uy = self.x.clone(), self.y.clone()
        self.upx, self.upy = torch.zeros(m, **f32), torch.zeros(m, **f32)
        self.gpx, self.gpy = torch.zeros(m, **f32), torch.zeros(m, **f32)
        self.gx, self.gy = torch.empty(m, **f32), torch.empty(m, **f32)
        # out4 | step statistics | real cells' out4 (fillers only)
        self.scal = torch.zeros(12, dtype=torch.float64, device=dev)
        self.work = torch.empty(1024, dtype=torch.float64, device=dev)
        self.k = 0
        self.a = 1.0
        bw = float(inst.bin_w)
        self.alpha_max0 = schedule.alpha_max0_bins * bw
        self.alpha_max = self.alpha_max0
        self.alpha_min = 0.01 * self.alpha_max
        self.gamma = gamma_of_tau(1.0, bw)
        self.lam = None
        self.last_hpwl = None
        self.history: List[Dict[str, float]] = []

    # -- device calls ------------------------------------------------------
    def _eval(self, lam: float, gamma: float, gx=None, gy=None):
        fftpl.eval(self.plan, self.prob, self.ux, self.uy, lam, gamma, self.sched.grad_mode,
                   self.gx if gx is None else gx, self.gy if gy is None else gy, self.scal[:4])
        if self.prob_real is not None:
            r = self.num_real
            fftpl.eval(self.plan, self.prob_real, self.ux[:r], self.uy[:r], lam, gamma,
                       self.sched.grad_mode, None, None, self.scal[8:12])

    def positions(self):
        """Current centres of the real cells (fillers dropped), on the host."""
        torch.cuda.synchronize()
        r = self.num_real
        return self.x[:r].cpu().numpy(), self.y[:r].cpu().numpy()

    def _stats(self, first: bool):
        lib = _lib.load()
        p = fftpl._ptr
        none = None
        st = lib.fftpl_step_stats(
            self.inst.num_cells, p(self.ux), p(self.uy),
            none if first else p(self.upx), none if first else p(self.upy),
            p(self.gx), p(self.gy), none if first else p(self.gpx),
            none if first else p(self.gpy), p(self.scal) + 32, p(self.work),
            self.work.numel(), fftpl._stream(None))
        fftpl._check(st, "fftpl_step_stats")

    def _cg_dots(self, first: bool):
        p = fftpl._ptr
        st = _lib.load().fftpl_cg_dots(
            self.inst.num_cells, p(self.gx), p(self.gy), None if first else p(self.gpx),
            None if first else p(self.gpy), None if first else p(self.upx),
            None if first else p(self.upy), p(self.scal) + 32, p(self.work),
            self.work.numel(), fftpl._stream(None))
        fftpl._check(st, "fftpl_cg_dots")

    def _cg_direction(self, beta: float):
        # the direction d lives in (upx, upy); max |d| into scal[7]
        p = fftpl._ptr
        st = _lib.load().fftpl_cg_direction(
            self.inst.num_cells, p(self.gx), p(self.gy), float(beta), p(self.upx),
            p(self.upy), p(self.scal) + 56, p(self.work), self.work.numel(),
            fftpl._stream(None))
        fftpl._check(st, "fftpl_cg_direction")

    def _cg_move(self, t: float, xo, yo):
        p = fftpl._ptr
        a = self.prob.arrays
        st = _lib.load().fftpl_cg_move(
            ctypes.byref(self.region.c()), self.inst.num_cells, p(a["w"]), p(a["h"]), p(self.x),
            p(self.y), p(self.upx), p(self.upy), float(t), p(xo), p(yo), fftpl._stream(None))
        fftpl._check(st, "fftpl_cg_move")

    def _update(self, step: float, beta: float):
        lib = _lib.load()
        p = fftpl._ptr
        a = self.prob.arrays
        st = lib.fftpl_nesterov_update(
            ctypes.byref(self.region.c()), self.inst.num_cells, p(a["w"]), p(a["h"]),
            p(self.x), p(self.y), p(self.ux), p(self.uy), p(self.upx), p(self.upy),
            p(self.gpx), p(self.gpy), p(self.gx), p(self.gy), float(step), float(beta),
            fftpl._stream(None))
        fftpl._check(st, "fftpl_nesterov_update")

    def initial_lambda(self) -> float:
        """lambda_0 = sum |grad W~| / sum |grad N| at the current positions."""
        m = self.inst.num_cells
        g0x, g0y = torch.empty(m, device="cuda"), torch.empty(m, device="cuda")
        self._eval(0.0, self.gamma, g0x, g0y)
        self._eval(1.0, self.gamma)
        gw = float(g0x.abs().sum() + g0y.abs().sum())
        gn = float((self.gx - g0x).abs().sum() + (self.gy - g0y).abs().sum())
        return gw / gn if gn > 0 else 1.0

    # -- the loop ----------------------------------------------------------
    def _cg_step(self, on_eval) -> Dict[str, float]:
        """One outer iteration of Algorithm 1 with the CG inner solver.  The
        gradient is taken at x (u = x); the direction is kept in (upx, upy)
        and the previous gradient in (gpx, gpy); trial points go to (ux, uy)."""
        first = self.k == 0
        self.ux.copy_(self.x)
        self.uy.copy_(self.y)
        self._eval(self.lam, self.gamma)
        self._cg_dots(first)
        s = self.scal.cpu().numpy()
        N, W, H, tau = (float(v) for v in s[:4])
        gg, ggp, gpgp, gd = (float(v) for v in s[4:8])
        if self.prob_real is not None:
            tau = float(s[11])
        if on_eval is not None:
            on_eval(self)
        f0 = W + self.lam * N
        beta = 0.0 if first else pr_beta(gg, ggp, gpgp)
        slope = -gg + beta * gd
        if beta > 0.0 and slope >= 0.0:      # not a descent direction: restart
            beta, slope = 0.0, -gg
        self._cg_direction(beta)
        dmax = float(self.scal[7].item())
        restarted = beta == 0.0

        def phi(alpha):
            t = alpha / dmax if dmax > 0 else 0.0
            self._cg_move(t, self.ux, self.uy)
            fftpl.eval(self.plan, self.prob, self.ux, self.uy, self.lam, self.gamma,
                       self.sched.grad_mode, None, None, self.scal[:4])
            o = self.scal[:2].cpu().numpy()
            return float(o[1]) + self.lam * float(o[0])

        alpha, f1, trials = backtrack(phi, f0, slope, self.alpha_max, self.alpha_min, dmax)
        # accept the last trial point: x = u; the gradient becomes the previous one
        self.x.copy_(self.ux)
        self.y.copy_(self.uy)
        self.gpx.copy_(self.gx)
        self.gpy.copy_(self.gy)
        rec = dict(k=self.k, energy=N, wa=W, hpwl=H, tau=tau, lam=self.lam, gamma=self.gamma,
                   alpha=alpha, f=f0, f_next=f1, trials=trials, beta=beta,
                   restart=float(restarted))
        self.history.append(rec)
        self.alpha_max = max(self.alpha_max0, 2.0 * alpha)
        self.alpha_min = 0.01 * self.alpha_max
        self.gamma = gamma_of_tau(tau, float(self.inst.bin_w))
        self._next_lambda(H)
        self.k += 1
        return rec

    def _next_lambda(self, H: float) -> None:
        if self.sched.lam_mode == "double":
            if (self.k + 1) % self.sched.lam_every == 0:
                self.lam *= 2.0
                if self.sched.restart_on_lambda:
                    self.a = 1.0
        else:
            if self.last_hpwl is not None:
                self.lam *= mu_of_hpwl_change(H - self.last_hpwl)
        self.last_hpwl = H

    def step(self, on_eval: Optional[Callable[["Placer"], None]] = None) -> Dict[str, float]:
        if self.lam is None:
            self.lam = self.initial_lambda()
        if self.sched.solver == "cg":
            return self._cg_step(on_eval)
        first = self.k == 0
        self._eval(self.lam, self.gamma)
        self._stats(first)
        s = self.scal.cpu().numpy()        # one small read per iteration
        N, W, H, tau, du2, dg2, gmax, _ = (float(v) for v in s[:8])
        if self.prob_real is not None:
            tau = float(s[11])             # the real cells' overflow
        if on_eval is not None:
            on_eval(self)
        alpha = step_length(du2, dg2, gmax, self.alpha_min, self.alpha_max, first)
        a1, beta = nesterov_beta(self.a)
        self._update(alpha / gmax if gmax > 0 else 0.0, beta)
        rec = dict(k=self.k, energy=N, wa=W, hpwl=H, tau=tau, lam=self.lam, gamma=self.gamma,
                   alpha=alpha)
        self.history.append(rec)
        # next iteration's parameters
        self.a = a1
        self.alpha_max = max(self.alpha_max0, 2.0 * alpha)
        self.alpha_min = 0.01 * self.alpha_max
        self.gamma = gamma_of_tau(tau, float(self.inst.bin_w))
        self._next_lambda(H)
        self.k += 1
        return rec

    def run(self, iters: int, on_eval: Optional[Callable[["Placer"], None]] = None,
            trace: Optional[str] = None, checkpoint: Optional[str] = None,
            checkpoint_every: int = 50) -> List[Dict[str, float]]:
        """``iters`` iterations (fewer if the schedule's stop test fires).
        ``trace``: a JSON-lines file that gets one record per iteration (k,
        energy N, wa W~, hpwl, tau, lam, gamma, alpha, ...), appended as the
        iterations complete.  ``checkpoint``: an .npz path saved every
        ``checkpoint_every`` iterations and after the last one (load() resumes
        from it)."""
        for _ in range(iters):
            rec = self.step(on_eval)
            if trace is not None:
                self._trace(trace, [rec])
            stop = self.sched.stop_tau is not None and rec["tau"] <= self.sched.stop_tau
            if checkpoint is not None and (self.k % checkpoint_every == 0 or stop):
                self.save(checkpoint)
            if stop:
                break
        if checkpoint is not None and self.k % checkpoint_every != 0:
            self.save(checkpoint)
        return self.history

    @staticmethod
    def _trace(path: str, recs) -> None:
        import json
        with open(path, "a") as f:
            for r in recs:
                f.write(json.dumps({k: (int(v) if k == "k" else float(v)) for k, v in r.items()})
                        + "\n")

    def run_device(self, iters: int, graph: bool = True,
                   between: Optional[Callable[[int], None]] = None,
                   trace: Optional[str] = None) -> List[Dict[str, float]]:
        """``iters`` Nesterov iterations with the schedule on the device: each
        is fftpl_eval_params, fftpl_step_stats, fftpl_nesterov_schedule and
        fftpl_nesterov_update_dev, with no host read until the end (with
        ``graph``, one iteration is captured in a HIP graph and replayed).
        The rule is step()'s (the first iteration, which has no previous point,
        runs through step()).  The exchange path and the Nesterov solver only,
        without fillers, stop_tau or a per-evaluation callback.  ``between(i)``,
        if given, runs on the host after the i-th device iteration is enqueued
        (a test hook: it may synchronise and read state).  ``trace``: as in
        run(), written when the device log is read back at the end."""
        if self.sched.solver != "nesterov":
            raise ValueError("run_device runs the Nesterov solver")
        if self.prob_real is not None or self.sched.stop_tau is not None:
            raise ValueError("run_device has no fillers and no stop test")
        if self.prob.path != "xch":
            raise ValueError("run_device needs the exchange path")
        if iters <= 0:
            return self.history
        if self.k == 0:
            self.step()
            if trace is not None:
                self._trace(trace, self.history[-1:])
            iters -= 1
            if iters == 0:
                return self.history
        dev = "cuda"
        last = float("nan") if self.last_hpwl is None else float(self.last_hpwl)
        st = torch.tensor([self.a, self.alpha_max, self.alpha_min, self.lam, self.gamma,
                           float(self.k), last, self.alpha_max0, float(self.inst.bin_w),
                           0.0 if self.sched.lam_mode == "double" else 1.0,
                           float(self.sched.lam_every),
                           1.0 if self.sched.restart_on_lambda else 0.0, 0.0, 0.0,
                           float(self.k), 0.0], dtype=torch.float64, device=dev)
        params = torch.tensor([self.lam, self.gamma], dtype=torch.float32, device=dev)
        log = torch.zeros(8 * iters, dtype=torch.float64, device=dev)
        lib = _lib.load()
        p = fftpl._ptr
        a = self.prob.arrays
        m = self.inst.num_cells

        def one():
            fftpl.eval_params(self.plan, self.prob, self.ux, self.uy, params,
                              self.sched.grad_mode, self.gx, self.gy, self.scal[:4])
            self._stats(False)
            s = fftpl._stream(None)
            fftpl._check(lib.fftpl_nesterov_schedule(
                p(self.scal) + 32, p(self.scal), p(st), p(params), p(log), iters, s),
                "fftpl_nesterov_schedule")
            fftpl._check(lib.fftpl_nesterov_update_dev(
                ctypes.byref(self.region.c()), m, p(a["w"]), p(a["h"]), p(self.x), p(self.y),
                p(self.ux), p(self.uy), p(self.upx), p(self.upy), p(self.gpx), p(self.gpy),
                p(self.gx), p(self.gy), p(st) + 12 * 8, s), "fftpl_nesterov_update_dev")

        if graph:
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                one()
            for i in range(iters):
                g.replay()
                if between is not None:
                    between(i)
        else:
            for i in range(iters):
                one()
                if between is not None:
                    between(i)
        torch.cuda.synchronize()
        sv = st.cpu().numpy()
        first = len(self.history)
        for r in log.cpu().numpy().reshape(iters, 8):
            self.history.append(dict(k=int(r[0]), energy=float(r[1]), wa=float(r[2]),
                                     hpwl=float(r[3]), tau=float(r[4]), lam=float(r[5]),
                                     gamma=float(r[6]), alpha=float(r[7])))
        if trace is not None:
            self._trace(trace, self.history[first:])
        self.a, self.alpha_max, self.alpha_min = float(sv[0]), float(sv[1]), float(sv[2])
        self.lam, self.gamma, self.k = float(sv[3]), float(sv[4]), int(sv[5])
        self.last_hpwl = None if math.isnan(sv[6]) else float(sv[6])
        return self.history

    # -- checkpoint / resume -------------------------------------------------
    def state(self) -> Dict[str, np.ndarray]:
        torch.cuda.synchronize()
        st = {name: getattr(self, name).cpu().numpy()
              for name in ("x", "y", "ux", "uy", "upx", "upy", "gpx", "gpy")}
        scal = dict(k=self.k, a=self.a, alpha_max=self.alpha_max, alpha_min=self.alpha_min,
                    gamma=self.gamma, lam=np.nan if self.lam is None else self.lam,
                    last_hpwl=np.nan if self.last_hpwl is None else self.last_hpwl)
        st["scalars"] = np.array([scal[k] for k in sorted(scal)], np.float64)
        st["scalar_names"] = np.array(sorted(scal))
        keys = sorted(self.history[0]) if self.history else []
        st["history"] = np.array([[h[k] for k in keys] for h in self.history], np.float64)
        st["history_names"] = np.array(keys)
        return st

    def save(self, path: str) -> None:
        np.savez(path, **self.state())

    def load(self, path: str) -> None:
        d = np.load(path, allow_pickle=False)
        for name in ("x", "y", "ux", "uy", "upx", "upy", "gpx", "gpy"):
            getattr(self, name).copy_(torch.as_tensor(d[name]))
        sc = dict(zip([str(s) for s in d["scalar_names"]], d["scalars"].tolist()))
        self.k = int(sc["k"])
        self.a = sc["a"]
        self.alpha_max, self.alpha_min = sc["alpha_max"], sc["alpha_min"]
        self.gamma = sc["gamma"]
        self.lam = None if math.isnan(sc["lam"]) else sc["lam"]
        self.last_hpwl = None if math.isnan(sc["last_hpwl"]) else sc["last_hpwl"]
        names = [str(s) for s in d["history_names"]]
        self.history = [dict(zip(names, row.tolist())) for row in d["history"]]
        for h in self.history:
            h["k"] = int(h["k"])
        torch.cuda.synchronize()

    def close(self) -> None:
        self.plan.close()
