"""Differentiation form: the objective W~ + lambda N as a torch.autograd
function whose backward recomputes the density and the spectral solve
instead of keeping grid-sized tensors, checked against the FP64 oracle's
exact gradient and against central finite differences of the objective."""
import numpy as np
import pytest

import gen
import oracle
from tests.gpu_common import RTOL, host, lib_or_build, say

pytestmark = pytest.mark.gpu

LAM = 1.5


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_or_build()
    from paper_1312_4587_amd import autograd, fftpl
    return fftpl, autograd


def _setup(F, inst):
    import torch
    fftpl, _ = F
    prob = fftpl.Problem.from_instance(inst)
    plan = fftpl.Plan(inst.n, "fft")
    x = torch.as_tensor(inst.x).cuda().requires_grad_(True)
    y = torch.as_tensor(inst.y).cuda().requires_grad_(True)
    return prob, plan, x, y


def test_autograd_against_oracle_and_finite_differences(F):
    # the differentiation workload: 500k cells, n = 512, mixed netlist
    import torch
    fftpl, ag = F
    inst = gen.make_config("diff_500k")
    say("autograd diff_500k", inst.num_cells, inst.num_pins)
    prob, plan, x, y = _setup(F, inst)
    loss, scalars = ag.objective(x, y, plan, prob, LAM, inst.gamma)
    loss.backward()
    torch.cuda.synchronize()
    gx, gy = host(x.grad), host(y.grad)
    ref = oracle.evaluate(inst, lam=LAM, grad_mode="exact")
    say("loss", float(loss), ref["loss"])
    assert abs(float(loss) - ref["loss"]) <= RTOL * abs(ref["loss"])
    assert abs(float(scalars[0]) - ref["energy"]) <= RTOL * abs(ref["energy"])
    err = np.linalg.norm(np.concatenate([gx - ref["gx"], gy - ref["gy"]])) / \
        np.linalg.norm(np.concatenate([ref["gx"], ref["gy"]]))
    say("gradient vs oracle rel-L2", err)
    assert err < RTOL
    # central differences (h = 1e-3 bin) on a random subset of 1000 cells
    cells = np.random.default_rng(40).choice(inst.num_cells, 1000, replace=False)
    fx, fy, kink = oracle.local_fd_gradient(inst, cells, 1e-3, LAM, psi=ref["psi"])
    ok = ~kink
    say("finite differences: cells", ok.sum(), "kink cells excluded", kink.sum())
    assert kink.sum() < 100
    got = np.concatenate([gx[cells][ok], gy[cells][ok]])
    fd = np.concatenate([fx[ok], fy[ok]])
    e_fd = np.linalg.norm(got - fd) / np.linalg.norm(fd)
    say("gradient vs finite differences rel-L2", e_fd)
    assert e_fd < RTOL
    plan.close()


def test_backward_recomputes_and_scales_at_n1024(F):
    # 2.1M cells at n = 1024: backward keeps only the positions, and its
    # gradient is the plain exact-mode evaluation's, times the upstream weight
    import torch
    fftpl, ag = F
    inst = gen.make_config("large_2m")
    say("autograd large_2m")
    prob, plan, x, y = _setup(F, inst)
    loss, _ = ag.objective(x, y, plan, prob, LAM, inst.gamma)
    saved = loss.grad_fn.saved_tensors
    assert len(saved) == 2 and all(t.numel() == inst.num_cells for t in saved)
    (3.0 * loss).backward()
    gx = torch.empty(inst.num_cells, device="cuda")
    gy = torch.empty_like(gx)
    out4 = torch.empty(4, dtype=torch.float64, device="cuda")
    fftpl.eval(plan, prob, x.detach(), y.detach(), LAM, inst.gamma, "exact", gx, gy, out4)
    torch.cuda.synchronize()
    rx = np.linalg.norm(host(x.grad) - 3.0 * host(gx)) / np.linalg.norm(3.0 * host(gx))
    ry = np.linalg.norm(host(y.grad) - 3.0 * host(gy)) / np.linalg.norm(3.0 * host(gy))
    say("backward vs eval", rx, ry)
    assert rx < 1e-6 and ry < 1e-6
    assert abs(float(loss) - (float(out4[1]) + LAM * float(out4[0]))) <= 1e-9 * abs(float(loss))
    plan.close()


def test_loss_only_evaluation_needs_an_index(F):
    import torch
    fftpl, ag = F
    inst = gen.make_config("small_2k")
    prob = fftpl.Problem.from_instance(inst, path="atomic")
    plan = fftpl.Plan(inst.n, "fft")
    x = torch.as_tensor(inst.x).cuda()
    y = torch.as_tensor(inst.y).cuda()
    out4 = torch.empty(4, dtype=torch.float64, device="cuda")
    with pytest.raises(fftpl.FFTPLError) as ei:
        fftpl.eval(plan, prob, x, y, 1.0, inst.gamma, "exact", None, None, out4)
    assert ei.value.status == fftpl.E_INVAL
    with pytest.raises(ValueError):
        ag.objective(x, y, plan, prob, 1.0, inst.gamma)
    plan.close()
