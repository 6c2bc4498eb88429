"""Helpers for the GPU parity tests (device upload, the HIP path through the
binding, and the oracle side).  Imports torch and the binding lazily."""
import os
import sys

import numpy as np

RTOL = 1e-5          # relative L2 bound for float32 GPU vs float64 oracle


def lib_or_build():
    """Load libfftpl.so, building it first when it is missing or was built
    from other sources than the ones in the tree."""
    from paper_1312_4587_amd import _lib, build
    build.ensure_built()
    _lib.load()


def dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def host(t):
    return t.detach().cpu().numpy()


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


class DeviceCells:
    def __init__(self, inst):
        import torch
        self.x = dev(inst.x, torch.float32)
        self.y = dev(inst.y, torch.float32)
        self.w = dev(inst.w, torch.float32)
        self.h = dev(inst.h, torch.float32)
