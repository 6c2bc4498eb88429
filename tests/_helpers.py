"""Small helpers shared by the tests (no method arithmetic here)."""
import dataclasses
import os

import numpy as np

import gen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def tiny_instance(seed=0, m=60, n=16, num_nets=50, util=0.6, macros=0,
                  macro_frac=0.0, **kw):
    return gen.make_instance(seed, num_cells=m, util=util, n=n,
                             num_nets=num_nets, num_macros=macros,
                             macro_area_frac=macro_frac, **kw)


def hand_instance(cells, n, bin_size=1.0, origin=0.0, nets=None):
    """An Instance from explicit (cx, cy, w, h) rows and explicit nets
    (lists of (cell, dx, dy))."""
    cells = np.asarray(cells, np.float64).reshape(-1, 4)
    nets = nets or []
    ptr = [0]
    pc, pdx, pdy = [], [], []
    for net in nets:
        for (c, dx, dy) in net:
            pc.append(c)
            pdx.append(dx)
            pdy.append(dy)
        ptr.append(len(pc))
    z = np.zeros(0, np.float32)
    return gen.Instance(
        n=n, xl=origin, yl=origin, bin_w=bin_size, bin_h=bin_size,
        target_density=1.0,
        x=cells[:, 0].astype(np.float32), y=cells[:, 1].astype(np.float32),
        w=cells[:, 2].astype(np.float32), h=cells[:, 3].astype(np.float32),
        fx=z, fy=z.copy(), fw=z.copy(), fh=z.copy(),
        net_ptr=np.asarray(ptr, np.int32), pin_cell=np.asarray(pc, np.int32),
        pin_dx=np.asarray(pdx, np.float32), pin_dy=np.asarray(pdy, np.float32),
        gamma=0.5 * bin_size, side=n * bin_size)


def with_macros(inst, macros):
    macros = np.asarray(macros, np.float32).reshape(-1, 4)
    return dataclasses.replace(inst, fx=macros[:, 0], fy=macros[:, 1],
                               fw=macros[:, 2], fh=macros[:, 3])


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.linalg.norm((a - b).ravel())
    s = np.linalg.norm(b.ravel())
    return d / s if s > 0 else d


def load_golden_density(name="tiny_density.txt"):
    cells, rows = [], []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "cell":
                cells.append([float(v) for v in t[1:5]])
            elif t[0] == "row":
                rows.append([float(v) for v in t[1:]])
    return cells, np.asarray(rows)
