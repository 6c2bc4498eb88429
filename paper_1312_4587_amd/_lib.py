"""ctypes loader for libfftpl.so.  Loading fails loudly when the HIP library
has not been built; there is no fallback implementation."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# FFTPL_ROCTX=1: the build with roctx ranges around the entry points
LIB_PATH = os.path.join(_HERE, "libfftpl_roctx.so" if os.environ.get("FFTPL_ROCTX") == "1"
                        else "libfftpl.so")

c_int = ctypes.c_int32
c_float = ctypes.c_float
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_char_p = ctypes.c_char_p


class fftpl_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("xl", c_double), ("yl", c_double),
                ("bin_w", c_double), ("bin_h", c_double),
                ("target_density", c_double)]


class fftpl_problem(ctypes.Structure):
    _fields_ = [("grid", fftpl_grid),
                ("num_cells", ctypes.c_int32), ("num_nets", ctypes.c_int32),
                ("num_pins", ctypes.c_int32), ("wl_model", ctypes.c_int32),
                ("w", c_void_p), ("h", c_void_p), ("base", c_void_p),
                ("cap", c_void_p), ("net_ptr", c_void_p), ("pin_cell", c_void_p),
                ("pin_dx", c_void_p), ("pin_dy", c_void_p),
                ("cell_ptr", c_void_p), ("pin_slot", c_void_p),
                ("work", c_void_p), ("work_bytes", ctypes.c_uint64),
                ("xindex", c_void_p), ("xindex_bytes", ctypes.c_uint64),
                ("max_degree", ctypes.c_int32), ("screening", ctypes.c_float),
                ("xindex_key", ctypes.c_uint64)]


_G = ctypes.POINTER(fftpl_grid)
_P = ctypes.POINTER(fftpl_problem)

# name -> (restype, argtypes); mirrors include/fftpl.h
SIGNATURES = {
    "fftpl_version": (c_int, []),
    "fftpl_status_string": (c_char_p, [c_int]),
    "fftpl_plan_create": (c_int, [ctypes.POINTER(c_void_p), c_int, c_int, c_int, c_void_p]),
    "fftpl_plan_destroy": (c_int, [c_void_p]),
    "fftpl_plan_info": (c_int, [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                ctypes.POINTER(c_int)]),
    "fftpl_plan_maps": (c_int, [c_void_p, ctypes.POINTER(c_void_p),
                                ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p)]),
    "fftpl_fixed_map": (c_int, [_G, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_void_p, c_void_p]),
    "fftpl_dark_nodes": (c_int, [c_double, c_double, c_double, c_double, c_int, c_void_p,
                                 c_int, c_void_p, ctypes.POINTER(c_int)]),
    "fftpl_density_map": (c_int, [_G, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p]),
    "fftpl_density_map_noalloc": (c_int, [_G, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p, c_void_p]),
    "fftpl_poisson_solve": (c_int, [c_void_p, _G, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_void_p]),
    "fftpl_helmholtz_solve": (c_int, [c_void_p, _G, c_float, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p]),
    "fftpl_field_gather": (c_int, [_G, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_int, c_float, c_int,
                                   c_void_p, c_void_p, c_void_p]),
    "fftpl_wa_grad": (c_int, [c_int, c_void_p, c_int, c_void_p, c_void_p, c_void_p,
                              c_int, c_void_p, c_void_p, c_float, c_int, c_void_p,
                              c_void_p, c_void_p, c_void_p, c_void_p]),
    "fftpl_lse_grad": (c_int, [c_int, c_void_p, c_int, c_void_p, c_void_p, c_void_p,
                               c_int, c_void_p, c_void_p, c_float, c_int, c_void_p,
                               c_void_p, c_void_p, c_void_p, c_void_p]),
    "fftpl_eval": (c_int, [c_void_p, _P, c_void_p, c_void_p, c_float, c_float, c_int,
                           c_void_p, c_void_p, c_void_p, c_void_p]),
    "fftpl_eval_params": (c_int, [c_void_p, _P, c_void_p, c_void_p, c_void_p, c_int,
                                  c_void_p, c_void_p, c_void_p, c_void_p]),
    "fftpl_eval_batch": (c_int, [c_void_p, c_int, ctypes.POINTER(_P),
                                 ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                 ctypes.POINTER(c_float), ctypes.POINTER(c_float), c_int,
                                 ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                 c_void_p, c_void_p]),
    "fftpl_debug_cell_bins": (c_int, [_G, c_int, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p]),
    "fftpl_problem_work_bytes": (c_int, [c_int, c_int, c_int, c_int,
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "fftpl_netlist_index": (c_int, [c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p]),
    "fftpl_xindex_bytes": (c_int, [c_int, c_int, c_int, c_int,
                                   ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(ctypes.c_uint64)]),
    "fftpl_xindex_build": (c_int, [c_int, c_int, c_int, c_void_p, c_void_p, c_int, c_void_p,
                                   ctypes.c_uint64, c_void_p, ctypes.c_uint64,
                                   ctypes.POINTER(ctypes.c_uint64), c_void_p]),
    "fftpl_problem_path": (c_int, [_P, ctypes.POINTER(c_int)]),
    "fftpl_problem_density": (c_int, [_P, c_void_p, c_void_p, c_void_p, c_void_p]),
    "fftpl_problem_wl_grad": (c_int, [_P, c_void_p, c_void_p, c_float, c_int, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p]),
    "fftpl_debug_net_values": (c_int, [_P, c_void_p, c_void_p, c_float, c_void_p, c_void_p,
                                       c_void_p]),
    "fftpl_step_stats": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 ctypes.c_uint64, c_void_p]),
    "fftpl_nesterov_update": (c_int, [_G, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_float, c_float,
                                      c_void_p]),
    "fftpl_nesterov_update_dev": (c_int, [_G, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "fftpl_nesterov_schedule": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_int, c_void_p]),
    "fftpl_cg_dots": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_void_p, c_void_p, c_void_p, ctypes.c_uint64, c_void_p]),
    "fftpl_cg_direction": (c_int, [c_int, c_void_p, c_void_p, c_float, c_void_p, c_void_p,
                                   c_void_p, c_void_p, ctypes.c_uint64, c_void_p]),
    "fftpl_cg_move": (c_int, [_G, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_void_p, c_float, c_void_p, c_void_p, c_void_p]),
    "fftpl_plan_timing": (c_int, [c_void_p, c_int]),
    "fftpl_plan_kernel_times": (c_int, [c_void_p, c_int, ctypes.POINTER(c_float),
                                        ctypes.POINTER(c_char_p), ctypes.POINTER(c_int)]),
}

_lib = None


def load():
    """Load libfftpl.so (once) and declare every entry point's signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -m paper_1312_4587_amd.build` "
            "(hipcc, gfx950).  There is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
