"""ctypes binding of libcpr.so: the C ABI of include/cpr.h, one Python
function per entry point with the same name, argument marshalling only.

Loading fails loudly (ImportError) if the library has not been built; there
is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpr.so")

CPR_ABI_VERSION = 2
CPR_OK, CPR_EINVAL, CPR_ENOMEM, CPR_EHIP, CPR_EUNSUPPORTED, CPR_ENONPHYSICAL = 0, -1, -2, -3, -4, -5
CPR_BC_PERIODIC, CPR_BC_TRANSMISSIVE = 0, 1
CPR_FP64, CPR_FP32_BULK = 0, 1
CPR_LIM_NONE, CPR_LIM_TVB_CHAR = 0, 1
CPR_SCHEME_GL_LP, CPR_SCHEME_GLL_CHAIN, CPR_SCHEME_GLL_LP = 0, 1, 2

# exported symbols declared in include/cpr.h
SYMBOLS = (
    "cpr_init", "cpr_destroy", "cpr_set_stream", "cpr_residual", "cpr_rk3_step", "cpr_limit",
    "cpr_residual_vjp", "cpr_adjoint_step", "cpr_rk3_step_stages", "cpr_adjoint_step_stages",
    "cpr_max_wavespeed", "cpr_integrals", "cpr_l2_diff",
    "cpr_point_coords", "cpr_tables", "cpr_scheme_tables", "cpr_set_time", "cpr_get_time", "cpr_troubled_total", "cpr_sync",
    "cpr_status_string", "cpr_last_error", "cpr_rk3_step_static",
)


class CprConfig(ctypes.Structure):
    _fields_ = [
        ("abi_version", c_int32),
        ("order_p", c_int32),
        ("nx", c_int32),
        ("ny", c_int32),
        ("x0", c_double),
        ("x1", c_double),
        ("y0", c_double),
        ("y1", c_double),
        ("bc", c_int32),
        ("precision", c_int32),
        ("gamma", c_double),
        ("limiter", c_int32),
        ("scheme", c_int32),
        ("tvb_m", c_double),
        ("cfl", c_double),
        ("t_end", c_double),
    ]


class CprError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libcpr.so (once) and declare every entry point's signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_1709_01619_amd.build)")
    try:
        # torch carries its own HIP runtime; it must be loaded first, so
        # that the library binds to the process's one runtime
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = POINTER
    sig = {
        "cpr_init": (c_int32, [P(CprConfig), c_void_p, P(c_void_p)]),
        "cpr_destroy": (c_int32, [c_void_p]),
        "cpr_set_stream": (c_int32, [c_void_p, c_void_p]),
        "cpr_residual": (c_int32, [c_void_p, c_void_p, c_void_p]),
        "cpr_rk3_step": (c_int32, [c_void_p, c_void_p, c_double, c_int32]),
        "cpr_limit": (c_int32, [c_void_p, c_void_p, c_void_p, P(c_int32)]),
        "cpr_residual_vjp": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
        "cpr_adjoint_step": (c_int32, [c_void_p, c_void_p, c_double, c_void_p, c_void_p]),
        "cpr_rk3_step_stages": (c_int32, [c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
        "cpr_adjoint_step_stages": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                              c_void_p, c_void_p]),
        "cpr_max_wavespeed": (c_int32, [c_void_p, c_void_p, P(c_double)]),
        "cpr_integrals": (c_int32, [c_void_p, c_void_p, P(c_double)]),
        "cpr_l2_diff": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, P(c_double)]),
        "cpr_point_coords": (c_int32, [c_void_p, c_void_p, c_void_p]),
        "cpr_tables": (c_int32, [c_int32, P(c_double), P(c_double), P(c_double), P(c_double)]),
        "cpr_scheme_tables": (c_int32, [c_int32, c_int32, P(c_double), P(c_double), P(c_double),
                                        P(c_double)]),
        "cpr_set_time": (c_int32, [c_void_p, c_double]),
        "cpr_get_time": (c_int32, [c_void_p, P(c_double), P(c_double)]),
        "cpr_troubled_total": (c_int32, [c_void_p, P(c_int64), c_int32]),
        "cpr_sync": (c_int32, [c_void_p]),
        "cpr_status_string": (ctypes.c_char_p, [c_int32]),
        "cpr_last_error": (ctypes.c_char_p, [c_void_p]),
        "cpr_rk3_step_static": (c_int32, [P(CprConfig), c_void_p, c_void_p, c_double,
                                          c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, ctx=None, what=""):
    if status == CPR_OK:
        return
    lib = load()
    msg = lib.cpr_status_string(status).decode()
    if ctx:
        detail = lib.cpr_last_error(ctx).decode()
        if detail:
            msg = f"{msg}: {detail}"
    raise CprError(status, f"{what}: {msg}" if what else msg)


def make_config(P, nx, ny, x0=0.0, x1=10.0, y0=0.0, y1=10.0, bc=CPR_BC_PERIODIC,
                precision=CPR_FP64, gamma=1.4, limiter=CPR_LIM_NONE, tvb_m=10.0, cfl=0.0,
                t_end=0.0, scheme=CPR_SCHEME_GL_LP):
    return CprConfig(CPR_ABI_VERSION, P, nx, ny, x0, x1, y0, y1, bc, precision, gamma,
                     limiter, scheme, tvb_m, cfl, t_end)


def tables(P, scheme=None):
    """(xi, w, gL', gR') from the library's own table builder: cpr_tables,
    or cpr_scheme_tables when a scheme is given."""
    lib = load()
    arrs = [(c_double * (P + 1))() for _ in range(4)]
    if scheme is None:
        check(lib.cpr_tables(P, *arrs), what="cpr_tables")
    else:
        check(lib.cpr_scheme_tables(scheme, P, *arrs), what="cpr_scheme_tables")
    return tuple([a[i] for i in range(P + 1)] for a in arrs)
