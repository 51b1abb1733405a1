"""ctypes declarations of the C ABI in include/simwave_hip.h.

torch is imported before the library is loaded so that the library binds to
the HIP runtime already loaded by torch (same soname) and device pointers and
streams are shared.  There is no fallback: if the library is missing, loading
raises.
"""
import ctypes
import os

import torch  # noqa: F401  (must precede loading the HIP library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsimwave_hip.so")

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
c_float_p = ctypes.POINTER(ctypes.c_float)

SW_CONST, SW_VD_STAGGERED, SW_VD_CENTRED = 0, 1, 2
SW_SRC, SW_REC = 0, 1
SW_INTERP_HICKS, SW_INTERP_LINEAR = 0, 1
SCHEMES = {"const": SW_CONST, "vd_staggered": SW_VD_STAGGERED, "vd_centred": SW_VD_CENTRED}
INTERPS = {"hicks": SW_INTERP_HICKS, "linear": SW_INTERP_LINEAR}
BCS = {"none": 0, "dirichlet": 1, "neumann": 2}

STATUS = {0: "SW_OK", 1: "SW_ERR_ARG", 2: "SW_ERR_UNSUPPORTED", 3: "SW_ERR_DOMAIN",
          4: "SW_ERR_CFL", 5: "SW_ERR_STATE", 6: "SW_ERR_WORKSPACE", 7: "SW_ERR_HIP",
          8: "SW_ERR_NONFINITE"}


class SimwaveError(RuntimeError):
    def __init__(self, call, status, message):
        super().__init__(f"{call}: {STATUS.get(status, status)}: {message}")
        self.status = status
        self.call = call


class Problem(ctypes.Structure):
    _fields_ = [("ndim", c_int32), ("n", c_int32 * 3), ("h", c_double * 3),
                ("space_order", c_int32), ("scheme", c_int32),
                ("nbl", (c_int32 * 2) * 3), ("bc", (c_int32 * 2) * 3),
                ("damp_alpha", c_double), ("damp_power", c_double), ("dt", c_double),
                ("nsteps", c_int32), ("dtype", c_int32)]


class Layout(ctypes.Structure):
    _fields_ = [("ndim", c_int32), ("dims", c_int32 * 3), ("halo", c_int32),
                ("padded", c_int32 * 3), ("origin", c_int64), ("field_elems", c_int64),
                ("grid_nodes", c_int64), ("physical_nodes", c_int64), ("nsrc", c_int32),
                ("nrec", c_int32), ("workspace_bytes", c_int64)]


class FwdIO(ctypes.Structure):
    _fields_ = [("workspace", c_void_p), ("wavelet", c_void_p), ("field", c_void_p * 2),
                ("traces", c_void_p), ("snaps", c_void_p), ("saving_stride", c_int32),
                ("ckpt", c_void_p), ("ckpt_every", c_int32), ("step0", c_int32),
                ("nsteps_run", c_int32), ("use_graph", c_int32), ("stencil_ms", c_float_p),
                ("field2", c_void_p * 2), ("check_finite", c_int32)]


class Fwd64IO(ctypes.Structure):
    _fields_ = [("workspace", c_void_p), ("wavelet", c_void_p), ("field", c_void_p * 2),
                ("traces", c_void_p), ("snaps", c_void_p), ("saving_stride", c_int32),
                ("step0", c_int32), ("nsteps_run", c_int32)]


class AdjIO(ctypes.Structure):
    _fields_ = [("workspace", c_void_p), ("vel", c_void_p), ("wavelet", c_void_p),
                ("residual", c_void_p), ("ckpt", c_void_p), ("ckpt_every", c_int32),
                ("field", c_void_p * 2), ("adj", c_void_p * 2), ("segment", c_void_p),
                ("grad_m", c_void_p), ("grad_vel", c_void_p), ("src_adjoint", c_void_p),
                ("grad_rho", c_void_p), ("vd_work", c_void_p)]


class Tiling(ctypes.Structure):
    _fields_ = [("tx", c_int32), ("nw", c_int32), ("zc", c_int32), ("nt", c_int32), ("pf", c_int32),
                ("wt", c_int32), ("ts", c_int32), ("occ", c_int32), ("order", c_int32)]


class BatchIO(ctypes.Structure):
    _fields_ = [("shots", ctypes.POINTER(FwdIO)), ("table", c_void_p), ("nsteps_run", c_int32),
                ("use_graph", c_int32)]


# every symbol the header declares, with its signature
SIGNATURES = {
    "sw_abi_version": (c_int32, []),
    "sw_status_str": (ctypes.c_char_p, [c_int32]),
    "sw_last_error": (ctypes.c_char_p, []),
    "sw_critical_dt": (c_int32, [c_int32, ctypes.POINTER(c_double), c_int32, c_double,
                                 ctypes.POINTER(c_double)]),
    "sw_steps_for": (c_int32, [c_double, c_double, ctypes.POINTER(c_int32)]),
    "sw_ricker": (c_int32, [c_double, c_double, c_double, c_int32, c_float_p]),
    "sw_plan_create": (c_int32, [ctypes.POINTER(Problem), ctypes.POINTER(c_void_p)]),
    "sw_plan_destroy": (c_int32, [c_void_p]),
    "sw_plan_layout": (c_int32, [c_void_p, ctypes.POINTER(Layout)]),
    "sw_plan_set_geometry": (c_int32, [c_void_p, c_int32, c_int32, ctypes.POINTER(c_double),
                                       c_int32, c_int32, c_double]),
    "sw_plan_points": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_int64),
                                 ctypes.POINTER(c_int64), ctypes.POINTER(c_int32), c_float_p]),
    "sw_model_prepare": (c_int32, [c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p]),
    "sw_forward": (c_int32, [c_void_p, ctypes.POINTER(FwdIO), c_void_p]),
    "sw_model_prepare_f64": (c_int32, [c_void_p, c_void_p, c_double, c_void_p, c_void_p]),
    "sw_forward_f64": (c_int32, [c_void_p, ctypes.POINTER(Fwd64IO), c_void_p]),
    "sw_adjoint": (c_int32, [c_void_p, ctypes.POINTER(AdjIO), c_void_p]),
    "sw_plan_set_tiling": (c_int32, [c_void_p, ctypes.POINTER(Tiling)]),
    "sw_plan_get_tiling": (c_int32, [c_void_p, ctypes.POINTER(Tiling)]),
    "sw_plan_occupancy": (c_int32, [c_void_p, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32)]),
    "sw_batch_create": (c_int32, [c_int32, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p)]),
    "sw_batch_destroy": (c_int32, [c_void_p]),
    "sw_batch_layout": (c_int32, [c_void_p, ctypes.POINTER(c_int64)]),
    "sw_batch_set_tiling": (c_int32, [c_void_p, ctypes.POINTER(Tiling), c_int32]),
    "sw_batch_get_tiling": (c_int32, [c_void_p, ctypes.POINTER(Tiling), ctypes.POINTER(c_int32)]),
    "sw_batch_forward": (c_int32, [c_void_p, ctypes.POINTER(BatchIO), c_void_p]),
    "sw_batch_forward_static": (c_int32, [c_void_p, ctypes.POINTER(BatchIO), c_void_p]),
    "sw_plan_autotune": (c_int32, [c_void_p, ctypes.POINTER(FwdIO), ctypes.c_char_p, c_void_p]),
    "sw_batch_autotune": (c_int32, [c_void_p, ctypes.POINTER(BatchIO), ctypes.c_char_p, c_void_p]),
}

_lib = None


def lib():
    """Load libsimwave_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(call, status):
    if status != 0:
        msg = lib().sw_last_error()
        raise SimwaveError(call, status, msg.decode() if msg else "")
