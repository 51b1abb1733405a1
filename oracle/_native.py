"""Build and load the oracle's C stepping core (oracle/wave.c) with gcc.

Test infrastructure (oracle): only tests, the smoke check and the benchmark's
CPU-baseline leg use this module.
"""
import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wave.c")
LIB = os.path.join(HERE, "_wave.so")

RMAX = 16


def build(force=False):
    """Compile wave.c into _wave.so (plain IEEE FP64: no fast-math)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class Grid(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("r", ctypes.c_int32),
        ("N", ctypes.c_int64 * 3),
        ("h", ctypes.c_double * 3),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("v", ctypes.c_double * (RMAX + 1)),
        ("w", ctypes.c_double * (RMAX + 1)),
        ("s", ctypes.c_double * (RMAX + 1)),
        ("m", ctypes.c_double * (RMAX + 1)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        gp = ctypes.POINTER(Grid)
        L.ow_step.argtypes = [gp, ctypes.c_int32, dp, dp, dp, dp, dp, dp, dp]
        L.ow_step.restype = None
        L.ow_apply_L.argtypes = [gp, ctypes.c_int32, dp, dp, dp]
        L.ow_apply_L.restype = None
        ip = ctypes.POINTER(ctypes.c_int64)
        L.ow_step_points.argtypes = [gp, ctypes.c_int32, dp, dp, dp, dp, dp, dp, ip, ctypes.c_int64, dp]
        L.ow_step_points.restype = None
        L.ow_threads.argtypes = []
        L.ow_threads.restype = ctypes.c_int32
        _lib = L
    return _lib
