"""MI355X-native explicit finite-difference acoustic propagator.

The numerical work (model preparation, stencil time stepping with the fused
absorbing layer, source injection, receiver recording, adjoint and imaging
condition) runs in libsimwave_hip.so, hand-written HIP for gfx950, behind the
C ABI declared in include/simwave_hip.h.  This package is the thin Python
binding over it.
"""
from .propagator import (Propagator, ForwardResult, AcousticForward, AcousticForwardVD, Batch,  # noqa: F401
                         critical_dt, steps_for, ricker, forward, remove_nbl)
from ._lib import SimwaveError, lib  # noqa: F401
