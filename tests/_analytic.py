"""Closed-form solutions used to pin the oracle (independent of it).

* Homogeneous-medium Green's functions of (1/c^2) p_tt - lap p = S(t) delta(x):
    3D: p(R, t) = S(t - R/c) / (4 pi R)
    2D: p(R, t) = (1/(2 pi)) int_0^{acosh(ct/R)} S(t - (R/c) cosh th) d th
  (the 2D form is the convolution of S with c / (2 pi sqrt(c^2 t^2 - R^2))).
* Manufactured solutions: sympy differentiates a chosen u*(x, t) and rho(x)
  to give the forcing f = u*_tt / c^2 - lap u* + (grad rho / rho) . grad u*
  of the expanded variable-density equation, and the exact operators
  lap u - (grad rho/rho).grad u and div(grad u / rho).
"""
import math

import numpy as np
import sympy as sp
from scipy.integrate import quad


def ricker(f, t, t0):
    a = (math.pi * f * (t - t0)) ** 2
    return (1.0 - 2.0 * a) * math.exp(-a)


def greens_3d(R, c, f, times, t0):
    return np.array([ricker(f, t - R / c, t0) for t in times]) / (4.0 * math.pi * R)


def greens_2d(R, c, f, times, t0):
    out = []
    for t in times:
        if c * t <= R:
            out.append(0.0)
            continue
        top = math.acosh(c * t / R)
        val, _ = quad(lambda th: ricker(f, t - (R / c) * math.cosh(th), t0), 0.0, top, limit=400)
        out.append(val / (2.0 * math.pi))
    return np.array(out)


X = sp.symbols("x0 x1 x2", real=True)
T = sp.Symbol("t", real=True)


def lambdify_space(expr, ndim):
    f = sp.lambdify(X[:ndim], expr, "numpy")

    def call(*coords):
        val = f(*coords)
        return np.broadcast_to(np.asarray(val, dtype=np.float64), np.broadcast(*coords).shape).copy()
    return call


def grid_coords(shape, h, origin=None):
    origin = origin or [0] * len(shape)
    return np.meshgrid(*[(np.arange(n) - o) * hi for n, hi, o in zip(shape, h, origin)],
                       indexing="ij")


def exact_operators(u, rho, ndim):
    """(lap u, lap u - grad rho/rho . grad u, div(grad u / rho)) as sympy."""
    lap = sum(sp.diff(u, X[i], 2) for i in range(ndim))
    centred = lap - sum(sp.diff(rho, X[i]) / rho * sp.diff(u, X[i]) for i in range(ndim))
    conservative = sum(sp.diff(sp.diff(u, X[i]) / rho, X[i]) for i in range(ndim))
    return lap, centred, conservative


def mms_forcing(u, rho, c, ndim):
    """f = u_tt/c^2 - lap u + (grad rho/rho).grad u (sympy, in x and t)."""
    _, centred, _ = exact_operators(u, rho, ndim)
    return sp.diff(u, T, 2) / c ** 2 - centred
