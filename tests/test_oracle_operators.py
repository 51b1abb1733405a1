"""Pins for the oracle's spatial operators.

Each discrete operator, applied to smooth fields, must match the continuous
operator (sympy) at interior nodes with an error falling as h^SO, and must be
exact on low-degree polynomials.  A dropped term, a wrong sign or an
off-by-one in the staggered face indexing fails these.
"""
import math

import numpy as np
import pytest
import sympy as sp

import oracle
from tests._analytic import X, exact_operators, lambdify_space, grid_coords

SCHEME_INDEX = {"const": 0, "vd_centred": 1, "vd_staggered": 2}


def _fields(ndim):
    x = X[:ndim]
    u = sp.sin(0.9 * x[0] + 0.2) * sp.cos(1.1 * x[1] + 0.1)
    rho = 2 + sp.sin(0.7 * x[0] + 0.4) * sp.cos(0.5 * x[1] - 0.3)
    if ndim == 3:
        u = u * sp.cos(0.8 * x[2] - 0.5)
        rho = rho + 0.5 * sp.cos(0.6 * x[2] + 0.1)
    return u, rho


def _operator_error(scheme, ndim, so, h, margin_phys, L=None):
    u, rho = _fields(ndim)
    exact = exact_operators(u, rho, ndim)[SCHEME_INDEX[scheme]]
    L = L or 2 * margin_phys + 4.0
    n = int(round(L / h)) + 1
    shape = (n,) * ndim
    prob = oracle.Problem(n=shape, h=(h,) * ndim, space_order=so, dt=1.0, nsteps=1, scheme=scheme)
    coords = grid_coords(shape, prob.h)
    rho_v = lambdify_space(rho, ndim)(*coords)
    st = oracle.prepare(prob, np.ones(shape), None if scheme == "const" else rho_v)
    got = oracle.apply_L(st, np.ascontiguousarray(lambdify_space(u, ndim)(*coords)))
    ref = lambdify_space(exact, ndim)(*coords)
    m = int(math.ceil(margin_phys / h - 1e-9))
    sl = tuple(slice(m, n - m) for _ in range(ndim))
    return np.max(np.abs(got[sl] - ref[sl]))


@pytest.mark.parametrize("scheme", ["const", "vd_centred", "vd_staggered"])
@pytest.mark.parametrize("so", [2, 4, 8])
def test_operator_converges_at_space_order_2d(scheme, so):
    hs = [0.3, 0.15] if so < 8 else [0.4, 0.2]
    margin = (so + 1) * hs[0]
    errs = [_operator_error(scheme, 2, so, h, margin) for h in hs]
    slope = math.log2(errs[0] / errs[1])
    assert so - 0.5 < slope < so + 0.8, (errs, slope)


@pytest.mark.parametrize("scheme", ["const", "vd_centred", "vd_staggered"])
def test_operator_converges_3d(scheme):
    so = 4
    errs = [_operator_error(scheme, 3, so, h, 5 * 0.5, L=8.0) for h in (0.5, 0.25)]
    slope = math.log2(errs[0] / errs[1])
    assert so - 0.5 < slope < so + 0.8, (errs, slope)


def test_high_order_operator_accuracy():
    # SO16: error far below the SO8 error on the same grid.
    e8 = _operator_error("const", 2, 8, 0.3, 6.0)
    e16 = _operator_error("const", 2, 16, 0.3, 6.0)
    assert e16 < 1e-3 * e8


@pytest.mark.parametrize("so", [2, 4, 8])
def test_staggered_exact_on_polynomials(so):
    # b = 1/rho linear and p quadratic: face interpolation, D+ and D- are all
    # exact, so div(b grad p) is reproduced to rounding at interior nodes.
    n = 30
    h = (0.5, 0.25)
    prob = oracle.Problem(n=(n, n), h=h, space_order=so, dt=1.0, nsteps=1, scheme="vd_staggered")
    z, x = grid_coords((n, n), h)
    b = 1.0 + 0.1 * z + 0.05 * x
    p = 0.3 * z ** 2 - 0.2 * x * z + 0.7 * x ** 2 + z
    st = oracle.prepare(prob, np.ones((n, n)), 1.0 / b)
    got = oracle.apply_L(st, np.ascontiguousarray(p))
    # div(b grad p) = b lap p + grad b . grad p
    ref = b * (0.6 + 1.4) + 0.1 * (0.6 * z - 0.2 * x + 1.0) + 0.05 * (-0.2 * z + 1.4 * x)
    m = so + 1
    assert np.max(np.abs(got[m:-m, m:-m] - ref[m:-m, m:-m])) < 1e-10


@pytest.mark.parametrize("so", [2, 4, 8])
def test_centred_vd_exact_on_polynomials(so):
    n = 30
    h = (0.5, 0.25)
    prob = oracle.Problem(n=(n, n), h=h, space_order=so, dt=1.0, nsteps=1, scheme="vd_centred")
    z, x = grid_coords((n, n), h)
    rho = 2.0 + 0.1 * z - 0.05 * x
    p = 0.3 * z ** 2 - 0.2 * x * z + 0.7 * x ** 2 + z
    st = oracle.prepare(prob, np.ones((n, n)), rho)
    got = oracle.apply_L(st, np.ascontiguousarray(p))
    ref = 2.0 - (0.1 * (0.6 * z - 0.2 * x + 1.0) - 0.05 * (-0.2 * z + 1.4 * x)) / rho
    m = so // 2 + 1
    assert np.max(np.abs(got[m:-m, m:-m] - ref[m:-m, m:-m])) < 1e-10


def test_staggered_constant_density_is_a_laplacian():
    # With constant rho the conservative operator is D- D+, a symmetric
    # 2r-wide second-derivative stencil: exact for quadratics.
    n = 24
    prob = oracle.Problem(n=(n, n), h=(1.0, 1.0), space_order=8, dt=1.0, nsteps=1,
                          scheme="vd_staggered")
    z, x = grid_coords((n, n), (1.0, 1.0))
    st = oracle.prepare(prob, np.ones((n, n)), np.full((n, n), 3.0))
    got = oracle.apply_L(st, np.ascontiguousarray(z ** 2 + 2 * x ** 2))
    assert np.max(np.abs(got[9:-9, 9:-9] - 6.0 / 3.0)) < 1e-11


def test_ghost_rules():
    # none: zero ghosts; dirichlet: odd mirror; neumann: even mirror.
    n = 12
    z, x = grid_coords((n, n), (1.0, 1.0))
    f = np.ascontiguousarray(np.cos(0.4 * x) + 0.0 * z)
    out = {}
    for bc in ("none", "neumann"):
        prob = oracle.Problem(n=(n, n), h=(1.0, 1.0), space_order=2, dt=1.0, nsteps=1,
                              bc=(("none", "none"), (bc, bc)))
        out[bc] = oracle.apply_L(oracle.prepare(prob, np.ones((n, n))), f)
    # at x = 0, the even mirror gives 2 (f1 - f0) along x
    expect_x = 2 * (f[5, 1] - f[5, 0])
    assert abs(out["neumann"][5, 0] - expect_x) < 1e-14
    assert abs(out["none"][5, 0] - (f[5, 1] - 2 * f[5, 0])) < 1e-14
    g = np.ascontiguousarray(np.sin(0.4 * x) + 0.0 * z)
    prob = oracle.Problem(n=(n, n), h=(1.0, 1.0), space_order=2, dt=1.0, nsteps=1,
                          bc=(("none", "none"), ("dirichlet", "dirichlet")))
    Lg = oracle.apply_L(oracle.prepare(prob, np.ones((n, n))), g)
    assert abs(Lg[5, 0] - (g[5, 1] - 2 * g[5, 0] - g[5, 1])) < 1e-14
