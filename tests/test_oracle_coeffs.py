"""Pins for the oracle's finite-difference coefficients and time-step rule.

Polynomial exactness fixes each coefficient family independently of the
closed forms used to produce it; the paper's printed step counts and grid
sizes fix the stability constant, the step-count rule and the placement of
the absorbing layer (section "Performance evaluation").
"""
import os
from fractions import Fraction

import pytest

from oracle import coeffs
from oracle.core import Problem

ORDERS = [2, 4, 6, 8, 10, 12, 14, 16]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_grid_and_steps.txt")


def _pow(x, k):
    return Fraction(1) if k == 0 else Fraction(x) ** k


@pytest.mark.parametrize("so", ORDERS)
def test_second_derivative_exact_to_order(so):
    v = coeffs.second_derivative(so)
    r = so // 2
    for k in range(0, so + 2):
        got = v[0] * _pow(0, k) + sum(v[j] * (_pow(j, k) + _pow(-j, k)) for j in range(1, r + 1))
        assert got == (2 if k == 2 else 0), (so, k)
    k = so + 2          # one degree beyond: must not be exact (maximal order)
    assert sum(v[j] * (_pow(j, k) + _pow(-j, k)) for j in range(1, r + 1)) != 0


@pytest.mark.parametrize("so", ORDERS)
def test_first_derivative_exact_to_order(so):
    w = coeffs.first_derivative_w(so)
    r = so // 2
    for k in range(0, so + 1):
        got = sum(w[j] * (_pow(j, k) - _pow(-j, k)) for j in range(1, r + 1)) / 2
        assert got == (1 if k == 1 else 0), (so, k)
    k = so + 1
    assert sum(w[j] * (_pow(j, k) - _pow(-j, k)) for j in range(1, r + 1)) != 0


@pytest.mark.parametrize("so", ORDERS)
def test_staggered_derivative_exact_to_order(so):
    s = coeffs.staggered(so)
    r = so // 2
    for k in range(0, so + 1):
        got = sum(s[j] * (_pow(Fraction(2 * j - 1, 2), k) - _pow(Fraction(1 - 2 * j, 2), k))
                  for j in range(1, r + 1))
        assert got == (1 if k == 1 else 0), (so, k)


@pytest.mark.parametrize("so", ORDERS)
def test_midpoint_interpolation_exact_to_order(so):
    m = coeffs.midpoint(so)
    r = so // 2
    for k in range(0, so):
        got = sum(m[j] * (_pow(Fraction(2 * j - 1, 2), k) + _pow(Fraction(1 - 2 * j, 2), k))
                  for j in range(1, r + 1))
        assert got == (1 if k == 0 else 0), (so, k)


def test_textbook_low_orders():
    assert coeffs.second_derivative(2) == [-2, 1]
    assert coeffs.second_derivative(4) == [Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12)]
    assert coeffs.first_derivative_w(2)[1] == 1           # (f_{k+1} - f_{k-1}) / (2 dx)
    assert coeffs.staggered(4)[1:] == [Fraction(9, 8), Fraction(-1, 24)]
    assert coeffs.midpoint(2)[1:] == [Fraction(1, 2)]


def test_paper_step_counts():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 6
    for ndim, h, tf, cmax, so, steps in rows:
        ndim, so, steps = int(ndim), int(so), int(steps)
        dt = coeffs.critical_dt([float(h)] * ndim, so, float(cmax))
        assert coeffs.steps_for(float(tf), dt) == steps


def test_critical_dt_unequal_spacing_reduces_to_uniform():
    a = coeffs.critical_dt((10.0, 10.0, 10.0), 8, 3000.0)
    b = 2 * 10.0 / (3000.0 * (3 * float(coeffs.a1d(8))) ** 0.5)
    assert abs(a - b) < 1e-15 * b
    assert coeffs.critical_dt((10.0, 20.0), 4, 3000.0) > coeffs.critical_dt((10.0, 10.0), 4, 3000.0)


def test_paper_grid_sizes_layer_is_added_outside():
    p2 = Problem(n=(351, 1701), h=(10, 10), space_order=4, dt=1e-3, nsteps=1,
                 nbl=((0, 70), (70, 70)))
    assert p2.N == (421, 1841) and p2.N[0] * p2.N[1] == 775061
    p3 = Problem(n=(207, 801, 801), h=(20, 20, 20), space_order=4, dt=1e-3, nsteps=1)
    assert p3.N[0] * p3.N[1] * p3.N[2] == 132811407


def test_bad_order_rejected():
    with pytest.raises(ValueError):
        coeffs.second_derivative(3)
