"""Finite-difference coefficients and the time-step limit, in exact arithmetic.

Test infrastructure (oracle): only tests, the smoke check and the benchmark's
CPU-baseline leg use this module.

* Centred second derivative of even order SO = 2r (paper, "Space
  discretization", second-derivative formula): v_0 .. v_r.  Closed form of the
  maximal-order central stencil,
      v_j = 2 (-1)^(j+1) (r!)^2 / (j^2 (r-j)! (r+j)!),   v_0 = -2 sum_j v_j.
* Centred first derivative (same section, first-derivative formula, which
  carries a 1/(2 dx) prefactor): the paper's w_j = 2 c_j with the standard
      c_j = (-1)^(j+1) (r!)^2 / (j (r-j)! (r+j)!).
* Staggered first derivative at half nodes and the matching midpoint
  interpolation, for the conservative variable-density operator: solved here
  from their Taylor (half-node Vandermonde) conditions with rational Gaussian
  elimination.
* Time-step limit (paper, "Time discretization", stability condition): the
  constant a is the sum of the magnitudes of the second-derivative
  coefficients entering the update, a1d = |v_0| + 2 sum |v_j| per axis; with
  unequal spacings the bound generalises to
      dt_crit = 2 / (c_max sqrt(sum_i a1d / dx_i^2)).
  The step count for a total time tf is ceil(tf / dt) + 1.
"""
from fractions import Fraction
from math import factorial, ceil, sqrt


def _check_order(space_order):
    if space_order < 2 or space_order % 2 or space_order > 32:
        raise ValueError(f"space order must be even in [2, 32], got {space_order}")
    return space_order // 2


def second_derivative(space_order):
    """[v_0, v_1, ..., v_r] as Fractions."""
    r = _check_order(space_order)
    fr = factorial(r) ** 2
    v = [Fraction(0)] * (r + 1)
    for j in range(1, r + 1):
        v[j] = Fraction(2 * (-1) ** (j + 1) * fr, j * j * factorial(r - j) * factorial(r + j))
    v[0] = -2 * sum(v[1:])
    return v


def first_derivative_c(space_order):
    """[0, c_1, ..., c_r]: f'(x) ~ (1/dx) sum_j c_j (f(x+j dx) - f(x-j dx))."""
    r = _check_order(space_order)
    fr = factorial(r) ** 2
    c = [Fraction(0)] * (r + 1)
    for j in range(1, r + 1):
        c[j] = Fraction((-1) ** (j + 1) * fr, j * factorial(r - j) * factorial(r + j))
    return c


def first_derivative_w(space_order):
    """Paper's weights w_j (with its 1/(2 dx) prefactor): w_j = 2 c_j."""
    return [2 * x for x in first_derivative_c(space_order)]


def _solve(A, b):
    """Exact Gaussian elimination over Fractions."""
    n = len(b)
    M = [list(row) + [rhs] for row, rhs in zip(A, b)]
    for col in range(n):
        piv = next(i for i in range(col, n) if M[i][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for i in range(n):
            if i != col and M[i][col] != 0:
                f = M[i][col] / M[col][col]
                M[i] = [a - f * c for a, c in zip(M[i], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


def staggered(space_order):
    """[0, s_1, ..., s_r]: (D+ q)_{k+1/2} = (1/dx) sum_j s_j (q_{k+j} - q_{k-j+1}).

    Taylor expansion about x_{k+1/2}: q_{k+j} - q_{k-j+1} only has odd powers
    of the offset (j - 1/2) dx, so the conditions are
        sum_j s_j * 2 (j - 1/2)            = 1
        sum_j s_j * (j - 1/2)^(2q+1)       = 0,   q = 1 .. r-1.
    """
    r = _check_order(space_order)
    A, b = [], []
    for q in range(r):
        p = 2 * q + 1
        A.append([2 * Fraction(2 * j - 1, 2) ** p for j in range(1, r + 1)])
        b.append(Fraction(1 if q == 0 else 0))
    return [Fraction(0)] + _solve(A, b)


def midpoint(space_order):
    """[0, m_1, ..., m_r]: b_{k+1/2} = sum_j m_j (b_{k+j} + b_{k-j+1}).

    Only even powers of (j - 1/2) dx survive, so
        sum_j 2 m_j                = 1
        sum_j m_j (j - 1/2)^(2q)   = 0,   q = 1 .. r-1.
    """
    r = _check_order(space_order)
    A, b = [], []
    for q in range(r):
        A.append([(2 if q == 0 else 1) * Fraction(2 * j - 1, 2) ** (2 * q) for j in range(1, r + 1)])
        b.append(Fraction(1 if q == 0 else 0))
    return [Fraction(0)] + _solve(A, b)


def a1d(space_order):
    """Sum of the magnitudes of the second-derivative stencil along one axis."""
    v = second_derivative(space_order)
    return abs(v[0]) + 2 * sum(abs(x) for x in v[1:])


def critical_dt(h, space_order, cmax):
    """Largest stable leapfrog step for grid spacings h (one per axis)."""
    a = float(a1d(space_order))
    return 2.0 / (cmax * sqrt(sum(a / (hi * hi) for hi in h)))


def steps_for(tf, dt):
    """Number of time levels for a total time tf: ceil(tf / dt) + 1."""
    return int(ceil(tf / dt)) + 1
