"""Pins for the oracle's source/receiver weights (paper, "Sources and
receivers": Kaiser-windowed sinc, and the figure of a point half a cell from
its neighbours with b = 6.31, r = 4)."""
import math

import numpy as np
import pytest
import scipy.special

from oracle import geometry as G


@pytest.mark.parametrize("x", [0.0, 0.5, 1.0, 3.7, 6.31, 12.0, 25.0])
def test_i0_matches_scipy(x):
    assert abs(G.bessel_i0(x) - scipy.special.i0(x)) <= 1e-14 * scipy.special.i0(x)


@pytest.mark.parametrize("r,b", [(4, 6.31), (3, 4.0), (6, 8.5)])
def test_kaiser_matches_numpy_window_at_integers(r, b):
    ref = np.kaiser(2 * r + 1, b)
    got = [G.kaiser(n, r, b) for n in range(-r, r + 1)]
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-15)
    assert G.kaiser(r + 0.01, r, b) == 0.0


def test_sinc_matches_numpy():
    xs = np.linspace(-4.3, 4.3, 57) + 0.013
    assert np.allclose([G.sinc(x) for x in xs], np.sinc(xs), rtol=1e-14, atol=1e-16)
    assert G.sinc(0.0) == 1.0 and G.sinc(3.0) == 0.0


@pytest.mark.parametrize("xi", [0.0, 7.0, 11.0])
def test_on_node_point_is_a_delta(xi):
    assert G.hicks_1d(xi, 4, 6.31) == [(int(xi), 1.0)]


def test_half_cell_point_of_the_kaiser_figure():
    # A point half-way between nodes 10 and 11: eight non-zero weights,
    # symmetric about the point, the two nearest the largest.
    ws = G.hicks_1d(10.5, 4, 6.31)
    nodes = [k for k, _ in ws]
    w = np.array([x for _, x in ws])
    assert nodes == list(range(7, 15))
    assert np.allclose(w, w[::-1], rtol=0, atol=1e-15)
    assert w[3] == w.max() and w[4] == w.max()
    assert np.all(np.sign(w[:4]) == [-1, 1, -1, 1])
    assert abs(w.sum() - 1.0) < 1e-3


@pytest.mark.parametrize("kfrac", [0.1, 0.3, 0.5])
def test_band_limited_interpolation(kfrac):
    # Interpolating cos(k x + 0.3) for k up to pi/2 per cell (the design band
    # of the Kaiser parameter) must be accurate: a wrong sign of alpha, an
    # unnormalised sinc or a misplaced centre node would give O(1) errors.
    k = kfrac * math.pi
    for xi in np.linspace(20.0, 21.0, 23):
        ws = G.hicks_1d(xi, 4, 6.31)
        val = sum(w * math.cos(k * n + 0.3) for n, w in ws)
        assert abs(val - math.cos(k * xi + 0.3)) < 1e-3


def test_linear_weights_reproduce_linear_functions():
    for xi in np.linspace(3.0, 4.0, 11):
        ws = G.linear_1d(xi)
        assert abs(sum(w for _, w in ws) - 1.0) < 1e-15
        assert abs(sum(w * n for n, w in ws) - xi) < 1e-13
    assert G.linear_1d(5.0) == [(5, 1.0)]


def test_separable_product_and_layer_offset():
    pts = G.point_weights((20.0, 35.0), (10.0, 10.0), (3, 5), interp="linear")
    d = {idx: w for idx, w in pts}
    assert set(d) == {(5, 8), (5, 9)}
    assert abs(d[(5, 8)] - 0.5) < 1e-15 and abs(d[(5, 9)] - 0.5) < 1e-15


def test_footprint_outside_grid_rejected():
    with pytest.raises(ValueError):
        G.weight_table([(1.0, 50.0)], (10.0, 10.0), (0, 0), (20, 20), "hicks", 4, 6.31)


def test_radius_without_kaiser_parameter_rejected():
    with pytest.raises(ValueError):
        G.point_weights((15.0, 15.0), (10.0, 10.0), (0, 0), "hicks", 3, None)
