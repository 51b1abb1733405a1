"""Source-injection and receiver-interpolation weights, FP64.

Test infrastructure (oracle): only tests, the smoke check and the benchmark's
CPU-baseline leg use this module.

Band-limited point (paper, "Sources and receivers", source term and Kaiser
window): the node at signed distance x = n + alpha (in cells) from the point
gets the weight W(x) sinc(x), with W the Kaiser window of half-width r and
shape b, W(x) = I0(b sqrt(1 - (x/r)^2)) / I0(b) for |x| <= r and 0 outside,
and sinc the normalised sinc.  alpha lies in (-0.5, 0.5]: with xi the point's
coordinate in cells, the centre node is k0 = floor(xi + 0.5) and alpha =
k0 - xi.  Multi-dimensional weights are the product of the per-axis weights.
The same weights interpolate the wavefield at a receiver: R = sum_n p_n d_n.

Linear (trilinear in 3D) interpolation, used where a configuration asks for
it: nodes floor(xi) and floor(xi)+1 with weights 1 - t and t, t = xi - floor(xi).

Zero weights are dropped.  Coordinates are in metres from the first node of the
physical grid; the returned node indices are on the extended grid (physical
grid plus absorbing layer).
"""
import math
import itertools
import numpy as np


def bessel_i0(x):
    """Modified Bessel function of the first kind, order 0, by its power series
    sum_k ((x/2)^k / k!)^2, summed until the terms stop contributing."""
    x = float(x)
    term = 1.0
    total = 1.0
    k = 0
    q = (x / 2.0) ** 2
    while True:
        k += 1
        term *= q / (k * k)
        total += term
        if term < 1e-18 * total:
            return total


def kaiser(x, r, b):
    """Kaiser window W(x) of half-width r and shape b."""
    if abs(x) > r:
        return 0.0
    return bessel_i0(b * math.sqrt(max(0.0, 1.0 - (x / r) ** 2))) / bessel_i0(b)


def sinc(x):
    """Normalised sinc, exactly 0 at non-zero integers."""
    if x == 0.0:
        return 1.0
    if float(x).is_integer():
        return 0.0
    return math.sin(math.pi * x) / (math.pi * x)


def hicks_1d(xi, r, b):
    """[(node, weight)] along one axis for a point at xi (cells)."""
    k0 = math.floor(xi + 0.5)
    alpha = k0 - xi
    out = []
    for n in range(-r, r + 1):
        x = n + alpha
        wgt = kaiser(x, r, b) * sinc(x)
        if wgt != 0.0:
            out.append((k0 + n, wgt))
    return out


def linear_1d(xi):
    k = math.floor(xi)
    t = xi - k
    out = [(k, 1.0 - t)]
    if t != 0.0:
        out.append((k + 1, t))
    return out


DEFAULT_KAISER_B = {4: 6.31}


def point_weights(coord, h, nbl_lo, interp="hicks", radius=4, kaiser_b=None):
    """Weights of one point.

    coord  : metres per axis from the physical grid's first node
    h      : spacing per axis
    nbl_lo : absorbing-layer width (cells) on the low side of each axis
    Returns a list of (index tuple on the extended grid, weight).
    """
    per_axis = []
    for c, hi, lo in zip(coord, h, nbl_lo):
        xi = c / hi
        if interp == "hicks":
            b = kaiser_b if kaiser_b is not None else DEFAULT_KAISER_B.get(radius)
            if b is None:
                raise ValueError("Kaiser b must be given for this radius")
            axis = hicks_1d(xi, radius, b)
        elif interp == "linear":
            axis = linear_1d(xi)
        else:
            raise ValueError(interp)
        per_axis.append([(k + lo, w) for k, w in axis])
    out = []
    for combo in itertools.product(*per_axis):
        idx = tuple(k for k, _ in combo)
        w = 1.0
        for _, wk in combo:
            w *= wk
        out.append((idx, w))
    return out


def weight_table(coords, h, nbl_lo, N, interp="hicks", radius=4, kaiser_b=None):
    """Flattened (node, point id, weight) arrays for a set of points on a grid
    of extents N (extended grid); raises if a footprint leaves the grid."""
    nodes, ids, wts = [], [], []
    for pid, coord in enumerate(coords):
        for idx, w in point_weights(coord, h, nbl_lo, interp, radius, kaiser_b):
            for k, n in zip(idx, N):
                if k < 0 or k >= n:
                    raise ValueError(f"point {pid} footprint leaves the grid")
            flat = 0
            for k, n in zip(idx, N):
                flat = flat * n + k
            nodes.append(flat)
            ids.append(pid)
            wts.append(w)
    return (np.asarray(nodes, dtype=np.int64), np.asarray(ids, dtype=np.int64),
            np.asarray(wts, dtype=np.float64))
