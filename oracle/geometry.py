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

Points near a side with a mirror ghost condition ("Boundary conditions and
domain truncation": null Dirichlet / null Neumann by ghost nodes) follow the
image method that defines those conditions: the grid is the half of a problem
doubled about the boundary node, with the model mirrored evenly.
* A source has an image across each mirrored side (reflected about the
  boundary node, amplitude times -1 for Dirichlet, +1 for Neumann; across two
  mirrored axes the image of the image).  The entries of the source and of its
  images that fall inside the grid are the ones that act on it; entries beyond
  a mirrored side belong to the other half.
* A receiver reads ghost nodes as the ghost condition defines them: an entry
  beyond a mirrored side reads its mirror node, times -1 for Dirichlet.
An entry beyond a side without a mirror condition is an error.
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


def _images(coord, h, nbl_lo, N, mirror):
    """(coordinate, sign) of a source and its images across mirrored sides.
    mirror[i] = (sign at the low side, sign at the high side), None where the
    side has no mirror condition."""
    out = [(list(coord), 1.0)]
    for i, (lo_s, hi_s) in enumerate(mirror):
        # boundary nodes of the extended grid, in metres from the physical origin
        sides = [(lo_s, -nbl_lo[i] * h[i]), (hi_s, (N[i] - 1 - nbl_lo[i]) * h[i])]
        new = []
        for c, sg in out:
            for sign, m in sides:
                if sign is not None:
                    d = list(c)
                    d[i] = 2.0 * m - c[i]
                    new.append((d, sg * sign))
        out += new
    return out


def weight_table(coords, h, nbl_lo, N, interp="hicks", radius=4, kaiser_b=None, mirror=None,
                 role="receiver"):
    """Flattened (node, point id, weight) arrays for a set of points on a grid
    of extents N (extended grid).  mirror: per axis (low sign, high sign) of the
    mirror ghost conditions (-1 Dirichlet, +1 Neumann, None without), or None;
    role: "source" or "receiver" (how entries beyond a mirrored side are
    treated).  Raises if a footprint leaves the grid across a side without a
    mirror condition."""
    ndim = len(N)
    mirror = mirror or [(None, None)] * ndim
    nodes, ids, wts = [], [], []

    def flat_of(idx):
        f = 0
        for k, n in zip(idx, N):
            f = f * n + k
        return f

    def beyond(idx):
        """Per axis: None inside the grid, else the mirror sign of the side crossed."""
        out = []
        for i, (k, n) in enumerate(zip(idx, N)):
            if 0 <= k < n:
                out.append(None)
                continue
            sign = mirror[i][0] if k < 0 else mirror[i][1]
            if sign is None:
                raise ValueError("point footprint leaves the grid")
            out.append(sign)
        return out

    for pid, coord in enumerate(coords):
        if role == "source":
            for j, (c, sg) in enumerate(_images(coord, h, nbl_lo, N, mirror)):
                for idx, w in point_weights(c, h, nbl_lo, interp, radius, kaiser_b):
                    if j == 0:
                        beyond(idx)          # the source itself may cross mirrored sides only
                    if all(0 <= k < n for k, n in zip(idx, N)):
                        nodes.append(flat_of(idx))
                        ids.append(pid)
                        wts.append(sg * w)
        elif role == "receiver":
            for idx, w in point_weights(coord, h, nbl_lo, interp, radius, kaiser_b):
                signs = beyond(idx)
                q = []
                for k, n, sign in zip(idx, N, signs):
                    if sign is not None:
                        k = -k if k < 0 else 2 * (n - 1) - k
                        if not 0 <= k < n:
                            raise ValueError("point footprint reaches past the mirror of the grid")
                        w = sign * w
                    q.append(k)
                nodes.append(flat_of(q))
                ids.append(pid)
                wts.append(w)
        else:
            raise ValueError(role)
    return (np.asarray(nodes, dtype=np.int64), np.asarray(ids, dtype=np.int64),
            np.asarray(wts, dtype=np.float64))
