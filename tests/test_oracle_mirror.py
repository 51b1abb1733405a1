"""Pins of the oracle's mirror ghost conditions, damping profile and injection.

Mirror ghosts (paper, "Boundary conditions and domain truncation": null
Dirichlet and null Neumann conditions by ghost nodes; "Space discretization"):
* The image method: a Dirichlet (Neumann) side is the symmetry plane of a
  problem doubled about the boundary node, with the model mirrored evenly and
  the sources mirrored with the opposite (same) sign.  A run with the mirror
  condition on the half grid must give the traces and wavefield of the doubled
  run with zero ghosts far away, for all three operators.  This pins the sign
  and the centre of the wavefield mirror, the hold of Dirichlet nodes at zero
  and the image of the model (velocity, density, face buoyancy) in the ghosts;
  a nearest-node copy of a density that varies at the side fails it.
* Manufactured solutions with density varying at mirrored sides (the
  "Verification" section's approach): a density that is itself symmetric about
  the sides converges at the space order (to the time-error floor with
  Dirichlet sides); a density with a non-zero normal derivative at the side is
  not the restriction of any symmetric problem, and the measured order falls to
  2 (Dirichlet) and about 3 (Neumann) for both variable-density operators.

Damping profile ("Boundary conditions and domain truncation": eta = alpha d^p
with d the distance to the physical domain): values at an edge node and at a
corner node, written out by hand.

Injection ("Sources and receivers", source term): the per-node sums of
injection_terms() equal what inject() adds.
"""
import math

import numpy as np
import pytest
import sympy as sp

import oracle
from oracle import coeffs
import tests.test_oracle_physics as phys
from tests._analytic import X, T


def _doubled_pair(scheme, bc, ndim, axis, side, so, nsteps=70, layer=5, depth=None,
                  rec_interp="linear"):
    """Traces and fields of (mirror run on the half grid, doubled run).  depth:
    the source's distance from the mirrored side in cells (default 31% of the
    axis); rec_interp: receiver interpolation (Kaiser-sinc footprints of
    receivers on or near the side cross it)."""
    n = (17, 23) if ndim == 2 else (11, 13, 12)
    h = (10.0, 12.5) if ndim == 2 else (10.0, 12.5, 11.0)
    rng = np.random.default_rng(11 + axis + 3 * side + 7 * ndim)
    c = 1800.0 + 500.0 * rng.random(n)
    rho = 1.0 + 2.0 * rng.random(n) if scheme != "const" else None
    nbl = [[layer, layer] for _ in range(ndim)]
    nbl[axis][side] = 0
    bcs = [["none", "none"] for _ in range(ndim)]
    bcs[axis][side] = bc

    def mirror(a):
        if a is None:
            return None
        a = np.moveaxis(a, axis, 0)
        d = np.concatenate([a[:0:-1], a]) if side == 0 else np.concatenate([a, a[-2::-1]])
        return np.ascontiguousarray(np.moveaxis(d, 0, axis))

    nd = list(n)
    nd[axis] = 2 * n[axis] - 1
    nbld = [list(p) for p in nbl]
    nbld[axis] = [layer, layer]
    dt = 0.5 * coeffs.critical_dt(h, so, float(c.max()))
    wav = oracle.ricker(25.0, dt, nsteps)
    # a source away from the mirrored side, receivers anywhere in the half grid
    ext = [(k - 1) * hh for k, hh in zip(n, h)]
    s = [0.37 * e for e in ext]
    dd = 0.31 * ext[axis] if depth is None else depth * h[axis]
    s[axis] = dd if side == 0 else ext[axis] - dd
    recs = [[0.2 * e for e in ext], [0.85 * e for e in ext], [0.5 * e for e in ext]]
    recs[0][axis] = 0.0 if side == 0 else ext[axis]         # on the mirrored side
    recs[1][axis] = (0.04 if side == 0 else 0.96) * ext[axis]
    sign = -1.0 if bc == "dirichlet" else 1.0
    # doubled grid: shift of the half grid's physical origin along the axis
    shift = (n[axis] - 1) * h[axis] if side == 0 else 0.0
    centre = (n[axis] - 1) * h[axis] if side == 0 else (n[axis] - 1) * h[axis]
    s_d = list(s)
    s_d[axis] = s[axis] + shift
    img = list(s_d)
    img[axis] = 2.0 * centre - s_d[axis]
    recs_d = [list(r) for r in recs]
    for r in recs_d:
        r[axis] += shift

    runs = []
    for nn, nb, bb, cc, rr, srcs, w, rec in (
            (n, nbl, bcs, c, rho, [s], wav[:, None], recs),
            (tuple(nd), nbld, None, mirror(c), mirror(rho), [s_d, img], np.stack([wav, sign * wav], 1), recs_d)):
        prob = oracle.Problem(n=nn, h=h, space_order=so, dt=dt, nsteps=nsteps, scheme=scheme,
                              nbl=[tuple(p) for p in nb],
                              bc=None if bb is None else [tuple(p) for p in bb])
        st = oracle.prepare(prob, cc, rr)
        fw = oracle.forward(st, w, oracle.geometry_table(prob, srcs, role="source"),
                            oracle.geometry_table(prob, rec, rec_interp, role="receiver"), len(rec))
        runs.append((fw, prob))
    (fh, ph), (fd, pd) = runs
    # the half grid's extended nodes inside the doubled extended grid
    off = pd.N[axis] - ph.N[axis] if side == 0 else 0
    sl = [slice(None)] * ndim
    sl[axis] = slice(off, off + ph.N[axis])
    return fh.traces, fd.traces, fh.p, fd.p[tuple(sl)]


CASES = [(2, 0, 0), (2, 0, 1), (2, 1, 0), (2, 1, 1), (3, 2, 0), (3, 0, 1)]


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
@pytest.mark.parametrize("depth", [0.0, 1.3, 3.41, 5.5])
def test_mirror_source_near_side_is_doubled_problem(bc, depth):
    # Kaiser-sinc source and receivers whose footprints cross the mirrored
    # side (on the boundary node itself at depth 0): image sources and ghost
    # reads make the half-grid run the doubled problem's restriction
    for scheme, ndim, axis, side in (("const", 2, 0, 0), ("vd_staggered", 2, 1, 1), ("vd_centred", 3, 2, 0)):
        th, td, ph, pd = _doubled_pair(scheme, bc, ndim, axis, side, 8 if ndim == 2 else 4,
                                       depth=depth, rec_interp="hicks")
        if bc == "dirichlet" and depth == 0.0:
            # a source on a Dirichlet plane is cancelled by its image
            assert np.max(np.abs(ph)) == 0.0 and np.max(np.abs(pd)) < 1e-30
            continue
        assert np.max(np.abs(pd)) > 0
        assert np.max(np.abs(ph - pd)) <= 1e-12 * np.max(np.abs(pd)), (scheme, ndim, axis, side)
        assert np.max(np.abs(th - td)) <= 1e-12 * np.max(np.abs(td)), (scheme, ndim, axis, side)


@pytest.mark.parametrize("scheme", ["const", "vd_staggered", "vd_centred"])
@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
@pytest.mark.parametrize("ndim,axis,side", CASES)
def test_mirror_is_doubled_problem(scheme, bc, ndim, axis, side):
    so = 8 if ndim == 2 else 4
    th, td, ph, pd = _doubled_pair(scheme, bc, ndim, axis, side, so)
    scale = np.max(np.abs(pd))
    assert scale > 0 and np.max(np.abs(td)) > 0
    assert np.max(np.abs(ph - pd)) <= 1e-12 * scale
    assert np.max(np.abs(th - td)) <= 1e-12 * np.max(np.abs(td))


def _sym_rho():
    L = 440.0
    return (2 + sp.cos(sp.pi * X[0] / L)) * (2 + sp.cos(sp.pi * X[1] / L))


def _lin_rho():
    L = 440.0
    return (2 + X[0] / L) * (2 + X[1] / L)


def _mms_errors(scheme, bc, rho, hs, so=4, dt=5e-6, tf=0.03):
    L, c = 440.0, 2000.0
    sx = sp.sin if bc == "dirichlet" else sp.cos
    u = sx(sp.pi * X[0] / L) * sx(sp.pi * X[1] / L) * sp.sin(20 * sp.pi * T) * sp.sin(20 * sp.pi * (T + dt))
    return [phys._mms_run(scheme, so, h, c, u, rho, (bc, bc), L, tf, dt, receiver=(40.0, 200.0))
            for h in hs]


@pytest.mark.parametrize("scheme", ["vd_staggered", "vd_centred"])
def test_mms_symmetric_density_dirichlet(scheme):
    # density symmetric about every side: the doubled problem is smooth, and the
    # error at h = 20 m reaches the time-error floor (a nearest-node copy of the
    # density into the ghosts leaves it above 2e-5)
    e40, e20 = _mms_errors(scheme, "dirichlet", _sym_rho(), (40.0, 20.0))
    assert e20 < 2e-7, (e40, e20)
    assert math.log2(e40 / e20) > 3.8, (e40, e20)


@pytest.mark.parametrize("scheme", ["vd_staggered", "vd_centred"])
def test_mms_symmetric_density_neumann(scheme):
    errs = _mms_errors(scheme, "neumann", _sym_rho(), (40.0, 20.0, 10.0))
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(slopes) > 3.5, (errs, slopes)


@pytest.mark.parametrize("scheme", ["vd_staggered", "vd_centred"])
@pytest.mark.parametrize("bc,lo,hi", [("dirichlet", 1.9, 2.5), ("neumann", 2.5, 3.4)])
def test_mms_density_gradient_at_side_order(scheme, bc, lo, hi):
    # a density whose normal derivative does not vanish at the side: measured
    # order 2 with Dirichlet and about 3 with Neumann sides, at SO4
    errs = _mms_errors(scheme, bc, _lin_rho(), (40.0, 20.0, 10.0))
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(lo < s < hi for s in slopes), (errs, slopes)


def test_damping_profile_values():
    # physical box: z nodes 3..7, x nodes 2..8 of a 12 x 14 extended grid;
    # alpha = 0.002, p = 3; values by hand
    prob = oracle.Problem(n=(5, 7), h=(10.0, 10.0), space_order=4, dt=1e-3, nsteps=1,
                          nbl=((3, 4), (2, 5)), alpha=0.002, power=3.0)
    eta = oracle.damping(prob)
    assert eta.shape == (12, 14)
    assert eta[5, 5] == 0.0                               # physical node
    assert eta[3, 2] == 0.0 and eta[7, 8] == 0.0          # physical corners
    assert eta[0, 5] == pytest.approx(0.054, rel=1e-14)  # 3 cells above the box: 0.002 * 27
    assert eta[11, 5] == pytest.approx(0.128, rel=1e-14)  # 4 cells below: 0.002 * 64
    assert eta[5, 13] == pytest.approx(0.25, rel=1e-14)   # 5 cells right: 0.002 * 125
    # corner node (0, 0): 3 cells in z, 2 in x, d = sqrt(13), d^3 = 46.872166581031856
    assert eta[0, 0] == pytest.approx(0.09374433316206371, rel=1e-13)
    # corner node (10, 12): 3 cells in z, 4 in x, d = 5
    assert eta[10, 12] == pytest.approx(0.25, rel=1e-14)


def test_injection_terms_match_inject():
    prob = oracle.Problem(n=(21, 19), h=(10.0, 8.0), space_order=4, dt=1e-3, nsteps=1,
                          nbl=((4, 4), (4, 4)))
    rng = np.random.default_rng(4)
    st = oracle.prepare(prob, 1500.0 + 1000.0 * rng.random((21, 19)))
    # overlapping footprints: two sources 1.3 cells apart share nodes
    table = oracle.geometry_table(prob, [(83.0, 71.3), (96.0, 76.1), (150.0, 20.0)])
    amps = np.array([0.7, -1.3, 2.1])
    field = np.zeros(int(np.prod(prob.N)))
    oracle.core.inject(st, field, table, amps)
    nodes, vals = oracle.injection_terms(st, table, amps)
    assert len(nodes) < len(table[0])                     # shared nodes exist
    assert np.allclose(field[nodes], vals, rtol=1e-14, atol=0.0)
    rest = np.ones(field.size, bool)
    rest[nodes] = False
    assert np.all(field[rest] == 0.0)
