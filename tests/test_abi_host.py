"""Host-side checks of the C ABI (no GPU): every declared symbol is exported,
host helpers and host tables agree with the oracle, invalid input is refused
before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from oracle import coeffs

from paper_2201_05278_amd import _lib as L
from paper_2201_05278_amd import Propagator, critical_dt, steps_for, ricker, SimwaveError

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "simwave_hip.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 14
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(L.SIGNATURES), set(names) - set(L.SIGNATURES)
    assert lib.sw_abi_version() == 1


@pytest.mark.parametrize("ndim,h,so,cmax", [(2, 10.0, 2, 4700.0), (2, 10.0, 8, 4700.0),
                                            (3, 20.0, 4, 6000.0), (3, 10.0, 16, 4500.0)])
def test_critical_dt_and_steps_match_oracle(ndim, h, so, cmax):
    a = critical_dt([h] * ndim, so, cmax)
    b = coeffs.critical_dt([h] * ndim, so, cmax)
    assert abs(a - b) <= 1e-14 * b
    assert steps_for(2.0, a) == coeffs.steps_for(2.0, b)


def test_ricker_matches_oracle():
    dt = 5e-4
    got = ricker(12.0, dt, 400).numpy()
    ref = oracle.ricker(12.0, dt, 400)
    assert np.max(np.abs(got - ref)) < 1e-7


def _compare_tables(prop, prob, which, coords, interp, radius=4):
    nodes, ids, w = prop.point_table(which)
    ref_nodes, ref_ids, ref_w = oracle.geometry_table(prob, coords, interp, radius,
                                                      role="source" if which == "src" else "receiver")
    lay = prop.layout
    # map padded-layout offsets back to extended-grid flat indices
    off = nodes - lay.origin
    if prop.ndim == 3:
        p1, p2 = lay.padded[1], lay.padded[2]
        z, r = np.divmod(off, p1 * p2)
        x, y = np.divmod(r, p2)
        flat = (z * lay.dims[1] + x) * lay.dims[2] + y
    else:
        z, x = np.divmod(off, lay.padded[1])
        flat = z * lay.dims[1] + x
    got = sorted(zip(ids.tolist(), flat.tolist(), w.tolist()))
    ref = sorted(zip(ref_ids.tolist(), ref_nodes.tolist(), ref_w.tolist()))
    assert [g[:2] for g in got] == [r[:2] for r in ref]
    assert np.allclose([g[2] for g in got], [r[2] for r in ref], rtol=2e-7, atol=1e-9)


@pytest.mark.parametrize("interp", ["hicks", "linear"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_point_tables_match_oracle(interp, ndim):
    n = (30, 41, 37)[:ndim]
    h = (10.0, 12.0, 8.0)[:ndim]
    nbl = ((5, 7), (6, 4), (3, 8))[:ndim]
    prob = oracle.Problem(n=n, h=h, space_order=8, dt=1e-3, nsteps=10, nbl=nbl)
    prop = Propagator(n, h, 8, 1e-3, 10, nbl=[list(x) for x in nbl])
    rng = np.random.default_rng(1)
    coords = rng.uniform(0.2, 0.8, size=(7, ndim)) * (np.array(n) - 1) * np.array(h)
    coords[0] = (np.array(n) // 2) * np.array(h)          # an on-node point
    prop.set_sources(coords, interp)
    prop.set_receivers(coords[::-1], interp)
    _compare_tables(prop, prob, "src", coords, interp)
    _compare_tables(prop, prob, "rec", coords[::-1], interp)


@pytest.mark.parametrize("interp", ["hicks", "linear"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_point_tables_with_mirror_sides_match_oracle(interp, ndim):
    # footprints crossing Dirichlet / Neumann sides: sources take their images,
    # receivers read ghosts (as the image method of those conditions defines)
    n = (30, 41, 37)[:ndim]
    h = (10.0, 12.0, 8.0)[:ndim]
    nbl = ((0, 7), (0, 0), (3, 0))[:ndim]
    bc = (("dirichlet", "none"), ("neumann", "dirichlet"), ("none", "neumann"))[:ndim]
    prob = oracle.Problem(n=n, h=h, space_order=8, dt=1e-3, nsteps=10, nbl=nbl, bc=bc)
    prop = Propagator(n, h, 8, 1e-3, 10, nbl=[list(x) for x in nbl], bc=[list(b) for b in bc])
    rng = np.random.default_rng(2)
    ext = (np.array(n) - 1) * np.array(h)
    coords = rng.uniform(0.2, 0.8, size=(6, ndim)) * ext
    coords[0, 0] = 1.3 * h[0]                 # near the Dirichlet top
    coords[1, 0] = 0.0                        # on it
    coords[2, 1] = 0.4 * h[1]                 # near the second axis' low side
    coords[3, 1] = ext[1] - 0.7 * h[1]        # near its high side
    coords[4, 0] = 2.2 * h[0]
    coords[4, 1] = 1.6 * h[1]                 # near a corner of two mirrored sides
    prop.set_sources(coords, interp)
    prop.set_receivers(coords[::-1], interp)
    _compare_tables(prop, prob, "src", coords, interp)
    _compare_tables(prop, prob, "rec", coords[::-1], interp)
    # a window reaching past the mirror of a short axis is refused on both sides
    short = (6,) + tuple(n[1:])
    prob_s = oracle.Problem(n=short, h=h, space_order=8, dt=1e-3, nsteps=10, nbl=((0, 0),) + nbl[1:], bc=bc)
    prop_s = Propagator(short, h, 8, 1e-3, 10, nbl=[[0, 0]] + [list(x) for x in nbl[1:]],
                        bc=[list(b) for b in bc])
    pt = [[2.5 * h[0]] + [0.5 * e for e in ext[1:]]]
    with pytest.raises(ValueError):
        oracle.geometry_table(prob_s, pt, "hicks", 4, role="receiver")
    _expect("SW_ERR_DOMAIN", prop_s.set_receivers, pt, "hicks")


def test_layout_is_aligned_and_padded():
    prop = Propagator((50, 60, 70), (10.0,) * 3, 8, 1e-3, 10, nbl=40)
    lay = prop.layout
    assert tuple(lay.dims) == (130, 140, 150)
    assert lay.padded[2] % 64 == 0
    assert lay.origin % 64 == 0                       # interior rows 256-byte aligned
    assert lay.field_elems == lay.padded[0] * lay.padded[1] * lay.padded[2]
    assert lay.halo == 4
    p2 = Propagator((50, 60), (10.0, 10.0), 4, 1e-3, 10, nbl=[(0, 70), (70, 70)])
    l2 = p2.layout
    assert tuple(l2.dims[:2]) == (120, 200) and l2.padded[1] % 64 == 0


def _expect(status_name, fn, *a, **k):
    with pytest.raises(SimwaveError) as e:
        fn(*a, **k)
    assert L.STATUS[e.value.status] == status_name, str(e.value)


def test_invalid_problems_refused():
    _expect("SW_ERR_UNSUPPORTED", Propagator, (20, 20), (1.0, 1.0), 3, 1e-3, 5)
    _expect("SW_ERR_UNSUPPORTED", Propagator, (20, 20), (1.0, 1.0), 22, 1e-3, 5)
    _expect("SW_ERR_ARG", Propagator, (20, 20), (1.0, -1.0), 4, 1e-3, 5)
    _expect("SW_ERR_ARG", Propagator, (20, 20), (1.0, 1.0), 4, -1e-3, 5)
    # a padded z plane too large for the 32-bit window offsets (9000^2 x 4 B x 18 planes)
    _expect("SW_ERR_UNSUPPORTED", Propagator, (4, 9000, 9000), (1.0,) * 3, 8, 1e-4, 5, nbl=0)
    Propagator((4, 2000, 2000), (1.0,) * 3, 8, 1e-4, 5, nbl=0)


def test_mirror_ghost_contract():
    # Dirichlet / Neumann sides are accepted for the forward ...
    prop = Propagator((20, 24, 28), (10.0,) * 3, 8, 1e-3, 5, nbl=2,
                      bc=[("dirichlet", "neumann"), ("none", "dirichlet"), ("neumann", "none")])
    # ... but not by the adjoint, batches, wave tiles or two-step sweeps
    io = L.AdjIO()
    st = L.lib().sw_adjoint(prop._plan, ctypes.byref(io), None)
    assert L.STATUS[st] == "SW_ERR_UNSUPPORTED"
    assert b"ghost" in L.lib().sw_last_error()
    plans = (ctypes.c_void_p * 1)(prop._plan.value)
    out = ctypes.c_void_p()
    st = L.lib().sw_batch_create(1, plans, ctypes.byref(out))
    assert L.STATUS[st] == "SW_ERR_UNSUPPORTED"
    _expect("SW_ERR_UNSUPPORTED", prop.set_tiling, 16, 4, wt=1)
    _expect("SW_ERR_UNSUPPORTED", prop.set_tiling, ts=2)
    prop.set_tiling(16, 8)
    # an axis shorter than the mirror depth plus one, and unknown conditions
    _expect("SW_ERR_UNSUPPORTED", Propagator, (3, 20), (10.0, 10.0), 8, 1e-3, 5, nbl=0,
            bc=[("dirichlet", "none"), ("none", "none")])
    Propagator((5, 20), (10.0, 10.0), 8, 1e-3, 5, nbl=0, bc=[("dirichlet", "none"), ("none", "none")])
    _expect("SW_ERR_UNSUPPORTED", Propagator, (7, 20), (10.0, 10.0), 8, 1e-3, 5, scheme="vd_staggered",
            nbl=0, bc=[("neumann", "none"), ("none", "none")])
    prob = L.Problem()
    prob.ndim, prob.space_order, prob.dt, prob.nsteps = 2, 4, 1e-3, 5
    prob.n[0] = prob.n[1] = 20
    prob.h[0] = prob.h[1] = 1.0
    prob.bc[0][0] = 7
    h = ctypes.c_void_p()
    st = L.lib().sw_plan_create(ctypes.byref(prob), ctypes.byref(h))
    assert L.STATUS[st] == "SW_ERR_ARG"


def test_points_outside_domain_refused():
    prop = Propagator((20, 20), (10.0, 10.0), 4, 1e-3, 5, nbl=0)
    _expect("SW_ERR_DOMAIN", prop.set_sources, [[-1.0, 50.0]])
    _expect("SW_ERR_DOMAIN", prop.set_sources, [[15.0, 50.0]], "hicks", 4)   # footprint leaves grid
    _expect("SW_ERR_ARG", prop.set_sources, [[100.0, 100.0]], "hicks", 3)    # no Kaiser b for r=3
    prop.set_sources([[100.0, 100.0]], "hicks", 3, 4.0)
    prop.set_sources([[0.0, 0.0]], "linear")


def test_cfl_violation_refused_before_device_work():
    prop = Propagator((20, 20), (10.0, 10.0), 8, 1e-2, 5, nbl=0)
    lib = L.lib()
    fake = ctypes.c_void_p(4096)
    st = lib.sw_model_prepare(prop._plan, fake, None, 1500.0, fake, None)
    assert L.STATUS[st] == "SW_ERR_CFL"
    assert b"stability" in lib.sw_last_error()
    st = lib.sw_model_prepare(prop._plan, fake, None, 1500.0, ctypes.c_void_p(4100), None)
    assert L.STATUS[st] == "SW_ERR_WORKSPACE"


def test_forward_before_prepare_refused():
    prop = Propagator((20, 20), (10.0, 10.0), 4, 1e-3, 5, nbl=0)
    io = L.FwdIO()
    st = L.lib().sw_forward(prop._plan, ctypes.byref(io), None)
    assert L.STATUS[st] == "SW_ERR_STATE"


def test_tiling_choices_validated():
    prop = Propagator((30, 30, 30), (10.0,) * 3, 8, 1e-3, 5, nbl=4)
    prop.set_tiling(ts=2)
    t = prop.tiling
    assert (t["ts"], t["tx"], t["nw"], t["wt"]) == (2, 8, 4, 0)
    prop.set_tiling(16, 8, ts=2)                 # 2 (5R+5) + 1 (3R+3) = 65 values fit at R = 4
    _expect("SW_ERR_UNSUPPORTED", prop.set_tiling, 16, 4, ts=2)   # 4 (5R+5) + 2 (3R+3) = 130
    _expect("SW_ERR_ARG", prop.set_tiling, ts=3)
    _expect("SW_ERR_ARG", prop.set_tiling, 8, 1, wt=1, ts=2)
    _expect("SW_ERR_UNSUPPORTED", prop.set_tiling, 32, 8, ts=2)
    prop.set_tiling()
    assert prop.tiling["ts"] in (1, 2)
    so16 = Propagator((30, 30, 30), (10.0,) * 3, 16, 1e-4, 5, nbl=4)
    _expect("SW_ERR_UNSUPPORTED", so16.set_tiling, 8, 4, ts=2)    # 2 * 45 + 4 * 27 > 95
    _expect("SW_ERR_UNSUPPORTED", so16.set_tiling, 8, 8, ts=2)    # 45 + 2 * 27 > 95
    _expect("SW_ERR_UNSUPPORTED", so16.set_tiling, ts=2)
    so14 = Propagator((30, 30, 30), (10.0,) * 3, 14, 1e-4, 5, nbl=4)
    so14.set_tiling(8, 8, ts=2)
    flat = Propagator((30, 30), (10.0,) * 2, 8, 1e-3, 5, nbl=4)
    _expect("SW_ERR_UNSUPPORTED", flat.set_tiling, ts=2)
    vd = Propagator((30, 30, 30), (10.0,) * 3, 8, 1e-3, 5, scheme="vd_staggered", nbl=4)
    _expect("SW_ERR_UNSUPPORTED", vd.set_tiling, ts=2)


def test_occupancy_cap_and_default_tiles():
    # default constant-density tiles by order, with their resident-block caps
    expect = {2: (8, 4, 4), 4: (8, 4, 4), 6: (24, 8, 0), 8: (24, 8, 0), 10: (24, 8, 0),
              12: (16, 4, 3), 14: (8, 4, 0), 16: (8, 4, 0)}
    for so, (tx, nw, occ) in expect.items():
        t = Propagator((40, 40, 40), (10.0,) * 3, so, 1e-4, 5, nbl=4).tiling
        assert (t["tx"], t["nw"], t["occ"], t["ts"], t["wt"]) == (tx, nw, occ, 1, 0), so
    prop = Propagator((40, 40, 40), (10.0,) * 3, 4, 1e-3, 5, nbl=4)
    prop.set_tiling(16, 4)                        # an explicit shape has no cap by default
    assert prop.tiling["occ"] == 0
    for occ in (0, 3, 4, 5, 6):
        prop.set_tiling(16, 4, occ=occ)
        assert prop.tiling["occ"] == occ
    for bad in (-2, 1, 2, 7, 64):
        _expect("SW_ERR_ARG", prop.set_tiling, 16, 4, occ=bad)
    prop.set_tiling(16, 4, wt=1, occ=4)           # wave tiles and two-step sweeps take no cap
    assert prop.tiling["occ"] == 0
    prop.set_tiling(ts=2, occ=4)
    assert prop.tiling["occ"] == 0
    prop.set_tiling()
    assert (prop.tiling["tx"], prop.tiling["occ"]) == (8, 4)
    vd = Propagator((40, 40, 40), (10.0,) * 3, 8, 1e-3, 5, scheme="vd_staggered", nbl=4)
    vd.set_tiling(8, 4, occ=5)
    assert vd.tiling["occ"] == 5


def test_variable_density_default_tiles():
    # default tile by scheme and order (measured per order)
    expect = {("vd_staggered", 4): (8, 4), ("vd_staggered", 8): (8, 4), ("vd_staggered", 14): (8, 4),
              ("vd_staggered", 16): (16, 8), ("vd_staggered", 18): (8, 8), ("vd_staggered", 20): (8, 8),
              ("vd_centred", 4): (8, 4), ("vd_centred", 8): (16, 8), ("vd_centred", 12): (8, 8),
              ("vd_centred", 16): (8, 8), ("vd_centred", 20): (8, 4)}
    for (scheme, so), (tx, nw) in expect.items():
        t = Propagator((40, 40, 40), (10.0,) * 3, so, 1e-4, 5, nbl=4, scheme=scheme).tiling
        assert (t["tx"], t["nw"]) == (tx, nw), (scheme, so)
    prop = Propagator((40, 40, 40), (10.0,) * 3, 16, 1e-4, 5, nbl=4, scheme="vd_staggered")
    prop.set_tiling(8, 4)
    assert (prop.tiling["tx"], prop.tiling["nw"]) == (8, 4)


def test_adjoint_scheme_contract():
    # the centred variable-density operator is not symmetric: no adjoint for it;
    # the staggered one is (it then needs a prepared plan like any other)
    io = L.AdjIO()
    cen = Propagator((20, 24, 28), (10.0,) * 3, 8, 1e-3, 5, scheme="vd_centred", nbl=2)
    st = L.lib().sw_adjoint(cen._plan, ctypes.byref(io), None)
    assert L.STATUS[st] == "SW_ERR_UNSUPPORTED"
    stag = Propagator((20, 24, 28), (10.0,) * 3, 8, 1e-3, 5, scheme="vd_staggered", nbl=2)
    st = L.lib().sw_adjoint(stag._plan, ctypes.byref(io), None)
    assert L.STATUS[st] == "SW_ERR_STATE"


def test_double_precision_contract():
    # a double-precision plan: constant density only; it is served by the _f64
    # entry points and refused by the single-precision ones (and vice versa)
    _expect("SW_ERR_UNSUPPORTED", Propagator, (20, 24, 28), (10.0,) * 3, 8, 1e-3, 5, scheme="vd_staggered",
            dtype="float64")
    p64 = Propagator((20, 24, 28), (10.0,) * 3, 8, 1e-3, 5, nbl=2, dtype="float64")
    p32 = Propagator((20, 24, 28), (10.0,) * 3, 8, 1e-3, 5, nbl=2)
    # doubles in the workspace
    assert p64.layout.workspace_bytes > p32.layout.workspace_bytes
    st = L.lib().sw_model_prepare(p64._plan, ctypes.c_void_p(256), None, 2000.0, ctypes.c_void_p(256), None)
    assert L.STATUS[st] == "SW_ERR_STATE"
    st = L.lib().sw_model_prepare_f64(p32._plan, ctypes.c_void_p(256), 2000.0, ctypes.c_void_p(256), None)
    assert L.STATUS[st] == "SW_ERR_STATE"
    io = L.FwdIO()
    st = L.lib().sw_forward(p64._plan, ctypes.byref(io), None)
    assert L.STATUS[st] in ("SW_ERR_STATE", "SW_ERR_ARG")
    # double precision takes its own tile shapes and a z chunk, nothing else
    _expect("SW_ERR_UNSUPPORTED", p64.set_tiling, 16, 4)
    _expect("SW_ERR_UNSUPPORTED", p64.set_tiling, 8, 8, ts=2)
    _expect("SW_ERR_UNSUPPORTED", p64.set_tiling, 8, 8, occ=4)
    assert (p64.tiling["tx"], p64.tiling["nw"]) == (8, 4)        # SO8 default
    p64.set_tiling(16, 8, 9)
    assert (p64.tiling["tx"], p64.tiling["nw"], p64.tiling["zc"]) == (16, 8, 9)
    p64.set_tiling()
    assert (p64.tiling["tx"], p64.tiling["nw"]) == (8, 4)
    hi = Propagator((20, 24, 28), (10.0,) * 3, 12, 1e-4, 5, nbl=2, dtype="float64")
    assert (hi.tiling["tx"], hi.tiling["nw"]) == (8, 8)


def test_batch_tiling_contract():
    lib = L.lib()

    def batch_of(props):
        arr = (ctypes.c_void_p * len(props))(*[p._plan.value for p in props])
        h = ctypes.c_void_p()
        assert L.STATUS[lib.sw_batch_create(len(props), arr, ctypes.byref(h))] == "SW_OK"
        return h

    def get(h):
        t, bpc = L.Tiling(), ctypes.c_int32()
        assert L.STATUS[lib.sw_batch_get_tiling(h, ctypes.byref(t), ctypes.byref(bpc))] == "SW_OK"
        return (t.tx, t.nw, t.zc, t.nt, t.pf, bpc.value)

    def put(h, cfg, bpc=0):
        t = None if cfg is None else L.Tiling(*cfg)
        return L.STATUS[lib.sw_batch_set_tiling(h, ctypes.byref(t) if t is not None else None, bpc)]

    shots = [Propagator((30, 34, 40), (10.0,) * 3, 8, 1e-3, 5, nbl=4),
             Propagator((26, 40, 30), (10.0,) * 3, 8, 1e-3, 5, nbl=4)]
    h = batch_of(shots)
    try:
        assert get(h) == (16, 4, 64, 1, 1, 0)
        assert put(h, (24, 8, 11, 0, 2, 0, 1, 0, 1), -1) == "SW_OK"
        assert get(h) == (24, 8, 11, 0, 2, -1)
        assert put(h, (8, 4, 0, 1, 1, 0, 1, 0, 1), 6) == "SW_OK"
        assert get(h)[2:] == (64, 1, 1, 6)
        assert put(h, (12, 4, 0, 1, 1, 0, 1, 0, 1)) == "SW_ERR_ARG"          # shape not instantiated
        assert put(h, (16, 4, 0, 1, 3, 0, 1, 0, 1)) == "SW_ERR_ARG"          # prefetch depth
        assert put(h, (16, 4, 0, 1, 1, 0, 1, 0, 1), -2) == "SW_ERR_ARG"      # grid option
        assert put(h, (16, 4, 0, 1, 1, 1, 1, 0, 1)) == "SW_ERR_UNSUPPORTED"  # wave tiles
        assert put(h, (16, 4, 0, 1, 1, 0, 2, 0, 1)) == "SW_ERR_UNSUPPORTED"  # two-step sweep
        assert put(h, None) == "SW_OK"
        assert get(h) == (16, 4, 64, 1, 1, 0)
    finally:
        lib.sw_batch_destroy(h)
    h = batch_of([Propagator((30, 34), (10.0,) * 2, 8, 1e-3, 5, nbl=4)])
    try:
        assert get(h)[:2] == (1, 1)
        assert put(h, (16, 4, 0, 1, 1, 0, 1, 0, 1)) == "SW_ERR_ARG"
        assert put(h, None) == "SW_OK"
        assert get(h)[:2] == (1, 1)
    finally:
        lib.sw_batch_destroy(h)


def test_roctx_ranges_open_the_tracing_library():
    # in a process without torch: the first enqueueing call (here refused for a
    # NULL plan) opens the roctx library for its range; SW_ROCTX=0 keeps it closed
    import subprocess
    import sys
    code = (
        "import ctypes, sys\n"
        "lib = ctypes.CDLL(sys.argv[1])\n"
        "maps = lambda: 'librocprofiler-sdk-roctx' in open('/proc/self/maps').read()\n"
        "before = maps()\n"
        "st = lib.sw_forward(None, None, None)\n"
        "print(int(before), int(maps()), st)\n")
    path = L.LIB_PATH
    for env, want in ((None, "0 1"), ("0", "0 0")):
        e = dict(os.environ)
        e.pop("SW_ROCTX", None)
        if env is not None:
            e["SW_ROCTX"] = env
        out = subprocess.run([sys.executable, "-c", code, path], capture_output=True, text=True, env=e,
                             timeout=120)
        assert out.returncode == 0, out.stderr
        before_after, st = out.stdout.split()[:2], int(out.stdout.split()[2])
        assert " ".join(before_after) == want, out.stdout
        assert L.STATUS[st] == "SW_ERR_ARG"
