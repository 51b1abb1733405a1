"""GPU parity on degenerate inputs: grids smaller than one tile and than the
stencil, missing absorbing layers on some sides, no sources or receivers with
a non-zero initial state, zero steps, single-plane chunks."""
import numpy as np
import pytest
import torch

import oracle
from tests._parity import assert_traces
import workloads
from paper_2201_05278_amd import Propagator

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _pair(n, so, nbl, nsteps, vel, src, rec, interp="linear", state=None, step0=0, scheme="const", rho=None):
    h = (10.0,) * len(n)
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(h, so, float(vel.max()))
    prob = oracle.Problem(n=n, h=h, space_order=so, dt=dt, nsteps=nsteps, scheme=scheme,
                          nbl=tuple(tuple(p) for p in nbl))
    st = oracle.prepare(prob, vel.astype(np.float64), None if rho is None else rho.astype(np.float64))
    empty = (np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0))
    src_t = oracle.geometry_table(prob, src, interp) if len(src) else empty
    rec_t = oracle.geometry_table(prob, rec, interp) if len(rec) else empty
    wav = np.stack([oracle.ricker(17.0, dt, nsteps)] * max(1, len(src)), axis=1)
    ostate = None if state is None else (state[0], state[1], step0)
    ref = oracle.forward(st, wav if len(src) else None, src_t, rec_t, len(rec), state=ostate,
                         nsteps=nsteps - step0)
    prop = Propagator(n, h, so, dt, nsteps, scheme=scheme, nbl=[list(p) for p in nbl])
    if len(src):
        prop.set_sources(src, interp)
    if len(rec):
        prop.set_receivers(rec, interp)
    prop.prepare(torch.from_numpy(vel).cuda(), None if rho is None else torch.from_numpy(rho).cuda())
    fields = None
    if state is not None:
        fields = (prop.new_field(), prop.new_field())
        prop.grid_view(fields[0]).copy_(torch.from_numpy(state[0].astype(np.float32)))
        prop.grid_view(fields[1]).copy_(torch.from_numpy(state[1].astype(np.float32)))
    res = prop.forward(torch.from_numpy(wav.astype(np.float32)).cuda(), fields=fields, step0=step0)
    torch.cuda.synchronize()
    return ref, res, prop


@pytest.mark.parametrize("scheme", ["const", "vd_staggered", "vd_centred"])
def test_grid_smaller_than_tile_and_stencil(scheme):
    # 3 x 5 x 7 nodes at SO8 (radius 4), layer only on some sides
    n = (3, 5, 7)
    nbl = [(0, 2), (1, 0), (0, 0)]
    print(f"case: tiny grid {n} SO8 {scheme}", flush=True)
    rng = np.random.default_rng(31)
    vel = (2000.0 + 100.0 * rng.standard_normal(n)).astype(np.float32)
    rho = (1800.0 + 50.0 * rng.standard_normal(n)).astype(np.float32) if scheme != "const" else None
    src = np.array([[11.0, 17.0, 33.0]])
    rec = np.array([[0.0, 0.0, 0.0], [20.0, 40.0, 60.0], [13.0, 27.0, 5.0]])
    ref, res, prop = _pair(n, 8, nbl, 40, vel, src, rec, scheme=scheme, rho=rho)
    assert_traces(res.traces, ref.traces)
    assert _rel(prop.grid_view(res.fields[res.current]).cpu().numpy(), ref.p) < 1e-4


def test_tiny_2d_so16():
    n = (4, 6)
    print("case: tiny 2D grid SO16", flush=True)
    vel = np.full(n, 1800.0, dtype=np.float32)
    ref, res, prop = _pair(n, 16, [(2, 0), (0, 3)], 30, vel, np.array([[15.0, 25.0]]),
                           np.array([[0.0, 50.0], [30.0, 0.0]]))
    assert_traces(res.traces, ref.traces)
    assert _rel(prop.grid_view(res.fields[res.current]).cpu().numpy(), ref.p) < 1e-4


def test_no_points_initial_state_and_zero_steps():
    # no sources or receivers; a seeded non-zero state at step 5 propagates
    n = (20, 24, 28)
    nbl = [(3, 3)] * 3
    print("case: no points, initial state", flush=True)
    rng = np.random.default_rng(32)
    vel = (2500.0 + 200.0 * rng.standard_normal(n)).astype(np.float32)
    N = tuple(k + 6 for k in n)
    p0 = rng.standard_normal(N)
    p1 = rng.standard_normal(N)
    ref, res, prop = _pair(n, 4, nbl, 35, vel, np.zeros((0, 3)), np.zeros((0, 3)), state=(p0, p1), step0=5)
    assert res.traces.numel() == 0
    assert _rel(prop.grid_view(res.fields[res.current]).cpu().numpy(), ref.p) < 1e-4
    # zero steps leave the fields as they are
    before = [prop.grid_view(f).clone() for f in res.fields]
    again = prop.forward(None, fields=res.fields, step0=35, nsteps_run=0)
    torch.cuda.synchronize()
    assert again.current == 0
    for f, b in zip(again.fields, before):
        assert torch.equal(prop.grid_view(f), b)


def test_single_plane_chunks_and_layerless_grid():
    # z chunks of one plane, no absorbing layer at all, every tiling path
    n = (9, 21, 70)
    print("case: one-plane chunks, no layer", flush=True)
    rng = np.random.default_rng(33)
    vel = (1500.0 + 300.0 * rng.random(n)).astype(np.float32)
    src = np.array([[40.0, 100.0, 350.0]])
    rec = np.array([[0.0, 10.0 * k, 9.0 * k] for k in range(20)])
    ref, res, prop = _pair(n, 8, [(0, 0)] * 3, 50, vel, src, rec)
    assert_traces(res.traces, ref.traces)
    wav = torch.from_numpy(np.stack([oracle.ricker(17.0, prop.dt, 50)], axis=1).astype(np.float32)).cuda()
    for tiling in [dict(tx=8, nw=4, zc=1), dict(tx=16, nw=8, zc=1, ts=2), dict(tx=8, nw=8, zc=2, ts=2)]:
        print(f"case: tiling {tiling}", flush=True)
        prop.set_tiling(**tiling)
        r = prop.forward(wav)
        torch.cuda.synchronize()
        assert torch.equal(r.traces, res.traces)
        assert torch.equal(prop.grid_view(r.fields[r.current]), prop.grid_view(res.fields[res.current]))


def test_finite_check():
    # a clean run passes the optional check; a wavelet holding an infinity makes
    # the traces and the field non-finite and the call reports SW_ERR_NONFINITE
    from paper_2201_05278_amd import SimwaveError
    from paper_2201_05278_amd import _lib as L
    n = (20, 24, 70)
    vel = np.full(n, 2000.0, dtype=np.float32)
    dt = 0.5 * oracle.coeffs.critical_dt((10.0,) * 3, 4, 2000.0)
    prop = Propagator(n, (10.0,) * 3, 4, dt, 30, nbl=3)
    prop.set_sources([[100.0, 120.0, 340.0]], "linear")
    prop.set_receivers([[20.0, 120.0, 300.0], [150.0, 50.0, 600.0]], "linear")
    prop.prepare(torch.from_numpy(vel).cuda())
    wav = torch.from_numpy(oracle.ricker(15.0, dt, 30)[:, None].astype(np.float32)).cuda()
    print("case: finite check, clean run", flush=True)
    prop.forward(wav, check_finite=True)
    bad = wav.clone()
    bad[7, 0] = float("inf")
    print("case: finite check, infinite wavelet sample", flush=True)
    with pytest.raises(SimwaveError) as e:
        prop.forward(bad, check_finite=True)
    assert L.STATUS[e.value.status] == "SW_ERR_NONFINITE"
    assert "non-finite" in str(e.value)
