"""The double-precision forward (the paper's dtype option; its benchmark runs
are float64) against the FP64 oracle, at an FP64 tolerance: traces and
fields within relative L2 1e-10 (single precision reaches about 1e-6 on the
same runs), in 3D with ragged tiles at space orders 2, 8 and 20, and in 2D
with a free surface, a layer and snapshots."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2201_05278_amd import Propagator
from tests._parity import trace_errors

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _pair(n, h, so, nbl, bc, nsteps, vel, src, rec, interp, dtype, saving_stride=0):
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(h, so, float(vel.max()))
    prob = oracle.Problem(n=n, h=h, space_order=so, dt=dt, nsteps=nsteps,
                          nbl=tuple(tuple(p) for p in nbl), bc=None if bc is None else tuple(tuple(b) for b in bc))
    st = oracle.prepare(prob, vel.astype(np.float64))
    wav = oracle.ricker(16.0, dt, nsteps)[:, None]
    roles = {} if bc is None else {"role": "source"}
    rrole = {} if bc is None else {"role": "receiver"}
    ref = oracle.forward(st, wav, oracle.geometry_table(prob, src, interp, **roles),
                         oracle.geometry_table(prob, rec, interp, **rrole), len(rec), snap_stride=saving_stride)
    prop = Propagator(n, h, so, dt, nsteps, nbl=[list(p) for p in nbl], bc=bc, dtype=dtype)
    prop.set_sources(src, interp)
    prop.set_receivers(rec, interp)
    prop.prepare(torch.from_numpy(vel.astype(np.float64)).cuda())
    res = prop.forward(torch.from_numpy(wav).cuda(), saving_stride=saving_stride)
    torch.cuda.synchronize()
    return ref, res, prop


@pytest.mark.parametrize("so", [2, 8, 20])
def test_fp64_3d_ragged(so):
    n = (29, 37, 70)
    rng = np.random.default_rng(80 + so)
    vel = workloads.layered(n, [1600.0, 2300.0, 3100.0], rng, 40.0).astype(np.float64)
    h = (10.0, 10.0, 10.0)
    src = np.array([[101.3, 171.7, 345.2]])
    rec = np.array([[5.0 * k, 10.0 * k, 9.0 * k + 3.3] for k in range(30)])
    print(f"case: fp64 3D {n} SO{so}", flush=True)
    ref, res, prop = _pair(n, h, so, [(6, 6)] * 3, None, 120, vel, src, rec, "hicks", "float64")
    assert res.traces.dtype == torch.float64
    total, worst, _ = trace_errors(res.traces, ref.traces)
    assert total < TOL64 and worst < TOL64, (total, worst)
    assert _rel(prop.grid_view(res.fields[res.current]).cpu().numpy(), ref.p) < TOL64
    if so == 8:
        # the same run in single precision stays at FP32 accuracy
        ref32, res32, _ = _pair(n, h, so, [(6, 6)] * 3, None, 120, vel, src, rec, "hicks", "float32")
        t32, _, _ = trace_errors(res32.traces, ref32.traces)
        assert 1e-9 < t32 < 1e-4, t32


def test_fp64_2d_free_surface_snapshots():
    n = (60, 90)
    vel = workloads.smooth_random(n, 21, factor=8).astype(np.float64)
    h = (10.0, 10.0)
    src = np.array([[25.0, 440.0]])
    rec = np.array([[20.0, 10.0 * k] for k in range(89)])
    print("case: fp64 2D free surface, layer elsewhere, snapshots", flush=True)
    ref, res, prop = _pair(n, h, 8, [(0, 10), (10, 10)], [("dirichlet", "none"), ("none", "none")], 150, vel,
                           src, rec, "linear", "float64", saving_stride=50)
    total, worst, _ = trace_errors(res.traces, ref.traces)
    assert total < TOL64 and worst < TOL64, (total, worst)
    assert _rel(prop.grid_view(res.fields[res.current]).cpu().numpy(), ref.p) < TOL64
    assert res.snaps.shape[0] == 3
    for k in range(3):
        assert _rel(res.snaps[k].cpu().numpy(), ref.snaps[k]) < TOL64


@pytest.mark.parametrize("so", [4, 20])
def test_fp64_tile_shapes_are_bitwise_identical(so):
    # every double-precision tile shape and chunk gives the same bits (ragged
    # tiles along x and y, mirror sides), and agrees with the oracle
    n = (33, 41, 75)
    rng = np.random.default_rng(90 + so)
    vel = workloads.layered(n, [1700.0, 2600.0], rng, 30.0).astype(np.float64)
    h = (10.0, 10.0, 10.0)
    src = np.array([[151.3, 201.7, 377.2]])
    rec = np.array([[10.0, 9.0 * k, 5.0 * k + 1.3] for k in range(40)])
    bc = (("neumann", "dirichlet"), ("dirichlet", "dirichlet"), ("dirichlet", "dirichlet"))
    print(f"case: fp64 tile shapes SO{so}", flush=True)
    ref, res, prop = _pair(n, h, so, [(0, 5), (4, 4), (3, 6)], bc, 90, vel, src, rec, "linear", "float64")
    total, worst, _ = trace_errors(res.traces, ref.traces)
    assert total < TOL64 and worst < TOL64, (total, worst)
    u0 = prop.grid_view(res.fields[res.current]).clone()
    tr0 = res.traces.clone()
    wav = torch.from_numpy(oracle.ricker(16.0, prop.dt, 90)[:, None]).cuda()
    for tx, nw, zc in [(16, 8, 0), (8, 4, 7), (24, 8, 13), (8, 8, 1)]:
        print(f"case: fp64 SO{so} tile {tx}x{nw} zc={zc}", flush=True)
        prop.set_tiling(tx, nw, zc)
        r = prop.forward(wav)
        torch.cuda.synchronize()
        assert torch.equal(r.traces, tr0)
        assert torch.equal(prop.grid_view(r.fields[r.current]), u0)
    prop.set_tiling()
