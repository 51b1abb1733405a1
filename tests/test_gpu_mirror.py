"""GPU parity of the Dirichlet / Neumann mirror ghost conditions (paper,
"Boundary conditions and domain truncation") against the FP64 oracle, for the
three operators in 3D and 2D, with and without absorbing layers on the
mirrored sides, plus tiling invariance and graph replay with ghosts."""
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


def _case(n, so, nbl, bc, scheme, nsteps, src, rec, seed, src_interp="linear"):
    rng = np.random.default_rng(seed)
    vel = (2200.0 + 300.0 * rng.random(n)).astype(np.float32)
    rho = (1500.0 + 800.0 * rng.random(n)).astype(np.float32) if scheme != "const" else None
    h = (10.0,) * len(n)
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(h, so, float(vel.max()))
    prob = oracle.Problem(n=n, h=h, space_order=so, dt=dt, nsteps=nsteps, scheme=scheme,
                          nbl=tuple(tuple(p) for p in nbl), bc=tuple(tuple(b) for b in bc))
    st = oracle.prepare(prob, vel.astype(np.float64), None if rho is None else rho.astype(np.float64))
    wav = oracle.ricker(18.0, dt, nsteps)[:, None]
    ref = oracle.forward(st, wav, oracle.geometry_table(prob, src, src_interp, role="source"),
                         oracle.geometry_table(prob, rec, "linear", role="receiver"), len(rec))
    prop = Propagator(n, h, so, dt, nsteps, scheme=scheme, nbl=[list(p) for p in nbl], bc=bc)
    prop.set_sources(src, src_interp)
    prop.set_receivers(rec, "linear")
    prop.prepare(torch.from_numpy(vel).cuda(), None if rho is None else torch.from_numpy(rho).cuda())
    w = torch.from_numpy(wav.astype(np.float32)).cuda()
    res = prop.forward(w)
    torch.cuda.synchronize()
    return ref, res, prop, w


@pytest.mark.parametrize("scheme", ["const", "vd_staggered", "vd_centred"])
@pytest.mark.parametrize("so", [4, 8])
def test_mirror_3d(scheme, so):
    # every side differs; layers only on some of them
    n = (26, 31, 70)
    nbl = [(0, 4), (3, 0), (0, 0)]
    bc = [("dirichlet", "neumann"), ("neumann", "none"), ("none", "dirichlet")]
    print(f"case: mirror 3D {scheme} SO{so}", flush=True)
    src = np.array([[30.0, 40.0, 650.0]])          # near the mirrored sides
    # receivers inside the grid (the Dirichlet planes z = 0 and y = 690 m hold zero)
    rec = np.array([[20.0, 10.0 * k, 9.0 * k + 4.0] for k in range(30)] + [[250.0, 300.0, 600.0]])
    ref, res, prop, _ = _case(n, so, nbl, bc, scheme, 90, src, rec, 50 + so)
    assert_traces(res.traces, ref.traces)
    assert _rel(prop.grid_view(res.fields[res.current]).cpu().numpy(), ref.p) < 1e-4


@pytest.mark.parametrize("scheme", ["const", "vd_staggered", "vd_centred"])
def test_free_surface_2d(scheme):
    # the paper's examples: a free surface (Dirichlet) on top, layers elsewhere,
    # and an all-Neumann box at SO16
    n = (60, 90)
    print(f"case: free surface 2D {scheme}", flush=True)
    src = np.array([[20.0, 440.0]])
    rec = np.array([[0.0, 300.0]] + [[20.0, 10.0 * k] for k in range(90)])
    ref, res, prop, _ = _case(n, 8, [(0, 10), (10, 10)], [("dirichlet", "none"), ("none", "none")],
                              scheme, 150, src, rec, 61)
    assert np.all(res.traces[:, 0].cpu().numpy() == 0.0)       # a receiver on the held surface
    assert_traces(res.traces[:, 1:], ref.traces[:, 1:])
    assert _rel(prop.grid_view(res.fields[res.current]).cpu().numpy(), ref.p) < 1e-4
    ref, res, prop, _ = _case((40, 50), 16, [(0, 0), (0, 0)], [("neumann", "neumann"), ("neumann", "neumann")],
                              scheme, 120, np.array([[150.0, 210.0]]), np.array([[0.0, 0.0], [390.0, 490.0]]), 62)
    assert_traces(res.traces, ref.traces)
    assert _rel(prop.grid_view(res.fields[res.current]).cpu().numpy(), ref.p) < 1e-4


def test_mirror_tilings_and_graph_bitwise():
    n = (24, 37, 75)
    bc = [("dirichlet", "neumann"), ("neumann", "dirichlet"), ("dirichlet", "neumann")]
    src = np.array([[100.0, 180.0, 370.0]])
    rec = np.array([[20.0, 10.0 * k + 5.0, 7.0 * k + 10.0] for k in range(30)])
    ref, res, prop, w = _case(n, 8, [(0, 0)] * 3, bc, "const", 70, src, rec, 71)
    assert_traces(res.traces, ref.traces)
    u = prop.grid_view(res.fields[res.current]).clone()
    for tiling in [dict(tx=16, nw=8, zc=5), dict(tx=24, nw=8, zc=1), dict(tx=8, nw=8, zc=0, nt=0),
                   dict(tx=8, nw=4, zc=9, occ=4)]:
        print(f"case: mirror tiling {tiling}", flush=True)
        prop.set_tiling(**tiling)
        r = prop.forward(w)
        torch.cuda.synchronize()
        assert torch.equal(r.traces, res.traces)
        assert torch.equal(prop.grid_view(r.fields[r.current]), u)
    prop.set_tiling()
    for _ in range(2):
        g = prop.forward(w, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(g.traces, res.traces)
        assert torch.equal(prop.grid_view(g.fields[g.current]), u)
