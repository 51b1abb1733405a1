"""GPU parity of the variable-density propagators (staggered conservative and
centred) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from tests._parity import assert_traces
import workloads
from paper_2201_05278_amd import Propagator
from tests.test_gpu_forward import run_pair, rel, field_np, TOL

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scheme", ["vd_staggered", "vd_centred"])
@pytest.mark.parametrize("so", [2, 4, 8])
def test_vd_3d_ragged(scheme, so):
    n = (35, 41, 70)
    print(f"case: {scheme} 3D {n} SO{so}", flush=True)
    rng = np.random.default_rng(40 + so)
    vel = workloads.layered(n, [1500.0, 2300.0, 3100.0], rng, 40.0)
    rho = (workloads.gardner(vel) * (1.0 + 0.3 * workloads.smooth_random(n, 7, factor=4,
                                                                         vmin=-1.0, vmax=1.0)))
    rho = rho.astype(np.float32)
    h = (10.0, 10.0, 10.0)
    src = np.array([[121.3, 203.7, 330.2]])
    rec = np.array([[5.0 * k, 10.0 * k, 6.0 * k + 2.2] for k in range(35)])
    ref, res, prop, _ = run_pair(n, h, so, 7, 130, vel, src, rec, f=18.0, scheme=scheme, rho=rho)
    assert_traces(res.traces, ref.traces)
    assert rel(field_np(prop, res), ref.p) < TOL


@pytest.mark.parametrize("scheme", ["vd_staggered", "vd_centred"])
@pytest.mark.parametrize("so", [4, 16, 18, 20])
def test_vd_2d(scheme, so):
    n = (70, 150)
    print(f"case: {scheme} 2D {n} SO{so}", flush=True)
    vel = workloads.smooth_random(n, 12, factor=8)
    rho = workloads.gardner(vel)
    h = (8.0, 10.0)
    src = np.array([[201.1, 733.3]])
    rec = np.array([[20.0, 10.0 * k] for k in range(0, 149, 3)])
    ref, res, prop, _ = run_pair(n, h, so, ((12, 20), (18, 9)), 220, vel, src, rec, f=15.0,
                                 scheme=scheme, rho=rho)
    assert_traces(res.traces, ref.traces)


@pytest.mark.parametrize("scheme", ["vd_staggered", "vd_centred"])
def test_vd_smooth_gardner_trilinear(scheme):
    # the variable-density configuration's recipe at a reduced size
    wl = workloads.smooth_3d(n=56, nsteps=150, scheme="vd_staggered", nrec_side=16,
                             rec_spacing=30.0)
    print(f"case: {scheme} smooth_3d {wl.n}", flush=True)
    ref, res, prop, _ = run_pair(wl.n, wl.h, 8, 10, wl.nsteps, wl.vel, wl.src, wl.rec,
                                 "linear", "linear", f=wl.f_peak, scheme=scheme, rho=wl.rho)
    assert_traces(res.traces, ref.traces)


def test_vd_density_scale_invariance():
    n = (30, 33, 66)
    vel = workloads.layered(n, [1800.0, 2600.0], np.random.default_rng(1), 30.0)
    rho = workloads.gardner(vel)
    h = (10.0,) * 3
    src = np.array([[100.0, 160.0, 320.0]])
    rec = np.array([[20.0, 10.0 * k, 300.0] for k in range(30)])
    _, r1, _, _ = run_pair(n, h, 8, 5, 80, vel, src, rec, scheme="vd_staggered", rho=rho)
    _, r2, _, _ = run_pair(n, h, 8, 5, 80, vel, src, rec, scheme="vd_staggered",
                           rho=(rho * 1000.0).astype(np.float32))
    assert rel(r2.traces.cpu().numpy(), r1.traces.cpu().numpy()) < 1e-5


@pytest.mark.parametrize("scheme", ["vd_staggered", "vd_centred"])
def test_vd_tilings_are_bitwise_identical(scheme):
    # the per-node (and per-face) arithmetic does not depend on the tile shape,
    # chunk length or cache policy
    n = (30, 37, 70)
    rng = np.random.default_rng(41)
    vel = workloads.layered(n, [1500.0, 2500.0, 3500.0], rng, 40.0)
    rho = workloads.gardner(vel)
    h = (10.0,) * 3
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(h, 8, float(vel.max()))
    prop = Propagator(n, h, 8, dt, 50, scheme=scheme, nbl=5)
    prop.set_sources([[150.0, 183.0, 344.0]])
    prop.set_receivers([[0.0, 10.0 * k + 3.0, 8.0 * k] for k in range(30)])
    prop.prepare(torch.from_numpy(vel).cuda(), torch.from_numpy(rho).cuda())
    wav = torch.from_numpy(oracle.ricker(15.0, dt, 50)[:, None].astype(np.float32)).cuda()
    ref = prop.forward(wav)
    torch.cuda.synchronize()
    u_ref = prop.grid_view(ref.fields[ref.current]).clone()
    tr_ref = ref.traces.clone()
    for tx, nw, zc, nt, occ in [(8, 8, 0, 1, 0), (16, 8, 7, 0, 0), (8, 4, 13, 1, 0), (16, 4, 25, 0, 0),
                                (8, 4, 1, 0, 0), (8, 4, 9, 1, 5), (16, 4, 0, 1, 3)]:
        print(f"case: {scheme} tiling {tx}x{nw} zc={zc} nt={nt} occ={occ}", flush=True)
        prop.set_tiling(tx, nw, zc, nt, occ=occ)
        r = prop.forward(wav)
        torch.cuda.synchronize()
        assert torch.equal(r.traces, tr_ref)
        assert torch.equal(prop.grid_view(r.fields[r.current]), u_ref)
    prop.set_tiling()
