"""GPU checks of the two-step sweep (constant density, 3D).

A two-step sweep evaluates the first step on ghost rows and columns around
each tile with exactly the arithmetic of the tile that owns them, and adds
each step's source in the sweep with the arithmetic of the stand-alone
injection, so every level it writes must equal, bit for bit, the level two
single sweeps write.  Checked over all tile shapes, ragged tiles and z chunks,
space orders 2 to 14, multi-node (Kaiser-sinc) sources on tile edges, step
counts that leave single steps over, checkpoints and snapshots at odd steps,
resumption and graph replay; one case goes to the oracle directly, and one
compares the two paths at the full 592^3 benchmark size.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2201_05278_amd import Propagator

pytestmark = pytest.mark.gpu


def _prop(n, so, nsteps, nbl=6, seed=7, src=None, rec=None, interp="hicks"):
    rng = np.random.default_rng(seed)
    vel = workloads.layered(n, [1500.0, 2300.0, 3100.0], rng, 50.0)
    h = (10.0, 10.0, 10.0)
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(h, so, float(vel.max()))
    prop = Propagator(n, h, so, dt, nsteps, nbl=nbl)
    if src is None:
        # near the corner shared by four tiles of the 8-row / (64 - 2R)-column grid
        src = [[10.0 * (n[0] // 2) + 3.3, 10.0 * (8 - nbl) - 4.1, 10.0 * (56 - nbl) + 2.7]]
    if rec is None:
        rec = [[0.0, 10.0 * k + 1.5, 7.0 * k + 3.3] for k in range(30)]
    prop.set_sources(src, interp)
    prop.set_receivers(rec, interp)
    prop.prepare(torch.from_numpy(vel).cuda())
    wav = torch.from_numpy(oracle.ricker(16.0, dt, nsteps)[:, None].astype(np.float32)).cuda()
    return prop, wav, vel, dt


def _run(prop, wav, **kw):
    r = prop.forward(wav, **kw)
    torch.cuda.synchronize()
    return r


def _same(prop, a, b):
    assert torch.equal(a.traces, b.traces)
    assert torch.equal(prop.grid_view(a.fields[a.current]), prop.grid_view(b.fields[b.current]))
    assert torch.equal(prop.grid_view(a.fields[1 - a.current]), prop.grid_view(b.fields[1 - b.current]))


@pytest.mark.parametrize("so", [2, 8, 14])
def test_two_step_equals_single_steps(so):
    n = (45, 61, 123)                      # ragged along every axis for every shape
    nsteps = 47                            # 11 four-step groups + 3 single steps
    prop, wav, _, _ = _prop(n, so, nsteps)
    ref = _run(prop, wav)
    shapes = [(8, 4), (16, 8), (8, 8), (16, 4)]
    r = so // 2
    cases = [(tx, nw, zc, nt) for tx, nw in shapes if (tx // nw) * (5 * r + 5) +
             ((2 * r + nw - 1) // nw) * (3 * r + 3) <= 95 for zc, nt in ((0, 1), (13, 0), (30, 1))]
    assert cases
    for tx, nw, zc, nt in cases:
        print(f"case: two-step SO{so} tiling {tx}x{nw} zc={zc} nt={nt}", flush=True)
        prop.set_tiling(tx, nw, zc, nt, ts=2)
        assert prop.tiling["ts"] == 2
        _same(prop, _run(prop, wav), ref)
    prop.set_tiling()


def test_two_step_outputs_resume_graph():
    n = (40, 50, 70)
    nsteps = 61
    prop, wav, _, _ = _prop(n, 8, nsteps, seed=11)
    ref = _run(prop, wav, saving_stride=7, checkpoint_every=9)
    prop.set_tiling(ts=2)
    print("case: two-step snapshots (stride 7), checkpoints (every 9)", flush=True)
    two = _run(prop, wav, saving_stride=7, checkpoint_every=9)
    _same(prop, two, ref)
    assert torch.equal(two.snaps, ref.snaps)
    for k in range(ref.ckpt.shape[0]):
        assert torch.equal(prop.grid_view(two.ckpt[k, 0]), prop.grid_view(ref.ckpt[k, 0])), k
        assert torch.equal(prop.grid_view(two.ckpt[k, 1]), prop.grid_view(ref.ckpt[k, 1])), k
    print("case: two-step resume at step 21 and graph replay", flush=True)
    f = (prop.new_field(), prop.new_field())
    a = _run(prop, wav, fields=f, step0=0, nsteps_run=21)
    nxt = (f[a.current], f[1 - a.current])
    b = _run(prop, wav, fields=nxt, step0=21, nsteps_run=nsteps - 21, traces=a.traces)
    assert torch.equal(b.traces, ref.traces)
    assert torch.equal(prop.grid_view(nxt[b.current]), prop.grid_view(ref.fields[ref.current]))
    g = _run(prop, wav, use_graph=True)
    g2 = _run(prop, wav, use_graph=True, fields=g.fields, traces=g.traces)
    _same(prop, g, ref)
    _same(prop, g2, ref)
    ms = np.zeros(nsteps, dtype=np.float32)
    t = _run(prop, wav, stencil_ms=ms)
    _same(prop, t, ref)
    assert np.all(ms > 0)
    assert np.all(ms[:60:2] == ms[1:60:2])   # a sweep's time is split over its two steps
    prop.set_tiling()


def test_two_step_many_sources_against_oracle():
    # several Kaiser-sinc sources (overlapping footprints, on tile edges) and
    # linear receivers, checked against the oracle directly
    n = (38, 52, 60)
    so = 8
    nsteps = 90
    src = [[150.0, 13.0, 497.0], [153.1, 17.5, 501.2], [60.0, 300.0, 100.0]]
    rec = [[5.0, 10.0 * k + 2.0, 11.0 * k + 1.0] for k in range(25)]
    prop, _, vel, dt = _prop(n, so, nsteps, nbl=5, seed=13, src=src, rec=rec)
    wavelet = np.stack([oracle.ricker(f, dt, nsteps) for f in (14.0, 17.0, 21.0)], axis=1)
    prop.set_tiling(ts=2)
    print("case: two-step 3 sources vs oracle", flush=True)
    res = _run(prop, torch.from_numpy(wavelet.astype(np.float32)).cuda())
    prob = oracle.Problem(n=n, h=(10.0,) * 3, space_order=so, dt=dt, nsteps=nsteps, nbl=((5, 5),) * 3)
    st = oracle.prepare(prob, vel.astype(np.float64))
    ref = oracle.forward(st, wavelet, oracle.geometry_table(prob, src, "hicks"),
                         oracle.geometry_table(prob, rec, "hicks"), len(rec))
    got = res.traces.double().cpu().numpy()
    assert np.linalg.norm(got - ref.traces) <= 1e-4 * np.linalg.norm(ref.traces)
    u = prop.grid_view(res.fields[res.current]).double().cpu().numpy()
    assert np.linalg.norm(u - ref.p) <= 1e-4 * np.linalg.norm(ref.p)
    prop.set_tiling()


def test_two_step_full_size_equals_single_steps():
    # the benchmark grid (512^3 + 40-cell layer = 592^3), default two-step tiling
    wl = workloads.smooth_3d(n=512, nsteps=8)
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(wl.h, wl.space_order, wl.cmax)
    prop = Propagator(wl.n, wl.h, wl.space_order, dt, wl.nsteps, nbl=wl.nbl)
    prop.set_sources(wl.src, wl.src_interp)
    prop.set_receivers(wl.rec, wl.rec_interp)
    prop.prepare(torch.from_numpy(wl.vel).cuda(), cmax=wl.cmax)
    wav = torch.from_numpy(oracle.ricker(wl.f_peak, dt, wl.nsteps)[:, None].astype(np.float32)).cuda()
    print("case: two-step vs single steps at 592^3, 8 steps", flush=True)
    prop.set_tiling(ts=1)
    ref = _run(prop, wav)
    tr = ref.traces.clone()
    u = prop.grid_view(ref.fields[ref.current]).clone()
    del ref
    prop.set_tiling(ts=2)
    two = _run(prop, wav)
    assert torch.equal(two.traces, tr)
    assert torch.equal(prop.grid_view(two.fields[two.current]), u)
    prop.set_tiling()
