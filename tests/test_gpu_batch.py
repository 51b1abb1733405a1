"""GPU checks of tiling invariance, batched shots and the autotuner.

The per-node arithmetic of the stencil does not depend on the tile shape,
z-chunk length, cache policy or on whether the grid is advanced alone or in a
batch, so all of these must agree bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2201_05278_amd import Propagator, Batch

pytestmark = pytest.mark.gpu


def _shot_prop(wl, nbl=6):
    dt = 0.5 * oracle.coeffs.critical_dt(wl.h, wl.space_order, wl.cmax)
    prop = Propagator(wl.n, wl.h, wl.space_order, dt, wl.nsteps, nbl=nbl)
    prop.set_sources(wl.src)
    prop.set_receivers(wl.rec)
    prop.prepare(torch.from_numpy(wl.vel).cuda())
    wav = torch.from_numpy(oracle.ricker(wl.f_peak, dt, wl.nsteps)[:, None].astype(np.float32)).cuda()
    return prop, wav


def test_tilings_are_bitwise_identical():
    wl = workloads.layered_3d(n=44, nsteps=60, space_order=8, nrec_side=8, rec_stride=5)
    prop, wav = _shot_prop(wl)
    ref = prop.forward(wav)
    torch.cuda.synchronize()
    u_ref = prop.grid_view(ref.fields[ref.current]).clone()
    tr_ref = ref.traces.clone()
    for tx, nw, zc, nt, pf, wt, occ in [(8, 4, 0, 0, 1, 0, 0), (32, 8, 13, 1, 2, 0, 0), (16, 8, 100, 1, 1, 0, 0),
                                        (16, 4, 9, 0, 2, 0, 0), (8, 8, 20, 1, 2, 0, 0), (16, 4, 17, 1, 0, 1, -1),
                                        (4, 1, 0, 0, 0, 1, -1), (8, 1, 31, 1, 0, 1, -1), (24, 8, 11, 1, 1, 0, 0),
                                        (24, 8, 0, 0, 2, 0, 0), (8, 4, 5, 1, 1, 0, 4), (16, 4, 0, 1, 2, 0, 3),
                                        (8, 8, 7, 0, 1, 0, 6), (24, 8, 3, 1, 1, 0, 3)]:
        print(f"case: tiling {tx}x{nw} zc={zc} nt={nt} pf={pf} wave={wt} occ={occ}", flush=True)
        prop.set_tiling(tx, nw, zc, nt, pf, wt, occ=occ)
        r = prop.forward(wav)
        torch.cuda.synchronize()
        assert torch.equal(r.traces, tr_ref)
        assert torch.equal(prop.grid_view(r.fields[r.current]), u_ref)


def test_batch_matches_single_shots_bitwise():
    shots = workloads.batch_3d(nshots=5, nsteps=70, nrec_side=6, size_scale=0.2)
    props, wavs = zip(*[_shot_prop(wl) for wl in shots])
    single = []
    for p, w in zip(props, wavs):
        r = p.forward(w)
        torch.cuda.synchronize()
        single.append((r.traces.clone(), p.grid_view(r.fields[r.current]).clone()))
    batch = Batch(props)
    for use_graph in (False, True, True):
        print(f"case: batch of {len(props)} shots, graph={use_graph}", flush=True)
        traces = batch.forward(wavs, use_graph=use_graph)
        torch.cuda.synchronize()
        for k, p in enumerate(props):
            assert torch.equal(traces[k], single[k][0]), k
            assert torch.equal(p.grid_view(batch.fields[k][batch.current]), single[k][1]), k
    # tilings and grids of the batch launch: one block per tile, a small
    # persistent grid (many tiles per block) and the default
    for cfg in [(24, 8, 11, 1, 1, -1), (8, 4, 0, 0, 2, 1), (16, 8, 7, 1, 1, 3), (32, 8, 100, 0, 1, -1),
                (0, 0, 0, 1, 1, 0)]:
        print(f"case: batch tiling {cfg}", flush=True)
        batch.set_tiling(*cfg)
        got = batch.tiling
        if cfg[0]:
            assert (got["tx"], got["nw"], got["blocks_per_cu"]) == (cfg[0], cfg[1], cfg[5])
        for use_graph in (False, True):
            traces = batch.forward(wavs, use_graph=use_graph)
            torch.cuda.synchronize()
            for k, p in enumerate(props):
                assert torch.equal(traces[k], single[k][0]), k
                assert torch.equal(p.grid_view(batch.fields[k][batch.current]), single[k][1]), k


def test_autotune_keeps_results_and_uses_cache(tmp_path):
    wl = workloads.layered_3d(n=40, nsteps=40, space_order=4, nrec_side=6, rec_stride=6)
    prop, wav = _shot_prop(wl)
    ref = prop.forward(wav)
    torch.cuda.synchronize()
    tr_ref = ref.traces.clone()
    cache = str(tmp_path / "tune.json")
    prop.autotune(cache)
    tuned = prop.forward(wav)
    torch.cuda.synchronize()
    assert torch.equal(tuned.traces, tr_ref)
    text = open(cache).read()
    assert "plan_s0_r2_d3" in text
    prop.set_tiling()            # back to defaults, then read the choice from the cache
    assert prop.tiling["tx"] > 0
    prop.autotune(cache)
    again = prop.forward(wav)
    torch.cuda.synchronize()
    assert torch.equal(again.traces, tr_ref)

    shots = workloads.batch_3d(nshots=3, nsteps=30, nrec_side=4, size_scale=0.15)
    props, wavs = zip(*[_shot_prop(w) for w in shots])
    singles = []
    for p, w in zip(props, wavs):
        r = p.forward(w)
        torch.cuda.synchronize()
        singles.append(r.traces.clone())
    batch = Batch(props)
    batch.autotune(wavs, cache)
    out = batch.forward(wavs)
    torch.cuda.synchronize()
    for k in range(len(props)):
        assert torch.equal(out[k], singles[k])
    assert "batch_r4_d3_n3" in open(cache).read()
