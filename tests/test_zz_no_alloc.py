"""The batched forward's no-allocation variant (sw_batch_forward_static):
the same run as sw_batch_forward with the descriptor table in the library's
own fixed device array instead of a caller-allocated one.  Two calls in a
row, the second with a smaller batch (fewer shots, fewer steps), each
compared bit for bit with the allocating entry point on the same shots."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2201_05278_amd import Propagator, Batch
from paper_2201_05278_amd import _lib as L

pytestmark = pytest.mark.gpu


def _shots(nshots, nsteps, seed):
    shots = workloads.batch_3d(nshots=nshots, nsteps=nsteps, nrec_side=5, size_scale=0.2, seed=seed)
    props, wavs = [], []
    for wl in shots:
        dt = 0.5 * oracle.coeffs.critical_dt(wl.h, wl.space_order, wl.cmax)
        p = Propagator(wl.n, wl.h, wl.space_order, dt, wl.nsteps, nbl=6)
        p.set_sources(wl.src)
        p.set_receivers(wl.rec)
        p.prepare(torch.from_numpy(wl.vel).cuda())
        props.append(p)
        wavs.append(torch.from_numpy(oracle.ricker(wl.f_peak, dt, nsteps)[:, None].astype(np.float32)).cuda())
    return props, wavs


def _check(nshots, nsteps, seed):
    props, wavs = _shots(nshots, nsteps, seed)
    batch = Batch(props)
    print(f"case: allocating batch, {nshots} shots, {nsteps} steps", flush=True)
    ref = [t.clone() for t in batch.forward(wavs)]
    ref_fields = [p.grid_view(batch.fields[k][batch.current]).clone() for k, p in enumerate(props)]
    for t in batch.traces:
        t.fill_(123.0)
    for f in batch.fields:
        f[0].fill_(7.0)
        f[1].fill_(7.0)
    print(f"case: static-table batch, {nshots} shots, {nsteps} steps", flush=True)
    got = batch.forward_static(wavs)
    torch.cuda.synchronize()
    for k, p in enumerate(props):
        assert torch.equal(got[k], ref[k]), k
        assert torch.equal(p.grid_view(batch.fields[k][batch.current]), ref_fields[k]), k


def test_static_table_batch_matches_allocating_batch_twice():
    # two calls in a row on the shared array, the second with a smaller batch
    # (fewer shots, fewer steps): the array keeps the first call's larger table
    _check(5, 60, 4)
    _check(2, 35, 9)


def test_static_table_refuses_graphs():
    props, wavs = _shots(2, 10, 4)
    batch = Batch(props)
    io = batch._io(wavs, 10, True)
    st = L.lib().sw_batch_forward_static(batch._batch, ctypes.byref(io), None)
    assert L.STATUS[st] == "SW_ERR_ARG"
    assert b"graph" in L.lib().sw_last_error()
