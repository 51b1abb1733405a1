"""The paper's benchmark shapes ("Performance evaluation": the 421 x 1841 2D
grid and the 207 x 801 x 801 3D grid) with the boundary set-up of its two
examples (Neumann top, Dirichlet elsewhere; in 2D a 70-cell layer on the
bottom and the sides), at dt = dt_crit as its step counts imply: single and
double precision against the FP64 oracle over a reduced number of steps
(300 in 2D, 12 in 3D), traces within 1e-4 (single) and 1e-10 (double)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2201_05278_amd import Propagator
from tests._parity import assert_traces, trace_errors

pytestmark = pytest.mark.gpu


def _oracle(wl, dt, nsteps, f_peak=None, t0=None):
    prob = oracle.Problem(n=wl.n, h=wl.h, space_order=wl.space_order, dt=dt, nsteps=nsteps,
                          nbl=wl.nbl, bc=wl.bc)
    st = oracle.prepare(prob, wl.vel.astype(np.float64))
    wav = oracle.ricker(f_peak or wl.f_peak, dt, nsteps, t0)[:, None]
    return oracle.forward(st, wav, oracle.geometry_table(prob, wl.src, wl.src_interp, role="source"),
                          oracle.geometry_table(prob, wl.rec, wl.rec_interp, role="receiver"), len(wl.rec)), wav


def _gpu(wl, dt, nsteps, wav, dtype):
    prop = Propagator(wl.n, wl.h, wl.space_order, dt, nsteps, nbl=[list(p) for p in wl.nbl],
                      bc=[list(b) for b in wl.bc], dtype=dtype)
    prop.set_sources(wl.src, wl.src_interp)
    prop.set_receivers(wl.rec, wl.rec_interp)
    tdt = torch.float64 if dtype == "float64" else torch.float32
    prop.prepare(torch.from_numpy(wl.vel.astype(np.float64)).to(tdt).cuda(), cmax=wl.extra["cmax"])
    res = prop.forward(torch.from_numpy(wav).to(tdt).cuda())
    torch.cuda.synchronize()
    return res.traces


@pytest.mark.parametrize("so", [2, 4, 8])
def test_paper_shape_2d(so):
    wl = workloads.paper_shape_2d(space_order=so)
    dt = oracle.coeffs.critical_dt(wl.h, so, wl.extra["cmax"])
    nsteps = 300
    print(f"case: paper shape 2D SO{so}, {nsteps} steps at dt_crit", flush=True)
    ref, wav = _oracle(wl, dt, nsteps)
    assert_traces(_gpu(wl, dt, nsteps, wav, "float32"), ref.traces)
    total, worst, _ = trace_errors(_gpu(wl, dt, nsteps, wav, "float64"), ref.traces)
    assert total < 1e-10 and worst < 1e-10, (total, worst)


def test_paper_shape_3d():
    wl = workloads.paper_shape_3d(space_order=8)
    dt = oracle.coeffs.critical_dt(wl.h, 8, wl.extra["cmax"])
    nsteps = 12
    print(f"case: paper shape 3D SO8, {nsteps} steps at dt_crit", flush=True)
    # a 25 Hz wavelet peaking at 8 ms, so that the 12 steps carry its main lobe
    ref, wav = _oracle(wl, dt, nsteps, 25.0, 0.008)
    near = np.argsort(np.abs(wl.rec[:, 1] - wl.src[0, 1]))[:11]     # receivers the wave reaches
    t32 = _gpu(wl, dt, nsteps, wav, "float32")[:, torch.from_numpy(near).cuda()]
    assert_traces(t32, ref.traces[:, near])
    t64 = _gpu(wl, dt, nsteps, wav, "float64")[:, torch.from_numpy(near).cuda()]
    total, worst, _ = trace_errors(t64, ref.traces[:, near])
    assert total < 1e-10 and worst < 1e-10, (total, worst)
