"""Graph replay after the plan changes: a cached HIP graph of the forward loop
must not be replayed once the point tables, the model or the tiling it baked
in have changed, even when every buffer address is the same."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2201_05278_amd import Propagator

pytestmark = pytest.mark.gpu


def test_graph_after_geometry_change_matches_eager():
    n = (40, 44, 70)
    h = (10.0,) * 3
    nsteps = 60
    rng = np.random.default_rng(5)
    vel = (2000.0 + 500.0 * rng.random(n)).astype(np.float32)
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(h, 8, float(vel.max()))
    prop = Propagator(n, h, 8, dt, nsteps, nbl=4)
    ext = (np.array(n) - 1) * np.array(h)
    rec_a = np.array([[30.0, 20.0 + 10.0 * k, 40.0 + 9.0 * k] for k in range(20)])
    rec_b = np.array([[50.0 + 3.0 * k, 400.0 - 7.0 * k, 600.0 - 11.0 * k] for k in range(35)])
    prop.set_sources([0.5 * ext], "linear")
    prop.set_receivers(rec_a, "linear")
    v = torch.from_numpy(vel).cuda()
    prop.prepare(v)
    w = torch.from_numpy(oracle.ricker(20.0, dt, nsteps).astype(np.float32)).cuda().reshape(nsteps, 1)
    fields = (prop.new_field(), prop.new_field())
    tbuf = torch.zeros(nsteps * 64, dtype=torch.float32, device="cuda")
    print("case: graph, 20 linear receivers", flush=True)
    r1 = prop.forward(w, use_graph=True, fields=fields, traces=tbuf[: nsteps * 20].view(nsteps, 20))
    torch.cuda.synchronize()
    first = r1.traces.clone()
    # new geometry: more receivers, a windowed-sinc source (more unique nodes)
    prop.set_sources([0.5 * ext + 3.3], "hicks")
    prop.set_receivers(rec_b, "linear")
    prop.prepare(v)
    print("case: graph after set_sources / set_receivers at the same addresses", flush=True)
    tbuf.zero_()
    r2 = prop.forward(w, use_graph=True, fields=fields, traces=tbuf[: nsteps * 35].view(nsteps, 35))
    torch.cuda.synchronize()
    got = r2.traces.clone()
    got_field = prop.grid_view(r2.fields[r2.current]).clone()
    print("case: eager run of the new geometry", flush=True)
    e = prop.forward(w)
    torch.cuda.synchronize()
    assert torch.equal(got, e.traces)
    assert torch.equal(got_field, prop.grid_view(e.fields[e.current]))
    assert not torch.equal(got[:, :20], first)
    # a tiling change and a second prepare with a new model: replay still follows
    prop.set_tiling(8, 4, 9)
    prop.prepare(v * 1.05)
    r3 = prop.forward(w, use_graph=True, fields=fields, traces=tbuf[: nsteps * 35].view(nsteps, 35))
    torch.cuda.synchronize()
    g3 = r3.traces.clone()
    e3 = prop.forward(w)
    torch.cuda.synchronize()
    assert torch.equal(g3, e3.traces)
