"""Full-size parity in the launch configuration the benchmark times.

At the full grid sizes the oracle cannot run whole simulations, so one step is
checked: both sides start from the same seeded random levels p^k, p^{k-1}
(every node non-zero, so every tile, halo and layer node is exercised); the
GPU advances one step with its default tiling (stencil, injection,
recording), and the oracle evaluates its own update node by node at sampled
nodes (random nodes, every layer corner and edge box, the source footprint,
every receiver footprint), adds its injection and forms the traces.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2201_05278_amd import Propagator

pytestmark = pytest.mark.gpu

STEP = 3


@pytest.fixture(scope="module")
def smooth512():
    return workloads.smooth_3d(n=512, nsteps=8, scheme="vd_staggered")


def _boxes(N, width=6):
    """Flat indices of small boxes at the 8 corners and the centre of the grid."""
    out = []
    for cz in (0, N[0] // 2, N[0] - width):
        for cx in (0, N[1] - width):
            for cy in (0, N[2] // 2, N[2] - width):
                z, x, y = np.meshgrid(np.arange(cz, cz + width), np.arange(cx, cx + width),
                                      np.arange(cy, cy + width), indexing="ij")
                out.append(((z * N[1] + x) * N[2] + y).ravel())
    return np.concatenate(out)


def _one_step_parity(wl, scheme, so=None):
    so = so or wl.space_order
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(wl.h, so, wl.cmax)
    nsteps = wl.nsteps
    nbl = wl.nbl
    prop = Propagator(wl.n, wl.h, so, dt, nsteps, scheme=scheme, nbl=nbl)
    prop.set_sources(wl.src, wl.src_interp)
    prop.set_receivers(wl.rec, wl.rec_interp)
    rho = None if scheme == "const" else wl.rho
    prop.prepare(torch.from_numpy(wl.vel).cuda(), None if rho is None else torch.from_numpy(rho).cuda(),
                 cmax=wl.cmax)
    dims = prop.grid_shape
    print(f"case: full-size one step, {scheme} SO{so} grid {dims}", flush=True)
    rng = np.random.default_rng(1234)
    p = rng.standard_normal(dims, dtype=np.float32)
    prev = rng.standard_normal(dims, dtype=np.float32)
    f0, f1 = prop.new_field(), prop.new_field()
    prop.grid_view(f0).copy_(torch.from_numpy(p))
    prop.grid_view(f1).copy_(torch.from_numpy(prev))
    wav = oracle.ricker(wl.f_peak, dt, nsteps)[:, None]
    traces = torch.zeros((nsteps, len(wl.rec)), dtype=torch.float32, device="cuda")
    res = prop.forward(torch.from_numpy(wav.astype(np.float32)).cuda(), fields=(f0, f1), step0=STEP,
                       nsteps_run=1, traces=traces)
    torch.cuda.synchronize()
    got = prop.grid_view(res.fields[res.current]).cpu().numpy().ravel()
    got_tr = traces[STEP].double().cpu().numpy()
    del f0, f1, res
    torch.cuda.empty_cache()

    prob = oracle.Problem(n=wl.n, h=wl.h, space_order=so, dt=dt, nsteps=nsteps, scheme=scheme,
                          nbl=((nbl, nbl),) * 3)
    st = oracle.prepare(prob, wl.vel.astype(np.float64), None if rho is None else rho.astype(np.float64))
    src_t = oracle.geometry_table(prob, wl.src, wl.src_interp)
    rec_t = oracle.geometry_table(prob, wl.rec, wl.rec_interp)
    N = prob.N
    idx = np.unique(np.concatenate([rng.integers(0, int(np.prod(N)), 200000), _boxes(N),
                                    src_t[0], rec_t[0]]))
    p64, prev64 = p.astype(np.float64), prev.astype(np.float64)
    vals = oracle.step_points(st, p64, prev64, idx)
    inj_nodes, inj_vals = oracle.injection_terms(st, src_t, wav[STEP].astype(np.float64))
    pos = np.searchsorted(idx, inj_nodes)
    vals[pos] += inj_vals
    err = np.abs(got[idx] - vals)
    scale = np.max(np.abs(vals))
    assert np.max(err) <= 2e-6 * scale, (np.max(err), scale)
    assert np.linalg.norm(got[idx] - vals) <= 1e-6 * np.linalg.norm(vals)
    # traces of the step: receiver weights on the oracle's updated values
    lookup = dict(zip(idx.tolist(), vals.tolist()))
    ref_tr = np.zeros(len(wl.rec))
    np.add.at(ref_tr, rec_t[1], rec_t[2] * np.array([lookup[k] for k in rec_t[0].tolist()]))
    assert np.linalg.norm(got_tr - ref_tr) <= 1e-5 * np.linalg.norm(ref_tr)


def test_smooth_512_constant_density(smooth512):
    _one_step_parity(smooth512, "const")


def test_smooth_512_staggered(smooth512):
    _one_step_parity(smooth512, "vd_staggered")


def test_smooth_512_centred(smooth512):
    _one_step_parity(smooth512, "vd_centred")


def test_layered_256_so16():
    _one_step_parity(workloads.layered_3d(n=256, nsteps=8), "const")


def _fullsize_prop(wl, scheme, nsteps):
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(wl.h, wl.space_order, wl.cmax)
    prop = Propagator(wl.n, wl.h, wl.space_order, dt, nsteps, scheme=scheme, nbl=wl.nbl)
    prop.set_sources(wl.src, wl.src_interp)
    prop.set_receivers(wl.rec, wl.rec_interp)
    return prop, dt


@pytest.mark.parametrize("scheme", ["const", "vd_staggered"])
def test_smooth_512_adjoint_dot_product(smooth512, scheme):
    # <F s, r> = <s, F^T r> at the benchmark size, default tiling, partial
    # checkpoint segment: a property of the adjoint that holds at any size
    wl = smooth512
    nsteps, every = 30, 12
    prop, dt = _fullsize_prop(wl, scheme, nsteps)
    rho = None if scheme == "const" else torch.from_numpy(wl.rho).cuda()
    prop.prepare(torch.from_numpy(wl.vel).cuda(), rho, cmax=wl.cmax)
    print(f"case: full-size adjoint dot product, {scheme}", flush=True)
    rng = np.random.default_rng(5)
    s = torch.from_numpy(rng.standard_normal((nsteps, 1)).astype(np.float32)).cuda()
    r = torch.from_numpy(rng.standard_normal((nsteps, len(wl.rec))).astype(np.float32)).cuda()
    fw = prop.forward(s, checkpoint_every=every)
    out = prop.adjoint(s, r, fw.ckpt, every, want_src_adjoint=True)
    torch.cuda.synchronize()
    lhs = float((fw.traces.double() * r.double()).sum())
    rhs = float((s.double() * out[1].double()).sum())
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), abs(rhs)), (lhs, rhs)


def test_smooth_512_vd_gradients_match_finite_differences(smooth512):
    # directional derivatives of the FP32 misfit against the velocity and the
    # density gradients at the benchmark size (smooth directions)
    wl = smooth512
    nsteps, every = 40, 16
    prop, dt = _fullsize_prop(wl, "vd_staggered", nsteps)
    vel = torch.from_numpy(wl.vel).cuda()
    rho = torch.from_numpy(wl.rho).cuda()
    wav = torch.from_numpy(oracle.ricker(25.0, dt, nsteps, t0=12 * dt)[:, None].astype(np.float32)).cuda()
    n = wl.n
    axes = [torch.sin(torch.pi * (torch.arange(k, device="cuda", dtype=torch.float32) + 0.5) / k) for k in n]
    bump = axes[0][:, None, None] * axes[1][None, :, None] * axes[2][None, None, :]

    def traces(v, r_):
        prop.prepare(v, r_, cmax=wl.cmax * 1.05)
        t = prop.forward(wav).traces.clone()
        torch.cuda.synchronize()
        return t

    print("case: full-size VD gradients vs finite differences", flush=True)
    d_obs = traces(vel * (1.0 + 0.03 * bump), rho * (1.0 - 0.05 * bump))
    prop.prepare(vel, rho, cmax=wl.cmax * 1.05)
    fw = prop.forward(wav, checkpoint_every=every)
    gv, _, _, gr = prop.adjoint(wav, fw.traces - d_obs, fw.ckpt, every)
    torch.cuda.synchronize()

    def misfit(v, r_):
        return 0.5 * float(((traces(v, r_).double() - d_obs.double()) ** 2).sum())

    for name, g, base in (("vel", gv, vel), ("rho", gr, rho)):
        eps = 2e-3 * float(base.mean())
        d = bump
        if name == "vel":
            fd = (misfit(vel + eps * d, rho) - misfit(vel - eps * d, rho)) / (2 * eps)
        else:
            fd = (misfit(vel, rho + eps * d) - misfit(vel, rho - eps * d)) / (2 * eps)
        an = float((g.double() * d.double()).sum())
        assert abs(fd - an) <= 2e-2 * abs(an), (name, fd, an)
