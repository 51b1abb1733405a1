"""GPU adjoint: dot-product test, gradient against the FP64 oracle and
against finite differences, and the autograd wrapper."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2201_05278_amd import Propagator, AcousticForward

pytestmark = pytest.mark.gpu


def _setup(n=(30, 34, 66), nbl=6, so=8, nsteps=120, seed=3, interp="hicks"):
    rng = np.random.default_rng(seed)
    vel = workloads.layered(n, [1700.0, 2300.0, 2800.0], rng, 40.0)
    h = (10.0,) * 3
    dt = 0.5 * oracle.coeffs.critical_dt(h, so, float(vel.max()))
    src = np.array([[41.3, 170.2, 250.7], [150.0, 100.0, 400.0]])
    rec = np.array([[10.0 + 3.0 * k, 12.0 * k + 5.0, 9.0 * k + 7.0] for k in range(25)])
    prop = Propagator(n, h, so, dt, nsteps, nbl=nbl)
    prop.set_sources(src, interp)
    prop.set_receivers(rec, interp)
    return prop, vel, src, rec, dt, rng


def test_dot_product():
    prop, vel, src, rec, dt, rng = _setup()
    print("case: adjoint dot product", flush=True)
    prop.prepare(torch.from_numpy(vel).cuda())
    s = torch.from_numpy(rng.standard_normal((prop.nsteps, 2)).astype(np.float32)).cuda()
    r = torch.from_numpy(rng.standard_normal((prop.nsteps, 25)).astype(np.float32)).cuda()
    fw = prop.forward(s, checkpoint_every=16)
    _, FTr, _ = prop.adjoint(s, r, fw.ckpt, 16, want_src_adjoint=True)
    torch.cuda.synchronize()
    lhs = float((fw.traces.double() * r.double()).sum())
    rhs = float((s.double() * FTr.double()).sum())
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), abs(rhs)), (lhs, rhs)


@pytest.mark.parametrize("every", [16, 120, 1])
def test_gradient_matches_oracle(every):
    prop, vel, src, rec, dt, rng = _setup()
    print(f"case: gradient vs oracle, checkpoint every {every}", flush=True)
    n, nsteps = prop.n, prop.nsteps
    wav = np.stack([oracle.ricker(15.0, dt, nsteps)] * 2, axis=1)
    d_obs = 0.5 * rng.standard_normal((nsteps, 25)) * 1e-4
    prob = oracle.Problem(n=n, h=(10.0,) * 3, space_order=8, dt=dt, nsteps=nsteps,
                          nbl=((6, 6),) * 3)
    st = oracle.prepare(prob, vel.astype(np.float64))
    src_t, rec_t = oracle.geometry_table(prob, src), oracle.geometry_table(prob, rec)
    fw_ref = oracle.forward(st, wav, src_t, rec_t, 25, keep_history=True)
    _, gc_ref, _ = oracle.gradient(st, rec_t, fw_ref.traces - d_obs, fw_ref.history)

    prop.prepare(torch.from_numpy(vel).cuda())
    wt = torch.from_numpy(wav.astype(np.float32)).cuda()
    fw = prop.forward(wt, checkpoint_every=every)
    resid = fw.traces - torch.from_numpy(d_obs.astype(np.float32)).cuda()
    g, _, _ = prop.adjoint(wt, resid, fw.ckpt, every)
    torch.cuda.synchronize()
    err = np.linalg.norm(g.double().cpu().numpy() - gc_ref) / np.linalg.norm(gc_ref)
    assert err < 1e-3, err


def test_autograd_matches_adjoint_and_finite_difference():
    prop, vel, src, rec, dt, rng = _setup(nsteps=100)
    print("case: autograd + finite differences", flush=True)
    nsteps = prop.nsteps
    wav = torch.from_numpy(np.stack([oracle.ricker(15.0, dt, nsteps)] * 2, axis=1).astype(np.float32)).cuda()
    v_true = torch.from_numpy(vel).cuda()
    with torch.no_grad():
        d_obs = AcousticForward.apply(v_true * 1.02, prop, wav, 20).detach().clone()
    v = v_true.clone().requires_grad_(True)
    tr = AcousticForward.apply(v, prop, wav, 20)
    loss = 0.5 * ((tr.double() - d_obs.double()) ** 2).sum()
    loss.backward()
    g = v.grad.double()
    # central difference of the FP32 misfit along a smooth direction
    dv = torch.from_numpy(workloads.smooth_random(prop.n, 9, factor=4, vmin=-1.0, vmax=1.0)).cuda()
    eps = 2.0
    with torch.no_grad():
        jp = 0.5 * ((AcousticForward.apply(v_true + eps * dv, prop, wav, 20).double() - d_obs.double()) ** 2).sum()
        jm = 0.5 * ((AcousticForward.apply(v_true - eps * dv, prop, wav, 20).double() - d_obs.double()) ** 2).sum()
    fd = float((jp - jm) / (2 * eps))
    an = float((g * dv.double()).sum())
    assert abs(fd - an) <= 1e-2 * abs(an), (fd, an)


def test_gradient_bitwise_over_checkpoint_intervals():
    # checkpointing and the pairing of imaging steps keep the gradient
    # accumulation in step order: the same bits for segments of 1 (nothing
    # paired), odd and even lengths, and one segment
    prop, vel, src, rec, dt, rng = _setup(nsteps=57, seed=9)
    prop.prepare(torch.from_numpy(vel).cuda())
    s = torch.from_numpy(rng.standard_normal((prop.nsteps, 2)).astype(np.float32)).cuda()
    r = torch.from_numpy(rng.standard_normal((prop.nsteps, 25)).astype(np.float32)).cuda()
    grads = {}
    for every in (1, 2, 7, 16, 57):
        print(f"case: gradient, checkpoints every {every}", flush=True)
        fw = prop.forward(s, checkpoint_every=every)
        g, _, _ = prop.adjoint(s, r, fw.ckpt, every)
        torch.cuda.synchronize()
        grads[every] = g.clone()
    for every in (2, 7, 16, 57):
        assert torch.equal(grads[every], grads[1]), every
