"""Stored oracle outputs of the full-size, full-length parity tests.

Writes tests/golden/fullsize_<case>.npz: the FP64 oracle's receiver traces
(or velocity-gradient samples) for the benchmark configurations at their full
grid sizes and step counts.  Only the oracle and the seeded input generators
(workloads) are called; no stored value comes from the GPU path.  The oracle
records a strided subset of each configuration's receivers (recording is
independent per receiver), so the files stay small; the GPU tests run the
whole configuration and compare that subset.

  python tests/golden/make_fullsize.py CASE [CASE ...]    (repository root)

Cases:
  layered256_so16   256^3 + 40-cell layer, 5 layers + N(0, 50^2), SO16,
                    1000 steps, Kaiser-sinc source, 128 x 128 receivers
                    (every 8th row and column of the receiver grid stored)
  smooth512_const   512^3 + layer, smooth random velocity, constant density,
                    SO8, the first 400 of the 2000 steps (the oracle takes
                    about 45 minutes for them on 8 host cores), trilinear
                    source / receivers (the headline grid; every 16th row
                    and column stored)
  batch_shots       the smallest and the largest of the 64 uneven batch
                    shots, SO8, 400 steps (every 4th receiver row and column)
  smooth200_stag    200^3 + layer, smooth random velocity, Gardner density,
                    staggered variable density, SO8, 400 steps (the oracle's
                    staggered operator runs at about 0.0025 Gpts/s here, so
                    the headline 512^3 grid is out of its reach), trilinear
                    source / receivers (every 10th row and column stored)
  smooth200_cent    the same configuration with the centred variable-density
                    operator (the paper's form), 400 steps
  gradient320       320^3 + layer layered + N(0, 50^2) model, 2 of the 8
                    shots, SO8, 300 steps, L2 misfit against data of the
                    unperturbed layered model; velocity gradient summed over
                    the two shots, sampled at fixed nodes
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle          # noqa: E402
import workloads       # noqa: E402

BATCH_STEPS = 400
SMOOTH_STEPS = 400
GRADIENT_STEPS = 300
GRADIENT_SHOTS = (0, 5)


def grid_subset(nside, stride):
    """Indices into a receiver grid stored row-major (nside x nside)."""
    k = np.arange(0, nside, stride)
    return (k[:, None] * nside + k[None, :]).ravel()


def _traces(wl, scheme, dt, nsteps, subset):
    nbl = ((wl.nbl, wl.nbl),) * len(wl.n)
    prob = oracle.Problem(n=wl.n, h=wl.h, space_order=wl.space_order, dt=dt, nsteps=nsteps,
                          scheme=scheme, nbl=nbl)
    rho = None if scheme == "const" else wl.rho.astype(np.float64)
    st = oracle.prepare(prob, wl.vel.astype(np.float64), rho)
    src = oracle.geometry_table(prob, wl.src, wl.src_interp, wl.radius)
    rec_pts = wl.rec[subset]
    rec = oracle.geometry_table(prob, rec_pts, wl.rec_interp, wl.radius)
    wav = np.stack([oracle.ricker(wl.f_peak, dt, nsteps)] * len(wl.src), axis=1)
    fw = oracle.forward(st, wav, src, rec, len(rec_pts))
    return fw.traces


def case_layered256_so16():
    wl = workloads.layered_3d()
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(wl.h, wl.space_order, wl.cmax)
    subset = grid_subset(128, 8)
    return {"dt": dt, "nsteps": wl.nsteps, "subset": subset,
            "traces": _traces(wl, "const", dt, wl.nsteps, subset)}


def case_smooth512_const():
    wl = workloads.smooth_3d(scheme="const")
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(wl.h, wl.space_order, wl.cmax)
    nside = int(round(np.sqrt(len(wl.rec))))
    subset = grid_subset(nside, 16)
    return {"dt": dt, "nsteps": SMOOTH_STEPS, "subset": subset,
            "traces": _traces(wl, "const", dt, SMOOTH_STEPS, subset)}


STAG_STEPS = 400


def case_smooth200_stag():
    wl = workloads.smooth_3d(n=200, nsteps=STAG_STEPS, scheme="vd_staggered")
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(wl.h, wl.space_order, wl.cmax)
    nside = int(round(np.sqrt(len(wl.rec))))
    subset = grid_subset(nside, 10)
    return {"dt": dt, "nsteps": STAG_STEPS, "subset": subset,
            "traces": _traces(wl, "vd_staggered", dt, STAG_STEPS, subset)}


def case_smooth200_cent():
    wl = workloads.smooth_3d(n=200, nsteps=STAG_STEPS, scheme="vd_centred")
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(wl.h, wl.space_order, wl.cmax)
    nside = int(round(np.sqrt(len(wl.rec))))
    subset = grid_subset(nside, 10)
    return {"dt": dt, "nsteps": STAG_STEPS, "subset": subset,
            "traces": _traces(wl, "vd_centred", dt, STAG_STEPS, subset)}


def batch_pick(shots):
    """Indices of the smallest and the largest shot by node count."""
    nodes = [np.prod([k + 2 * s.nbl for k in s.n]) for s in shots]
    return int(np.argmin(nodes)), int(np.argmax(nodes))


def case_batch_shots():
    shots = workloads.batch_3d(nshots=64, nsteps=BATCH_STEPS)
    picks = batch_pick(shots)
    subset = grid_subset(64, 4)
    out = {"picks": np.array(picks), "nsteps": BATCH_STEPS, "subset": subset}
    for k in picks:
        wl = shots[k]
        dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(wl.h, wl.space_order, wl.cmax)
        out[f"dt_{k}"] = dt
        out[f"traces_{k}"] = _traces(wl, "const", dt, BATCH_STEPS, subset)
    return out


def gradient_samples(n, seed=50):
    """Physical node indices where the gradient is stored: every second node of
    the source plane (z index 2) and seeded random nodes of the whole grid."""
    k = np.arange(0, n, 2)
    plane = ((2 * n + k[:, None]) * n + k[None, :]).ravel()
    rng = np.random.default_rng(seed)
    rand = rng.choice(n ** 3, 30000, replace=False)
    return np.unique(np.concatenate([plane, rand])).astype(np.int64)


def case_gradient320():
    wl = workloads.gradient_3d(nsteps=GRADIENT_STEPS)
    ref_model = wl.extra["reference"]
    cmax = max(float(wl.vel.max()), float(ref_model.max()))
    dt = workloads.CFL_FRACTION * oracle.coeffs.critical_dt(wl.h, wl.space_order, cmax)
    nbl = ((wl.nbl, wl.nbl),) * 3
    prob = oracle.Problem(n=wl.n, h=wl.h, space_order=wl.space_order, dt=dt, nsteps=GRADIENT_STEPS,
                          nbl=nbl)
    st_ref = oracle.prepare(prob, ref_model.astype(np.float64))
    st = oracle.prepare(prob, wl.vel.astype(np.float64))
    rec = oracle.geometry_table(prob, wl.rec, wl.rec_interp, wl.radius)
    wav = oracle.ricker(wl.f_peak, dt, GRADIENT_STEPS)[:, None]
    samples = gradient_samples(wl.n[0])
    grad = np.zeros(len(samples))
    misfit = 0.0
    for s in GRADIENT_SHOTS:
        src = oracle.geometry_table(prob, wl.src[s:s + 1], wl.src_interp, wl.radius)
        d_obs = oracle.forward(st_ref, wav, src, rec, len(wl.rec)).traces
        # checkpoints every 25 steps (the gradient is the same bits for any spacing)
        _, gc, tr = oracle.gradient_checkpointed(st, wav, src, rec, len(wl.rec),
                                                 lambda t, d=d_obs: t - d, 25)
        grad += gc.reshape(-1)[samples]
        misfit += 0.5 * float(np.sum((tr - d_obs) ** 2))
        del d_obs, gc, tr
    return {"dt": dt, "nsteps": GRADIENT_STEPS, "shots": np.array(GRADIENT_SHOTS),
            "samples": samples, "grad": grad, "misfit": misfit}


CASES = {name[5:]: fn for name, fn in globals().items() if name.startswith("case_")}


def main(names):
    for name in names:
        t0 = time.time()
        out = CASES[name]()
        path = os.path.join(HERE, f"fullsize_{name}.npz")
        np.savez_compressed(path, **out)
        print(f"{name}: {time.time() - t0:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
