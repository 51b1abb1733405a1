"""Pins for the oracle's adjoint, imaging condition and checkpointing.

* Dot-product test <F s, r> = <s, F^T r> and a brute-force transpose of the
  whole source-to-trace map on a tiny grid: any index slip in the adjoint
  recursion (which residual sample enters which step, which level is
  imaged) breaks them.
* The velocity gradient against central finite differences of the misfit.
* Checkpointed recomputation gives the stored-history gradient bit for bit.
"""
import numpy as np
import pytest

import oracle
from oracle import coeffs


def _setup(n=(24, 28), nbl=6, so=4, nt=90, seed=11, interp="hicks", src_pts=None, rec_pts=None):
    h = (10.0, 10.0)
    rng = np.random.default_rng(seed)
    c = 1800.0 + 600.0 * rng.random(n)
    dt = 0.5 * coeffs.critical_dt(h, so, c.max())
    prob = oracle.Problem(n=n, h=h, space_order=so, dt=dt, nsteps=nt,
                          nbl=((nbl, nbl), (nbl, nbl)))
    src_pts = src_pts or [(61.3, 77.7), (150.0, 190.0)]
    rec_pts = rec_pts or [(20.0 + 13.0 * k, 30.0 + 17.0 * k) for k in range(9)]
    src = oracle.geometry_table(prob, src_pts, interp)
    rec = oracle.geometry_table(prob, rec_pts, interp)
    return prob, c, src, rec, len(src_pts), len(rec_pts), rng


@pytest.mark.parametrize("interp", ["hicks", "linear"])
def test_dot_product(interp):
    prob, c, src, rec, nsrc, nrec, rng = _setup(interp=interp)
    st = oracle.prepare(prob, c)
    s = rng.standard_normal((prob.nsteps, nsrc))
    r = rng.standard_normal((prob.nsteps, nrec))
    fw = oracle.forward(st, s, src, rec, nrec, keep_history=True)
    _, _, FTr = oracle.gradient(st, rec, r, fw.history, src=src, nsrc=nsrc)
    lhs = np.sum(fw.traces * r)
    rhs = np.sum(s * FTr)
    assert abs(lhs - rhs) < 1e-13 * max(abs(lhs), abs(rhs))


def test_brute_force_transpose():
    # 12 x 12 grid (with layer), 20 steps, one source, two receivers: build F
    # column by column from unit impulses and F^T row by row from unit
    # residuals; they must be transposes of each other.
    prob, c, src, rec, nsrc, nrec, _ = _setup(n=(12, 12), nbl=3, so=4, nt=20,
                                              src_pts=[(55.0, 53.0)],
                                              rec_pts=[(20.0, 70.0), (90.0, 40.0)])
    st = oracle.prepare(prob, c)
    nt = prob.nsteps
    F = np.zeros((nt * nrec, nt * nsrc))
    hist0 = None
    for j in range(nt * nsrc):
        s = np.zeros(nt * nsrc)
        s[j] = 1.0
        fw = oracle.forward(st, s.reshape(nt, nsrc), src, rec, nrec, keep_history=True)
        F[:, j] = fw.traces.ravel()
        hist0 = fw.history
    FT = np.zeros((nt * nsrc, nt * nrec))
    for i in range(nt * nrec):
        r = np.zeros(nt * nrec)
        r[i] = 1.0
        _, _, a = oracle.gradient(st, rec, r.reshape(nt, nrec), hist0, src=src, nsrc=nsrc)
        FT[:, i] = a.ravel()
    assert np.max(np.abs(FT - F.T)) < 1e-13 * np.max(np.abs(F))
    assert np.count_nonzero(np.abs(F) > 1e-14 * np.max(np.abs(F))) > 10


def _misfit(prob, c, src, rec, nrec, wav, d_obs):
    st = oracle.prepare(prob, c)
    tr = oracle.forward(st, wav, src, rec, nrec).traces
    return 0.5 * np.sum((tr - d_obs) ** 2)


@pytest.mark.parametrize("nbl", [0, 6])
def test_gradient_matches_finite_differences(nbl):
    prob, c, src, rec, nsrc, nrec, rng = _setup(nbl=nbl)
    wav = np.stack([oracle.ricker(18.0, prob.dt, prob.nsteps)] * nsrc, axis=1)
    c_true = c * (1.0 + 0.05 * rng.standard_normal(c.shape))
    d_obs = oracle.forward(oracle.prepare(prob, c_true), wav, src, rec, nrec).traces
    st = oracle.prepare(prob, c)
    fw = oracle.forward(st, wav, src, rec, nrec, keep_history=True)
    _, gc, _ = oracle.gradient(st, rec, fw.traces - d_obs, fw.history)
    dc = rng.standard_normal(c.shape)
    eps = 1e-6 * np.linalg.norm(c) / np.linalg.norm(dc)
    jp = _misfit(prob, c + eps * dc, src, rec, nrec, wav, d_obs)
    jm = _misfit(prob, c - eps * dc, src, rec, nrec, wav, d_obs)
    fd = (jp - jm) / (2 * eps)
    an = np.sum(gc * dc)
    assert abs(fd - an) < 1e-6 * abs(an)


def test_layer_fold_is_transpose_of_replication():
    prob = oracle.Problem(n=(5, 7), h=(1.0, 1.0), space_order=2, dt=1.0, nsteps=1,
                          nbl=((2, 3), (1, 4)))
    rng = np.random.default_rng(0)
    a = rng.standard_normal(prob.n)
    g = rng.standard_normal(prob.N)
    assert abs(np.sum(oracle.extend(a, prob) * g) - np.sum(a * oracle.fold_to_physical(prob, g))) \
        < 1e-12


def test_checkpointed_gradient_is_bitwise_equal():
    prob, c, src, rec, nsrc, nrec, rng = _setup(nt=83)
    wav = np.stack([oracle.ricker(18.0, prob.dt, prob.nsteps)] * nsrc, axis=1)
    d_obs = 0.3 * rng.standard_normal((prob.nsteps, nrec))
    st = oracle.prepare(prob, c)
    fw = oracle.forward(st, wav, src, rec, nrec, keep_history=True)
    gM, gc, _ = oracle.gradient(st, rec, fw.traces - d_obs, fw.history)
    gM2, gc2, tr2 = oracle.gradient_checkpointed(st, wav, src, rec, nrec,
                                                 lambda tr: tr - d_obs, every=10)
    assert np.array_equal(tr2, fw.traces)
    assert np.array_equal(gM, gM2) and np.array_equal(gc, gc2)
