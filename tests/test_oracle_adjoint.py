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


# ---- staggered variable-density adjoint --------------------------------------

def _vd_setup(n=(24, 28), nbl=5, so=4, nt=80, seed=5, points=True):
    h = tuple(10.0 for _ in n)
    rng = np.random.default_rng(seed)
    c = 1800.0 + 600.0 * rng.random(n)
    rho = 1500.0 + 1000.0 * rng.random(n)
    dt = 0.5 * coeffs.critical_dt(h, so, c.max())
    prob = oracle.Problem(n=n, h=h, space_order=so, dt=dt, nsteps=nt, scheme="vd_staggered",
                          nbl=tuple((nbl, nbl + 1) for _ in n))
    if not points:
        return prob, c, rho
    if len(n) == 2:
        src_pts, rec_pts = [(61.3, 77.7), (150.0, 190.0)], [(20.0 + 13.0 * k, 30.0 + 17.0 * k) for k in range(9)]
    else:
        src_pts, rec_pts = [(41.3, 47.7, 52.2)], [(10.0 + 7.0 * k, 20.0 + 5.0 * k, 15.0 + 6.0 * k) for k in range(8)]
    src = oracle.geometry_table(prob, src_pts, "hicks")
    rec = oracle.geometry_table(prob, rec_pts, "hicks")
    wav = np.stack([oracle.ricker(18.0 + 3.0 * k, prob.dt, prob.nsteps) for k in range(len(src_pts))], axis=1)
    return prob, c, rho, src, rec, len(rec_pts), wav, rng


def _face_buoyancy(st, b, axis):
    # b_{m+1/2} = sum_j m_j (b_{m+j} + b_{m-j+1}) on faces m = -r .. n + r - 2,
    # node indices clamped to the grid (nearest node outside it)
    r = st.prob.r
    mj = coeffs.midpoint(st.prob.space_order)
    bm = np.moveaxis(b, axis, 0)
    n = bm.shape[0]
    out = np.zeros((n + 2 * r - 1,) + bm.shape[1:])
    for t, m in enumerate(range(-r, n + r - 1)):
        for j in range(1, r + 1):
            out[t] += float(mj[j]) * (bm[min(max(m + j, 0), n - 1)] + bm[min(max(m - j + 1, 0), n - 1)])
    return np.moveaxis(out, 0, axis)


@pytest.mark.parametrize("n,so", [((13, 17), 4), ((13, 17), 8), ((7, 9, 8), 6)])
def test_staggered_operator_energy_form(n, so):
    # <L u, v> = -sum_i <b_i D+_i u, D+_i v> over every face the divergence
    # reads: pins the face range and D- = -(D+)^T of the half-node differences
    # against the C operator, and makes L symmetric.
    prob, c, rho = _vd_setup(n=n, so=so, nbl=2, nt=1, points=False)
    st = oracle.prepare(prob, c, rho)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(prob.N)
    v = rng.standard_normal(prob.N)
    Lu, Lv = oracle.apply_L(st, u), oracle.apply_L(st, v)
    energy = -sum(np.sum(_face_buoyancy(st, st.aux, i) * oracle.face_difference(st, u, i) *
                         oracle.face_difference(st, v, i)) for i in range(prob.ndim))
    scale = np.sum(np.abs(Lu * v))
    assert abs(np.sum(Lu * v) - energy) < 1e-12 * scale
    assert abs(np.sum(Lu * v) - np.sum(u * Lv)) < 1e-12 * scale


def test_midpoint_transpose_is_adjoint_of_interpolation():
    prob, c, rho = _vd_setup(n=(9, 11, 7), so=8, nbl=1, nt=1, points=False)
    st = oracle.prepare(prob, c, rho)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(prob.N)
    for i in range(3):
        F = rng.standard_normal(_face_buoyancy(st, b, i).shape)
        lhs = np.sum(F * _face_buoyancy(st, b, i))
        rhs = np.sum(oracle.midpoint_transpose(st, F, i) * b)
        assert abs(lhs - rhs) < 1e-12 * np.sum(np.abs(F))


def _vd_misfit(prob, c, rho, src, rec, nrec, wav, d_obs):
    st = oracle.prepare(prob, c, rho)
    tr = oracle.forward(st, wav, src, rec, nrec).traces
    return 0.5 * np.sum((tr - d_obs) ** 2)


@pytest.mark.parametrize("n,nbl,so", [((24, 28), 5, 4), ((20, 22), 0, 8), ((10, 11, 12), 3, 4)])
def test_vd_gradients_match_finite_differences(n, nbl, so):
    prob, c, rho, src, rec, nrec, wav, rng = _vd_setup(n=n, nbl=nbl, so=so, nt=70 if len(n) == 2 else 45)
    d_obs = oracle.forward(oracle.prepare(prob, c * (1.0 + 0.05 * rng.standard_normal(n)),
                                          rho * (1.0 + 0.1 * rng.standard_normal(n))),
                           wav, src, rec, nrec).traces
    st = oracle.prepare(prob, c, rho)
    fw = oracle.forward(st, wav, src, rec, nrec, keep_history=True)
    gc, grho, *_ = oracle.gradient_vd(st, wav, src, rec, fw.traces - d_obs, fw.history)
    # a random direction, and single physical nodes: a corner (its layer
    # copies and the clamped buoyancy reads), an edge node and a node under
    # the first source
    dirs = [rng.standard_normal(n)]
    for idx in [(0,) * len(n), (n[0] - 1,) + (3,) * (len(n) - 1), tuple(int(round(x / 10.0)) for x in
                                                                         ((61.3, 77.7) if len(n) == 2 else (41.3, 47.7, 52.2)))]:
        e = np.zeros(n)
        e[idx] = 1.0
        dirs.append(e)
    for d in dirs:
        for which, g, base in (("c", gc, c), ("rho", grho, rho)):
            eps = 1e-6 * np.linalg.norm(base) / np.linalg.norm(d) if d.sum() != 1.0 else 1e-6 * base.mean()
            args_p = (c + eps * d, rho) if which == "c" else (c, rho + eps * d)
            args_m = (c - eps * d, rho) if which == "c" else (c, rho - eps * d)
            fd = (_vd_misfit(prob, *args_p, src, rec, nrec, wav, d_obs) -
                  _vd_misfit(prob, *args_m, src, rec, nrec, wav, d_obs)) / (2 * eps)
            an = np.sum(g * d)
            assert abs(fd - an) < 2e-6 * max(abs(an), 1e-3 * np.abs(g).max()), (which, fd, an)


@pytest.mark.parametrize("n", [(24, 28), (10, 11, 12)])
def test_vd_dot_product(n):
    # <F s, r> = <s, F^T r> for the staggered scheme's source-to-trace map
    prob, c, rho, src, rec, nrec, wav, rng = _vd_setup(n=n, nbl=4, so=4, nt=50)
    st = oracle.prepare(prob, c, rho)
    nsrc = wav.shape[1]
    s = rng.standard_normal((prob.nsteps, nsrc))
    r = rng.standard_normal((prob.nsteps, nrec))
    fw = oracle.forward(st, s, src, rec, nrec, keep_history=True)
    FTr = oracle.gradient_vd(st, s, src, rec, r, fw.history, nsrc=nsrc)[5]
    lhs, rhs = np.sum(fw.traces * r), np.sum(s * FTr)
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), abs(rhs))


def test_vd_gradients_so2_single_step_and_no_layer():
    # the shortest stencil, one time step, and no absorbing layer
    for n, nbl, so, nt in [((24, 28), 3, 2, 30), ((24, 28), 0, 4, 1)]:
        prob, c, rho, src, rec, nrec, wav, rng = _vd_setup(n=n, nbl=nbl, so=so, nt=nt)
        d_obs = 1e-3 * rng.standard_normal((nt, nrec))
        st = oracle.prepare(prob, c, rho)
        fw = oracle.forward(st, wav, src, rec, nrec, keep_history=True)
        gc, grho, *_ = oracle.gradient_vd(st, wav, src, rec, fw.traces - d_obs, fw.history)
        d = rng.standard_normal(n)
        for which, g, base in (("c", gc, c), ("rho", grho, rho)):
            eps = 1e-6 * np.linalg.norm(base) / np.linalg.norm(d)
            pa = (c + eps * d, rho) if which == "c" else (c, rho + eps * d)
            ma = (c - eps * d, rho) if which == "c" else (c, rho - eps * d)
            fd = (_vd_misfit(prob, *pa, src, rec, nrec, wav, d_obs) -
                  _vd_misfit(prob, *ma, src, rec, nrec, wav, d_obs)) / (2 * eps)
            an = np.sum(g * d)
            assert abs(fd - an) < 2e-6 * max(abs(an), 1e-12), (n, so, nt, which, fd, an)


def test_vd_gradient_of_zero_residual_is_zero():
    prob, c, rho, src, rec, nrec, wav, _ = _vd_setup(n=(24, 28), nbl=2, so=4, nt=20)
    st = oracle.prepare(prob, c, rho)
    fw = oracle.forward(st, wav, src, rec, nrec, keep_history=True)
    gc, grho, gK, gM, gb, _ = oracle.gradient_vd(st, wav, src, rec, np.zeros((20, nrec)), fw.history)
    assert not np.any(gc) and not np.any(grho) and not np.any(gK) and not np.any(gM) and not np.any(gb)
