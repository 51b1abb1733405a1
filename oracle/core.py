"""FP64 forward propagator, adjoint and velocity gradient (oracle).

Test infrastructure: only tests, the smoke check and the benchmark's
CPU-baseline leg use this module.  It shares no code with the HIP library.

Problem statement (paper, "Governing equations", "Boundary conditions and
domain truncation", "Time discretization", "Sources and receivers"):

* The physical grid (n nodes per axis, spacing h) is extended by an absorbing
  layer of nbl cells per side; velocity and density are copied from the
  nearest physical node into the layer.
* Inside the layer eta = alpha d^p, d the Euclidean distance in cells from the
  node to the physical node box; eta = 0 in the physical grid.
* Time levels: p^{-1} = p^0 = 0.  For n = 0 .. N-1
      p^{n+1} = A (2 p^n + K (L p^n)) - B p^{n-1}              (stencil)
      p^{n+1} += A M (d_s / dV) S_s(t_n)   at each source node    (injection)
      rec[n]   = sum_k d_k p^{n+1}                                (recording)
  with M = dt^2 c^2, K = M (or dt^2 rho c^2 for the staggered operator),
  A = 1/(1 + eta dt), B = (1 - eta dt)/(1 + eta dt), dV the cell volume.
  The source enters as c^2 dt^2 S(t) delta(x - x_s): the discrete delta is the
  interpolation weight divided by the cell volume.

Adjoint of the forward map (velocity gradient of J = 1/2 sum (rec - d_obs)^2,
constant density, ghost condition "none" so that L is symmetric):
      phi^{N+1} = phi^{N+2} = 0
      phi^m = A (2 phi^{m+1} + M L phi^{m+1} + M P_r^T r^{m-1}) - B phi^{m+2},
      m = N .. 1, with r^n = rec[n] - d_obs[n] and P_r^T the receiver weights
      spread back onto their nodes,
      dJ/dM = sum_{n=0}^{N-1} phi^{n+1} [(1+eta dt) u^{n+1} - 2 u^n + (1-eta dt) u^{n-1}] / M^2,
      dJ/dc = dJ/dM * 2 dt^2 c, summed back from the layer onto the physical
      node each layer node copies.
  phi = M A mu where mu is the Lagrange multiplier of the update equation.
  The adjoint of the source map is (F^T r)_s^n = sum_x (d_s/dV) phi^{n+1}.

Adjoint of the staggered variable-density forward map (velocity and density
gradients; ghost condition "none").  With zero ghosts the half-node
difference D+ (nodes -> faces m + 1/2, every face the divergence reads,
m = -r .. n + r - 2 per axis) and the node difference D- satisfy D- = -(D+)^T,
so L = -sum_i (D+_i)^T diag(b_i) D+_i is symmetric (b_i the face buoyancies).
The update is u^{n+1} = A (2 u^n + K L u^n + M q^n) - B u^{n-1}, K = dt^2 rho c^2,
M = dt^2 c^2, q^n the source term (d_s / dV) S_s(t_n).  Taking the Lagrange
multiplier mu^n of step n and phi^{n+1} = K A mu^n:
      phi^m = A (2 phi^{m+1} + K L phi^{m+1} + K P_r^T r^{m-1}) - B phi^{m+2}
  (the forward stencil again, the residual entering with weight A K), and
      dJ/dK      = sum_n phi^{n+1} (L u^n) / K
      dJ/dM      = sum_n phi^{n+1} q^n / K                (source nodes only)
      dJ/db_face = -sum_n (D+_i phi^{n+1}) (D+_i u^n)      per axis and face
      dJ/db      = the transpose of the midpoint interpolation
                   b_{m+1/2} = sum_j m_j (b_{m+j} + b_{m-j+1}) (indices clamped
                   to the grid, as the forward reads b) applied to dJ/db_face
      dJ/dc      = dJ/dK 2 dt^2 rho c + dJ/dM 2 dt^2 c
      dJ/drho    = dJ/dK dt^2 c^2 - dJ/db / rho^2
  each summed back from the layer onto the physical node it copies.  The
  source enters with M = K / rho, so the adjoint of the source map is
  (F^T r)_s^n = sum_x (d_s / (dV rho)) phi^{n+1}.  The paper
  states no adjoint: this is the exact adjoint of the discrete forward map,
  pinned by finite differences of that map.
"""
from dataclasses import dataclass, field
import ctypes
import numpy as np

from . import coeffs
from . import geometry
from ._native import lib, Grid, RMAX

SCHEMES = {"const": 0, "vd_staggered": 1, "vd_centred": 2}
BCS = {"none": 0, "dirichlet": 1, "neumann": 2}


@dataclass
class Problem:
    n: tuple                     # physical nodes per axis (z, x[, y])
    h: tuple                     # spacing per axis (m)
    space_order: int
    dt: float
    nsteps: int
    scheme: str = "const"
    nbl: tuple = None            # ((lo, hi), ...) cells
    bc: tuple = None             # (("none", "none"), ...)
    alpha: float = 0.001
    power: float = 3.0

    def __post_init__(self):
        self.n = tuple(int(x) for x in self.n)
        self.h = tuple(float(x) for x in self.h)
        if self.nbl is None:
            self.nbl = tuple((0, 0) for _ in self.n)
        if self.bc is None:
            self.bc = tuple(("none", "none") for _ in self.n)
        self.nbl = tuple((int(a), int(b)) for a, b in self.nbl)

    @property
    def ndim(self):
        return len(self.n)

    @property
    def r(self):
        return self.space_order // 2

    @property
    def N(self):
        return tuple(n + lo + hi for n, (lo, hi) in zip(self.n, self.nbl))

    @property
    def dV(self):
        return float(np.prod(self.h))

    @property
    def nbl_lo(self):
        return tuple(lo for lo, _ in self.nbl)


def extend(a, prob):
    """Physical-grid array -> extended grid by edge replication."""
    return np.pad(np.asarray(a, dtype=np.float64), prob.nbl, mode="edge")


def damping(prob):
    """eta over the extended grid."""
    N = prob.N
    d2 = np.zeros(N)
    for i, (n, (lo, hi)) in enumerate(zip(prob.n, prob.nbl)):
        k = np.arange(N[i])
        e = np.maximum(0, np.maximum(lo - k, k - (lo + n - 1))).astype(np.float64)
        shape = [1] * prob.ndim
        shape[i] = N[i]
        d2 = d2 + (e ** 2).reshape(shape)
    return prob.alpha * np.sqrt(d2) ** prob.power


def make_grid(prob):
    g = Grid()
    g.ndim = prob.ndim
    g.r = prob.r
    if prob.r > RMAX:
        raise ValueError("space order too high for the oracle")
    N = list(prob.N) + [1] * (3 - prob.ndim)
    h = list(prob.h) + [1.0] * (3 - prob.ndim)
    for i in range(3):
        g.N[i] = N[i]
        g.h[i] = h[i]
    for i in range(prob.ndim):
        for s in range(2):
            g.bc[i][s] = BCS[prob.bc[i][s]]
    v = coeffs.second_derivative(prob.space_order)
    w = coeffs.first_derivative_w(prob.space_order)
    sj = coeffs.staggered(prob.space_order)
    mj = coeffs.midpoint(prob.space_order)
    for j in range(prob.r + 1):
        g.v[j] = float(v[j])
        g.w[j] = float(w[j])
        g.s[j] = float(sj[j])
        g.m[j] = float(mj[j])
    return g


def _ptr(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Setup:
    prob: Problem
    grid: Grid
    c: np.ndarray       # extended velocity
    M: np.ndarray       # dt^2 c^2
    K: np.ndarray       # multiplier of L p in the update
    A: np.ndarray
    B: np.ndarray
    eta: np.ndarray
    aux: np.ndarray     # b = 1/rho (staggered), rho (centred), or None


def prepare(prob, vel, rho=None):
    if prob.scheme != "const" and rho is None:
        raise ValueError("variable-density schemes need a density model")
    c = extend(vel, prob)
    M = prob.dt ** 2 * c ** 2
    eta = damping(prob)
    A = 1.0 / (1.0 + eta * prob.dt)
    B = (1.0 - eta * prob.dt) / (1.0 + eta * prob.dt)
    aux = None
    K = M
    if prob.scheme == "vd_staggered":
        r = extend(rho, prob)
        K = M * r
        aux = np.ascontiguousarray(1.0 / r)
    elif prob.scheme == "vd_centred":
        aux = np.ascontiguousarray(extend(rho, prob))
    return Setup(prob, make_grid(prob), c, np.ascontiguousarray(M), np.ascontiguousarray(K),
                 np.ascontiguousarray(A), np.ascontiguousarray(B), eta, aux)


MIRROR_SIGN = {"none": None, "dirichlet": -1.0, "neumann": 1.0}


def geometry_table(prob, coords, interp="hicks", radius=4, kaiser_b=None, role=None):
    """(nodes, ids, weights) on the extended grid for points given in metres.
    role ("source" or "receiver") says how a footprint crossing a side with a
    mirror ghost condition is treated (image sources, ghost reads); it must be
    given when the problem has such a side."""
    mirror = [tuple(MIRROR_SIGN[b] for b in side) for side in prob.bc]
    if any(s is not None for side in mirror for s in side):
        if role not in ("source", "receiver"):
            raise ValueError("geometry_table needs role='source' or 'receiver' with mirror ghost conditions")
    return geometry.weight_table(coords, prob.h, prob.nbl_lo, prob.N, interp, radius, kaiser_b,
                                 mirror=mirror, role=role or "receiver")


def step(st, p, prev, lap_out=None):
    """One stencil update: prev (p^{n-1}) becomes p^{n+1}."""
    lib().ow_step(ctypes.byref(st.grid), SCHEMES[st.prob.scheme], _ptr(p), _ptr(prev),
                  _ptr(st.K), _ptr(st.A), _ptr(st.B), _ptr(st.aux), _ptr(lap_out))


def step_points(st, p, prev, idx):
    """p^{n+1} (before injection) at the flat extended-grid indices idx, from
    p^n = p and p^{n-1} = prev, without touching either."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(len(idx))
    lib().ow_step_points(ctypes.byref(st.grid), SCHEMES[st.prob.scheme], _ptr(p), _ptr(prev),
                         _ptr(st.K), _ptr(st.A), _ptr(st.B), _ptr(st.aux),
                         idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(idx), _ptr(out))
    return out


def injection_terms(st, table, amplitudes):
    """(nodes, values): what inject() adds at each node of a source table."""
    nodes, ids, w = table
    vals = st.A.ravel()[nodes] * st.M.ravel()[nodes] * (w / st.prob.dV) * amplitudes[ids]
    u, inv = np.unique(nodes, return_inverse=True)
    acc = np.zeros(len(u))
    np.add.at(acc, inv, vals)
    return u, acc


def apply_L(st, p):
    out = np.empty_like(p)
    lib().ow_apply_L(ctypes.byref(st.grid), SCHEMES[st.prob.scheme], _ptr(p), _ptr(st.aux),
                     _ptr(out))
    return out


def inject(st, field_flat, table, amplitudes, divide_by_volume=True, weight=None):
    """field[node] += A W w (/dV) * amplitude[id] for every table entry, W = M
    unless another multiplier field is given."""
    nodes, ids, w = table
    if len(nodes) == 0:
        return
    W = st.M if weight is None else weight
    scale = w / st.prob.dV if divide_by_volume else w
    np.add.at(field_flat, nodes, st.A.ravel()[nodes] * W.ravel()[nodes] * scale * amplitudes[ids])


def record(field_flat, table, npts):
    nodes, ids, w = table
    out = np.zeros(npts)
    if len(nodes):
        np.add.at(out, ids, w * field_flat[nodes])
    return out


@dataclass
class ForwardResult:
    traces: np.ndarray              # (nsteps, nrec)
    p: np.ndarray                   # last level u^N (extended grid)
    p_prev: np.ndarray              # u^{N-1}
    snaps: list = field(default_factory=list)
    history: list = None            # u^0 .. u^N when requested
    checkpoints: dict = None        # step k -> (u^k, u^{k-1})


def forward(st, wavelet, src, rec, nrec, snap_stride=0, keep_history=False,
            forcing=None, state=None, nsteps=None, checkpoint_every=0):
    """Run the forward propagator.

    wavelet : (nsteps, nsrc) source amplitudes S_s(t_n)
    src/rec : geometry tables from geometry_table
    forcing : optional callable n -> distributed source f^n on the extended
              grid, added as A M f^n (no volume division)
    state   : optional (u^{k}, u^{k-1}, k) to resume from step k
    """
    prob = st.prob
    N = prob.N
    total = prob.nsteps if nsteps is None else nsteps
    if state is None:
        p = np.zeros(N)
        prev = np.zeros(N)
        k0 = 0
    else:
        p = np.array(state[0], dtype=np.float64, copy=True).reshape(N)
        prev = np.array(state[1], dtype=np.float64, copy=True).reshape(N)
        k0 = state[2]
    traces = np.zeros((total, nrec))
    snaps = []
    history = [p.copy()] if keep_history else None
    ckpts = {} if checkpoint_every else None
    for n in range(k0, k0 + total):
        if ckpts is not None and n % checkpoint_every == 0:
            ckpts[n] = (p.copy(), prev.copy())
        step(st, p, prev)
        nxt = prev
        flat = nxt.reshape(-1)
        if wavelet is not None:
            inject(st, flat, src, wavelet[n])
        if forcing is not None:
            flat += (st.A * st.M * forcing(n)).reshape(-1)
        traces[n - k0] = record(flat, rec, nrec)
        if snap_stride and (n + 1) % snap_stride == 0:
            snaps.append(nxt.copy())
        if keep_history:
            history.append(nxt.copy())
        p, prev = nxt, p
    return ForwardResult(traces, p, prev, snaps, history, ckpts)


def second_difference(st, u_next, u, u_prev):
    """(1 + eta dt) u^{n+1} - 2 u^n + (1 - eta dt) u^{n-1}."""
    e = st.eta * st.prob.dt
    return (1.0 + e) * u_next - 2.0 * u + (1.0 - e) * u_prev


def fold_to_physical(prob, g_ext):
    """Sum an extended-grid field back onto the physical node each layer node
    copies (the transpose of edge replication)."""
    out = g_ext
    for i, (n, (lo, hi)) in enumerate(zip(prob.n, prob.nbl)):
        out = np.moveaxis(out, i, 0)
        core = out[lo:lo + n].copy()
        if lo:
            core[0] += out[:lo].sum(axis=0)
        if hi:
            core[-1] += out[lo + n:].sum(axis=0)
        out = np.moveaxis(core, 0, i)
    return out


class AdjointState:
    """Adjoint wavefield pair carried across checkpoint segments."""

    def __init__(self, N):
        self.phi1 = np.zeros(N)    # phi^{m+1}
        self.phi2 = np.zeros(N)    # phi^{m+2}


def adjoint_segment(st, rec, residual, history_fn, m_hi, m_lo, state, gM, src=None, src_adj=None):
    """Adjoint steps m = m_hi .. m_lo (descending).  history_fn(n) returns u^n
    (u^{-1} = 0).  Accumulates dJ/dM into gM and, if src is given, the source
    adjoint into src_adj[m-1]."""
    prob = st.prob
    for m in range(m_hi, m_lo - 1, -1):
        step(st, state.phi1, state.phi2)            # phi2 <- phi^m before injection
        phi = state.phi2
        flat = phi.reshape(-1)
        inject(st, flat, rec, residual[m - 1], divide_by_volume=False, weight=st.K)
        if src is not None:
            src_adj[m - 1] = record(flat, (src[0], src[1], src[2] / prob.dV), src_adj.shape[1])
        d2u = second_difference(st, history_fn(m), history_fn(m - 1), history_fn(m - 2))
        gM += phi * d2u / st.M ** 2
        state.phi1, state.phi2 = phi, state.phi1


def gradient(st, rec, residual, history, src=None, nsrc=0):
    """dJ/dM (extended grid), dJ/dc (physical grid) and, optionally, F^T r.

    history: list u^0 .. u^N from forward(keep_history=True)."""
    prob = st.prob
    if prob.scheme != "const":
        raise NotImplementedError("the adjoint covers constant density")
    if any(b != "none" for side in prob.bc for b in side):
        raise NotImplementedError("the adjoint assumes the zero ghost condition")
    N = prob.N
    nsteps = len(history) - 1
    zero = np.zeros(N)

    def u(n):
        return zero if n < 0 else history[n]

    gM = np.zeros(N)
    src_adj = np.zeros((nsteps, nsrc)) if src is not None else None
    state = AdjointState(N)
    adjoint_segment(st, rec, residual, u, nsteps, 1, state, gM, src, src_adj)
    gc = fold_to_physical(prob, gM * 2.0 * prob.dt ** 2 * st.c)
    return gM, gc, src_adj


def face_difference(st, q, axis):
    """(D+ q)_{m+1/2} along `axis` on the faces m = -r .. n + r - 2 (array index
    m + r), zero ghosts:  (1/h) sum_l s_l (q_{m+l} - q_{m-l+1})."""
    prob = st.prob
    r = prob.r
    s = coeffs.staggered(prob.space_order)
    g = np.moveaxis(q, axis, 0)
    n = g.shape[0]
    padded = np.zeros((n + 4 * r,) + g.shape[1:])
    padded[2 * r:2 * r + n] = g                # node k at index k + 2r
    nf = n + 2 * r - 1
    out = np.zeros((nf,) + g.shape[1:])
    for l in range(1, r + 1):
        # face m sits at index t = m + r: q_{m+l} at t + r + l, q_{m-l+1} at t + r - l + 1
        out += float(s[l]) * (padded[r + l:r + l + nf] - padded[r - l + 1:r - l + 1 + nf])
    return np.moveaxis(out / prob.h[axis], 0, axis)


def midpoint_transpose(st, F, axis):
    """Transpose of the face buoyancy interpolation along `axis`: node values
    from face values F (faces m = -r .. n + r - 2), where the forward takes
    b_{m+1/2} = sum_j m_j (b_{m+j} + b_{m-j+1}) with node indices clamped to
    the grid."""
    prob = st.prob
    r = prob.r
    mj = coeffs.midpoint(prob.space_order)
    Fm = np.moveaxis(F, axis, 0)
    n = Fm.shape[0] - 2 * r + 1
    out = np.zeros((n,) + Fm.shape[1:])
    m = np.arange(-r, n + r - 1)
    for j in range(1, r + 1):
        np.add.at(out, np.clip(m + j, 0, n - 1), float(mj[j]) * Fm)
        np.add.at(out, np.clip(m - j + 1, 0, n - 1), float(mj[j]) * Fm)
    return np.moveaxis(out, 0, axis)


def source_term(st, table, amplitudes):
    """q: sum over table entries of (w / dV) amplitude[id] at each node."""
    nodes, ids, w = table
    q = np.zeros(int(np.prod(st.prob.N)))
    if len(nodes):
        np.add.at(q, nodes, (w / st.prob.dV) * amplitudes[ids])
    return q.reshape(st.prob.N)


def gradient_vd(st, wavelet, src, rec, residual, history, nsrc=0):
    """Velocity and density gradients of 1/2 sum (rec - d_obs)^2 for the
    staggered variable-density scheme, from the stored history u^0 .. u^N:
    (dJ/dc, dJ/drho) on the physical grid, (dJ/dK, dJ/dM, dJ/db) on the
    extended grid and, when nsrc > 0, the adjoint of the source map F^T r."""
    prob = st.prob
    if prob.scheme != "vd_staggered":
        raise ValueError("gradient_vd covers the staggered variable-density scheme")
    if any(b != "none" for side in prob.bc for b in side):
        raise NotImplementedError("the adjoint assumes the zero ghost condition")
    N = prob.N
    nsteps = len(history) - 1
    gK = np.zeros(N)
    gMsrc = np.zeros(N)
    gface = [np.zeros(tuple(N[a] + (2 * prob.r - 1 if a == i else 0) for a in range(prob.ndim)))
             for i in range(prob.ndim)]
    state = AdjointState(N)
    src_adj = np.zeros((nsteps, nsrc)) if nsrc else None
    for m in range(nsteps, 0, -1):
        step(st, state.phi1, state.phi2)           # phi2 <- phi^m before injection
        phi = state.phi2
        inject(st, phi.reshape(-1), rec, residual[m - 1], divide_by_volume=False, weight=st.K)
        if nsrc:
            nodes, ids, w = src
            src_adj[m - 1] = record(phi.reshape(-1), (nodes, ids, w * st.aux.ravel()[nodes] / prob.dV), nsrc)
        u = history[m - 1]                         # u^n with n = m - 1
        gK += phi * apply_L(st, u) / st.K
        if wavelet is not None:
            gMsrc += phi * source_term(st, src, wavelet[m - 1]) / st.K
        for i in range(prob.ndim):
            gface[i] -= face_difference(st, phi, i) * face_difference(st, u, i)
        state.phi1, state.phi2 = phi, state.phi1
    gb = sum(midpoint_transpose(st, gface[i], i) for i in range(prob.ndim))
    rho = 1.0 / st.aux
    dt2 = prob.dt ** 2
    gc_ext = gK * 2.0 * dt2 * rho * st.c + gMsrc * 2.0 * dt2 * st.c
    grho_ext = gK * dt2 * st.c ** 2 - gb / rho ** 2
    return (fold_to_physical(prob, gc_ext), fold_to_physical(prob, grho_ext), gK, gMsrc, gb, src_adj)


def gradient_checkpointed(st, wavelet, src, rec, nrec, residual_fn, every):
    """Same gradient with forward checkpoints every `every` steps and segment
    recomputation in the backward pass.  residual_fn(traces) -> residual."""
    prob = st.prob
    N = prob.N
    nsteps = prob.nsteps
    fw = forward(st, wavelet, src, rec, nrec, checkpoint_every=every)
    residual = residual_fn(fw.traces)
    gM = np.zeros(N)
    state = AdjointState(N)
    zero = np.zeros(N)
    starts = sorted(fw.checkpoints)
    for k in reversed(starts):
        seg_len = min(every, nsteps - k)
        u_k, u_km1 = fw.checkpoints[k]
        seg = forward(st, wavelet, src, rec, nrec, keep_history=True,
                      state=(u_k, u_km1, k), nsteps=seg_len)
        levels = {k - 1: u_km1, **{k + i: seg.history[i] for i in range(seg_len + 1)}}

        def u(n, levels=levels):
            return zero if n < 0 else levels[n]

        adjoint_segment(st, rec, residual, u, k + seg_len, k + 1, state, gM)
    gc = fold_to_physical(prob, gM * 2.0 * prob.dt ** 2 * st.c)
    return gM, gc, fw.traces


def ricker(f_peak, dt, nsteps, t0=None):
    """Ricker wavelet of peak frequency f, peak amplitude 1, delayed by
    t0 = 1/f, sampled at t_n = n dt:
        S(t) = (1 - 2 pi^2 f^2 (t - t0)^2) exp(-pi^2 f^2 (t - t0)^2)."""
    t0 = 1.0 / f_peak if t0 is None else t0
    t = np.arange(nsteps) * dt - t0
    a = (np.pi * f_peak * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)
