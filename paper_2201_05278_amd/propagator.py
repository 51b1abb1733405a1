"""Python front-end over the C ABI: argument marshalling and torch buffers.

Every numerical step runs in the HIP library; this module only allocates
device buffers with torch, fills the ABI structs and calls the library on the
current torch stream.

Vocabulary follows the paper ("Example of use"): a physical grid with spacing
h, a space order, an absorbing layer added on each side, sources and
receivers at coordinates in metres, a wavelet per source, and forward()
returning receiver traces and wavefields.
"""
import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _pairs(v, ndim):
    if isinstance(v, int):
        return [(v, v)] * ndim
    return [tuple(int(a) for a in x) for x in v]


def critical_dt(h, space_order, cmax):
    h = list(h)
    arr = (ctypes.c_double * 3)(*(h + [1.0] * (3 - len(h))))
    out = ctypes.c_double()
    L.check("sw_critical_dt", L.lib().sw_critical_dt(len(h), arr, space_order, cmax, ctypes.byref(out)))
    return out.value


def steps_for(tf, dt):
    out = ctypes.c_int32()
    L.check("sw_steps_for", L.lib().sw_steps_for(tf, dt, ctypes.byref(out)))
    return out.value


def ricker(f_peak, dt, nsteps, t0=0.0):
    buf = (ctypes.c_float * max(1, nsteps))()
    L.check("sw_ricker", L.lib().sw_ricker(f_peak, t0, dt, nsteps, buf))
    return torch.tensor(list(buf)[:nsteps], dtype=torch.float32)


def remove_nbl(prop, grid):
    """Physical part of an extended-grid array of plan `prop` (the paper's
    remove_nbl)."""
    return prop.physical_view(grid)


def forward(vel, h, space_order, dt, nsteps, src, rec, wavelet=None, f_peak=10.0, rho=None, scheme="const",
            nbl=0, bc=None, src_interp="hicks", rec_interp="hicks", radius=4, saving_stride=0, cmax=None,
            dtype="float32", alpha=0.001, power=3.0, device="cuda"):
    """A whole forward run in one call (the paper's solver forward): plan,
    sources and receivers (coordinates in metres), model (physical-grid
    velocity and, for the variable-density schemes, density), nsteps steps.
    wavelet: (nsteps, nsrc) or (nsteps,) samples; None: a Ricker wavelet of
    peak frequency f_peak at every source.  Returns (traces (nsteps, nrec),
    the last wavefield on the physical grid, the snapshots taken every
    saving_stride steps on the physical grid, or None)."""
    import numpy as np
    vel = torch.as_tensor(vel)
    n = tuple(vel.shape)
    prop = Propagator(n, h, space_order, dt, nsteps, scheme=scheme, nbl=nbl, alpha=alpha, power=power,
                      device=device, bc=bc, dtype=dtype)
    src = np.asarray(src, dtype=np.float64).reshape(-1, len(n))
    prop.set_sources(src, src_interp, radius)
    prop.set_receivers(np.asarray(rec, dtype=np.float64).reshape(-1, len(n)), rec_interp, radius)
    prop.prepare(vel.to(prop.device), None if rho is None else torch.as_tensor(rho).to(prop.device), cmax=cmax)
    if wavelet is None:
        wavelet = ricker(f_peak, dt, nsteps).reshape(-1, 1).repeat(1, len(src))
    wavelet = torch.as_tensor(wavelet).reshape(nsteps, -1)
    if wavelet.shape[1] == 1 and len(src) > 1:
        wavelet = wavelet.repeat(1, len(src))
    res = prop.forward(wavelet.to(prop.device), saving_stride=saving_stride)
    last = prop.physical_view(prop.grid_view(res.fields[res.current])).clone()
    snaps = None
    if res.snaps is not None:
        snaps = res.snaps[(slice(None),) + tuple(
            slice(int(prop.prob.nbl[i][0]), int(prop.prob.nbl[i][0]) + n[i]) for i in range(len(n)))].clone()
    return res.traces, last, snaps


@dataclass
class ForwardResult:
    traces: torch.Tensor        # (nsteps, nrec)
    fields: tuple               # the two wavefield buffers (padded layout)
    current: int                # index in fields of the last level p^{end}
    snaps: torch.Tensor = None  # (nsnap, *grid dims)
    ckpt: torch.Tensor = None   # (nckpt, 2, field_elems)
    checkpoint_every: int = 0


class Propagator:
    """One plan: grid, scheme, time axis, absorbing layer, geometry, model."""

    def __init__(self, n, h, space_order, dt, nsteps, scheme="const", nbl=0, alpha=0.001,
                 power=3.0, device="cuda", bc=None, dtype="float32"):
        ndim = len(n)
        prob = L.Problem()
        prob.ndim = ndim
        for i in range(3):
            prob.n[i] = int(n[i]) if i < ndim else 1
            prob.h[i] = float(h[i]) if i < ndim else 1.0
        prob.space_order = int(space_order)
        prob.scheme = L.SCHEMES[scheme]
        for i, (a, b) in enumerate(_pairs(nbl, ndim)):
            prob.nbl[i][0] = a
            prob.nbl[i][1] = b
        if bc is not None:              # per axis (low, high): "none", "dirichlet" or "neumann"
            for i, (a, b) in enumerate(bc):
                prob.bc[i][0] = L.BCS[a]
                prob.bc[i][1] = L.BCS[b]
        prob.damp_alpha = float(alpha)
        prob.damp_power = float(power)
        prob.dt = float(dt)
        prob.nsteps = int(nsteps)
        if dtype not in ("float32", "float64"):
            raise ValueError("dtype must be 'float32' or 'float64'")
        prob.dtype = 1 if dtype == "float64" else 0
        self.dtype = dtype
        self.torch_dtype = torch.float64 if dtype == "float64" else torch.float32
        self.prob = prob
        self.ndim = ndim
        self.n = tuple(int(x) for x in n)
        self.scheme = scheme
        self.nsteps = int(nsteps)
        self.dt = float(dt)
        self.device = torch.device(device)
        handle = ctypes.c_void_p()
        L.check("sw_plan_create", L.lib().sw_plan_create(ctypes.byref(prob), ctypes.byref(handle)))
        self._plan = handle
        self.workspace = None
        self._vel = None

    def __del__(self):
        try:
            if getattr(self, "_plan", None):
                L.lib().sw_plan_destroy(self._plan)
                self._plan = None
        except Exception:
            pass

    # ---- layout -----------------------------------------------------------
    @property
    def layout(self):
        lay = L.Layout()
        L.check("sw_plan_layout", L.lib().sw_plan_layout(self._plan, ctypes.byref(lay)))
        return lay

    @property
    def grid_shape(self):
        lay = self.layout
        return tuple(lay.dims[:self.ndim])

    def new_field(self):
        return torch.zeros(self.layout.field_elems, dtype=self.torch_dtype, device=self.device)

    def grid_view(self, buf):
        """Extended-grid view of a padded-layout buffer (no copy)."""
        lay = self.layout
        off = buf.storage_offset() + lay.origin
        if self.ndim == 3:
            p1, p2 = lay.padded[1], lay.padded[2]
            return buf.as_strided(tuple(lay.dims[:3]), (p1 * p2, p2, 1), off)
        p1 = lay.padded[1]
        return buf.as_strided(tuple(lay.dims[:2]), (p1, 1), off)

    def physical_view(self, grid):
        """Physical part of an extended-grid array (paper: remove_nbl)."""
        sl = tuple(slice(int(self.prob.nbl[i][0]), int(self.prob.nbl[i][0]) + self.n[i])
                   for i in range(self.ndim))
        return grid[sl]

    # ---- geometry and model -------------------------------------------------
    def _set_points(self, which, coords, interp, radius, kaiser_b):
        import numpy as np
        c = np.ascontiguousarray(np.asarray(coords, dtype=np.float64).reshape(-1, self.ndim))
        arr = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        L.check("sw_plan_set_geometry",
                L.lib().sw_plan_set_geometry(self._plan, which, c.shape[0], arr, L.INTERPS[interp],
                                             int(radius), float(kaiser_b or 0.0)))

    def set_sources(self, coords, interp="hicks", radius=4, kaiser_b=None):
        self._set_points(L.SW_SRC, coords, interp, radius, kaiser_b)
        self._vel = None

    def set_receivers(self, coords, interp="hicks", radius=4, kaiser_b=None):
        self._set_points(L.SW_REC, coords, interp, radius, kaiser_b)
        self._vel = None

    def point_table(self, which):
        """Host table (nodes, ids, weights) of sources ('src') or receivers ('rec')."""
        import numpy as np
        w = L.SW_SRC if which == "src" else L.SW_REC
        n = ctypes.c_int64(0)
        L.check("sw_plan_points", L.lib().sw_plan_points(self._plan, w, ctypes.byref(n), None, None, None))
        nodes = np.zeros(max(1, n.value), np.int64)
        ids = np.zeros(max(1, n.value), np.int32)
        wts = np.zeros(max(1, n.value), np.float32)
        L.check("sw_plan_points", L.lib().sw_plan_points(
            self._plan, w, ctypes.byref(n), nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            wts.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return nodes[:n.value], ids[:n.value], wts[:n.value]

    def prepare(self, vel, rho=None, cmax=None):
        """Build the device model arrays from physical-grid velocity (and density)."""
        if self.dtype == "float64":
            return self._prepare64(vel, cmax)
        vel = vel.to(self.device, torch.float32).contiguous()
        if rho is not None:
            rho = rho.to(self.device, torch.float32).contiguous()
        if tuple(vel.shape) != self.n:
            raise ValueError(f"velocity shape {tuple(vel.shape)} != grid {self.n}")
        lay = self.layout
        nbytes = int(lay.workspace_bytes)
        if self.workspace is None or self.workspace.numel() < nbytes:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        cmax = float(vel.max().item()) if cmax is None else float(cmax)
        L.check("sw_model_prepare", L.lib().sw_model_prepare(
            self._plan, _ptr(vel), _ptr(rho), cmax, _ptr(self.workspace), _stream()))
        self._vel = vel
        self._rho = rho
        return self

    def _prepare64(self, vel, cmax):
        vel = vel.to(self.device, torch.float64).contiguous()
        if tuple(vel.shape) != self.n:
            raise ValueError(f"velocity shape {tuple(vel.shape)} != grid {self.n}")
        nbytes = int(self.layout.workspace_bytes)
        if self.workspace is None or self.workspace.numel() < nbytes:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        cmax = float(vel.max().item()) if cmax is None else float(cmax)
        L.check("sw_model_prepare_f64", L.lib().sw_model_prepare_f64(
            self._plan, _ptr(vel), cmax, _ptr(self.workspace), _stream()))
        self._vel = vel
        self._rho = None
        return self

    def _forward64(self, wavelet, saving_stride, fields, step0, nsteps_run, traces):
        lay = self.layout
        nrun = self.nsteps - step0 if nsteps_run is None else int(nsteps_run)
        self._keep = None
        if fields is None:
            fields = (self.new_field(), self.new_field())
        if lay.nsrc:
            wavelet = wavelet.to(self.device, torch.float64).reshape(self.nsteps, lay.nsrc).contiguous()
        if traces is None:
            traces = torch.zeros((self.nsteps, max(0, lay.nrec)), dtype=torch.float64, device=self.device)
        snaps = None
        if saving_stride:
            snaps = torch.zeros((self.nsteps // saving_stride,) + self.grid_shape, dtype=torch.float64,
                                device=self.device)
        io = L.Fwd64IO()
        io.workspace = _ptr(self.workspace).value
        io.wavelet = _ptr(wavelet if lay.nsrc else None).value
        io.field[0] = fields[0].data_ptr()
        io.field[1] = fields[1].data_ptr()
        io.traces = traces.data_ptr() if lay.nrec else None
        io.snaps = snaps.data_ptr() if snaps is not None else None
        io.saving_stride = int(saving_stride)
        io.step0 = int(step0)
        io.nsteps_run = nrun
        self._keep = (wavelet, fields, traces, snaps)
        L.check("sw_forward_f64", L.lib().sw_forward_f64(self._plan, ctypes.byref(io), _stream()))
        return ForwardResult(traces, fields, nrun % 2, snaps, None, 0)

    # ---- tiling -------------------------------------------------------------
    def set_tiling(self, tx=0, nw=0, zc=0, nt=-1, pf=0, wt=0, ts=0, occ=-1, order=0):
        """Stencil tile shape, z-chunk length, cache policy, prefetch distance,
        wave-tile mode, time steps per sweep, resident-block cap per CU and
        block order (0 / -1: default; occ=0: no cap; order 1: y tiles fastest,
        2: x tiles fastest)."""
        t = L.Tiling(tx, nw, zc, nt, pf, wt, ts, occ, order)
        L.check("sw_plan_set_tiling", L.lib().sw_plan_set_tiling(self._plan, ctypes.byref(t)))

    @property
    def tiling(self):
        t = L.Tiling()
        L.check("sw_plan_get_tiling", L.lib().sw_plan_get_tiling(self._plan, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in L.Tiling._fields_}

    @property
    def occupancy(self):
        """(resident blocks per CU, CUs) of the stencil kernel under the current
        tiling: 3D constant-density block tiles on a device, else (0, 0)."""
        n, c = ctypes.c_int32(), ctypes.c_int32()
        L.check("sw_plan_occupancy", L.lib().sw_plan_occupancy(self._plan, ctypes.byref(n), ctypes.byref(c)))
        return n.value, c.value

    def autotune(self, cache_path=None):
        """Time candidate tilings on scratch buffers and keep the fastest (or
        reuse the choice cached in the JSON file cache_path)."""
        fields = (self.new_field(), self.new_field())
        io = L.FwdIO()
        io.workspace = _ptr(self.workspace).value
        io.field[0], io.field[1] = fields[0].data_ptr(), fields[1].data_ptr()
        spare = self._spare_fields(force=True)
        if spare is not None:
            io.field2[0], io.field2[1] = spare[0].data_ptr(), spare[1].data_ptr()
        L.check("sw_plan_autotune", L.lib().sw_plan_autotune(
            self._plan, ctypes.byref(io), cache_path.encode() if cache_path else None, _stream()))

    def _spare_fields(self, force=False):
        """The two extra wavefield buffers of two-step sweeps (3D constant
        density), allocated once when the tiling uses them (or force)."""
        if self.ndim != 3 or self.scheme != "const":
            return None
        if not force and self.tiling["ts"] != 2:
            return None
        if getattr(self, "_field2", None) is None:
            self._field2 = (self.new_field(), self.new_field())
        return self._field2

    def _fwd_io(self, wavelet, fields, traces):
        lay = self.layout
        io = L.FwdIO()
        io.workspace = _ptr(self.workspace).value
        io.wavelet = wavelet.data_ptr() if lay.nsrc else None
        io.field[0], io.field[1] = fields[0].data_ptr(), fields[1].data_ptr()
        io.traces = traces.data_ptr() if lay.nrec else None
        return io

    # ---- propagation --------------------------------------------------------
    def forward(self, wavelet, saving_stride=0, checkpoint_every=0, use_graph=False, fields=None,
                step0=0, nsteps_run=None, traces=None, stencil_ms=None, check_finite=False):
        """Run steps step0 .. step0+nsteps_run-1 (all by default).  check_finite:
        wait for the run and raise (SW_ERR_NONFINITE) if a trace sample written
        or a value of the final wavefield is not finite.  stencil_ms: a
        host float32 numpy array of nsteps_run entries to receive each stencil
        launch's duration (the call then waits for the GPU)."""
        if self._vel is None:
            raise RuntimeError("prepare() must be called after the geometry is set")
        if self.dtype == "float64":
            if checkpoint_every or use_graph or stencil_ms is not None or check_finite:
                raise ValueError("the double-precision forward has no checkpoints, graphs, timing or checks")
            return self._forward64(wavelet, saving_stride, fields, step0, nsteps_run, traces)
        lay = self.layout
        nrun = self.nsteps - step0 if nsteps_run is None else int(nsteps_run)
        # drop the previous call's buffers first, so that the allocator can
        # hand them out again (work queued on the stream keeps its order)
        self._keep = None
        if fields is None:
            fields = (self.new_field(), self.new_field())
        if lay.nsrc:
            wavelet = wavelet.to(self.device, torch.float32).reshape(self.nsteps, lay.nsrc).contiguous()
        if traces is None:
            traces = torch.zeros((self.nsteps, max(0, lay.nrec)), dtype=torch.float32, device=self.device)
        snaps = None
        if saving_stride:
            nsnap = self.nsteps // saving_stride
            snaps = torch.zeros((nsnap,) + self.grid_shape, dtype=torch.float32, device=self.device)
        ckpt = None
        if checkpoint_every:
            nck = (self.nsteps + checkpoint_every - 1) // checkpoint_every
            ckpt = torch.zeros((nck, 2, lay.field_elems), dtype=torch.float32, device=self.device)
        io = L.FwdIO()
        io.workspace = _ptr(self.workspace).value
        io.wavelet = _ptr(wavelet if lay.nsrc else None).value
        io.field[0] = fields[0].data_ptr()
        io.field[1] = fields[1].data_ptr()
        io.traces = traces.data_ptr() if lay.nrec else None
        io.snaps = snaps.data_ptr() if snaps is not None else None
        io.saving_stride = int(saving_stride)
        io.ckpt = ckpt.data_ptr() if ckpt is not None else None
        io.ckpt_every = int(checkpoint_every)
        io.step0 = int(step0)
        io.nsteps_run = nrun
        io.use_graph = 1 if use_graph else 0
        io.check_finite = 1 if check_finite else 0
        if stencil_ms is not None:
            assert stencil_ms.dtype.name == "float32" and stencil_ms.size >= nrun
            io.stencil_ms = stencil_ms.ctypes.data_as(L.c_float_p)
        spare = self._spare_fields()
        if spare is not None:
            io.field2[0], io.field2[1] = spare[0].data_ptr(), spare[1].data_ptr()
        self._keep = (wavelet, fields, traces, snaps, ckpt)
        L.check("sw_forward", L.lib().sw_forward(self._plan, ctypes.byref(io), _stream()))
        return ForwardResult(traces, fields, nrun % 2, snaps, ckpt, int(checkpoint_every))

    def adjoint(self, wavelet, residual, ckpt, checkpoint_every, want_src_adjoint=False):
        """Velocity gradient (physical grid) of 1/2 |traces - d_obs|^2 given the
        residual dJ/dtraces and the forward checkpoints: (dJ/dc, F^T r or None,
        dJ/dM on the extended grid).  Staggered variable-density plans return a
        fourth element, dJ/drho on the physical grid."""
        lay = self.layout
        fe = lay.field_elems
        dev = self.device
        vd = self.scheme == "vd_staggered"
        self._keep_adj = None          # the previous call's scratch can be reused
        work = [torch.empty(fe, dtype=torch.float32, device=dev) for _ in range(4)]
        segment = torch.empty(((2 if vd else 1) * checkpoint_every, fe), dtype=torch.float32, device=dev)
        grad_m = torch.empty(fe, dtype=torch.float32, device=dev)
        grad_vel = torch.empty(self.n, dtype=torch.float32, device=dev)
        grad_rho = torch.empty(self.n, dtype=torch.float32, device=dev) if vd else None
        vd_work = torch.empty((4, fe), dtype=torch.float32, device=dev) if vd else None
        src_adj = None
        if want_src_adjoint and lay.nsrc:
            src_adj = torch.zeros((self.nsteps, lay.nsrc), dtype=torch.float32, device=dev)
        residual = residual.to(dev, torch.float32).reshape(self.nsteps, lay.nrec).contiguous()
        if lay.nsrc:
            wavelet = wavelet.to(dev, torch.float32).reshape(self.nsteps, lay.nsrc).contiguous()
        io = L.AdjIO()
        io.workspace = _ptr(self.workspace).value
        io.vel = self._vel.data_ptr()
        io.wavelet = wavelet.data_ptr() if lay.nsrc else None
        io.residual = residual.data_ptr()
        io.ckpt = ckpt.data_ptr()
        io.ckpt_every = int(checkpoint_every)
        io.field[0], io.field[1] = work[0].data_ptr(), work[1].data_ptr()
        io.adj[0], io.adj[1] = work[2].data_ptr(), work[3].data_ptr()
        io.segment = segment.data_ptr()
        io.grad_m = grad_m.data_ptr()
        io.grad_vel = grad_vel.data_ptr()
        io.src_adjoint = src_adj.data_ptr() if src_adj is not None else None
        if vd:
            io.grad_rho = grad_rho.data_ptr()
            io.vd_work = vd_work.data_ptr()
        self._keep_adj = (work, segment, grad_m, residual, wavelet, vd_work)
        L.check("sw_adjoint", L.lib().sw_adjoint(self._plan, ctypes.byref(io), _stream()))
        if vd:
            return grad_vel, src_adj, grad_m, grad_rho
        return grad_vel, src_adj, grad_m


class Batch:
    """Many prepared constant-density propagators (shots) advanced together:
    one persistent stencil launch per step over the tiles of all shots, one
    batched injection and one batched recording launch."""

    def __init__(self, props):
        self.props = list(props)
        arr = (ctypes.c_void_p * len(self.props))(*[p._plan.value for p in self.props])
        handle = ctypes.c_void_p()
        L.check("sw_batch_create", L.lib().sw_batch_create(len(self.props), arr, ctypes.byref(handle)))
        self._batch = handle
        nbytes = ctypes.c_int64()
        L.check("sw_batch_layout", L.lib().sw_batch_layout(self._batch, ctypes.byref(nbytes)))
        dev = self.props[0].device
        self.table = torch.empty(max(256, nbytes.value), dtype=torch.uint8, device=dev)
        self.fields = [(p.new_field(), p.new_field()) for p in self.props]
        self.traces = [torch.zeros((p.nsteps, max(0, p.layout.nrec)), dtype=torch.float32, device=dev)
                       for p in self.props]

    def __del__(self):
        try:
            if getattr(self, "_batch", None):
                L.lib().sw_batch_destroy(self._batch)
                self._batch = None
        except Exception:
            pass

    def _io(self, wavelets, nsteps_run, use_graph):
        self._wav = [w.to(p.device, torch.float32).reshape(p.nsteps, -1).contiguous()
                     for p, w in zip(self.props, wavelets)]
        shots = (L.FwdIO * len(self.props))()
        for k, p in enumerate(self.props):
            shots[k] = p._fwd_io(self._wav[k], self.fields[k], self.traces[k])
        io = L.BatchIO()
        io.shots = shots
        io.table = self.table.data_ptr()
        io.nsteps_run = int(nsteps_run)
        io.use_graph = 1 if use_graph else 0
        self._shots = shots
        return io

    def set_tiling(self, tx=0, nw=0, zc=0, nt=1, pf=1, blocks_per_cu=0):
        """Tile shape, z-chunk length, cache policy and prefetch distance of the
        batch launch, and its grid (blocks_per_cu 0: default persistent grid,
        -1: one block per tile); tx 0: the defaults."""
        t = L.Tiling(tx, nw, zc, nt, pf, 0, 1, 0, 1) if tx else None
        L.check("sw_batch_set_tiling", L.lib().sw_batch_set_tiling(
            self._batch, ctypes.byref(t) if t is not None else None, int(blocks_per_cu)))

    @property
    def tiling(self):
        t, bpc = L.Tiling(), ctypes.c_int32()
        L.check("sw_batch_get_tiling", L.lib().sw_batch_get_tiling(self._batch, ctypes.byref(t), ctypes.byref(bpc)))
        out = {k: getattr(t, k) for k in ("tx", "nw", "zc", "nt", "pf")}
        out["blocks_per_cu"] = bpc.value
        return out

    def autotune(self, wavelets, cache_path=None):
        io = self._io(wavelets, self.props[0].nsteps, False)
        L.check("sw_batch_autotune", L.lib().sw_batch_autotune(
            self._batch, ctypes.byref(io), cache_path.encode() if cache_path else None, _stream()))

    def forward(self, wavelets, nsteps_run=None, use_graph=False):
        """Run all shots; returns the list of trace tensors (one per shot)."""
        n = self.props[0].nsteps if nsteps_run is None else nsteps_run
        io = self._io(wavelets, n, use_graph)
        L.check("sw_batch_forward", L.lib().sw_batch_forward(self._batch, ctypes.byref(io), _stream()))
        self.current = n % 2
        return self.traces


    def forward_static(self, wavelets, nsteps_run=None):
        """The same run through the no-allocation entry point: the descriptor
        table lives in the library's fixed device array (self.table unused);
        launches are enqueued eagerly."""
        n = self.props[0].nsteps if nsteps_run is None else nsteps_run
        io = self._io(wavelets, n, False)
        io.table = None
        L.check("sw_batch_forward_static", L.lib().sw_batch_forward_static(self._batch, ctypes.byref(io),
                                                                            _stream()))
        self.current = n % 2
        return self.traces


class AcousticForward(torch.autograd.Function):
    """traces = F(vel); backward gives dJ/dvel by the hand-written adjoint with
    checkpointed recomputation of the forward wavefield."""

    @staticmethod
    def forward(ctx, vel, prop, wavelet, checkpoint_every):
        vel = vel.detach().to(prop.device, torch.float32).contiguous()
        prop.prepare(vel)
        res = prop.forward(wavelet, checkpoint_every=checkpoint_every)
        ctx.prop = prop
        ctx.vel = vel
        ctx.wavelet = wavelet
        ctx.ckpt = res.ckpt
        ctx.every = checkpoint_every
        return res.traces.clone()

    @staticmethod
    def backward(ctx, grad_traces):
        prop = ctx.prop
        if prop._vel is None or prop._vel.data_ptr() != ctx.vel.data_ptr():
            prop.prepare(ctx.vel)      # the plan was re-prepared since this forward
        g, _, _ = prop.adjoint(ctx.wavelet, grad_traces, ctx.ckpt, ctx.every)
        return g, None, None, None


class AcousticForwardVD(torch.autograd.Function):
    """traces = F(vel, rho) for a staggered variable-density propagator;
    backward gives (dJ/dvel, dJ/drho) by the hand-written adjoint with
    checkpointed recomputation of the forward wavefield."""

    @staticmethod
    def forward(ctx, vel, rho, prop, wavelet, checkpoint_every):
        if prop.scheme != "vd_staggered":
            raise ValueError("AcousticForwardVD needs a staggered variable-density propagator")
        vel = vel.detach().to(prop.device, torch.float32).contiguous()
        rho = rho.detach().to(prop.device, torch.float32).contiguous()
        prop.prepare(vel, rho)
        res = prop.forward(wavelet, checkpoint_every=checkpoint_every)
        ctx.prop = prop
        ctx.vel, ctx.rho = vel, rho
        ctx.wavelet = wavelet
        ctx.ckpt = res.ckpt
        ctx.every = checkpoint_every
        return res.traces.clone()

    @staticmethod
    def backward(ctx, grad_traces):
        prop = ctx.prop
        if (prop._vel is None or prop._vel.data_ptr() != ctx.vel.data_ptr() or
                prop._rho is None or prop._rho.data_ptr() != ctx.rho.data_ptr()):
            prop.prepare(ctx.vel, ctx.rho)      # the plan was re-prepared since this forward
        gv, _, _, gr = prop.adjoint(ctx.wavelet, grad_traces, ctx.ckpt, ctx.every)
        return gv, gr, None, None, None
