"""Seeded synthetic workloads: velocity/density models, geometry and sizes.

This module holds inputs only: model arrays, point coordinates, grid sizes,
step counts, seeds, peak frequencies and the CFL fraction.  It contains none
of the propagator's arithmetic (no stencil coefficients, no stability limit,
no wavelet, no interpolation weights): each side computes those itself from
these inputs.

The configurations stand in for the paper's Marmousi2 / Overthrust models,
which are not available here; they have the shapes, value ranges and
structure of the configurations listed in the benchmark plan:

  homogeneous_2d   201 x 201, h = 10 m, v = 1500 m/s, SO8, 500 steps, Ricker
                   10 Hz at the centre node, 101 receivers at 50 m depth.
  layered_3d       256^3, h = 10 m, 5 flat layers 1500..4500 m/s plus
                   i.i.d. N(0, 50^2) per node (seed 2), SO16, 1000 steps,
                   Ricker 15 Hz off-grid source (Kaiser-sinc r = 4),
                   128 x 128 surface receivers every 2 nodes.
  smooth_3d        512^3, h = 10 m, smooth random velocity 1500..4500 m/s
                   (white noise on a 64^3 grid, seed 3, Gaussian filter of
                   1.5 coarse cells with wrap-around, trilinear upsampling by
                   8, affine map), density from Gardner's rule 310 v^0.25,
                   SO8, 2000 steps, Ricker 12 Hz, trilinear source and
                   256 x 256 receivers.
  batch_3d         64 shots on grids drawn from U{160..256} x U{160..320}^2
                   (seed 4), each with 3..8 flat layers (seed 400 + shot),
                   Ricker 10..20 Hz, SO8, 1000 steps, 64 x 64 receivers.
  gradient_3d      320^3 layered + N(0, 50^2) model (seed 5) and the smooth
                   layered reference it perturbs, 8 sources on a 2 x 4
                   surface grid, 64 x 64 receivers, SO8, 1500 steps.

Every configuration adds a 40-cell absorbing layer on each side.  Sizes can be
scaled down for tests with the `n` / `nsteps` arguments.

The paper's own benchmark shapes ("Performance evaluation", with the boundary
set-up of its two examples) are stand-ins too (the Marmousi2 and Overthrust
models are not used):

  paper_shape_2d   351 x 1701 physical nodes, h = 10 m, layer 70 cells on the
                   bottom and both sides, none on top; Neumann top, Dirichlet
                   elsewhere; 6 flat layers 1500..4700 m/s + N(0, 20^2)
                   (seed 7, capped at 4700); 101 receivers at 10 m depth.
  paper_shape_3d   207 x 801 x 801 nodes, h = 20 m, no layer; Neumann top,
                   Dirichlet elsewhere; the same recipe up to 6000 m/s.
"""
from dataclasses import dataclass, field

import numpy as np

CFL_FRACTION = 0.5     # dt = 0.5 * dt_crit(c_max of the model)
LAYER = 40


@dataclass
class Workload:
    name: str
    n: tuple
    h: tuple
    space_order: int
    nsteps: int
    f_peak: float
    vel: np.ndarray
    rho: np.ndarray = None
    scheme: str = "const"
    nbl: int = LAYER
    src: np.ndarray = None          # (nsrc, ndim) metres
    rec: np.ndarray = None          # (nrec, ndim) metres
    src_interp: str = "hicks"
    rec_interp: str = "hicks"
    radius: int = 4
    extra: dict = field(default_factory=dict)
    bc: tuple = None                # per axis (low, high) ghost condition, None: zero ghosts

    @property
    def cmax(self):
        return float(self.vel.max())

    @property
    def ndim(self):
        return len(self.n)


def layered(shape, speeds, rng=None, sigma=0.0):
    """Flat layers of equal thickness along axis 0, plus N(0, sigma^2) noise."""
    v = np.empty(shape, dtype=np.float32)
    edges = np.linspace(0, shape[0], len(speeds) + 1).round().astype(int)
    for k, s in enumerate(speeds):
        v[edges[k]:edges[k + 1]] = s
    if sigma > 0.0:
        v += rng.normal(0.0, sigma, size=shape).astype(np.float32)
    return v


def smooth_random(shape, seed, factor=8, sigma=1.5, vmin=1500.0, vmax=4500.0):
    """Smooth random field mapped affinely onto [vmin, vmax]."""
    import torch
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    coarse_shape = tuple(max(2, -(-s // factor)) for s in shape)
    w = gaussian_filter(rng.standard_normal(coarse_shape), sigma, mode="wrap")
    t = torch.from_numpy(w.astype(np.float32))[None, None]
    mode = "trilinear" if len(shape) == 3 else "bilinear"
    up = torch.nn.functional.interpolate(t, size=tuple(c * factor for c in coarse_shape), mode=mode,
                                         align_corners=False)[0, 0].numpy()
    up = up[tuple(slice(0, s) for s in shape)]
    lo, hi = float(up.min()), float(up.max())
    return (vmin + (vmax - vmin) * (up - lo) / (hi - lo)).astype(np.float32)


def gardner(vel):
    return (310.0 * np.power(vel.astype(np.float64), 0.25)).astype(np.float32)


def homogeneous_2d(n=201, nsteps=500, h=10.0):
    vel = np.full((n, n), 1500.0, dtype=np.float32)
    centre = (n - 1) // 2 * h
    rec_x = np.arange(0.0, (n - 1) * h + 1e-9, 2 * h)
    rec = np.stack([np.full_like(rec_x, 5 * h), rec_x], axis=1)
    return Workload("homogeneous_2d", (n, n), (h, h), 8, nsteps, 10.0, vel,
                    src=np.array([[centre, centre]]), rec=rec)


def layered_3d(n=256, nsteps=1000, h=10.0, space_order=16, seed=2, rec_stride=2, nrec_side=128):
    rng = np.random.default_rng(seed)
    vel = layered((n, n, n), [1500.0, 2250.0, 3000.0, 3750.0, 4500.0], rng, 50.0)
    centre = (n // 2) * h
    src = np.array([[2 * h + 0.3 * h, centre + 0.25 * h, centre + 0.4 * h]])
    k = np.arange(min(nrec_side, (n - 1) // rec_stride + 1)) * rec_stride * h
    gx, gy = np.meshgrid(k, k, indexing="ij")
    rec = np.stack([np.zeros(gx.size), gx.ravel(), gy.ravel()], axis=1)
    return Workload("layered_3d", (n, n, n), (h, h, h), space_order, nsteps, 15.0, vel,
                    src=src, rec=rec)


def smooth_3d(n=512, nsteps=2000, h=10.0, scheme="vd_staggered", seed=3, nrec_side=256,
              rec_spacing=20.0):
    vel = smooth_random((n, n, n), seed)
    rho = gardner(vel) if scheme != "const" else None
    ext = (n - 1) * h
    src = np.array([[5.23 * h, 0.5008 * ext, 0.4993 * ext]])
    k = 0.5 * h + rec_spacing * np.arange(nrec_side)
    k = k[k <= ext]
    gx, gy = np.meshgrid(k, k, indexing="ij")
    rec = np.stack([np.full(gx.size, 2.46 * h), gx.ravel(), gy.ravel()], axis=1)
    return Workload("smooth_3d", (n, n, n), (h, h, h), 8, nsteps, 12.0, vel, rho=rho,
                    scheme=scheme, src=src, rec=rec, src_interp="linear", rec_interp="linear")


def gradient_3d(n=320, nsteps=1500, h=10.0, seed=5, nrec_side=64, rec_stride=5):
    rng = np.random.default_rng(seed)
    speeds = [1500.0, 2250.0, 3000.0, 3750.0, 4500.0]
    reference = layered((n, n, n), speeds)
    current = layered((n, n, n), speeds, rng, 50.0)
    ext = (n - 1) * h
    sx = np.linspace(0.25, 0.75, 2) * ext
    sy = np.linspace(0.2, 0.8, 4) * ext
    src = np.array([[2 * h, a, b] for a in sx for b in sy])
    k = np.arange(min(nrec_side, (n - 1) // rec_stride + 1)) * rec_stride * h
    gx, gy = np.meshgrid(k, k, indexing="ij")
    rec = np.stack([np.zeros(gx.size), gx.ravel(), gy.ravel()], axis=1)
    return Workload("gradient_3d", (n, n, n), (h, h, h), 8, nsteps, 10.0, current,
                    src=src, rec=rec, extra={"reference": reference})


def batch_3d(nshots=64, nsteps=1000, h=10.0, seed=4, nrec_side=64, size_scale=1.0):
    """Shot list for batched propagation: uneven grids, own layered models."""
    rng = np.random.default_rng(seed)
    shots = []
    for s in range(nshots):
        nz = int(rng.integers(160, 257) * size_scale)
        nx = int(rng.integers(160, 321) * size_scale)
        ny = int(rng.integers(160, 321) * size_scale)
        r2 = np.random.default_rng(400 + s)
        nl = int(r2.integers(3, 9))
        speeds = np.sort(r2.uniform(1500.0, 4500.0, nl)).astype(np.float32)
        vel = layered((nz, nx, ny), list(speeds))
        f = float(r2.uniform(10.0, 20.0))
        src = np.array([[2 * h, (nx - 1) // 2 * h, (ny - 1) // 2 * h]])
        kx = np.linspace(0, nx - 1, nrec_side).round() * h
        ky = np.linspace(0, ny - 1, nrec_side).round() * h
        gx, gy = np.meshgrid(kx, ky, indexing="ij")
        rec = np.stack([np.zeros(gx.size), gx.ravel(), gy.ravel()], axis=1)
        shots.append(Workload(f"shot{s}", (nz, nx, ny), (h, h, h), 8, nsteps, f, vel,
                              src=src, rec=rec))
    return shots


def _paper_layers(n, cmax, seed=7):
    rng = np.random.default_rng(seed)
    speeds = np.linspace(1500.0, cmax, 6)
    vel = layered(n, list(speeds))
    return np.minimum(vel + rng.normal(0.0, 20.0, n).astype(np.float32), np.float32(cmax)).astype(np.float32)


def paper_shape_2d(space_order=8, nsteps=None, tf=2.0):
    """The 2D benchmark shape (421 x 1841 nodes with the layer); nsteps None:
    the caller takes the step count from the stability limit and tf."""
    n, h, cmax = (351, 1701), 10.0, 4700.0
    vel = _paper_layers(n, cmax)
    ext = [h * (k - 1) for k in n]
    src = np.array([[2 * h, ext[1] / 2]])
    rec = np.array([[h, ext[1] * (i / 100.0)] for i in range(101)])
    wl = Workload("paper_shape_2d", n, (h, h), space_order, nsteps or 0, 10.0, vel,
                  nbl=((0, 70), (70, 70)), src=src, rec=rec, src_interp="linear", rec_interp="linear",
                  extra={"cmax": cmax, "tf": tf},
                  bc=(("neumann", "dirichlet"), ("dirichlet", "dirichlet")))
    return wl


def paper_shape_3d(space_order=8, nsteps=None, tf=4.0):
    """The 3D benchmark shape (207 x 801 x 801 nodes, no layer)."""
    n, h, cmax = (207, 801, 801), 20.0, 6000.0
    vel = _paper_layers(n, cmax)
    ext = [h * (k - 1) for k in n]
    src = np.array([[2 * h, ext[1] / 2, ext[2] / 2]])
    rec = np.array([[h, ext[1] * (i / 100.0), ext[2] / 2] for i in range(101)])
    return Workload("paper_shape_3d", n, (h, h, h), space_order, nsteps or 0, 10.0, vel,
                    nbl=((0, 0), (0, 0), (0, 0)), src=src, rec=rec, src_interp="linear", rec_interp="linear",
                    extra={"cmax": cmax, "tf": tf},
                    bc=(("neumann", "dirichlet"), ("dirichlet", "dirichlet"), ("dirichlet", "dirichlet")))
