/*
 * simwave_hip — explicit finite-difference acoustic propagator for MI355X (gfx950).
 *
 * C ABI of libsimwave_hip.so.  Every entry point is extern "C", takes plain
 * host or device pointers and sizes, never throws, never exits and never
 * allocates caller-visible device memory: the caller (for instance PyTorch)
 * allocates every device buffer with the sizes reported by sw_plan_layout or
 * sw_batch_layout and passes a HIP stream (hipStream_t, as void*).  Calls that
 * launch work only enqueue it on that stream and return.  On any error the
 * call returns a non-zero sw_status before enqueueing anything, and
 * sw_last_error() gives a message for the calling thread.
 *
 * The problem statement follows the paper (sections "Governing equations",
 * "Boundary conditions and domain truncation", "Time discretization",
 * "Space discretization", "Sources and receivers", "Example of use"):
 *
 *   - a regular grid of n[i] physical nodes with spacing h[i] per axis, axis
 *     order (z, x) in 2D and (z, x, y) in 3D, the last axis fastest;
 *   - an absorbing layer of nbl[i][side] cells added outside the physical
 *     grid, where the damped equation p_tt + 2 eta p_t - c^2 lap p = f holds
 *     with eta = damp_alpha * d^damp_power, d the Euclidean distance in cells
 *     to the physical node box (eta = 0 inside); velocity and density are
 *     copied from the nearest physical node into the layer;
 *   - second-order central differences in time, giving the explicit update
 *       p^{n+1} = A (2 p^n + K (L p^n)) - B p^{n-1},
 *       A = 1/(1 + eta dt),  B = (1 - eta dt)/(1 + eta dt),
 *     with p^{-1} = p^0 = 0;
 *   - the spatial operator L of space order SO = 2r (even, 2..20):
 *       SW_CONST        centred Laplacian, K = dt^2 c^2;
 *       SW_VD_CENTRED   Laplacian minus (grad rho / rho) . grad p with centred
 *                       first derivatives (the paper's expanded
 *                       variable-density form), K = dt^2 c^2;
 *       SW_VD_STAGGERED conservative div(b grad p), b = 1/rho, with half-node
 *                       first derivatives and order-SO midpoint interpolation
 *                       of b, K = dt^2 rho c^2;
 *   - sources injected after the stencil update as
 *       p^{n+1} += A dt^2 c^2 (d / dV) S_s(t_n)
 *     (d the interpolation weight, dV the cell volume) and receivers recording
 *       rec[n] = sum d p^{n+1}
 *     with Kaiser-windowed sinc weights (half-width r_w, shape b) or linear
 *     (trilinear in 3D) weights.
 *
 * Device memory layout of wavefield and model buffers ("padded layout"):
 * an array of padded[0] x padded[1] x padded[2] floats (2D: padded[2] = 1 is
 * not used; the last used axis is the pitch axis) whose node (i0, i1[, i2]) of
 * the extended grid sits at element
 *     origin + (i0 * padded[1] + i1) * padded[2] + i2          (3D)
 *     origin + i0 * padded[1] + i1                             (2D)
 * The halo around the extended grid is stored and must stay zero in
 * wavefield buffers (the library never writes it after clearing the buffer).
 * Interior rows start on 256-byte boundaries if the buffer base is 256-byte
 * aligned.
 */
#ifndef SIMWAVE_HIP_H
#define SIMWAVE_HIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SW_ABI_VERSION 1

typedef enum sw_status {
    SW_OK = 0,
    SW_ERR_ARG = 1,          /* invalid argument (null pointer, bad size, ...) */
    SW_ERR_UNSUPPORTED = 2,  /* valid but not provided (odd or >16 order, mirror ghosts in
                                the adjoint, ...) */
    SW_ERR_DOMAIN = 3,       /* a point lies outside the physical grid or its footprint
                                leaves the extended grid */
    SW_ERR_CFL = 4,          /* dt above the stability limit */
    SW_ERR_STATE = 5,        /* call out of order (e.g. forward before model prepare) */
    SW_ERR_WORKSPACE = 6,    /* workspace missing or misaligned */
    SW_ERR_HIP = 7,          /* a HIP runtime call failed */
    SW_ERR_NONFINITE = 8     /* non-finite values found where a check was requested */
} sw_status;

enum { SW_CONST = 0, SW_VD_STAGGERED = 1, SW_VD_CENTRED = 2 };
enum { SW_BC_NONE = 0, SW_BC_DIRICHLET = 1, SW_BC_NEUMANN = 2 };
enum { SW_SRC = 0, SW_REC = 1 };
enum { SW_INTERP_HICKS = 0, SW_INTERP_LINEAR = 1 };
enum { SW_F32 = 0, SW_F64 = 1 };

/* Problem description (paper: SpaceModel, config_boundary, TimeModel). */
typedef struct sw_problem {
    int32_t ndim;           /* 2 or 3 */
    int32_t n[3];           /* physical nodes per axis (z, x[, y]); unused axis: 1 */
    double  h[3];           /* grid spacing per axis, metres */
    int32_t space_order;    /* even, 2..20 (paper, "Space discretization") */
    int32_t scheme;         /* SW_CONST, SW_VD_STAGGERED or SW_VD_CENTRED */
    int32_t nbl[3][2];      /* absorbing layer cells (low side, high side) per axis */
    int32_t bc[3][2];       /* ghost condition per side at the edge of the extended grid
                               (paper, "Boundary conditions and domain truncation"):
                               SW_BC_NONE (ghosts read zero), SW_BC_DIRICHLET (odd
                               mirror about the boundary node, which is held at zero)
                               or SW_BC_NEUMANN (even mirror).  Mirror sides need at
                               least R + 1 nodes (2R staggered) along their axis, are
                               served by the forward with single sweeps of block
                               tiles, and are refused by the adjoint and batches. */
    double  damp_alpha;     /* alpha of eta = alpha d^p (paper default 0.001) */
    double  damp_power;     /* p (paper default 3) */
    double  dt;             /* time step, seconds */
    int32_t nsteps;         /* number of time steps N */
    int32_t dtype;          /* SW_F32 (0: single precision, every entry point) or SW_F64
                               (double precision, as the paper's dtype option: constant
                               density forward only, through sw_model_prepare_f64 and
                               sw_forward_f64) */
} sw_problem;

/* Sizes of every caller-allocated buffer for a plan. */
typedef struct sw_layout {
    int32_t ndim;
    int32_t dims[3];        /* extended grid extents (physical + layer) */
    int32_t halo;           /* zero ghost cells stored on each side */
    int32_t padded[3];      /* padded extents, last used axis = pitch */
    int64_t origin;         /* element offset of extended-grid node 0 */
    int64_t field_elems;    /* floats per wavefield or model buffer */
    int64_t grid_nodes;     /* nodes of the extended grid */
    int64_t physical_nodes; /* nodes of the physical grid */
    int32_t nsrc;           /* sources set with sw_plan_set_geometry */
    int32_t nrec;           /* receivers set with sw_plan_set_geometry */
    int64_t workspace_bytes;/* device workspace (model arrays and tables) */
} sw_layout;

/* ---- version and errors ------------------------------------------------ */

/* SW_ABI_VERSION of the built library. */
int32_t sw_abi_version(void);
/* Static string naming a status code. */
const char *sw_status_str(sw_status s);
/* Message of the last failed call on this thread ("" if none); valid until
 * the next call on this thread. */
const char *sw_last_error(void);

/* ---- host helpers (no device work) ------------------------------------- */

/* Stability limit of the leapfrog update (paper, "Time discretization",
 * stability condition): dt_crit = 2 / (cmax sqrt(sum_i a / h_i^2)) with
 * a = |v_0| + 2 sum_j |v_j| the magnitude sum of the order-`space_order`
 * second-derivative coefficients.  h has ndim entries.  Writes *dt. */
sw_status sw_critical_dt(int32_t ndim, const double *h, int32_t space_order, double cmax,
                         double *dt);
/* Number of time levels for total time tf: ceil(tf / dt) + 1.  Writes *n. */
sw_status sw_steps_for(double tf, double dt, int32_t *n);
/* Ricker wavelet of peak frequency f (paper, "Sources and receivers", default
 * wavelet): S(t) = (1 - 2 pi^2 f^2 (t - t0)^2) exp(-pi^2 f^2 (t - t0)^2)
 * sampled at t_k = k dt, k = 0..n-1, into the host array out[n].  t0 <= 0
 * selects t0 = 1/f. */
sw_status sw_ricker(double f, double t0, double dt, int32_t n, float *out);

/* ---- plans --------------------------------------------------------------- */

typedef struct sw_plan sw_plan;

/* Validate the problem and build a plan (host tables: coefficients, damping
 * table).  Checks dt against the stability limit is left to the model
 * prepare call, which knows c_max.  *out receives a plan owned by the caller
 * and released with sw_plan_destroy.  SW_ERR_UNSUPPORTED if a padded z plane
 * times (4R + 2) reaches 2^31 bytes (the kernels address a window of planes
 * with 32-bit offsets), e.g. planes beyond about 3800^2 nodes at SO16. */
sw_status sw_plan_create(const sw_problem *prob, sw_plan **out);
sw_status sw_plan_destroy(sw_plan *plan);
/* Fill *out with the buffer sizes of the plan (after geometry is set the
 * workspace size includes the point tables). */
sw_status sw_plan_layout(const sw_plan *plan, sw_layout *out);

/* Set the sources (which = SW_SRC) or receivers (SW_REC) of the plan.
 * coords: host array count x ndim of positions in metres measured from the
 * first physical node, axis order as the grid.  interp: SW_INTERP_HICKS
 * (Kaiser-windowed sinc of half-width `radius`, 1..10, shape kaiser_b; a
 * kaiser_b <= 0 selects 6.31 for radius 4 and is an error otherwise) or
 * SW_INTERP_LINEAR (radius and kaiser_b ignored).  Errors: SW_ERR_DOMAIN if a
 * point lies outside the physical grid or its footprint leaves the extended
 * grid.  count may be 0.  Invalidates a previous model prepare. */
sw_status sw_plan_set_geometry(sw_plan *plan, int32_t which, int32_t count, const double *coords,
                               int32_t interp, int32_t radius, double kaiser_b);

/* Host copy of a point table, for inspection: entries (padded-layout element
 * offset of the node, point index, interpolation weight), grouped by point.
 * Call with nodes = ids = weights = NULL to get the entry count in *nent;
 * then pass arrays of at least *nent entries (any of them may be NULL). */
sw_status sw_plan_points(const sw_plan *plan, int32_t which, int64_t *nent, int64_t *nodes,
                         int32_t *ids, float *weights);

/* Build the device model arrays of the plan in `workspace` (device, at least
 * layout.workspace_bytes, 256-byte aligned) from the physical-grid velocity
 * vel_dev (device floats, physical_nodes, C order) and, for the
 * variable-density schemes, density rho_dev (same shape; NULL otherwise):
 * edge replication into the layer and ghosts, dt^2 c^2 (and rho or 1/rho),
 * the damping table and the point tables.  cmax is the largest velocity of
 * the model (the caller knows it; used for the stability check):
 * SW_ERR_CFL if dt exceeds the limit.  Enqueued on `stream`. */
sw_status sw_model_prepare(sw_plan *plan, const float *vel_dev, const float *rho_dev,
                           double cmax, void *workspace, void *stream);

/* ---- forward propagation (paper: Solver.forward) ------------------------ */

typedef struct sw_fwd_io {
    void *workspace;          /* prepared by sw_model_prepare */
    const float *wavelet;     /* device [nsteps][nsrc]: S_s(t_n) */
    float *field[2];          /* device, field_elems floats each.  On entry field[0]
                                 holds p^{step0} and field[1] p^{step0-1}; if step0 == 0
                                 both are cleared first.  On return p^{end} is in
                                 field[nsteps_run % 2] and p^{end-1} in the other. */
    float *traces;            /* device [nsteps][nrec]; row n written for the steps run;
                                 may be NULL when nrec == 0 */
    float *snaps;             /* device [nsteps / saving_stride][grid_nodes] dense
                                 extended-grid snapshots of p^{n+1} for every step n with
                                 (n+1) % saving_stride == 0, slot (n+1)/saving_stride - 1;
                                 NULL or saving_stride == 0 for none */
    int32_t saving_stride;
    float *ckpt;              /* device [ceil(nsteps/ckpt_every)][2][field_elems]:
                                 slot k holds (p^{k e}, p^{k e - 1}), e = ckpt_every;
                                 NULL for none */
    int32_t ckpt_every;
    int32_t step0;            /* first step to run (0 = start) */
    int32_t nsteps_run;       /* number of steps to run */
    int32_t use_graph;        /* 1: capture the step loop in a HIP graph and launch it */
    float *stencil_ms;        /* host [nsteps_run] or NULL: if given, HIP events are recorded
                                 on `stream` around each stencil launch, the call waits for
                                 them and writes, for every step, the duration in
                                 milliseconds of the launch that advanced it divided by
                                 the number of steps that launch advanced (1 or 2)
                                 (not combinable with use_graph) */
    float *field2[2];         /* device, field_elems floats each, or NULL: two more
                                 wavefield buffers.  With both given and a tiling of
                                 ts = 2, steps run in two-step sweeps (four steps at a
                                 time: field -> field2 -> field); remaining steps and
                                 all other cases run singly.  Contents on return are
                                 unspecified; the result is in field[] as above. */
    int32_t check_finite;     /* 1: after the run, count the non-finite values among the
                                 trace rows written and the final wavefield p^{end}
                                 (waits for the stream); the call then returns
                                 SW_ERR_NONFINITE if there are any (an unstable dt or
                                 model), with the count in the error message */
} sw_fwd_io;

sw_status sw_forward(sw_plan *plan, const sw_fwd_io *io, void *stream);

/* ---- double precision (SW_F64 plans) ------------------------------------ */

/* Model preparation of an SW_F64 plan: K = dt^2 c^2 in double precision from
 * the device velocity vel_dev [physical_nodes] (double), the damping table and
 * the point coefficients, into the workspace (sw_plan_layout's
 * workspace_bytes, which counts 8-byte values for such a plan).  Errors as
 * for sw_model_prepare; SW_ERR_STATE for a single-precision plan. */
sw_status sw_model_prepare_f64(sw_plan *plan, const double *vel_dev, double cmax, void *workspace,
                               void *stream);

/* Buffers of the double-precision forward; meaning, sizes and ownership as in
 * sw_fwd_io, with double elements. */
typedef struct sw_fwd64_io {
    void *workspace;          /* prepared by sw_model_prepare_f64 */
    const double *wavelet;    /* device [nsteps][nsrc] */
    double *field[2];         /* device, field_elems doubles each (as sw_fwd_io) */
    double *traces;           /* device [nsteps][nrec] */
    double *snaps;            /* device [nsteps / saving_stride][grid_nodes] or NULL */
    int32_t saving_stride;
    int32_t step0;
    int32_t nsteps_run;
} sw_fwd64_io;

/* The forward of an SW_F64 plan (paper, "Time discretization" update with the
 * damped source term), stencil, injection, recording and mirror ghosts in
 * double precision; the same steps and outputs as sw_forward (no checkpoints,
 * graphs, two-step sweeps or timing).  Enqueue only. */
sw_status sw_forward_f64(sw_plan *plan, const sw_fwd64_io *io, void *stream);

/* ---- adjoint and velocity gradient -------------------------------------- */

typedef struct sw_adj_io {
    void *workspace;          /* as for the forward */
    const float *vel;         /* device [physical_nodes]: velocity the plan was prepared with */
    const float *wavelet;     /* the forward's wavelet */
    const float *residual;    /* device [nsteps][nrec]: dJ/d rec[n] */
    const float *ckpt;        /* forward checkpoints (ckpt_every as for the forward) */
    int32_t ckpt_every;
    float *field[2];          /* device work buffers (field_elems each) */
    float *adj[2];            /* device adjoint wavefield buffers (field_elems each) */
    float *segment;           /* device [ckpt_every][field_elems] recomputed
                                 dt^2 c^2 (L u^n + source) levels; staggered scheme:
                                 [2][ckpt_every][field_elems], the K L u^n levels and
                                 the levels u^n themselves */
    float *grad_m;            /* device field_elems: dJ/d(dt^2 c^2) on the extended grid
                                 (staggered scheme: dJ/dK, K = dt^2 rho c^2; cleared and
                                 accumulated by the call) */
    float *grad_vel;          /* device [physical_nodes]: dJ/dc (written) */
    float *src_adjoint;       /* device [nsteps][nsrc] adjoint of the source map, or NULL */
    /* staggered variable density only (ignored otherwise): */
    float *grad_rho;          /* device [physical_nodes]: dJ/drho (written) */
    float *vd_work;           /* device [4][field_elems] scratch: per-axis face imaging
                                 sums and the source imaging term */
} sw_adj_io;

/* Velocity gradient of J = 1/2 sum_n sum_k (rec[n][k] - d_obs[n][k])^2 for a
 * constant-density plan with zero ghosts: the adjoint wavefield
 *   phi^m = A (2 phi^{m+1} + M L phi^{m+1} + M P_r^T r^{m-1}) - B phi^{m+2}
 * (M = dt^2 c^2) is stepped from m = N down to 1 by the forward stencil, with
 * the residual spread by the receiver weights; the zero-lag imaging condition
 * accumulates dJ/dM = sum_n phi^{n+1} M (L u^n + Q s^n) / M^2 with u^n
 * recomputed segment by segment from the checkpoints; dJ/dc = dJ/dM 2 dt^2 c
 * summed back from the layer onto the physical node it copies.
 *
 * Staggered variable-density plans (zero ghosts) get velocity and density
 * gradients.  The operator L = -sum_i (D+_i)^T diag(b_i) D+_i is symmetric, so
 * the adjoint is the same stencil with K = dt^2 rho c^2 and the residual
 * entering with weight A K; per step n the call accumulates
 *   dJ/dK     += phi^{n+1} K L u^n / K^2          (fused into the stencil)
 *   dJ/db_f   -= (D+_i phi^{n+1}) (D+_i u^n)       (every face of every axis)
 *   S         += phi^{n+1} M q^n                   (source nodes; dJ/dM = S / (K M))
 * and then, per extended node, dJ/db by the transpose of the face buoyancy
 * interpolation, dJ/dc = 2 dt^2 c (dJ/dK rho + dJ/dM) and
 * dJ/drho = dJ/dK dt^2 c^2 - dJ/db / rho^2, folded onto the physical grid.
 * The centred variable-density scheme and mirror ghosts: SW_ERR_UNSUPPORTED. */
sw_status sw_adjoint(sw_plan *plan, const sw_adj_io *io, void *stream);

/* Stencil tiling of a plan.  Results never depend on it.
 *   tx, nw  rows per block and waves per block.  3D constant density:
 *           block tiles (16,4), (8,4), (32,8), (16,8), (8,8), (24,8), or with wt = 1
 *           wave tiles (16,4), (32,4), (4,1), (8,1), (16,2) (each wave owns
 *           tx / nw rows); 3D variable density: (16,8), (8,8), (8,4), (16,4);
 *           2D grids: fixed.  0, 0: default.
 *   zc      z-chunk length (0: default)
 *   nt      1: non-temporal loads/stores for the streamed arrays, 0: cached,
 *           -1: default
 *   pf      planes of loads in flight ahead of the update (1 or 2; 0: default;
 *           block tiles only)
 *   wt      1: wave tiles (see tx, nw)
 *   ts      time steps per sweep: 0 default, 1, or 2 (constant density, 3D,
 *           forward only: one launch reads p^n, p^{n-1}, K and writes
 *           p^{n+1}, p^{n+2}, evaluating the first step also on R ghost rows
 *           and columns around the tile; the tile is tx rows x (64 - 2R)
 *           columns; shapes (8,4), (16,8), (8,8), (16,4) where the register
 *           queues fit: (tx/nw)(5R+5) + ceil(2R/nw)(3R+3) <= 95, so up to R = 7).  Takes
 *           effect when sw_fwd_io.field2 is given.
 *   occ     resident blocks per CU at most, for single-step block tiles: the
 *           launch reserves 160 KiB / occ of LDS per block, so that fewer
 *           z streams share each L2 (3 .. 6; 0: no cap; -1: default).  The
 *           cap only lowers occupancy; where registers or LDS already allow
 *           fewer blocks it has no effect.  Other values: SW_ERR_ARG.
 *   order   block order of single-step block tiles within a z chunk: 0
 *           default, 1 y tiles fastest, 2 x tiles fastest (tiles that share
 *           the taller x halos then run side by side on an XCD). */
typedef struct sw_tiling {
    int32_t tx, nw, zc, nt, pf, wt, ts, occ, order;
} sw_tiling;

/* Set (t != NULL) or reset to the defaults (t == NULL) the tiling of a plan.
 * SW_F64 plans take a tile shape (8x8, 16x8, 8x4 or 24x8 in 3D) and a z chunk
 * only: wave tiles, two-step sweeps and occupancy caps are refused, and the
 * cache policy, prefetch depth and block order are ignored. */
sw_status sw_plan_set_tiling(sw_plan *plan, const sw_tiling *t);
/* The tiling the plan's stencil launches use (defaults resolved).  For 3D
 * block tiles in single precision on a device (every scheme), the default
 * z chunk is the one with the fewest whole rounds of resident blocks times
 * planes per block (chunks of 4r .. 100 planes making at least three rounds);
 * elsewhere (and without a device, or where no chunk qualifies) about 16000
 * waves per launch, chunks of at most 74 planes. */
sw_status sw_plan_get_tiling(const sw_plan *plan, sw_tiling *out);
/* Resident blocks per compute unit of the plan's stencil kernel under its
 * current tiling (the runtime's occupancy calculator) and the device's
 * compute units: set for 3D block tiles (every scheme and precision), 0
 * and 0 otherwise or without a device. */
sw_status sw_plan_occupancy(const sw_plan *plan, int32_t *blocks_per_cu, int32_t *cus);

/* ---- batched shots and autotuning --------------------------------------- */

typedef struct sw_batch sw_batch;

/* Group `nshots` prepared constant-density plans (each with its own grid
 * size, dt, model, geometry and workspace; all with the same ndim, space
 * order and step count) so that every time step advances all shots with one
 * stencil launch over a tile list spanning all shots, one batched
 * injection and one batched recording launch.  The plans stay owned by the
 * caller and must outlive the batch. */
sw_status sw_batch_create(int32_t nshots, sw_plan *const *plans, sw_batch **out);
sw_status sw_batch_destroy(sw_batch *batch);
/* Tiling of the batch stencil launch (t NULL: the defaults) and its grid:
 * blocks_per_cu > 0 persistent blocks per compute unit looping over the tile
 * list, -1 one block per tile, 0 the default (one block per tile for 3D
 * shots, 8 looping blocks per compute unit for 2D shots).  Plain tile
 * shapes only (wt 0, ts 1, occ 0; order is ignored; zc 0: the default chunk).
 * Results do not depend on any of it. */
sw_status sw_batch_set_tiling(sw_batch *batch, const sw_tiling *t, int32_t blocks_per_cu);
sw_status sw_batch_get_tiling(const sw_batch *batch, sw_tiling *out, int32_t *blocks_per_cu);
/* Bytes of the device descriptor table the caller allocates for the batch. */
sw_status sw_batch_layout(const sw_batch *batch, int64_t *table_bytes);

typedef struct sw_batch_io {
    const sw_fwd_io *shots;   /* host array [nshots]: per-shot workspace, wavelet, field[2],
                                 traces (snaps, ckpt, step0, nsteps_run ignored) */
    void *table;              /* device, sw_batch_layout bytes, 256-byte aligned */
    int32_t nsteps_run;       /* steps 0 .. nsteps_run-1 for every shot (fields cleared first) */
    int32_t use_graph;        /* 1: capture the loop in a HIP graph and launch it */
} sw_batch_io;

/* Run the batch (enqueue only).  On return shot s has p^{nsteps_run} in
 * shots[s].field[nsteps_run % 2]. */
sw_status sw_batch_forward(sw_batch *batch, const sw_batch_io *io, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the run of
 * sw_batch_forward with the batch's descriptor table held in a fixed device
 * array owned by the library (1 MiB per GPU, about 1400 shots; kept until
 * the process ends) instead of io->table, which is ignored.  Nothing is
 * allocated: the array's address is resolved once per device, and the call
 * enqueues the table upload and the launches on `stream` (io->use_graph must
 * be 0: the caller may capture them in a graph of its own).  A batch whose
 * table is larger than the array is refused (SW_ERR_UNSUPPORTED) before
 * anything is enqueued.  Every call on one GPU shares the array: calls that
 * overlap on the same GPU (other streams or threads) race on it and must be
 * serialised by the caller.  Results are bitwise those of sw_batch_forward. */
sw_status sw_batch_forward_static(sw_batch *batch, const sw_batch_io *io, void *stream);

/* Pick the tile shape (rows per tile, waves per block), the z-chunk length,
 * cache policy and prefetch depth, for single plans also the two-step sweep
 * (when io->field2 is given) and a cap of 4 resident blocks per CU, and (for
 * batches) the launch grid (one block per tile or a looping grid), by timing a few steps of each
 * candidate on the given buffers (their contents are overwritten), or reuse
 * the choice stored under the same problem key in the JSON file `cache_path`
 * (may be NULL: no cache).  The choice is kept in the plan / batch and
 * written back to the cache.  Synchronises `stream`. */
sw_status sw_plan_autotune(sw_plan *plan, const sw_fwd_io *io, const char *cache_path, void *stream);
sw_status sw_batch_autotune(sw_batch *batch, const sw_batch_io *io, const char *cache_path,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SIMWAVE_HIP_H */
