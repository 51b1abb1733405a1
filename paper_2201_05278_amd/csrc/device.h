// Kernel parameter blocks and launcher declarations shared by the HIP
// translation units and the C ABI layer.
#pragma once

#include <cstdint>
#include <hip/hip_runtime.h>

namespace sw {

// Extended grid in the internal (z, x, y) view plus its padded layout.
struct Geom {
    int Z, X, Y;            // extended grid extents
    int px, py;             // padded x extent and row pitch
    int64_t origin;         // element offset of node (0, 0, 0)
    int64_t base;           // element offset of the first padded element of plane z = 0
    int xy0;                // in-plane offset of node (x, y) = (0, 0) from that element
    int lo[3];              // layer width on the low side (physical box start)
    int np[3];              // physical extents
};

__host__ __device__ inline int64_t elem(const Geom &g, int z, int x, int y)
{
    return g.origin + (int64_t(z) * g.px + x) * g.py + y;
}

enum StencilMode { MODE_FWD = 0, MODE_STORE = 1, MODE_IMAGE = 2, MODE_IMAGE2 = 3 };

// Blocks are dealt round-robin to the 8 XCDs; remap the flat block index so
// that each XCD receives a contiguous range of tiles (neighbouring tiles then
// share halos through the same L2).  A bijection on [0, n).
__device__ inline int xcd_remap(int bid, int n)
{
    const int per = n / 8, rem = n % 8;
    const int xcd = bid % 8, k = bid / 8;
    return (xcd < rem) ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

// Tile (tx, ty, z chunk) of block index bid: y tiles fastest, or x tiles
// fastest (neighbours along x, which share the larger halos, then run side by
// side on an XCD).
__device__ inline void tile_of(int bid, int ntx, int nty, int xfast, int &tx, int &ty, int &zc)
{
    if (xfast) {
        tx = bid % ntx;
        ty = (bid / ntx) % nty;
    } else {
        ty = bid % nty;
        tx = (bid / nty) % ntx;
    }
    zc = bid / (ntx * nty);
}

// Pair type of a value type: the (A, B) damping entries.
template <typename T> struct Pair;
template <> struct Pair<float> { using type = float2; };
template <> struct Pair<double> { using type = double2; };

// Parameters of one stencil launch over values of type T (float, or double
// for the double-precision forward).
template <typename T>
struct StencilParamsT {
    T *nxt;                 // p^{n-1} on entry, p^{n+1} on exit (in place)
    const T *cur;           // p^n
    const T *K;             // multiplier of (L p): dt^2 c^2, or dt^2 rho c^2
    const T *aux;           // b = 1/rho (staggered) or rho (centred); unused otherwise
    const typename Pair<T>::type *damp;   // (A, B) by squared layer distance
    int ndamp;              // entries of damp
    T *store;               // MODE_STORE: K (L p) written; MODE_IMAGE: read
    T *grad;                // MODE_IMAGE: += p * store / K^2
    T *store2;              // MODE_IMAGE2: the next step's stored level, imaged against p^{n-1}
    T *ustore;              // MODE_STORE, staggered scheme: p^n written (the level imaged by the face term)
    Geom g;
    T c0;                   // sum over axes of v_0 / h^2
    T cz[11], cx[11], cy[11];   // second-derivative v_j / h^2 per axis (j <= R <= 10)
    T sz[11], sx[11], sy[11];   // staggered s_j / h, or centred c_j / h (first derivative)
    T mj[11];               // midpoint interpolation weights
    int ntx, nty, nzc, zc;  // tiling: tiles along x, y; z chunks and chunk length
    int xfast;              // tile order within a z chunk: 1 x tiles fastest, 0 y tiles fastest
    int bcm[3][2];          // ghost condition per internal axis (z, x, y) and side: 0 zero, 1 Dirichlet, 2 Neumann
    int gh;                 // ghost layers held in the stored halo (mirror sides)
};
using StencilParams = StencilParamsT<float>;

// Whether the wavefield at coordinate v of an axis of extent n is read from
// memory: grid nodes, and ghost nodes within the stored halo on a side with a
// mirror condition (filled before the sweep); other positions read zero.
__device__ inline bool axis_read(int v, int n, int lo, int hi, int h)
{
    return (v >= 0 && v < n) || (v < 0 && lo != 0 && v >= -h) || (v >= n && hi != 0 && v < n + h);
}

// Grid node whose model value coordinate v (axis extent n) takes: the even
// mirror about the boundary node across a side with a mirror condition (lo /
// hi non-zero: the image of the model), then the nearest node (edge
// replication; also where a mirror reaches past the far side).
__host__ __device__ inline int model_axis(int v, int n, int lo, int hi)
{
    if (v < 0 && lo) v = -v;
    if (v >= n && hi) v = 2 * (n - 1) - v;
    return v < 0 ? 0 : (v > n - 1 ? n - 1 : v);
}

// Whether coordinate v lies on a side held at zero by a Dirichlet condition.
__device__ inline bool axis_dirichlet(int v, int n, int lo, int hi)
{
    return (v == 0 && lo == 1) || (v == n - 1 && hi == 1);
}

// Tiling chosen by the host for one stencil launch.
struct Tiling {
    int tx;                 // rows (x) per tile
    int nw;                 // waves per block
    int zc;                 // z-chunk length
    int nt;                 // 1: non-temporal loads/stores for the streamed arrays
    int pf;                 // planes of loads kept in flight ahead of the update (1 or 2)
    int wt;                 // 1: wave tiles (each wave owns tx / nw rows, no block barrier)
    int ts;                 // time steps per sweep (1, or 2 for the two-step constant-density sweep)
    int occ;                // resident blocks per CU at most (0: as registers and LDS allow; else 3..6)
    int xfast;              // 1: x tiles fastest in the block order (block tiles, single steps)
};

// Dynamic LDS bytes that hold a kernel with `static_lds` bytes of its own to
// at most `occ` resident blocks per CU (0 = no cap).  A CU has 160 KiB of LDS;
// each block is given 160 KiB / occ in total, rounded down to a multiple of
// 2560 bytes (a multiple of every LDS allocation granule), which leaves no
// room for block occ + 1 for occ <= 6.  Where the static LDS alone already
// exceeds that share the kernel is left as it is.
inline unsigned occ_pad_bytes(int occ, int static_lds)
{
    if (occ <= 0) return 0;
    const int share = (160 * 1024 / occ) / 2560 * 2560;
    return share > static_lds ? unsigned(share - static_lds) : 0u;
}

// Static LDS bytes of kernel KERN (read once per kernel and cached: one
// instantiation, and so one cached value, per kernel).
template <auto KERN>
int static_lds_of()
{
    static const int bytes = [] {
        hipFuncAttributes a{};
        return hipFuncGetAttributes(&a, reinterpret_cast<const void *>(KERN)) == hipSuccess
                   ? int(a.sharedSizeBytes) : 0;
    }();
    return bytes;
}

// Second output and injection of a two-step sweep (P.cur = p^n, P.nxt = p^{n-1}
// read only): p^{n+1} -> out1, p^{n+2} -> out2; inj[which * nuniq + u] is added
// to node unode[u] after step n + which; box = inclusive (z, x, y) bounds of
// the injection nodes (empty when nuniq == 0).
struct TwoStepParams {
    float *out1;
    float *out2;
    const int64_t *unode;
    const float *inj;
    int nuniq;
    int box[6];
};

hipError_t launch_const(int r, int ndim, int mode, const Tiling &t, StencilParams &P, hipStream_t s);
// Resident blocks per CU of the 3D constant-density forward block-tile kernel
// of tiling t at radius r (0: wave tiles, two-step sweeps, or no device).
int const_resident_blocks(int r, const Tiling &t);
// The same for the 3D variable-density forward kernels (scheme 1 staggered,
// 2 centred).
int vd_resident_blocks(int scheme, int r, const Tiling &t);
hipError_t launch_const_two(int r, const Tiling &t, StencilParams &P, const TwoStepParams &T, hipStream_t s);
hipError_t launch_vd(int scheme, int mode, int r, int ndim, const Tiling &t, StencilParams &P, hipStream_t s);

// ---- point and utility kernels ----
struct PointTableDev {
    const int32_t *ptr;     // by point: entries ptr[k] .. ptr[k+1]
    const int64_t *node;
    const int32_t *pid;
    const int32_t *d2;
    const int64_t *phys;
    const float *weight;
    const int64_t *unode;   // by unique node
    const int32_t *uptr;
    const int32_t *uent;
    float *coef_a;
    float *coef_s;
    float *wscaled;
    int count, nent, nuniq, max_per_point, max_per_node;
};

// Points of one shot of a batch: tables, the shot's two wavefield buffers,
// wavelet [nsteps][nsrc] and traces [nsteps][nrec].
struct ShotPoints {
    PointTableDev src, rec;
    float *field[2];
    const float *wavelet;
    float *traces;
};

hipError_t launch_const_batch(int r, int ndim, const Tiling &t, const StencilParams *shots,
                              const int *tile_start, int nshots, int parity, int nblocks,
                              hipStream_t s);
// Injection / recording for every shot of a batch at step `step`; the new
// level is in field[parity ^ 1].
hipError_t launch_inject_batch(const ShotPoints *shots, int nshots, int max_uniq, int max_per_node,
                               int step, int parity, hipStream_t s);
hipError_t launch_record_batch(const ShotPoints *shots, int nshots, int max_count, int max_per_point,
                               int step, int parity, hipStream_t s);

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t s);
// *count = number of non-finite values among a[0 .. n) (count cleared first).
hipError_t launch_count_nonfinite(const float *a, int64_t n, uint32_t *count, hipStream_t s);
// Mirror ghosts of a wavefield: for every side with a Dirichlet (odd) or
// Neumann (even) condition, ghost layer k = 1..depth takes +-p at the node k
// inside the boundary node, along z, then x, then y.
hipError_t launch_ghost_fill(const Geom &g, const int (*bcm)[2], int depth, float *field, hipStream_t s);
hipError_t launch_copy(float *dst, const float *src, int64_t n, hipStream_t s);
// Model arrays over the padded layout; bcm (per internal axis and side, 0 for
// zero ghosts) selects the even mirror image of the model in the ghosts of
// mirrored sides, the nearest node elsewhere.
hipError_t launch_model_prep(const Geom &g, const int (*bcm)[2], int halo_z, int halo_x, int pz, int scheme,
                             double dt, const float *vel, const float *rho, float *K, float *aux,
                             hipStream_t s);
// rho_inj (or NULL) scales the injection multiplier to dt^2 rho c^2; rho_rec
// (or NULL) divides the recording weights by rho (see k_point_coef).
hipError_t launch_point_coef(const PointTableDev &t, const float2 *damp, const float *vel, const float *rho_inj,
                             const float *rho_rec, double dt, double inv_dv, hipStream_t s);
hipError_t launch_inject(const PointTableDev &t, float *field, float *store, const float *amp,
                         hipStream_t s);
// The values launch_inject would add, for two consecutive steps:
// out[u] (amplitudes amp0) and out[nuniq + u] (amplitudes amp1).
hipError_t launch_inject_values(const PointTableDev &t, const float *amp0, const float *amp1, float *out,
                                hipStream_t s);
hipError_t launch_record(const PointTableDev &t, const float *field, float *out, hipStream_t s);
hipError_t launch_snapshot(const Geom &g, const float *field, float *out, hipStream_t s);
// Fold dJ/dM from the extended grid onto the physical grid and scale by
// 2 dt^2 c; tmp0 / tmp1 hold Z*X*ny and Z*nx*ny floats.
hipError_t launch_fold_gradient(const Geom &g, const float *grad_m, const float *vel, double dt,
                                float *grad_vel, float *tmp0, float *tmp1, hipStream_t s);
// Fold an extended-grid field (padded layout) onto the physical grid, unscaled.
hipError_t launch_fold(const Geom &g, const float *in, float *out, float *tmp0, float *tmp1, hipStream_t s);

// ---- staggered variable-density imaging (k_adjoint_vd.hip) ----
// F[axis] -= (D+ phi[k])(D+ u[k]) on every face of each used axis, for the np
// (1 or 2) level pairs k in order; sj[axis][1..r] = s_j / h.
hipError_t launch_face_image(const Geom &g, int ndim, int r, const float *const *sj, int np,
                             const float *const *phi, const float *const *u, float *const *F, hipStream_t s);
// S += phi * (source part of the update) at the source nodes.
hipError_t launch_src_image(const PointTableDev &t, const float *phi, const float *amp, float *S,
                            hipStream_t s);
// Per extended node: x = (gK + S / K^2) / b and y = gK K b - (dJ/db) b^2.
hipError_t launch_vd_chain(const Geom &g, int r, int ndim, const float *mj, const float *gK,
                           const float *const *F, const float *S, const float *K, const float *b,
                           float *xout, float *yout, hipStream_t s);

}  // namespace sw
