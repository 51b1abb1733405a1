// C ABI of the propagator (declarations and contracts in include/simwave_hip.h).
#include <algorithm>
#include <limits>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "runtime.h"
#include "device64.h"

namespace sw {
const std::string &last_error();
}  // namespace sw

using namespace sw;


namespace sw {

Geom make_geom(const sw_plan *p)
{
    Geom g{};
    g.Z = p->dims[0];
    g.X = p->dims[1];
    g.Y = p->dims[2];
    g.px = p->pad[1];
    g.py = p->pad[2];
    g.origin = p->origin;
    g.xy0 = p->hx * p->pad[2] + kRowAlign;
    g.base = p->origin - g.xy0;
    for (int i = 0; i < 3; ++i) {
        g.lo[i] = p->lo[i];
        g.np[i] = p->nphys[i];
    }
    return g;
}

PointTableDev table_dev(const sw_plan *p, const PointSet &ps, const WorkspaceMap::Pts &o, void *ws)
{
    PointTableDev t{};
    t.ptr = at<int32_t>(ws, o.ptr);
    t.node = at<int64_t>(ws, o.node);
    t.pid = at<int32_t>(ws, o.pid);
    t.d2 = at<int32_t>(ws, o.d2);
    t.phys = at<int64_t>(ws, o.phys);
    t.weight = at<float>(ws, o.weight);
    t.unode = at<int64_t>(ws, o.unode);
    t.uptr = at<int32_t>(ws, o.uptr);
    t.uent = at<int32_t>(ws, o.uent);
    t.coef_a = at<float>(ws, o.coef_a);
    t.coef_s = at<float>(ws, o.coef_s);
    t.wscaled = at<float>(ws, o.wscaled);
    t.count = ps.count;
    t.nent = int(ps.node.size());
    t.nuniq = int(ps.unode.size());
    t.max_per_point = ps.max_per_point;
    t.max_per_node = ps.max_per_node;
    (void)p;
    return t;
}

// Defaults from the tiling sweep of the 592^3 SO8 forward on MI355X.
constexpr int kDefaultNT = 1;
constexpr int kDefaultPF = 1;

bool const_shape_ok(int tx, int nw)
{
    return (tx == 16 && nw == 4) || (tx == 8 && nw == 4) || (tx == 32 && nw == 8) || (tx == 16 && nw == 8) ||
           (tx == 8 && nw == 8) || (tx == 24 && nw == 8);
}

bool wave_shape_ok(int tx, int nw)
{
    return (tx == 16 && nw == 4) || (tx == 32 && nw == 4) || (tx == 4 && nw == 1) || (tx == 8 && nw == 1) ||
           (tx == 16 && nw == 2);
}

bool vd_shape_ok(int tx, int nw)
{
    return (tx == 16 && nw == 8) || (tx == 8 && nw == 8) || (tx == 8 && nw == 4) || (tx == 16 && nw == 4) ||
           (tx == 16 && nw == 16);
}

// Two-step sweep shapes whose register queues fit (same rule as the kernel).
bool tb_shape_ok(int r, int tx, int nw)
{
    const bool listed = (tx == 8 && nw == 4) || (tx == 16 && nw == 8) || (tx == 8 && nw == 8) ||
                        (tx == 16 && nw == 4);
    return listed && (tx / nw) * (5 * r + 5) + ((2 * r + nw - 1) / nw) * (3 * r + 3) <= 95;
}

// Columns of a tile along y: 64, or 64 - 2R for the two-step sweep.
static int tile_cols(const sw_plan *p, int ts)
{
    return ts == 2 ? 64 - 2 * p->r : 64;
}

// z-chunk length giving about `want` blocks in total (at least 4R planes).
int default_zc(const sw_plan *p, int tx, int64_t want, int ts)
{
    const int ntx = (p->dims[1] + tx - 1) / tx;
    const int nty = (p->dims[2] + tile_cols(p, ts) - 1) / tile_cols(p, ts);
    const int64_t tiles = int64_t(ntx) * nty;
    const int nzc = int(std::max<int64_t>(1, (want + tiles - 1) / tiles));
    const int zc = (p->dims[0] + nzc - 1) / nzc;
    return std::max(zc, std::min(p->dims[0], 4 * p->r));
}

// Resident blocks per CU of the plan's 3D forward kernel for tiling t
// (queried once per plan and tiling; 0 without a device).
int resident_blocks(const sw_plan *p, const Tiling &t)
{
    const uint64_t key = (uint64_t(t.tx) << 40) | (uint64_t(t.nw) << 32) | (uint64_t(t.nt) << 24) |
                         (uint64_t(t.pf) << 16) | (uint64_t(t.wt) << 12) | (uint64_t(t.ts) << 8) |
                         uint64_t(t.occ & 0xff);
    for (const auto &e : p->resident_cache)
        if (e.first == key) return e.second;
    int dev = 0, n = 0;
    if (!p->ncu)
        p->ncu = (hipGetDevice(&dev) == hipSuccess &&
                  hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
                     ? n
                     : -1;
    const int r = p->ncu <= 0                    ? 0
                  : p->prob.dtype == SW_F64    ? f64_resident_blocks(p->r, t.tx, t.nw)
                  : p->prob.scheme == SW_CONST ? const_resident_blocks(p->r, t)
                                               : vd_resident_blocks(p->prob.scheme, p->r, t);
    p->resident_cache.emplace_back(key, r);
    return r;
}

// z-chunk length from whole rounds of resident blocks: a launch of B blocks
// runs in about ceil(B / resident) rounds, each as long as one block's march
// over its chunk and the 2R planes around it, so the chunk with the least
// rounds x (zc + 2R) is taken (ties: the shorter chunk), among chunks of
// 4R .. kMaxChunk planes that make at least kMinRounds rounds (launches of
// fewer, longer blocks ran up to 14% slower on a 400^3 grid whatever their
// rounds); 0 if no chunk qualifies.
constexpr int kMaxChunk = 100;
constexpr int kMinRounds = 3;
int rounds_zc(const sw_plan *p, const Tiling &t, int64_t resident)
{
    const int Z = p->dims[0];
    const int64_t tiles = int64_t((p->dims[1] + t.tx - 1) / t.tx) * ((p->dims[2] + 63) / 64);
    int best = 0;
    int64_t best_cost = std::numeric_limits<int64_t>::max();
    for (int nzc = 1; nzc <= Z; ++nzc) {
        const int zc = (Z + nzc - 1) / nzc;
        if (zc > kMaxChunk) continue;
        if (zc < 4 * p->r) break;
        const int64_t blocks = tiles * ((Z + zc - 1) / zc);
        if (blocks < kMinRounds * resident) continue;
        const int64_t cost = ((blocks + resident - 1) / resident) * (zc + 2 * p->r);
        if (cost <= best_cost) {
            best_cost = cost;
            best = zc;
        }
    }
    return best;
}

// Default variable-density block tile by radius, from a sweep of the forward
// stencils at 592^3 over SO 4 .. 20 (all shapes in one process): the
// staggered kernel keeps 8x4 tiles up to radius 7 and needs fewer registers
// per thread beyond (16x8 at radius 8: 2.90 against 6.69 ms; 8x8 at 9 and
// 10: 4.67 against 16.3 ms at SO20); the centred kernel takes 8x4 at radius
// 1 .. 2 and 9 .. 10, 16x8 at 3 .. 4, 8x8 at 5 .. 8.
void vd_default(int scheme, int r, int &tx, int &nw)
{
    if (scheme == SW_VD_STAGGERED) {
        tx = (r == 8) ? 16 : 8;
        nw = (r <= 7) ? 4 : 8;
        return;
    }
    if (r <= 2 || r >= 9) {
        tx = 8;
        nw = 4;
    } else if (r <= 4) {
        tx = 16;
        nw = 8;
    } else {
        tx = 8;
        nw = 8;
    }
}

// Default constant-density block tile and resident-block cap by radius, from a
// sweep of the forward stencil at 592^3 over space orders 2 .. 16: short
// stencils stream fastest with 8x4 tiles held to 4 blocks per CU (fewer z
// streams per L2), medium ones with 24x8 tiles, long ones with 8x4 or 16x4
// tiles whose register queues leave few blocks per CU anyway.
struct ConstDefault {
    int tx, nw, occ;
};
static ConstDefault const_default(int r)
{
    if (r <= 2) return {8, 4, 4};
    if (r <= 5) return {24, 8, 0};
    if (r == 6) return {16, 4, 3};
    return {8, 4, 0};            // r = 7 .. 10
}

Tiling choose_tiling(const sw_plan *p)
{
    Tiling t{};
    int def_occ = 0;
    if (p->ndim == 2) {
        t.tx = 1;
        t.nw = 1;
    } else if (p->prob.dtype == SW_F64) {
        t.tx = p->tile_tx ? p->tile_tx : kTile64X;
        t.nw = p->tile_tx ? p->tile_nw : f64_default_nw(p->r);
    } else if (p->prob.scheme != SW_CONST) {
        if (p->tile_tx) {
            t.tx = p->tile_tx;
            t.nw = p->tile_nw;
        } else {
            vd_default(p->prob.scheme, p->r, t.tx, t.nw);
        }
    } else if (p->tile_tx) {
        t.tx = p->tile_tx;
        t.nw = p->tile_nw;
        t.wt = p->mirror ? 0 : p->tile_wt;
        if (p->tile_wt && p->mirror) {   // wave tiles read no ghosts: the default block tile instead
            t.tx = 8;
            t.nw = 4;
        }
        t.ts = p->tile_ts == 2 ? 2 : 1;
    } else if (p->tile_ts == 2) {
        t.tx = 8;
        t.nw = tb_shape_ok(p->r, 8, 4) ? 4 : 8;
        t.ts = 2;
    } else {
        const ConstDefault d = const_default(p->r);
        t.tx = d.tx;
        t.nw = d.nw;
        def_occ = d.occ;
    }
    if (t.ts == 0) t.ts = 1;
    // z chunks of about 74 planes (fewer if the grid has few tiles per plane:
    // about 16000 waves in 3D).  At 592^3 this gives 74-plane chunks for both
    // 8x4 and 24x8 tiles; for 24x8, 74 planes (2000 blocks, just under four
    // rounds of resident blocks) ran 3% faster than 66 (2250 blocks, a mostly
    // idle fifth round).
    t.zc = p->tile_zc ? std::min(p->tile_zc, p->dims[0])
                      : std::min(std::min(74, p->dims[0]),
                                 default_zc(p, t.tx, p->ndim == 2 ? 1024 : 16000 / t.nw, t.ts));
    t.nt = p->tile_nt < 0 ? kDefaultNT : p->tile_nt;
    t.pf = p->tile_pf ? p->tile_pf : kDefaultPF;
    // the occupancy cap applies to single-step block tiles
    t.occ = (t.wt || t.ts == 2) ? 0 : (p->tile_occ < 0 ? def_occ : p->tile_occ);
    // 3D block tiles in single precision on a device: chunks by rounds of
    // resident blocks (the fixed wave target where no chunk makes enough
    // rounds; in double precision the rule picked chunks 3-5% slower than the
    // wave target on the paper's 3D shape at SO2 and SO4, so it keeps that)
    if (!p->tile_zc && p->ndim == 3 && p->prob.dtype == SW_F32 && !t.wt && t.ts == 1) {
        const int res = resident_blocks(p, t);
        if (res > 0) {
            const int zc = rounds_zc(p, t, int64_t(res) * p->ncu);
            if (zc > 0) t.zc = zc;
        }
    }
    // block order: y tiles fastest unless x tiles fastest is asked (block tiles only)
    t.xfast = (t.wt || t.ts == 2) ? 0 : (p->tile_order == 2 ? 1 : 0);
    return t;
}

void fill_params(const sw_plan *p, void *ws, StencilParams &P)
{
    std::memset(&P, 0, sizeof(P));
    P.g = make_geom(p);
    P.K = at<float>(ws, p->ws.model_k);
    P.aux = (p->prob.scheme != SW_CONST) ? at<float>(ws, p->ws.model_aux) : nullptr;
    P.damp = at<float2>(ws, p->ws.damp);
    P.ndamp = p->damp_n;
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s) P.bcm[a][s] = p->bcm[a][s];
    P.gh = p->ghost;
    double c0 = 0.0;
    const double h2z = p->hh[0] * p->hh[0], h2x = p->hh[1] * p->hh[1], h2y = p->hh[2] * p->hh[2];
    c0 += p->v2[0] / h2z + p->v2[0] / h2y;
    if (p->ndim == 3) c0 += p->v2[0] / h2x;
    P.c0 = float(c0);
    for (int j = 1; j <= p->r; ++j) {
        P.cz[j] = float(p->v2[j] / h2z);
        P.cx[j] = (p->ndim == 3) ? float(p->v2[j] / h2x) : 0.0f;
        P.cy[j] = float(p->v2[j] / h2y);
        const bool stag = p->prob.scheme == SW_VD_STAGGERED;
        const double *d = stag ? p->sg : p->w1;
        P.sz[j] = float(d[j] / p->hh[0]);
        P.sx[j] = (p->ndim == 3) ? float(d[j] / p->hh[1]) : 0.0f;
        P.sy[j] = float(d[j] / p->hh[2]);
        P.mj[j] = float(p->mp[j]);
    }
}

void set_tiles(const sw_plan *p, const Tiling &t, StencilParams &P)
{
    const int cols = tile_cols(p, t.ts);
    // a z window (chunk plus 4R planes) stays below 2^31 bytes: 32-bit buffer offsets
    const int64_t pbytes = int64_t(p->pad[1]) * p->pad[2] * (p->prob.dtype == SW_F64 ? 8 : 4);
    const int zmax = int(std::max<int64_t>(1, (int64_t(1) << 31) / pbytes - 4 * p->r - 2));
    P.ntx = (p->dims[1] + t.tx - 1) / t.tx;
    P.nty = (p->dims[2] + cols - 1) / cols;
    P.zc = std::min(t.zc, zmax);
    P.xfast = t.xfast;
    P.nzc = (p->dims[0] + P.zc - 1) / P.zc;
}

hipError_t stencil(const sw_plan *p, int mode, StencilParams &P, hipStream_t s)
{
    Tiling t = choose_tiling(p);
    t.ts = 1;
    // the staggered imaging stencil holds two more values per node than the
    // other modes: 8 x 4 tiles leave it 2 waves per SIMD, 8 x 8 tiles 4 (1.77
    // against 2.03 ms per launch at 592^3 SO8), so it takes 8 x 8 by default
    if ((mode == MODE_IMAGE || mode == MODE_IMAGE2) && p->prob.scheme == SW_VD_STAGGERED && p->ndim == 3 &&
        !p->tile_tx) {
        t.tx = 8;
        t.nw = 8;
    }
    set_tiles(p, t, P);
    if (p->prob.scheme == SW_CONST) return launch_const(p->r, p->ndim, mode, t, P, s);
    return launch_vd(p->prob.scheme, mode, p->r, p->ndim, t, P, s);
}

bool two_step_ready(const sw_plan *p, const sw_fwd_io *io)
{
    return p->ndim == 3 && p->prob.scheme == SW_CONST && !p->mirror && io->field2[0] && io->field2[1] &&
           choose_tiling(p).ts == 2;
}

hipError_t stencil_two(const sw_plan *p, const sw_fwd_io *io, int n, const float *cur, const float *prv,
                       float *out1, float *out2, bool sources, hipStream_t s)
{
    void *ws = io->workspace;
    StencilParams P;
    fill_params(p, ws, P);
    const Tiling t = choose_tiling(p);
    set_tiles(p, t, P);
    P.cur = cur;
    P.nxt = const_cast<float *>(prv);
    TwoStepParams T{};
    T.out1 = out1;
    T.out2 = out2;
    const PointTableDev src = table_dev(p, p->src, p->ws.src, ws);
    T.nuniq = sources ? src.nuniq : 0;
    T.unode = src.unode;
    float *inj = at<float>(ws, p->ws.src.inj);
    T.inj = inj;
    T.box[0] = T.box[2] = T.box[4] = 1;       // empty box
    T.box[1] = T.box[3] = T.box[5] = 0;
    if (T.nuniq > 0) {
        const int64_t plane = int64_t(p->pad[1]) * p->pad[2];
        T.box[0] = T.box[2] = T.box[4] = 1 << 30;
        T.box[1] = T.box[3] = T.box[5] = -1;
        for (const int64_t e : p->src.unode) {
            const int64_t rel = e - p->origin;
            const int c[3] = {int(rel / plane), int((rel / p->pad[2]) % p->pad[1]), int(rel % p->pad[2])};
            for (int a = 0; a < 3; ++a) {
                T.box[2 * a] = std::min(T.box[2 * a], c[a]);
                T.box[2 * a + 1] = std::max(T.box[2 * a + 1], c[a]);
            }
        }
        const hipError_t e = launch_inject_values(src, io->wavelet + size_t(n) * src.count,
                                                  io->wavelet + size_t(n + 1) * src.count, inj, s);
        if (e != hipSuccess) return e;
    }
    return launch_const_two(p->r, t, P, T, s);
}

sw_status check_problem(const sw_problem *q)
{
    if (!q) return fail(SW_ERR_ARG, "problem is NULL");
    if (q->ndim != 2 && q->ndim != 3) return fail(SW_ERR_UNSUPPORTED, "ndim must be 2 or 3");
    if (q->space_order < 2 || q->space_order > 20 || q->space_order % 2)
        return fail(SW_ERR_UNSUPPORTED, "space order must be even in 2..20");
    if (q->scheme != SW_CONST && q->scheme != SW_VD_STAGGERED && q->scheme != SW_VD_CENTRED)
        return fail(SW_ERR_ARG, "unknown scheme");
    if (q->dtype != SW_F32 && q->dtype != SW_F64) return fail(SW_ERR_ARG, "dtype must be SW_F32 or SW_F64");
    if (q->dtype == SW_F64 && q->scheme != SW_CONST)
        return fail(SW_ERR_UNSUPPORTED, "double precision covers the constant-density scheme");
    const int r = q->space_order / 2;
    for (int i = 0; i < q->ndim; ++i) {
        if (q->n[i] < 1) return fail(SW_ERR_ARG, "grid extents must be >= 1");
        if (!(q->h[i] > 0.0) || !std::isfinite(q->h[i]))
            return fail(SW_ERR_ARG, "grid spacing must be positive");
        for (int s = 0; s < 2; ++s) {
            if (q->nbl[i][s] < 0) return fail(SW_ERR_ARG, "layer widths must be >= 0");
            if (q->bc[i][s] != SW_BC_NONE && q->bc[i][s] != SW_BC_DIRICHLET && q->bc[i][s] != SW_BC_NEUMANN)
                return fail(SW_ERR_ARG, "unknown ghost condition");
        }
        if (int64_t(q->n[i]) + q->nbl[i][0] + q->nbl[i][1] > (1 << 20))
            return fail(SW_ERR_ARG, "grid extent too large");
    }
    if (!(q->dt > 0.0) || !std::isfinite(q->dt)) return fail(SW_ERR_ARG, "dt must be positive");
    if (q->nsteps < 0) return fail(SW_ERR_ARG, "nsteps must be >= 0");
    if (!(q->damp_alpha >= 0.0) || !(q->damp_power >= 0.0))
        return fail(SW_ERR_ARG, "damping parameters must be >= 0");
    (void)r;
    return SW_OK;
}

sw_status check_prepared(const sw_plan *p, void *ws)
{
    if (!p->prepared) return fail(SW_ERR_STATE, "sw_model_prepare must run after the last geometry change");
    if (ws != p->prepared_ws) return fail(SW_ERR_WORKSPACE, "workspace differs from the prepared one");
    return SW_OK;
}

}  // namespace sw

extern "C" {

int32_t sw_abi_version(void) { return SW_ABI_VERSION; }

const char *sw_status_str(sw_status s)
{
    switch (s) {
    case SW_OK: return "SW_OK";
    case SW_ERR_ARG: return "SW_ERR_ARG";
    case SW_ERR_UNSUPPORTED: return "SW_ERR_UNSUPPORTED";
    case SW_ERR_DOMAIN: return "SW_ERR_DOMAIN";
    case SW_ERR_CFL: return "SW_ERR_CFL";
    case SW_ERR_STATE: return "SW_ERR_STATE";
    case SW_ERR_WORKSPACE: return "SW_ERR_WORKSPACE";
    case SW_ERR_HIP: return "SW_ERR_HIP";
    case SW_ERR_NONFINITE: return "SW_ERR_NONFINITE";
    }
    return "SW_ERR_UNKNOWN";
}

const char *sw_last_error(void) { return sw::last_error().c_str(); }

sw_status sw_critical_dt(int32_t ndim, const double *h, int32_t space_order, double cmax, double *dt)
{
    set_error("");
    if ((ndim != 2 && ndim != 3) || !h || !dt) return fail(SW_ERR_ARG, "bad arguments");
    if (space_order < 2 || space_order > 20 || space_order % 2)
        return fail(SW_ERR_UNSUPPORTED, "space order must be even in 2..20");
    if (!(cmax > 0.0)) return fail(SW_ERR_ARG, "cmax must be positive");
    const double a = a1d(space_order);
    double s = 0.0;
    for (int i = 0; i < ndim; ++i) {
        if (!(h[i] > 0.0)) return fail(SW_ERR_ARG, "spacing must be positive");
        s += a / (h[i] * h[i]);
    }
    *dt = 2.0 / (cmax * std::sqrt(s));
    return SW_OK;
}

sw_status sw_steps_for(double tf, double dt, int32_t *n)
{
    set_error("");
    if (!n || !(dt > 0.0) || !(tf >= 0.0)) return fail(SW_ERR_ARG, "bad arguments");
    const double k = std::ceil(tf / dt) + 1.0;
    if (k > 2.0e9) return fail(SW_ERR_ARG, "too many steps");
    *n = int32_t(k);
    return SW_OK;
}

sw_status sw_ricker(double f, double t0, double dt, int32_t n, float *out)
{
    set_error("");
    if (!(f > 0.0) || !(dt > 0.0) || n < 0 || (n > 0 && !out)) return fail(SW_ERR_ARG, "bad arguments");
    if (t0 <= 0.0) t0 = 1.0 / f;
    for (int32_t k = 0; k < n; ++k) {
        const double t = k * dt - t0;
        const double a = M_PI * M_PI * f * f * t * t;
        out[k] = float((1.0 - 2.0 * a) * std::exp(-a));
    }
    return SW_OK;
}

sw_status sw_plan_create(const sw_problem *prob, sw_plan **out)
{
    set_error("");
    if (!out) return fail(SW_ERR_ARG, "out is NULL");
    *out = nullptr;
    sw_status st = check_problem(prob);
    if (st != SW_OK) return st;
    sw_plan *p = new (std::nothrow) sw_plan();
    if (!p) return fail(SW_ERR_ARG, "out of host memory");
    p->prob = *prob;
    if (p->prob.ndim == 2) {
        p->prob.n[2] = 1;
        p->prob.h[2] = 1.0;
        p->prob.nbl[2][0] = p->prob.nbl[2][1] = 0;
    }
    build_layout(p);
    // ghost conditions on the internal axes (z, x, y); a 2D grid is (z, 1, x)
    p->ghost = p->prob.scheme == SW_VD_STAGGERED ? 2 * p->r - 1 : p->r;
    for (int s = 0; s < 2; ++s) {
        p->bcm[0][s] = p->prob.bc[0][s];
        p->bcm[1][s] = p->ndim == 3 ? p->prob.bc[1][s] : SW_BC_NONE;
        p->bcm[2][s] = p->ndim == 3 ? p->prob.bc[2][s] : p->prob.bc[1][s];
    }
    for (int a = 0; a < 3; ++a)
        if (p->bcm[a][0] || p->bcm[a][1]) {
            p->mirror = true;
            if (p->dims[a] < p->ghost + 1) {
                delete p;
                return fail(SW_ERR_UNSUPPORTED, "a mirror ghost condition needs at least " +
                                                    std::to_string(p->ghost + 1) + " nodes along its axis");
            }
        }
    // stencil launches address a window of at most (4R + 2) z planes with
    // 32-bit byte offsets
    const int64_t es = p->prob.dtype == SW_F64 ? 8 : 4;
    if (int64_t(p->pad[1]) * p->pad[2] * es * (4 * p->r + 2) >= (int64_t(1) << 31)) {
        delete p;
        return fail(SW_ERR_UNSUPPORTED, "a z plane of the padded grid is too large for 32-bit window offsets "
                                        "(plane bytes x (4R + 2) must stay below 2^31)");
    }
    *out = p;
    return SW_OK;
}

sw_status sw_plan_set_tiling(sw_plan *p, const sw_tiling *t)
{
    set_error("");
    if (!p) return fail(SW_ERR_ARG, "plan is NULL");
    if (p->prob.dtype == SW_F64 && t) {
        // double precision: a tile shape and a z chunk (one cache policy and
        // prefetch depth, no wave tiles, two-step sweeps or occupancy caps)
        if (t->wt || t->ts == 2 || t->occ > 0)
            return fail(SW_ERR_UNSUPPORTED, "double-precision plans take a tile shape and a z chunk only");
        if (t->zc < 0) return fail(SW_ERR_ARG, "zc must be >= 0");
        if ((t->tx || t->nw) && (p->ndim != 3 || !f64_shape_ok(t->tx, t->nw)))
            return fail(SW_ERR_UNSUPPORTED, "tile shape not provided in double precision");
        p->tile_tx = t->tx;
        p->tile_nw = t->nw;
        p->tile_zc = t->zc;
        if (p->graph_exec) {
            (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(p->graph_exec));
            p->graph_exec = nullptr;
        }
        return SW_OK;
    }
    sw_tiling d{0, 0, 0, -1, 0, 0, 0, -1, 0};
    if (t) d = *t;
    if (d.order < 0 || d.order > 2) return fail(SW_ERR_ARG, "order must be 0 (default), 1 or 2");
    if (d.zc < 0) return fail(SW_ERR_ARG, "zc must be >= 0");
    if (d.occ < -1 || d.occ == 1 || d.occ == 2 || d.occ > 6)
        return fail(SW_ERR_ARG, "occ must be -1 (default), 0 (no cap) or 3 .. 6");
    if (d.ts < 0 || d.ts > 2) return fail(SW_ERR_ARG, "ts must be 0, 1 or 2");
    if (d.ts == 2) {
        if (p->ndim != 3 || p->prob.scheme != SW_CONST)
            return fail(SW_ERR_UNSUPPORTED, "two-step sweeps cover 3D constant density");
        if (d.wt) return fail(SW_ERR_ARG, "two-step sweeps use block tiles");
        if ((d.tx || d.nw) && !tb_shape_ok(p->r, d.tx, d.nw))
            return fail(SW_ERR_UNSUPPORTED, "tile shape not provided for two-step sweeps at this order");
        if (!d.tx && !d.nw && !tb_shape_ok(p->r, 8, 4) && !tb_shape_ok(p->r, 8, 8))
            return fail(SW_ERR_UNSUPPORTED, "no two-step tile shape at this order");
    }
    if (d.pf < 0 || d.pf > 2) return fail(SW_ERR_ARG, "pf must be 0, 1 or 2");
    if (d.wt && p->prob.scheme != SW_CONST) return fail(SW_ERR_UNSUPPORTED, "wave tiles cover constant density");
    if ((d.wt || d.ts == 2) && p->mirror)
        return fail(SW_ERR_UNSUPPORTED, "wave tiles and two-step sweeps read no mirror ghosts");
    if (d.tx || d.nw) {
        if (p->ndim != 3) return fail(SW_ERR_UNSUPPORTED, "2D grids have a fixed tile shape");
        const bool ok = p->prob.scheme != SW_CONST ? vd_shape_ok(d.tx, d.nw)
                        : (d.wt ? wave_shape_ok(d.tx, d.nw) : const_shape_ok(d.tx, d.nw));
        if (!ok) return fail(SW_ERR_UNSUPPORTED, "tile shape not provided");
    } else if (d.wt) {
        return fail(SW_ERR_ARG, "wave tiles need an explicit shape");
    }
    p->tile_tx = d.tx;
    p->tile_nw = d.nw;
    p->tile_zc = d.zc;
    p->tile_nt = d.nt < 0 ? -1 : (d.nt ? 1 : 0);
    p->tile_pf = d.pf;
    p->tile_wt = d.wt ? 1 : 0;
    p->tile_ts = d.ts;
    p->tile_occ = d.occ;
    p->tile_order = d.order;
    if (p->graph_exec) {
        (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(p->graph_exec));
        p->graph_exec = nullptr;
    }
    return SW_OK;
}

sw_status sw_plan_get_tiling(const sw_plan *p, sw_tiling *out)
{
    set_error("");
    if (!p || !out) return fail(SW_ERR_ARG, "NULL argument");
    const Tiling t = choose_tiling(p);
    *out = sw_tiling{t.tx, t.nw, t.zc, t.nt, t.pf, t.wt, t.ts, t.occ, t.xfast ? 2 : 1};
    return SW_OK;
}

sw_status sw_plan_occupancy(const sw_plan *p, int32_t *blocks_per_cu, int32_t *cus)
{
    set_error("");
    if (!p || !blocks_per_cu || !cus) return fail(SW_ERR_ARG, "NULL argument");
    *blocks_per_cu = 0;
    *cus = 0;
    const Tiling t = choose_tiling(p);
    if (p->ndim != 3 || t.wt || t.ts != 1) return SW_OK;
    const int n = resident_blocks(p, t);
    if (n > 0 && p->ncu > 0) {
        *blocks_per_cu = n;
        *cus = p->ncu;
    }
    return SW_OK;
}

sw_status sw_plan_destroy(sw_plan *plan)
{
    set_error("");
    if (!plan) return SW_OK;
    if (plan->graph_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(plan->graph_exec));
    if (plan->capture_stream) (void)hipStreamDestroy(static_cast<hipStream_t>(plan->capture_stream));
    delete plan;
    return SW_OK;
}

sw_status sw_plan_layout(const sw_plan *p, sw_layout *out)
{
    set_error("");
    if (!p || !out) return fail(SW_ERR_ARG, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->ndim = p->ndim;
    if (p->ndim == 3) {
        for (int i = 0; i < 3; ++i) out->dims[i] = p->dims[i];
        out->padded[0] = p->pad[0];
        out->padded[1] = p->pad[1];
        out->padded[2] = p->pad[2];
    } else {
        out->dims[0] = p->dims[0];
        out->dims[1] = p->dims[2];
        out->dims[2] = 1;
        out->padded[0] = p->pad[0];
        out->padded[1] = p->pad[2];
        out->padded[2] = 1;
    }
    out->halo = p->halo;
    out->origin = p->origin;
    out->field_elems = p->field_elems;
    out->grid_nodes = p->grid_nodes;
    out->physical_nodes = p->phys_nodes;
    out->nsrc = p->src.count;
    out->nrec = p->rec.count;
    out->workspace_bytes = int64_t(p->ws.total);
    return SW_OK;
}

sw_status sw_plan_set_geometry(sw_plan *p, int32_t which, int32_t count, const double *coords,
                               int32_t interp, int32_t radius, double kaiser_b)
{
    set_error("");
    if (!p) return fail(SW_ERR_ARG, "plan is NULL");
    if (which != SW_SRC && which != SW_REC) return fail(SW_ERR_ARG, "which must be SW_SRC or SW_REC");
    sw_status st = build_points(p, which == SW_SRC ? p->src : p->rec, count, coords, interp, radius,
                                kaiser_b, which == SW_SRC);
    if (st != SW_OK) return st;
    p->prepared = false;
    ++p->generation;
    return SW_OK;
}

sw_status sw_plan_points(const sw_plan *p, int32_t which, int64_t *nent, int64_t *nodes,
                         int32_t *ids, float *weights)
{
    set_error("");
    if (!p || !nent) return fail(SW_ERR_ARG, "NULL argument");
    if (which != SW_SRC && which != SW_REC) return fail(SW_ERR_ARG, "which must be SW_SRC or SW_REC");
    const PointSet &ps = which == SW_SRC ? p->src : p->rec;
    const int64_t n = int64_t(ps.node.size());
    if (nodes || ids || weights) {
        if (*nent < n) return fail(SW_ERR_ARG, "arrays too small");
        for (int64_t e = 0; e < n; ++e) {
            if (nodes) nodes[e] = ps.node[e];
            if (ids) ids[e] = ps.pid[e];
            if (weights) weights[e] = ps.weight[e];
        }
    }
    *nent = n;
    return SW_OK;
}

static sw_status upload_points(sw_plan *p, const PointSet &ps, const WorkspaceMap::Pts &o, void *ws,
                               hipStream_t s)
{
    auto up = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(static_cast<char *>(ws) + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    SW_HIP(up(o.ptr, ps.ptr.data(), ps.ptr.size() * sizeof(int32_t)));
    SW_HIP(up(o.node, ps.node.data(), ps.node.size() * sizeof(int64_t)));
    SW_HIP(up(o.pid, ps.pid.data(), ps.pid.size() * sizeof(int32_t)));
    SW_HIP(up(o.d2, ps.d2.data(), ps.d2.size() * sizeof(int32_t)));
    SW_HIP(up(o.phys, ps.phys.data(), ps.phys.size() * sizeof(int64_t)));
    SW_HIP(up(o.weight, ps.weight.data(), ps.weight.size() * sizeof(float)));
    SW_HIP(up(o.unode, ps.unode.data(), ps.unode.size() * sizeof(int64_t)));
    SW_HIP(up(o.uptr, ps.uptr.data(), ps.uptr.size() * sizeof(int32_t)));
    SW_HIP(up(o.uent, ps.uent.data(), ps.uent.size() * sizeof(int32_t)));
    (void)p;
    return SW_OK;
}

sw_status sw_model_prepare(sw_plan *p, const float *vel, const float *rho, double cmax, void *ws,
                           void *stream)
{
    Range range_("sw_model_prepare");
    set_error("");
    if (!p || !vel || !ws) return fail(SW_ERR_ARG, "NULL argument");
    if (p->prob.dtype == SW_F64) return fail(SW_ERR_STATE, "a double-precision plan is prepared by sw_model_prepare_f64");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(SW_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (p->prob.scheme != SW_CONST && !rho) return fail(SW_ERR_ARG, "variable density needs rho");
    if (!(cmax > 0.0)) return fail(SW_ERR_ARG, "cmax must be positive");
    double dtc = 0.0;
    sw_status st = sw_critical_dt(p->ndim, p->ndim == 3 ? p->prob.h : p->prob.h, p->prob.space_order,
                                  cmax, &dtc);
    if (st != SW_OK) return st;
    if (p->prob.dt > dtc * (1.0 + 1e-12))
        return fail(SW_ERR_CFL, "dt " + std::to_string(p->prob.dt) + " exceeds the stability limit " +
                                    std::to_string(dtc));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Geom g = make_geom(p);
    float *K = at<float>(ws, p->ws.model_k);
    float *aux = (p->prob.scheme != SW_CONST) ? at<float>(ws, p->ws.model_aux) : nullptr;
    SW_HIP(launch_model_prep(g, p->bcm, p->hz, p->hx, p->pad[0], p->prob.scheme, p->prob.dt, vel, rho, K, aux, s));
    SW_HIP(hipMemcpyAsync(at<char>(ws, p->ws.damp), p->damp.data(), p->damp.size() * sizeof(float),
                          hipMemcpyHostToDevice, s));
    st = upload_points(p, p->src, p->ws.src, ws, s);
    if (st != SW_OK) return st;
    st = upload_points(p, p->rec, p->ws.rec, ws, s);
    if (st != SW_OK) return st;
    const float2 *damp = at<float2>(ws, p->ws.damp);
    // staggered scheme: receivers inject the adjoint residual with the
    // stencil's multiplier K, and the source adjoint is recorded with w / rho
    const float *rho_stag = p->prob.scheme == SW_VD_STAGGERED ? rho : nullptr;
    SW_HIP(launch_point_coef(table_dev(p, p->src, p->ws.src, ws), damp, vel, nullptr, rho_stag, p->prob.dt,
                             1.0 / p->dV, s));
    SW_HIP(launch_point_coef(table_dev(p, p->rec, p->ws.rec, ws), damp, vel, rho_stag, nullptr, p->prob.dt,
                             1.0, s));
    p->prepared = true;
    p->prepared_ws = ws;
    ++p->generation;
    return SW_OK;
}

// Enqueue the forward steps of io on s.
static sw_status enqueue_forward(sw_plan *p, const sw_fwd_io *io, hipStream_t s)
{
    void *ws = io->workspace;
    StencilParams P;
    fill_params(p, ws, P);
    const PointTableDev src = table_dev(p, p->src, p->ws.src, ws);
    const PointTableDev rec = table_dev(p, p->rec, p->ws.rec, ws);
    const Geom g = make_geom(p);
    if (io->step0 == 0) {
        SW_HIP(launch_fill(io->field[0], p->field_elems, 0.0f, s));
        SW_HIP(launch_fill(io->field[1], p->field_elems, 0.0f, s));
    }
    std::vector<hipEvent_t> ev;
    if (io->stencil_ms) {
        ev.resize(2 * size_t(io->nsteps_run));
        for (auto &e : ev) SW_HIP(hipEventCreate(&e));
    }
    auto release = [&]() {
        for (auto &e : ev) (void)hipEventDestroy(e);
    };
    // checkpoint slot of step n: (p^n, p^{n-1})
    auto checkpoint = [&](int n, const float *cur, const float *prv) -> hipError_t {
        if (!io->ckpt || n % io->ckpt_every != 0) return hipSuccess;
        float *slot = io->ckpt + size_t(n / io->ckpt_every) * 2 * p->field_elems;
        hipError_t e = launch_copy(slot, cur, p->field_elems, s);
        if (e == hipSuccess) e = launch_copy(slot + p->field_elems, prv, p->field_elems, s);
        return e;
    };
    // receivers and snapshot of step n, whose new level p^{n+1} is in f
    auto outputs = [&](int n, const float *f) -> hipError_t {
        hipError_t e = hipSuccess;
        if (rec.count) e = launch_record(rec, f, io->traces + size_t(n) * rec.count, s);
        if (e == hipSuccess && io->snaps && io->saving_stride > 0 && (n + 1) % io->saving_stride == 0)
            e = launch_snapshot(g, f, io->snaps + size_t((n + 1) / io->saving_stride - 1) * p->grid_nodes, s);
        return e;
    };
    // span[k]: steps advanced by the launch bracketed by events 2k, 2k+1 (0: none)
    std::vector<int> span(size_t(io->nsteps_run), 0);
    const bool two = two_step_ready(p, io);
    int k = 0;
    while (k < io->nsteps_run) {
        const int n = io->step0 + k;
        float *cur = io->field[k % 2];
        float *nxt = io->field[(k + 1) % 2];
        if (two && io->nsteps_run - k >= 4) {
            // four steps in two sweeps: (cur, nxt) -> field2 -> (cur, nxt)
            float *t1 = io->field2[0], *t2 = io->field2[1];
            const float *in[2][2] = {{cur, nxt}, {t2, t1}};
            float *out[2][2] = {{t1, t2}, {nxt, cur}};
            for (int h = 0; h < 2; ++h) {
                const int m = n + 2 * h, km = k + 2 * h;
                SW_HIP(checkpoint(m, in[h][0], in[h][1]));
                if (!ev.empty()) SW_HIP(hipEventRecord(ev[2 * km], s));
                SW_HIP(stencil_two(p, io, m, in[h][0], in[h][1], out[h][0], out[h][1], true, s));
                if (!ev.empty()) SW_HIP(hipEventRecord(ev[2 * km + 1], s));
                span[km] = 2;
                SW_HIP(checkpoint(m + 1, out[h][0], in[h][0]));
                SW_HIP(outputs(m, out[h][0]));
                SW_HIP(outputs(m + 1, out[h][1]));
            }
            k += 4;
            continue;
        }
        SW_HIP(checkpoint(n, cur, nxt));
        if (p->mirror) SW_HIP(launch_ghost_fill(g, p->bcm, p->ghost, cur, s));
        P.cur = cur;
        P.nxt = nxt;
        if (!ev.empty()) SW_HIP(hipEventRecord(ev[2 * k], s));
        SW_HIP(stencil(p, MODE_FWD, P, s));
        if (!ev.empty()) SW_HIP(hipEventRecord(ev[2 * k + 1], s));
        span[k] = 1;
        if (src.count) SW_HIP(launch_inject(src, nxt, nullptr, io->wavelet + size_t(n) * src.count, s));
        SW_HIP(outputs(n, nxt));
        ++k;
    }
    if (!ev.empty()) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            release();
            return fail(SW_ERR_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
        }
        for (int j = 0; j < io->nsteps_run; ++j) {
            if (span[j] == 0) continue;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, ev[2 * j], ev[2 * j + 1]);
            for (int q = 0; q < span[j]; ++q) io->stencil_ms[j + q] = ms / span[j];
        }
    }
    release();
    return SW_OK;
}

static sw_status forward_impl(sw_plan *p, const sw_fwd_io *io, void *stream)
{
    if (!p || !io) return fail(SW_ERR_ARG, "NULL argument");
    if (p->prob.dtype == SW_F64) return fail(SW_ERR_STATE, "a double-precision plan runs by sw_forward_f64");
    sw_status st = check_prepared(p, io->workspace);
    if (st != SW_OK) return st;
    if (!io->field[0] || !io->field[1] || io->field[0] == io->field[1])
        return fail(SW_ERR_ARG, "two distinct wavefield buffers are required");
    if (io->step0 < 0 || io->nsteps_run < 0 || int64_t(io->step0) + io->nsteps_run > p->prob.nsteps)
        return fail(SW_ERR_ARG, "step range outside [0, nsteps]");
    if (p->src.count && !io->wavelet) return fail(SW_ERR_ARG, "wavelet is NULL");
    if (p->rec.count && !io->traces) return fail(SW_ERR_ARG, "traces is NULL");
    if (io->ckpt && io->ckpt_every <= 0) return fail(SW_ERR_ARG, "ckpt_every must be > 0");
    if (io->snaps && io->saving_stride < 0) return fail(SW_ERR_ARG, "saving_stride must be >= 0");
    if (io->stencil_ms && io->use_graph) return fail(SW_ERR_ARG, "stencil timing is not available with graphs");
    if ((io->field2[0] || io->field2[1]) &&
        (!io->field2[0] || !io->field2[1] || io->field2[0] == io->field2[1] || io->field2[0] == io->field[0] ||
         io->field2[0] == io->field[1] || io->field2[1] == io->field[0] || io->field2[1] == io->field[1]))
        return fail(SW_ERR_ARG, "field2 must be two more distinct wavefield buffers (or both NULL)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!io->use_graph) return enqueue_forward(p, io, s);

    // Capture the whole loop once, on a private stream (the legacy default
    // stream cannot be captured), and replay the graph on the caller's stream
    // whenever the same run is asked again.
    const std::vector<uint64_t> key = {
        uint64_t(uintptr_t(io->workspace)), uint64_t(uintptr_t(io->wavelet)),
        uint64_t(uintptr_t(io->field[0])), uint64_t(uintptr_t(io->field[1])),
        uint64_t(uintptr_t(io->field2[0])), uint64_t(uintptr_t(io->field2[1])),
        uint64_t(uintptr_t(io->traces)), uint64_t(uintptr_t(io->snaps)), uint64_t(io->saving_stride),
        uint64_t(uintptr_t(io->ckpt)), uint64_t(io->ckpt_every), uint64_t(io->step0),
        uint64_t(io->nsteps_run), p->generation, uint64_t(p->src.count), uint64_t(p->src.unode.size()),
        uint64_t(p->rec.count), uint64_t(p->rec.node.size())};
    if (!p->graph_exec || p->graph_key != key) {
        if (p->graph_exec) {
            (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(p->graph_exec));
            p->graph_exec = nullptr;
        }
        if (!p->capture_stream) {
            hipStream_t cs = nullptr;
            SW_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            p->capture_stream = cs;
        }
        hipStream_t cs = static_cast<hipStream_t>(p->capture_stream);
        SW_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        st = enqueue_forward(p, io, cs);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(cs, &graph);
        if (st != SW_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (ec != hipSuccess) return fail(SW_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(SW_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        p->graph_exec = exec;
        p->graph_key = key;
    }
    SW_HIP(hipGraphLaunch(static_cast<hipGraphExec_t>(p->graph_exec), s));
    return SW_OK;
}

sw_status sw_forward(sw_plan *p, const sw_fwd_io *io, void *stream)
{
    Range range_("sw_forward");
    set_error("");
    sw_status st = forward_impl(p, io, stream);
    if (st != SW_OK || !io->check_finite) return st;
    // optional check: non-finite trace samples of the steps run and final field values
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t *cnt = at<uint32_t>(io->workspace, p->ws.counter);
    uint32_t bad[2] = {0u, 0u};
    if (p->rec.count && io->nsteps_run) {
        SW_HIP(launch_count_nonfinite(io->traces + int64_t(io->step0) * p->rec.count,
                                      int64_t(io->nsteps_run) * p->rec.count, cnt, s));
        SW_HIP(hipMemcpyAsync(&bad[0], cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        SW_HIP(hipStreamSynchronize(s));
    }
    SW_HIP(launch_count_nonfinite(io->field[io->nsteps_run % 2], p->field_elems, cnt, s));
    SW_HIP(hipMemcpyAsync(&bad[1], cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SW_HIP(hipStreamSynchronize(s));
    if (bad[0] || bad[1])
        return fail(SW_ERR_NONFINITE, std::to_string(bad[0]) + " non-finite trace samples and " +
                                          std::to_string(bad[1]) + " non-finite wavefield values");
    return SW_OK;
}

sw_status sw_adjoint(sw_plan *p, const sw_adj_io *io, void *stream)
{
    Range range_("sw_adjoint");
    set_error("");
    if (!p || !io) return fail(SW_ERR_ARG, "NULL argument");
    if (p->prob.scheme == SW_VD_CENTRED)
        return fail(SW_ERR_UNSUPPORTED, "the adjoint covers the constant-density and staggered schemes");
    if (p->prob.dtype == SW_F64) return fail(SW_ERR_UNSUPPORTED, "the adjoint runs in single precision");
    if (p->mirror)
        return fail(SW_ERR_UNSUPPORTED, "the adjoint covers zero ghosts (no Dirichlet / Neumann sides)");
    sw_status st = check_prepared(p, io->workspace);
    if (st != SW_OK) return st;
    if (!io->residual || !io->ckpt || io->ckpt_every <= 0 || !io->field[0] || !io->field[1] ||
        !io->adj[0] || !io->adj[1] || !io->segment || !io->grad_m || !io->grad_vel || !io->vel)
        return fail(SW_ERR_ARG, "missing buffer");
    const bool vd = p->prob.scheme == SW_VD_STAGGERED;
    if (vd && (!io->grad_rho || !io->vd_work))
        return fail(SW_ERR_ARG, "the staggered scheme needs grad_rho and vd_work");
    if (p->src.count && !io->wavelet) return fail(SW_ERR_ARG, "wavelet is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = io->workspace;
    const int64_t fe = p->field_elems;
    const int N = p->prob.nsteps;
    const int E = io->ckpt_every;
    const PointTableDev src = table_dev(p, p->src, p->ws.src, ws);
    const PointTableDev rec = table_dev(p, p->rec, p->ws.rec, ws);
    StencilParams P;
    fill_params(p, ws, P);
    SW_HIP(launch_fill(io->grad_m, fe, 0.0f, s));
    SW_HIP(launch_fill(io->adj[0], fe, 0.0f, s));
    SW_HIP(launch_fill(io->adj[1], fe, 0.0f, s));
    // staggered scheme: per-axis face sums (vd_work[0..2]) and the source term (vd_work[3])
    float *face_sum[3] = {nullptr, nullptr, nullptr};
    float *src_sum = nullptr;
    const float *sj[3] = {P.sz, P.sx, P.sy};
    if (vd) {
        SW_HIP(launch_fill(io->vd_work, 4 * fe, 0.0f, s));
        for (int a = 0; a < 3; ++a) face_sum[a] = io->vd_work + size_t(a) * fe;
        src_sum = io->vd_work + size_t(3) * fe;
    }
    float *acur = io->adj[0];   // phi^{m+1}
    float *anxt = io->adj[1];   // phi^{m+2}, overwritten by phi^m
    const int nseg = (N + E - 1) / E;
    const Geom gm = make_geom(p);
    // staggered face term, formed two steps at a time: the term of step m
    // (phi^{m+1} against u^m) is deferred to the start of step m - 1, where
    // phi^{m+1} is still held (anxt) next to phi^m (acur); a step left over at
    // the end of a segment is formed alone
    auto u_level = [&](int m, int k) -> const float * { return io->segment + size_t(E + m - k) * fe; };
    // block tiles: imaging steps in pairs (one gradient pass per two steps)
    const bool pair_image = !choose_tiling(p).wt;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int k = seg * E;
        const int L = std::min(E, N - k);
        // restore (u^k, u^{k-1}) and recompute u^{k+1..k+L}, storing K L u^n plus,
        // for constant density, the source part M Q s^n (the staggered scheme
        // images the source separately and also keeps u^n for the face term)
        const float *slot = io->ckpt + size_t(seg) * 2 * fe;
        SW_HIP(launch_copy(io->field[0], slot, fe, s));
        SW_HIP(launch_copy(io->field[1], slot + fe, fe, s));
        for (int i = 0; i < L; ++i) {
            const int n = k + i;
            float *cur = io->field[i % 2];
            float *nxt = io->field[(i + 1) % 2];
            float *lvl = io->segment + size_t(i) * fe;
            P.cur = cur;
            P.nxt = nxt;
            P.store = lvl;
            P.grad = nullptr;
            P.ustore = vd ? io->segment + size_t(E + i) * fe : nullptr;
            SW_HIP(stencil(p, MODE_STORE, P, s));
            if (src.count)
                SW_HIP(launch_inject(src, nxt, vd ? nullptr : lvl, io->wavelet + size_t(n) * src.count, s));
        }
        P.ustore = nullptr;
        // adjoint steps m = top .. k (top = N in the last segment)
        const int top = (seg == nseg - 1) ? N : k + L - 1;
        int pend = -1;              // imaging step whose face term is deferred
        int gpend = -1;             // step whose imaging term is deferred
        for (int m = top; m >= k; --m) {
            P.cur = acur;
            P.nxt = anxt;
            if (m <= N - 1) {
                if (vd) {
                    if (pend == m + 1) {   // (phi^{m+2}, u^{m+1}) then (phi^{m+1}, u^m), before anxt is overwritten
                        const float *ph[2] = {anxt, acur};
                        const float *uu[2] = {u_level(m + 1, k), u_level(m, k)};
                        SW_HIP(launch_face_image(gm, p->ndim, p->r, sj, 2, ph, uu, face_sum, s));
                        pend = -1;
                    } else {
                        pend = m;
                    }
                    if (src.count)   // phi^{m+1} (acur, left unchanged by the step) at the sources
                        SW_HIP(launch_src_image(src, acur, io->wavelet + size_t(m) * src.count, src_sum, s));
                }
                if (pair_image && gpend == m + 1) {
                    // this step's imaging term and the one deferred from step m + 1:
                    // phi^{m+2}, the p^{n-1} this launch reads, against that step's level
                    P.store = io->segment + size_t(m - k) * fe;
                    P.store2 = io->segment + size_t(m + 1 - k) * fe;
                    P.grad = io->grad_m;
                    SW_HIP(stencil(p, MODE_IMAGE2, P, s));
                    gpend = -1;
                } else if (pair_image && m > k) {
                    // deferred to step m - 1 of this segment (the gradient is then
                    // read and written once per two steps)
                    P.store = nullptr;
                    P.grad = nullptr;
                    SW_HIP(stencil(p, MODE_FWD, P, s));
                    gpend = m;
                } else {
                    P.store = io->segment + size_t(m - k) * fe;
                    P.grad = io->grad_m;
                    SW_HIP(stencil(p, MODE_IMAGE, P, s));
                }
            } else {
                P.store = nullptr;
                P.grad = nullptr;
                SW_HIP(stencil(p, MODE_FWD, P, s));
            }
            if (m >= 1) {
                if (rec.count) SW_HIP(launch_inject(rec, anxt, nullptr, io->residual + size_t(m - 1) * rec.count, s));
                if (io->src_adjoint && src.count)
                    SW_HIP(launch_record(src, anxt, io->src_adjoint + size_t(m - 1) * src.count, s));
            }
            std::swap(acur, anxt);   // phi^m becomes the current level
        }
        if (pend >= 0) {   // step k alone: phi^{k+1} is now anxt
            const float *ph[1] = {anxt};
            const float *uu[1] = {u_level(pend, k)};
            SW_HIP(launch_face_image(gm, p->ndim, p->r, sj, 1, ph, uu, face_sum, s));
        }
    }
    // the forward work buffers are free now and hold the fold's partial sums
    if (!vd) {
        SW_HIP(launch_fold_gradient(make_geom(p), io->grad_m, io->vel, p->prob.dt, io->grad_vel, io->field[0],
                                    io->field[1], s));
        return SW_OK;
    }
    // staggered: x = (dJ/dK + S / K^2) / b -> dJ/dc = fold(x) 2 dt^2 c;
    // y = dJ/dK K b - dJ/db b^2 -> dJ/drho = fold(y)
    const Geom g = make_geom(p);
    const float *Kf = at<float>(ws, p->ws.model_k);
    const float *bf = at<float>(ws, p->ws.model_aux);
    SW_HIP(launch_vd_chain(g, p->r, p->ndim, P.mj, io->grad_m, face_sum, src_sum, Kf, bf, io->field[0],
                           io->field[1], s));
    SW_HIP(launch_fold_gradient(g, io->field[0], io->vel, p->prob.dt, io->grad_vel, io->adj[0], io->adj[1], s));
    SW_HIP(launch_fold(g, io->field[1], io->grad_rho, io->adj[0], io->adj[1], s));
    return SW_OK;
}

}  // extern "C"
