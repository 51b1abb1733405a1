// C ABI of the double-precision forward (SW_F64 plans, constant density):
// model preparation and the time loop, with the plan's host tables (the
// same coefficients, damping and point tables as single precision, kept in
// double) and double values in the workspace.
#include <algorithm>
#include <cstring>
#include <string>

#include <hip/hip_runtime.h>

#include "device64.h"
#include "runtime.h"

using namespace sw;

namespace {

PointTable64 table64(const PointSet &ps, const WorkspaceMap::Pts &o, void *ws)
{
    PointTable64 t{};
    t.ptr = at<int32_t>(ws, o.ptr);
    t.node = at<int64_t>(ws, o.node);
    t.pid = at<int32_t>(ws, o.pid);
    t.d2 = at<int32_t>(ws, o.d2);
    t.phys = at<int64_t>(ws, o.phys);
    t.weight = at<double>(ws, o.weight);
    t.unode = at<int64_t>(ws, o.unode);
    t.uptr = at<int32_t>(ws, o.uptr);
    t.uent = at<int32_t>(ws, o.uent);
    t.coef_a = at<double>(ws, o.coef_a);
    t.wscaled = at<double>(ws, o.wscaled);
    t.count = ps.count;
    t.nent = int(ps.node.size());
    t.nuniq = int(ps.unode.size());
    t.max_per_point = ps.max_per_point;
    t.max_per_node = ps.max_per_node;
    return t;
}

sw_status upload64(const PointSet &ps, const WorkspaceMap::Pts &o, void *ws, hipStream_t s)
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
    SW_HIP(up(o.weight, ps.weight64.data(), ps.weight64.size() * sizeof(double)));
    SW_HIP(up(o.unode, ps.unode.data(), ps.unode.size() * sizeof(int64_t)));
    SW_HIP(up(o.uptr, ps.uptr.data(), ps.uptr.size() * sizeof(int32_t)));
    SW_HIP(up(o.uent, ps.uent.data(), ps.uent.size() * sizeof(int32_t)));
    return SW_OK;
}

// Stencil parameters in double precision (coefficients as in fill_params).
void fill_params64(const sw_plan *p, void *ws, StencilParamsT<double> &P)
{
    std::memset(&P, 0, sizeof(P));
    P.g = make_geom(p);
    P.K = at<double>(ws, p->ws.model_k);
    P.damp = at<double2>(ws, p->ws.damp);
    P.ndamp = p->damp_n;
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 2; ++k) P.bcm[a][k] = p->bcm[a][k];
    P.gh = p->ghost;
    const double h2z = p->hh[0] * p->hh[0], h2x = p->hh[1] * p->hh[1], h2y = p->hh[2] * p->hh[2];
    P.c0 = p->v2[0] / h2z + p->v2[0] / h2y + (p->ndim == 3 ? p->v2[0] / h2x : 0.0);
    for (int j = 1; j <= p->r; ++j) {
        P.cz[j] = p->v2[j] / h2z;
        P.cx[j] = (p->ndim == 3) ? p->v2[j] / h2x : 0.0;
        P.cy[j] = p->v2[j] / h2y;
    }
    const Tiling t = choose_tiling(p);
    const int64_t pbytes = int64_t(p->pad[1]) * p->pad[2] * int64_t(sizeof(double));
    const int zmax = int(std::max<int64_t>(1, (int64_t(1) << 31) / pbytes - 4 * p->r - 2));
    P.ntx = (p->dims[1] + t.tx - 1) / t.tx;
    P.nty = (p->dims[2] + 63) / 64;
    P.zc = std::min(t.zc, zmax);
    P.nzc = (p->dims[0] + P.zc - 1) / P.zc;
    P.xfast = t.xfast;
}

}  // namespace

extern "C" {

sw_status sw_model_prepare_f64(sw_plan *p, const double *vel, double cmax, void *ws, void *stream)
{
    Range range_("sw_model_prepare_f64");
    set_error("");
    if (!p || !vel || !ws) return fail(SW_ERR_ARG, "NULL argument");
    if (p->prob.dtype != SW_F64) return fail(SW_ERR_STATE, "a single-precision plan is prepared by sw_model_prepare");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(SW_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (!(cmax > 0.0)) return fail(SW_ERR_ARG, "cmax must be positive");
    double dtc = 0.0;
    sw_status st = sw_critical_dt(p->ndim, p->prob.h, p->prob.space_order, cmax, &dtc);
    if (st != SW_OK) return st;
    if (p->prob.dt > dtc * (1.0 + 1e-12))
        return fail(SW_ERR_CFL, "dt " + std::to_string(p->prob.dt) + " exceeds the stability limit " +
                                    std::to_string(dtc));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Geom g = make_geom(p);
    SW_HIP(launch_prep64(g, p->bcm, p->hz, p->hx, p->pad[0], p->prob.dt, vel, at<double>(ws, p->ws.model_k), s));
    SW_HIP(hipMemcpyAsync(at<char>(ws, p->ws.damp), p->damp64.data(), p->damp64.size() * sizeof(double),
                          hipMemcpyHostToDevice, s));
    st = upload64(p->src, p->ws.src, ws, s);
    if (st != SW_OK) return st;
    st = upload64(p->rec, p->ws.rec, ws, s);
    if (st != SW_OK) return st;
    const double2 *damp = at<double2>(ws, p->ws.damp);
    SW_HIP(launch_point_coef64(table64(p->src, p->ws.src, ws), damp, vel, p->prob.dt, 1.0 / p->dV, s));
    SW_HIP(launch_point_coef64(table64(p->rec, p->ws.rec, ws), damp, vel, p->prob.dt, 1.0, s));
    p->prepared = true;
    p->prepared_ws = ws;
    ++p->generation;
    return SW_OK;
}

sw_status sw_forward_f64(sw_plan *p, const sw_fwd64_io *io, void *stream)
{
    Range range_("sw_forward_f64");
    set_error("");
    if (!p || !io) return fail(SW_ERR_ARG, "NULL argument");
    if (p->prob.dtype != SW_F64) return fail(SW_ERR_STATE, "a single-precision plan runs by sw_forward");
    sw_status st = check_prepared(p, io->workspace);
    if (st != SW_OK) return st;
    if (!io->field[0] || !io->field[1] || io->field[0] == io->field[1])
        return fail(SW_ERR_ARG, "two distinct wavefield buffers are required");
    if (io->step0 < 0 || io->nsteps_run < 0 || int64_t(io->step0) + io->nsteps_run > p->prob.nsteps)
        return fail(SW_ERR_ARG, "step range outside [0, nsteps]");
    if (p->src.count && !io->wavelet) return fail(SW_ERR_ARG, "wavelet is NULL");
    if (p->rec.count && !io->traces) return fail(SW_ERR_ARG, "traces is NULL");
    if (io->snaps && io->saving_stride < 0) return fail(SW_ERR_ARG, "saving_stride must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = io->workspace;
    StencilParamsT<double> P;
    fill_params64(p, ws, P);
    const Tiling t = choose_tiling(p);
    const PointTable64 src = table64(p->src, p->ws.src, ws);
    const PointTable64 rec = table64(p->rec, p->ws.rec, ws);
    const Geom g = make_geom(p);
    if (io->step0 == 0) {
        SW_HIP(launch_fill64(io->field[0], p->field_elems, s));
        SW_HIP(launch_fill64(io->field[1], p->field_elems, s));
    }
    for (int k = 0; k < io->nsteps_run; ++k) {
        const int n = io->step0 + k;
        double *cur = io->field[k % 2];
        double *nxt = io->field[(k + 1) % 2];
        if (p->mirror) SW_HIP(launch_ghost64(g, p->bcm, p->ghost, cur, s));
        P.cur = cur;
        P.nxt = nxt;
        SW_HIP(launch_const64(p->r, p->ndim, t.tx, t.nw, P, s));
        if (src.count) SW_HIP(launch_inject64(src, nxt, io->wavelet + size_t(n) * src.count, s));
        if (rec.count) SW_HIP(launch_record64(rec, nxt, io->traces + size_t(n) * rec.count, s));
        if (io->snaps && io->saving_stride > 0 && (n + 1) % io->saving_stride == 0)
            SW_HIP(launch_snapshot64(g, nxt, io->snaps + size_t((n + 1) / io->saving_stride - 1) * p->grid_nodes,
                                     s));
    }
    return SW_OK;
}

}  // extern "C"
