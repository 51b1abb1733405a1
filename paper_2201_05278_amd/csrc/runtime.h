// Host runtime helpers shared by the C ABI translation units.
#pragma once

#include <string>

#include <hip/hip_runtime.h>

#include "device.h"
#include "plan.h"

#define SW_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return sw::fail(SW_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

namespace sw {

template <typename T>
T *at(void *ws, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

Geom make_geom(const sw_plan *p);
PointTableDev table_dev(const sw_plan *p, const PointSet &ps, const WorkspaceMap::Pts &o, void *ws);
bool const_shape_ok(int tx, int nw);
bool vd_shape_ok(int tx, int nw);
bool wave_shape_ok(int tx, int nw);
int default_zc(const sw_plan *p, int tx, int64_t want, int ts = 1);
Tiling choose_tiling(const sw_plan *p);
void fill_params(const sw_plan *p, void *ws, StencilParams &P);
void set_tiles(const sw_plan *p, const Tiling &t, StencilParams &P);
hipError_t stencil(const sw_plan *p, int mode, StencilParams &P, hipStream_t s);
bool tb_shape_ok(int r, int tx, int nw);
bool two_step_ready(const sw_plan *p, const sw_fwd_io *io);
// One two-step sweep from (cur = p^n, prv = p^{n-1}) to out1 = p^{n+1},
// out2 = p^{n+2}, with the sources of steps n and n+1 if `sources`.
hipError_t stencil_two(const sw_plan *p, const sw_fwd_io *io, int n, const float *cur, const float *prv,
                       float *out1, float *out2, bool sources, hipStream_t s);
sw_status check_prepared(const sw_plan *p, void *ws);
// A named roctx range over the enclosing scope (no-op without the roctx
// library; trace.cpp).
class Range {
public:
    explicit Range(const char *name);
    ~Range();
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;

private:
    bool active_ = false;
};
// Device address and size of the no-allocation batch's fixed descriptor table
// on the current device (resolved once per device; k_points.hip).
hipError_t static_batch_table(void **ptr, size_t *bytes);

}  // namespace sw
