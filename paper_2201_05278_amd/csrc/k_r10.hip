// Stencil kernels instantiated for radius 10 (space order 20).  No
// two-step sweep at this radius: its register queues do not fit.
#include "stencil_const.h"
#include "stencil_vd.h"

namespace sw {

hipError_t launch_const_r10(int ndim, int mode, const Tiling &t, StencilParams &P, hipStream_t s)
{
    return launch_const_radius<10>(ndim, mode, t, P, s);
}

int const_resident_r10(const Tiling &t) { return const_resident_radius<10>(t); }

int vd_resident_r10(int scheme, const Tiling &t) { return vd_resident_radius<10>(scheme, t); }

hipError_t launch_batch_r10(int ndim, const Tiling &t, const StencilParams *shots, const int *tile_start,
                            int nshots, int parity, int nblocks, hipStream_t s)
{
    return launch_batch_radius<10>(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
}

hipError_t launch_vd_r10(int scheme, int mode, int ndim, const Tiling &t, StencilParams &P, hipStream_t s)
{
    return launch_vd_radius<10>(scheme, mode, ndim, t, P, s);
}

}  // namespace sw
