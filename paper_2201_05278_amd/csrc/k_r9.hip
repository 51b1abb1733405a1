// Stencil kernels instantiated for radius 9 (space order 18).  No
// two-step sweep at this radius: its register queues do not fit.
#include "stencil_const.h"
#include "stencil_vd.h"

namespace sw {

hipError_t launch_const_r9(int ndim, int mode, const Tiling &t, StencilParams &P, hipStream_t s)
{
    return launch_const_radius<9>(ndim, mode, t, P, s);
}

int const_resident_r9(const Tiling &t) { return const_resident_radius<9>(t); }

int vd_resident_r9(int scheme, const Tiling &t) { return vd_resident_radius<9>(scheme, t); }

hipError_t launch_batch_r9(int ndim, const Tiling &t, const StencilParams *shots, const int *tile_start,
                            int nshots, int parity, int nblocks, hipStream_t s)
{
    return launch_batch_radius<9>(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
}

hipError_t launch_vd_r9(int scheme, int mode, int ndim, const Tiling &t, StencilParams &P, hipStream_t s)
{
    return launch_vd_radius<9>(scheme, mode, ndim, t, P, s);
}

}  // namespace sw
