// Stencil kernels instantiated for radius 4 (space order 8).
#include "stencil_const.h"
#include "stencil_vd.h"
#include "stencil_tb.h"

namespace sw {

hipError_t launch_const_r4(int ndim, int mode, const Tiling &t, StencilParams &P, hipStream_t s)
{
    return launch_const_radius<4>(ndim, mode, t, P, s);
}

int const_resident_r4(const Tiling &t) { return const_resident_radius<4>(t); }

int vd_resident_r4(int scheme, const Tiling &t) { return vd_resident_radius<4>(scheme, t); }

hipError_t launch_batch_r4(int ndim, const Tiling &t, const StencilParams *shots, const int *tile_start,
                            int nshots, int parity, int nblocks, hipStream_t s)
{
    return launch_batch_radius<4>(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
}

hipError_t launch_tb_r4(const Tiling &t, StencilParams &P, const TwoStepParams &T, hipStream_t s)
{
    return launch_tb_radius<4>(t, P, T, s);
}

hipError_t launch_vd_r4(int scheme, int mode, int ndim, const Tiling &t, StencilParams &P, hipStream_t s)
{
    return launch_vd_radius<4>(scheme, mode, ndim, t, P, s);
}

}  // namespace sw
