// Stencil kernels instantiated for radius 8 (space order 16).
#include "stencil_const.h"
#include "stencil_vd.h"
#include "stencil_tb.h"

namespace sw {

hipError_t launch_const_r8(int ndim, int mode, const Tiling &t, StencilParams &P, hipStream_t s)
{
    return launch_const_radius<8>(ndim, mode, t, P, s);
}

int const_resident_r8(const Tiling &t) { return const_resident_radius<8>(t); }

int vd_resident_r8(int scheme, const Tiling &t) { return vd_resident_radius<8>(scheme, t); }

hipError_t launch_batch_r8(int ndim, const Tiling &t, const StencilParams *shots, const int *tile_start,
                            int nshots, int parity, int nblocks, hipStream_t s)
{
    return launch_batch_radius<8>(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
}

hipError_t launch_tb_r8(const Tiling &t, StencilParams &P, const TwoStepParams &T, hipStream_t s)
{
    return launch_tb_radius<8>(t, P, T, s);
}

hipError_t launch_vd_r8(int scheme, int mode, int ndim, const Tiling &t, StencilParams &P, hipStream_t s)
{
    return launch_vd_radius<8>(scheme, mode, ndim, t, P, s);
}

}  // namespace sw
