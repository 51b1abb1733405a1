// Variable-density stencils (staggered conservative and centred forms).
#include "device.h"

namespace sw {

hipError_t launch_vd(int scheme, int r, int ndim, const Tiling &t, StencilParams &P, hipStream_t s)
{
    (void)scheme; (void)r; (void)ndim; (void)t; (void)P; (void)s;
    return hipErrorNotSupported;
}

}  // namespace sw
