// Radius dispatch of the stencil launchers (one translation unit per radius).
#include "device.h"

namespace sw {

hipError_t launch_const_r1(int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_batch_r1(int, const Tiling &, const StencilParams *, const int *, int, int, int, hipStream_t);
hipError_t launch_vd_r1(int, int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_const_r2(int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_batch_r2(int, const Tiling &, const StencilParams *, const int *, int, int, int, hipStream_t);
hipError_t launch_vd_r2(int, int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_const_r3(int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_batch_r3(int, const Tiling &, const StencilParams *, const int *, int, int, int, hipStream_t);
hipError_t launch_vd_r3(int, int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_const_r4(int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_batch_r4(int, const Tiling &, const StencilParams *, const int *, int, int, int, hipStream_t);
hipError_t launch_vd_r4(int, int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_const_r5(int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_batch_r5(int, const Tiling &, const StencilParams *, const int *, int, int, int, hipStream_t);
hipError_t launch_vd_r5(int, int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_const_r6(int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_batch_r6(int, const Tiling &, const StencilParams *, const int *, int, int, int, hipStream_t);
hipError_t launch_vd_r6(int, int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_const_r7(int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_batch_r7(int, const Tiling &, const StencilParams *, const int *, int, int, int, hipStream_t);
hipError_t launch_vd_r7(int, int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_const_r8(int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_batch_r8(int, const Tiling &, const StencilParams *, const int *, int, int, int, hipStream_t);
hipError_t launch_vd_r8(int, int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_const_r9(int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_batch_r9(int, const Tiling &, const StencilParams *, const int *, int, int, int, hipStream_t);
hipError_t launch_vd_r9(int, int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_const_r10(int, int, const Tiling &, StencilParams &, hipStream_t);
hipError_t launch_batch_r10(int, const Tiling &, const StencilParams *, const int *, int, int, int, hipStream_t);
hipError_t launch_vd_r10(int, int, int, const Tiling &, StencilParams &, hipStream_t);

int vd_resident_r1(int, const Tiling &);
int vd_resident_r2(int, const Tiling &);
int vd_resident_r3(int, const Tiling &);
int vd_resident_r4(int, const Tiling &);
int vd_resident_r5(int, const Tiling &);
int vd_resident_r6(int, const Tiling &);
int vd_resident_r7(int, const Tiling &);
int vd_resident_r8(int, const Tiling &);
int vd_resident_r9(int, const Tiling &);
int vd_resident_r10(int, const Tiling &);
int const_resident_r1(const Tiling &);
int const_resident_r2(const Tiling &);
int const_resident_r3(const Tiling &);
int const_resident_r4(const Tiling &);
int const_resident_r5(const Tiling &);
int const_resident_r6(const Tiling &);
int const_resident_r7(const Tiling &);
int const_resident_r8(const Tiling &);
int const_resident_r9(const Tiling &);
int const_resident_r10(const Tiling &);

hipError_t launch_tb_r1(const Tiling &, StencilParams &, const TwoStepParams &, hipStream_t);
hipError_t launch_tb_r2(const Tiling &, StencilParams &, const TwoStepParams &, hipStream_t);
hipError_t launch_tb_r3(const Tiling &, StencilParams &, const TwoStepParams &, hipStream_t);
hipError_t launch_tb_r4(const Tiling &, StencilParams &, const TwoStepParams &, hipStream_t);
hipError_t launch_tb_r5(const Tiling &, StencilParams &, const TwoStepParams &, hipStream_t);
hipError_t launch_tb_r6(const Tiling &, StencilParams &, const TwoStepParams &, hipStream_t);
hipError_t launch_tb_r7(const Tiling &, StencilParams &, const TwoStepParams &, hipStream_t);
hipError_t launch_tb_r8(const Tiling &, StencilParams &, const TwoStepParams &, hipStream_t);

hipError_t launch_const(int r, int ndim, int mode, const Tiling &t, StencilParams &P, hipStream_t s)
{
    switch (r) {
    case 1: return launch_const_r1(ndim, mode, t, P, s);
    case 2: return launch_const_r2(ndim, mode, t, P, s);
    case 3: return launch_const_r3(ndim, mode, t, P, s);
    case 4: return launch_const_r4(ndim, mode, t, P, s);
    case 5: return launch_const_r5(ndim, mode, t, P, s);
    case 6: return launch_const_r6(ndim, mode, t, P, s);
    case 7: return launch_const_r7(ndim, mode, t, P, s);
    case 8: return launch_const_r8(ndim, mode, t, P, s);
    case 9: return launch_const_r9(ndim, mode, t, P, s);
    case 10: return launch_const_r10(ndim, mode, t, P, s);
    default: return hipErrorInvalidValue;
    }
}

int vd_resident_blocks(int scheme, int r, const Tiling &t)
{
    switch (r) {
    case 1: return vd_resident_r1(scheme, t);
    case 2: return vd_resident_r2(scheme, t);
    case 3: return vd_resident_r3(scheme, t);
    case 4: return vd_resident_r4(scheme, t);
    case 5: return vd_resident_r5(scheme, t);
    case 6: return vd_resident_r6(scheme, t);
    case 7: return vd_resident_r7(scheme, t);
    case 8: return vd_resident_r8(scheme, t);
    case 9: return vd_resident_r9(scheme, t);
    case 10: return vd_resident_r10(scheme, t);
    default: return 0;
    }
}

int const_resident_blocks(int r, const Tiling &t)
{
    switch (r) {
    case 1: return const_resident_r1(t);
    case 2: return const_resident_r2(t);
    case 3: return const_resident_r3(t);
    case 4: return const_resident_r4(t);
    case 5: return const_resident_r5(t);
    case 6: return const_resident_r6(t);
    case 7: return const_resident_r7(t);
    case 8: return const_resident_r8(t);
    case 9: return const_resident_r9(t);
    case 10: return const_resident_r10(t);
    default: return 0;
    }
}

hipError_t launch_const_batch(int r, int ndim, const Tiling &t, const StencilParams *shots,
                              const int *tile_start, int nshots, int parity, int nblocks, hipStream_t s)
{
    switch (r) {
    case 1: return launch_batch_r1(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
    case 2: return launch_batch_r2(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
    case 3: return launch_batch_r3(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
    case 4: return launch_batch_r4(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
    case 5: return launch_batch_r5(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
    case 6: return launch_batch_r6(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
    case 7: return launch_batch_r7(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
    case 8: return launch_batch_r8(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
    case 9: return launch_batch_r9(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
    case 10: return launch_batch_r10(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_const_two(int r, const Tiling &t, StencilParams &P, const TwoStepParams &T, hipStream_t s)
{
    switch (r) {
    case 1: return launch_tb_r1(t, P, T, s);
    case 2: return launch_tb_r2(t, P, T, s);
    case 3: return launch_tb_r3(t, P, T, s);
    case 4: return launch_tb_r4(t, P, T, s);
    case 5: return launch_tb_r5(t, P, T, s);
    case 6: return launch_tb_r6(t, P, T, s);
    case 7: return launch_tb_r7(t, P, T, s);
    case 8: return launch_tb_r8(t, P, T, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_vd(int scheme, int mode, int r, int ndim, const Tiling &t, StencilParams &P, hipStream_t s)
{
    switch (r) {
    case 1: return launch_vd_r1(scheme, mode, ndim, t, P, s);
    case 2: return launch_vd_r2(scheme, mode, ndim, t, P, s);
    case 3: return launch_vd_r3(scheme, mode, ndim, t, P, s);
    case 4: return launch_vd_r4(scheme, mode, ndim, t, P, s);
    case 5: return launch_vd_r5(scheme, mode, ndim, t, P, s);
    case 6: return launch_vd_r6(scheme, mode, ndim, t, P, s);
    case 7: return launch_vd_r7(scheme, mode, ndim, t, P, s);
    case 8: return launch_vd_r8(scheme, mode, ndim, t, P, s);
    case 9: return launch_vd_r9(scheme, mode, ndim, t, P, s);
    case 10: return launch_vd_r10(scheme, mode, ndim, t, P, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sw
