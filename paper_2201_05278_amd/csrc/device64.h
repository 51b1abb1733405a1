// Double-precision forward (constant density): point tables and launchers
// shared by k_f64.hip and the C ABI layer.
#pragma once

#include "device.h"

namespace sw {

// Tiles of the double-precision stencil in 3D (rows, waves); 2D uses (1, 1).
// Default: 8x4 up to radius 4 (0.93 / 0.96 / 1.00 ms per step at SO2/4/8 on
// the paper's 207x801x801 shape, against 0.98 / 1.03 / 1.08 for 8x8), 8x8
// (one row per thread, the fewest registers) beyond.
constexpr int f64_default_nw(int r) { return r <= 4 ? 4 : 8; }
constexpr int kTile64X = 8;
#define SW_F64_SHAPES(X) X(8, 8) X(16, 8) X(8, 4) X(24, 8)
constexpr bool f64_shape_ok(int tx, int nw)
{
    return (tx == 8 && nw == 8) || (tx == 16 && nw == 8) || (tx == 8 && nw == 4) || (tx == 24 && nw == 8);
}

// Point table with double weights and coefficients (indices as in PointTableDev).
struct PointTable64 {
    const int32_t *ptr;     // by point: entries ptr[k] .. ptr[k+1]
    const int64_t *node;
    const int32_t *pid;
    const int32_t *d2;
    const int64_t *phys;
    const double *weight;
    const int64_t *unode;   // by unique node
    const int32_t *uptr;
    const int32_t *uent;
    double *coef_a;         // A(node) dt^2 c^2 w scale: injection
    double *wscaled;        // w scale: recording
    int count, nent, nuniq, max_per_point, max_per_node;
};

hipError_t launch_fill64(double *p, int64_t n, hipStream_t s);
hipError_t launch_prep64(const Geom &g, const int (*bcm)[2], int hz, int hx, int pz, double dt, const double *vel,
                         double *K, hipStream_t s);
hipError_t launch_point_coef64(const PointTable64 &t, const double2 *damp, const double *vel, double dt,
                               double scale, hipStream_t s);
hipError_t launch_inject64(const PointTable64 &t, double *field, const double *amp, hipStream_t s);
hipError_t launch_record64(const PointTable64 &t, const double *field, double *out, hipStream_t s);
hipError_t launch_ghost64(const Geom &g, const int (*bcm)[2], int depth, double *field, hipStream_t s);
hipError_t launch_snapshot64(const Geom &g, const double *field, double *out, hipStream_t s);
hipError_t launch_const64(int r, int ndim, int tx, int nw, StencilParamsT<double> &P, hipStream_t s);
// Resident blocks per CU of the 3D double-precision stencil of a tile shape (0: unknown).
int f64_resident_blocks(int r, int tx, int nw);

}  // namespace sw
