// Double-precision instance of the constant-density forward (the precision
// of the paper's benchmark runs): model preparation, point coefficients,
// injection, recording, mirror ghosts, snapshots, and the block-tile stencil
// (the same tile code as single precision, instantiated for double with one
// tile shape per dimension).
#include "stencil_const.h"

#include "device64.h"
#include "ghost.h"

namespace sw {

namespace {

constexpr int kBlock = 256;

int blocks_for64(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return int(b);
}

__global__ void k_fill64(double *__restrict__ p, int64_t n)
{
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0.0;
}

// K = dt^2 c^2 at every padded position, from the model node of its
// coordinates (mirror image across mirrored sides, nearest node elsewhere).
__global__ void k_prep64(Geom g, int m0, int m1, int m2, int m3, int m4, int m5, int hz, int hx, int pz,
                         double dt2, const double *__restrict__ vel, double *__restrict__ K)
{
    const int64_t total = int64_t(pz) * g.px * g.py;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int yy = int(i % g.py);
        const int64_t t = i / g.py;
        const int xx = int(t % g.px);
        const int zz = int(t / g.px);
        const int z = model_axis(zz - hz, g.Z, m0, m1);
        const int x = model_axis(xx - hx, g.X, m2, m3);
        const int y = model_axis(yy - 64, g.Y, m4, m5);
        const int pzc = min(max(z - g.lo[0], 0), g.np[0] - 1);
        const int pxc = min(max(x - g.lo[1], 0), g.np[1] - 1);
        const int pyc = min(max(y - g.lo[2], 0), g.np[2] - 1);
        const double c = vel[(int64_t(pzc) * g.np[1] + pxc) * g.np[2] + pyc];
        K[i] = dt2 * c * c;
    }
}

// Injection coefficient A(node) dt^2 c^2 w / dV and recording weight w (the
// weight times `scale`, 1 / dV for sources).
__global__ void k_point_coef64(PointTable64 t, const double2 *__restrict__ damp, const double *__restrict__ vel,
                               double dt, double scale)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= t.nent) return;
    const double c = vel[t.phys[e]];
    const double w = t.weight[e] * scale;
    t.coef_a[e] = damp[t.d2[e]].x * (dt * dt * c * c) * w;
    t.wscaled[e] = w;
}

template <int G>
__device__ inline double group_sum64(double v)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

// Deterministic gather per unique node, as the single-precision injection.
template <int G>
__global__ void __launch_bounds__(kBlock) k_inject64(PointTable64 t, double *__restrict__ field,
                                                     const double *__restrict__ amp)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int u = gid / G, sub = gid % G;
    double sa = 0.0;
    if (u < t.nuniq)
        for (int k = t.uptr[u] + sub; k < t.uptr[u + 1]; k += G) {
            const int e = t.uent[k];
            sa = fma(t.coef_a[e], amp[t.pid[e]], sa);
        }
    sa = group_sum64<G>(sa);
    if (u < t.nuniq && sub == 0) field[t.unode[u]] += sa;
}

template <int G>
__global__ void __launch_bounds__(kBlock) k_record64(PointTable64 t, const double *__restrict__ field,
                                                     double *__restrict__ out)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int pt = gid / G, sub = gid % G;
    double acc = 0.0;
    if (pt < t.count)
        for (int e = t.ptr[pt] + sub; e < t.ptr[pt + 1]; e += G) acc += t.wscaled[e] * field[t.node[e]];
    acc = group_sum64<G>(acc);
    if (pt < t.count && sub == 0) out[pt] = acc;
}

__global__ void k_snapshot64(Geom g, const double *__restrict__ f, double *__restrict__ out)
{
    const int64_t total = int64_t(g.Z) * g.X * g.Y;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int y = int(i % g.Y);
        const int64_t t = i / g.Y;
        const int x = int(t % g.X);
        const int z = int(t / g.X);
        out[i] = f[elem(g, z, x, y)];
    }
}

template <int R, int NDIM, int TX, int NW>
__global__ void __launch_bounds__(64 * NW) k_const64(StencilParamsT<double> P)
{
    const_tile<double, R, NDIM, TX, NW, MODE_FWD, 1, 1>(P, xcd_remap(blockIdx.x, gridDim.x));
}

template <int R>
hipError_t launch_k_const64(int ndim, int tx, int nw, StencilParamsT<double> &P, hipStream_t s)
{
    const dim3 grid(P.ntx * P.nty * P.nzc);
    if (ndim == 2) {
        hipLaunchKernelGGL((k_const64<R, 2, 1, 1>), grid, dim3(64), 0, s, P);
        return hipGetLastError();
    }
#define SW_X(TXV, NWV)                                                                         \
    if (tx == TXV && nw == NWV) {                                                              \
        hipLaunchKernelGGL((k_const64<R, 3, TXV, NWV>), grid, dim3(64 * NWV), 0, s, P);        \
        return hipGetLastError();                                                              \
    }
    SW_F64_SHAPES(SW_X)
#undef SW_X
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_fill64(double *p, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill64, dim3(blocks_for64(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_prep64(const Geom &g, const int (*bcm)[2], int hz, int hx, int pz, double dt, const double *vel,
                         double *K, hipStream_t s)
{
    const int64_t total = int64_t(pz) * g.px * g.py;
    hipLaunchKernelGGL(k_prep64, dim3(blocks_for64(total)), dim3(kBlock), 0, s, g, bcm[0][0] != 0, bcm[0][1] != 0,
                       bcm[1][0] != 0, bcm[1][1] != 0, bcm[2][0] != 0, bcm[2][1] != 0, hz, hx, pz, dt * dt, vel, K);
    return hipGetLastError();
}

hipError_t launch_point_coef64(const PointTable64 &t, const double2 *damp, const double *vel, double dt,
                               double scale, hipStream_t s)
{
    if (t.nent <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_point_coef64, dim3((t.nent + kBlock - 1) / kBlock), dim3(kBlock), 0, s, t, damp, vel,
                       dt, scale);
    return hipGetLastError();
}

static int group_of(int n)
{
    int g = 1;
    while (g < n && g < 64) g *= 2;
    return g;
}

#define SW_G64(G, KERNEL, N, ...)                                                                          \
    switch (G) {                                                                                           \
    case 1: hipLaunchKernelGGL(KERNEL<1>, dim3((int64_t(N) * 1 + kBlock - 1) / kBlock), dim3(kBlock), 0, __VA_ARGS__); break;   \
    case 2: hipLaunchKernelGGL(KERNEL<2>, dim3((int64_t(N) * 2 + kBlock - 1) / kBlock), dim3(kBlock), 0, __VA_ARGS__); break;   \
    case 4: hipLaunchKernelGGL(KERNEL<4>, dim3((int64_t(N) * 4 + kBlock - 1) / kBlock), dim3(kBlock), 0, __VA_ARGS__); break;   \
    case 8: hipLaunchKernelGGL(KERNEL<8>, dim3((int64_t(N) * 8 + kBlock - 1) / kBlock), dim3(kBlock), 0, __VA_ARGS__); break;   \
    case 16: hipLaunchKernelGGL(KERNEL<16>, dim3((int64_t(N) * 16 + kBlock - 1) / kBlock), dim3(kBlock), 0, __VA_ARGS__); break; \
    case 32: hipLaunchKernelGGL(KERNEL<32>, dim3((int64_t(N) * 32 + kBlock - 1) / kBlock), dim3(kBlock), 0, __VA_ARGS__); break; \
    default: hipLaunchKernelGGL(KERNEL<64>, dim3((int64_t(N) * 64 + kBlock - 1) / kBlock), dim3(kBlock), 0, __VA_ARGS__); break; \
    }

hipError_t launch_inject64(const PointTable64 &t, double *field, const double *amp, hipStream_t s)
{
    if (t.nuniq <= 0) return hipSuccess;
    const int G = group_of(t.max_per_node);
    SW_G64(G, k_inject64, t.nuniq, s, t, field, amp);
    return hipGetLastError();
}

hipError_t launch_record64(const PointTable64 &t, const double *field, double *out, hipStream_t s)
{
    if (t.count <= 0) return hipSuccess;
    const int G = group_of(t.max_per_point);
    SW_G64(G, k_record64, t.count, s, t, field, out);
    return hipGetLastError();
}

#undef SW_G64

hipError_t launch_ghost64(const Geom &g, const int (*bcm)[2], int depth, double *field, hipStream_t s)
{
    const GhostSides sd = ghost_sides(g, bcm, depth);
    const int64_t total = sd.items[0] + sd.items[1] + sd.items[2];
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ghost_all<double>, dim3(blocks_for64(total)), dim3(kBlock), 0, s, g, sd, depth, field);
    return hipGetLastError();
}

hipError_t launch_snapshot64(const Geom &g, const double *field, double *out, hipStream_t s)
{
    const int64_t total = int64_t(g.Z) * g.X * g.Y;
    hipLaunchKernelGGL(k_snapshot64, dim3(blocks_for64(total)), dim3(kBlock), 0, s, g, field, out);
    return hipGetLastError();
}

template <int R, int TX, int NW>
int resident64_shape()
{
    constexpr auto kern = k_const64<R, 3, TX, NW>;
    int n = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, 64 * NW, 0) == hipSuccess ? n : 0;
}

template <int R>
int resident64(int tx, int nw)
{
#define SW_X(TXV, NWV) \
    if (tx == TXV && nw == NWV) return resident64_shape<R, TXV, NWV>();
    SW_F64_SHAPES(SW_X)
#undef SW_X
    return 0;
}

int f64_resident_blocks(int r, int tx, int nw)
{
    switch (r) {
    case 1: return resident64<1>(tx, nw);
    case 2: return resident64<2>(tx, nw);
    case 3: return resident64<3>(tx, nw);
    case 4: return resident64<4>(tx, nw);
    case 5: return resident64<5>(tx, nw);
    case 6: return resident64<6>(tx, nw);
    case 7: return resident64<7>(tx, nw);
    case 8: return resident64<8>(tx, nw);
    case 9: return resident64<9>(tx, nw);
    case 10: return resident64<10>(tx, nw);
    default: return 0;
    }
}

hipError_t launch_const64(int r, int ndim, int tx, int nw, StencilParamsT<double> &P, hipStream_t s)
{
    switch (r) {
    case 1: return launch_k_const64<1>(ndim, tx, nw, P, s);
    case 2: return launch_k_const64<2>(ndim, tx, nw, P, s);
    case 3: return launch_k_const64<3>(ndim, tx, nw, P, s);
    case 4: return launch_k_const64<4>(ndim, tx, nw, P, s);
    case 5: return launch_k_const64<5>(ndim, tx, nw, P, s);
    case 6: return launch_k_const64<6>(ndim, tx, nw, P, s);
    case 7: return launch_k_const64<7>(ndim, tx, nw, P, s);
    case 8: return launch_k_const64<8>(ndim, tx, nw, P, s);
    case 9: return launch_k_const64<9>(ndim, tx, nw, P, s);
    case 10: return launch_k_const64<10>(ndim, tx, nw, P, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sw
