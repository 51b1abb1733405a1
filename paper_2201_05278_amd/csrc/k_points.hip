// Point kernels (source injection, receiver recording) and small utility
// kernels (buffer fill/copy, model preparation, snapshots, gradient fold).
//
// Injection is a gather over unique grid nodes: each node sums its table
// entries in a fixed order and adds the sum once, so results are deterministic
// and no atomics are needed.  Recording sums each receiver's entries.  Both
// give a group of G lanes (a power of two up to the wavefront width) to one
// node or receiver and finish with a butterfly reduction inside the group.
#include "device.h"
#include "ghost.h"

#include <mutex>

namespace sw {

// Descriptor table of the batched forward's no-allocation variant
// (sw_batch_forward_static): a fixed array in device memory, one copy per GPU
// the library runs on, held until the process ends.  Host code never passes
// the symbol itself to a kernel or a copy: static_batch_table resolves its
// device address once per device.
constexpr size_t kStaticTableBytes = size_t(1) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticTableBytes];

hipError_t static_batch_table(void **ptr, size_t *bytes)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kStaticTableBytes;
    return hipSuccess;
}

namespace {

constexpr int kBlock = 256;

// Per internal axis (z, x, y) and side: non-zero where a mirror ghost
// condition (Dirichlet or Neumann) holds.
struct Sides {
    int m[3][2];
};

Sides sides_of(const int (*bcm)[2])
{
    Sides sd{};
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 2; ++k) sd.m[a][k] = bcm ? bcm[a][k] != 0 : 0;
    return sd;
}

__global__ void k_fill(float *__restrict__ p, int64_t n, float v)
{
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_u32(uint32_t *c) { *c = 0u; }

// One atomic per wavefront: each lane counts its non-finite values, the wave
// sums its lanes, lane 0 adds the sum.
__global__ void k_count_nonfinite(const float *__restrict__ a, int64_t n, uint32_t *__restrict__ count)
{
    uint32_t c = 0;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        c += isfinite(a[i]) ? 0u : 1u;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

__global__ void k_copy(float *__restrict__ d, const float *__restrict__ s, int64_t n)
{
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        d[i] = s[i];
}

// Every element of the padded arrays receives a model value: the physical
// node nearest to its model node (edge replication into the layer; mirror
// images in the ghosts of mirrored sides; nearest node in the other ghosts and
// the row slack).
__global__ void k_model_prep(Geom g, Sides sd, int hz, int hx, int pz, int scheme, float dt2,
                             const float *__restrict__ vel, const float *__restrict__ rho,
                             float *__restrict__ K, float *__restrict__ aux)
{
    const int64_t total = int64_t(pz) * g.px * g.py;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int yy = int(i % g.py);
        const int64_t t = i / g.py;
        const int xx = int(t % g.px);
        const int zz = int(t / g.px);
        const int z = model_axis(zz - hz, g.Z, sd.m[0][0], sd.m[0][1]);
        const int x = model_axis(xx - hx, g.X, sd.m[1][0], sd.m[1][1]);
        const int y = model_axis(yy - 64, g.Y, sd.m[2][0], sd.m[2][1]);
        const int pzc = min(max(z - g.lo[0], 0), g.np[0] - 1);
        const int pxc = min(max(x - g.lo[1], 0), g.np[1] - 1);
        const int pyc = min(max(y - g.lo[2], 0), g.np[2] - 1);
        const int64_t ph = (int64_t(pzc) * g.np[1] + pxc) * g.np[2] + pyc;
        const float c = vel[ph];
        const float m = dt2 * c * c;
        if (scheme == 0) {
            K[i] = m;
        } else if (scheme == 1) {   // staggered: K = dt^2 rho c^2, aux = 1/rho
            const float r = rho[ph];
            K[i] = m * r;
            aux[i] = 1.0f / r;
        } else {                    // centred: K = dt^2 c^2, aux = rho
            K[i] = m;
            aux[i] = rho[ph];
        }
    }
}

// Per entry: A(node) W w s (injection), W w s (the source part of the stored
// levels of the imaging condition) and w s / R (recording), with s = 1/dV for
// sources and 1 for receivers.  W = dt^2 c^2, or dt^2 rho c^2 when rho_inj is
// given (the receivers of a staggered variable-density plan, whose adjoint
// spreads the residual with the stencil's multiplier K); R = 1, or rho when
// rho_rec is given (the sources of such a plan: its adjoint level is K A mu,
// and the source entered with M = K / rho).
__global__ void k_point_coef(PointTableDev t, const float2 *__restrict__ damp,
                             const float *__restrict__ vel, const float *__restrict__ rho_inj,
                             const float *__restrict__ rho_rec, double dt, double scale)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= t.nent) return;
    const double c = vel[t.phys[e]];
    const double m = dt * dt * c * c * (rho_inj ? double(rho_inj[t.phys[e]]) : 1.0);
    const double a = damp[t.d2[e]].x;
    const double w = double(t.weight[e]) * scale;
    t.coef_a[e] = float(a * m * w);
    t.coef_s[e] = float(m * w);
    t.wscaled[e] = float(rho_rec ? w / double(rho_rec[t.phys[e]]) : w);
}

template <int G>
__device__ inline float group_sum(float v)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

template <int G>
__global__ void __launch_bounds__(kBlock) k_inject(PointTableDev t, float *__restrict__ field,
                                                   float *__restrict__ store,
                                                   const float *__restrict__ amp)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int u = gid / G, sub = gid % G;
    float sa = 0.0f, ss = 0.0f;
    if (u < t.nuniq) {
        for (int k = t.uptr[u] + sub; k < t.uptr[u + 1]; k += G) {
            const int e = t.uent[k];
            const float s = amp[t.pid[e]];
            sa = fmaf(t.coef_a[e], s, sa);
            ss = fmaf(t.coef_s[e], s, ss);
        }
    }
    sa = group_sum<G>(sa);
    ss = group_sum<G>(ss);
    if (u < t.nuniq && sub == 0) {
        const int64_t n = t.unode[u];
        field[n] += sa;
        if (store) store[n] += ss;
    }
}

// The sums k_inject adds, for the amplitudes of two steps (blockIdx.y).
template <int G>
__global__ void __launch_bounds__(kBlock) k_inject_values(PointTableDev t, const float *__restrict__ amp0,
                                                          const float *__restrict__ amp1,
                                                          float *__restrict__ out)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int u = gid / G, sub = gid % G;
    const float *amp = blockIdx.y ? amp1 : amp0;
    float sa = 0.0f;
    if (u < t.nuniq)
        for (int k = t.uptr[u] + sub; k < t.uptr[u + 1]; k += G) {
            const int e = t.uent[k];
            sa = fmaf(t.coef_a[e], amp[t.pid[e]], sa);
        }
    sa = group_sum<G>(sa);
    if (u < t.nuniq && sub == 0) out[blockIdx.y * t.nuniq + u] = sa;
}

template <int G>
__global__ void __launch_bounds__(kBlock) k_record(PointTableDev t, const float *__restrict__ field,
                                                   float *__restrict__ out)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int pt = gid / G, sub = gid % G;
    float acc = 0.0f;
    if (pt < t.count)
        for (int e = t.ptr[pt] + sub; e < t.ptr[pt + 1]; e += G) acc += t.wscaled[e] * field[t.node[e]];
    acc = group_sum<G>(acc);
    if (pt < t.count && sub == 0) out[pt] = acc;
}

// Batched versions: blockIdx.y selects the shot.
template <int G>
__global__ void __launch_bounds__(kBlock) k_inject_batch(const ShotPoints *__restrict__ shots, int step,
                                                         int parity)
{
    const ShotPoints &S = shots[blockIdx.y];
    const PointTableDev &t = S.src;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int u = gid / G, sub = gid % G;
    const float *amp = S.wavelet + size_t(step) * t.count;
    float sa = 0.0f;
    if (u < t.nuniq)
        for (int k = t.uptr[u] + sub; k < t.uptr[u + 1]; k += G) {
            const int e = t.uent[k];
            sa = fmaf(t.coef_a[e], amp[t.pid[e]], sa);
        }
    sa = group_sum<G>(sa);
    if (u < t.nuniq && sub == 0) S.field[parity ^ 1][t.unode[u]] += sa;
}

template <int G>
__global__ void __launch_bounds__(kBlock) k_record_batch(const ShotPoints *__restrict__ shots, int step,
                                                         int parity)
{
    const ShotPoints &S = shots[blockIdx.y];
    const PointTableDev &t = S.rec;
    const float *field = S.field[parity ^ 1];
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int pt = gid / G, sub = gid % G;
    float acc = 0.0f;
    if (pt < t.count)
        for (int e = t.ptr[pt] + sub; e < t.ptr[pt + 1]; e += G) acc += t.wscaled[e] * field[t.node[e]];
    acc = group_sum<G>(acc);
    if (pt < t.count && sub == 0) S.traces[size_t(step) * t.count + pt] = acc;
}

__global__ void k_snapshot(Geom g, const float *__restrict__ f, float *__restrict__ out)
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

// Fold onto the physical grid (dJ/dc when scaled by 2 dt^2 c, or unscaled when
// vel is NULL).  Every extended-grid node copies its model from
// the nearest physical node, so the transpose of that copy sums the layer
// cells of each axis onto the physical edge cell.  The sum is separable and is
// done one axis at a time (y, then x, then z), each pass summing at most
// layer+1 inputs per output in a fixed order; `in` and `out` use dense
// (z, x, y) arrays of the stated extents, except that pass 0 reads the padded
// extended-grid layout.
__global__ void k_fold_axis(Geom g, int pass, const float *__restrict__ in, float *__restrict__ out,
                            const float *__restrict__ vel, float two_dt2)
{
    // extents of the input (iz, ix, iy) and output (oz, ox, oy) of this pass
    const int iz = g.Z, ix = (pass == 0) ? g.X : (pass == 1 ? g.X : g.np[1]);
    const int iy = (pass == 0) ? g.Y : g.np[2];
    const int oz = (pass == 2) ? g.np[0] : g.Z;
    const int ox = (pass >= 1) ? g.np[1] : g.X;
    const int oy = g.np[2];
    (void)iz;
    const int64_t total = int64_t(oz) * ox * oy;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int y = int(i % oy);
        const int64_t t = i / oy;
        const int x = int(t % ox);
        const int z = int(t / ox);
        const int ax = (pass == 0) ? 2 : (pass == 1 ? 1 : 0);      // axis folded in this pass
        const int c = (ax == 2) ? y : (ax == 1 ? x : z);           // physical index on that axis
        const int ext = (ax == 2) ? g.Y : (ax == 1 ? g.X : g.Z);
        int a = c + g.lo[ax], b = a;
        if (c == 0) a = 0;
        if (c == g.np[ax] - 1) b = ext - 1;
        float s = 0.0f;
        for (int k = a; k <= b; ++k) {
            if (pass == 0) s += in[elem(g, z, x, k)];
            else if (pass == 1) s += in[(int64_t(z) * ix + k) * iy + y];
            else s += in[(int64_t(k) * ix + x) * iy + y];
        }
        out[i] = (pass == 2 && vel) ? s * two_dt2 * vel[i] : s;
    }
}

// Grid size for the grid-stride kernels (capped) ...
int blocks_for(int64_t n, int per = kBlock)
{
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return int(b);
}

// ... and for the one-thread-per-item point kernels (not capped).
int blocks_exact(int64_t n)
{
    const int64_t b = (n + kBlock - 1) / kBlock;
    return int(b < 1 ? 1 : b);
}

int group_size(int max_entries)
{
    int g = 1;
    while (g < max_entries && g < 64) g <<= 1;
    return g;
}

}  // namespace

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy(float *dst, const float *src, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(blocks_for(n)), dim3(kBlock), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_model_prep(const Geom &g, const int (*bcm)[2], int halo_z, int halo_x, int pz, int scheme,
                             double dt, const float *vel, const float *rho, float *K, float *aux,
                             hipStream_t s)
{
    const int64_t total = int64_t(pz) * g.px * g.py;
    hipLaunchKernelGGL(k_model_prep, dim3(blocks_for(total)), dim3(kBlock), 0, s, g, sides_of(bcm), halo_z,
                       halo_x, pz, scheme, float(dt * dt), vel, rho, K, aux);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float *a, int64_t n, uint32_t *count, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, count);
    if (n > 0)
        hipLaunchKernelGGL(k_count_nonfinite, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, n, count);
    return hipGetLastError();
}

hipError_t launch_ghost_fill(const Geom &g, const int (*bcm)[2], int depth, float *field, hipStream_t s)
{
    const GhostSides sd = ghost_sides(g, bcm, depth);
    const int64_t total = sd.items[0] + sd.items[1] + sd.items[2];
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ghost_all<float>, dim3(blocks_for(total)), dim3(kBlock), 0, s, g, sd, depth, field);
    return hipGetLastError();
}

hipError_t launch_point_coef(const PointTableDev &t, const float2 *damp, const float *vel, const float *rho_inj,
                             const float *rho_rec, double dt, double scale, hipStream_t s)
{
    if (t.nent <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_point_coef, dim3(blocks_for(t.nent)), dim3(kBlock), 0, s, t, damp, vel, rho_inj,
                       rho_rec, dt, scale);
    return hipGetLastError();
}

#define SW_GROUP_DISPATCH(G, KERNEL, N, ...)                                                    \
    switch (G) {                                                                                \
    case 1: hipLaunchKernelGGL(KERNEL<1>, dim3(blocks_exact(int64_t(N) * 1)), dim3(kBlock), 0, __VA_ARGS__); break;   \
    case 2: hipLaunchKernelGGL(KERNEL<2>, dim3(blocks_exact(int64_t(N) * 2)), dim3(kBlock), 0, __VA_ARGS__); break;   \
    case 4: hipLaunchKernelGGL(KERNEL<4>, dim3(blocks_exact(int64_t(N) * 4)), dim3(kBlock), 0, __VA_ARGS__); break;   \
    case 8: hipLaunchKernelGGL(KERNEL<8>, dim3(blocks_exact(int64_t(N) * 8)), dim3(kBlock), 0, __VA_ARGS__); break;   \
    case 16: hipLaunchKernelGGL(KERNEL<16>, dim3(blocks_exact(int64_t(N) * 16)), dim3(kBlock), 0, __VA_ARGS__); break; \
    case 32: hipLaunchKernelGGL(KERNEL<32>, dim3(blocks_exact(int64_t(N) * 32)), dim3(kBlock), 0, __VA_ARGS__); break; \
    default: hipLaunchKernelGGL(KERNEL<64>, dim3(blocks_exact(int64_t(N) * 64)), dim3(kBlock), 0, __VA_ARGS__); break; \
    }

hipError_t launch_inject(const PointTableDev &t, float *field, float *store, const float *amp,
                         hipStream_t s)
{
    if (t.nuniq <= 0) return hipSuccess;
    const int G = group_size(t.max_per_node);
    SW_GROUP_DISPATCH(G, k_inject, t.nuniq, s, t, field, store, amp);
    return hipGetLastError();
}

hipError_t launch_record(const PointTableDev &t, const float *field, float *out, hipStream_t s)
{
    if (t.count <= 0) return hipSuccess;
    const int G = group_size(t.max_per_point);
    SW_GROUP_DISPATCH(G, k_record, t.count, s, t, field, out);
    return hipGetLastError();
}

#define SW_GROUP_DISPATCH2(G, KERNEL, N, NY, ...)                                                \
    switch (G) {                                                                                  \
    case 1: hipLaunchKernelGGL(KERNEL<1>, dim3(blocks_exact(int64_t(N) * 1), NY), dim3(kBlock), 0, __VA_ARGS__); break;   \
    case 2: hipLaunchKernelGGL(KERNEL<2>, dim3(blocks_exact(int64_t(N) * 2), NY), dim3(kBlock), 0, __VA_ARGS__); break;   \
    case 4: hipLaunchKernelGGL(KERNEL<4>, dim3(blocks_exact(int64_t(N) * 4), NY), dim3(kBlock), 0, __VA_ARGS__); break;   \
    case 8: hipLaunchKernelGGL(KERNEL<8>, dim3(blocks_exact(int64_t(N) * 8), NY), dim3(kBlock), 0, __VA_ARGS__); break;   \
    case 16: hipLaunchKernelGGL(KERNEL<16>, dim3(blocks_exact(int64_t(N) * 16), NY), dim3(kBlock), 0, __VA_ARGS__); break; \
    case 32: hipLaunchKernelGGL(KERNEL<32>, dim3(blocks_exact(int64_t(N) * 32), NY), dim3(kBlock), 0, __VA_ARGS__); break; \
    default: hipLaunchKernelGGL(KERNEL<64>, dim3(blocks_exact(int64_t(N) * 64), NY), dim3(kBlock), 0, __VA_ARGS__); break; \
    }

hipError_t launch_inject_values(const PointTableDev &t, const float *amp0, const float *amp1, float *out,
                                hipStream_t s)
{
    if (t.nuniq <= 0) return hipSuccess;
    const int G = group_size(t.max_per_node);
    SW_GROUP_DISPATCH2(G, k_inject_values, t.nuniq, 2, s, t, amp0, amp1, out);
    return hipGetLastError();
}

hipError_t launch_inject_batch(const ShotPoints *shots, int nshots, int max_uniq, int max_per_node,
                               int step, int parity, hipStream_t s)
{
    if (max_uniq <= 0 || nshots <= 0) return hipSuccess;
    const int G = group_size(max_per_node);
    SW_GROUP_DISPATCH2(G, k_inject_batch, max_uniq, nshots, s, shots, step, parity);
    return hipGetLastError();
}

hipError_t launch_record_batch(const ShotPoints *shots, int nshots, int max_count, int max_per_point,
                               int step, int parity, hipStream_t s)
{
    if (max_count <= 0 || nshots <= 0) return hipSuccess;
    const int G = group_size(max_per_point);
    SW_GROUP_DISPATCH2(G, k_record_batch, max_count, nshots, s, shots, step, parity);
    return hipGetLastError();
}

hipError_t launch_snapshot(const Geom &g, const float *field, float *out, hipStream_t s)
{
    const int64_t total = int64_t(g.Z) * g.X * g.Y;
    hipLaunchKernelGGL(k_snapshot, dim3(blocks_for(total)), dim3(kBlock), 0, s, g, field, out);
    return hipGetLastError();
}

hipError_t launch_fold_gradient(const Geom &g, const float *grad_m, const float *vel, double dt,
                                float *grad_vel, float *tmp0, float *tmp1, hipStream_t s)
{
    const float two_dt2 = float(2.0 * dt * dt);
    const int64_t n0 = int64_t(g.Z) * g.X * g.np[2];
    const int64_t n1 = int64_t(g.Z) * g.np[1] * g.np[2];
    const int64_t n2 = int64_t(g.np[0]) * g.np[1] * g.np[2];
    hipLaunchKernelGGL(k_fold_axis, dim3(blocks_for(n0)), dim3(kBlock), 0, s, g, 0, grad_m, tmp0, vel, two_dt2);
    hipLaunchKernelGGL(k_fold_axis, dim3(blocks_for(n1)), dim3(kBlock), 0, s, g, 1, tmp0, tmp1, vel, two_dt2);
    hipLaunchKernelGGL(k_fold_axis, dim3(blocks_for(n2)), dim3(kBlock), 0, s, g, 2, tmp1, grad_vel, vel, two_dt2);
    return hipGetLastError();
}

hipError_t launch_fold(const Geom &g, const float *in, float *out, float *tmp0, float *tmp1, hipStream_t s)
{
    return launch_fold_gradient(g, in, nullptr, 0.0, out, tmp0, tmp1, s);
}

}  // namespace sw
