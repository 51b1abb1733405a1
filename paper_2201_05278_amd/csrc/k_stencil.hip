// Constant-density leapfrog stencil (paper, "Time discretization" update with
// the "Space discretization" centred second derivatives), damping fused:
//
//   p^{n+1} = A (2 p^n + K (L p^n)) - B p^{n-1},
//   L p = c0 p + sum_j [cz_j (p_{z+j} + p_{z-j}) + cx_j (...) + cy_j (...)],
//
// with (A, B) looked up from the squared layer distance of the node (1, 1 in
// the physical grid), so no damping array is read.
//
// Blocking: a block owns a TX x 64 tile of the (x, y) plane (y, the
// contiguous axis, across the 64 lanes of a wavefront) and marches along z
// through a chunk of planes.  Each thread keeps the 2R+1 values of its column
// p[z-R .. z+R] in a register queue; the current plane of the tile plus an
// R-wide halo in x and y is staged in LDS (double buffered, one barrier per
// plane) for the in-plane neighbours.  Loads for plane z+1 are issued before
// plane z is computed.  Grid points outside the extended grid read as zero.
// The flat block index is remapped so that each XCD (blocks are dealt
// round-robin to the 8 XCDs) works on a contiguous range of tiles, which keeps
// neighbouring tiles' halos in the same L2.
//
// Modes: MODE_FWD plain step; MODE_STORE also writes K (L p) (the recomputed
// forward level of the imaging condition); MODE_IMAGE also accumulates
// grad += p * store / K^2 (zero-lag imaging of the adjoint field p against the
// stored level).
#include "device.h"

namespace sw {

__device__ inline int xcd_remap(int bid, int n)
{
    const int per = n / 8, rem = n % 8;
    const int xcd = bid % 8, k = bid / 8;
    return (xcd < rem) ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

namespace {

template <int R, int NDIM, int TX, int NW, int MODE>
__global__ void __launch_bounds__(64 * NW) k_const(StencilParams P)
{
    static_assert(TX % NW == 0, "rows must split evenly over waves");
    constexpr int RPT = TX / NW;                 // rows per thread
    constexpr int HXR = (NDIM == 3) ? R : 0;     // LDS halo rows in x
    constexpr int LY = 64 + 2 * R;
    constexpr int LX = TX + 2 * HXR;
    constexpr int NT = 64 * NW;
    constexpr int HXN = (NDIM == 3) ? (2 * R + NW - 1) / NW : 0;   // x-halo rows per wave
    constexpr int YHN = (TX * 2 * R + NT - 1) / NT;                 // y-halo items per thread
    __shared__ float lds[2][LX][LY];

    const Geom &g = P.g;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int ty = bid % P.nty;
    const int rest = bid / P.nty;
    const int tx = rest % P.ntx;
    const int zc = rest / P.ntx;
    const int y0 = ty * 64;
    const int y = y0 + lane;
    const int x0 = tx * TX;
    const int zb = zc * P.zc;
    const int ze = min(zb + P.zc, g.Z);
    const int64_t sz = int64_t(g.px) * g.py;
    const bool yin = y < g.Y;
    const int ey = max(0, max(g.lo[2] - y, y - (g.lo[2] + g.np[2] - 1)));

    int64_t roff[RPT];
    bool rin[RPT];
    int ex2[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int x = x0 + wave * RPT + i;
        rin[i] = yin && x < g.X;
        roff[i] = g.origin + int64_t(x) * g.py + y;
        const int ex = max(0, max(g.lo[1] - x, x - (g.lo[1] + g.np[1] - 1)));
        ex2[i] = ex * ex + ey * ey;
    }
    int64_t hxoff[HXN > 0 ? HXN : 1];
    bool hxin[HXN > 0 ? HXN : 1], hxok[HXN > 0 ? HXN : 1];
    int hxrow[HXN > 0 ? HXN : 1];
#pragma unroll
    for (int s = 0; s < HXN; ++s) {
        const int hr = wave + s * NW;
        hxok[s] = hr < 2 * R;
        const int x = (hr < R) ? x0 - R + hr : x0 + TX + hr - R;
        hxin[s] = hxok[s] && yin && x >= 0 && x < g.X;
        hxrow[s] = (hr < R) ? hr : TX + hr;
        hxoff[s] = g.origin + int64_t(x) * g.py + y;
    }
    int64_t hyoff[YHN];
    bool hyin[YHN], hyok[YHN];
    int hyrow[YHN], hycol[YHN];
#pragma unroll
    for (int s = 0; s < YHN; ++s) {
        const int e = threadIdx.x + s * NT;
        hyok[s] = e < TX * 2 * R;
        const int row = e / (2 * R), c = e % (2 * R);
        const int yy = (c < R) ? y0 - R + c : y0 + 64 + c - R;
        const int x = x0 + row;
        hyin[s] = hyok[s] && x < g.X && yy >= 0 && yy < g.Y;
        hyrow[s] = HXR + row;
        hycol[s] = (c < R) ? c : 64 + c;
        hyoff[s] = g.origin + int64_t(x) * g.py + yy;
    }

    const float *__restrict__ cur = P.cur;
    float *__restrict__ nxt = P.nxt;
    const float *__restrict__ Km = P.K;

    float q[RPT][2 * R + 1];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) {
            const int z = zb - R + k;
            q[i][k] = (rin[i] && z >= 0 && z < g.Z) ? cur[roff[i] + z * sz] : 0.0f;
        }

    // registers filled one plane ahead
    float nf[RPT], np_[RPT], nk[RPT], na[RPT], nb[RPT], nd[RPT], ng[RPT];
    float nhx[HXN > 0 ? HXN : 1], nhy[YHN];
    auto load = [&](int z) {
        const int zf = z + R;
        const int ez = max(0, max(g.lo[0] - z, z - (g.lo[0] + g.np[0] - 1)));
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int64_t o = roff[i] + z * sz;
            nf[i] = (rin[i] && zf < g.Z) ? cur[roff[i] + zf * sz] : 0.0f;
            np_[i] = rin[i] ? nxt[o] : 0.0f;
            nk[i] = rin[i] ? Km[o] : 0.0f;
            const int d2 = ez * ez + ex2[i];
            na[i] = 1.0f;
            nb[i] = 1.0f;
            if (rin[i] && d2 > 0) {
                const float2 ab = P.damp[d2];
                na[i] = ab.x;
                nb[i] = ab.y;
            }
            if constexpr (MODE == MODE_IMAGE) {
                nd[i] = rin[i] ? P.store[o] : 0.0f;
                ng[i] = rin[i] ? P.grad[o] : 0.0f;
            }
        }
#pragma unroll
        for (int s = 0; s < HXN; ++s) nhx[s] = hxin[s] ? cur[hxoff[s] + z * sz] : 0.0f;
#pragma unroll
        for (int s = 0; s < YHN; ++s) nhy[s] = hyin[s] ? cur[hyoff[s] + z * sz] : 0.0f;
    };

    load(zb);
    int buf = 0;
    for (int z = zb; z < ze; ++z) {
        float pp[RPT], pk[RPT], pa[RPT], pb[RPT], pd[RPT], pg[RPT];
        float hx[HXN > 0 ? HXN : 1], hy[YHN];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            q[i][2 * R] = nf[i];
            pp[i] = np_[i];
            pk[i] = nk[i];
            pa[i] = na[i];
            pb[i] = nb[i];
            if constexpr (MODE == MODE_IMAGE) {
                pd[i] = nd[i];
                pg[i] = ng[i];
            }
        }
#pragma unroll
        for (int s = 0; s < HXN; ++s) hx[s] = nhx[s];
#pragma unroll
        for (int s = 0; s < YHN; ++s) hy[s] = nhy[s];
        if (z + 1 < ze) load(z + 1);

        float(*T)[LY] = lds[buf];
#pragma unroll
        for (int i = 0; i < RPT; ++i) T[HXR + wave * RPT + i][R + lane] = q[i][R];
#pragma unroll
        for (int s = 0; s < HXN; ++s)
            if (hxok[s]) T[hxrow[s]][R + lane] = hx[s];
#pragma unroll
        for (int s = 0; s < YHN; ++s)
            if (hyok[s]) T[hyrow[s]][hycol[s]] = hy[s];
        __syncthreads();

#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int lx = HXR + wave * RPT + i, ly = R + lane;
            const float c = q[i][R];
            float lap = P.c0 * c;
#pragma unroll
            for (int j = 1; j <= R; ++j) lap = fmaf(P.cz[j], q[i][R + j] + q[i][R - j], lap);
            if constexpr (NDIM == 3) {
#pragma unroll
                for (int j = 1; j <= R; ++j) lap = fmaf(P.cx[j], T[lx + j][ly] + T[lx - j][ly], lap);
            }
#pragma unroll
            for (int j = 1; j <= R; ++j) lap = fmaf(P.cy[j], T[lx][ly + j] + T[lx][ly - j], lap);
            const float out = pa[i] * fmaf(pk[i], lap, 2.0f * c) - pb[i] * pp[i];
            if (rin[i]) {
                const int64_t o = roff[i] + z * sz;
                nxt[o] = out;
                if constexpr (MODE == MODE_STORE) P.store[o] = pk[i] * lap;
                if constexpr (MODE == MODE_IMAGE) P.grad[o] = fmaf(c, pd[i] / (pk[i] * pk[i]), pg[i]);
            }
        }
        buf ^= 1;
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) q[i][k] = q[i][k + 1];
    }
}

template <int R, int NDIM, int TX, int NW>
hipError_t launch_const_mode(int mode, const Tiling &t, StencilParams &P, hipStream_t s)
{
    const int nblocks = P.ntx * P.nty * P.nzc;
    const dim3 grid(nblocks), block(64 * NW);
    switch (mode) {
    case MODE_FWD: hipLaunchKernelGGL((k_const<R, NDIM, TX, NW, MODE_FWD>), grid, block, 0, s, P); break;
    case MODE_STORE: hipLaunchKernelGGL((k_const<R, NDIM, TX, NW, MODE_STORE>), grid, block, 0, s, P); break;
    default: hipLaunchKernelGGL((k_const<R, NDIM, TX, NW, MODE_IMAGE>), grid, block, 0, s, P); break;
    }
    (void)t;
    return hipGetLastError();
}

template <int R>
hipError_t launch_const_r(int ndim, int mode, const Tiling &t, StencilParams &P, hipStream_t s)
{
    if (ndim == 2) return launch_const_mode<R, 2, 1, 1>(mode, t, P, s);
    if (t.tx == 16 && t.nw == 4) return launch_const_mode<R, 3, 16, 4>(mode, t, P, s);
    if (t.tx == 8 && t.nw == 4) return launch_const_mode<R, 3, 8, 4>(mode, t, P, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_const(int r, int ndim, int mode, const Tiling &t, StencilParams &P, hipStream_t s)
{
    switch (r) {
    case 1: return launch_const_r<1>(ndim, mode, t, P, s);
    case 2: return launch_const_r<2>(ndim, mode, t, P, s);
    case 3: return launch_const_r<3>(ndim, mode, t, P, s);
    case 4: return launch_const_r<4>(ndim, mode, t, P, s);
    case 5: return launch_const_r<5>(ndim, mode, t, P, s);
    case 6: return launch_const_r<6>(ndim, mode, t, P, s);
    case 7: return launch_const_r<7>(ndim, mode, t, P, s);
    case 8: return launch_const_r<8>(ndim, mode, t, P, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sw
