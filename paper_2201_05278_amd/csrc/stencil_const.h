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
// Addresses are a per-plane base pointer (uniform) plus an unsigned 32-bit
// lane offset.  With NT = 1 the streamed arrays (p^{n-1}, K and the output)
// use non-temporal loads and stores so that the caches keep the p^n planes
// that neighbouring tiles re-read as halos.
//
// Modes: MODE_FWD plain step; MODE_STORE also writes K (L p) (the recomputed
// forward level of the imaging condition); MODE_IMAGE also accumulates
// grad += p * store / K^2 (zero-lag imaging of the adjoint field p against the
// stored level); MODE_IMAGE2 also takes the imaging term of the next adjoint
// step, deferred to this one, from the level p^{n-1} it reads anyway and the
// next step's stored level: grad = p store / K^2 + (p^{n-1} store2 / K^2 +
// grad), the two single steps' fused multiply-adds in their order, with the
// gradient read and written once for both.
#pragma once

#include "device.h"

namespace sw {

template <int NT>
__device__ __forceinline__ float ld_stream(const float *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <int NT>
__device__ __forceinline__ void st_stream(float v, float *p)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// The leapfrog update A (2 c + K lap) - B prev with its rounding pinned by
// explicit fused multiply-adds, so that every kernel that evaluates it (block
// tiles, wave tiles, batches, two-step sweeps) produces the same bits.
__device__ __forceinline__ float leapfrog(float a, float b, float k, float lap, float c, float prev)
{
    return fmaf(a, fmaf(k, lap, 2.0f * c), -(b * prev));
}

__device__ __forceinline__ double leapfrog(double a, double b, double k, double lap, double c, double prev)
{
    return fma(a, fma(k, lap, 2.0 * c), -(b * prev));
}

// Fused multiply-add of either value type.
__device__ __forceinline__ float fmat(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return fma(a, b, c); }

// Buffer addressing: a resource descriptor (base, byte size) per array and
// per z window, a per-thread 32-bit byte offset inside a plane and a uniform
// (scalar) byte offset of the plane, so that a load costs no vector address
// arithmetic.  Reads past the descriptor's size return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_res(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, int(bytes), 0x00020000);
}

template <int NT>
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, NT ? 2 : 0));
}

template <int NT>
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, NT ? 2 : 0);
}

__device__ __forceinline__ float2 buf_ld2(__amdgpu_buffer_rsrc_t r, int voff)
{
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0));
}

// The same accesses for a value type T (float: the functions above; double:
// 8-byte loads and stores, 16-byte damping pairs).
template <typename T, int NT>
__device__ __forceinline__ T buf_ldt(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    if constexpr (sizeof(T) == 4) return buf_ld<NT>(r, voff, soff);
    else return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, NT ? 2 : 0));
}

template <typename T, int NT>
__device__ __forceinline__ void buf_stt(T v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    if constexpr (sizeof(T) == 4) {
        buf_st<NT>(v, r, voff, soff);
    } else {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, NT ? 2 : 0);
    }
}

template <typename T>
__device__ __forceinline__ typename Pair<T>::type buf_ld2t(__amdgpu_buffer_rsrc_t r, int voff)
{
    if constexpr (sizeof(T) == 4) return buf_ld2(r, voff);
    else return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0));
}

// keep a loaded value (mask ~0) or replace it by +0 (mask 0)
__device__ __forceinline__ float keep_mask(float v, unsigned m)
{
    return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, v) & m);
}
__device__ __forceinline__ double keep_mask(double v, unsigned m)
{
    return __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, v) &
                                          ((unsigned long long)(m) << 32 | m));
}

// Register-queue length of the block tile: at least 2R + 1 planes, rounded
// up to a multiple of the slot and LDS-buffer periods so that a fully
// unrolled round of Q planes addresses every queue entry, load slot and LDS
// buffer with compile-time indices (no register moves).
template <int R, int PF>
constexpr int queue_len()
{
    constexpr int period = (PF + 1) % 2 == 0 ? PF + 1 : 2 * (PF + 1);
    return (2 * R + 1 + period - 1) / period * period;
}

// One tile (TX x 64 columns, one z chunk) of one grid; `bid` is the tile's
// index in (z chunk, x tile, y tile) order.  T: value type (float, or double
// for the double-precision forward).
template <typename T, int R, int NDIM, int TX, int NW, int MODE, int NT, int PF>
__device__ __forceinline__ void const_tile(const StencilParamsT<T> &P, int bid)
{
    using T2 = typename Pair<T>::type;
    constexpr int ES = int(sizeof(T));           // bytes per value
    static_assert(TX % NW == 0, "rows must split evenly over waves");
    static_assert(PF == 1 || PF == 2, "one or two planes of loads in flight");
    constexpr int RPT = TX / NW;                 // rows per thread
    constexpr int HXR = (NDIM == 3) ? R : 0;     // LDS halo rows in x
    constexpr int LY = 64 + 2 * R;
    constexpr int LX = TX + 2 * HXR;
    constexpr int NTH = 64 * NW;
    constexpr int HXN = (NDIM == 3) ? (2 * R + NW - 1) / NW : 0;   // x-halo rows per wave
    constexpr int YHN = (TX * 2 * R + NTH - 1) / NTH;               // y-halo items per thread
    constexpr int NS = PF + 1;                   // load slots
    constexpr int Q = queue_len<R, PF>();
    __shared__ T lds[2][LX + 1][LY];              // row LX: sink for idle halo lanes

    const Geom &g = P.g;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int tx, ty, zc;
    tile_of(bid, P.ntx, P.nty, P.xfast, tx, ty, zc);
    const int y0 = ty * 64;
    const int y = y0 + lane;
    const int x0 = tx * TX;
    const int zb = zc * P.zc;
    const int ze = min(zb + P.zc, g.Z);
    const int64_t sz = int64_t(g.px) * g.py;
    const bool yin = y < g.Y;
    const int ey = max(0, max(g.lo[2] - y, y - (g.lo[2] + g.np[2] - 1)));
    // z window of this chunk: planes zw .. zt - 1, plane z at byte offset (z - zw) * pb
    // (planes off the grid lie in the stored halo: they hold mirror ghosts, or are
    // masked to zero)
    const int zw = zb - R;
    const int zt = ze + R;
    const int pb = int(sz) * ES;
    const uint32_t wbytes = uint32_t(zt - zw) * uint32_t(pb);
    const int64_t w0 = g.base + int64_t(zw) * sz;
    const auto rc = buf_res(P.cur + w0, wbytes);
    const auto rn = buf_res(P.nxt + w0, wbytes);
    const auto rk = buf_res(P.K + w0, wbytes);
    const auto rd = buf_res(P.damp, uint32_t(P.ndamp) * uint32_t(sizeof(T2)));
    constexpr bool kImage = (MODE == MODE_IMAGE || MODE == MODE_IMAGE2);
    __amdgpu_buffer_rsrc_t rs = rk, rg = rk, rs2 = rk;
    if constexpr (MODE != MODE_FWD) rs = buf_res(P.store + w0, wbytes);
    if constexpr (kImage) rg = buf_res(P.grad + w0, wbytes);
    if constexpr (MODE == MODE_IMAGE2) rs2 = buf_res(P.store2 + w0, wbytes);
    // byte offset of plane z in the window
    auto soff = [&](int z) -> int { return (z - zw) * pb; };
    // planes read from memory: grid planes and mirror ghost planes
    auto zmask = [&](int z) -> unsigned {
        return axis_read(z, g.Z, P.bcm[0][0], P.bcm[0][1], P.gh) ? ~0u : 0u;
    };
    auto zdir = [&](int z) -> bool { return axis_dirichlet(z, g.Z, P.bcm[0][0], P.bcm[0][1]); };
    // in-plane byte offsets: (xy0 + x py + y) * ES; nodes off the grid (other
    // than mirror ghosts, for reads) get an offset past every window, so their
    // loads read zero and their stores are dropped
    auto off = [&](int x, int yy) -> int { return (g.xy0 + x * g.py + yy) * ES; };
    constexpr int kOut = 0x7ffffe00;
    auto rd_ok = [&](int x, int yy) -> bool {
        return axis_read(x, g.X, P.bcm[1][0], P.bcm[1][1], P.gh) &&
               axis_read(yy, g.Y, P.bcm[2][0], P.bcm[2][1], P.gh);
    };

    // the tile lies inside the physical box along x and y: (A, B) = (1, 1) on
    // every plane whose z is outside the layer, no table reads there
    const bool inner_xy = x0 >= g.lo[1] && x0 + TX <= g.lo[1] + g.np[1] && y0 >= g.lo[2] &&
                          y0 + 64 <= g.lo[2] + g.np[2];
    int ro[RPT], rr[RPT], ex2[RPT];
    bool rin[RPT], rdir[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int x = x0 + wave * RPT + i;
        rin[i] = yin && x < g.X;
        ro[i] = rin[i] ? off(x, y) : kOut;              // stores and per-node arrays
        rr[i] = rd_ok(x, y) ? off(x, y) : kOut;         // wavefield reads
        rdir[i] = axis_dirichlet(x, g.X, P.bcm[1][0], P.bcm[1][1]) ||
                  axis_dirichlet(y, g.Y, P.bcm[2][0], P.bcm[2][1]);
        const int ex = max(0, max(g.lo[1] - x, x - (g.lo[1] + g.np[1] - 1)));
        ex2[i] = rin[i] ? ex * ex + ey * ey : 0;      // keeps table reads in range
    }
    int hxo[HXN > 0 ? HXN : 1], hxrow[HXN > 0 ? HXN : 1];
    bool hxin[HXN > 0 ? HXN : 1], hxok[HXN > 0 ? HXN : 1];
#pragma unroll
    for (int s = 0; s < HXN; ++s) {
        const int hr = wave + s * NW;
        hxok[s] = hr < 2 * R;
        const int x = (hr < R) ? x0 - R + hr : x0 + TX + hr - R;
        hxin[s] = hxok[s] && rd_ok(x, y);
        hxrow[s] = !hxok[s] ? LX : (hr < R) ? hr : TX + hr;
        hxo[s] = hxin[s] ? off(x, y) : kOut;
    }
    int hyo[YHN], hyrow[YHN], hycol[YHN];
    bool hyin[YHN], hyok[YHN];
#pragma unroll
    for (int s = 0; s < YHN; ++s) {
        const int e = threadIdx.x + s * NTH;
        hyok[s] = e < TX * 2 * R;
        const int row = e / (2 * R), c = e % (2 * R);
        const int yy = (c < R) ? y0 - R + c : y0 + 64 + c - R;
        const int x = x0 + row;
        hyin[s] = hyok[s] && rd_ok(x, yy);
        hyrow[s] = hyok[s] ? HXR + row : LX;
        hycol[s] = (c < R) ? c : 64 + c;
        hyo[s] = hyin[s] ? off(x, yy) : kOut;
    }

    // q[i][(u + k) % Q] = p^n at plane z - R + k (k = 0 .. 2R) in unrolled step u
    T q[RPT][Q];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
        const int z = zb - R + k;
        const unsigned zm = zmask(z);
        const int so = soff(z);
#pragma unroll
        for (int i = 0; i < RPT; ++i) q[i][k] = keep_mask(buf_ldt<T, 0>(rc, rr[i], so), zm);
    }

    struct Slot {
        T f[RPT], p[RPT], k[RPT], d[RPT], g[RPT], d2[MODE == MODE_IMAGE2 ? RPT : 1];
        T2 ab[RPT];
        T hx[HXN > 0 ? HXN : 1], hy[YHN];
    };
    Slot S[NS];
    auto load = [&](int z, Slot &L) {
        const int zf = z + R;
        const unsigned fm = zmask(zf);
        const int so = soff(z), sf = soff(zf);
        const int ez = max(0, max(g.lo[0] - z, z - (g.lo[0] + g.np[0] - 1)));
        // (A, B) by squared layer distance (entry 0 is (1, 1)); skipped on interior tile planes
        if (!inner_xy || ez > 0) {
#pragma unroll
            for (int i = 0; i < RPT; ++i) L.ab[i] = buf_ld2t<T>(rd, (ez * ez + ex2[i]) * int(sizeof(T2)));
        } else {
#pragma unroll
            for (int i = 0; i < RPT; ++i) L.ab[i] = T2{T(1), T(1)};
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            L.f[i] = keep_mask(buf_ldt<T, 0>(rc, rr[i], sf), fm);
            L.p[i] = buf_ldt<T, NT>(rn, ro[i], so);
            L.k[i] = buf_ldt<T, NT>(rk, ro[i], so);
            if constexpr (kImage) {
                L.d[i] = buf_ldt<T, NT>(rs, ro[i], so);
                L.g[i] = buf_ldt<T, NT>(rg, ro[i], so);
            }
            if constexpr (MODE == MODE_IMAGE2) L.d2[i] = buf_ldt<T, NT>(rs2, ro[i], so);
        }
#pragma unroll
        for (int s = 0; s < HXN; ++s) L.hx[s] = buf_ldt<T, 0>(rc, hxo[s], so);
#pragma unroll
        for (int s = 0; s < YHN; ++s) L.hy[s] = buf_ldt<T, 0>(rc, hyo[s], so);
    };

#pragma unroll
    for (int j = 0; j < PF; ++j)
        if (zb + j < ze) load(zb + j, S[j]);
    for (int zz = zb; zz < ze; zz += Q) {
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            const int z = zz + u;
            if (z < ze) {
                Slot &W = S[u % NS];
                if (z + PF < ze) load(z + PF, S[(u + PF) % NS]);
                T(*Tl)[LY] = lds[u % 2];
#pragma unroll
                for (int i = 0; i < RPT; ++i) q[i][(u + 2 * R) % Q] = W.f[i];
#pragma unroll
                for (int i = 0; i < RPT; ++i) Tl[HXR + wave * RPT + i][R + lane] = q[i][(u + R) % Q];
#pragma unroll
                for (int s = 0; s < HXN; ++s) Tl[hxrow[s]][R + lane] = W.hx[s];
#pragma unroll
                for (int s = 0; s < YHN; ++s) Tl[hyrow[s]][hycol[s]] = W.hy[s];
                __syncthreads();

                const int so = soff(z);
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int lx = HXR + wave * RPT + i, ly = R + lane;
                    const T c = q[i][(u + R) % Q];
                    T lap = P.c0 * c;
#pragma unroll
                    for (int j = 1; j <= R; ++j)
                        lap = fmat(P.cz[j], q[i][(u + R + j) % Q] + q[i][(u + R - j) % Q], lap);
                    if constexpr (NDIM == 3) {
#pragma unroll
                        for (int j = 1; j <= R; ++j) lap = fmat(P.cx[j], Tl[lx + j][ly] + Tl[lx - j][ly], lap);
                    }
#pragma unroll
                    for (int j = 1; j <= R; ++j) lap = fmat(P.cy[j], Tl[lx][ly + j] + Tl[lx][ly - j], lap);
                    T out = leapfrog(W.ab[i].x, W.ab[i].y, W.k[i], lap, c, W.p[i]);
                    if (rdir[i] || zdir(z)) out = T(0);     // held by a Dirichlet condition
                    buf_stt<T, NT>(out, rn, ro[i], so);
                    if constexpr (MODE == MODE_STORE) buf_stt<T, NT>(W.k[i] * lap, rs, ro[i], so);
                    if constexpr (MODE == MODE_IMAGE)
                        buf_stt<T, NT>(fmat(c, W.d[i] / (W.k[i] * W.k[i]), W.g[i]), rg, ro[i], so);
                    if constexpr (MODE == MODE_IMAGE2) {
                        const T k2 = W.k[i] * W.k[i];
                        buf_stt<T, NT>(fmat(c, W.d[i] / k2, fmat(W.p[i], W.d2[i] / k2, W.g[i])), rg, ro[i], so);
                    }
                }
            }
        }
    }
}

// Wave tiles: every wavefront owns RW consecutive x rows of 64 columns and
// marches along z on its own.  The x neighbours inside the wave's rows are the
// centres of its own register queues; the R rows above and below come from
// halo loads of the current plane; the y neighbours go through a row buffer in
// LDS private to the wave.  No block-wide barrier is needed (a block is NWB
// independent waves, RW * NWB rows).
template <int R, int NDIM, int RW, int NWB, int MODE, int NT>
__device__ __forceinline__ void const_wave_tile(const StencilParams &P, int bid)
{
    constexpr int HX = (NDIM == 3) ? R : 0;
    constexpr int LY = 64 + 2 * R;
    constexpr int YH = (RW * 2 * R + 63) / 64;      // y-halo items per lane
    __shared__ float lds[NWB][RW][LY];

    const Geom &g = P.g;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int tx, ty, zc;
    tile_of(bid, P.ntx, P.nty, P.xfast, tx, ty, zc);
    const int y0 = ty * 64;
    const int y = y0 + lane;
    const int xw = tx * (RW * NWB) + wave * RW;     // first row of this wave
    const int zb = zc * P.zc;
    const int ze = min(zb + P.zc, g.Z);
    const int64_t sz = int64_t(g.px) * g.py;
    const bool yin = y < g.Y;
    const int ey = max(0, max(g.lo[2] - y, y - (g.lo[2] + g.np[2] - 1)));
    auto off = [&](int x, int yy) -> unsigned { return unsigned(g.xy0 + x * g.py + yy); };
    const float *cur0 = P.cur + g.base;
    float *nxt0 = P.nxt + g.base;
    const float *k0 = P.K + g.base;
    float(*T)[LY] = lds[wave];

    unsigned ro[RW];
    bool rin[RW];
    int ex2[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int x = xw + i;
        rin[i] = yin && x < g.X;
        ro[i] = rin[i] ? off(x, y) : 0u;
        const int ex = max(0, max(g.lo[1] - x, x - (g.lo[1] + g.np[1] - 1)));
        ex2[i] = ex * ex + ey * ey;
    }
    // halo rows xw-R .. xw-1 (lo) and xw+RW .. xw+RW+R-1 (hi)
    unsigned hlo[HX > 0 ? HX : 1], hhi[HX > 0 ? HX : 1];
    bool ilo[HX > 0 ? HX : 1], ihi[HX > 0 ? HX : 1];
#pragma unroll
    for (int j = 0; j < HX; ++j) {
        const int xl = xw - R + j, xh = xw + RW + j;
        ilo[j] = yin && xl >= 0 && xl < g.X;
        ihi[j] = yin && xh < g.X;
        hlo[j] = ilo[j] ? off(xl, y) : 0u;
        hhi[j] = ihi[j] ? off(xh, y) : 0u;
    }
    // y-halo items: RW rows x 2R columns spread over the lanes
    unsigned hyo[YH];
    bool hyin[YH], hyok[YH];
    int hyrow[YH], hycol[YH];
#pragma unroll
    for (int s = 0; s < YH; ++s) {
        const int e = lane + 64 * s;
        hyok[s] = e < RW * 2 * R;
        const int row = e / (2 * R), c = e % (2 * R);
        const int yy = (c < R) ? y0 - R + c : y0 + 64 + c - R;
        const int x = xw + row;
        hyin[s] = hyok[s] && x < g.X && yy >= 0 && yy < g.Y;
        hyrow[s] = hyok[s] ? row : 0;
        hycol[s] = (c < R) ? c : 64 + c;
        hyo[s] = hyin[s] ? off(x, yy) : 0u;
    }

    float q[RW][2 * R + 1];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
        const int z = zb - R + k;
        const bool zin = z >= 0 && z < g.Z;
        const float *pl = cur0 + int64_t(z) * sz;
#pragma unroll
        for (int i = 0; i < RW; ++i) q[i][k] = (rin[i] && zin) ? pl[ro[i]] : 0.0f;
    }

    struct Slot {
        float f[RW], p[RW], k[RW], a[RW], b[RW], d[RW], g[RW];
        float lo[HX > 0 ? HX : 1], hi[HX > 0 ? HX : 1], hy[YH];
    };
    auto load = [&](int z, Slot &S) {
        const int zf = z + R;
        const int ez = max(0, max(g.lo[0] - z, z - (g.lo[0] + g.np[0] - 1)));
        const float *pc = cur0 + int64_t(z) * sz;
        const float *pf = cur0 + int64_t(zf) * sz;
        const float *pn = nxt0 + int64_t(z) * sz;
        const float *pk = k0 + int64_t(z) * sz;
        const bool fin = zf < g.Z;
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            S.f[i] = (rin[i] && fin) ? pf[ro[i]] : 0.0f;
            S.p[i] = rin[i] ? ld_stream<NT>(pn + ro[i]) : 0.0f;
            S.k[i] = rin[i] ? ld_stream<NT>(pk + ro[i]) : 0.0f;
            const int d2 = ez * ez + ex2[i];
            S.a[i] = 1.0f;
            S.b[i] = 1.0f;
            if (rin[i] && d2 > 0) {
                const float2 ab = P.damp[d2];
                S.a[i] = ab.x;
                S.b[i] = ab.y;
            }
            if constexpr (MODE == MODE_IMAGE) {
                const int64_t o = int64_t(z) * sz + g.base + ro[i];
                S.d[i] = rin[i] ? ld_stream<NT>(P.store + o) : 0.0f;
                S.g[i] = rin[i] ? ld_stream<NT>(P.grad + o) : 0.0f;
            }
        }
#pragma unroll
        for (int j = 0; j < HX; ++j) {
            S.lo[j] = ilo[j] ? pc[hlo[j]] : 0.0f;
            S.hi[j] = ihi[j] ? pc[hhi[j]] : 0.0f;
        }
#pragma unroll
        for (int s = 0; s < YH; ++s) S.hy[s] = hyin[s] ? pc[hyo[s]] : 0.0f;
    };

    Slot S;
    load(zb, S);
    for (int z = zb; z < ze; ++z) {
        const Slot W = S;
        if (z + 1 < ze) load(z + 1, S);
#pragma unroll
        for (int i = 0; i < RW; ++i) q[i][2 * R] = W.f[i];
        // y neighbours through the wave's own LDS rows (DS operations of one
        // wave complete in order; the fence keeps the compiler from moving
        // this plane's reads across the writes)
#pragma unroll
        for (int i = 0; i < RW; ++i) T[i][R + lane] = q[i][R];
#pragma unroll
        for (int s = 0; s < YH; ++s)
            if (hyok[s]) T[hyrow[s]][hycol[s]] = W.hy[s];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        float *pn = nxt0 + int64_t(z) * sz;
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const float c = q[i][R];
            float lap = P.c0 * c;
#pragma unroll
            for (int j = 1; j <= R; ++j) lap = fmaf(P.cz[j], q[i][R + j] + q[i][R - j], lap);
            if constexpr (NDIM == 3) {
#pragma unroll
                for (int j = 1; j <= R; ++j) {
                    const float up = (i + j < RW) ? q[(i + j) % RW][R] : W.hi[(i + j - RW) % (HX > 0 ? HX : 1)];
                    const float dn = (i - j >= 0) ? q[(i - j + RW) % RW][R] : W.lo[(R + i - j) % (HX > 0 ? HX : 1)];
                    lap = fmaf(P.cx[j], up + dn, lap);
                }
            }
#pragma unroll
            for (int j = 1; j <= R; ++j) lap = fmaf(P.cy[j], T[i][R + lane + j] + T[i][R + lane - j], lap);
            const float out = leapfrog(W.a[i], W.b[i], W.k[i], lap, c, W.p[i]);
            if (rin[i]) {
                st_stream<NT>(out, pn + ro[i]);
                const int64_t o = int64_t(z) * sz + g.base + ro[i];
                if constexpr (MODE == MODE_STORE) st_stream<NT>(W.k[i] * lap, P.store + o);
                if constexpr (MODE == MODE_IMAGE)
                    st_stream<NT>(fmaf(c, W.d[i] / (W.k[i] * W.k[i]), W.g[i]), P.grad + o);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int i = 0; i < RW; ++i)
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) q[i][k] = q[i][k + 1];
    }
}

template <int R, int NDIM, int RW, int NWB, int MODE, int NT>
__global__ void __launch_bounds__(64 * NWB) k_const_wave(StencilParams P)
{
    const_wave_tile<R, NDIM, RW, NWB, MODE, NT>(P, xcd_remap(blockIdx.x, gridDim.x));
}

// Tall tiles of 8 waves (3 or more rows per thread) are held to 128 VGPRs so
// that two blocks share a CU (up to radius 4; larger radii would spill).
template <int R, int TX, int NW>
constexpr int const_min_waves()
{
    return (R <= 4 && NW == 8 && TX / NW >= 3) ? 4 : 1;
}

template <int R, int NDIM, int TX, int NW, int MODE, int NT, int PF>
__global__ void __launch_bounds__(64 * NW, (const_min_waves<R, TX, NW>())) k_const(StencilParams P)
{
    const_tile<float, R, NDIM, TX, NW, MODE, NT, PF>(P, xcd_remap(blockIdx.x, gridDim.x));
}

// Many grids (shots) in one launch: the tiles of all shots form one list
// (shot s owns [tile_start[s], tile_start[s+1])); each block takes tiles
// blockIdx, blockIdx + gridDim, ... (XCD-aware; one tile when the grid has a
// block per tile), looks up the shot and runs the same tile code on that
// shot's arrays.  `parity` swaps the two wavefield buffers of every shot.
template <int R, int NDIM, int TX, int NW, int NT, int PF>
__global__ void __launch_bounds__(64 * NW) k_const_batch(const StencilParams *__restrict__ shots,
                                                         const int *__restrict__ tile_start,
                                                         int nshots, int parity)
{
    const int total = tile_start[nshots];
    const int first = xcd_remap(blockIdx.x, gridDim.x);
    for (int t = first; t < total; t += gridDim.x) {
        int lo = 0, hi = nshots - 1;          // last shot with tile_start <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_start[mid] <= t) lo = mid; else hi = mid - 1;
        }
        StencilParams P = shots[lo];
        if (parity) {
            float *c = const_cast<float *>(P.cur);
            P.cur = P.nxt;
            P.nxt = c;
        }
        const_tile<float, R, NDIM, TX, NW, MODE_FWD, NT, PF>(P, t - tile_start[lo]);
        __syncthreads();                      // LDS is reused by the next tile
    }
}

// Tile shapes (rows, waves) instantiated for 3D grids; 2D grids use (1, 1).
#define SW_CONST_SHAPES(X) X(16, 4) X(8, 4) X(32, 8) X(16, 8) X(8, 8) X(24, 8)

template <int R, int NDIM, int TX, int NW, int MODE, int NT, int PF>
void launch_const_mode(int occ, StencilParams &P, hipStream_t s)
{
    constexpr auto kern = k_const<R, NDIM, TX, NW, MODE, NT, PF>;
    const unsigned pad = occ ? occ_pad_bytes(occ, static_lds_of<kern>()) : 0u;
    hipLaunchKernelGGL(kern, dim3(P.ntx * P.nty * P.nzc), dim3(64 * NW), pad, s, P);
}

template <int R, int NDIM, int TX, int NW, int NT, int PF>
hipError_t launch_const_shape(int mode, int occ, StencilParams &P, hipStream_t s)
{
    switch (mode) {
    case MODE_FWD: launch_const_mode<R, NDIM, TX, NW, MODE_FWD, NT, PF>(occ, P, s); break;
    case MODE_STORE: launch_const_mode<R, NDIM, TX, NW, MODE_STORE, NT, PF>(occ, P, s); break;
    case MODE_IMAGE: launch_const_mode<R, NDIM, TX, NW, MODE_IMAGE, NT, PF>(occ, P, s); break;
    case MODE_IMAGE2: launch_const_mode<R, NDIM, TX, NW, MODE_IMAGE2, NT, PF>(occ, P, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Wave-tile shapes (rows per wave, waves per block).
#define SW_WAVE_SHAPES(X) X(4, 4) X(8, 4) X(4, 1) X(8, 1) X(8, 2)

template <int R, int NDIM, int RW, int NWB, int NT>
hipError_t launch_wave_shape(int mode, StencilParams &P, hipStream_t s)
{
    const dim3 grid(P.ntx * P.nty * P.nzc), block(64 * NWB);
    switch (mode) {
    case MODE_FWD: hipLaunchKernelGGL((k_const_wave<R, NDIM, RW, NWB, MODE_FWD, NT>), grid, block, 0, s, P); break;
    case MODE_STORE: hipLaunchKernelGGL((k_const_wave<R, NDIM, RW, NWB, MODE_STORE, NT>), grid, block, 0, s, P); break;
    case MODE_IMAGE: hipLaunchKernelGGL((k_const_wave<R, NDIM, RW, NWB, MODE_IMAGE, NT>), grid, block, 0, s, P); break;
    default: return hipErrorInvalidValue;       // the paired imaging step runs on block tiles
    }
    return hipGetLastError();
}

template <int R, int NT, int PF>
hipError_t launch_const_v(int ndim, int mode, const Tiling &t, StencilParams &P, hipStream_t s)
{
    if (ndim == 2) return launch_const_shape<R, 2, 1, 1, NT, PF>(mode, t.occ, P, s);
    if (t.wt) {
#define SW_X(RWV, NWV) \
        if (t.tx == RWV * NWV && t.nw == NWV) return launch_wave_shape<R, 3, RWV, NWV, NT>(mode, P, s);
        SW_WAVE_SHAPES(SW_X)
#undef SW_X
        return hipErrorInvalidValue;
    }
#define SW_X(TXV, NWV) \
    if (t.tx == TXV && t.nw == NWV) return launch_const_shape<R, 3, TXV, NWV, NT, PF>(mode, t.occ, P, s);
    SW_CONST_SHAPES(SW_X)
#undef SW_X
    return hipErrorInvalidValue;
}

// Resident blocks per CU of the forward block-tile kernel of a 3D tiling (with
// its occupancy cap), from the runtime's occupancy calculator; 0 if unknown.
template <int R, int TX, int NW, int NT, int PF>
int const_resident_shape(int occ)
{
    constexpr auto kern = k_const<R, 3, TX, NW, MODE_FWD, NT, PF>;
    const unsigned pad = occ ? occ_pad_bytes(occ, static_lds_of<kern>()) : 0u;
    int n = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, 64 * NW, pad) == hipSuccess ? n : 0;
}

template <int R, int NT, int PF>
int const_resident_v(const Tiling &t)
{
#define SW_X(TXV, NWV) \
    if (t.tx == TXV && t.nw == NWV) return const_resident_shape<R, TXV, NWV, NT, PF>(t.occ);
    SW_CONST_SHAPES(SW_X)
#undef SW_X
    return 0;
}

template <int R>
int const_resident_radius(const Tiling &t)
{
    if (t.wt || t.ts == 2) return 0;
    if (t.pf == 2) return t.nt ? const_resident_v<R, 1, 2>(t) : const_resident_v<R, 0, 2>(t);
    return t.nt ? const_resident_v<R, 1, 1>(t) : const_resident_v<R, 0, 1>(t);
}

template <int R>
hipError_t launch_const_radius(int ndim, int mode, const Tiling &t, StencilParams &P, hipStream_t s)
{
    if (t.pf == 2)
        return t.nt ? launch_const_v<R, 1, 2>(ndim, mode, t, P, s) : launch_const_v<R, 0, 2>(ndim, mode, t, P, s);
    return t.nt ? launch_const_v<R, 1, 1>(ndim, mode, t, P, s) : launch_const_v<R, 0, 1>(ndim, mode, t, P, s);
}

template <int R, int NT, int PF>
hipError_t launch_batch_v(int ndim, const Tiling &t, const StencilParams *shots, const int *tile_start,
                          int nshots, int parity, int nblocks, hipStream_t s)
{
    if (ndim == 2) {
        hipLaunchKernelGGL((k_const_batch<R, 2, 1, 1, NT, PF>), dim3(nblocks), dim3(64), 0, s, shots,
                           tile_start, nshots, parity);
        return hipGetLastError();
    }
#define SW_X(TXV, NWV)                                                                               \
    if (t.tx == TXV && t.nw == NWV) {                                                                \
        hipLaunchKernelGGL((k_const_batch<R, 3, TXV, NWV, NT, PF>), dim3(nblocks), dim3(64 * NWV), 0, s, \
                           shots, tile_start, nshots, parity);                                       \
        return hipGetLastError();                                                                    \
    }
    SW_CONST_SHAPES(SW_X)
#undef SW_X
    return hipErrorInvalidValue;
}

template <int R>
hipError_t launch_batch_radius(int ndim, const Tiling &t, const StencilParams *shots, const int *tile_start,
                               int nshots, int parity, int nblocks, hipStream_t s)
{
    if (t.pf == 2)
        return t.nt ? launch_batch_v<R, 1, 2>(ndim, t, shots, tile_start, nshots, parity, nblocks, s)
                    : launch_batch_v<R, 0, 2>(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
    return t.nt ? launch_batch_v<R, 1, 1>(ndim, t, shots, tile_start, nshots, parity, nblocks, s)
                : launch_batch_v<R, 0, 1>(ndim, t, shots, tile_start, nshots, parity, nblocks, s);
}

}  // namespace sw
