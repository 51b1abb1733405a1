// Variable-density leapfrog stencils, damping fused as in the constant-density
// kernel (A, B from the squared layer distance).
//
// Staggered (conservative) operator, K = dt^2 rho c^2, b = 1/rho:
//   L p = sum_i D-_i (b_{i+1/2} D+_i p)
//   (D+ q)_{k+1/2} = sum_j s_j (q_{k+j} - q_{k-j+1}) / h
//   (D- F)_k       = sum_j s_j (F_{k+j-1/2} - F_{k-j+1/2}) / h
//   b_{k+1/2}      = sum_j m_j (b_{k+j} + b_{k-j+1})
// Every face flux is formed once per face.  Along z the fluxes are produced as
// the march reaches each face and kept in a register queue, fed by register
// queues of p and b in front of the node; the x and y fluxes of the tile's
// plane are formed once into LDS from LDS tiles of p and b (halo 2R - 1) and
// differenced from there.  The face buoyancies are interpolated from b inside
// the kernel, so the sweep streams p^n, p^{n-1}, K and b (20 bytes per node)
// rather than three stored face arrays.
//
// Centred operator (paper, "Time discretization": expanded variable-density
// equation), K = dt^2 c^2:
//   L p = sum_i [ D2_i p - (D1_i rho / rho) D1_i p ]
// with the centred second and first derivatives; rho is staged like p (halo R)
// with its own register queue along z.
//
// Model values outside the extended grid are those of its model node (mirror
// image across mirrored sides, nearest node elsewhere): the staggered kernel
// reads b from the stored halo, which model preparation fills that way; the
// centred kernel maps rho's coordinates itself.  Wavefield values outside it
// are zero or mirror ghosts.
#pragma once

#include "device.h"
#include "stencil_const.h"

namespace sw {


template <int R, int NDIM, int TX, int NW, int NT, int MODE = MODE_FWD>
__global__ void __launch_bounds__(64 * NW) k_stag(StencilParams P)
{
    static_assert(TX % NW == 0, "rows must split evenly over waves");
    static_assert(NDIM == 3 || TX == 1, "2D grids use one row per tile");
    constexpr int RPT = TX / NW;
    constexpr int H = 2 * R - 1;                  // node halo of the face fluxes
    constexpr int HX = (NDIM == 3) ? H : 0;
    constexpr int LY = 64 + 2 * H;
    constexpr int LX = TX + 2 * HX;
    constexpr int FX = (NDIM == 3) ? TX + 2 * R - 1 : 1;   // x faces x0-R+t+1/2, t < FX
    constexpr int FY = 64 + 2 * R - 1;                     // y faces y0-R+c+1/2, c < FY
    constexpr int NTH = 64 * NW;
    constexpr int HXN = (NDIM == 3) ? (2 * HX + NW - 1) / NW : 0;   // x-halo rows per wave
    constexpr int YHN = (TX * 2 * H + NTH - 1) / NTH;               // y-halo items per thread
    constexpr int FXR = (NDIM == 3) ? FX : 0;     // x-face rows
    // face items: runs of MX consecutive x faces of one column (NRX runs per
    // column: the 64 columns of a run index fill a wavefront), then runs of MY
    // consecutive y faces of one tile row.  A run reads its p and b values once
    // into registers (y runs with 16-byte LDS reads) and forms each face flux
    // from them.
    // (short runs: about 6 x faces, 4 y faces; longer runs that fit all items
    // in one pass of the block's threads ran slower at 592^3: more registers,
    // fewer resident waves)
    constexpr int NRX = (NDIM == 3) ? (FXR + 5) / 6 : 0;
    constexpr int MX = (NDIM == 3) ? (FXR + NRX - 1) / NRX : 1;
    constexpr int MY = 4;
    constexpr int NRY = (FY + MY - 1) / MY;
    constexpr int NVY = (MY + 2 * R - 1 + 3) / 4 * 4;       // values a y run reads (float4 multiple)
    constexpr int LYP = (NRY * MY + 2 * R - 1 + 3) / 4 * 4 > LY ? (NRY * MY + 2 * R - 1 + 3) / 4 * 4 : LY;
    constexpr int SPR = NRX * MX + 2 * R - 1 > LX + 1 ? NRX * MX + 2 * R - 1 : LX + 1;
    constexpr int NI = NRX * 64 + TX * NRY;
    constexpr int NIT = (NI + NTH - 1) / NTH;     // face items per thread
    constexpr int Q = 2 * R;                      // queue length (even: slots alternate)
    constexpr int kOut = 0x7ffffe00;
    // p and b of the plane (row LX: sink for idle halo items; rows past it are
    // only read by the faces of the last x run beyond the tile's faces);
    // 16-byte aligned rows for the y runs' vector reads
    __shared__ __align__(16) float sp[SPR][LYP];
    __shared__ __align__(16) float sb[SPR][LYP];
    __shared__ float sfx[NRX * MX + 1][64];
    __shared__ __align__(16) float sfy[TX + 1][NRY * MY];

    const Geom &g = P.g;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
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
    // z window: planes zw .. zt - 1 (the queues reach 2R - 1 planes ahead; planes
    // off the grid lie in the stored halo of 2R planes: wavefield planes there
    // hold mirror ghosts or are masked, model planes hold the model's ghosts)
    const int zw = zb - 2 * R + 1;
    const int zt = ze + 2 * R - 1;
    const int pb = int(sz) * 4;
    const uint32_t wbytes = uint32_t(zt - zw) * uint32_t(pb);
    const int64_t w0 = g.base + int64_t(zw) * sz;
    const auto rc = buf_res(P.cur + w0, wbytes);
    const auto rn = buf_res(P.nxt + w0, wbytes);
    const auto rb = buf_res(P.aux + w0, wbytes);
    const auto rk = buf_res(P.K + w0, wbytes);
    const auto rd = buf_res(P.damp, uint32_t(P.ndamp) * 8u);
    // imaging arrays share the wavefield layout and window
    __amdgpu_buffer_rsrc_t rs = rk, ru = rk, rg = rk;
    // imaging modes: one term per step, or (MODE_IMAGE2) this step's and the
    // next step's deferred term, from the p^{n-1} level read anyway and that
    // step's stored level (the two single steps' fused multiply-adds in order)
    constexpr bool kImage = (MODE == MODE_IMAGE || MODE == MODE_IMAGE2);
    __amdgpu_buffer_rsrc_t rs2 = rk;
    if constexpr (MODE != MODE_FWD) rs = buf_res(P.store + w0, wbytes);
    if constexpr (MODE == MODE_STORE) ru = buf_res(P.ustore + w0, wbytes);
    if constexpr (kImage) rg = buf_res(P.grad + w0, wbytes);
    if constexpr (MODE == MODE_IMAGE2) rs2 = buf_res(P.store2 + w0, wbytes);
    auto soff = [&](int z) -> int { return (z - zw) * pb; };
    auto zmask = [&](int z) -> unsigned {
        return axis_read(z, g.Z, P.bcm[0][0], P.bcm[0][1], P.gh) ? ~0u : 0u;
    };
    auto keep = [](float v, unsigned m) -> float {
        return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, v) & m);
    };
    // byte offsets in a plane: wavefield (zero off the grid); wavefield reads
    // (also mirror ghosts within the stored halo); model reads (the whole stored
    // halo of 2R nodes, which feeds every face of the grid's nodes; positions
    // beyond it only feed nodes off the grid and read zero)
    auto off = [&](int x, int yy) -> int {
        return (x >= 0 && x < g.X && yy >= 0 && yy < g.Y) ? (g.xy0 + x * g.py + yy) * 4 : kOut;
    };
    auto roff = [&](int x, int yy) -> int {
        const bool ok = axis_read(x, g.X, P.bcm[1][0], P.bcm[1][1], P.gh) &&
                        axis_read(yy, g.Y, P.bcm[2][0], P.bcm[2][1], P.gh);
        return ok ? (g.xy0 + x * g.py + yy) * 4 : kOut;
    };
    auto moff = [&](int x, int yy) -> int {
        const bool ok = (NDIM == 2 || (x >= -2 * R && x < g.X + 2 * R)) && yy >= -2 * R && yy < g.Y + 2 * R;
        return ok ? (g.xy0 + x * g.py + yy) * 4 : kOut;
    };

    int ro[RPT], rr[RPT], rm[RPT], ex2[RPT];
    bool rdir[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int x = x0 + wave * RPT + i;
        const bool in = yin && x < g.X;
        ro[i] = off(x, y);
        rr[i] = roff(x, y);
        rm[i] = moff(x, y);
        rdir[i] = axis_dirichlet(x, g.X, P.bcm[1][0], P.bcm[1][1]) ||
                  axis_dirichlet(y, g.Y, P.bcm[2][0], P.bcm[2][1]);
        const int ex = max(0, max(g.lo[1] - x, x - (g.lo[1] + g.np[1] - 1)));
        ex2[i] = in ? ex * ex + ey * ey : 0;
    }
    int hxo[HXN > 0 ? HXN : 1], hxm[HXN > 0 ? HXN : 1], hxrow[HXN > 0 ? HXN : 1];
#pragma unroll
    for (int s = 0; s < HXN; ++s) {
        const int hr = wave + s * NW;
        const bool ok = hr < 2 * HX;
        const int x = (hr < HX) ? x0 - HX + hr : x0 + TX + hr - HX;
        hxo[s] = ok ? roff(x, y) : kOut;
        hxm[s] = ok ? moff(x, y) : kOut;
        hxrow[s] = !ok ? LX : (hr < HX) ? hr : TX + hr;
    }
    int hyo[YHN], hym[YHN], hyrow[YHN], hycol[YHN];
#pragma unroll
    for (int s = 0; s < YHN; ++s) {
        const int e = threadIdx.x + s * NTH;
        const bool ok = e < TX * 2 * H;
        const int row = e / (2 * H), c = e % (2 * H);
        const int yy = (c < H) ? y0 - H + c : y0 + 64 + c - H;
        const int x = x0 + row;
        hyo[s] = ok ? roff(x, yy) : kOut;
        hym[s] = ok ? moff(x, yy) : kOut;
        hyrow[s] = ok ? HX + row : LX;
        hycol[s] = (c < H) ? c : 64 + c;
    }

    // queues, rotating with the unrolled step u: pq[(u + k) % Q] = p(z + k) and
    // bq[(u + k) % Q] = b(z + k), fq[(u + k) % Q] = z flux at face (z - R + k) + 1/2
    float pq[RPT][Q], bq[RPT][Q], fq[RPT][Q];
    const int zs = zb - 2 * R + 1;
#pragma unroll
    for (int k = 0; k < 2 * R - 1; ++k) {
        const int z = zs + k;
        const unsigned m = zmask(z);
        const int so = soff(z);
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            pq[i][k] = keep(buf_ld<0>(rc, rr[i], so), m);
            bq[i][k] = buf_ld<0>(rb, rm[i], so);
        }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) fq[i][k] = 0.0f;

    struct Slot {
        float fp[RPT], fb[RPT], p[RPT], k[RPT];
        float2 ab[RPT];
        float hxp[HXN > 0 ? HXN : 1], hxb[HXN > 0 ? HXN : 1], hyp[YHN], hyb[YHN];
        float d[kImage ? RPT : 1], gr[kImage ? RPT : 1], d2[MODE == MODE_IMAGE2 ? RPT : 1];
    };
    // loads of plane z: the queue inputs p and b at z + 2R - 1, and for z >= zb
    // the plane's own p^{n-1}, K, (A, B) and the halos of p and b
    auto load = [&](int z, Slot &L) {
        const int zf = z + 2 * R - 1;
        const unsigned mf = zmask(zf);
        const int sf = soff(zf);
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            L.fp[i] = keep(buf_ld<0>(rc, rr[i], sf), mf);
            L.fb[i] = buf_ld<0>(rb, rm[i], sf);
        }
        if (z < zb) return;
        const int so = soff(z);
        const int ez = max(0, max(g.lo[0] - z, z - (g.lo[0] + g.np[0] - 1)));
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            L.p[i] = buf_ld<NT>(rn, ro[i], so);
            L.k[i] = buf_ld<NT>(rk, ro[i], so);
            L.ab[i] = buf_ld2(rd, (ez * ez + ex2[i]) * 8);
            if constexpr (kImage) {
                L.d[i] = buf_ld<NT>(rs, ro[i], so);
                L.gr[i] = buf_ld<NT>(rg, ro[i], so);
            }
            if constexpr (MODE == MODE_IMAGE2) L.d2[i] = buf_ld<NT>(rs2, ro[i], so);
        }
#pragma unroll
        for (int s = 0; s < HXN; ++s) {
            L.hxp[s] = buf_ld<0>(rc, hxo[s], so);
            L.hxb[s] = buf_ld<0>(rb, hxm[s], so);
        }
#pragma unroll
        for (int s = 0; s < YHN; ++s) {
            L.hyp[s] = buf_ld<0>(rc, hyo[s], so);
            L.hyb[s] = buf_ld<0>(rb, hym[s], so);
        }
    };

    // face buoyancy b_{m+1/2} = sum_l m_l (b_{m+l} + b_{m-l+1}), fused
    // multiply-adds in the order l = 1 .. R, from values v(k) = b_{m+k}
    auto bface = [&](auto v) -> float {
        float acc = 0.0f;
#pragma unroll
        for (int l = 1; l <= R; ++l) acc = fmaf(P.mj[l], v(l) + v(1 - l), acc);
        return acc;
    };

    Slot S[2];
    load(zs, S[0]);
    for (int zz = zs; zz < ze; zz += Q) {
#pragma unroll
    for (int u = 0; u < Q; ++u) {
        const int z = zz + u;
        if (z >= ze) break;
        Slot &W = S[u % 2];
        if (z + 1 < ze) load(z + 1, S[(u + 1) % 2]);
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            pq[i][(u + 2 * R - 1) % Q] = W.fp[i];
            bq[i][(u + 2 * R - 1) % Q] = W.fb[i];
        }
        // z flux at face (z + R - 1) + 1/2
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            float dp = 0.0f;
#pragma unroll
            for (int l = 1; l <= R; ++l)
                dp = fmaf(P.sz[l], pq[i][(u + R - 1 + l) % Q] - pq[i][(u + R - l) % Q], dp);
            const float bf = bface([&](int k) { return bq[i][(u + R - 1 + k + Q) % Q]; });
            fq[i][(u + 2 * R - 1) % Q] = bf * dp;
        }

        if (z >= zb) {
            // phase one: stage p and b of plane z with an H-node halo
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                sp[HX + wave * RPT + i][H + lane] = pq[i][u % Q];
                sb[HX + wave * RPT + i][H + lane] = bq[i][u % Q];
            }
#pragma unroll
            for (int s = 0; s < HXN; ++s) {
                sp[hxrow[s]][H + lane] = W.hxp[s];
                sb[hxrow[s]][H + lane] = W.hxb[s];
            }
#pragma unroll
            for (int s = 0; s < YHN; ++s) {
                sp[hyrow[s]][hycol[s]] = W.hyp[s];
                sb[hyrow[s]][hycol[s]] = W.hyb[s];
            }
            __syncthreads();

            // phase two: every x and y face flux of the tile, once, by runs
#pragma unroll
            for (int s = 0; s < NIT; ++s) {
                const int e = threadIdx.x + s * NTH;
                if (NDIM == 3 && e < NRX * 64) {
                    // x run: faces t0 .. t0 + MX - 1 of column c (face t lies
                    // between rows x0 - R + t and x0 - R + t + 1; it reads LDS
                    // rows t .. t + 2R - 1)
                    const int c = e & 63, t0 = (e >> 6) * MX;
                    float vp[MX + 2 * R - 1], vb[MX + 2 * R - 1];
#pragma unroll
                    for (int j = 0; j < MX + 2 * R - 1; ++j) {
                        vp[j] = sp[t0 + j][H + c];
                        vb[j] = sb[t0 + j][H + c];
                    }
#pragma unroll
                    for (int f = 0; f < MX; ++f) {
                        float dp = 0.0f;
#pragma unroll
                        for (int l = 1; l <= R; ++l) dp = fmaf(P.sx[l], vp[f + R - 1 + l] - vp[f + R - l], dp);
                        const float bf = bface([&](int k) { return vb[f + R - 1 + k]; });
                        sfx[t0 + f][c] = bf * dp;
                    }
                } else if (e < NI) {
                    // y run: faces c0 .. c0 + MY - 1 of tile row r (face c lies
                    // between columns y0 - R + c and y0 - R + c + 1; it reads LDS
                    // columns c .. c + 2R - 1)
                    const int q = e - NRX * 64;
                    const int r = q / NRY, c0 = (q % NRY) * MY;
                    float vp[NVY], vb[NVY], out[MY];
                    static_assert(MY % 4 == 0, "y runs store float4s");
#pragma unroll
                    for (int j = 0; j < NVY / 4; ++j) {
                        const float4 a = *reinterpret_cast<const float4 *>(&sp[HX + r][c0 + 4 * j]);
                        const float4 bb = *reinterpret_cast<const float4 *>(&sb[HX + r][c0 + 4 * j]);
                        vp[4 * j] = a.x; vp[4 * j + 1] = a.y; vp[4 * j + 2] = a.z; vp[4 * j + 3] = a.w;
                        vb[4 * j] = bb.x; vb[4 * j + 1] = bb.y; vb[4 * j + 2] = bb.z; vb[4 * j + 3] = bb.w;
                    }
#pragma unroll
                    for (int f = 0; f < MY; ++f) {
                        float dp = 0.0f;
#pragma unroll
                        for (int l = 1; l <= R; ++l) dp = fmaf(P.sy[l], vp[f + R - 1 + l] - vp[f + R - l], dp);
                        const float bf = bface([&](int k) { return vb[f + R - 1 + k]; });
                        out[f] = bf * dp;
                    }
#pragma unroll
                    for (int j = 0; j < MY / 4; ++j)
                        *reinterpret_cast<float4 *>(&sfy[r][c0 + 4 * j]) =
                            make_float4(out[4 * j], out[4 * j + 1], out[4 * j + 2], out[4 * j + 3]);
                }
            }
            __syncthreads();

            // phase three: divergence and update
            const int so = soff(z);
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int rr = wave * RPT + i;
                float dzs = 0.0f, dxs = 0.0f, dys = 0.0f;
#pragma unroll
                for (int j = 1; j <= R; ++j) {
                    dzs = fmaf(P.sz[j], fq[i][(u + R + j - 1) % Q] - fq[i][(u + R - j) % Q], dzs);
                    if constexpr (NDIM == 3) dxs = fmaf(P.sx[j], sfx[rr + R + j - 1][lane] - sfx[rr + R - j][lane], dxs);
                    dys = fmaf(P.sy[j], sfy[rr][lane + R + j - 1] - sfy[rr][lane + R - j], dys);
                }
                const float lap = dzs + dxs + dys;
                const float c = pq[i][u % Q];
                float out = leapfrog(W.ab[i].x, W.ab[i].y, W.k[i], lap, c, W.p[i]);
                if (rdir[i] || axis_dirichlet(z, g.Z, P.bcm[0][0], P.bcm[0][1])) out = 0.0f;
                buf_st<NT>(out, rn, ro[i], so);
                if constexpr (MODE == MODE_STORE) {
                    buf_st<NT>(W.k[i] * lap, rs, ro[i], so);
                    buf_st<NT>(c, ru, ro[i], so);
                }
                if constexpr (MODE == MODE_IMAGE)
                    buf_st<NT>(fmaf(c, W.d[i] / (W.k[i] * W.k[i]), W.gr[i]), rg, ro[i], so);
                if constexpr (MODE == MODE_IMAGE2) {
                    const float k2 = W.k[i] * W.k[i];
                    buf_st<NT>(fmaf(c, W.d[i] / k2, fmaf(W.p[i], W.d2[i] / k2, W.gr[i])), rg, ro[i], so);
                }
            }
        }
    }
    }
}

template <int R, int NDIM, int TX, int NW, int NT>
__global__ void __launch_bounds__(64 * NW) k_cent(StencilParams P)
{
    static_assert(TX % NW == 0, "rows must split evenly over waves");
    constexpr int RPT = TX / NW;
    constexpr int HXR = (NDIM == 3) ? R : 0;
    constexpr int LY = 64 + 2 * R;
    constexpr int LX = TX + 2 * HXR;
    constexpr int NTH = 64 * NW;
    constexpr int HXN = (NDIM == 3) ? (2 * R + NW - 1) / NW : 0;
    constexpr int YHN = (TX * 2 * R + NTH - 1) / NTH;
    __shared__ float sp[2][LX][LY];
    __shared__ float sr[2][LX][LY];

    const Geom &g = P.g;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    int tx, ty, zc;
    tile_of(bid, P.ntx, P.nty, P.xfast, tx, ty, zc);
    const int y0 = ty * 64;
    const int y = y0 + lane;
    const int x0 = tx * TX;
    const int zb = zc * P.zc;
    const int ze = min(zb + P.zc, g.Z);
    const int64_t sz = int64_t(g.px) * g.py;
    const bool yin = y < g.Y;
    const int yc = model_axis(y, g.Y, P.bcm[2][0], P.bcm[2][1]);   // model reads: mirror images / nearest node
    const int ey = max(0, max(g.lo[2] - y, y - (g.lo[2] + g.np[2] - 1)));
    // plane base pointers + unsigned 32-bit lane offsets off(x, y) = xy0 + x py + y
    auto off = [&](int x, int yy) -> unsigned { return unsigned(g.xy0 + x * g.py + yy); };
    const float *cur = P.cur + g.base;
    const float *rm = P.aux + g.base;
    float *nxt = P.nxt + g.base;
    const float *km = P.K + g.base;

    // wavefield reads: grid nodes and mirror ghosts within the stored halo
    auto pread = [&](int x, int yy) -> bool {
        return axis_read(x, g.X, P.bcm[1][0], P.bcm[1][1], P.gh) &&
               axis_read(yy, g.Y, P.bcm[2][0], P.bcm[2][1], P.gh);
    };
    auto zread = [&](int z) -> bool { return axis_read(z, g.Z, P.bcm[0][0], P.bcm[0][1], P.gh); };
    unsigned roff[RPT], rroff[RPT], rpo[RPT];
    bool rin[RPT], rp[RPT], rdir[RPT];
    int ex2[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int x = x0 + wave * RPT + i;
        rin[i] = yin && x < g.X;
        roff[i] = rin[i] ? off(x, y) : 0u;
        rp[i] = pread(x, y);
        rpo[i] = rp[i] ? off(x, y) : 0u;
        rdir[i] = axis_dirichlet(x, g.X, P.bcm[1][0], P.bcm[1][1]) ||
                  axis_dirichlet(y, g.Y, P.bcm[2][0], P.bcm[2][1]);
        rroff[i] = off(model_axis(x, g.X, P.bcm[1][0], P.bcm[1][1]), yc);
        const int ex = max(0, max(g.lo[1] - x, x - (g.lo[1] + g.np[1] - 1)));
        ex2[i] = ex * ex + ey * ey;
    }
    unsigned hxo[HXN > 0 ? HXN : 1], hxro[HXN > 0 ? HXN : 1];
    bool hxin[HXN > 0 ? HXN : 1], hxok[HXN > 0 ? HXN : 1];
    int hxrow[HXN > 0 ? HXN : 1];
#pragma unroll
    for (int s = 0; s < HXN; ++s) {
        const int hr = wave + s * NW;
        hxok[s] = hr < 2 * R;
        const int x = (hr < R) ? x0 - R + hr : x0 + TX + hr - R;
        hxin[s] = hxok[s] && pread(x, y);
        hxrow[s] = (hr < R) ? hr : TX + hr;
        hxo[s] = hxin[s] ? off(x, y) : 0u;
        hxro[s] = off(model_axis(x, g.X, P.bcm[1][0], P.bcm[1][1]), yc);
    }
    unsigned hyo[YHN], hyro[YHN];
    bool hyin[YHN], hyok[YHN];
    int hyrow[YHN], hycol[YHN];
#pragma unroll
    for (int s = 0; s < YHN; ++s) {
        const int e = threadIdx.x + s * NTH;
        hyok[s] = e < TX * 2 * R;
        const int row = e / (2 * R), c = e % (2 * R);
        const int yy = (c < R) ? y0 - R + c : y0 + 64 + c - R;
        const int x = x0 + row;
        hyin[s] = hyok[s] && pread(x, yy);
        hyrow[s] = HXR + row;
        hycol[s] = (c < R) ? c : 64 + c;
        hyo[s] = hyin[s] ? off(x, yy) : 0u;
        hyro[s] = off(model_axis(x, g.X, P.bcm[1][0], P.bcm[1][1]),
                     model_axis(yy, g.Y, P.bcm[2][0], P.bcm[2][1]));
    }

    float q[RPT][2 * R + 1], qr[RPT][2 * R + 1];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) {
            const int z = zb - R + k;
            q[i][k] = (rp[i] && zread(z)) ? (cur + int64_t(z) * sz)[rpo[i]] : 0.0f;
            qr[i][k] = (rm + int64_t(model_axis(z, g.Z, P.bcm[0][0], P.bcm[0][1])) * sz)[rroff[i]];
        }

    float nf[RPT], nfr[RPT], np_[RPT], nk[RPT], na[RPT], nb[RPT];
    float nhx[HXN > 0 ? HXN : 1], nhxr[HXN > 0 ? HXN : 1], nhy[YHN], nhyr[YHN];
    auto load = [&](int z) {
        const int zf = z + R;
        const int ez = max(0, max(g.lo[0] - z, z - (g.lo[0] + g.np[0] - 1)));
        const int64_t zo = int64_t(z) * sz;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            nf[i] = (rp[i] && zread(zf)) ? cur[rpo[i] + int64_t(zf) * sz] : 0.0f;
            nfr[i] = rm[rroff[i] + int64_t(model_axis(zf, g.Z, P.bcm[0][0], P.bcm[0][1])) * sz];
            np_[i] = rin[i] ? ld_stream<NT>(nxt + zo + roff[i]) : 0.0f;
            nk[i] = rin[i] ? ld_stream<NT>(km + zo + roff[i]) : 0.0f;
            const int d2 = ez * ez + ex2[i];
            na[i] = 1.0f;
            nb[i] = 1.0f;
            if (rin[i] && d2 > 0) {
                const float2 ab = P.damp[d2];
                na[i] = ab.x;
                nb[i] = ab.y;
            }
        }
#pragma unroll
        for (int s = 0; s < HXN; ++s) {
            nhx[s] = hxin[s] ? (cur + zo)[hxo[s]] : 0.0f;
            nhxr[s] = hxok[s] ? (rm + zo)[hxro[s]] : 0.0f;
        }
#pragma unroll
        for (int s = 0; s < YHN; ++s) {
            nhy[s] = hyin[s] ? (cur + zo)[hyo[s]] : 0.0f;
            nhyr[s] = hyok[s] ? (rm + zo)[hyro[s]] : 0.0f;
        }
    };

    load(zb);
    int buf = 0;
    for (int z = zb; z < ze; ++z) {
        float pp[RPT], pk[RPT], pa[RPT], pb[RPT];
        float hx[HXN > 0 ? HXN : 1], hxr[HXN > 0 ? HXN : 1], hy[YHN], hyr[YHN];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            q[i][2 * R] = nf[i];
            qr[i][2 * R] = nfr[i];
            pp[i] = np_[i];
            pk[i] = nk[i];
            pa[i] = na[i];
            pb[i] = nb[i];
        }
#pragma unroll
        for (int s = 0; s < HXN; ++s) {
            hx[s] = nhx[s];
            hxr[s] = nhxr[s];
        }
#pragma unroll
        for (int s = 0; s < YHN; ++s) {
            hy[s] = nhy[s];
            hyr[s] = nhyr[s];
        }
        if (z + 1 < ze) load(z + 1);

        float(*T)[LY] = sp[buf];
        float(*U)[LY] = sr[buf];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            T[HXR + wave * RPT + i][R + lane] = q[i][R];
            U[HXR + wave * RPT + i][R + lane] = qr[i][R];
        }
#pragma unroll
        for (int s = 0; s < HXN; ++s)
            if (hxok[s]) {
                T[hxrow[s]][R + lane] = hx[s];
                U[hxrow[s]][R + lane] = hxr[s];
            }
#pragma unroll
        for (int s = 0; s < YHN; ++s)
            if (hyok[s]) {
                T[hyrow[s]][hycol[s]] = hy[s];
                U[hyrow[s]][hycol[s]] = hyr[s];
            }
        __syncthreads();

#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int lx = HXR + wave * RPT + i, ly = R + lane;
            const float c = q[i][R];
            float lap = P.c0 * c;
            float dpz = 0.0f, drz = 0.0f, dpx = 0.0f, drx = 0.0f, dpy = 0.0f, dry = 0.0f;
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                lap = fmaf(P.cz[j], q[i][R + j] + q[i][R - j], lap);
                dpz = fmaf(P.sz[j], q[i][R + j] - q[i][R - j], dpz);
                drz = fmaf(P.sz[j], qr[i][R + j] - qr[i][R - j], drz);
            }
            if constexpr (NDIM == 3) {
#pragma unroll
                for (int j = 1; j <= R; ++j) {
                    lap = fmaf(P.cx[j], T[lx + j][ly] + T[lx - j][ly], lap);
                    dpx = fmaf(P.sx[j], T[lx + j][ly] - T[lx - j][ly], dpx);
                    drx = fmaf(P.sx[j], U[lx + j][ly] - U[lx - j][ly], drx);
                }
            }
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                lap = fmaf(P.cy[j], T[lx][ly + j] + T[lx][ly - j], lap);
                dpy = fmaf(P.sy[j], T[lx][ly + j] - T[lx][ly - j], dpy);
                dry = fmaf(P.sy[j], U[lx][ly + j] - U[lx][ly - j], dry);
            }
            const float grad = fmaf(drz, dpz, fmaf(drx, dpx, dry * dpy));
            const float Lp = lap - grad / qr[i][R];
            float out = pa[i] * fmaf(pk[i], Lp, 2.0f * c) - pb[i] * pp[i];
            if (rdir[i] || axis_dirichlet(z, g.Z, P.bcm[0][0], P.bcm[0][1])) out = 0.0f;
            if (rin[i]) st_stream<NT>(out, nxt + int64_t(z) * sz + roff[i]);
        }
        buf ^= 1;
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) {
                q[i][k] = q[i][k + 1];
                qr[i][k] = qr[i][k + 1];
            }
    }
}

// Tile shapes (rows, waves) of the variable-density kernels in 3D; 2D uses (1, 1).
#define SW_VD_SHAPES(X) X(16, 8) X(8, 8) X(8, 4) X(16, 4) X(16, 16)

template <int R, int NDIM, int TX, int NW, int NT, int MODE>
void launch_stag_mode(int occ, StencilParams &P, hipStream_t s)
{
    constexpr auto kern = k_stag<R, NDIM, TX, NW, NT, MODE>;
    hipLaunchKernelGGL(kern, dim3(P.ntx * P.nty * P.nzc), dim3(64 * NW),
                       occ ? occ_pad_bytes(occ, static_lds_of<kern>()) : 0u, s, P);
}

template <int R, int NDIM, int TX, int NW, int NT>
hipError_t launch_vd_shape(int scheme, int mode, int occ, StencilParams &P, hipStream_t s)
{
    const dim3 grid(P.ntx * P.nty * P.nzc), block(64 * NW);
    if (scheme == 1) {
        if (mode == MODE_STORE) launch_stag_mode<R, NDIM, TX, NW, NT, MODE_STORE>(occ, P, s);
        else if (mode == MODE_IMAGE) launch_stag_mode<R, NDIM, TX, NW, NT, MODE_IMAGE>(occ, P, s);
        else if (mode == MODE_IMAGE2) launch_stag_mode<R, NDIM, TX, NW, NT, MODE_IMAGE2>(occ, P, s);
        else launch_stag_mode<R, NDIM, TX, NW, NT, MODE_FWD>(occ, P, s);
    } else {
        constexpr auto kern = k_cent<R, NDIM, TX, NW, NT>;
        hipLaunchKernelGGL(kern, grid, block, occ ? occ_pad_bytes(occ, static_lds_of<kern>()) : 0u, s, P);
    }
    return hipGetLastError();
}

template <int R, int NT>
hipError_t launch_vd_nt(int scheme, int mode, int ndim, const Tiling &t, StencilParams &P, hipStream_t s)
{
    if (ndim == 2) return launch_vd_shape<R, 2, 1, 1, NT>(scheme, mode, t.occ, P, s);
#define SW_X(TXV, NWV) \
    if (t.tx == TXV && t.nw == NWV) return launch_vd_shape<R, 3, TXV, NWV, NT>(scheme, mode, t.occ, P, s);
    SW_VD_SHAPES(SW_X)
#undef SW_X
    return hipErrorInvalidValue;
}

// Resident blocks per CU of the 3D forward kernel of a scheme (1 staggered,
// else centred) and tiling, from the runtime's occupancy calculator; 0 if
// unknown.
template <auto KERN>
int resident_of(int nw, int occ)
{
    const unsigned pad = occ ? occ_pad_bytes(occ, static_lds_of<KERN>()) : 0u;
    int n = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, KERN, 64 * nw, pad) == hipSuccess ? n : 0;
}

template <int R, int NT>
int vd_resident_nt(int scheme, const Tiling &t)
{
#define SW_X(TXV, NWV)                                                                     \
    if (t.tx == TXV && t.nw == NWV)                                                        \
        return scheme == 1 ? resident_of<k_stag<R, 3, TXV, NWV, NT, MODE_FWD>>(NWV, t.occ) \
                           : resident_of<k_cent<R, 3, TXV, NWV, NT>>(NWV, t.occ);
    SW_VD_SHAPES(SW_X)
#undef SW_X
    return 0;
}

template <int R>
int vd_resident_radius(int scheme, const Tiling &t)
{
    return t.nt ? vd_resident_nt<R, 1>(scheme, t) : vd_resident_nt<R, 0>(scheme, t);
}

template <int R>
hipError_t launch_vd_radius(int scheme, int mode, int ndim, const Tiling &t, StencilParams &P, hipStream_t s)
{
    return t.nt ? launch_vd_nt<R, 1>(scheme, mode, ndim, t, P, s) : launch_vd_nt<R, 0>(scheme, mode, ndim, t, P, s);
}

}  // namespace sw
