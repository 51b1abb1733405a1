// Two leapfrog steps per sweep of the constant-density update (3D).
//
// One launch reads p^n, p^{n-1} and K once and writes p^{n+1} and p^{n+2}:
// 20 bytes of HBM traffic per node for two steps instead of 32.  A block owns
// a TX x (64 - 2R) output tile of the (x, y) plane and one z chunk.  Its 64
// lanes cover the output columns plus R ghost columns on each side, and its
// rows are the TX output rows plus R ghost rows on each side; on these
// (TX + 2R) x 64 nodes it evaluates the first step, so that the second step
// finds every in-plane neighbour of p^{n+1} in the block.  Along z the block
// marches two fronts R planes apart: step one at plane z1, step two at
// z2 = z1 - R, each with a register queue of its input level (p^n for step
// one, p^{n+1} for step two, which step one pushes into).  One LDS buffer pair
// per plane (double buffered, one barrier per plane) holds p^n at z1 with a 2R
// halo and p^{n+1} at z2.  The first step is evaluated R planes beyond both
// ends of the chunk.  Ghost work repeats exactly the arithmetic of the
// neighbouring tile, so the result is bitwise that of two single sweeps.
//
// The source of each step is added in the sweep (to ghost nodes as well):
// the value of every injection node for step n and n+1 is formed beforehand
// by the same arithmetic as the stand-alone injection, and a node of the
// injection box looks itself up in that list.
#pragma once

#include "device.h"
#include "stencil_const.h"

namespace sw {

template <int R, int TX, int NW, int NT>
__global__ void __launch_bounds__(64 * NW) k_const2(StencilParams P, TwoStepParams T)
{
    static_assert(TX % NW == 0, "rows must split evenly over waves");
    constexpr int RPT = TX / NW;                  // output rows per thread
    constexpr int NG = 2 * R;                     // ghost rows of step one
    constexpr int GPT = (NG + NW - 1) / NW;       // ghost (and halo) rows per wave
    constexpr int YO = 64 - 2 * R;                // output columns per tile
    constexpr int AX = TX + 4 * R, AY = 64 + 2 * R;
    constexpr int BX = TX + 2 * R;
    constexpr int NTH = 64 * NW;
    constexpr int YHN = (BX * 2 * R + NTH - 1) / NTH;   // y-halo items of tile A per thread
    constexpr int Q = 2 * R + 2;                  // queue length: even, a multiple of R + 1
    constexpr int G = R + 1;                      // short queues (K, ghost p^{n+1})
    constexpr int kOut = 0x7ffffe00;              // byte offset past every window: reads 0, stores dropped
    __shared__ float sa[2][AX + 1][AY];           // p^n, rows x0-2R.., columns y(lane 0)-R..; last row: sink
    __shared__ float sb[2][BX + 1][64];           // p^{n+1}, rows x0-R.., columns of the lanes; last row: sink

    const Geom &g = P.g;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int ty = bid % P.nty;
    const int rest = bid / P.nty;
    const int tx = rest % P.ntx;
    const int zc = rest / P.ntx;
    const int yl0 = ty * YO - R;                  // column of lane 0
    const int y = yl0 + lane;
    const int x0 = tx * TX;
    const int zb = zc * P.zc;
    const int ze = min(zb + P.zc, g.Z);
    const int64_t sz = int64_t(g.px) * g.py;
    const bool yin = y >= 0 && y < g.Y;
    const bool ycol = lane >= R && lane < 64 - R && yin;     // an output column
    const int ey = max(0, max(g.lo[2] - y, y - (g.lo[2] + g.np[2] - 1)));
    const int ly2 = min(max(lane, R), 63 - R);    // step-two column (clamped on ghost lanes)
    // z window: planes zw .. zt - 1
    const int zw = max(zb - 2 * R, 0);
    const int zt = min(ze + 2 * R, g.Z);
    const int pb = int(sz) * 4;
    const uint32_t wbytes = uint32_t(zt - zw) * uint32_t(pb);
    const int64_t w0 = g.base + int64_t(zw) * sz;
    const auto rc = buf_res(P.cur + w0, wbytes);
    const auto rp = buf_res(P.nxt + w0, wbytes);
    const auto rk = buf_res(P.K + w0, wbytes);
    const auto r1 = buf_res(T.out1 + w0, wbytes);
    const auto r2 = buf_res(T.out2 + w0, wbytes);
    const auto rd = buf_res(P.damp, uint32_t(P.ndamp) * 8u);
    auto soff = [&](int z) -> int { return min(max(z, zw), zt - 1) - zw; };   // in planes
    auto keep = [](float v, unsigned m) -> float {
        return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, v) & m);
    };
    auto off = [&](int x, int yy) -> int { return (g.xy0 + x * g.py + yy) * 4; };

    // output rows
    int ro[RPT], rs[RPT], rx[RPT], ex2[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int x = x0 + wave * RPT + i;
        const bool in = yin && x < g.X;
        rx[i] = x;
        ro[i] = in ? off(x, y) : kOut;
        rs[i] = (in && ycol) ? ro[i] : kOut;       // stores: owned nodes only
        const int ex = max(0, max(g.lo[1] - x, x - (g.lo[1] + g.np[1] - 1)));
        ex2[i] = in ? ex * ex + ey * ey : 0;
    }
    // ghost rows (step one only) and the tile-A halo rows beyond them
    int go[GPT], ho[GPT], gx[GPT], gex2[GPT], gra[GPT], grb[GPT], hra[GPT];
#pragma unroll
    for (int s = 0; s < GPT; ++s) {
        const int e = wave + s * NW;
        const bool ok = e < NG;
        const int x = (e < R) ? x0 - R + e : x0 + TX + e - R;
        const bool in = ok && yin && x >= 0 && x < g.X;
        gx[s] = x;
        go[s] = in ? off(x, y) : kOut;
        gra[s] = !ok ? AX : (e < R) ? R + e : TX + R + e;
        grb[s] = !ok ? BX : (e < R) ? e : TX + e;
        const int ex = max(0, max(g.lo[1] - x, x - (g.lo[1] + g.np[1] - 1)));
        gex2[s] = in ? ex * ex + ey * ey : 0;
        const int xh = (e < R) ? x0 - 2 * R + e : x0 + TX + e;
        ho[s] = (ok && yin && xh >= 0 && xh < g.X) ? off(xh, y) : kOut;
        hra[s] = !ok ? AX : (e < R) ? e : TX + 2 * R + e;
    }
    // y halo of tile A: the (TX + 2R) step-one rows x R columns on each side
    int yo[YHN], yra[YHN], yca[YHN];
#pragma unroll
    for (int s = 0; s < YHN; ++s) {
        const int e = threadIdx.x + s * NTH;
        const bool ok = e < BX * 2 * R;
        const int row = e / (2 * R), c = e % (2 * R);
        const int yy = (c < R) ? yl0 - R + c : yl0 + 64 + c - R;
        const int x = x0 - R + row;
        yo[s] = (ok && x >= 0 && x < g.X && yy >= 0 && yy < g.Y) ? off(x, yy) : kOut;
        yra[s] = ok ? R + row : AX;
        yca[s] = (c < R) ? c : 64 + c;
    }
    // injection: only blocks whose node box meets the injection box look nodes up
    const bool inj_blk = T.nuniq > 0 && zb - R <= T.box[1] && ze + R - 1 >= T.box[0] && x0 - R <= T.box[3] &&
                         x0 + TX + R - 1 >= T.box[2] && yl0 <= T.box[5] && yl0 + 63 >= T.box[4];
    // (called only for planes z inside the box)
    auto inject = [&](int which, int z, int x, float v) -> float {
        if (x < T.box[2] || x > T.box[3] || y < T.box[4] || y > T.box[5]) return v;
        const int64_t node = g.origin + (int64_t(z) * g.px + x) * g.py + y;
        for (int u = 0; u < T.nuniq; ++u)
            if (T.unode[u] == node) v = v + T.inj[which * T.nuniq + u];
        return v;
    };

    // queues (index rotates with the unrolled step u):
    //   qa[i][(u + k) % Q] = p^n at z1 - R + k,        k = 0 .. 2R
    //   qb[i][(u + k) % Q] = p^{n+1} at z2 - R + k,    k = 0 .. 2R   (z2 = z1 - R)
    //   kq[i][(u + k) % G] = K at z2 + k,               k = 0 .. R
    //   qg[s][(u + k) % Q] = p^n of ghost rows at z1 - R + k
    //   gb[s][(u + k) % G] = p^{n+1} of ghost rows at z2 + k
    float qa[RPT][Q], qb[RPT][Q], kq[RPT][G], qg[GPT][Q], gb[GPT][G];
    const int zs = zb - R;                        // first plane of step one
    const int zl = ze + R;                        // one past its last plane
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
        const int z = zs - R + k;
        const unsigned m = (z >= 0 && z < g.Z) ? ~0u : 0u;
        const int so = soff(z) * pb;
#pragma unroll
        for (int i = 0; i < RPT; ++i) qa[i][k] = keep(buf_ld<0>(rc, ro[i], so), m);
#pragma unroll
        for (int s = 0; s < GPT; ++s) qg[s][k] = keep(buf_ld<0>(rc, go[s], so), m);
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
#pragma unroll
        for (int k = 0; k < Q; ++k) qb[i][k] = 0.0f;
#pragma unroll
        for (int k = 0; k < G; ++k) kq[i][k] = 0.0f;
    }
#pragma unroll
    for (int s = 0; s < GPT; ++s)
#pragma unroll
        for (int k = 0; k < G; ++k) gb[s][k] = 0.0f;

    // loads of step-one plane z: p^n at z + R, p^{n-1} and K at z (zero off the
    // grid), tile-A halos at z; (A, B) of step one at z and of step two at z - R
    struct Slot {
        float f[RPT], p[RPT], k[RPT];
        float2 a1[RPT], a2[RPT];
        float fg[GPT], pg[GPT], kg[GPT], h[GPT];
        float2 ag[GPT];
        float hy[YHN];
    };
    Slot S[2];
    auto load = [&](int z, Slot &L) {
        const int zf = z + R, z2 = z - R;
        const unsigned mf = zf < g.Z ? ~0u : 0u;
        const unsigned mz = (z >= 0 && z < g.Z) ? ~0u : 0u;
        const int so = soff(z) * pb, sf = soff(zf) * pb;
        // layer distance along z of the nearest grid plane (off the grid the
        // update yields zero whatever (A, B) are, since p^n, p^{n-1} and K read zero)
        const int zc1 = min(max(z, 0), g.Z - 1), zc2 = min(max(z2, 0), g.Z - 1);
        const int ez = max(0, max(g.lo[0] - zc1, zc1 - (g.lo[0] + g.np[0] - 1)));
        const int ez2 = max(0, max(g.lo[0] - zc2, zc2 - (g.lo[0] + g.np[0] - 1)));
        const int dz = ez * ez, dz2 = ez2 * ez2;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            L.f[i] = keep(buf_ld<0>(rc, ro[i], sf), mf);
            L.p[i] = keep(buf_ld<NT>(rp, ro[i], so), mz);
            L.k[i] = keep(buf_ld<0>(rk, ro[i], so), mz);
            L.a1[i] = buf_ld2(rd, (dz + ex2[i]) * 8);
            L.a2[i] = buf_ld2(rd, (dz2 + ex2[i]) * 8);
        }
#pragma unroll
        for (int s = 0; s < GPT; ++s) {
            L.fg[s] = keep(buf_ld<0>(rc, go[s], sf), mf);
            L.pg[s] = keep(buf_ld<0>(rp, go[s], so), mz);
            L.kg[s] = keep(buf_ld<0>(rk, go[s], so), mz);
            L.ag[s] = buf_ld2(rd, (dz + gex2[s]) * 8);
            L.h[s] = keep(buf_ld<0>(rc, ho[s], so), mz);
        }
#pragma unroll
        for (int s = 0; s < YHN; ++s) L.hy[s] = keep(buf_ld<0>(rc, yo[s], so), mz);
    };

    load(zs, S[0]);
    for (int zz = zs; zz < zl; zz += Q) {
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            const int z1 = zz + u;
            if (z1 < zl) {
                Slot &W = S[u % 2];
                if (z1 + 1 < zl) load(z1 + 1, S[(u + 1) % 2]);
                const int z2 = z1 - R;
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    qa[i][(u + 2 * R) % Q] = W.f[i];
                    kq[i][(u + R) % G] = W.k[i];
                }
#pragma unroll
                for (int s = 0; s < GPT; ++s) qg[s][(u + 2 * R) % Q] = W.fg[s];

                float(*A)[AY] = sa[u % 2];
                float(*B)[64] = sb[u % 2];
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    A[2 * R + wave * RPT + i][R + lane] = qa[i][(u + R) % Q];
                    B[R + wave * RPT + i][lane] = qb[i][(u + R) % Q];
                }
#pragma unroll
                for (int s = 0; s < GPT; ++s) {
                    A[gra[s]][R + lane] = qg[s][(u + R) % Q];
                    A[hra[s]][R + lane] = W.h[s];
                    B[grb[s]][lane] = gb[s][u % G];
                }
#pragma unroll
                for (int s = 0; s < YHN; ++s) A[yra[s]][yca[s]] = W.hy[s];
                __syncthreads();

                // step one at plane z1 (zero off the grid: p^n, p^{n-1} and K read zero there)
                const int so1 = soff(z1) * pb;
                const bool inj1 = inj_blk && z1 >= T.box[0] && z1 <= T.box[1];
                const bool inj2 = inj_blk && z2 >= T.box[0] && z2 <= T.box[1];
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int ra = 2 * R + wave * RPT + i, ca = R + lane;
                    const float c = qa[i][(u + R) % Q];
                    float lap = P.c0 * c;
#pragma unroll
                    for (int j = 1; j <= R; ++j)
                        lap = fmaf(P.cz[j], qa[i][(u + R + j) % Q] + qa[i][(u + R - j) % Q], lap);
#pragma unroll
                    for (int j = 1; j <= R; ++j) lap = fmaf(P.cx[j], A[ra + j][ca] + A[ra - j][ca], lap);
#pragma unroll
                    for (int j = 1; j <= R; ++j) lap = fmaf(P.cy[j], A[ra][ca + j] + A[ra][ca - j], lap);
                    float out = leapfrog(W.a1[i].x, W.a1[i].y, W.k[i], lap, c, W.p[i]);
                    if (inj1) out = inject(0, z1, rx[i], out);
                    qb[i][(u + 2 * R) % Q] = out;
                    if (z1 >= zb && z1 < ze) buf_st<NT>(out, r1, rs[i], so1);
                }
#pragma unroll
                for (int s = 0; s < GPT; ++s) {
                    const int ra = gra[s], ca = R + lane;
                    const float c = qg[s][(u + R) % Q];
                    float lap = P.c0 * c;
#pragma unroll
                    for (int j = 1; j <= R; ++j)
                        lap = fmaf(P.cz[j], qg[s][(u + R + j) % Q] + qg[s][(u + R - j) % Q], lap);
#pragma unroll
                    for (int j = 1; j <= R; ++j) lap = fmaf(P.cx[j], A[ra + j][ca] + A[ra - j][ca], lap);
#pragma unroll
                    for (int j = 1; j <= R; ++j) lap = fmaf(P.cy[j], A[ra][ca + j] + A[ra][ca - j], lap);
                    float out = leapfrog(W.ag[s].x, W.ag[s].y, W.kg[s], lap, c, W.pg[s]);
                    if (inj1 && go[s] != kOut) out = inject(0, z1, gx[s], out);
                    gb[s][(u + R) % G] = out;
                }

                // step two at plane z2 (output rows)
                if (z2 >= zb) {
                    const int so2 = soff(z2) * pb;
#pragma unroll
                    for (int i = 0; i < RPT; ++i) {
                        const int rb = R + wave * RPT + i;
                        const float c = qb[i][(u + R) % Q];
                        float lap = P.c0 * c;
#pragma unroll
                        for (int j = 1; j <= R; ++j)
                            lap = fmaf(P.cz[j], qb[i][(u + R + j) % Q] + qb[i][(u + R - j) % Q], lap);
#pragma unroll
                        for (int j = 1; j <= R; ++j) lap = fmaf(P.cx[j], B[rb + j][ly2] + B[rb - j][ly2], lap);
#pragma unroll
                        for (int j = 1; j <= R; ++j) lap = fmaf(P.cy[j], B[rb][ly2 + j] + B[rb][ly2 - j], lap);
                        float out = leapfrog(W.a2[i].x, W.a2[i].y, kq[i][u % G], lap, c, qa[i][u % Q]);
                        if (inj2) out = inject(1, z2, rx[i], out);
                        buf_st<NT>(out, r2, rs[i], so2);
                    }
                }
            }
        }
    }
}

// Shapes (rows, waves) of the two-step sweep whose register queues fit:
// RPT (2Q + G) + GPT (Q + G) <= 95 values per thread, Q = 2R + 2, G = R + 1.
template <int R, int TX, int NW>
constexpr bool tb_fits()
{
    return (TX / NW) * (5 * R + 5) + ((2 * R + NW - 1) / NW) * (3 * R + 3) <= 95;
}

#define SW_TB_SHAPES(X) X(8, 4) X(16, 8) X(8, 8) X(16, 4)

template <int R, int TX, int NW, int NT>
hipError_t launch_tb_shape(StencilParams &P, const TwoStepParams &T, hipStream_t s)
{
    if constexpr (tb_fits<R, TX, NW>()) {
        const dim3 grid(P.ntx * P.nty * P.nzc), block(64 * NW);
        hipLaunchKernelGGL((k_const2<R, TX, NW, NT>), grid, block, 0, s, P, T);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <int R>
hipError_t launch_tb_radius(const Tiling &t, StencilParams &P, const TwoStepParams &T, hipStream_t s)
{
#define SW_X(TXV, NWV)                                                                      \
    if (t.tx == TXV && t.nw == NWV)                                                         \
        return t.nt ? launch_tb_shape<R, TXV, NWV, 1>(P, T, s) : launch_tb_shape<R, TXV, NWV, 0>(P, T, s);
    SW_TB_SHAPES(SW_X)
#undef SW_X
    return hipErrorInvalidValue;
}

}  // namespace sw
