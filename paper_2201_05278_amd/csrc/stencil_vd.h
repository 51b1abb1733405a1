// Variable-density leapfrog stencils, damping fused as in the constant-density
// kernel (A, B from the squared layer distance).
//
// Staggered (conservative) operator, K = dt^2 rho c^2, b = 1/rho:
//   L p = sum_i D-_i (b_{i+1/2} D+_i p)
//   (D+ q)_{k+1/2} = sum_j s_j (q_{k+j} - q_{k-j+1}) / h
//   (D- F)_k       = sum_j s_j (F_{k+j-1/2} - F_{k-j+1/2}) / h
//   b_{k+1/2}      = sum_j m_j (b_{k+j} + b_{k-j+1})
// Fluxes along z are produced once per face as the march reaches it and kept
// in a register queue (with register queues of p and b in front of the
// node); fluxes along x are computed by each wave for its own rows from a
// column of the LDS plane tile; fluxes along y are computed once per face into
// LDS and differenced from there.  p and b planes are staged with a 2R halo.
//
// Centred operator (paper, "Time discretization": expanded variable-density
// equation), K = dt^2 c^2:
//   L p = sum_i [ D2_i p - (D1_i rho / rho) D1_i p ]
// with the centred second and first derivatives; rho is staged like p (halo R)
// with its own register queue along z.
//
// Model values outside the extended grid are read from the nearest grid node
// (coordinates clamped), wavefield values outside it are zero.
#pragma once

#include "device.h"
#include "stencil_const.h"

namespace sw {

__device__ inline int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

template <int R, int NDIM, int TX, int NW, int NT>
__global__ void __launch_bounds__(64 * NW) k_stag(StencilParams P)
{
    static_assert(TX % NW == 0, "rows must split evenly over waves");
    constexpr int RPT = TX / NW;
    constexpr int H2 = 2 * R;
    constexpr int HX = (NDIM == 3) ? H2 : 0;
    constexpr int LY = 64 + 2 * H2;
    constexpr int LX = TX + 2 * HX;
    constexpr int FY = 64 + 2 * R;
    constexpr int NTH = 64 * NW;
    constexpr int NCOL = RPT + 4 * R - 2;
    constexpr int NFX = RPT + 2 * R - 1;
    constexpr int HXN = (NDIM == 3) ? (2 * HX + NW - 1) / NW : 0;
    constexpr int YHN = (TX * 2 * H2 + NTH - 1) / NTH;
    __shared__ float sp[LX][LY];
    __shared__ float sb[LX][LY];
    __shared__ float sfy[TX][FY];

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
    const int yc = clampi(y, 0, g.Y - 1);
    const int ey = max(0, max(g.lo[2] - y, y - (g.lo[2] + g.np[2] - 1)));
    // plane base pointers + unsigned 32-bit lane offsets off(x, y) = xy0 + x py + y
    auto off = [&](int x, int yy) -> unsigned { return unsigned(g.xy0 + x * g.py + yy); };
    const float *cur = P.cur + g.base;
    const float *bm = P.aux + g.base;
    float *nxt = P.nxt + g.base;
    const float *km = P.K + g.base;

    unsigned roff[RPT], rboff[RPT];
    bool rin[RPT];
    int ex2[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int x = x0 + wave * RPT + i;
        rin[i] = yin && x < g.X;
        roff[i] = rin[i] ? off(x, y) : 0u;
        rboff[i] = off(clampi(x, 0, g.X - 1), yc);
        const int ex = max(0, max(g.lo[1] - x, x - (g.lo[1] + g.np[1] - 1)));
        ex2[i] = ex * ex + ey * ey;
    }
    // x-halo rows (3D): 2R rows on each side, one lane per column
    unsigned hxo[HXN > 0 ? HXN : 1], hxbo[HXN > 0 ? HXN : 1];
    bool hxin[HXN > 0 ? HXN : 1], hxok[HXN > 0 ? HXN : 1];
    int hxrow[HXN > 0 ? HXN : 1];
#pragma unroll
    for (int s = 0; s < HXN; ++s) {
        const int hr = wave + s * NW;
        hxok[s] = hr < 2 * HX;
        const int x = (hr < HX) ? x0 - HX + hr : x0 + TX + hr - HX;
        hxin[s] = hxok[s] && yin && x >= 0 && x < g.X;
        hxrow[s] = (hr < HX) ? hr : TX + hr;
        hxo[s] = hxin[s] ? off(x, y) : 0u;
        hxbo[s] = off(clampi(x, 0, g.X - 1), yc);
    }
    // y-halo columns: 2R on each side of every tile row
    unsigned hyo[YHN], hybo[YHN];
    bool hyin[YHN], hyok[YHN];
    int hyrow[YHN], hycol[YHN];
#pragma unroll
    for (int s = 0; s < YHN; ++s) {
        const int e = threadIdx.x + s * NTH;
        hyok[s] = e < TX * 2 * H2;
        const int row = e / (2 * H2), c = e % (2 * H2);
        const int yy = (c < H2) ? y0 - H2 + c : y0 + 64 + c - H2;
        const int x = x0 + row;
        hyin[s] = hyok[s] && x < g.X && yy >= 0 && yy < g.Y;
        hyrow[s] = HX + row;
        hycol[s] = (c < H2) ? c : 64 + c;
        hyo[s] = hyin[s] ? off(x, yy) : 0u;
        hybo[s] = off(clampi(x, 0, g.X - 1), clampi(yy, 0, g.Y - 1));
    }

    auto pz_ = [&](int i, int z) -> float {
        return (rin[i] && z >= 0 && z < g.Z) ? (cur + int64_t(z) * sz)[roff[i]] : 0.0f;
    };
    auto bz_ = [&](int i, int z) -> float {
        return (bm + int64_t(clampi(z, 0, g.Z - 1)) * sz)[rboff[i]];
    };

    // queues: pq[k] = p(z + k), bq[k] = b(z + k), fq[k] = z-flux at face (z - R + k) + 1/2
    float pq[RPT][2 * R], bq[RPT][2 * R], fq[RPT][2 * R];
    const int zs = zb - 2 * R + 1;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
#pragma unroll
        for (int k = 0; k < 2 * R - 1; ++k) {
            pq[i][k] = pz_(i, zs + k);
            bq[i][k] = bz_(i, zs + k);
        }
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) fq[i][k] = 0.0f;
    }

    float fp[RPT], fb[RPT], np_[RPT], nk[RPT], na[RPT], nb[RPT];
    float nhxp[HXN > 0 ? HXN : 1], nhxb[HXN > 0 ? HXN : 1], nhyp[YHN], nhyb[YHN];
    auto load = [&](int z) {
        const int zf = z + 2 * R - 1;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            fp[i] = pz_(i, zf);
            fb[i] = bz_(i, zf);
        }
        if (z < zb) return;
        const int ez = max(0, max(g.lo[0] - z, z - (g.lo[0] + g.np[0] - 1)));
        const int64_t zo = int64_t(z) * sz;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
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
            nhxp[s] = hxin[s] ? (cur + zo)[hxo[s]] : 0.0f;
            nhxb[s] = hxok[s] ? (bm + zo)[hxbo[s]] : 0.0f;
        }
#pragma unroll
        for (int s = 0; s < YHN; ++s) {
            nhyp[s] = hyin[s] ? (cur + zo)[hyo[s]] : 0.0f;
            nhyb[s] = hyok[s] ? (bm + zo)[hybo[s]] : 0.0f;
        }
    };

    load(zs);
    for (int z = zs; z < ze; ++z) {
        const bool out_plane = z >= zb;
        float pp[RPT], pk[RPT], pa[RPT], pb[RPT];
        float hxp[HXN > 0 ? HXN : 1], hxb[HXN > 0 ? HXN : 1], hyp[YHN], hyb[YHN];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            pq[i][2 * R - 1] = fp[i];
            bq[i][2 * R - 1] = fb[i];
            pp[i] = np_[i];
            pk[i] = nk[i];
            pa[i] = na[i];
            pb[i] = nb[i];
        }
#pragma unroll
        for (int s = 0; s < HXN; ++s) {
            hxp[s] = nhxp[s];
            hxb[s] = nhxb[s];
        }
#pragma unroll
        for (int s = 0; s < YHN; ++s) {
            hyp[s] = nhyp[s];
            hyb[s] = nhyb[s];
        }
        if (z + 1 < ze) load(z + 1);

        // new z-flux at face (z + R - 1) + 1/2
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            float bf = 0.0f, dp = 0.0f;
#pragma unroll
            for (int l = 1; l <= R; ++l) {
                bf = fmaf(P.mj[l], bq[i][R - 1 + l] + bq[i][R - l], bf);
                dp = fmaf(P.sz[l], pq[i][R - 1 + l] - pq[i][R - l], dp);
            }
            fq[i][2 * R - 1] = bf * dp;
        }

        if (out_plane) {
            // phase 1: stage p and b of plane z
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                sp[HX + wave * RPT + i][H2 + lane] = pq[i][0];
                sb[HX + wave * RPT + i][H2 + lane] = bq[i][0];
            }
#pragma unroll
            for (int s = 0; s < HXN; ++s)
                if (hxok[s]) {
                    sp[hxrow[s]][H2 + lane] = hxp[s];
                    sb[hxrow[s]][H2 + lane] = hxb[s];
                }
#pragma unroll
            for (int s = 0; s < YHN; ++s)
                if (hyok[s]) {
                    sp[hyrow[s]][hycol[s]] = hyp[s];
                    sb[hyrow[s]][hycol[s]] = hyb[s];
                }
            __syncthreads();

            // phase 2: y-fluxes into LDS; x-fluxes and their differences per wave
            float dx[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int lr = HX + wave * RPT + i;
#pragma unroll
                for (int rep = 0; rep < 2; ++rep) {
                    const int k = lane + rep * 64;
                    if (rep == 1 && lane >= 2 * R - 1) break;
                    float bf = 0.0f, dp = 0.0f;
#pragma unroll
                    for (int l = 1; l <= R; ++l) {
                        bf = fmaf(P.mj[l], sb[lr][k + l + R] + sb[lr][k - l + 1 + R], bf);
                        dp = fmaf(P.sy[l], sp[lr][k + l + R] - sp[lr][k - l + 1 + R], dp);
                    }
                    sfy[wave * RPT + i][k] = bf * dp;
                }
                dx[i] = 0.0f;
            }
            if constexpr (NDIM == 3) {
                float cp[NCOL], cb[NCOL], fx[NFX];
#pragma unroll
                for (int t = 0; t < NCOL; ++t) {
                    cp[t] = sp[wave * RPT + 1 + t][H2 + lane];
                    cb[t] = sb[wave * RPT + 1 + t][H2 + lane];
                }
#pragma unroll
                for (int f = 0; f < NFX; ++f) {
                    float bf = 0.0f, dp = 0.0f;
#pragma unroll
                    for (int l = 1; l <= R; ++l) {
                        bf = fmaf(P.mj[l], cb[f + l + R - 1] + cb[f - l + R], bf);
                        dp = fmaf(P.sx[l], cp[f + l + R - 1] - cp[f - l + R], dp);
                    }
                    fx[f] = bf * dp;
                }
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    float d = 0.0f;
#pragma unroll
                    for (int j = 1; j <= R; ++j) d = fmaf(P.sx[j], fx[i + j - 1 + R] - fx[i - j + R], d);
                    dx[i] = d;
                }
            }
            __syncthreads();

            // phase 3: assemble and update
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int row = wave * RPT + i;
                float dzs = 0.0f, dys = 0.0f;
#pragma unroll
                for (int j = 1; j <= R; ++j) {
                    dzs = fmaf(P.sz[j], fq[i][R + j - 1] - fq[i][R - j], dzs);
                    dys = fmaf(P.sy[j], sfy[row][lane + j - 1 + R] - sfy[row][lane - j + R], dys);
                }
                const float lap = dzs + dx[i] + dys;
                const float c = pq[i][0];
                const float out = pa[i] * fmaf(pk[i], lap, 2.0f * c) - pb[i] * pp[i];
                if (rin[i]) st_stream<NT>(out, nxt + int64_t(z) * sz + roff[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int k = 0; k < 2 * R - 1; ++k) {
                pq[i][k] = pq[i][k + 1];
                bq[i][k] = bq[i][k + 1];
                fq[i][k] = fq[i][k + 1];
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
    const int yc = clampi(y, 0, g.Y - 1);
    const int ey = max(0, max(g.lo[2] - y, y - (g.lo[2] + g.np[2] - 1)));
    // plane base pointers + unsigned 32-bit lane offsets off(x, y) = xy0 + x py + y
    auto off = [&](int x, int yy) -> unsigned { return unsigned(g.xy0 + x * g.py + yy); };
    const float *cur = P.cur + g.base;
    const float *rm = P.aux + g.base;
    float *nxt = P.nxt + g.base;
    const float *km = P.K + g.base;

    unsigned roff[RPT], rroff[RPT];
    bool rin[RPT];
    int ex2[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int x = x0 + wave * RPT + i;
        rin[i] = yin && x < g.X;
        roff[i] = rin[i] ? off(x, y) : 0u;
        rroff[i] = off(clampi(x, 0, g.X - 1), yc);
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
        hxin[s] = hxok[s] && yin && x >= 0 && x < g.X;
        hxrow[s] = (hr < R) ? hr : TX + hr;
        hxo[s] = hxin[s] ? off(x, y) : 0u;
        hxro[s] = off(clampi(x, 0, g.X - 1), yc);
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
        hyin[s] = hyok[s] && x < g.X && yy >= 0 && yy < g.Y;
        hyrow[s] = HXR + row;
        hycol[s] = (c < R) ? c : 64 + c;
        hyo[s] = hyin[s] ? off(x, yy) : 0u;
        hyro[s] = off(clampi(x, 0, g.X - 1), clampi(yy, 0, g.Y - 1));
    }

    float q[RPT][2 * R + 1], qr[RPT][2 * R + 1];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) {
            const int z = zb - R + k;
            q[i][k] = (rin[i] && z >= 0 && z < g.Z) ? (cur + int64_t(z) * sz)[roff[i]] : 0.0f;
            qr[i][k] = (rm + int64_t(clampi(z, 0, g.Z - 1)) * sz)[rroff[i]];
        }

    float nf[RPT], nfr[RPT], np_[RPT], nk[RPT], na[RPT], nb[RPT];
    float nhx[HXN > 0 ? HXN : 1], nhxr[HXN > 0 ? HXN : 1], nhy[YHN], nhyr[YHN];
    auto load = [&](int z) {
        const int zf = z + R;
        const int ez = max(0, max(g.lo[0] - z, z - (g.lo[0] + g.np[0] - 1)));
        const int64_t zo = int64_t(z) * sz;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            nf[i] = (rin[i] && zf < g.Z) ? cur[roff[i] + int64_t(zf) * sz] : 0.0f;
            nfr[i] = rm[rroff[i] + int64_t(min(zf, g.Z - 1)) * sz];
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
            const float out = pa[i] * fmaf(pk[i], Lp, 2.0f * c) - pb[i] * pp[i];
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
#define SW_VD_SHAPES(X) X(16, 8) X(8, 8) X(8, 4) X(16, 4)

template <int R, int NT>
hipError_t launch_vd_nt(int scheme, int ndim, const Tiling &t, StencilParams &P, hipStream_t s)
{
    const dim3 grid(P.ntx * P.nty * P.nzc);
    if (ndim == 2) {
        if (scheme == 1) hipLaunchKernelGGL((k_stag<R, 2, 1, 1, NT>), grid, dim3(64), 0, s, P);
        else hipLaunchKernelGGL((k_cent<R, 2, 1, 1, NT>), grid, dim3(64), 0, s, P);
        return hipGetLastError();
    }
#define SW_X(TXV, NWV)                                                                             \
    if (t.tx == TXV && t.nw == NWV) {                                                              \
        if (scheme == 1) hipLaunchKernelGGL((k_stag<R, 3, TXV, NWV, NT>), grid, dim3(64 * NWV), 0, s, P); \
        else hipLaunchKernelGGL((k_cent<R, 3, TXV, NWV, NT>), grid, dim3(64 * NWV), 0, s, P);    \
        return hipGetLastError();                                                                  \
    }
    SW_VD_SHAPES(SW_X)
#undef SW_X
    return hipErrorInvalidValue;
}

template <int R>
hipError_t launch_vd_radius(int scheme, int ndim, const Tiling &t, StencilParams &P, hipStream_t s)
{
    return t.nt ? launch_vd_nt<R, 1>(scheme, ndim, t, P, s) : launch_vd_nt<R, 0>(scheme, ndim, t, P, s);
}

}  // namespace sw
