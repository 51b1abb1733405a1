// Imaging kernels of the staggered variable-density adjoint.
//
// With zero ghosts the staggered operator is L = -sum_i (D+_i)^T diag(b_i) D+_i
// (b_i the face buoyancies), so its adjoint is the forward stencil itself; the
// density enters the gradient through K = dt^2 rho c^2 and through the face
// buoyancies.  Per adjoint step (level phi^{n+1} against the recomputed
// forward level u^n):
//   face term    F_i(m) -= (D+_i phi^{n+1})_{m+1/2} (D+_i u^n)_{m+1/2}
//                for every face m = -r .. n_i + r - 2 the divergence reads
//   source term  S(x)   += phi^{n+1}(x) M q^n(x) at the source nodes
// and once at the end, per extended node,
//   dJ/db   = transpose of b_{m+1/2} = sum_j m_j (b_{clamp(m+j)} + b_{clamp(m-j+1)})
//             applied to the face sums,
//   x       = (dJ/dK + S / K^2) / b          (dJ/dc = fold(x) 2 dt^2 c)
//   y       = dJ/dK K b - dJ/db b^2          (dJ/drho = fold(y))
// with dJ/dK accumulated by the imaging stencil and M = K b.
#include <algorithm>

#include "device.h"
#include "stencil_const.h"

namespace sw {

namespace {

constexpr int kBlock = 256;

struct AxisCoef {
    float s[11];    // s_j / h along the axis
};

struct MidCoef {
    float m[11];    // midpoint interpolation weights m_j
};

int grid_blocks(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return int(b);
}

// Faces outside the grid's node range, one thread each: m = -r .. -1 and
// m = n .. n + r - 2 along `axis` (the 2r - 1 faces that no grid node owns),
// the grid along the other two axes.  The face sum of face m lives at the
// padded position of node m, inside the stored halo.
__global__ void k_face_image_outer(Geom g, int axis, int r, AxisCoef c, const float *__restrict__ phi,
                                   const float *__restrict__ u, float *__restrict__ F)
{
    const int n[3] = {g.Z, g.X, g.Y};
    int e[3] = {n[0], n[1], n[2]};
    e[axis] = 2 * r - 1;
    const int64_t total = int64_t(e[0]) * e[1] * e[2];
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        int k[3];
        k[2] = int(i % e[2]);
        const int64_t t = i / e[2];
        k[1] = int(t % e[1]);
        k[0] = int(t / e[1]);
        k[axis] = (k[axis] < r) ? k[axis] - r : n[axis] + k[axis] - r;   // face index m
        const int m = k[axis];
        auto at = [&](const float *f, int v) -> float {  // node v along the axis, zero off the grid
            if (v < 0 || v >= n[axis]) return 0.0f;
            int q[3] = {k[0], k[1], k[2]};
            q[axis] = v;
            return f[elem(g, q[0], q[1], q[2])];
        };
        float dp = 0.0f, du = 0.0f;
        for (int l = 1; l <= r; ++l) {
            dp = fmaf(c.s[l], at(phi, m + l) - at(phi, m - l + 1), dp);
            du = fmaf(c.s[l], at(u, m + l) - at(u, m - l + 1), du);
        }
        const int64_t o = elem(g, k[0], k[1], k[2]);
        F[o] = fmaf(-dp, du, F[o]);
    }
}

struct FaceTileParams {
    Geom g;
    float sz[11], sx[11], sy[11];   // s_j / h per axis
    const float *phi[2], *u[2];     // level pairs, accumulated in this order
    float *F[3];
    int ntx, nty, nzc, zc;
};

// The faces k + 1/2 of every grid node k along each axis for NP level pairs
// (phi, u) at once, one tile of TX = NW * RPT rows x 64 columns per block
// marching along a z chunk (each thread owns RPT rows of one column): the face
// sums are read and written once for all pairs.  z differences come from
// rotating register queues (2R planes, compile-time slots), x and y
// differences from the plane staged in LDS with R - 1 nodes of halo below and
// R above: the tile's own nodes from the queues, the halo from memory.
// Buffer addressing as in the stencils: one descriptor per array over the
// block's z window, 32-bit in-plane byte offsets fixed before the march (the
// halo items of each thread included), off-grid x / y positions at an offset
// past the descriptor (loads read zero, stores are dropped) and off-grid z
// planes masked to zero.
template <int R, int NDIM, int NW, int RPT, int NP>
__global__ void __launch_bounds__(64 * NW) k_face_tile(FaceTileParams P)
{
    constexpr int TX = NW * RPT;
    constexpr int HL = R - 1;
    constexpr int LXR = (NDIM == 3) ? TX + 2 * R - 1 : 1;
    constexpr int LYC = 64 + 2 * R - 1;
    constexpr int Q = 2 * R;
    constexpr int NTH = 64 * NW;
    constexpr int NF = 2 * NP;                   // staged fields: phi and u of each pair
    constexpr int R0 = (NDIM == 3) ? HL : 0;     // LDS row of the tile's first row (2D: one row, no x halo)
    constexpr int NXH = (NDIM == 3) ? (2 * R - 1) * LYC : 0;   // halo items: x-halo rows (all columns)
    constexpr int NH = NXH + TX * (2 * R - 1);                  // and the y-halo columns of the tile's rows
    constexpr int NHT = (NH + NTH - 1) / NTH;                   // halo items per thread
    constexpr int kOut = 0x7ffffe00;
    static_assert(NDIM == 3 || (NW == 1 && RPT == 1), "2D tiles are one row");
    __shared__ float sf[NF][LXR * LYC + 1];      // element LXR * LYC: sink of idle halo items
    const Geom &g = P.g;
    const float *src[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) src[f] = (f & 1) ? P.u[f >> 1] : P.phi[f >> 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int ty = bid % P.nty;
    const int rest = bid / P.nty;
    const int tx = rest % P.ntx;
    const int zc = rest / P.ntx;
    const int y0 = ty * 64, x0 = tx * TX;
    const int y = y0 + lane;
    const int zb = zc * P.zc;
    const int ze = min(zb + P.zc, g.Z);
    // windows: planes zw .. zt - 1 of the staged fields, zb .. ze - 1 of the face sums
    const int zw = zb - R + 1, zt = ze + R;
    const int64_t sz = int64_t(g.px) * g.py;
    const int pb = int(sz) * 4;
    const int64_t w0 = g.base + int64_t(zw) * sz, f0e = g.base + int64_t(zb) * sz;
    __amdgpu_buffer_rsrc_t rs[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) rs[f] = buf_res(src[f] + w0, uint32_t(zt - zw) * uint32_t(pb));
    const uint32_t fbytes = uint32_t(ze - zb) * uint32_t(pb);
    const auto rf0 = buf_res(P.F[0] + f0e, fbytes);
    const auto rf1 = buf_res(P.F[NDIM == 3 ? 1 : 0] + f0e, fbytes);
    const auto rf2 = buf_res(P.F[2] + f0e, fbytes);
    auto off = [&](int x, int yy) -> int {
        return (x >= 0 && x < g.X && yy >= 0 && yy < g.Y) ? (g.xy0 + x * g.py + yy) * 4 : kOut;
    };
    auto zmask = [&](int z) -> unsigned { return (z >= 0 && z < g.Z) ? ~0u : 0u; };
    int ro[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) ro[i] = off(x0 + wave * RPT + i, y);
    int ho[NHT], hl[NHT];
#pragma unroll
    for (int t = 0; t < NHT; ++t) {
        const int e = threadIdx.x + t * NTH;
        int row = 0, col = 0;
        if (e < NXH) {                       // rows 0 .. HL - 1 and R0 + TX .. LXR - 1, every column
            const int k = e / LYC;
            col = e % LYC;
            row = (k < HL) ? k : R0 + TX + (k - HL);
        } else {                             // columns 0 .. HL - 1 and HL + 64 .. LYC - 1 of the tile's rows
            const int e2 = e - NXH;
            const int k = e2 % (2 * R - 1);
            row = R0 + e2 / (2 * R - 1);
            col = (k < HL) ? k : HL + 64 + (k - HL);
        }
        const bool ok = e < NH;
        ho[t] = ok ? off((NDIM == 3) ? x0 - HL + row : 0, y0 - HL + col) : kOut;
        hl[t] = ok ? row * LYC + col : LXR * LYC;
    }
    // slot (s + k) % Q of field f, row i holds the value at z - R + 1 + k on step s (z = zz + s)
    float q[NF][RPT][Q];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int k = 0; k < Q - 1; ++k)
                q[f][i][k] = keep_mask(buf_ld<0>(rs[f], ro[i], k * pb), zmask(zw + k));
    for (int zz = zb; zz < ze; zz += Q) {
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const int z = zz + s;
            if (z >= ze) break;
            const int fo = (z - zb) * pb;
            // this plane's face sums are loaded first, so that they arrive
            // while the plane is staged
            float f0[RPT], f1[RPT], f2[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                f0[i] = buf_ld<1>(rf0, ro[i], fo);
                f1[i] = (NDIM == 3) ? buf_ld<1>(rf1, ro[i], fo) : 0.0f;
                f2[i] = buf_ld<1>(rf2, ro[i], fo);
                const unsigned m = zmask(z + R);
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    q[f][i][(s + Q - 1) % Q] = keep_mask(buf_ld<0>(rs[f], ro[i], (z + R - zw) * pb), m);
                    sf[f][(R0 + wave * RPT + i) * LYC + HL + lane] = q[f][i][(s + R - 1) % Q];
                }
            }
#pragma unroll
            for (int t = 0; t < NHT; ++t)
#pragma unroll
                for (int f = 0; f < NF; ++f) sf[f][hl[t]] = buf_ld<0>(rs[f], ho[t], (z - zw) * pb);
            __syncthreads();
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int ci = R0 + wave * RPT + i, cj = HL + lane;
                float a0 = f0[i], a1 = f1[i], a2 = f2[i];
#pragma unroll
                for (int pr = 0; pr < NP; ++pr) {
                    const int fp = 2 * pr, fu = 2 * pr + 1;
                    float dpz = 0.0f, duz = 0.0f, dpx = 0.0f, dux = 0.0f, dpy = 0.0f, duy = 0.0f;
#pragma unroll
                    for (int l = 1; l <= R; ++l) {
                        dpz = fmaf(P.sz[l], q[fp][i][(s + R - 1 + l) % Q] - q[fp][i][(s + R - l) % Q], dpz);
                        duz = fmaf(P.sz[l], q[fu][i][(s + R - 1 + l) % Q] - q[fu][i][(s + R - l) % Q], duz);
                        if constexpr (NDIM == 3) {
                            dpx = fmaf(P.sx[l], sf[fp][(ci + l) * LYC + cj] - sf[fp][(ci - l + 1) * LYC + cj], dpx);
                            dux = fmaf(P.sx[l], sf[fu][(ci + l) * LYC + cj] - sf[fu][(ci - l + 1) * LYC + cj], dux);
                        }
                        dpy = fmaf(P.sy[l], sf[fp][ci * LYC + cj + l] - sf[fp][ci * LYC + cj - l + 1], dpy);
                        duy = fmaf(P.sy[l], sf[fu][ci * LYC + cj + l] - sf[fu][ci * LYC + cj - l + 1], duy);
                    }
                    a0 = fmaf(-dpz, duz, a0);
                    if constexpr (NDIM == 3) a1 = fmaf(-dpx, dux, a1);
                    a2 = fmaf(-dpy, duy, a2);
                }
                buf_st<1>(a0, rf0, ro[i], fo);
                if constexpr (NDIM == 3) buf_st<1>(a1, rf1, ro[i], fo);
                buf_st<1>(a2, rf2, ro[i], fo);
            }
            __syncthreads();
        }
    }
}

// 3D tiles of 8 waves (faster than 4 or 16 at 592^3 SO8), with 2 rows per
// thread for one pair up to radius 4 and 1 row otherwise (the queues take the
// registers); 2D tiles of one row.
constexpr int face_waves(int) { return 8; }
constexpr int face_rows_per_thread(int r, int np) { return (r <= 4 && np == 1) ? 2 : 1; }

template <int R, int NP>
void launch_face_tile_np(int ndim, FaceTileParams &P, hipStream_t s)
{
    if (ndim == 2)
        hipLaunchKernelGGL((k_face_tile<R, 2, 1, 1, NP>), dim3(P.ntx * P.nty * P.nzc), dim3(64), 0, s, P);
    else
        hipLaunchKernelGGL((k_face_tile<R, 3, face_waves(R), face_rows_per_thread(R, NP), NP>),
                           dim3(P.ntx * P.nty * P.nzc), dim3(64 * face_waves(R)), 0, s, P);
}

template <int R>
void launch_face_tile(int ndim, int np, FaceTileParams &P, hipStream_t s)
{
    if (np == 2) launch_face_tile_np<R, 2>(ndim, P, s);
    else launch_face_tile_np<R, 1>(ndim, P, s);
}

// One thread per unique source node: S(x) += phi(x) sum_e coef_s[e] amp[pid[e]]
// (coef_s = M w / dV, the stored source part of the forward update).
__global__ void k_src_image(PointTableDev t, const float *__restrict__ phi, const float *__restrict__ amp,
                            float *__restrict__ S)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= t.nuniq) return;
    float q = 0.0f;
    for (int k = t.uptr[u]; k < t.uptr[u + 1]; ++k) {
        const int e = t.uent[k];
        q = fmaf(t.coef_s[e], amp[t.pid[e]], q);
    }
    const int64_t n = t.unode[u];
    S[n] = fmaf(phi[n], q, S[n]);
}

// Sum of the face sums F over faces m in [a, b] clipped to the face range.
__device__ inline float face_range_sum(const Geom &g, const float *F, int axis, int n, int r,
                                       const int k[3], int a, int b)
{
    a = max(a, -r);
    b = min(b, n + r - 2);
    float s = 0.0f;
    int q[3] = {k[0], k[1], k[2]};
    for (int m = a; m <= b; ++m) {
        q[axis] = m;
        s += F[elem(g, q[0], q[1], q[2])];
    }
    return s;
}

// Per extended node: dJ/db from the face sums, then x and y (see the header).
__global__ void k_vd_chain(Geom g, int r, int ndim, MidCoef c, const float *__restrict__ gK,
                           const float *__restrict__ F0, const float *__restrict__ F1,
                           const float *__restrict__ F2, const float *__restrict__ S,
                           const float *__restrict__ K, const float *__restrict__ b,
                           float *__restrict__ xout, float *__restrict__ yout)
{
    const int n[3] = {g.Z, g.X, g.Y};
    const float *F[3] = {F0, F1, F2};
    const int64_t total = int64_t(g.Z) * g.X * g.Y;
    constexpr int kInf = 1 << 29;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        int k[3];
        k[2] = int(i % g.Y);
        const int64_t t = i / g.Y;
        k[1] = int(t % g.X);
        k[0] = int(t / g.X);
        float gb = 0.0f;
        for (int axis = 0; axis < 3; ++axis) {
            if (ndim == 2 && axis == 1) continue;       // a 2D grid is (z, 1, x): no faces along x
            const int v = k[axis], na = n[axis];
            // node indices that clamp onto v: [lo, hi]
            const int lo = (v == 0) ? -kInf : v;
            const int hi = (v == na - 1) ? kInf : v;
            for (int j = 1; j <= r; ++j) {
                // faces m with m + j in [lo, hi], and with m - j + 1 in [lo, hi]
                const float a = face_range_sum(g, F[axis], axis, na, r, k, lo == -kInf ? -kInf : lo - j,
                                               hi == kInf ? kInf : hi - j);
                const float bb = face_range_sum(g, F[axis], axis, na, r, k, lo == -kInf ? -kInf : lo + j - 1,
                                                hi == kInf ? kInf : hi + j - 1);
                gb = fmaf(c.m[j], a + bb, gb);
            }
        }
        const int64_t o = elem(g, k[0], k[1], k[2]);
        const float kk = K[o], bo = b[o], gk = gK[o];
        xout[o] = (gk + S[o] / (kk * kk)) / bo;
        yout[o] = gk * kk * bo - gb * bo * bo;
    }
}

}  // namespace

hipError_t launch_face_image(const Geom &g, int ndim, int r, const float *const *sj, int np,
                             const float *const *phi, const float *const *u, float *const *F, hipStream_t s)
{
    if (r < 1 || r > 10 || np < 1 || np > 2) return hipErrorInvalidValue;
    // faces of the grid nodes: z-marching tiles
    FaceTileParams T{};
    T.g = g;
    for (int l = 1; l <= r; ++l) {
        T.sz[l] = sj[0][l];
        T.sx[l] = sj[1][l];
        T.sy[l] = sj[2][l];
    }
    for (int k = 0; k < np; ++k) {
        T.phi[k] = phi[k];
        T.u[k] = u[k];
    }
    for (int a = 0; a < 3; ++a) T.F[a] = F[a];
    const int tx = (ndim == 2) ? 1 : face_waves(r) * face_rows_per_thread(r, np);
    T.ntx = (g.X + tx - 1) / tx;
    T.nty = (g.Y + 63) / 64;
    T.zc = (ndim == 2) ? 16 : 32;
    // a block's window (chunk plus 2r - 1 planes) stays below 2^31 bytes: 32-bit buffer offsets
    const int64_t pbytes = int64_t(g.px) * g.py * 4;
    const int64_t zmax = ((int64_t(1) << 31) - 1) / pbytes - (2 * r - 1);
    if (zmax < 1) return hipErrorInvalidValue;
    T.zc = int(std::min<int64_t>(T.zc, zmax));
    T.nzc = (g.Z + T.zc - 1) / T.zc;
    switch (r) {
    case 1: launch_face_tile<1>(ndim, np, T, s); break;
    case 2: launch_face_tile<2>(ndim, np, T, s); break;
    case 3: launch_face_tile<3>(ndim, np, T, s); break;
    case 4: launch_face_tile<4>(ndim, np, T, s); break;
    case 5: launch_face_tile<5>(ndim, np, T, s); break;
    case 6: launch_face_tile<6>(ndim, np, T, s); break;
    case 7: launch_face_tile<7>(ndim, np, T, s); break;
    case 8: launch_face_tile<8>(ndim, np, T, s); break;
    case 9: launch_face_tile<9>(ndim, np, T, s); break;
    default: launch_face_tile<10>(ndim, np, T, s); break;
    }
    // faces no grid node owns (m < 0 or m >= n along each axis), pair by pair
    const int n[3] = {g.Z, g.X, g.Y};
    for (int k = 0; k < np; ++k)
        for (int axis = 0; axis < 3; ++axis) {
            if (ndim == 2 && axis == 1) continue;
            AxisCoef c{};
            for (int l = 1; l <= r; ++l) c.s[l] = sj[axis][l];
            int e[3] = {n[0], n[1], n[2]};
            e[axis] = 2 * r - 1;
            const int64_t total = int64_t(e[0]) * e[1] * e[2];
            hipLaunchKernelGGL(k_face_image_outer, dim3(grid_blocks(total)), dim3(kBlock), 0, s, g, axis, r, c,
                               phi[k], u[k], F[axis]);
        }
    return hipGetLastError();
}

hipError_t launch_src_image(const PointTableDev &t, const float *phi, const float *amp, float *S,
                            hipStream_t s)
{
    if (t.nuniq <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_src_image, dim3((t.nuniq + kBlock - 1) / kBlock), dim3(kBlock), 0, s, t, phi, amp, S);
    return hipGetLastError();
}

hipError_t launch_vd_chain(const Geom &g, int r, int ndim, const float *mj, const float *gK,
                           const float *const *F, const float *S, const float *K, const float *b,
                           float *xout, float *yout, hipStream_t s)
{
    MidCoef c{};
    for (int l = 1; l <= r; ++l) c.m[l] = mj[l];
    const int64_t total = int64_t(g.Z) * g.X * g.Y;
    hipLaunchKernelGGL(k_vd_chain, dim3(grid_blocks(total)), dim3(kBlock), 0, s, g, r, ndim, c, gK, F[0],
                       F[1], F[2], S, K, b, xout, yout);
    return hipGetLastError();
}

}  // namespace sw
