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
#include "device.h"

namespace sw {

namespace {

constexpr int kBlock = 256;

struct AxisCoef {
    float s[9];     // s_j / h along the axis
};

struct MidCoef {
    float m[9];     // midpoint interpolation weights m_j
};

int grid_blocks(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return int(b);
}

// One thread per face of `axis`: the face box is m = -r .. n + r - 2 along the
// axis and the grid along the other two; the face sum of face m lives at the
// padded position of node m (inside the stored halo for m < 0 or m >= n).
__global__ void k_face_image(Geom g, int axis, int r, AxisCoef c, const float *__restrict__ phi,
                             const float *__restrict__ u, float *__restrict__ F)
{
    const int n[3] = {g.Z, g.X, g.Y};
    int e[3] = {n[0], n[1], n[2]};
    e[axis] = n[axis] + 2 * r - 1;
    const int64_t total = int64_t(e[0]) * e[1] * e[2];
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        int k[3];
        k[2] = int(i % e[2]);
        const int64_t t = i / e[2];
        k[1] = int(t % e[1]);
        k[0] = int(t / e[1]);
        k[axis] -= r;                                   // face index m
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

hipError_t launch_face_image(const Geom &g, int ndim, int r, const float *const *sj, const float *phi,
                             const float *u, float *const *F, hipStream_t s)
{
    const int n[3] = {g.Z, g.X, g.Y};
    for (int axis = 0; axis < 3; ++axis) {
        if (ndim == 2 && axis == 1) continue;
        AxisCoef c{};
        for (int l = 1; l <= r; ++l) c.s[l] = sj[axis][l];
        int e[3] = {n[0], n[1], n[2]};
        e[axis] += 2 * r - 1;
        const int64_t total = int64_t(e[0]) * e[1] * e[2];
        hipLaunchKernelGGL(k_face_image, dim3(grid_blocks(total)), dim3(kBlock), 0, s, g, axis, r, c, phi, u,
                           F[axis]);
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
