// Host-side plan: coefficients, padded layout, damping table, point tables.
//
// Coefficients (paper, "Space discretization"): central differences of even
// order SO = 2r, computed from their closed forms in double precision:
//   second derivative  v_j = 2 (-1)^{j+1} (r!)^2 / (j^2 (r-j)! (r+j)!),  v_0 = -2 sum v_j
//   first derivative   c_j = (-1)^{j+1} (r!)^2 / (j (r-j)! (r+j)!)      (f' ~ sum c_j (f_{+j} - f_{-j}) / dx)
//   staggered          s_j = (-1)^{j+1} ((2r-1)!!)^2 / ((2j-1)^2 (r-j)! (r+j-1)! 4^{r-1})
//   midpoint           m_j = (-1)^{j+1} ((2r-1)!!)^2 / ((2j-1) (r-j)! (r+j-1)! 2^{2r-1})
// (the last two are the half-node derivative and interpolation weights of the
// conservative variable-density operator).
//
// Points (paper, "Sources and receivers"): Kaiser-windowed sinc weights
// W(n + alpha) sinc(n + alpha) with alpha = k0 - xi, k0 = floor(xi + 0.5), or
// linear weights; products over axes; zero weights dropped.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace sw {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
const std::string &last_error() { return g_err; }

sw_status fail(sw_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

static double fact(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

static double dfact_odd(int n)  // n!! for odd n
{
    double f = 1.0;
    for (int i = n; i > 1; i -= 2) f *= i;
    return f;
}

static void coefficients(sw_plan *p)
{
    const int r = p->r;
    double sum = 0.0;
    for (int j = 1; j <= r; ++j) {
        const double sgn = (j % 2) ? 1.0 : -1.0;
        const double fr = fact(r) * fact(r);
        p->v2[j] = 2.0 * sgn * fr / (double(j) * j * fact(r - j) * fact(r + j));
        p->w1[j] = sgn * fr / (double(j) * fact(r - j) * fact(r + j));
        const double df = dfact_odd(2 * r - 1);
        const double den = fact(r - j) * fact(r + j - 1);
        p->sg[j] = sgn * (df / (double(2 * j - 1) * (2 * j - 1))) * (df / den) / std::pow(4.0, r - 1);
        p->mp[j] = sgn * (df / double(2 * j - 1)) * (df / den) / std::pow(2.0, 2 * r - 1);
        sum += p->v2[j];
    }
    p->v2[0] = -2.0 * sum;
}

double a1d(int space_order)
{
    sw_plan tmp;
    tmp.r = space_order / 2;
    coefficients(&tmp);
    double a = std::fabs(tmp.v2[0]);
    for (int j = 1; j <= tmp.r; ++j) a += 2.0 * std::fabs(tmp.v2[j]);
    return a;
}

static int64_t round_up(int64_t a, int64_t m) { return (a + m - 1) / m * m; }

sw_status build_layout(sw_plan *p)
{
    const sw_problem &q = p->prob;
    p->ndim = q.ndim;
    p->r = q.space_order / 2;
    p->halo = (q.scheme == SW_VD_STAGGERED) ? 2 * p->r : p->r;
    // internal 3D view: (z, x, y); a 2D grid (z, x) becomes (z, 1, x)
    int phys[3], lo[3], hi[3];
    double h[3];
    if (q.ndim == 3) {
        for (int i = 0; i < 3; ++i) {
            phys[i] = q.n[i];
            lo[i] = q.nbl[i][0];
            hi[i] = q.nbl[i][1];
            h[i] = q.h[i];
        }
    } else {
        phys[0] = q.n[0]; lo[0] = q.nbl[0][0]; hi[0] = q.nbl[0][1]; h[0] = q.h[0];
        phys[1] = 1;      lo[1] = 0;           hi[1] = 0;           h[1] = 1.0;
        phys[2] = q.n[1]; lo[2] = q.nbl[1][0]; hi[2] = q.nbl[1][1]; h[2] = q.h[1];
    }
    for (int i = 0; i < 3; ++i) {
        p->nphys[i] = phys[i];
        p->lo[i] = lo[i];
        p->dims[i] = phys[i] + lo[i] + hi[i];
        p->hh[i] = h[i];
    }
    p->hz = p->halo;
    p->hx = (q.ndim == 3) ? p->halo : 0;
    p->pad[0] = p->dims[0] + 2 * p->hz;
    p->pad[1] = p->dims[1] + 2 * p->hx;
    p->pad[2] = int(round_up(kRowAlign + p->dims[2] + p->halo, kRowAlign));
    p->origin = (int64_t(p->hz) * p->pad[1] + p->hx) * p->pad[2] + kRowAlign;
    p->field_elems = int64_t(p->pad[0]) * p->pad[1] * p->pad[2];
    p->grid_nodes = int64_t(p->dims[0]) * p->dims[1] * p->dims[2];
    p->phys_nodes = int64_t(phys[0]) * phys[1] * phys[2];
    p->dV = 1.0;
    for (int i = 0; i < q.ndim; ++i) p->dV *= q.h[i];
    coefficients(p);
    // damping table by squared distance (in cells) to the physical box
    int64_t maxd2 = 0;
    for (int i = 0; i < 3; ++i) {
        const int m = std::max(lo[i], hi[i]);
        maxd2 += int64_t(m) * m;
    }
    p->damp_n = int(maxd2 + 1);
    p->damp.assign(2 * size_t(p->damp_n), 0.0f);
    p->damp64.assign(2 * size_t(p->damp_n), 0.0);
    for (int d2 = 0; d2 < p->damp_n; ++d2) {
        const double d = std::sqrt(double(d2));
        const double eta = (d2 == 0) ? 0.0 : q.damp_alpha * std::pow(d, q.damp_power);
        const double e = eta * q.dt;
        p->damp64[2 * d2] = 1.0 / (1.0 + e);
        p->damp64[2 * d2 + 1] = (1.0 - e) / (1.0 + e);
        p->damp[2 * d2] = float(p->damp64[2 * d2]);
        p->damp[2 * d2 + 1] = float(p->damp64[2 * d2 + 1]);
    }
    build_workspace_map(p);
    return SW_OK;
}

void build_workspace_map(sw_plan *p)
{
    WorkspaceMap &w = p->ws;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    // values are 4 bytes, or 8 for a double-precision plan
    const size_t es = p->prob.dtype == SW_F64 ? sizeof(double) : sizeof(float);
    const size_t fb = size_t(p->field_elems) * es;
    w.model_k = take(fb);
    w.model_aux = (p->prob.scheme != SW_CONST) ? take(fb) : 0;
    w.damp = take(size_t(p->damp_n) * 2 * es);
    w.counter = take(sizeof(uint32_t));
    auto pts = [&](const PointSet &ps, WorkspaceMap::Pts &o) {
        const size_t ne = std::max<size_t>(1, ps.node.size());
        const size_t nu = std::max<size_t>(1, ps.unode.size());
        o.ptr = take((ps.count + 1) * sizeof(int32_t));
        o.node = take(ne * sizeof(int64_t));
        o.pid = take(ne * sizeof(int32_t));
        o.d2 = take(ne * sizeof(int32_t));
        o.phys = take(ne * sizeof(int64_t));
        o.weight = take(ne * es);
        o.unode = take(nu * sizeof(int64_t));
        o.uptr = take((nu + 1) * sizeof(int32_t));
        o.uent = take(ne * sizeof(int32_t));
        o.coef_a = take(ne * es);
        o.coef_s = take(ne * es);
        o.wscaled = take(ne * es);
        o.inj = take(2 * nu * es);
    };
    pts(p->src, w.src);
    pts(p->rec, w.rec);
    w.total = off;
}

static double bessel_i0(double x)
{
    // power series sum ((x/2)^k / k!)^2
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / (double(k) * k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

static double sinc_norm(double x)
{
    if (x == 0.0) return 1.0;
    if (x == std::floor(x)) return 0.0;     // exact zero at the other integers
    const double px = M_PI * x;
    return std::sin(px) / px;
}

struct AxisW {
    int k;
    double w;
};

static void axis_weights(double xi, int interp, int radius, double b, std::vector<AxisW> &out)
{
    out.clear();
    if (interp == SW_INTERP_LINEAR) {
        const double k = std::floor(xi);
        const double t = xi - k;
        out.push_back({int(k), 1.0 - t});
        if (t != 0.0) out.push_back({int(k) + 1, t});
        return;
    }
    const double k0 = std::floor(xi + 0.5);
    const double alpha = k0 - xi;
    const double i0b = bessel_i0(b);
    for (int n = -radius; n <= radius; ++n) {
        const double x = n + alpha;
        if (std::fabs(x) > radius) continue;
        const double arg = 1.0 - (x / radius) * (x / radius);
        const double win = bessel_i0(b * std::sqrt(std::max(0.0, arg))) / i0b;
        const double w = win * sinc_norm(x);
        if (w != 0.0) out.push_back({int(k0) + n, w});
    }
}

sw_status build_points(sw_plan *p, PointSet &ps, int count, const double *coords, int interp,
                       int radius, double kaiser_b, bool source)
{
    const sw_problem &q = p->prob;
    if (count < 0) return fail(SW_ERR_ARG, "point count must be >= 0");
    if (count > 0 && !coords) return fail(SW_ERR_ARG, "coords is NULL");
    if (interp != SW_INTERP_HICKS && interp != SW_INTERP_LINEAR)
        return fail(SW_ERR_ARG, "interp must be SW_INTERP_HICKS or SW_INTERP_LINEAR");
    if (interp == SW_INTERP_HICKS) {
        if (radius < 1 || radius > 10) return fail(SW_ERR_ARG, "window radius must be in 1..10");
        if (kaiser_b <= 0.0) {
            if (radius != 4)
                return fail(SW_ERR_ARG, "Kaiser shape b must be given for window radius != 4");
            kaiser_b = 6.31;
        }
    }
    PointSet out;
    out.count = count;
    out.interp = interp;
    out.radius = radius;
    out.kaiser_b = kaiser_b;
    out.coords.assign(coords, coords + size_t(count) * q.ndim);
    out.ptr.assign(1, 0);
    // map problem axes to the internal (z, x, y) axes
    int axmap[3];
    if (q.ndim == 3) { axmap[0] = 0; axmap[1] = 1; axmap[2] = 2; }
    else { axmap[0] = 0; axmap[1] = 2; axmap[2] = -1; }
    // a point and, for a source, its images across sides with a mirror ghost
    // condition: the problem doubled about the boundary node of such a side
    // carries the source reflected about that node, times -1 (Dirichlet) or
    // +1 (Neumann); across two mirrored sides, the image of the image
    struct Image {
        double c[3];
        double sign;
    };
    std::vector<Image> imgs;
    std::vector<AxisW> aw[3];
    for (int pt = 0; pt < count; ++pt) {
        Image o{{0.0, 0.0, 0.0}, 1.0};
        for (int a = 0; a < q.ndim; ++a) {
            const double c = coords[size_t(pt) * q.ndim + a];
            const double ext = double(q.n[a] - 1) * q.h[a];
            if (!(c >= 0.0 && c <= ext))
                return fail(SW_ERR_DOMAIN, "point " + std::to_string(pt) +
                                               " lies outside the physical grid");
            o.c[a] = c;
        }
        imgs.assign(1, o);
        if (source)
            for (int a = 0; a < q.ndim; ++a) {
                const int ia = axmap[a];
                const size_t n0 = imgs.size();
                for (size_t j = 0; j < n0; ++j)
                    for (int side = 0; side < 2; ++side) {
                        const int bc = p->bcm[ia][side];
                        if (!bc) continue;
                        // boundary node of the extended grid, metres from physical node 0
                        const double m = side == 0 ? -double(p->lo[ia]) * q.h[a]
                                                   : double(p->dims[ia] - 1 - p->lo[ia]) * q.h[a];
                        Image im = imgs[j];
                        im.c[a] = 2.0 * m - imgs[j].c[a];
                        im.sign = imgs[j].sign * (bc == SW_BC_DIRICHLET ? -1.0 : 1.0);
                        imgs.push_back(im);
                    }
            }
        for (size_t j = 0; j < imgs.size(); ++j) {
            for (int i = 0; i < 3; ++i) aw[i].assign(1, AxisW{0, 1.0});
            for (int a = 0; a < q.ndim; ++a) {
                const int ia = axmap[a];
                axis_weights(imgs[j].c[a] / q.h[a], interp, radius, kaiser_b, aw[ia]);
                std::vector<AxisW> kept;
                for (auto &e : aw[ia]) {
                    int k = e.k + p->lo[ia];
                    double w = e.w;
                    if (k < 0 || k >= p->dims[ia]) {
                        const int bc = p->bcm[ia][k < 0 ? 0 : 1];
                        if (j == 0 && !bc)
                            return fail(SW_ERR_DOMAIN, "footprint of point " + std::to_string(pt) +
                                                           " leaves the extended grid");
                        // a source's entries beyond a mirrored side belong to
                        // the other half of the doubled problem
                        if (source) continue;
                        // a receiver reads the ghost node: its mirror node,
                        // times -1 across a Dirichlet side
                        k = k < 0 ? -k : 2 * (p->dims[ia] - 1) - k;
                        if (k < 0 || k >= p->dims[ia])
                            return fail(SW_ERR_DOMAIN, "footprint of point " + std::to_string(pt) +
                                                           " reaches past the mirror of the grid");
                        if (bc == SW_BC_DIRICHLET) w = -w;
                    }
                    kept.push_back({k - p->lo[ia], w});
                }
                aw[ia].swap(kept);
            }
            for (auto &ez : aw[0])
                for (auto &ex : aw[1])
                    for (auto &ey : aw[2]) {
                        const int z = ez.k + p->lo[0], x = ex.k + p->lo[1], y = ey.k + p->lo[2];
                        const double w = imgs[j].sign * ez.w * ex.w * ey.w;
                        if (w == 0.0) continue;
                        out.node.push_back(p->origin + (int64_t(z) * p->pad[1] + x) * p->pad[2] + y);
                        out.pid.push_back(pt);
                        // squared distance (cells) from the node to the physical box
                        int64_t d2 = 0;
                        const int c3[3] = {z, x, y};
                        int64_t phys = 0;
                        for (int i = 0; i < 3; ++i) {
                            const int e = std::max(0, std::max(p->lo[i] - c3[i],
                                                               c3[i] - (p->lo[i] + p->nphys[i] - 1)));
                            d2 += int64_t(e) * e;
                            const int pc = std::min(std::max(c3[i] - p->lo[i], 0), p->nphys[i] - 1);
                            phys = phys * p->nphys[i] + pc;
                        }
                        out.d2.push_back(int32_t(d2));
                        out.phys.push_back(phys);
                        out.weight.push_back(float(w));
                        out.weight64.push_back(w);
                    }
        }
        out.ptr.push_back(int32_t(out.node.size()));
        out.max_per_point = std::max(out.max_per_point, out.ptr[pt + 1] - out.ptr[pt]);
    }
    // group entries by node (stable: ties keep point order) for the gather
    std::vector<int32_t> order(out.node.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return out.node[a] < out.node[b]; });
    out.uptr.assign(1, 0);
    for (size_t i = 0; i < order.size(); ++i) {
        if (i == 0 || out.node[order[i]] != out.node[order[i - 1]]) {
            if (i) out.uptr.push_back(int32_t(i));
            out.unode.push_back(out.node[order[i]]);
        }
        out.uent.push_back(order[i]);
    }
    if (!order.empty()) out.uptr.push_back(int32_t(order.size()));
    for (size_t u = 0; u + 1 < out.uptr.size(); ++u)
        out.max_per_node = std::max(out.max_per_node, out.uptr[u + 1] - out.uptr[u]);
    ps = std::move(out);
    build_workspace_map(p);
    return SW_OK;
}

}  // namespace sw
