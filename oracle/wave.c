/*
 * FP64 CPU oracle for the explicit acoustic finite-difference propagator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP implementation.
 *
 * What lives here is the inner work of one leapfrog time step over the whole
 * extended grid, written as plain loops with a ghost-node accessor:
 *
 *   (L p)  spatial operator, one of
 *     - constant density: the centred high-order Laplacian
 *         sum_i dx_i^-2 ( v_0 p_k + sum_j v_j (p_{k+j} + p_{k-j}) )
 *       (paper, "Space discretization", second-derivative formula);
 *     - variable density, centred: the Laplacian minus (grad rho / rho).grad p,
 *       each first derivative the centred formula with the 1/(2 dx) prefactor
 *       (paper, "Time discretization", expanded variable-density equation, and
 *       "Space discretization", first-derivative formula);
 *     - variable density, staggered: sum_i D-_i ( b_{i+1/2} D+_i p ), b = 1/rho,
 *       half-node first derivatives and order-matched midpoint interpolation of b.
 *
 *   update  p^{n+1} = A (2 p^n + K (L p)) - B p^{n-1}
 *           A = 1/(1 + eta dt), B = (1 - eta dt)/(1 + eta dt)
 *     which is the second-order central time difference of the damped wave
 *     equation (paper, "Time discretization" central differences applied to the
 *     damped equation of "Boundary conditions and domain truncation"); K is
 *     dt^2 c^2, or dt^2 rho c^2 for the staggered operator.
 *
 * Ghost nodes outside the grid follow the per-side boundary condition:
 *   none      -> 0
 *   dirichlet -> odd mirror about the boundary node (boundary node held at 0)
 *   neumann   -> even mirror about the boundary node
 * Model fields (b or rho) outside the grid: on a mirrored side the even
 * mirror about the boundary node (the image of the model, so that the
 * mirrored problem is the restriction of the problem doubled about that
 * node, which is what the image method of the ghost conditions means); on a
 * side without a mirror condition the nearest grid value.
 *
 * Arrays are C-ordered over (N0, N1, N2); a 2D grid uses N2 = 1 and ndim = 2.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <omp.h>

enum { OW_CONST = 0, OW_VD_STAGGERED = 1, OW_VD_CENTRED = 2 };
enum { OW_BC_NONE = 0, OW_BC_DIRICHLET = 1, OW_BC_NEUMANN = 2 };

#define OW_RMAX 16

typedef struct {
    int32_t ndim;
    int32_t r;                  /* stencil radius: space order / 2 */
    int64_t N[3];               /* grid extents (unused axes: 1) */
    double h[3];                /* spacing per axis */
    int32_t bc[3][2];           /* per axis, (low side, high side) */
    double v[OW_RMAX + 1];      /* centred 2nd derivative: v_0 .. v_r */
    double w[OW_RMAX + 1];      /* centred 1st derivative, paper's w_j (j = 1..r) */
    double s[OW_RMAX + 1];      /* staggered 1st derivative s_j (j = 1..r) */
    double m[OW_RMAX + 1];      /* midpoint interpolation m_j (j = 1..r) */
} ow_grid;

static int64_t lin(const ow_grid *g, const int64_t k[3])
{
    return (k[0] * g->N[1] + k[1]) * g->N[2] + k[2];
}

/* Wavefield value at node k (possibly a ghost node). */
static double pval(const ow_grid *g, const double *p, const int64_t k[3])
{
    int64_t q[3];
    double sign = 1.0;
    for (int i = 0; i < 3; ++i) {
        int64_t x = k[i];
        if (x < 0) {
            int bc = g->bc[i][0];
            if (bc == OW_BC_NONE) return 0.0;
            if (bc == OW_BC_DIRICHLET) sign = -sign;
            x = -x;
        } else if (x >= g->N[i]) {
            int bc = g->bc[i][1];
            if (bc == OW_BC_NONE) return 0.0;
            if (bc == OW_BC_DIRICHLET) sign = -sign;
            x = 2 * (g->N[i] - 1) - x;
        }
        q[i] = x;
    }
    return sign * p[lin(g, q)];
}

/* Model value at node k: the even mirror about the boundary node on a side
 * with a Dirichlet or Neumann condition, the nearest grid node (edge
 * replication) on a side without one. */
static double mval(const ow_grid *g, const double *a, const int64_t k[3])
{
    int64_t q[3];
    for (int i = 0; i < 3; ++i) {
        int64_t x = k[i];
        if (x < 0) x = (g->bc[i][0] != OW_BC_NONE) ? -x : 0;
        if (x >= g->N[i]) x = (g->bc[i][1] != OW_BC_NONE) ? 2 * (g->N[i] - 1) - x : g->N[i] - 1;
        /* a mirror reaching past the far side (fewer nodes than the stencil
         * reach) falls back to the nearest node */
        if (x < 0) x = 0;
        if (x >= g->N[i]) x = g->N[i] - 1;
        q[i] = x;
    }
    return a[lin(g, q)];
}

/* Value of p at k shifted by d along axis i. */
static double p_at(const ow_grid *g, const double *p, const int64_t k[3], int i, int64_t d)
{
    int64_t q[3] = {k[0], k[1], k[2]};
    q[i] += d;
    return pval(g, p, q);
}

static double m_at(const ow_grid *g, const double *a, const int64_t k[3], int i, int64_t d)
{
    int64_t q[3] = {k[0], k[1], k[2]};
    q[i] += d;
    return mval(g, a, q);
}

/* Centred second derivative along axis i at node k. */
static double d2(const ow_grid *g, const double *p, const int64_t k[3], int i)
{
    double t = g->v[0] * p_at(g, p, k, i, 0);
    for (int j = 1; j <= g->r; ++j)
        t += g->v[j] * (p_at(g, p, k, i, j) + p_at(g, p, k, i, -j));
    return t / (g->h[i] * g->h[i]);
}

/* Centred first derivative along axis i at node k; f is a wavefield (ghost
 * rule) when is_model == 0, a model field (model ghost rule) otherwise. */
static double d1(const ow_grid *g, const double *f, const int64_t k[3], int i, int is_model)
{
    double t = 0.0;
    for (int j = 1; j <= g->r; ++j) {
        double fp = is_model ? m_at(g, f, k, i, j) : p_at(g, f, k, i, j);
        double fm = is_model ? m_at(g, f, k, i, -j) : p_at(g, f, k, i, -j);
        t += g->w[j] * (fp - fm);
    }
    return t / (2.0 * g->h[i]);
}

/* Staggered flux b_{m+1/2} (D+ p)_{m+1/2} along axis i, for the face between
 * node m and node m+1 (m is the axis-i index; other indices from k). */
static double face_flux(const ow_grid *g, const double *p, const double *b,
                        const int64_t k[3], int i, int64_t m)
{
    int64_t base[3] = {k[0], k[1], k[2]};
    base[i] = m;
    double bf = 0.0, dp = 0.0;
    for (int l = 1; l <= g->r; ++l) {
        bf += g->m[l] * (m_at(g, b, base, i, l) + m_at(g, b, base, i, 1 - l));
        dp += g->s[l] * (p_at(g, p, base, i, l) - p_at(g, p, base, i, 1 - l));
    }
    return bf * dp / g->h[i];
}

/* (L p) at node k for the chosen operator.  aux is b = 1/rho (staggered) or
 * rho (centred variable density); unused for constant density. */
static double apply_L(const ow_grid *g, int scheme, const double *p, const double *aux,
                      const int64_t k[3])
{
    double acc = 0.0;
    if (scheme == OW_VD_STAGGERED) {
        for (int i = 0; i < g->ndim; ++i) {
            double t = 0.0;
            for (int j = 1; j <= g->r; ++j)
                t += g->s[j] * (face_flux(g, p, aux, k, i, k[i] + j - 1) -
                                face_flux(g, p, aux, k, i, k[i] - j));
            acc += t / g->h[i];
        }
        return acc;
    }
    for (int i = 0; i < g->ndim; ++i) acc += d2(g, p, k, i);
    if (scheme == OW_VD_CENTRED) {
        double rho = mval(g, aux, k);
        for (int i = 0; i < g->ndim; ++i)
            acc -= (d1(g, aux, k, i, 1) / rho) * d1(g, p, k, i, 0);
    }
    return acc;
}

static void unlin(const ow_grid *g, int64_t idx, int64_t k[3])
{
    k[2] = idx % g->N[2];
    idx /= g->N[2];
    k[1] = idx % g->N[1];
    k[0] = idx / g->N[1];
}

static int64_t nnodes(const ow_grid *g) { return g->N[0] * g->N[1] * g->N[2]; }

/* out = L p over the whole grid. */
void ow_apply_L(const ow_grid *g, int32_t scheme, const double *p, const double *aux, double *out)
{
    const int64_t n = nnodes(g);
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < n; ++idx) {
        int64_t k[3];
        unlin(g, idx, k);
        out[idx] = apply_L(g, scheme, p, aux, k);
    }
}

/* Whether node k lies on a side held at zero by a Dirichlet condition. */
static int on_dirichlet_side(const ow_grid *g, const int64_t k[3])
{
    for (int i = 0; i < g->ndim; ++i) {
        if (k[i] == 0 && g->bc[i][0] == OW_BC_DIRICHLET) return 1;
        if (k[i] == g->N[i] - 1 && g->bc[i][1] == OW_BC_DIRICHLET) return 1;
    }
    return 0;
}

/* The updated value p^{n+1} at node idx from p^n (p) and p^{n-1} (prev). */
static double update_at(const ow_grid *g, int32_t scheme, const double *p, const double *prev,
                        const double *K, const double *A, const double *B, const double *aux,
                        int64_t idx, double *lap)
{
    int64_t k[3];
    unlin(g, idx, k);
    double Lp = apply_L(g, scheme, p, aux, k);
    if (lap) *lap = Lp;
    double next = A[idx] * (2.0 * p[idx] + K[idx] * Lp) - B[idx] * prev[idx];
    if (on_dirichlet_side(g, k)) next = 0.0;
    return next;
}

/* One leapfrog step.  p holds p^n; prev holds p^{n-1} on entry and p^{n+1}
 * on return (each node reads only its own previous value, so the overwrite is
 * safe).  If lap_out is not NULL it receives (L p^n). */
void ow_step(const ow_grid *g, int32_t scheme, const double *p, double *prev,
             const double *K, const double *A, const double *B, const double *aux,
             double *lap_out)
{
    const int64_t n = nnodes(g);
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < n; ++idx) {
        double lap;
        double next = update_at(g, scheme, p, prev, K, A, B, aux, idx, &lap);
        if (lap_out) lap_out[idx] = lap;
        prev[idx] = next;
    }
}

/* The same update evaluated only at the nodes idx[0..n-1] (out[s] receives
 * p^{n+1} at idx[s]); p and prev are not modified. */
void ow_step_points(const ow_grid *g, int32_t scheme, const double *p, const double *prev,
                    const double *K, const double *A, const double *B, const double *aux,
                    const int64_t *idx, int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s)
        out[s] = update_at(g, scheme, p, prev, K, A, B, aux, idx[s], 0);
}

/* Threads the parallel loops above run with (for timing reports). */
int32_t ow_threads(void) { return (int32_t)omp_get_max_threads(); }
