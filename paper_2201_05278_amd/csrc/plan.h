// Internal host-side plan of the propagator: layout, coefficients, damping
// table and point (source/receiver) tables.  Not part of the C ABI.
#pragma once

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/simwave_hip.h"

namespace sw {

constexpr int kMaxRadius = 10;     // space order 20
constexpr int kRowAlign = 64;      // floats: interior rows start on 256-byte boundaries

// Per-thread error message for sw_last_error().
void set_error(const std::string &msg);
sw_status fail(sw_status s, const std::string &msg);

// A point table flattened into entries (one per non-zero weight).
struct PointSet {
    int count = 0;
    int interp = SW_INTERP_HICKS;
    int radius = 4;
    double kaiser_b = 0.0;
    std::vector<double> coords;          // count * ndim, metres
    // entries, grouped by point (CSR by point)
    std::vector<int32_t> ptr;            // count + 1
    std::vector<int64_t> node;           // padded-layout element offset
    std::vector<int32_t> pid;            // point the entry belongs to
    std::vector<int32_t> d2;             // squared layer distance of the node (damping index)
    std::vector<int64_t> phys;           // physical-grid index the node copies its model from
    std::vector<float> weight;           // interpolation weight
    std::vector<double> weight64;        // the same weight in double precision (SW_F64 plans)
    // the same entries grouped by unique node (CSR by node, deterministic gather)
    std::vector<int64_t> unode;          // unique nodes
    std::vector<int32_t> uptr;           // nunique + 1
    std::vector<int32_t> uent;           // entry index, grouped by unique node
    int max_per_point = 0;
    int max_per_node = 0;
};

// Byte offsets of the device arrays inside the caller's workspace.
struct WorkspaceMap {
    size_t model_k = 0;      // float[field_elems]: K (dt^2 c^2, or dt^2 rho c^2)
    size_t model_aux = 0;    // float[field_elems]: b = 1/rho or rho (variable density)
    size_t damp = 0;         // float2[damp_n]: (A, B) by squared layer distance
    size_t counter = 0;      // uint32: non-finite count of the optional finite check
    struct Pts {
        size_t ptr = 0, node = 0, pid = 0, d2 = 0, phys = 0, weight = 0;   // by point
        size_t unode = 0, uptr = 0, uent = 0;                     // by node
        size_t coef_a = 0;   // float[nent]: A M w (/dV for sources): injection
        size_t coef_s = 0;   // float[nent]: M w / dV: source term of stored M (L u + Q s)
        size_t wscaled = 0;  // float[nent]: w / dV (sources) or w (receivers): recording
        size_t inj = 0;      // float[2][nuniq]: injected values of the two steps of a sweep
    } src, rec;
    size_t total = 0;
};

}  // namespace sw

struct sw_plan {
    sw_problem prob{};
    int bcm[3][2] = {{0, 0}, {0, 0}, {0, 0}};   // ghost condition per internal axis (z, x, y) and side
    int ghost = 0;                  // mirror ghost layers a sweep reads (R, or 2R - 1 staggered)
    bool mirror = false;            // any side with a Dirichlet or Neumann condition
    int ndim = 3;
    int r = 4;
    int halo = 4;
    // internal 3D view: 2D grids are (Z, 1, X)
    int dims[3] = {1, 1, 1};       // extended grid
    int nphys[3] = {1, 1, 1};      // physical grid
    int lo[3] = {0, 0, 0};         // layer width on the low side
    int hz = 0, hx = 0;            // stored halo along z and x (x: 0 in 2D)
    int pad[3] = {1, 1, 1};        // padded extents (z, x, pitch)
    int64_t origin = 0;
    int64_t field_elems = 0;
    int64_t grid_nodes = 0;
    int64_t phys_nodes = 0;
    double hh[3] = {1, 1, 1};      // spacing in the internal axis order
    double dV = 1.0;
    // coefficients (double, exact closed forms / solved systems)
    double v2[sw::kMaxRadius + 1] = {};   // centred second derivative
    double w1[sw::kMaxRadius + 1] = {};   // centred first derivative (1/dx prefactor)
    double sg[sw::kMaxRadius + 1] = {};   // staggered first derivative
    double mp[sw::kMaxRadius + 1] = {};   // midpoint interpolation
    // damping table (A, B) by squared layer distance
    std::vector<float> damp;      // 2 * damp_n
    std::vector<double> damp64;   // the same (A, B) pairs in double precision
    int damp_n = 1;
    sw::PointSet src, rec;
    sw::WorkspaceMap ws;
    bool prepared = false;
    void *prepared_ws = nullptr;
    // stencil tiling chosen by sw_plan_set_tiling / sw_plan_autotune (tx == 0: default)
    int tile_tx = 0, tile_nw = 0, tile_zc = 0, tile_nt = -1, tile_pf = 0, tile_wt = 0, tile_ts = 0,
        tile_occ = -1, tile_order = 0;
    // bumped by every call that changes what a captured launch bakes in
    // (point tables and counts, model, tiling); part of the graph keys
    uint64_t generation = 1;
    // resident blocks per CU of the constant-density block-tile kernels, by
    // tiling key (queried once per kernel), and the device's CU count
    mutable std::vector<std::pair<uint64_t, int>> resident_cache;
    mutable int ncu = 0;
    // cached HIP graph of a forward run, captured on a private stream
    void *graph_exec = nullptr;
    void *capture_stream = nullptr;
    std::vector<uint64_t> graph_key;
};

namespace sw {
sw_status build_layout(sw_plan *p);
void build_workspace_map(sw_plan *p);
// source: true for the source table (images across mirrored sides), false
// for receivers (ghost reads across mirrored sides).
sw_status build_points(sw_plan *p, PointSet &ps, int count, const double *coords, int interp,
                       int radius, double kaiser_b, bool source);
double a1d(int space_order);
}  // namespace sw
