// Mirror ghosts of every mirrored side in one launch (the image method of the
// free surface: a ghost node at distance k outside the boundary node takes
// sign * p at distance k inside it, odd for Dirichlet, even for Neumann).
// The three axes are independent: each reads only nodes inside the grid along
// its own axis and writes only its own ghosts, over the grid's extent along
// the other two (corner ghosts are never read, every operator being
// axis-aligned).  Items of the z and x axes run along y across the lanes
// (contiguous rows); items of the y axis, the contiguous one, take the ghost
// layer fastest, so a row's ghost run is written by neighbouring lanes.
#pragma once

#include "device.h"

namespace sw {

struct GhostSides {
    int lo[3], hi[3];           // per axis: 0 none, 1 Dirichlet (odd), 2 Neumann (even)
    int64_t items[3];           // items per axis (0 if the axis has no mirrored side)
};

inline GhostSides ghost_sides(const Geom &g, const int (*bcm)[2], int depth)
{
    const int n[3] = {g.Z, g.X, g.Y};
    GhostSides s{};
    for (int a = 0; a < 3; ++a) {
        s.lo[a] = bcm[a][0];
        s.hi[a] = bcm[a][1];
        const int a1 = a == 0 ? 1 : 0, a2 = a == 2 ? 1 : 2;
        s.items[a] = (bcm[a][0] || bcm[a][1]) ? int64_t(n[a1]) * n[a2] * depth * 2 : 0;
    }
    return s;
}

template <typename T>
__global__ void k_ghost_all(Geom g, GhostSides sd, int depth, T *__restrict__ f)
{
    const int n[3] = {g.Z, g.X, g.Y};
    const int64_t total = sd.items[0] + sd.items[1] + sd.items[2];
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        int axis = 0;
        int64_t j = i;
        if (j >= sd.items[0]) {
            j -= sd.items[0];
            axis = 1;
            if (j >= sd.items[1]) {
                j -= sd.items[1];
                axis = 2;
            }
        }
        const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
        const int64_t rows = int64_t(n[a1]) * n[a2];
        int64_t r;
        int k, side;
        if (axis < 2) {                         // row fastest
            r = j % rows;
            k = 1 + int((j / rows) % depth);
            side = int(j / (rows * depth));
        } else {                                // ghost layer fastest, then side
            k = 1 + int(j % depth);
            side = int((j / depth) % 2);
            r = j / (2 * int64_t(depth));
        }
        const int bc = side ? sd.hi[axis] : sd.lo[axis];
        if (bc == 0) continue;
        int src[3] = {0, 0, 0}, dst[3] = {0, 0, 0};
        src[a1] = dst[a1] = int(r / n[a2]);
        src[a2] = dst[a2] = int(r % n[a2]);
        if (side == 0) {
            dst[axis] = -k;
            src[axis] = k;
        } else {
            dst[axis] = n[axis] - 1 + k;
            src[axis] = n[axis] - 1 - k;
        }
        if (src[axis] < 0 || src[axis] >= n[axis]) continue;   // extent below the ghost depth
        const T v = f[elem(g, src[0], src[1], src[2])];
        f[elem(g, dst[0], dst[1], dst[2])] = bc == 1 ? -v : v;
    }
}

}  // namespace sw
