// vrt_cullwalk.h -- exact integer culling walk with hierarchical empty-space skipping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vrt {

// floor(n / m) for m > 0 (exact; binary64 estimate corrected in integers)
__host__ __device__ inline long long walk_floor_div(long long n, long long m) {
    long long q = (long long)floor((double)n / (double)m);
    while (q * m > n) --q;
    while ((q + 1) * m <= n) ++q;
    return q;
}

// Counts the blocking voxels met by the open segment from the centre of voxel
// (x, y, z) to the eye E (both in 1/256 voxel), stopping at `limit`.
//
// The walk is the exact integer grid walk of Section 3.2's culling rays: with
// c the start, D = E - c, and g_a the distance from c to the next voxel
// boundary ahead on axis a, the next crossing is the axis minimizing
// g_a / |D_a| (compared as g_a |D_b| < g_b |D_a|); tied axes step together, so
// voxels met only along an edge or at a corner are not visited.  It stops at
// the grid boundary, at the eye, or once it is past the bounding box of all
// blocking voxels.
//
// Cells of S^3 voxels (S = 64, then 8) that hold no blocking voxel are crossed
// in one jump: the exit time t = gb_m / |D_m| is the first crossing of the
// cell's far faces; on the exit axes the walk enters the next cell, on every
// other axis a it enters the voxel containing c_a + t D_a, half-open in the
// direction of travel:
//   D_a > 0: floor((c_a |D_m| + gb_m D_a) / (Q |D_m|)),
//   D_a < 0: floor((c_a |D_m| + gb_m D_a - 1) / (Q |D_m|)),
// which is the voxel the unskipped walk occupies right after t.  Skipped voxels
// hold no blocker, so the count is unchanged.
//
// Cells: `cells` provides
//   bool super_empty(x, y, z)  -- the 64^3 cell holding voxel (x,y,z) has no blocker
//   bool brick_empty(x, y, z)  -- the 8^3 brick holding voxel (x,y,z) has no blocker
//   bool blocking(x, y, z)     -- the voxel blocks (only asked in non-empty bricks)
template <class Cells>
__host__ __device__ inline int culling_walk(const int *G, int x, int y, int z, const long long *E, int limit,
                                            const int *bbox, const Cells &cells) {
    constexpr long long Q = 256;
    long long c[3], adel[3], g[3];
    int step[3], cur[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
        c[a] = (long long)cur[a] * Q + Q / 2;
        long long dl = E[a] - c[a];
        step[a] = dl > 0 ? 1 : (dl < 0 ? -1 : 0);
        adel[a] = dl < 0 ? -dl : dl;
        g[a] = Q / 2;
    }
    int n = 0;
    for (;;) {
        bool gone = false;  // past the blocking box for good
        for (int a = 0; a < 3; ++a) {
            if (step[a] > 0 && cur[a] > bbox[3 + a]) gone = true;
            if (step[a] < 0 && cur[a] < bbox[a]) gone = true;
            if (step[a] == 0 && (cur[a] < bbox[a] || cur[a] > bbox[3 + a])) gone = true;
        }
        if (gone) break;
        int S = 1;
        if (cells.super_empty(cur[0], cur[1], cur[2])) S = 64;
        else if (cells.brick_empty(cur[0], cur[1], cur[2])) S = 8;
        if (S == 1) {
            int m = -1;
            for (int a = 0; a < 3; ++a) {
                if (step[a] == 0) continue;
                if (m < 0 || g[a] * adel[m] < g[m] * adel[a]) m = a;
            }
            if (m < 0 || !(g[m] < adel[m])) break;  // eye reached
            const long long gm = g[m], am = adel[m];
            bool out = false;
            for (int a = 0; a < 3; ++a) {
                if (step[a] != 0 && g[a] * am == gm * adel[a]) {
                    cur[a] += step[a];
                    g[a] += Q;
                    if (cur[a] < 0 || cur[a] >= G[a]) out = true;
                }
            }
            if (out) break;
        } else {
            long long gb[3];
            int m = -1;
            for (int a = 0; a < 3; ++a) {
                gb[a] = 0;
                if (step[a] == 0) continue;
                const long long cell = cur[a] / S;  // cur >= 0
                const long long bnd = (step[a] > 0 ? cell + 1 : cell) * S * Q;
                gb[a] = step[a] > 0 ? bnd - c[a] : c[a] - bnd;
                if (m < 0 || gb[a] * adel[m] < gb[m] * adel[a]) m = a;
            }
            if (m < 0 || !(gb[m] < adel[m])) break;  // the eye lies inside this empty cell
            const long long gm = gb[m], am = adel[m];
            bool out = false;
            int nxt[3];
            for (int a = 0; a < 3; ++a) {
                nxt[a] = cur[a];
                if (step[a] == 0) continue;
                if (gb[a] * am == gm * adel[a]) {
                    const int cell = cur[a] / S;
                    nxt[a] = step[a] > 0 ? (cell + 1) * S : cell * S - 1;
                    if (nxt[a] < 0 || nxt[a] >= G[a]) out = true;
                } else {
                    const long long num = c[a] * am + (long long)step[a] * gm * adel[a];
                    nxt[a] = (int)walk_floor_div(step[a] > 0 ? num : num - 1, Q * am);
                    if (nxt[a] < 0 || nxt[a] >= G[a]) out = true;  // left the grid inside a 64^3 cell
                }
            }
            if (out) break;
            for (int a = 0; a < 3; ++a) {
                cur[a] = nxt[a];
                if (step[a] == 0) continue;
                const long long bnd = (step[a] > 0 ? (long long)cur[a] + 1 : (long long)cur[a]) * Q;
                g[a] = step[a] > 0 ? bnd - c[a] : c[a] - bnd;
            }
        }
        if (!cells.brick_empty(cur[0], cur[1], cur[2]) && cells.blocking(cur[0], cur[1], cur[2])) {
            if (++n >= limit) break;
        }
    }
    return n;
}

}  // namespace vrt
