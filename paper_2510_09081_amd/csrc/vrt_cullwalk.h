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

// Element k (0..2) of a three-vector held in registers (no indexed memory).
template <class T>
__host__ __device__ inline T wpick(const T (&v)[3], int k) {
    return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]);
}

// Product of two non-negative values below 2^32 (one 32x32->64 multiply).
__host__ __device__ inline long long wmul(long long a, long long b) {
    return (long long)((unsigned long long)(uint32_t)a * (unsigned long long)(uint32_t)b);
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
// Magnitudes: positions below 2^18 (1024 voxels), |D| below 2^23 (the eye
// within 2^22 of the grid corner), so every g and |D| fits 32 bits and every
// product fits 64.  Three-vectors are only indexed by loop constants or
// through wpick, so they stay in registers.
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
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c[a] = (long long)cur[a] * Q + Q / 2;
        const long long dl = E[a] - c[a];
        step[a] = dl > 0 ? 1 : (dl < 0 ? -1 : 0);
        adel[a] = dl < 0 ? -dl : dl;
        g[a] = Q / 2;
    }
    int n = 0;
    bool be = cells.brick_empty(x, y, z);  // brick_empty of the current voxel
    for (;;) {
        bool gone = false;  // past the blocking box for good
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (step[a] > 0 && cur[a] > bbox[3 + a]) gone = true;
            if (step[a] < 0 && cur[a] < bbox[a]) gone = true;
            if (step[a] == 0 && (cur[a] < bbox[a] || cur[a] > bbox[3 + a])) gone = true;
        }
        if (gone) break;
        int S = 1;
        if (be) S = cells.super_empty(cur[0], cur[1], cur[2]) ? 64 : 8;
        if (S == 1) {
            int m = -1;
            long long gm = 0, am = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (step[a] == 0) continue;
                if (m < 0 || wmul(g[a], am) < wmul(gm, adel[a])) {
                    m = a;
                    gm = g[a];
                    am = adel[a];
                }
            }
            if (m < 0 || !(gm < am)) break;  // eye reached
            bool out = false;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (step[a] != 0 && wmul(g[a], am) == wmul(gm, adel[a])) {
                    cur[a] += step[a];
                    g[a] += Q;
                    if (cur[a] < 0 || cur[a] >= G[a]) out = true;
                }
            }
            if (out) break;
        } else {
            long long gb[3];
            int m = -1;
            long long gm = 0, am = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                gb[a] = 0;
                if (step[a] == 0) continue;
                const long long cell = cur[a] / S;  // cur >= 0
                const long long bnd = (step[a] > 0 ? cell + 1 : cell) * S * Q;
                gb[a] = step[a] > 0 ? bnd - c[a] : c[a] - bnd;
                if (m < 0 || wmul(gb[a], am) < wmul(gm, adel[a])) {
                    m = a;
                    gm = gb[a];
                    am = adel[a];
                }
            }
            if (m < 0 || !(gm < am)) break;  // the eye lies inside this empty cell
            bool out = false;
            int nxt[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                nxt[a] = cur[a];
                if (step[a] == 0) continue;
                if (wmul(gb[a], am) == wmul(gm, adel[a])) {
                    const int cell = cur[a] / S;
                    nxt[a] = step[a] > 0 ? (cell + 1) * S : cell * S - 1;
                    if (nxt[a] < 0 || nxt[a] >= G[a]) out = true;
                } else {
                    const long long num = wmul(c[a], am) + (long long)step[a] * wmul(gm, adel[a]);
                    nxt[a] = (int)walk_floor_div(step[a] > 0 ? num : num - 1, Q * am);
                    if (nxt[a] < 0 || nxt[a] >= G[a]) out = true;  // left the grid inside a 64^3 cell
                }
            }
            if (out) break;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                cur[a] = nxt[a];
                if (step[a] == 0) continue;
                const long long bnd = (step[a] > 0 ? (long long)cur[a] + 1 : (long long)cur[a]) * Q;
                g[a] = step[a] > 0 ? bnd - c[a] : c[a] - bnd;
            }
        }
        be = cells.brick_empty(cur[0], cur[1], cur[2]);
        if (!be && cells.blocking(cur[0], cur[1], cur[2])) {
            if (++n >= limit) break;
        }
    }
    return n;
}

}  // namespace vrt
