// vrt_cullwalk.h -- exact integer culling walk with hierarchical empty-space skipping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vrt {

// floor((num) / den) for 0 <= num < 64 * den (den > 0): an estimate from a
// binary32 reciprocal, corrected exactly in integers.
__host__ __device__ inline long long walk_small_quot(long long num, long long den) {
#ifdef __HIP_DEVICE_COMPILE__
    long long q = (long long)((float)num * __builtin_amdgcn_rcpf((float)den));
#else
    long long q = num / den;
#endif
    while (q > 0 && q * den > num) --q;
    while ((q + 1) * den <= num) ++q;
    return q;
}

// Counts the blocking voxels met by the open segment from the centre of voxel
// (x, y, z) to the eye E (both in 1/256 voxel), stopping at `limit`.
//
// The walk is the exact integer grid walk of Section 3.2's culling rays: with
// c the start, D = E - c, and g_a the distance from c to the next voxel
// boundary ahead on axis a, the next crossing is the axis minimizing
// g_a / |D_a|; tied axes step together, so voxels met only along an edge or at
// a corner are not visited.  It stops at the grid boundary, at the eye, or once
// it is past the bounding box of all blocking voxels.
//
// Crossing times are kept as integers T_a = g_a * L_a, where L_a is the product
// of |D_b| over the other moving axes: T_a < T_b exactly when
// g_a / |D_a| < g_b / |D_b|, crossing axis a adds dT_a = Q L_a, and the eye is
// reached once the smallest T is at least P = |D_a| L_a (the product of all
// moving |D|).  A step is then additions and comparisons only.  Magnitudes:
// |D| < 2^22.1 (the eye within 2^22 of the grid corner), g below 2^18.1
// (1024 voxels), so T < 2^62.3; P is clamped to 2^63 - 1 when larger (the eye
// then lies beyond every reachable crossing).
//
// Cells of S^3 voxels (S = 64, then 8) that hold no blocking voxel are crossed
// in one jump: with Te the smallest time at which the walk crosses the cell's
// far face on some axis, every moving axis a makes all its crossings with
// T <= Te, n_a = floor((Te - T_a) / dT_a) + 1 of them (none if Te < T_a);
// on the exit axes that is exactly into the next cell, and crossings tied
// with Te are taken together as in the voxel walk.  Skipped voxels hold no
// blocker, so the count is unchanged.
//
// Cells: `cells` provides
//   bool super_empty(x, y, z)  -- the 64^3 cell holding voxel (x,y,z) has no blocker
//   bool brick_empty(x, y, z)  -- the 8^3 brick holding voxel (x,y,z) has no blocker
//   bool blocking(x, y, z)     -- the voxel blocks (only asked in non-empty bricks)
template <class Cells>
__host__ __device__ inline int culling_walk(const int *G, int x, int y, int z, const long long *E, int limit,
                                            const int *bbox, const Cells &cells) {
    constexpr long long Q = 256;
    constexpr long long kNever = 0x7FFFFFFFFFFFFFFFll;
    long long adel[3], T[3], dT[3];
    int step[3], cur[3] = {x, y, z};
    int nmov = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long c = (long long)cur[a] * Q + Q / 2;
        const long long dl = E[a] - c;
        step[a] = dl > 0 ? 1 : (dl < 0 ? -1 : 0);
        adel[a] = dl < 0 ? -dl : dl;
        nmov += step[a] != 0;
    }
    if (nmov == 0) return 0;  // the eye is at this voxel's centre
    long long P = kNever;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        long long L = 1;
#pragma unroll
        for (int b = 0; b < 3; ++b)
            if (b != a && step[b] != 0) L *= adel[b];
        T[a] = step[a] != 0 ? (Q / 2) * L : kNever;
        dT[a] = step[a] != 0 ? Q * L : kNever;
        if (step[a] != 0 && (double)adel[a] * (double)L < 9.0e18) P = adel[a] * L;
    }
    // The walk is monotone on every axis, so it can stop as soon as it leaves
    // the grid or the box of blocking voxels: lim[a] is the last coordinate
    // worth visiting in the direction of travel.
    int lim[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (step[a] == 0 && (cur[a] < bbox[a] || cur[a] > bbox[3 + a])) return 0;
        lim[a] = step[a] > 0 ? (G[a] - 1 < bbox[3 + a] ? G[a] - 1 : bbox[3 + a]) : (bbox[a] > 0 ? bbox[a] : 0);
        if ((step[a] > 0 && cur[a] > lim[a]) || (step[a] < 0 && cur[a] < lim[a])) return 0;
    }
    int n = 0;
    bool be = cells.brick_empty(x, y, z);  // brick_empty of the current voxel
    for (;;) {
        int S = 1;
        if (be) S = cells.super_empty(cur[0], cur[1], cur[2]) ? 64 : 8;
        if (S == 1) {
            long long tm = T[0] < T[1] ? T[0] : T[1];
            tm = T[2] < tm ? T[2] : tm;
            if (!(tm < P)) break;  // eye reached
            bool out = false;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (T[a] == tm) {
                    cur[a] += step[a];
                    T[a] += dT[a];
                    if (step[a] > 0 ? cur[a] > lim[a] : cur[a] < lim[a]) out = true;
                }
            }
            if (out) break;
        } else {
            long long Tc[3];
            const int sh = S == 64 ? 6 : 3;  // S = 2^sh
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                Tc[a] = kNever;
                if (step[a] == 0) continue;
                const int cs = (cur[a] >> sh) << sh;  // cur >= 0
                const unsigned k = (unsigned)(step[a] > 0 ? cs + S - 1 - cur[a] : cur[a] - cs);
                Tc[a] = T[a] + (long long)((unsigned long long)dT[a] * k);
            }
            long long te = Tc[0] < Tc[1] ? Tc[0] : Tc[1];
            te = Tc[2] < te ? Tc[2] : te;
            if (!(te < P)) break;  // the eye lies inside this empty cell
            bool out = false;
            long long na[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                na[a] = 0;
                if (step[a] == 0 || te < T[a]) continue;
                na[a] = walk_small_quot(te - T[a], dT[a]) + 1;
                const long long nx = cur[a] + step[a] * na[a];
                if (step[a] > 0 ? nx > lim[a] : nx < lim[a]) out = true;
            }
            if (out) break;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                cur[a] += step[a] * (int)na[a];
                if (na[a]) T[a] += (long long)((unsigned long long)dT[a] * (unsigned)na[a]);
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
