// vrt_cullwalk.h -- exact integer culling walk with hierarchical empty-space skipping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vrt {

// Within a brick: index of the 2^3 cell holding voxel (x, y, z), and the mask
// of the eight 2^3 cells of its 4^3 cell, in a brick's 64-bit mask of
// 2^3 cells (bit 16 Z + 4 Y + X for cell (X, Y, Z), 0 <= X, Y, Z < 4).
__host__ __device__ inline int walk_cell2(int x, int y, int z) {
    return (((z & 7) >> 1) << 4) | (((y & 7) >> 1) << 2) | ((x & 7) >> 1);
}
__host__ __device__ inline uint64_t walk_cell4_mask(int x, int y, int z) {
    return 0x00330033ull << ((((z & 7) >> 2) << 5) | (((y & 7) >> 2) << 3) | (((x & 7) >> 2) << 1));
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
// Cells of S^3 voxels that hold no blocking voxel are crossed in one jump (S =
// 64, 32, 16 or 8 in bricks without a blocker, else 4 or 2 from the brick's
// mask of 2^3 cells): with Te the smallest time at which the walk crosses the cell's
// far face on some axis, every moving axis a makes all its crossings with
// T <= Te, n_a = floor((Te - T_a) / dT_a) + 1 of them (none if Te < T_a);
// on the exit axes that is exactly into the next cell, and crossings tied
// with Te are taken together as in the voxel walk.  Skipped voxels hold no
// blocker, so the count is unchanged.
//
// Cells: `cells` provides
//   bool brick_empty(x, y, z)  -- the 8^3 brick holding voxel (x,y,z) has no blocker
//   int empty_shift(x, y, z)   -- log2 of the largest of the 64^3, 32^3 and 16^3
//                                 cells and the brick holding it with no blocker
//                                 (only asked in empty bricks)
//   uint64_t sub_mask(x, y, z) -- the 2^3 cells of that brick holding a blocker
//                                 (only asked in non-empty bricks)
//   uint64_t slice_bits(x, y, z) -- the blocking voxels of the brick's z-slice holding
//                                 voxel (x, y, z), bit 8 (y mod 8) + (x mod 8)
//                                 (only asked in non-empty bricks)
//
// State of one culling walk between steps (everything in registers).
struct CullWalk {
    int cur[3], step[3], lim[3];
    long long T[3], dT[3], P;
    float rdT[3];  // 1 / dT in binary32 (0 on a still axis): the estimate of a jump's crossing counts
    uint64_t m2;  // sub_mask of the brick with key k2
    int k2;       // packed brick coordinates of m2, or -1
    int n;        // blocking voxels met so far
    bool be;      // the current voxel's brick holds no blocker
    bool done;    // n is the result
};

// Brick key of voxel (x, y, z): brick coordinates below 2^10 each.
__host__ __device__ inline int walk_brick_key(int x, int y, int z) {
    return ((z >> 3) << 20) | ((y >> 3) << 10) | (x >> 3);
}

// The brick flag of the current voxel, the 2^3-cell mask of its brick when
// that holds a blocker, and whether the current voxel blocks.  In a brick
// with a blocker the voxel's blocking bits (its z-slice of the brick) are
// read together with the brick's mask when that is new, so the two reads
// overlap instead of waiting one after the other.
template <class Cells>
__host__ __device__ inline bool walk_enter(CullWalk &w, const Cells &cells) {
    w.be = cells.brick_empty(w.cur[0], w.cur[1], w.cur[2]);
    if (w.be) return false;
    const uint64_t slice = cells.slice_bits(w.cur[0], w.cur[1], w.cur[2]);
    const int key = walk_brick_key(w.cur[0], w.cur[1], w.cur[2]);
    if (key != w.k2) {
        w.m2 = cells.sub_mask(w.cur[0], w.cur[1], w.cur[2]);
        w.k2 = key;
    }
    const bool cell = (w.m2 >> walk_cell2(w.cur[0], w.cur[1], w.cur[2])) & 1ull;
    return cell && ((slice >> (((w.cur[1] & 7) << 3) | (w.cur[0] & 7))) & 1ull);
}

// Sets up the walk from voxel (x, y, z); done at once when the eye is at the
// voxel's centre or no blocking voxel can lie ahead.
template <class Cells>
__host__ __device__ inline void walk_begin(CullWalk &w, const int *G, int x, int y, int z, const long long *E,
                                           const int *bbox, const Cells &cells) {
    constexpr long long Q = 256;
    constexpr long long kNever = 0x7FFFFFFFFFFFFFFFll;
    constexpr long long kStill = kNever - 64;
    long long adel[3];
    w.cur[0] = x;
    w.cur[1] = y;
    w.cur[2] = z;
    w.n = 0;
    w.done = false;
    int nmov = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long c = (long long)w.cur[a] * Q + Q / 2;
        const long long dl = E[a] - c;
        w.step[a] = dl > 0 ? 1 : (dl < 0 ? -1 : 0);
        adel[a] = dl < 0 ? -dl : dl;
        nmov += w.step[a] != 0;
    }
    w.P = kNever;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        long long L = 1;
#pragma unroll
        for (int b = 0; b < 3; ++b)
            if (b != a && w.step[b] != 0) L *= adel[b];
        // a still axis never crosses: its crossing time stays above every reachable one
        // (kStill + dT * 63 < kNever) and its crossing count at zero
        w.T[a] = w.step[a] != 0 ? (Q / 2) * L : kStill;
        w.dT[a] = w.step[a] != 0 ? Q * L : 1;
        w.rdT[a] = w.step[a] != 0 ? 1.0f / (float)(Q * L) : 0.0f;
        // the product fits in int64 when its binary32 estimate (relative error below 2^-22) is below 9e18
        if (w.step[a] != 0 && (float)adel[a] * (float)L < 9.0e18f) w.P = adel[a] * L;
    }
    // The walk is monotone on every axis, so it can stop as soon as it leaves
    // the grid or the box of blocking voxels: lim[a] is the last coordinate
    // worth visiting in the direction of travel.
    bool none = nmov == 0;  // the eye is at this voxel's centre
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int st = w.step[a];
        if (st == 0 && (w.cur[a] < bbox[a] || w.cur[a] > bbox[3 + a])) none = true;
        w.lim[a] = st > 0 ? (G[a] - 1 < bbox[3 + a] ? G[a] - 1 : bbox[3 + a]) : (bbox[a] > 0 ? bbox[a] : 0);
        if ((st > 0 && w.cur[a] > w.lim[a]) || (st < 0 && w.cur[a] < w.lim[a])) none = true;
    }
    w.done = none;
    w.k2 = -1;
    w.m2 = 0;
    w.be = true;
    if (!none) walk_enter(w, cells);
}

// q = floor(num / den) for 0 <= num < 64 den (den > 0, 65 den < 2^63), from
// the binary32 estimate num * rden (rden = 1 / den rounded) corrected by one
// multiply and compare each way: the estimate's relative error is below
// 2^-20, so with q < 64 it is off by at most one.  Also returns q * den in `qd`.
__host__ __device__ inline int walk_small_quot_est(long long num, long long den, float rden, long long &qd) {
    // num in binary32 from its two 32-bit halves (relative error below 2^-22)
    const float fn = fmaf((float)(uint32_t)((unsigned long long)num >> 32), 4294967296.0f, (float)(uint32_t)num);
    int q = (int)(fn * rden);
    q = q < 0 ? 0 : (q > 63 ? 63 : q);
    long long p = den * q;
    const bool over = p > num;
    q -= over ? 1 : 0;
    p -= over ? den : 0;
    const bool under = p + den <= num;
    q += under ? 1 : 0;
    p += under ? den : 0;
    qd = p;
    return q;
}

// One step of the walk: the cell of S^3 voxels holding the current voxel is
// crossed (S = 1 for a voxel, larger for a cell without a blocker), then the
// blocking test of the voxel entered.  A voxel is the cell with S = 1: every
// axis whose next crossing ties the smallest steps once, the others not at
// all, as in the voxel walk; one code path serves both, so the lanes of a
// wave that step voxels and those that jump cells run it together.  Sets done
// when the walk ends.
template <class Cells>
__host__ __device__ inline void walk_step(CullWalk &w, int limit, const Cells &cells) {
    int sh = 0;  // the cell crossed has S = 2^sh voxels a side
    if (w.be) {
        sh = cells.empty_shift(w.cur[0], w.cur[1], w.cur[2]);
    } else if (!((w.m2 >> walk_cell2(w.cur[0], w.cur[1], w.cur[2])) & 1ull)) {
        sh = (w.m2 & walk_cell4_mask(w.cur[0], w.cur[1], w.cur[2])) ? 1 : 2;
    }
    long long Tc[3];
    const int s1 = (1 << sh) - 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {  // crossings to the cell's far face on axis a (cur >= 0)
        const int low = w.cur[a] & s1;
        const unsigned k = (unsigned)(w.step[a] > 0 ? s1 - low : low);
        Tc[a] = w.T[a] + (long long)((unsigned long long)w.dT[a] * k);
    }
    long long te = Tc[0] < Tc[1] ? Tc[0] : Tc[1];
    te = Tc[2] < te ? Tc[2] : te;
    if (!(te < w.P)) {  // the eye lies inside this cell (or is reached at its exit)
        w.done = true;
        return;
    }
    bool out = false;
    int na[3];
    long long nd[3];  // na * dT
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // an axis crosses when te reaches its next crossing (a still axis never: its T is above every reachable te)
        const long long num = te - w.T[a];
        const bool moves = num >= 0;
        long long qd;
        const int q = walk_small_quot_est(moves ? num : 0, w.dT[a], w.rdT[a], qd);
        na[a] = moves ? q + 1 : 0;
        nd[a] = moves ? qd + w.dT[a] : 0;
        // past the limit on this axis: step (cur + step na) > step lim
        out |= w.step[a] * (w.cur[a] + w.step[a] * na[a]) > w.step[a] * w.lim[a];
    }
    if (out) {
        w.done = true;
        return;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        w.cur[a] += w.step[a] * na[a];
        w.T[a] += nd[a];
    }
    if (walk_enter(w, cells) && ++w.n >= limit) w.done = true;
}

// The whole walk: the number of blocking voxels met, at most `limit`.
template <class Cells>
__host__ __device__ inline int culling_walk(const int *G, int x, int y, int z, const long long *E, int limit,
                                            const int *bbox, const Cells &cells) {
    CullWalk w;
    walk_begin(w, G, x, y, z, E, bbox, cells);
    while (!w.done) walk_step(w, limit, cells);
    return w.n;
}

}  // namespace vrt
