// vrt_cull.hip -- Section 3.2 (erosion, culling rays, culling pyramid) and
// Section 3.3 (scan of visible counts, voxelization pass 2 into the lists).
#include <climits>

#include "vrt_cullwalk.h"
#include "vrt_internal.h"

namespace vrt {
namespace {

__device__ __forceinline__ void b_cull_reset(uint8_t *__restrict__ vis3, int64_t nb, uint8_t *__restrict__ vis_hi,
                                             int64_t n_hi, DevStatus *__restrict__ st, unsigned bid_, unsigned nblk_) {
    int64_t i = (int64_t)bid_ * blockDim.x + threadIdx.x;
    if (i < nb) vis3[i] = 0;
    if (i < n_hi) vis_hi[i] = 0;
    if (i == 0) st->n_listed = 0;
    if (i < kStripes) {
        int *p = st->stripe[i].vbox;
        p[0] = p[1] = p[2] = INT_MAX;
        p[3] = p[4] = p[5] = INT_MIN;
        st->stripe[i].vvis = 0;
    }
}

__global__ void k_cull_reset(uint8_t *__restrict__ vis3, int64_t nb, uint8_t *__restrict__ vis_hi, int64_t n_hi,
                             DevStatus *__restrict__ st) {
    b_cull_reset(vis3, nb, vis_hi, n_hi, st, blockIdx.x, gridDim.x);
}

// Blocking flags the culling walk reads: one byte per 64^3 and 32^3 cell, one
// bit per 16^3 cell and brick, and per brick holding a blocker one bit per
// voxel (64 voxels per word) and one per 2^3 cell.
struct CullCells {
    const uint8_t *super_blk, *c32_blk;
    const uint32_t *brick_bits, *c16_bits;
    const uint64_t *blk_bits;
    int nb0, nb1, ns0, ns1;
    int n16x, n16y, n32x, n32y;
    // indices below 2^24 (at most 128^3 bricks): 24-bit multiplies
    __device__ unsigned brick_of(int x, int y, int z) const {
        return __umul24(__umul24((unsigned)(z >> 3), (unsigned)nb1) + (unsigned)(y >> 3), (unsigned)nb0) +
               (unsigned)(x >> 3);
    }
    // log2 of the largest of the 64^3, 32^3, 16^3 cells and the brick holding
    // voxel (x, y, z) with no blocker, the brick being empty
    __device__ int empty_shift(int x, int y, int z) const {
        const bool e64 = !super_blk[__umul24(__umul24((unsigned)(z >> 6), (unsigned)ns1) + (unsigned)(y >> 6),
                                             (unsigned)ns0) + (unsigned)(x >> 6)];
        const unsigned c32 = __umul24(__umul24((unsigned)(z >> 5), (unsigned)n32y) + (unsigned)(y >> 5), (unsigned)n32x) +
                             (unsigned)(x >> 5);
        const unsigned c16 = __umul24(__umul24((unsigned)(z >> 4), (unsigned)n16y) + (unsigned)(y >> 4), (unsigned)n16x) +
                             (unsigned)(x >> 4);
        const bool e32 = !c32_blk[c32];
        const bool e16 = !((c16_bits[c16 >> 5] >> (c16 & 31u)) & 1u);
        return e64 ? 6 : (e32 ? 5 : (e16 ? 4 : 3));
    }
    __device__ bool brick_empty(int x, int y, int z) const {
        const unsigned b = brick_of(x, y, z);
        return !((brick_bits[b >> 5] >> (b & 31u)) & 1u);
    }
    __device__ uint64_t sub_mask(int x, int y, int z) const { return blk_bits[brick_of(x, y, z) * 16u + 8u]; }
    __device__ uint64_t slice_bits(int x, int y, int z) const { return blk_bits[brick_of(x, y, z) * 16u + (unsigned)(z & 7)]; }
};

// Bytes of the brick and cell flags when staged in LDS.
__host__ __device__ inline size_t cull_lds_bytes(int64_t nwords, int64_t nflags) {
    return (size_t)nwords * 4 + (size_t)nflags;
}
constexpr size_t kCullLdsMax = 48 * 1024;  // larger grids read the flags from global memory

struct CullArgs {
    GridArgs g;
    long long E[3];
    int limit;  // < 0: no culling
};

// One thread per occupied voxel (Section 3.2): visible iff its culling ray
// meets fewer than `limit` blocking voxels.  Writes level-0 visibility of
// occupied voxels only; k_cull_brick completes the rest of the brick.
// With kLds the block first copies the brick bits and cell flags into LDS
// (cull_lds_bytes of dynamic shared memory), so that only the voxel bits are
// global loads inside the walk.
extern __shared__ __align__(16) uint32_t vrt_cull_lds[];

template <bool kLds>
__device__ __forceinline__ void b_cull_walk(CullArgs a, CullCells cells, const uint32_t *__restrict__ occ_list,
                                                   const DevStatus *__restrict__ st, uint8_t *__restrict__ vis0, unsigned bid_, unsigned nblk_) {
    __shared__ int bbox[6];
    if (threadIdx.x < 6) {  // combine the stripes of the blocking box
        const int k = threadIdx.x;
        int v = k < 3 ? INT_MAX : INT_MIN;
        for (int s = 0; s < kStripes; ++s) {
            const int u = st->stripe[s].bbox[k];
            v = k < 3 ? (u < v ? u : v) : (u > v ? u : v);
        }
        bbox[k] = v;
    }
    if (kLds) {
        const CellFlagLayout cl = cell_flag_layout(a.g.nb);
        const int nw = (int)cl.words, nf = (int)cl.bytes;
        for (int i = threadIdx.x; i < nw; i += blockDim.x) vrt_cull_lds[i] = cells.brick_bits[i];
        uint8_t *s_flags = reinterpret_cast<uint8_t *>(vrt_cull_lds + nw);
        for (int i = threadIdx.x; i < nf; i += blockDim.x) s_flags[i] = cells.super_blk[i];
        cells.brick_bits = vrt_cull_lds;
        cells.c16_bits = vrt_cull_lds + cl.w16;
        cells.super_blk = s_flags;
        cells.c32_blk = s_flags + cl.b32;
    }
    __syncthreads();
    const unsigned n = st->n_occ;
    for (unsigned i = bid_ * blockDim.x + threadIdx.x; i < n; i += nblk_ * blockDim.x) {
        const uint32_t v = occ_list[i];
        const int l = (int)(v & 511u);
        int bx, by, bz;
        brick_xyz(v >> 9, a.g.nb, bx, by, bz);
        const int x = bx * 8 + (l & 7), y = by * 8 + ((l >> 3) & 7), z = bz * 8 + (l >> 6);
        const int nblk = culling_walk(a.g.G, x, y, z, a.E, a.limit, bbox, cells);
        vis0[v] = nblk < a.limit ? 1 : 0;
    }
}

template <bool kLds>
__global__ void __launch_bounds__(512) k_cull_walk(CullArgs a, CullCells cells, const uint32_t *__restrict__ occ_list,
                                                   const DevStatus *__restrict__ st, uint8_t *__restrict__ vis0) { b_cull_walk<kLds>(a, cells, occ_list, st, vis0, blockIdx.x, gridDim.x); }

// One workgroup per occupied brick: final level-0 visibility (unoccupied
// voxels are invisible; without culling every occupied voxel is visible), the
// in-brick culling mips 1..3 (parent = OR of children), and the brick's
// visible-fragment total.  The coarser culling levels are ORs too: a visible
// brick sets its cell on levels 4 .. kMarkTop (cleared by the reset); the few
// cells above are left to the brick scan.
constexpr int kMarkTop = 6;  // highest culling level set brick by brick

__device__ __forceinline__ void b_cull_brick(int limit, GridArgs g, const uint32_t *__restrict__ words,
                                                    const int32_t *__restrict__ list, DevStatus *__restrict__ st,
                                                    uint8_t *__restrict__ vis0, uint8_t *__restrict__ vis1,
                                                    uint8_t *__restrict__ vis2, uint8_t *__restrict__ vis3,
                                                    uint8_t *__restrict__ vis_hi, const Level *levels, int n_levels,
                                                    uint32_t *__restrict__ brick_total, unsigned bid_, unsigned nblk_) {
    __shared__ uint8_t s0[512];
    __shared__ uint8_t s1[64];
    __shared__ uint8_t s2[8];
    __shared__ unsigned wsum[8];
    const unsigned nbk = st->n_bricks;
    const int t = threadIdx.x;
    for (unsigned sl = bid_; sl < nbk; sl += nblk_) {
        int64_t b = list[sl];
        unsigned cnt = words[b * kBrickVox + t] & 0xFFFFu;
        uint8_t v = 0;
        if (cnt) v = limit < 0 ? 1 : vis0[b * kBrickVox + t];
        vis0[b * kBrickVox + t] = v;
        s0[t] = v;
        unsigned c = v ? cnt : 0u;
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if ((t & 63) == 0) wsum[t >> 6] = c;
        __syncthreads();
        if (t < 64) {
            int X = t & 3, Y = (t >> 2) & 3, Z = t >> 4;
            uint8_t o = 0;
            for (int k = 0; k < 8; ++k)
                o |= s0[((2 * Z + (k >> 2)) << 6) | ((2 * Y + ((k >> 1) & 1)) << 3) | (2 * X + (k & 1))];
            s1[t] = o;
            vis1[b * 64 + t] = o;
        }
        __syncthreads();
        if (t < 8) {
            int X = t & 1, Y = (t >> 1) & 1, Z = t >> 2;
            uint8_t o = 0;
            for (int k = 0; k < 8; ++k)
                o |= s1[((2 * Z + (k >> 2)) << 4) | ((2 * Y + ((k >> 1) & 1)) << 2) | (2 * X + (k & 1))];
            s2[t] = o;
            vis2[b * 8 + t] = o;
        }
        __syncthreads();
        if (t == 0) {
            uint8_t o = 0;
            for (int k = 0; k < 8; ++k) o |= s2[k];
            vis3[b] = o;
            unsigned tot = 0;
            for (int k = 0; k < 8; ++k) tot += wsum[k];
            brick_total[sl] = tot;
            if (o) {
                int bx, by, bz;
                brick_xyz((uint32_t)b, g.nb, bx, by, bz);
                int *p = st->stripe[bid_ % kStripes].vbox;
                atomicMin(&p[0], bx); atomicMin(&p[1], by); atomicMin(&p[2], bz);
                atomicMax(&p[3], bx); atomicMax(&p[4], by); atomicMax(&p[5], bz);
                for (int L = 4; L < n_levels && L <= kMarkTop; ++L) {
                    const int s = L - 3;
                    const Level &lv = levels[L];
                    vis_hi[lv.offset + ((int64_t)(bz >> s) * lv.dims[1] + (by >> s)) * lv.dims[0] + (bx >> s)] = 1;
                }
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(512) k_cull_brick(int limit, GridArgs g, const uint32_t *__restrict__ words,
                                                    const int32_t *__restrict__ list, DevStatus *__restrict__ st,
                                                    uint8_t *__restrict__ vis0, uint8_t *__restrict__ vis1,
                                                    uint8_t *__restrict__ vis2, uint8_t *__restrict__ vis3,
                                                    uint8_t *__restrict__ vis_hi, LevelChain ch,
                                                    uint32_t *__restrict__ brick_total) {
    b_cull_brick(limit, g, words, list, st, vis0, vis1, vis2, vis3, vis_hi, ch.lv, ch.n, brick_total, blockIdx.x,
                 gridDim.x);
}

// Culling levels L0, L0 + 1, ... from level L0 - 1 (src, sx x sy x sz) by one
// block, level after level: parent = OR of its children inside the grid.
__device__ void mip_or_levels(int L0, const uint8_t *src, int sx, int sy, int sz, uint8_t *hi, const Level *levels,
                              int n_levels) {
    for (int L = L0; L < n_levels; ++L) {
        const Level &lv = levels[L];
        uint8_t *dst = hi + lv.offset;
        const int64_t n = (int64_t)lv.dims[0] * lv.dims[1] * lv.dims[2];
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            const int x = (int)(i % lv.dims[0]), y = (int)((i / lv.dims[0]) % lv.dims[1]);
            const int z = (int)(i / ((int64_t)lv.dims[0] * lv.dims[1]));
            uint8_t o = 0;
            for (int k = 0; k < 8; ++k) {
                const int cx = 2 * x + (k & 1), cy = 2 * y + ((k >> 1) & 1), cz = 2 * z + (k >> 2);
                if (cx < sx && cy < sy && cz < sz) o |= src[((int64_t)cz * sy + cy) * sx + cx];
            }
            dst[i] = o;
        }
        __syncthreads();
        src = dst;
        sx = lv.dims[0];
        sy = lv.dims[1];
        sz = lv.dims[2];
    }
}

// Single workgroup: exclusive scan of the per-brick visible totals in
// ascending brick order (the grand total is the number of listed fragments),
// then the culling levels above kMarkTop.
__device__ __forceinline__ void b_scan_bricks(const uint32_t *__restrict__ tot, uint32_t *__restrict__ base,
                                                      DevStatus *__restrict__ st, int64_t capacity,
                                                      uint8_t *__restrict__ vis_hi, const Level *levels, int n_levels,
                                                      unsigned bid_, unsigned nblk_) {
    __shared__ unsigned long long wt[16];
    __shared__ unsigned long long carry;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const unsigned n = st->n_bricks;
    if (t == 0) carry = 0;
    __syncthreads();
    for (unsigned start = 0; start < n; start += blockDim.x) {
        unsigned i = start + t;
        unsigned long long v = i < n ? tot[i] : 0ull;
        unsigned long long incl = v;
        for (int o = 1; o < 64; o <<= 1) {
            unsigned long long u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) wt[w] = incl;
        __syncthreads();
        unsigned long long wb = 0;
        for (int k = 0; k < w; ++k) wb += wt[k];
        unsigned long long ex = carry + wb + incl - v;
        if (i < n) base[i] = (uint32_t)ex;
        __syncthreads();
        if (t == (int)blockDim.x - 1) carry = ex + v;
        __syncthreads();
    }
    if (t == 0) {
        st->n_listed = carry;
        if ((long long)carry > capacity) atomicOr(&st->err, kErrCapacity);
    }
    if (n_levels > kMarkTop + 1) {
        const Level &l = levels[kMarkTop];
        mip_or_levels(kMarkTop + 1, vis_hi + l.offset, l.dims[0], l.dims[1], l.dims[2], vis_hi, levels, n_levels);
    }
}

__global__ void __launch_bounds__(1024) k_scan_bricks(const uint32_t *__restrict__ tot, uint32_t *__restrict__ base,
                                                      DevStatus *__restrict__ st, int64_t capacity,
                                                      uint8_t *__restrict__ vis_hi, LevelChain ch) {
    b_scan_bricks(tot, base, st, capacity, vis_hi, ch.lv, ch.n, blockIdx.x, gridDim.x);
}

// One workgroup per occupied brick: list start of every voxel = brick base +
// exclusive prefix of visible counts inside the brick (x fastest).
__device__ __forceinline__ void b_list_offsets(const uint32_t *__restrict__ words,
                                                      const uint8_t *__restrict__ vis0,
                                                      const int32_t *__restrict__ list,
                                                      const uint32_t *__restrict__ base,
                                                      DevStatus *__restrict__ st,
                                                      uint32_t *__restrict__ cursor, uint64_t *__restrict__ cell,
                                                      uint64_t *__restrict__ lmask, uint64_t *__restrict__ lmask2,
                                                      unsigned bid_, unsigned nblk_) {
    __shared__ unsigned wt[8];
    __shared__ unsigned sq[8];
    const unsigned nbk = st->n_bricks;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    unsigned nvis = 0;  // visible voxels seen by this wave
    for (unsigned sl = bid_; sl < nbk; sl += nblk_) {
        int64_t b = list[sl];
        unsigned c = vis0[b * kBrickVox + t] ? (words[b * kBrickVox + t] & 0xFFFFu) : 0u;
        unsigned incl = c;
        for (int o = 1; o < 64; o <<= 1) {
            unsigned u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) wt[w] = incl;
        __syncthreads();
        unsigned wb = 0;
        for (int k = 0; k < w; ++k) wb += wt[k];
        const uint32_t start = base[sl] + wb + incl - c;
        cursor[b * kBrickVox + t] = start;
        cell[b * kBrickVox + t] = (uint64_t)start | ((uint64_t)c << 32);
        const unsigned long long nonempty = __ballot(c != 0u);  // the wave holds local voxels 64w .. 64w + 63
        if (lane == 0) lmask[b * 8 + w] = nonempty;
        nvis += (unsigned)__popcll(nonempty);
        {  // the slice's 2x2 squares holding such a voxel: bit 4 Y + X for square (X, Y)
            unsigned long long s2 = nonempty | (nonempty >> 1);
            s2 |= s2 >> 8;  // bit 16 Y + 2 X: the square's OR
            const unsigned long long m = __ballot(lane < 16 && ((s2 >> (16 * (lane >> 2) + 2 * (lane & 3))) & 1ull));
            if (lane == 0) sq[w] = (unsigned)m & 0xFFFFu;
        }
        __syncthreads();
        if (t == 0) {
            uint64_t cells = 0;
            for (int Z = 0; Z < 4; ++Z) cells |= (uint64_t)(sq[2 * Z] | sq[2 * Z + 1]) << (16 * Z);
            lmask2[b] = cells;
        }
    }
    if (lane == 0 && nvis) atomicAdd(&st->stripe[bid_ % kStripes].vvis, (unsigned long long)nvis);
}

__global__ void __launch_bounds__(512) k_list_offsets(const uint32_t *__restrict__ words,
                                                      const uint8_t *__restrict__ vis0,
                                                      const int32_t *__restrict__ list,
                                                      const uint32_t *__restrict__ base,
                                                      DevStatus *__restrict__ st,
                                                      uint32_t *__restrict__ cursor, uint64_t *__restrict__ cell,
                                                      uint64_t *__restrict__ lmask, uint64_t *__restrict__ lmask2) {
    b_list_offsets(words, vis0, list, base, st, cursor, cell, lmask, lmask2, blockIdx.x, gridDim.x);
}

struct ScatterArgs {
    const VRec *vrec;
    int64_t nv;
    int mode;  // VRT_VOX_*
    long long rq;
    int G[3];
    int nb[3];
    const uint8_t *vis0;
    const uint8_t *vis3;
    uint32_t *cursor;
    uint32_t *ids;
    int64_t capacity;
};

// Pass 2 (Section 3.3) for one segment with global atomics: a segment whose
// capsule AABB touches no visible brick is skipped; otherwise its voxel set is
// walked again and every visible voxel gets the segment id at an atomically
// claimed slot of its list.
__device__ __forceinline__ void scatter_segment(const ScatterArgs &a, int64_t i) {
    if (i + 1 >= a.nv) return;
    VRec A = a.vrec[i];
    if (!(A.flags & kSegValid)) return;
    VRec B = a.vrec[i + 1];
    long long dx = (long long)B.x - A.x, dy = (long long)B.y - A.y, dz = (long long)B.z - A.z;
    if (dx >= 65536 || dx <= -65536 || dy >= 65536 || dy <= -65536 || dz >= 65536 || dz <= -65536) return;
    SlabSpan s = make_span(make_int3(A.x, A.y, A.z), make_int3(B.x, B.y, B.z), a.rq, a.G, a.mode);
    if (s.empty) return;
    // voxel ranges back on (x, y, z)
    const int lx = s.a0 == 0 ? s.vlo0 : (s.a1 == 0 ? s.vlo1 : s.vlo2), hx = s.a0 == 0 ? s.vhi0 : (s.a1 == 0 ? s.vhi1 : s.vhi2);
    const int ly = s.a0 == 1 ? s.vlo0 : (s.a1 == 1 ? s.vlo1 : s.vlo2), hy = s.a0 == 1 ? s.vhi0 : (s.a1 == 1 ? s.vhi1 : s.vhi2);
    const int lz = s.a0 == 2 ? s.vlo0 : (s.a1 == 2 ? s.vlo1 : s.vlo2), hz = s.a0 == 2 ? s.vhi0 : (s.a1 == 2 ? s.vhi1 : s.vhi2);
    bool any = false;
    for (int bz = lz >> 3; bz <= hz >> 3 && !any; ++bz)
        for (int by = ly >> 3; by <= hy >> 3 && !any; ++by)
            for (int bx = lx >> 3; bx <= hx >> 3; ++bx)
                if (a.vis3[((int64_t)bz * a.nb[1] + by) * a.nb[0] + bx]) {
                    any = true;
                    break;
                }
    if (!any) return;
    const uint32_t id = (uint32_t)i;
    for_each_voxel(s, [&](int x, int y, int z) {
        int64_t v = brick_index_of(x, y, z, a.nb[0], a.nb[1]) * kBrickVox + local_of(x, y, z);
        if (a.vis0[v]) {
            uint32_t slot = atomicAdd(&a.cursor[v], 1u);
            if ((int64_t)slot < a.capacity) a.ids[slot] = id;
        }
    });
}

// Pass 2, one thread per segment (the batched form's path).
__device__ __forceinline__ void b_scatter(ScatterArgs a, unsigned bid_, unsigned nblk_) {
    scatter_segment(a, (int64_t)bid_ * blockDim.x + threadIdx.x);
}

struct ScatterBinArgs {
    ScatterArgs sa;
    const int32_t *cand;
    const uint2 *bin_range;
    const uint32_t *bins;
    const uint32_t *long_ids;
};

// Pass 2 by brick (the per-context path): one workgroup per visible binned
// brick walks its bin's segments inside the brick and claims list slots from
// LDS copies of the brick's cursors, so a brick's ids land in its own
// contiguous range of the list array; the cursors are stored back for the
// long segments that follow.
template <int kMode>
__device__ __forceinline__ void b_scatter_brick(ScatterBinArgs a, const DevStatus *__restrict__ st, unsigned bid_,
                                                unsigned nblk_) {
    __shared__ uint32_t cur[kBrickVox];
    __shared__ uint8_t vis[kBrickVox];
    const ScatterArgs &s = a.sa;
    const unsigned n = st->n_cand;
    const int t = threadIdx.x;
    for (unsigned sl = bid_; sl < n; sl += nblk_) {
        const int b = a.cand[sl];
        if (!s.vis3[b]) continue;  // the whole workgroup skips
        for (int v = t; v < kBrickVox; v += blockDim.x) {
            vis[v] = s.vis0[(int64_t)b * kBrickVox + v];
            cur[v] = s.cursor[(int64_t)b * kBrickVox + v];
        }
        __syncthreads();
        const uint2 r = a.bin_range[b];
        const int bx = b % s.nb[0], by = (b / s.nb[0]) % s.nb[1], bz = b / (s.nb[0] * s.nb[1]);
        for (uint32_t k = t; k < r.y; k += blockDim.x) {
            const uint32_t id = a.bins[r.x + k];
            const VRec A = s.vrec[id], B = s.vrec[id + 1];
            const SlabSpan sp = make_span(make_int3(A.x, A.y, A.z), make_int3(B.x, B.y, B.z), s.rq, s.G, s.mode);
            for_each_voxel_in_brick<kMode>(sp, bx, by, bz, [&](int x, int y, int z) {
                const int l = local_of(x, y, z);
                if (vis[l]) {
                    const uint32_t slot = atomicAdd(&cur[l], 1u);
                    if ((int64_t)slot < s.capacity) s.ids[slot] = id;
                }
            });
        }
        __syncthreads();
        for (int v = t; v < kBrickVox; v += blockDim.x) s.cursor[(int64_t)b * kBrickVox + v] = cur[v];
        __syncthreads();
    }
}

// Pass 2 for the long segments (after the binned bricks).
__device__ __forceinline__ void b_scatter_long(ScatterBinArgs a, const DevStatus *__restrict__ st, unsigned bid_,
                                               unsigned nblk_) {
    const unsigned n = st->n_long;
    for (unsigned k = bid_ * blockDim.x + threadIdx.x; k < n; k += nblk_ * blockDim.x) scatter_segment(a.sa, a.long_ids[k]);
}

__global__ void __launch_bounds__(256) k_scatter(ScatterArgs a) { b_scatter(a, blockIdx.x, gridDim.x); }
template <int kMode>
__global__ void __launch_bounds__(256) k_scatter_brick(ScatterBinArgs a, const DevStatus *__restrict__ st) {
    b_scatter_brick<kMode>(a, st, blockIdx.x, gridDim.x);
}
__global__ void __launch_bounds__(256) k_scatter_long(ScatterBinArgs a, const DevStatus *__restrict__ st) {
    b_scatter_long(a, st, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------------
// Optional in-voxel order (Section 3.3 leaves the order of a voxel's list
// undefined, and the slot atomics of pass 2 make it vary between runs): every
// visible voxel's list sorted ascending, which makes the whole id array a
// deterministic function of the frame.

constexpr int kSortShort = 64;     // lists up to this length: one wave, one id per lane
constexpr int kSortLds = 4096;     // longer lists up to this padded length: the workgroup sorts in LDS

// Comparator step of an ascending bitonic network over P = 2^p keys: for the
// first step of a merge of blocks of size `span` the partner is the mirror
// index in the block, afterwards the element `half` away; every comparator
// moves the smaller key to the lower index, so keys past the list's end can
// stand for +inf without being stored.
template <class Load, class Store>
__device__ __forceinline__ void bitonic_steps(uint32_t P, uint32_t n, Load &&ld, Store &&st) {
    for (uint32_t span = 2; span <= P; span <<= 1) {
        for (uint32_t half = span >> 1; half > 0; half >>= 1) {
            for (uint32_t c = threadIdx.x; c < P / 2; c += blockDim.x) {
                const uint32_t blk = c / half, off = c % half;
                const uint32_t i = blk * 2 * half + off;
                const uint32_t j = half == span / 2 ? (i / span) * span + span - 1 - (i % span) : i + half;
                if (j < n) {  // j >= n holds +inf: nothing moves
                    const uint32_t a = ld(i), b = ld(j);
                    if (b < a) {
                        st(i, b);
                        st(j, a);
                    }
                }
            }
            __syncthreads();
        }
    }
}

// One workgroup (512 threads) per occupied brick, grid-stride over the bricks.
__device__ __forceinline__ void b_sort_lists(const uint64_t *__restrict__ cell, const int32_t *__restrict__ list,
                                             const DevStatus *__restrict__ st, uint32_t *__restrict__ ids,
                                             int64_t capacity, unsigned bid_, unsigned nblk_) {
    __shared__ uint32_t keys[kSortLds];
    __shared__ unsigned long long longm[8];
    const unsigned nbk = st->n_bricks;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (st->n_listed > (unsigned long long)capacity) return;  // lists undefined after a capacity overflow
    for (unsigned sl = bid_; sl < nbk; sl += nblk_) {
        const int64_t b = list[sl];
        const uint64_t cd = cell[b * kBrickVox + t];
        const uint32_t n = (uint32_t)(cd >> 32);
        // the wave's 64 voxels one after another: a list of 2..64 ids is loaded one id per lane (the rest
        // padded with the largest key) and sorted by a bitonic network across the lanes
        unsigned long long todo = __ballot(n > 1 && n <= (uint32_t)kSortShort);
        while (todo) {
            const int l = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const uint64_t c = __shfl(cd, l, 64);
            const uint32_t s = (uint32_t)c, len = (uint32_t)(c >> 32);
            uint32_t key = (uint32_t)lane < len ? ids[s + lane] : 0xFFFFFFFFu;
            for (int k = 2; k <= 64; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1) {
                    const uint32_t other = __shfl_xor(key, j, 64);
                    const bool up = (lane & k) == 0, low = (lane & j) == 0;
                    key = (low == up) ? (key < other ? key : other) : (key < other ? other : key);
                }
            if ((uint32_t)lane < len) ids[s + lane] = key;
        }
        const unsigned long long m = __ballot(n > (uint32_t)kSortShort);
        if (lane == 0) longm[w] = m;
        __syncthreads();
        for (int ww = 0; ww < 8; ++ww) {
            unsigned long long mm = longm[ww];
            while (mm) {
                const int l = __ffsll((long long)mm) - 1;
                mm &= mm - 1;
                const uint64_t c2 = cell[b * kBrickVox + 64 * ww + l];
                const uint32_t s = (uint32_t)c2, len = (uint32_t)(c2 >> 32);
                uint32_t P = 1;
                while (P < len) P <<= 1;
                if (P <= (uint32_t)kSortLds) {
                    for (uint32_t i = t; i < len; i += blockDim.x) keys[i] = ids[s + i];
                    __syncthreads();
                    bitonic_steps(P, len, [&](uint32_t i) { return keys[i]; },
                                  [&](uint32_t i, uint32_t v) { keys[i] = v; });
                    for (uint32_t i = t; i < len; i += blockDim.x) ids[s + i] = keys[i];
                } else {
                    bitonic_steps(P, len, [&](uint32_t i) { return ids[s + i]; },
                                  [&](uint32_t i, uint32_t v) { ids[s + i] = v; });
                }
                __syncthreads();
            }
        }
        __syncthreads();  // longm is rewritten for the next brick
    }
}

__global__ void __launch_bounds__(512) k_sort_lists(const uint64_t *__restrict__ cell, const int32_t *__restrict__ list,
                                                    const DevStatus *__restrict__ st, uint32_t *__restrict__ ids,
                                                    int64_t capacity) {
    b_sort_lists(cell, list, st, ids, capacity, blockIdx.x, gridDim.x);
}

}  // namespace

// Blocks of the LDS-staged walk: each copies the flags once, then takes
// occupied voxels grid-stride.  More blocks than fit at once, so a compute
// unit whose blocks drew short walks starts another block while others are
// still walking (1024 blocks: 12% slower on the benchmark frame, 4096: 2%).
static constexpr unsigned kCullWalkBlocks = 2048;

// Arguments of every culling and list kernel for one view of context c.
struct CullPlan {
    int64_t nb, nv;
    int64_t nw, nf;  // words of the brick and 16^3 cell bits, bytes of the 64^3 and 32^3 cell flags
    int limit;  // < 0: no culling
    GridArgs g;
    CullArgs ca;
    CullCells cells;
    ScatterArgs sa;
    ScatterBinArgs sb;
};

static CullPlan make_cull_plan(const vrt_ctx *c, const int64_t E[3], int64_t limit) {
    const Arenas &A = c->a;
    CullPlan p;
    for (int k = 0; k < 3; ++k) {
        p.g.G[k] = c->dims[k];
        p.g.nb[k] = c->dims[k] / 8;
        p.g.ns[k] = (c->dims[k] + 63) / 64;
    }
    p.nb = (int64_t)p.g.nb[0] * p.g.nb[1] * p.g.nb[2];
    p.nv = c->n_vertices;
    p.limit = limit < 0 ? -1 : (int)(limit > INT_MAX ? INT_MAX : limit);
    p.ca.g = p.g;
    for (int k = 0; k < 3; ++k) p.ca.E[k] = E[k];
    p.ca.limit = p.limit;
    const CellFlagLayout cl = cell_flag_layout(p.g.nb);
    p.nw = cl.words;
    p.nf = cl.bytes;
    p.cells.super_blk = A.super_blk;
    p.cells.c32_blk = A.super_blk + cl.b32;
    p.cells.brick_bits = A.brick_bits;
    p.cells.c16_bits = A.brick_bits + cl.w16;
    p.cells.blk_bits = A.blk_bits;
    p.cells.nb0 = p.g.nb[0];
    p.cells.nb1 = p.g.nb[1];
    p.cells.ns0 = p.g.ns[0];
    p.cells.ns1 = p.g.ns[1];
    p.cells.n16x = cl.n16[0];
    p.cells.n16y = cl.n16[1];
    p.cells.n32x = cl.n32[0];
    p.cells.n32y = cl.n32[1];
    p.sa.vrec = A.vrec;
    p.sa.nv = c->n_vertices;
    p.sa.mode = c->voxelizer;
    p.sa.rq = c->rq;
    for (int k = 0; k < 3; ++k) {
        p.sa.G[k] = p.g.G[k];
        p.sa.nb[k] = p.g.nb[k];
    }
    p.sa.vis0 = A.vis0;
    p.sa.vis3 = A.vis3;
    p.sa.cursor = A.cursor;
    p.sa.ids = A.ids;
    p.sa.capacity = c->desc.max_fragments;
    p.sb.sa = p.sa;
    p.sb.cand = A.cand;
    p.sb.bin_range = A.bin_range;
    p.sb.bins = A.bins;
    p.sb.long_ids = A.long_ids;
    return p;
}

hipError_t launch_cull(vrt_ctx *c, const int64_t E[3], int64_t limit, hipStream_t st) {
    Arenas &A = c->a;
    const CullPlan p = make_cull_plan(c, E, limit);
    LevelChain ch;
    ch.n = c->n_levels;
    for (int L = 0; L < kMaxLevels; ++L) ch.lv[L] = c->levels[L];
    const int64_t n_hi = hi_used(c);
    VRT_LAUNCH(c, "k_cull_reset", st,
               k_cull_reset<<<(unsigned)(((p.nb > n_hi ? p.nb : n_hi) + 255) / 256), 256, 0, st>>>(A.vis3, p.nb, A.vis_hi,
                                                                                              n_hi, A.status));
    if (p.limit >= 0) {
        const size_t lds = cull_lds_bytes(p.nw, p.nf);
        if (lds <= kCullLdsMax)
            VRT_LAUNCH(c, "k_cull_walk", st,
                       k_cull_walk<true><<<kCullWalkBlocks, 512, lds, st>>>(p.ca, p.cells, A.occ_list, A.status, A.vis0));
        else
            VRT_LAUNCH(c, "k_cull_walk", st,
                       k_cull_walk<false><<<8192, 512, 0, st>>>(p.ca, p.cells, A.occ_list, A.status, A.vis0));
    }
    VRT_LAUNCH(c, "k_cull_brick", st,
               k_cull_brick<<<4096, 512, 0, st>>>(p.limit, p.g, A.words, A.brick_list, A.status, A.vis0, A.vis1, A.vis2,
                                                  A.vis3, A.vis_hi, ch, A.brick_total));
    VRT_LAUNCH(c, "k_scan_bricks", st,
               k_scan_bricks<<<1, 1024, 0, st>>>(A.brick_total, A.brick_base, A.status, c->desc.max_fragments, A.vis_hi,
                                                 ch));
    VRT_LAUNCH(c, "k_list_offsets", st,
               k_list_offsets<<<4096, 512, 0, st>>>(A.words, A.vis0, A.brick_list, A.brick_base, A.status, A.cursor,
                                                    A.cell, A.lmask, A.lmask2));
    if (c->voxelizer == VRT_VOX_THIN)
        VRT_LAUNCH(c, "k_scatter_brick", st, k_scatter_brick<VRT_VOX_THIN><<<kBrickBlocks, 256, 0, st>>>(p.sb, A.status));
    else if (c->voxelizer == VRT_VOX_AABB)
        VRT_LAUNCH(c, "k_scatter_brick", st, k_scatter_brick<VRT_VOX_AABB><<<kBrickBlocks, 256, 0, st>>>(p.sb, A.status));
    else
        VRT_LAUNCH(c, "k_scatter_brick", st,
                   k_scatter_brick<VRT_VOX_CAPSULE><<<kBrickBlocks, 256, 0, st>>>(p.sb, A.status));
    VRT_LAUNCH(c, "k_scatter_long", st, k_scatter_long<<<256, 256, 0, st>>>(p.sb, A.status));
    return hipGetLastError();
}

hipError_t launch_sort_lists(vrt_ctx *c, hipStream_t st) {
    Arenas &A = c->a;
    VRT_LAUNCH(c, "k_sort_lists", st,
               k_sort_lists<<<4096, 512, 0, st>>>(A.cell, A.brick_list, A.status, A.ids, c->desc.max_fragments));
    return hipGetLastError();
}

}  // namespace vrt
