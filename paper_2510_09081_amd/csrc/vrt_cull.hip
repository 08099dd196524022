// vrt_cull.hip -- Section 3.2 (erosion, culling rays, culling pyramid) and
// Section 3.3 (scan of visible counts, voxelization pass 2 into the lists).
#include <climits>

#include "vrt_internal.h"

namespace vrt {
namespace {

__global__ void k_cull_reset(uint8_t *__restrict__ vis3, uint8_t *__restrict__ brick_blk, int64_t nb,
                             DevStatus *__restrict__ st) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) {
        vis3[i] = 0;
        brick_blk[i] = 0;
    }
    if (i == 0) {
        st->n_listed = 0;
        st->bbox[0] = st->bbox[1] = st->bbox[2] = INT_MAX;
        st->bbox[3] = st->bbox[4] = st->bbox[5] = INT_MIN;
    }
}

struct GridArgs {
    int G[3];
    int nb[3];  // bricks per axis
};

// Level-0 occupancy of any voxel (0 outside the grid and in empty bricks).
__device__ __forceinline__ unsigned occ_at(const GridArgs &g, const uint16_t *__restrict__ occ0,
                                           const int32_t *__restrict__ slot, int x, int y, int z) {
    if (x < 0 || y < 0 || z < 0 || x >= g.G[0] || y >= g.G[1] || z >= g.G[2]) return 0;
    int64_t b = brick_index_of(x, y, z, g.nb[0], g.nb[1]);
    if (slot[b] < 0) return 0;
    return occ0[b * kBrickVox + local_of(x, y, z)];
}

// Erosion (Section 3.2): minimum occupancy over the voxel and its 6 face
// neighbours; the voxel blocks culling rays when that minimum is full.
__global__ void __launch_bounds__(512) k_erode(GridArgs g, const uint16_t *__restrict__ occ0,
                                               const int32_t *__restrict__ list, const int32_t *__restrict__ slot,
                                               DevStatus *__restrict__ st, uint8_t *__restrict__ blk,
                                               uint8_t *__restrict__ brick_blk) {
    __shared__ int bb[6];
    const unsigned nbk = st->n_bricks;
    const int t = threadIdx.x;
    for (unsigned sl = blockIdx.x; sl < nbk; sl += gridDim.x) {
        int64_t b = list[sl];
        if (t < 3) bb[t] = INT_MAX;
        else if (t < 6) bb[t] = INT_MIN;
        __syncthreads();
        int bx = (int)(b % g.nb[0]), by = (int)((b / g.nb[0]) % g.nb[1]), bz = (int)(b / ((int64_t)g.nb[0] * g.nb[1]));
        int x = bx * 8 + (t & 7), y = by * 8 + ((t >> 3) & 7), z = bz * 8 + (t >> 6);
        unsigned e = occ0[b * kBrickVox + t];
        if (e >= 256u) {
            unsigned n;
            n = occ_at(g, occ0, slot, x - 1, y, z); e = n < e ? n : e;
            n = occ_at(g, occ0, slot, x + 1, y, z); e = n < e ? n : e;
            n = occ_at(g, occ0, slot, x, y - 1, z); e = n < e ? n : e;
            n = occ_at(g, occ0, slot, x, y + 1, z); e = n < e ? n : e;
            n = occ_at(g, occ0, slot, x, y, z - 1); e = n < e ? n : e;
            n = occ_at(g, occ0, slot, x, y, z + 1); e = n < e ? n : e;
        }
        bool blocking = e >= 256u;
        blk[b * kBrickVox + t] = blocking ? 1 : 0;
        if (blocking) {
            atomicMin(&bb[0], x); atomicMin(&bb[1], y); atomicMin(&bb[2], z);
            atomicMax(&bb[3], x); atomicMax(&bb[4], y); atomicMax(&bb[5], z);
        }
        int any = __syncthreads_or(blocking ? 1 : 0);
        if (t == 0) {
            brick_blk[b] = any ? 1 : 0;
            if (any) {
                atomicMin(&st->bbox[0], bb[0]); atomicMin(&st->bbox[1], bb[1]); atomicMin(&st->bbox[2], bb[2]);
                atomicMax(&st->bbox[3], bb[3]); atomicMax(&st->bbox[4], bb[4]); atomicMax(&st->bbox[5], bb[5]);
            }
        }
        __syncthreads();
    }
}

// Blocking voxels met by the open segment from the centre of voxel (x,y,z) to
// the eye, up to `limit`: exact integer grid walk; the next crossing on each
// axis is found by comparing g_a*|D_b| with g_b*|D_a| (g: distance from the
// start to the next boundary, D: start-to-eye vector); tied axes step
// together.  Stops at the grid boundary, at the eye, or once the walk has left
// the bounding box of all blocking voxels.
__device__ int culling_ray(const GridArgs &g, int x, int y, int z, const long long *E, int limit, const int *bbox,
                           const uint8_t *__restrict__ blk, const uint8_t *__restrict__ brick_blk) {
    long long adel[3], gd[3];
    int step[3], cur[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
        long long c = (long long)cur[a] * kQ + kQ / 2;
        long long dl = E[a] - c;
        step[a] = dl > 0 ? 1 : (dl < 0 ? -1 : 0);
        adel[a] = dl < 0 ? -dl : dl;
        gd[a] = kQ / 2;
    }
    int n = 0;
    for (;;) {
        // leaving the blocking box for good
        bool gone = false;
        for (int a = 0; a < 3; ++a) {
            if (step[a] > 0 && cur[a] > bbox[3 + a]) gone = true;
            if (step[a] < 0 && cur[a] < bbox[a]) gone = true;
            if (step[a] == 0 && (cur[a] < bbox[a] || cur[a] > bbox[3 + a])) gone = true;
        }
        if (gone) break;
        int m = -1;
        for (int a = 0; a < 3; ++a) {
            if (step[a] == 0) continue;
            if (m < 0 || gd[a] * adel[m] < gd[m] * adel[a]) m = a;
        }
        if (m < 0 || !(gd[m] < adel[m])) break;
        bool out = false;
        long long gm = gd[m], am = adel[m];
        for (int a = 0; a < 3; ++a) {
            if (step[a] != 0 && gd[a] * am == gm * adel[a]) {
                cur[a] += step[a];
                gd[a] += kQ;
                if (cur[a] < 0 || cur[a] >= g.G[a]) out = true;
            }
        }
        if (out) break;
        int64_t b = brick_index_of(cur[0], cur[1], cur[2], g.nb[0], g.nb[1]);
        if (brick_blk[b] && blk[b * kBrickVox + local_of(cur[0], cur[1], cur[2])]) {
            if (++n >= limit) break;
        }
    }
    return n;
}

struct CullArgs {
    GridArgs g;
    long long E[3];
    int limit;  // < 0: no culling
};

// One workgroup per occupied brick: level-0 visibility (occupied and fewer
// than `limit` blockers toward the eye), the in-brick culling mips 1..3
// (parent = OR of children), and the brick's visible-fragment total.
__global__ void __launch_bounds__(512) k_cull_vis(CullArgs a, const uint32_t *__restrict__ words,
                                                  const int32_t *__restrict__ list, const DevStatus *__restrict__ st,
                                                  const uint8_t *__restrict__ blk,
                                                  const uint8_t *__restrict__ brick_blk, uint8_t *__restrict__ vis0,
                                                  uint8_t *__restrict__ vis1, uint8_t *__restrict__ vis2,
                                                  uint8_t *__restrict__ vis3, uint32_t *__restrict__ brick_total) {
    __shared__ uint8_t s0[512];
    __shared__ uint8_t s1[64];
    __shared__ uint8_t s2[8];
    __shared__ unsigned wsum[8];
    __shared__ int bbox[6];
    const unsigned nbk = st->n_bricks;
    const int t = threadIdx.x;
    if (t < 6) bbox[t] = st->bbox[t];
    __syncthreads();
    for (unsigned sl = blockIdx.x; sl < nbk; sl += gridDim.x) {
        int64_t b = list[sl];
        int bx = (int)(b % a.g.nb[0]), by = (int)((b / a.g.nb[0]) % a.g.nb[1]);
        int bz = (int)(b / ((int64_t)a.g.nb[0] * a.g.nb[1]));
        int x = bx * 8 + (t & 7), y = by * 8 + ((t >> 3) & 7), z = bz * 8 + (t >> 6);
        unsigned cnt = words[b * kBrickVox + t] & 0xFFFFu;
        uint8_t v = 0;
        if (cnt) {
            if (a.limit < 0) v = 1;
            else v = culling_ray(a.g, x, y, z, a.E, a.limit, bbox, blk, brick_blk) < a.limit ? 1 : 0;
        }
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
        }
        __syncthreads();
    }
}

__global__ void k_mip_or(const uint8_t *__restrict__ src, int sx, int sy, int sz, uint8_t *__restrict__ dst, int dx,
                         int dy, int dz) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)dx * dy * dz) return;
    int x = (int)(i % dx), y = (int)((i / dx) % dy), z = (int)(i / ((int64_t)dx * dy));
    uint8_t o = 0;
    for (int k = 0; k < 8; ++k) {
        int cx = 2 * x + (k & 1), cy = 2 * y + ((k >> 1) & 1), cz = 2 * z + (k >> 2);
        if (cx < sx && cy < sy && cz < sz) o |= src[((int64_t)cz * sy + cy) * sx + cx];
    }
    dst[i] = o;
}

// Single workgroup: exclusive scan of the per-brick visible totals in
// ascending brick order; the grand total is the number of listed fragments.
__global__ void __launch_bounds__(1024) k_scan_bricks(const uint32_t *__restrict__ tot, uint32_t *__restrict__ base,
                                                      DevStatus *__restrict__ st, int64_t capacity) {
    __shared__ unsigned long long wt[16];
    __shared__ unsigned long long carry;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const unsigned n = st->n_bricks;
    if (t == 0) carry = 0;
    __syncthreads();
    for (unsigned start = 0; start < n; start += 1024) {
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
        if (t == 1023) carry = ex + v;
        __syncthreads();
    }
    if (t == 0) {
        st->n_listed = carry;
        if ((long long)carry > capacity) atomicOr(&st->err, kErrCapacity);
    }
}

// One workgroup per occupied brick: list start of every voxel = brick base +
// exclusive prefix of visible counts inside the brick (x fastest).
__global__ void __launch_bounds__(512) k_list_offsets(const uint32_t *__restrict__ words,
                                                      const uint8_t *__restrict__ vis0,
                                                      const int32_t *__restrict__ list,
                                                      const uint32_t *__restrict__ base,
                                                      const DevStatus *__restrict__ st,
                                                      uint32_t *__restrict__ cursor) {
    __shared__ unsigned wt[8];
    const unsigned nbk = st->n_bricks;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (unsigned sl = blockIdx.x; sl < nbk; sl += gridDim.x) {
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
        cursor[b * kBrickVox + t] = base[sl] + wb + incl - c;
        __syncthreads();
    }
}

struct ScatterArgs {
    const VRec *vrec;
    int64_t nv;
    long long rq;
    int G[3];
    int nb[3];
    const uint8_t *vis0;
    const uint8_t *vis3;
    uint32_t *cursor;
    uint32_t *ids;
    int64_t capacity;
};

// Pass 2 (Section 3.3): a segment whose capsule AABB touches no visible brick
// is skipped; otherwise its voxel set is walked again and every visible voxel
// gets the segment id at an atomically claimed slot of its list.
__global__ void __launch_bounds__(256) k_scatter(ScatterArgs a) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i + 1 >= a.nv) return;
    VRec A = a.vrec[i];
    if (!(A.flags & kSegValid)) return;
    VRec B = a.vrec[i + 1];
    long long dx = (long long)B.x - A.x, dy = (long long)B.y - A.y, dz = (long long)B.z - A.z;
    if (dx >= 65536 || dx <= -65536 || dy >= 65536 || dy <= -65536 || dz >= 65536 || dz <= -65536) return;
    SlabSpan s = make_span(make_int3(A.x, A.y, A.z), make_int3(B.x, B.y, B.z), a.rq, a.G);
    if (s.empty) return;
    bool any = false;
    for (int bz = s.vlo[2] >> 3; bz <= s.vhi[2] >> 3 && !any; ++bz)
        for (int by = s.vlo[1] >> 3; by <= s.vhi[1] >> 3 && !any; ++by)
            for (int bx = s.vlo[0] >> 3; bx <= s.vhi[0] >> 3; ++bx)
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

}  // namespace

hipError_t launch_cull(vrt_ctx *c, const int64_t E[3], int64_t limit, hipStream_t st) {
    Arenas &A = c->a;
    GridArgs g;
    for (int k = 0; k < 3; ++k) {
        g.G[k] = c->dims[k];
        g.nb[k] = c->dims[k] / 8;
    }
    const int64_t nb = (int64_t)g.nb[0] * g.nb[1] * g.nb[2];
    VRT_LAUNCH(c, "k_cull_reset", st, k_cull_reset<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(A.vis3, A.brick_blk, nb, A.status));
    VRT_LAUNCH(c, "k_erode", st, k_erode<<<4096, 512, 0, st>>>(g, A.occ0, A.brick_list, A.brick_slot, A.status, A.blk, A.brick_blk));
    CullArgs ca;
    ca.g = g;
    for (int k = 0; k < 3; ++k) ca.E[k] = E[k];
    ca.limit = limit < 0 ? -1 : (int)(limit > INT_MAX ? INT_MAX : limit);
    VRT_LAUNCH(c, "k_cull_vis", st, k_cull_vis<<<4096, 512, 0, st>>>(ca, A.words, A.brick_list, A.status, A.blk, A.brick_blk, A.vis0, A.vis1, A.vis2,
                                     A.vis3, A.brick_total));
    const uint8_t *src = A.vis3;
    int sx = g.nb[0], sy = g.nb[1], sz = g.nb[2];
    for (int L = 4; L < c->n_levels; ++L) {
        const Level &lv = c->levels[L];
        uint8_t *dst = A.vis_hi + lv.offset;
        int64_t n = (int64_t)lv.dims[0] * lv.dims[1] * lv.dims[2];
        VRT_LAUNCH(c, "k_mip_or", st, k_mip_or<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(src, sx, sy, sz, dst, lv.dims[0], lv.dims[1], lv.dims[2]));
        src = dst;
        sx = lv.dims[0];
        sy = lv.dims[1];
        sz = lv.dims[2];
    }
    VRT_LAUNCH(c, "k_scan_bricks", st, k_scan_bricks<<<1, 1024, 0, st>>>(A.brick_total, A.brick_base, A.status, c->desc.max_fragments));
    VRT_LAUNCH(c, "k_list_offsets", st, k_list_offsets<<<4096, 512, 0, st>>>(A.words, A.vis0, A.brick_list, A.brick_base, A.status, A.cursor));
    ScatterArgs sa;
    sa.vrec = A.vrec;
    sa.nv = c->n_vertices;
    sa.rq = c->rq;
    for (int k = 0; k < 3; ++k) {
        sa.G[k] = g.G[k];
        sa.nb[k] = g.nb[k];
    }
    sa.vis0 = A.vis0;
    sa.vis3 = A.vis3;
    sa.cursor = A.cursor;
    sa.ids = A.ids;
    sa.capacity = c->desc.max_fragments;
    VRT_LAUNCH(c, "k_scatter", st, k_scatter<<<(unsigned)((c->n_vertices + 255) / 256), 256, 0, st>>>(sa));
    return hipGetLastError();
}

}  // namespace vrt
