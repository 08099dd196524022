// vrt_voxelize.hip -- Section 3.1: ingest, voxelization pass 1 and the occupancy pyramid.
#include <climits>

#include "vrt_internal.h"

namespace vrt {
namespace {

// Zeroes the level-0 words of every brick the previous frame occupied.
__device__ __forceinline__ void b_clear_prev(uint32_t *__restrict__ words, const int32_t *__restrict__ brick_list,
                             const DevStatus *__restrict__ st, unsigned bid_, unsigned nblk_) {
    const unsigned nb = st->n_bricks;
    uint4 *w4 = reinterpret_cast<uint4 *>(words);
    for (unsigned slot = bid_; slot < nb; slot += nblk_) {
        int64_t b = brick_list[slot];
        for (int t = threadIdx.x; t < kBrickVox / 4; t += blockDim.x) w4[b * (kBrickVox / 4) + t] = make_uint4(0, 0, 0, 0);
    }
}

__global__ void k_clear_prev(uint32_t *__restrict__ words, const int32_t *__restrict__ brick_list,
                             const DevStatus *__restrict__ st) { b_clear_prev(words, brick_list, st, blockIdx.x, gridDim.x); }

// Clears the per-frame brick-level state: level-3 occupancy, blocking flags
// of bricks and 64^3 cells, the blocking box and the frame counters.
// Threads of the per-frame reset: bricks, flag words and flag bytes.
__host__ __device__ inline int64_t reset_items(int64_t nb, int64_t nw, int64_t nf) {
    const int64_t m = nb > nw ? nb : nw;
    return m > nf ? m : nf;
}

__device__ __forceinline__ void b_reset(uint16_t *__restrict__ occ3, uint32_t *__restrict__ bin_count,
                        uint32_t *__restrict__ brick_bits, int64_t nbricks, int64_t nwords,
                        uint8_t *__restrict__ super_blk, int64_t nflags, DevStatus *__restrict__ st, unsigned bid_, unsigned nblk_) {
    int64_t i = (int64_t)bid_ * blockDim.x + threadIdx.x;
    if (i < nbricks) {
        occ3[i] = 0;
        bin_count[i * kBinStride] = 0u;
    }
    if (i < nwords) brick_bits[i] = 0u;
    if (i < nflags) super_blk[i] = 0;
    if (i == 0) {
        st->n_fragments = 0;
        st->n_cand = 0;
        st->n_long = 0;
        st->bin_total = 0;
        st->n_items = 0;
        st->n_occ = 0;
    }
    if (i < kStripes) {
        StatStripe &p = st->stripe[i];
        p.frag = 0;
        p.csum = 0;
        p.bbox[0] = p.bbox[1] = p.bbox[2] = INT_MAX;
        p.bbox[3] = p.bbox[4] = p.bbox[5] = INT_MIN;
    }
}

__global__ void k_reset(uint16_t *__restrict__ occ3, uint32_t *__restrict__ bin_count, uint32_t *__restrict__ brick_bits,
                        int64_t nbricks, int64_t nwords, uint8_t *__restrict__ super_blk, int64_t nflags,
                        DevStatus *__restrict__ st) {
    b_reset(occ3, bin_count, brick_bits, nbricks, nwords, super_blk, nflags, st, blockIdx.x, gridDim.x);
}

// fixed-point coordinate: rint((x - origin) * s) as two binary32 operations
__device__ __forceinline__ bool quantize1(float x, float o, float s, int &q) {
    float u = (x - o) * s;
    if (!(fabsf(u) < 1048576.0f)) {
        q = 0;
        return false;
    }
    q = (int)rintf(u);
    return q < (1 << 20) && q > -(1 << 20);
}

__device__ __forceinline__ bool quantize3(const float *__restrict__ xyz, int64_t i, const float *o, float s, int *q) {
    bool ok = quantize1(xyz[3 * i + 0], o[0], s, q[0]);
    ok &= quantize1(xyz[3 * i + 1], o[1], s, q[1]);
    ok &= quantize1(xyz[3 * i + 2], o[2], s, q[2]);
    return ok;
}

struct IngestArgs {
    const float *xyz;
    const int32_t *off;
    int64_t np, nv;
    float o[3];
    float s;
};

// One thread per vertex: polyline lookup by binary search over the offsets,
// quantization, segment/interior flags and the central-difference clip normal.
__device__ __forceinline__ void b_ingest(IngestArgs a, VRec *__restrict__ out, DevStatus *__restrict__ st, unsigned bid_, unsigned nblk_) {
    const int64_t i0 = (int64_t)bid_ * blockDim.x;  // the block's first vertex
    int64_t i = i0 + threadIdx.x;
    if (i0 >= a.nv) return;
    // polyline of the block's first vertex (largest p with off[p] <= i0), the
    // same search in every lane: from the proportional guess, doubling steps
    // until the polyline is bracketed, then halving; each lane then scans
    // forward to its own
    int64_t g = (int64_t)((float)i0 * ((float)a.np / (float)a.nv));  // a guess only: the search corrects it
    g = g < 0 ? 0 : (g > a.np - 1 ? a.np - 1 : g);
    int64_t lo, hi;  // off[lo] <= i0 (or lo = 0), and hi = np or off[hi] > i0
    if ((int64_t)a.off[g] <= i0) {
        lo = g;
        hi = g + 1;
        for (int64_t s = 1; hi < a.np && (int64_t)a.off[hi] <= i0; s <<= 1) {
            lo = hi;
            hi = lo + 2 * s;
        }
        hi = hi > a.np ? a.np : hi;
    } else {
        hi = g;
        lo = g - 1;
        for (int64_t s = 1; lo > 0 && (int64_t)a.off[lo] > i0; s <<= 1) {
            hi = lo;
            lo = hi - 2 * s;
        }
        lo = lo < 0 ? 0 : lo;
    }
    while (lo + 1 < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)a.off[mid] <= i0) lo = mid;
        else hi = mid;
    }
    if (i >= a.nv) return;
    if (i == 0 && (a.off[0] != 0 || a.off[a.np] != a.nv)) set_err(st, kErrInvalid);
    while (lo + 1 < a.np && (int64_t)a.off[lo + 1] <= i) ++lo;
    int64_t pa = a.off[lo], pb = a.off[lo + 1];
    VRec r;
    int q[3];
    bool ok = quantize3(a.xyz, i, a.o, a.s, q);
    r.x = q[0];
    r.y = q[1];
    r.z = q[2];
    r.flags = 0;
    r.nx = r.ny = r.nz = r.pad = 0.0f;
    if (!(pa <= i && i < pb) || pa < 0 || pb > a.nv) {  // offsets not a partition of [0, nv)
        set_err(st, kErrInvalid);
    } else {
        if (i + 1 < pb) r.flags |= kSegValid;
        if (i > pa && i + 1 < pb) {
            int qp[3], qn[3];
            ok &= quantize3(a.xyz, i - 1, a.o, a.s, qp);
            ok &= quantize3(a.xyz, i + 1, a.o, a.s, qn);
            long long T0 = (long long)qn[0] - qp[0], T1 = (long long)qn[1] - qp[1], T2 = (long long)qn[2] - qp[2];
            long long TT = T0 * T0 + T1 * T1 + T2 * T2;
            if (TT > 0) {
                float len = sqrtf((float)TT);
                r.nx = (float)T0 / len;
                r.ny = (float)T1 / len;
                r.nz = (float)T2 / len;
                r.flags |= kInterior;
            }
        }
    }
    if (!ok) set_err(st, kErrRange);
    out[i] = r;
}

__global__ void k_ingest(IngestArgs a, VRec *__restrict__ out, DevStatus *__restrict__ st) { b_ingest(a, out, st, blockIdx.x, gridDim.x); }

// Occupancy quantum of one (segment, voxel) pair: the clipped-capsule SDF at
// the voxel centre with the PWAA radius clamp (Alg. 2, Alg. 3), evaluated as a
// fixed binary32 sequence (no contraction, sums left to right).  Lengths in
// 1/256 voxel.  Returns rint(256 * occupancy) in [0, 256].
__device__ __forceinline__ int occupancy_quantum(const VRec &A, const VRec &B, float rc, float corr, int vx, int vy,
                                                 int vz) {
    int px = vx * kQ + kQ / 2, py = vy * kQ + kQ / 2, pz = vz * kQ + kQ / 2;
    float pax = (float)(px - A.x), pay = (float)(py - A.y), paz = (float)(pz - A.z);
    float pbx = (float)(px - B.x), pby = (float)(py - B.y), pbz = (float)(pz - B.z);
    float dx = (float)(B.x - A.x), dy = (float)(B.y - A.y), dz = (float)(B.z - A.z);
    float num = pax * dx;
    num = num + pay * dy;
    num = num + paz * dz;
    float den = dx * dx;
    den = den + dy * dy;
    den = den + dz * dz;
    float h = 0.0f;
    if (den > 0.0f) h = fminf(fmaxf(num / den, 0.0f), 1.0f);
    float ex = pax - dx * h, ey = pay - dy * h, ez = paz - dz * h;
    float ss = ex * ex;
    ss = ss + ey * ey;
    ss = ss + ez * ez;
    float sdf = sqrtf(ss) - rc;
    if (A.flags & kInterior) {
        float s0 = pax * A.nx;
        s0 = s0 + pay * A.ny;
        s0 = s0 + paz * A.nz;
        sdf = fmaxf(sdf, -s0);
    }
    if (B.flags & kInterior) {
        float s1 = pbx * B.nx;
        s1 = s1 + pby * B.ny;
        s1 = s1 + pbz * B.nz;
        sdf = fmaxf(sdf, s1);
    }
    float occ = fminf(fmaxf(0.5f - sdf / 256.0f, 0.0f), 1.0f) * corr;
    return (int)rintf(occ * 256.0f);
}

// FP16 form: one record per segment with its endpoints relative to the centre
// of the brick holding its midpoint (binary16, voxel units) and its clip
// normals in 16-bit signed fixed point.  Quantized positions are multiples of 1/256 voxel, so
// offsets below 8 voxels are exact; a segment with a longer offset (one that
// reaches beyond the neighbouring bricks) is marked to be read from its plain
// vertex records instead.
__device__ __forceinline__ void b_pack16(const VRec *__restrict__ vrec, int64_t nv, SRec16 *__restrict__ out, unsigned bid_, unsigned nblk_) {
    const int64_t i = (int64_t)bid_ * blockDim.x + threadIdx.x;
    if (i + 1 >= nv) return;
    const VRec A = vrec[i];
    if (!(A.flags & kSegValid)) return;
    const VRec B = vrec[i + 1];
    const long long mx = ((long long)A.x + B.x) >> 1, my = ((long long)A.y + B.y) >> 1, mz = ((long long)A.z + B.z) >> 1;
    const long long bx = mx >> 11, by = my >> 11, bz = mz >> 11;  // 8 voxels = 2^11 steps
    const long long cx = bx * 2048 + 1024, cy = by * 2048 + 1024, cz = bz * 2048 + 1024;
    SRec16 r;
    r.a[0] = __float2half((float)(A.x - cx) * (1.0f / kQ));
    r.a[1] = __float2half((float)(A.y - cy) * (1.0f / kQ));
    r.a[2] = __float2half((float)(A.z - cz) * (1.0f / kQ));
    r.b[0] = __float2half((float)(B.x - cx) * (1.0f / kQ));
    r.b[1] = __float2half((float)(B.y - cy) * (1.0f / kQ));
    r.b[2] = __float2half((float)(B.z - cz) * (1.0f / kQ));
    r.n0[0] = (short)rintf(A.nx * 32767.0f);
    r.n0[1] = (short)rintf(A.ny * 32767.0f);
    r.n0[2] = (short)rintf(A.nz * 32767.0f);
    r.n1[0] = (short)rintf(B.nx * 32767.0f);
    r.n1[1] = (short)rintf(B.ny * 32767.0f);
    r.n1[2] = (short)rintf(B.nz * 32767.0f);
    r.bx = (short)bx;
    r.by = (short)by;
    r.bz = (short)bz;
    const long long ox[6] = {A.x - cx, A.y - cy, A.z - cz, B.x - cx, B.y - cy, B.z - cz};
    bool exact = true;
#pragma unroll
    for (int k = 0; k < 6; ++k) exact &= ox[k] > -2048 && ox[k] < 2048;  // |offset| < 8 voxels
    r.flags = (unsigned short)(((A.flags & kInterior) ? 1 : 0) | ((B.flags & kInterior) ? 2 : 0) |
                               (exact ? 0u : kSRecPlain));
    out[i] = r;
}

__global__ void k_pack16(const VRec *__restrict__ vrec, int64_t nv, SRec16 *__restrict__ out) { b_pack16(vrec, nv, out, blockIdx.x, gridDim.x); }

struct CountArgs {
    const VRec *vrec;
    int64_t nv;
    int mode;  // VRT_VOX_*
    long long rq;
    float rc, corr;
    int G[3];
    int nbx, nby;
    uint32_t *words;
    uint8_t *brick_flag;
};

// Pass 1 for one segment with global atomics: walks its voxel set and adds
// 1 + (q << 16) to each voxel's packed word (count low, occupancy high).
// The adds return nothing: a count field that wraps past 65535 is found
// afterwards, because the count fields then sum to less than the number of
// fragments (each wrap loses exactly 65536).  Returns the fragments.
__device__ __forceinline__ unsigned long long vox_count_segment(const CountArgs &a, int64_t i, DevStatus *st) {
    if (i + 1 >= a.nv) return 0;
    const VRec A = a.vrec[i];
    if (!(A.flags & kSegValid)) return 0;
    const VRec B = a.vrec[i + 1];
    const long long dx = (long long)B.x - A.x, dy = (long long)B.y - A.y, dz = (long long)B.z - A.z;
    if (dx >= 65536 || dx <= -65536 || dy >= 65536 || dy <= -65536 || dz >= 65536 || dz <= -65536) {
        set_err(st, kErrRange);
        return 0;
    }
    SlabSpan s = make_span(make_int3(A.x, A.y, A.z), make_int3(B.x, B.y, B.z), a.rq, a.G, a.mode);
    int64_t last_b = -1;
    return for_each_voxel(s, [&](int x, int y, int z) {
        int q = occupancy_quantum(A, B, a.rc, a.corr, x, y, z);
        int64_t b = brick_index_of(x, y, z, a.nbx, a.nby);
        atomicAdd(&a.words[b * kBrickVox + local_of(x, y, z)], 1u + ((uint32_t)q << 16));
        if (b != last_b) {
            a.brick_flag[b] = 1;
            last_b = b;
        }
    });
}

// Pass 1, one thread per segment (the batched form's path).
__device__ __forceinline__ void b_vox_count(CountArgs a, DevStatus *__restrict__ st, unsigned bid_, unsigned nblk_) {
    unsigned long long nfrag = vox_count_segment(a, (int64_t)bid_ * blockDim.x + threadIdx.x, st);
    nfrag = wave_sum_u64(nfrag);
    if ((threadIdx.x & 63) == 0 && nfrag) atomicAdd(&st->stripe[bid_ % kStripes].frag, nfrag);
}

// ------------------------------------------------------------------------
// Pass 1 by brick (the per-context path).  Segments are first binned by the
// bricks of their voxel box; then one workgroup per binned brick adds the
// brick's fragments in LDS and stores its 512 words once.  Device-wide atomics
// go from one per fragment to about one per run of consecutive segments in a
// brick; words are written with plain coalesced stores.

struct BinArgs {
    const VRec *vrec;
    int64_t nv;
    long long rq;
    int G[3];
    int nb[3];
    uint32_t *bin_count;
    uint2 *bin_range;
    int32_t *cand;
    uint32_t *bins;
    int64_t bin_cap;
    uint32_t *long_ids;
    uint2 *items;
};

// Brick box of segment i's voxel set; 0 bricks when the segment is not
// valid, out of range (flagged when `flag`) or its set is empty.
__device__ __forceinline__ int seg_brick_box(const BinArgs &a, int64_t i, DevStatus *st, bool flag, int &bx0,
                                             int &bx1, int &by0, int &by1, int &bz0, int &bz1) {
    if (i + 1 >= a.nv) return 0;
    const VRec A = a.vrec[i];
    if (!(A.flags & kSegValid)) return 0;
    const VRec B = a.vrec[i + 1];
    const long long dx = (long long)B.x - A.x, dy = (long long)B.y - A.y, dz = (long long)B.z - A.z;
    if (dx >= 65536 || dx <= -65536 || dy >= 65536 || dy <= -65536 || dz >= 65536 || dz <= -65536) {
        if (flag) set_err(st, kErrRange);
        return 0;
    }
    // the voxel range of the closed capsule AABB, clipped to the grid (the box make_span computes)
    int lo[3], hi[3];
    const int pa[3] = {A.x, A.y, A.z}, pb[3] = {B.x, B.y, B.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const long long l = (long long)(pa[k] < pb[k] ? pa[k] : pb[k]) - a.rq - 1;
        const long long h = (long long)(pa[k] < pb[k] ? pb[k] : pa[k]) + a.rq;
        long long vl = l >> 8, vh = h >> 8;  // floor division by kQ = 256
        vl = vl < 0 ? 0 : vl;
        vh = vh > a.G[k] - 1 ? a.G[k] - 1 : vh;
        if (vl > vh) return 0;
        lo[k] = (int)vl >> 3;
        hi[k] = (int)vh >> 3;
    }
    bx0 = lo[0], bx1 = hi[0], by0 = lo[1], by1 = hi[1], bz0 = lo[2], bz1 = hi[2];
    return (bx1 - bx0 + 1) * (by1 - by0 + 1) * (bz1 - bz0 + 1);
}

// Brick k (0-based, x fastest) of a brick box.
__device__ __forceinline__ int box_brick(const BinArgs &a, int k, int bx0, int bx1, int by0, int by1, int bz0) {
    const int wx = bx1 - bx0 + 1, wy = by1 - by0 + 1;
    const int bx = bx0 + k % wx, by = by0 + (k / wx) % wy, bz = bz0 + k / (wx * wy);
    return (bz * a.nb[1] + by) * a.nb[0] + bx;
}

// Runs of consecutive lanes whose segment lies in one brick (key >= 0): true
// for the first lane of a run, with the run's length.
__device__ __forceinline__ bool run_head(int key, int lane, unsigned long long &heads, unsigned &len) {
    const int prev = __shfl_up(key, 1, 64);
    const bool head = key >= 0 && (lane == 0 || prev != key);
    heads = __ballot(head);
    const unsigned long long single = __ballot(key >= 0);
    const unsigned long long stop = (heads | ~single) & ~((2ull << lane) - 1ull);  // lanes after this one
    len = (unsigned)((stop ? __ffsll((long long)stop) - 1 : 64) - lane);
    return head;
}

// Bin sizes: one thread per segment.  A brick whose count leaves zero is
// appended to the candidate list; segments spanning more than kMaxBinBricks
// bricks go to the long list.
__device__ __forceinline__ void b_bin_count(BinArgs a, DevStatus *__restrict__ st, unsigned bid_, unsigned nblk_) {
    const int64_t i = (int64_t)bid_ * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int bx0 = 0, bx1 = 0, by0 = 0, by1 = 0, bz0 = 0, bz1 = 0;
    const int nbr = seg_brick_box(a, i, st, true, bx0, bx1, by0, by1, bz0, bz1);
    const int nbin = nbr <= kMaxBinBricks ? nbr : 0;
    // the k-th bricks of consecutive segments along a polyline mostly agree:
    // one atomic per run of equal bricks
    for (int k = 0; __ballot(k < nbin); ++k) {
        const int key = k < nbin ? box_brick(a, k, bx0, bx1, by0, by1, bz0) : -1;
        unsigned long long heads;
        unsigned len;
        const bool head = run_head(key, lane, heads, len);
        bool fresh = false;
        if (head) fresh = atomicAdd(&a.bin_count[(int64_t)key * kBinStride], len) == 0u;
        wave_append(fresh, key, &st->n_cand, a.cand);
    }
    wave_append(nbr > kMaxBinBricks, (uint32_t)i, &st->n_long, a.long_ids);
}

// Bin ranges and work items: per wave, inclusive scans of the candidates'
// counts and chunk counts and one atomic on each running total.
__device__ __forceinline__ void b_bin_alloc(BinArgs a, DevStatus *__restrict__ st, unsigned bid_, unsigned nblk_) {
    const unsigned n = st->n_cand;
    const int lane = threadIdx.x & 63;
    const unsigned stride = nblk_ * blockDim.x;
    for (unsigned base = bid_ * blockDim.x + (threadIdx.x & ~63u); base < n; base += stride) {
        const unsigned k = base + lane;
        int b = -1;
        unsigned c = 0;
        if (k < n) {
            b = a.cand[k];
            c = a.bin_count[(int64_t)b * kBinStride];
        }
        const unsigned nch = (c + kBinChunk - 1) / kBinChunk;
        unsigned incl = c, inch = nch;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned u = __shfl_up(incl, o, 64), v = __shfl_up(inch, o, 64);
            if (lane >= o) {
                incl += u;
                inch += v;
            }
        }
        unsigned long long start = 0;
        unsigned first = 0;
        if (lane == 63) {
            start = atomicAdd(&st->bin_total, (unsigned long long)incl);
            first = atomicAdd(&st->n_items, inch);
        }
        start = __shfl(start, 63, 64);
        first = __shfl(first, 63, 64);
        if (k < n) {
            a.bin_range[b] = make_uint2((uint32_t)(start + incl - c), c);
            for (unsigned j = 0; j < nch; ++j) a.items[first + inch - nch + j] = make_uint2((uint32_t)b, j);
        }
    }
}

// Bin entries: the same enumeration as b_bin_count; each run (or brick of a
// multi-brick segment) takes its slots by counting its bin back down to zero.
__device__ __forceinline__ void b_bin_fill(BinArgs a, DevStatus *__restrict__ st, unsigned bid_, unsigned nblk_) {
    const int64_t i = (int64_t)bid_ * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int bx0 = 0, bx1 = 0, by0 = 0, by1 = 0, bz0 = 0, bz1 = 0;
    const int nbr = seg_brick_box(a, i, st, false, bx0, bx1, by0, by1, bz0, bz1);
    const int nbin = nbr <= kMaxBinBricks ? nbr : 0;
    for (int k = 0; __ballot(k < nbin); ++k) {
        const int key = k < nbin ? box_brick(a, k, bx0, bx1, by0, by1, bz0) : -1;
        unsigned long long heads;
        unsigned len;
        const bool head = run_head(key, lane, heads, len);
        unsigned old = 0;
        if (head) old = atomicSub(&a.bin_count[(int64_t)key * kBinStride], len);
        // each lane of a run takes its slot from the run's head (the last head at or below it)
        const int h = key >= 0 ? 63 - __clzll((long long)(heads & ((2ull << lane) - 1ull))) : lane;
        const unsigned old_h = __shfl(old, h, 64), len_h = __shfl(len, h, 64);
        if (key >= 0) {
            const uint64_t slot = (uint64_t)a.bin_range[key].x + (old_h - len_h) + (unsigned)(lane - h);
            if ((int64_t)slot < a.bin_cap) a.bins[slot] = (uint32_t)i;
        }
    }
}

struct AccumArgs {
    CountArgs ca;
    const uint2 *items;
    const uint2 *bin_range;
    const uint32_t *bins;
};

// Words of the binned bricks: one workgroup per (brick, chunk) item adds the
// chunk's fragments in LDS, then stores the brick's 512 words (a brick of one
// chunk) or adds them to the words (every word is zero at the start of a
// frame: the previous frame's occupied bricks are cleared), and flags the
// brick when it holds a fragment.
template <int kMode>
__device__ __forceinline__ void b_brick_accum(AccumArgs a, DevStatus *__restrict__ st, unsigned bid_, unsigned nblk_) {
    __shared__ uint32_t w[kBrickVox];
    const CountArgs &c = a.ca;
    const unsigned n = st->n_items;
    const int t = threadIdx.x;
    unsigned long long nfrag = 0;
    for (unsigned it = bid_; it < n; it += nblk_) {
        const uint2 item = a.items[it];
        const int b = (int)item.x;
        const uint2 r = a.bin_range[b];
        const uint32_t k0 = item.y * kBinChunk, len = min(r.y - k0, (uint32_t)kBinChunk);
        for (int v = t; v < kBrickVox; v += blockDim.x) w[v] = 0u;
        __syncthreads();
        const int bx = b % c.nbx, by = (b / c.nbx) % c.nby, bz = b / (c.nbx * c.nby);
        for (uint32_t u = t; u < ((len + 63u) & ~63u); u += blockDim.x) {
            const uint32_t kk = spread64(u);
            if (kk >= len) continue;
            const uint32_t id = a.bins[r.x + k0 + kk];
            const VRec A = c.vrec[id], B = c.vrec[id + 1];
            const SlabSpan s = make_span(make_int3(A.x, A.y, A.z), make_int3(B.x, B.y, B.z), c.rq, c.G, c.mode);
            nfrag += for_each_voxel_in_brick<kMode>(s, bx, by, bz, [&](int x, int y, int z) {
                const int q = occupancy_quantum(A, B, c.rc, c.corr, x, y, z);
                atomicAdd(&w[local_of(x, y, z)], 1u + ((uint32_t)q << 16));
            });
        }
        __syncthreads();
        const bool whole = r.y <= (uint32_t)kBinChunk;
        unsigned any = 0;
        for (int v = t; v < kBrickVox; v += blockDim.x) {
            const uint32_t wd = w[v];
            if (whole) c.words[(int64_t)b * kBrickVox + v] = wd;
            else if (wd) atomicAdd(&c.words[(int64_t)b * kBrickVox + v], wd);
            any |= wd & 0xFFFFu;
        }
        if (__syncthreads_or(any != 0u) && t == 0) c.brick_flag[b] = 1;
    }
    nfrag = wave_sum_u64(nfrag);
    if ((t & 63) == 0 && nfrag) atomicAdd(&st->stripe[bid_ % kStripes].frag, nfrag);
}

// Pass 1 for the long segments, after the binned bricks' words are stored.
__device__ __forceinline__ void b_vox_long(CountArgs a, const uint32_t *__restrict__ long_ids, DevStatus *__restrict__ st,
                                           unsigned bid_, unsigned nblk_) {
    const unsigned n = st->n_long;
    unsigned long long nfrag = 0;
    for (unsigned k = bid_ * blockDim.x + threadIdx.x; k < n; k += nblk_ * blockDim.x)
        nfrag += vox_count_segment(a, long_ids[k], st);
    nfrag = wave_sum_u64(nfrag);
    if ((threadIdx.x & 63) == 0 && nfrag) atomicAdd(&st->stripe[bid_ % kStripes].frag, nfrag);
}

__global__ void __launch_bounds__(256) k_vox_count(CountArgs a, DevStatus *__restrict__ st) { b_vox_count(a, st, blockIdx.x, gridDim.x); }
__global__ void __launch_bounds__(256) k_bin_count(BinArgs a, DevStatus *__restrict__ st) { b_bin_count(a, st, blockIdx.x, gridDim.x); }
__global__ void __launch_bounds__(256) k_bin_alloc(BinArgs a, DevStatus *__restrict__ st) { b_bin_alloc(a, st, blockIdx.x, gridDim.x); }
__global__ void __launch_bounds__(256) k_bin_fill(BinArgs a, DevStatus *__restrict__ st) { b_bin_fill(a, st, blockIdx.x, gridDim.x); }
template <int kMode>
__global__ void __launch_bounds__(256) k_brick_accum(AccumArgs a, DevStatus *__restrict__ st) { b_brick_accum<kMode>(a, st, blockIdx.x, gridDim.x); }
__global__ void __launch_bounds__(256) k_vox_long(CountArgs a, const uint32_t *__restrict__ long_ids, DevStatus *__restrict__ st) { b_vox_long(a, long_ids, st, blockIdx.x, gridDim.x); }

// One workgroup compacts the touched-brick flags of bricks [first, last) into
// the ascending list of occupied bricks, starting at list position carry0;
// writes each brick's slot (or -1) and clears the flags.  Rounds of 16 flags
// per thread (coalesced), a block-wide exclusive scan of the per-thread counts
// and a running carry keep the list in brick order.  Returns the position
// after the range (in every thread).
__device__ __forceinline__ unsigned compact_range(uint8_t *__restrict__ flag, int64_t nb, int64_t first, int64_t last,
                                                  unsigned carry0, int32_t *__restrict__ list,
                                                  int32_t *__restrict__ slot) {
    __shared__ unsigned wtot[16];
    __shared__ unsigned carry;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = blockDim.x >> 6;
    if (t == 0) carry = carry0;
    __syncthreads();
    for (int64_t base = first; base < last; base += (int64_t)blockDim.x * 16) {
        const int64_t b0 = base + (int64_t)t * 16;
        uint8_t f[16];
        if (b0 + 16 <= nb) {
            const uint4 q = *reinterpret_cast<const uint4 *>(flag + b0);
            const uint32_t qq[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int k = 0; k < 16; ++k) f[k] = (uint8_t)(qq[k >> 2] >> (8 * (k & 3)));
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) f[k] = b0 + k < nb ? flag[b0 + k] : 0;
        }
        unsigned cnt = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) cnt += f[k] ? 1u : 0u;
        unsigned incl = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        if (lane == 63) wtot[w] = incl;
        __syncthreads();
        unsigned pos = carry + incl - cnt, round = 0;
        for (int k = 0; k < nw; ++k) {
            if (k < w) pos += wtot[k];
            round += wtot[k];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int64_t b = b0 + k;
            if (b >= nb) break;
            if (f[k]) {
                list[pos] = (int32_t)b;
                slot[b] = (int32_t)pos;
                ++pos;
                flag[b] = 0;
            } else {
                slot[b] = -1;
            }
        }
        __syncthreads();
        if (t == 0) carry += round;
        __syncthreads();
    }
    return carry;
}

// Single workgroup over all bricks (the batched form's path).
__device__ __forceinline__ void b_brick_compact(uint8_t *__restrict__ flag, int64_t nb,
                                                int32_t *__restrict__ list, int32_t *__restrict__ slot,
                                                DevStatus *__restrict__ st, unsigned bid_, unsigned nblk_) {
    const unsigned n = compact_range(flag, nb, 0, nb, 0u, list, slot);
    if (threadIdx.x == 0) st->n_bricks = n;
}

// The per-context path: one workgroup per chunk of kCompactChunk bricks,
// first counting each chunk's touched bricks, then compacting every chunk at
// the position after the chunks before it.
constexpr int kCompactChunk = 1024 * 16;

__global__ void __launch_bounds__(1024) k_compact_count(const uint8_t *__restrict__ flag, int64_t nb,
                                                        uint32_t *__restrict__ chunk_cnt) {
    __shared__ unsigned wsum[16];
    const int64_t b0 = (int64_t)blockIdx.x * kCompactChunk + (int64_t)threadIdx.x * 16;
    unsigned cnt = 0;
    if (b0 + 16 <= nb) {
        const uint4 q = *reinterpret_cast<const uint4 *>(flag + b0);
        const uint32_t qq[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) cnt += ((qq[k >> 2] >> (8 * (k & 3))) & 0xFFu) ? 1u : 0u;
    } else {
        for (int k = 0; k < 16; ++k) cnt += (b0 + k < nb && flag[b0 + k]) ? 1u : 0u;
    }
    cnt = (unsigned)wave_sum_u64(cnt);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned tot = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) tot += wsum[k];
        chunk_cnt[blockIdx.x] = tot;
    }
}

__global__ void __launch_bounds__(1024) k_compact_write(uint8_t *__restrict__ flag, int64_t nb,
                                                        const uint32_t *__restrict__ chunk_cnt,
                                                        int32_t *__restrict__ list, int32_t *__restrict__ slot,
                                                        DevStatus *__restrict__ st) {
    __shared__ unsigned base;
    if (threadIdx.x == 0) {
        unsigned s = 0;
        for (unsigned k = 0; k < blockIdx.x; ++k) s += chunk_cnt[k];
        base = s;
    }
    __syncthreads();
    const int64_t first = (int64_t)blockIdx.x * kCompactChunk;
    const int64_t last = first + kCompactChunk < nb ? first + kCompactChunk : nb;
    const unsigned end = compact_range(flag, nb, first, last, base, list, slot);
    if (threadIdx.x == 0 && blockIdx.x + 1 == gridDim.x) st->n_bricks = end;
}

// One workgroup (512 threads) per occupied brick: level-0 occupancy (saturated
// at 1.0; a voxel with 256 or more fragments is full) and the in-brick mips
// 1..3, each parent floor((sum of 8 children + 4) / 8).
__device__ __forceinline__ void b_occ_brick(const uint32_t *__restrict__ words,
                                                   const int32_t *__restrict__ list, DevStatus *__restrict__ st,
                                                   uint16_t *__restrict__ occ0, uint16_t *__restrict__ occ1,
                                                   uint16_t *__restrict__ occ2, uint16_t *__restrict__ occ3,
                                                   uint32_t *__restrict__ occ_list, unsigned bid_, unsigned nblk_) {
    __shared__ uint16_t s0[512];
    __shared__ uint16_t s1[64];
    __shared__ uint16_t s2[8];
    __shared__ unsigned wcnt[8];
    __shared__ unsigned base;
    const unsigned nbk = st->n_bricks;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    // this block's bricks: one contiguous range of slots, so that the occupied
    // list takes one atomic per block (same-address atomics serialize)
    const unsigned per = (nbk + nblk_ - 1) / nblk_;
    const unsigned sl0 = bid_ * per < nbk ? bid_ * per : nbk, sl1 = sl0 + per < nbk ? sl0 + per : nbk;
    if (sl0 >= sl1) return;  // the whole block
    unsigned occ_t = 0;
    for (unsigned sl = sl0; sl < sl1; ++sl) occ_t += (words[(int64_t)list[sl] * kBrickVox + t] & 0xFFFFu) != 0u;
    occ_t = (unsigned)wave_sum_u64(occ_t);
    if (lane == 0) wcnt[w] = occ_t;
    __syncthreads();
    if (t == 0) {
        unsigned tot = 0;
        for (int k = 0; k < 8; ++k) tot += wcnt[k];
        base = tot ? atomicAdd(&st->n_occ, tot) : 0u;
    }
    __syncthreads();
    unsigned run = base;  // the block's next occupied-list position (same in every thread)
    unsigned long long csum = 0;  // count fields seen by this thread
    for (unsigned sl = sl0; sl < sl1; ++sl) {
        int64_t b = list[sl];
        uint32_t wd = words[b * kBrickVox + t];
        uint32_t cnt = wd & 0xFFFFu, sum = wd >> 16;
        csum += cnt;
        uint16_t o = (uint16_t)(cnt >= 256u ? 256u : (sum > 256u ? 256u : sum));
        occ0[b * kBrickVox + t] = o;
        s0[t] = o;
        // append the brick's occupied voxels (x-fastest inside the brick) to the occupied list
        const unsigned long long m = __ballot(cnt != 0u);
        if (lane == 0) wcnt[w] = (unsigned)__popcll(m);
        __syncthreads();
        if (cnt) {
            unsigned pos = run + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
            for (int k = 0; k < w; ++k) pos += wcnt[k];
            occ_list[pos] = (uint32_t)(b * kBrickVox + t);
        }
        for (int k = 0; k < 8; ++k) run += wcnt[k];
        if (t < 64) {
            int X = t & 3, Y = (t >> 2) & 3, Z = t >> 4;
            unsigned s = 0;
            for (int k = 0; k < 8; ++k)
                s += s0[((2 * Z + (k >> 2)) << 6) | ((2 * Y + ((k >> 1) & 1)) << 3) | (2 * X + (k & 1))];
            uint16_t p = (uint16_t)((s + 4u) >> 3);
            s1[t] = p;
            occ1[b * 64 + t] = p;
        }
        __syncthreads();
        if (t < 8) {
            int X = t & 1, Y = (t >> 1) & 1, Z = t >> 2;
            unsigned s = 0;
            for (int k = 0; k < 8; ++k)
                s += s1[((2 * Z + (k >> 2)) << 4) | ((2 * Y + ((k >> 1) & 1)) << 2) | (2 * X + (k & 1))];
            uint16_t p = (uint16_t)((s + 4u) >> 3);
            s2[t] = p;
            occ2[b * 8 + t] = p;
        }
        __syncthreads();
        if (t == 0) {
            unsigned s = 0;
            for (int k = 0; k < 8; ++k) s += s2[k];
            occ3[b] = (uint16_t)((s + 4u) >> 3);
        }
        __syncthreads();
    }
    csum = wave_sum_u64(csum);
    if (lane == 0 && csum) atomicAdd(&st->stripe[bid_ % kStripes].csum, csum);
}

__global__ void __launch_bounds__(512) k_occ_brick(const uint32_t *__restrict__ words,
                                                   const int32_t *__restrict__ list, DevStatus *__restrict__ st,
                                                   uint16_t *__restrict__ occ0, uint16_t *__restrict__ occ1,
                                                   uint16_t *__restrict__ occ2, uint16_t *__restrict__ occ3,
                                                   uint32_t *__restrict__ occ_list) { b_occ_brick(words, list, st, occ0, occ1, occ2, occ3, occ_list, blockIdx.x, gridDim.x); }

// Level-0 occupancy of any voxel (0 outside the grid and in empty bricks).
__device__ __forceinline__ unsigned occ_at(const GridArgs &g, const uint16_t *__restrict__ occ0,
                                           const int32_t *__restrict__ slot, int x, int y, int z) {
    if (x < 0 || y < 0 || z < 0 || x >= g.G[0] || y >= g.G[1] || z >= g.G[2]) return 0;
    int64_t b = brick_index_of(x, y, z, g.nb[0], g.nb[1]);
    if (slot[b] < 0) return 0;
    return occ0[b * kBrickVox + local_of(x, y, z)];
}

// Erosion (Section 3.2): the minimum occupancy over the voxel and its 6 face
// neighbours; the voxel blocks culling rays when that minimum is full.  Also
// marks bricks and 64^3 cells holding a blocking voxel and the blocking box.
__device__ __forceinline__ void b_erode(GridArgs g, const uint16_t *__restrict__ occ0,
                                               const int32_t *__restrict__ list, const int32_t *__restrict__ slot,
                                               DevStatus *__restrict__ st, uint8_t *__restrict__ blk,
                                               uint64_t *__restrict__ blk_bits, uint32_t *__restrict__ brick_bits,
                                               uint8_t *__restrict__ super_blk, unsigned bid_, unsigned nblk_) {
    __shared__ int bb[6];
    __shared__ unsigned m2[8];
    const unsigned nbk = st->n_bricks;
    const int t = threadIdx.x;
    // pass 1 is complete: total the fragment stripes; a count field wrapped iff
    // the fields sum to less than the fragments
    if (bid_ == 0 && t < 64) {
        const unsigned long long f = wave_sum_u64(t < kStripes ? st->stripe[t].frag : 0ull);
        const unsigned long long c = wave_sum_u64(t < kStripes ? st->stripe[t].csum : 0ull);
        if (t == 0) {
            st->n_fragments = f;
            if (c != f) set_err(st, kErrCount);
        }
    }
    // box of the blocking voxels of all this workgroup's bricks, added to the
    // stripes once at the end
    if (t < 3) bb[t] = INT_MAX;
    else if (t < 6) bb[t] = INT_MIN;
    __syncthreads();
    for (unsigned sl = bid_; sl < nbk; sl += nblk_) {
        int64_t b = list[sl];
        int bx, by, bz;
        brick_xyz((uint32_t)b, g.nb, bx, by, bz);
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
        const unsigned long long bits = __ballot(blocking);  // the wave holds local voxels 64w .. 64w + 63
        if ((t & 63) == 0) blk_bits[b * 16 + (t >> 6)] = bits;
        {  // the slice's 2x2 squares holding a blocker: bit 4 Y + X for square (X, Y)
            unsigned long long c = bits | (bits >> 1);
            c |= c >> 8;  // bit 16 Y + 2 X: the square's OR
            const int lane = t & 63;
            const unsigned long long sq = __ballot(lane < 16 && ((c >> (16 * (lane >> 2) + 2 * (lane & 3))) & 1ull));
            if (lane == 0) m2[t >> 6] = (unsigned)sq & 0xFFFFu;
        }
        if (bits) {  // the wave's box first, then one LDS update per wave
            int v[6] = {blocking ? x : INT_MAX, blocking ? y : INT_MAX, blocking ? z : INT_MAX,
                        blocking ? x : INT_MIN, blocking ? y : INT_MIN, blocking ? z : INT_MIN};
            for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int lo = __shfl_xor(v[k], o, 64), hi = __shfl_xor(v[3 + k], o, 64);
                    v[k] = lo < v[k] ? lo : v[k];
                    v[3 + k] = hi > v[3 + k] ? hi : v[3 + k];
                }
            }
            if ((t & 63) == 0) {
                atomicMin(&bb[0], v[0]); atomicMin(&bb[1], v[1]); atomicMin(&bb[2], v[2]);
                atomicMax(&bb[3], v[3]); atomicMax(&bb[4], v[4]); atomicMax(&bb[5], v[5]);
            }
        }
        int any = __syncthreads_or(blocking ? 1 : 0);
        if (t == 0 && any) {
            uint64_t cells = 0;  // bit 16 Z + 4 Y + X for the 2^3 cell (X, Y, Z)
            for (int Z = 0; Z < 4; ++Z) cells |= (uint64_t)(m2[2 * Z] | m2[2 * Z + 1]) << (16 * Z);
            blk_bits[b * 16 + 8] = cells;
            atomicOr(&brick_bits[b >> 5], 1u << (b & 31));
            const CellFlagLayout cl = cell_flag_layout(g.nb);
            const int64_t c16 = ((int64_t)(bz >> 1) * cl.n16[1] + (by >> 1)) * cl.n16[0] + (bx >> 1);
            atomicOr(&brick_bits[cl.w16 + (c16 >> 5)], 1u << (c16 & 31));
            super_blk[((int64_t)(bz >> 3) * g.ns[1] + (by >> 3)) * g.ns[0] + (bx >> 3)] = 1;
            super_blk[cl.b32 + ((int64_t)(bz >> 2) * cl.n32[1] + (by >> 2)) * cl.n32[0] + (bx >> 2)] = 1;
        }
        __syncthreads();
    }
    if (t == 0 && bb[0] <= bb[3]) {
        int *p = st->stripe[bid_ % kStripes].bbox;
        atomicMin(&p[0], bb[0]); atomicMin(&p[1], bb[1]); atomicMin(&p[2], bb[2]);
        atomicMax(&p[3], bb[3]); atomicMax(&p[4], bb[4]); atomicMax(&p[5], bb[5]);
    }
}

__global__ void __launch_bounds__(512) k_erode(GridArgs g, const uint16_t *__restrict__ occ0,
                                               const int32_t *__restrict__ list, const int32_t *__restrict__ slot,
                                               DevStatus *__restrict__ st, uint8_t *__restrict__ blk,
                                               uint64_t *__restrict__ blk_bits, uint32_t *__restrict__ brick_bits,
                                               uint8_t *__restrict__ super_blk) { b_erode(g, occ0, list, slot, st, blk, blk_bits, brick_bits, super_blk, blockIdx.x, gridDim.x); }

// Averaging step on dense grids (levels >= 3): parent = floor((sum of the
// children inside the grid + 4) / 8), parent dims = ceil(child dims / 2).
__device__ __forceinline__ void b_mip_avg(const uint16_t *__restrict__ src, int sx, int sy, int sz, uint16_t *__restrict__ dst, int dx,
                          int dy, int dz, unsigned bid_, unsigned nblk_) {
    int64_t i = (int64_t)bid_ * blockDim.x + threadIdx.x;
    if (i >= (int64_t)dx * dy * dz) return;
    int x = (int)(i % dx), y = (int)((i / dx) % dy), z = (int)(i / ((int64_t)dx * dy));
    unsigned s = 0;
    for (int k = 0; k < 8; ++k) {
        int cx = 2 * x + (k & 1), cy = 2 * y + ((k >> 1) & 1), cz = 2 * z + (k >> 2);
        if (cx < sx && cy < sy && cz < sz) s += src[((int64_t)cz * sy + cy) * sx + cx];
    }
    dst[i] = (uint16_t)((s + 4u) >> 3);
}

// Occupancy levels L0, L0 + 1, ... from level L0 - 1 (src, sx x sy x sz), by
// one block, level after level.
__device__ void mip_avg_levels(int L0, const uint16_t *src, int sx, int sy, int sz, uint16_t *hi,
                               const Level *levels, int n_levels) {
    for (int L = L0; L < n_levels; ++L) {
        const Level &lv = levels[L];
        uint16_t *dst = hi + lv.offset;
        const int64_t n = (int64_t)lv.dims[0] * lv.dims[1] * lv.dims[2];
        for (unsigned vb = 0; (int64_t)vb * blockDim.x < n; ++vb)
            b_mip_avg(src, sx, sy, sz, dst, lv.dims[0], lv.dims[1], lv.dims[2], vb, 0u);
        __syncthreads();
        src = dst;
        sx = lv.dims[0];
        sy = lv.dims[1];
        sz = lv.dims[2];
    }
}

// Regions of the occupancy tree: one per 8^3 cells of level 4.
__host__ __device__ inline unsigned mip_tree_regions(const Level *levels) {
    const Level &l4 = levels[4];
    return (unsigned)(((l4.dims[0] + 7) / 8) * ((l4.dims[1] + 7) / 8) * ((l4.dims[2] + 7) / 8));
}

// Occupancy levels 4..7 from the dense level 3 (nb bricks per axis).  Block
// vb (of mip_tree_regions) takes an 8^3 region of level 4 and averages it up
// to level 7 in LDS: the regions of level 4 + k are aligned (8 >> k)^3 blocks
// of cells, so every parent's children lie in its block.  Levels above 7 are
// left to mip_avg_levels.
__device__ void b_mip_avg_tree(const uint16_t *__restrict__ occ3, const int *nb, uint16_t *__restrict__ hi,
                               const Level *levels, int n_levels, unsigned vb) {
    __shared__ uint16_t s[512 + 64 + 8];
    const Level &l4 = levels[4];
    const int nrx = (l4.dims[0] + 7) / 8, nry = (l4.dims[1] + 7) / 8;
    const int ox = (int)(vb % nrx), oy = (int)((vb / nrx) % nry), oz = (int)(vb / ((unsigned)nrx * nry));
    for (int t = threadIdx.x; t < 512; t += blockDim.x) {
        const int x = ox * 8 + (t & 7), y = oy * 8 + ((t >> 3) & 7), z = oz * 8 + (t >> 6);
        unsigned v = 0;
        if (x < l4.dims[0] && y < l4.dims[1] && z < l4.dims[2]) {
            unsigned sum = 0;
            for (int k = 0; k < 8; ++k) {
                const int cx = 2 * x + (k & 1), cy = 2 * y + ((k >> 1) & 1), cz = 2 * z + (k >> 2);
                if (cx < nb[0] && cy < nb[1] && cz < nb[2]) sum += occ3[((int64_t)cz * nb[1] + cy) * nb[0] + cx];
            }
            v = (sum + 4u) >> 3;
            hi[l4.offset + ((int64_t)z * l4.dims[1] + y) * l4.dims[0] + x] = (uint16_t)v;
        }
        s[t] = (uint16_t)v;
    }
    __syncthreads();
    int in = 0, out = 512;  // LDS offsets of the child and parent cells
    for (int k = 1; k <= 3 && 4 + k < n_levels; ++k) {
        const int m = 8 >> k, cm = 2 * m;  // cells per region axis: parent, child
        const Level &lc = levels[3 + k], &lv = levels[4 + k];
        for (int t = threadIdx.x; t < m * m * m; t += blockDim.x) {
            const int lx = t % m, ly = (t / m) % m, lz = t / (m * m);
            const int x = ox * m + lx, y = oy * m + ly, z = oz * m + lz;
            unsigned v = 0;
            if (x < lv.dims[0] && y < lv.dims[1] && z < lv.dims[2]) {
                unsigned sum = 0;
                for (int c = 0; c < 8; ++c) {
                    const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
                    if (2 * x + dx < lc.dims[0] && 2 * y + dy < lc.dims[1] && 2 * z + dz < lc.dims[2])
                        sum += s[in + ((2 * lz + dz) * cm + (2 * ly + dy)) * cm + 2 * lx + dx];
                }
                v = (sum + 4u) >> 3;
                hi[lv.offset + ((int64_t)z * lv.dims[1] + y) * lv.dims[0] + x] = (uint16_t)v;
            }
            s[out + t] = (uint16_t)v;
        }
        __syncthreads();
        in = out;
        out += m * m * m;
    }
}

__global__ void __launch_bounds__(512) k_mip_avg_tree(const uint16_t *__restrict__ occ3, GridArgs g,
                                                      uint16_t *__restrict__ hi, LevelChain ch) {
    b_mip_avg_tree(occ3, g.nb, hi, ch.lv, ch.n, blockIdx.x);
}

// Occupancy levels above 7, from level 7, by one block.
__device__ void b_mip_avg_top(uint16_t *__restrict__ hi, const Level *levels, int n_levels) {
    const Level &l7 = levels[7];
    mip_avg_levels(8, hi + l7.offset, l7.dims[0], l7.dims[1], l7.dims[2], hi, levels, n_levels);
}

__global__ void __launch_bounds__(1024) k_mip_avg_top(uint16_t *__restrict__ hi, LevelChain ch) {
    b_mip_avg_top(hi, ch.lv, ch.n);
}

}  // namespace

// Arguments of every voxelization kernel for one frame of context c.
struct VoxPlan {
    int64_t nb, ns, nv;
    int64_t nw, nf;  // words of the brick and 16^3 cell bits, bytes of the 64^3 and 32^3 cell flags
    bool fp16;
    GridArgs g;
    IngestArgs ia;
    CountArgs ca;
    BinArgs ba;
    AccumArgs aa;
};

static VoxPlan make_vox_plan(const vrt_ctx *c, const vrt_lines *L, float s_q) {
    const Arenas &A = c->a;
    VoxPlan p;
    for (int k = 0; k < 3; ++k) {
        p.g.G[k] = c->dims[k];
        p.g.nb[k] = c->dims[k] / 8;
        p.g.ns[k] = (c->dims[k] + 63) / 64;
    }
    p.nb = (int64_t)p.g.nb[0] * p.g.nb[1] * p.g.nb[2];
    p.ns = (int64_t)p.g.ns[0] * p.g.ns[1] * p.g.ns[2];
    const CellFlagLayout cl = cell_flag_layout(p.g.nb);
    p.nw = cl.words;
    p.nf = cl.bytes;
    p.nv = L->n_vertices;
    p.fp16 = c->desc.form == VRT_FORM_FP16;
    p.ia.xyz = L->xyz;
    p.ia.off = L->poly_offsets;
    p.ia.np = L->n_polylines;
    p.ia.nv = L->n_vertices;
    for (int k = 0; k < 3; ++k) p.ia.o[k] = c->origin[k];
    p.ia.s = s_q;
    p.ca.vrec = A.vrec;
    p.ca.nv = L->n_vertices;
    p.ca.mode = c->voxelizer;
    p.ca.rq = c->rq;
    const int64_t rcl = c->rq > kRMinQ ? c->rq : kRMinQ;
    const double ratio = (double)c->rq / (double)rcl;
    p.ca.rc = (float)rcl;
    p.ca.corr = (float)(ratio * ratio);
    for (int k = 0; k < 3; ++k) p.ca.G[k] = c->dims[k];
    p.ca.nbx = c->dims[0] / 8;
    p.ca.nby = c->dims[1] / 8;
    p.ca.words = A.words;
    p.ca.brick_flag = A.brick_flag;
    p.ba.vrec = A.vrec;
    p.ba.nv = L->n_vertices;
    p.ba.rq = c->rq;
    for (int k = 0; k < 3; ++k) {
        p.ba.G[k] = p.g.G[k];
        p.ba.nb[k] = p.g.nb[k];
    }
    p.ba.bin_count = A.bin_count;
    p.ba.bin_range = A.bin_range;
    p.ba.cand = A.cand;
    p.ba.bins = A.bins;
    p.ba.bin_cap = (int64_t)kMaxBinBricks * c->desc.max_vertices;
    p.ba.long_ids = A.long_ids;
    p.ba.items = A.items;
    p.aa.ca = p.ca;
    p.aa.items = A.items;
    p.aa.bin_range = A.bin_range;
    p.aa.bins = A.bins;
    return p;
}

// Workgroups of the per-brick passes (grid-stride over the binned bricks).
static constexpr unsigned kBrickBlocks = 8192;

hipError_t launch_voxelize(vrt_ctx *c, const vrt_lines *L, float s_q, hipStream_t st) {
    Arenas &A = c->a;
    const VoxPlan p = make_vox_plan(c, L, s_q);
    const unsigned eb = (unsigned)((p.nv + 255) / 256);
    VRT_LAUNCH(c, "k_clear_prev", st, k_clear_prev<<<2048, 128, 0, st>>>(A.words, A.brick_list, A.status));
    VRT_LAUNCH(c, "k_reset", st,
               k_reset<<<(unsigned)((reset_items(p.nb, p.nw, p.nf) + 255) / 256), 256, 0, st>>>(
                   A.occ3, A.bin_count, A.brick_bits, p.nb, p.nw, A.super_blk, p.nf, A.status));
    VRT_LAUNCH(c, "k_ingest", st, k_ingest<<<eb, 256, 0, st>>>(p.ia, A.vrec, A.status));
    if (p.fp16) VRT_LAUNCH(c, "k_pack16", st, k_pack16<<<eb, 256, 0, st>>>(A.vrec, p.nv, A.srec16));
    VRT_LAUNCH(c, "k_bin_count", st, k_bin_count<<<eb, 256, 0, st>>>(p.ba, A.status));
    VRT_LAUNCH(c, "k_bin_alloc", st, k_bin_alloc<<<64, 256, 0, st>>>(p.ba, A.status));
    VRT_LAUNCH(c, "k_bin_fill", st, k_bin_fill<<<eb, 256, 0, st>>>(p.ba, A.status));
    if (c->voxelizer == VRT_VOX_THIN)
        VRT_LAUNCH(c, "k_brick_accum", st, k_brick_accum<VRT_VOX_THIN><<<kBrickBlocks, 256, 0, st>>>(p.aa, A.status));
    else if (c->voxelizer == VRT_VOX_AABB)
        VRT_LAUNCH(c, "k_brick_accum", st, k_brick_accum<VRT_VOX_AABB><<<kBrickBlocks, 256, 0, st>>>(p.aa, A.status));
    else
        VRT_LAUNCH(c, "k_brick_accum", st, k_brick_accum<VRT_VOX_CAPSULE><<<kBrickBlocks, 256, 0, st>>>(p.aa, A.status));
    VRT_LAUNCH(c, "k_vox_long", st, k_vox_long<<<256, 256, 0, st>>>(p.ca, A.long_ids, A.status));
    const unsigned nchunks = (unsigned)((p.nb + kCompactChunk - 1) / kCompactChunk);
    VRT_LAUNCH(c, "k_compact_count", st,
               k_compact_count<<<nchunks, 1024, 0, st>>>(A.brick_flag, p.nb, A.chunk_cnt));
    VRT_LAUNCH(c, "k_compact_write", st,
               k_compact_write<<<nchunks, 1024, 0, st>>>(A.brick_flag, p.nb, A.chunk_cnt, A.brick_list, A.brick_slot,
                                                         A.status));
    VRT_LAUNCH(c, "k_occ_brick", st,
               k_occ_brick<<<1024, 512, 0, st>>>(A.words, A.brick_list, A.status, A.occ0, A.occ1, A.occ2, A.occ3,
                                                 A.occ_list));
    VRT_LAUNCH(c, "k_erode", st,
               k_erode<<<4096, 512, 0, st>>>(p.g, A.occ0, A.brick_list, A.brick_slot, A.status, A.blk, A.blk_bits,
                                             A.brick_bits, A.super_blk));
    // levels >= 4 from the dense level 3
    if (c->n_levels > 4) {
        LevelChain ch;
        ch.n = c->n_levels;
        for (int L = 0; L < kMaxLevels; ++L) ch.lv[L] = c->levels[L];
        VRT_LAUNCH(c, "k_mip_avg_tree", st,
                   k_mip_avg_tree<<<mip_tree_regions(ch.lv), 512, 0, st>>>(A.occ3, p.g, A.occ_hi, ch));
        if (c->n_levels > 8) VRT_LAUNCH(c, "k_mip_avg_top", st, k_mip_avg_top<<<1, 1024, 0, st>>>(A.occ_hi, ch));
    }
    return hipGetLastError();
}

}  // namespace vrt
