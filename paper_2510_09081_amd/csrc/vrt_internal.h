// vrt_internal.h -- shared declarations of the HIP implementation (not part of the ABI).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vrt.h"

namespace vrt {

constexpr int kQ = 256;            // fixed-point steps per voxel
constexpr int kRMinQ = 128;        // PWAA minimum radius: half a voxel (Alg. 3)
constexpr int kBrick = 8;          // brick edge in voxels
constexpr int kBrickVox = 512;     // voxels per brick
constexpr int kMaxLevels = 12;     // 1024 -> 1 needs 11 halvings

// device status bits
constexpr unsigned kErrInvalid = 1u, kErrRange = 2u, kErrCapacity = 4u, kErrCount = 8u;

// Vertex record: quantized position, flags and binary32 clip normal (32 B).
// flags bit 0: the vertex starts a segment; bit 1: interior vertex (clip plane).
struct __align__(16) VRec {
    int x, y, z, flags;
    float nx, ny, nz, pad;
};
constexpr int kSegValid = 1, kInterior = 2;

// FP16-form segment record (32 B): endpoints as binary16 offsets (voxel units)
// from the centre of brick (bx, by, bz), clip normals as 16-bit signed
// fixed point (n * 32767: a unit vector's components keep an absolute error
// below 2^-16, where binary16 would leave up to 2^-12), flags bit 0:
// interior A (clip with n0), bit 1: interior B (clip with n1), bit 2: an
// offset is 8 voxels or more, where binary16 no longer holds every multiple
// of 1/256 voxel -- the tracer then reads the segment's plain vertex records.
struct __align__(16) SRec16 {
    __half a[3], b[3];
    short n0[3], n1[3];
    short bx, by, bz;
    unsigned short flags;
};
static_assert(sizeof(SRec16) == 32, "SRec16 is 32 bytes");
constexpr unsigned kSRecPlain = 4u;

// Device-wide atomics on one cache line serialize (about 11 ns each on
// MI355X), so per-block tallies go to the stripe of their block (one 128-byte
// line each) and the readers combine the stripes.
constexpr int kStripes = 64;
struct alignas(128) StatStripe {
    unsigned long long frag;  // pass-1 fragments
    unsigned long long csum;  // sum of the 16-bit count fields
    int bbox[6];              // blocking-voxel bounds
    int vbox[6];              // visible-brick bounds
    unsigned long long vvis;  // visible voxels (those with a list)
};

struct DevStatus {
    unsigned int err;
    unsigned int n_bricks;
    unsigned long long n_fragments;  // final value (sum of the stripes, written after pass 1)
    unsigned long long n_listed;
    unsigned int n_occ;  // occupied voxels (entries of occ_list)
    int vbox[6];         // visible-brick bounds: min bx,by,bz then max (bricks), combined at trace start
    unsigned int n_queue;  // rays queued by the trace's march phase
    unsigned int n_cont;   // queued rays whose walk stopped at the limit, resumed after the shade phase
    unsigned int n_cand;           // bricks with a non-empty segment bin (entries of cand)
    unsigned int n_long;           // segments too long for the bins (entries of long_ids)
    unsigned long long bin_total;  // bin entries allocated
    unsigned int n_items;          // (brick, chunk) work items of the per-brick passes
    StatStripe stripe[kStripes];
};

// A segment is binned into every brick of its voxel box when that box has at
// most this many bricks; longer segments take the per-segment path.
constexpr int kMaxBinBricks = 8;
// Walk entries per pixel of max_pixels: the trace's walk phase gives every
// queued ray walk_entries / n_queue entries (at most kWalkMax), so rays are
// walked in full unless most pixels reach a list.
constexpr int kWalkPerPixel = 8;  // at least 4: a ray's slot also holds its resume state (32 B)
constexpr int kWalkMax = 4096;
// Bins are processed in chunks of at most this many segments (one workgroup
// each), so that crowded bricks are spread over several workgroups.
constexpr int kBinChunk = 1024;
// Words between the bin counters of consecutive bricks: each counter has a
// 128-byte line of its own, so that device atomics on different bricks'
// counters do not queue behind each other.
constexpr int kBinStride = 32;

// Workgroup order for launches whose neighbouring work items read the same
// data.  The workgroups of a launch go to the eight XCDs in turn (workgroup b
// to XCD b mod 8) and each XCD has an L2 of its own, so consecutive items
// would be spread over all eight L2s.  A kernel that takes item
// xcd_order(b, nb) (+ multiples of nb) in workgroup b gives each XCD runs of
// kXcdChunk consecutive items, the XCDs' runs interleaved (run c of XCD x is
// the (8c + x)-th), so each L2 sees neighbouring items and every XCD still
// takes a share of every part of the item list.  Identity when nb does not
// split evenly.
constexpr unsigned kXcdChunk = 64;
__device__ __forceinline__ unsigned xcd_order(unsigned b, unsigned nb) {
    if (nb % (8u * kXcdChunk) != 0u) return b;
    const unsigned x = b % 8u, j = b / 8u;
    return ((j / kXcdChunk) * 8u + x) * kXcdChunk + j % kXcdChunk;
}

// Index of the k-th item of a chunk in the order its workgroup reads it:
// within every group of 64, lane L takes entry 8 (L % 8) + L / 8, so that the
// lanes of a wave take segments eight apart in the bin (consecutive segments
// of a polyline share voxels, and LDS atomics on one address serialize).
__device__ __forceinline__ uint32_t spread64(uint32_t u) {
    const uint32_t l = u & 63u;
    return (u & ~63u) | ((l & 7u) << 3) | (l >> 3);
}

struct Arenas {
    VRec *vrec = nullptr;
    uint32_t *words = nullptr;      // [max_bricks * 512]
    uint16_t *occ0 = nullptr;       // [max_bricks * 512]
    uint16_t *occ1 = nullptr;       // [max_bricks * 64]
    uint16_t *occ2 = nullptr;       // [max_bricks * 8]
    uint16_t *occ3 = nullptr;       // [max_bricks]
    uint16_t *occ_hi = nullptr;     // levels >= 4
    uint8_t *blk = nullptr;         // [max_bricks * 512]
    uint64_t *blk_bits = nullptr;   // [max_bricks * 16] per brick: words 0..7 blocking voxels, one bit each
                                    // (64 voxels per word), word 8 its 2^3 cells holding a blocker
    uint32_t *brick_bits = nullptr; // [cell_flag_layout(max).words] bricks and 16^3 cells holding a blocker, one bit each
    uint8_t *super_blk = nullptr;   // [cell_flag_layout(max).bytes] 64^3 and 32^3 cells holding a blocker
    uint32_t *occ_list = nullptr;   // [max_bricks * 512] brick-major index of every occupied voxel
    uint8_t *vis0 = nullptr;        // [max_bricks * 512]
    uint8_t *vis1 = nullptr;        // [max_bricks * 64]
    uint8_t *vis2 = nullptr;        // [max_bricks * 8]
    uint8_t *vis3 = nullptr;        // [max_bricks]
    uint8_t *bskip = nullptr;       // [max_bricks] 0: visible brick, else the shift of the largest invisible cell holding it
    uint8_t *vis_hi = nullptr;      // levels >= 4
    uint32_t *cursor = nullptr;     // [max_bricks * 512] list start, then end after pass 2
    uint64_t *cell = nullptr;       // [max_bricks * 512] list start (low 32) | visible count (high 32)
    uint64_t *lmask = nullptr;      // [max_bricks * 8] voxels with a non-empty list, one bit each (64 per word)
    uint64_t *lmask2 = nullptr;     // [max_bricks] 2^3 cells holding such a voxel, bit 16 Z + 4 Y + X
    uint4 *queue = nullptr;         // [max_pixels] rays that reached a list
    uint2 *walk = nullptr;          // [walk_entries] list voxels of the queued rays, in walk order (voxel, entry t)
    uint32_t *cont = nullptr;       // [max_pixels] queued rays resumed after the walk limit
    SRec16 *srec16 = nullptr;       // [max_vertices] FP16-form segment records (FP16 form only)
    uint32_t *ids = nullptr;        // [max_fragments]
    uint8_t *brick_flag = nullptr;  // [max_bricks]
    uint32_t *bin_count = nullptr;  // [max_bricks * kBinStride] segments binned per brick, brick b at b * kBinStride (zero between frames)
    uint2 *bin_range = nullptr;     // [max_bricks] (first entry, length) of a brick's bin in bins
    int32_t *cand = nullptr;        // [max_bricks] bricks with a non-empty bin, in no particular order
    uint32_t *bins = nullptr;       // [kMaxBinBricks * max_vertices] segment ids grouped by brick
    uint32_t *long_ids = nullptr;   // [max_vertices] segments whose voxel box spans more bricks
    uint2 *items = nullptr;         // (brick, chunk) work items of the per-brick passes
    uint32_t *chunk_cnt = nullptr;  // touched bricks per compaction chunk
    int32_t *brick_list = nullptr;  // [max_bricks]
    int32_t *brick_slot = nullptr;  // [max_bricks] slot in brick_list or -1
    uint32_t *brick_total = nullptr;// [max_bricks] visible fragments per occupied brick (by slot)
    uint32_t *brick_base = nullptr; // [max_bricks] exclusive scan of brick_total
    DevStatus *status = nullptr;
    // trace statistics (inspection only)
    float *lit = nullptr;                   // [max_bricks * 512] voxel-space shading of the visible voxels
    uint8_t *stat_vox = nullptr;            // [max_bricks * 512] voxel list read
    uint8_t *stat_seg = nullptr;            // [max_vertices] segment tested
    unsigned long long *stat_acc = nullptr; // [16]
};

// Grid extents shared by the per-brick kernels.
struct GridArgs {
    int G[3];
    int nb[3];  // bricks per axis
    int ns[3];  // 64^3 cells per axis
};

// Brick coordinates of brick index b, x fastest.  Grids are at most 1024
// voxels a side, so b < 2^21 and 32-bit division is exact (64-bit division
// is a long emulated sequence).
__device__ __forceinline__ void brick_xyz(uint32_t b, const int *nb, int &bx, int &by, int &bz) {
    const uint32_t n0 = (uint32_t)nb[0], n1 = (uint32_t)nb[1];
    const uint32_t q = b / n0;
    bx = (int)(b - q * n0);
    bz = (int)(q / n1);
    by = (int)(q - (uint32_t)bz * n1);
}

// Blocker flags above the voxel level, each array x fastest.  Bits, in one
// word array: one per brick, then one per 16^3 cell (2^3 bricks) from word
// w16.  Bytes, in one byte array: one per 64^3 cell, then one per 32^3 cell
// (4^3 bricks) from byte b32.
struct CellFlagLayout {
    int n16[3], n32[3], n64[3];
    int64_t w16, words;
    int64_t b32, bytes;
};
__host__ __device__ inline CellFlagLayout cell_flag_layout(const int *nb) {
    CellFlagLayout c;
    int64_t tb = 1, t16 = 1, t32 = 1, t64 = 1;
    for (int k = 0; k < 3; ++k) {
        c.n16[k] = (nb[k] + 1) / 2;
        c.n32[k] = (nb[k] + 3) / 4;
        c.n64[k] = (nb[k] + 7) / 8;
        tb *= nb[k];
        t16 *= c.n16[k];
        t32 *= c.n32[k];
        t64 *= c.n64[k];
    }
    c.w16 = (tb + 31) / 32;
    c.words = c.w16 + (t16 + 31) / 32;
    c.b32 = t64;
    c.bytes = t64 + t32;
    return c;
}

// Event-pair profiler (host side); disabled unless vrt_profile_enable.
struct Profiler {
    static constexpr int kMaxPairs = 65536;
    bool enabled = false;
    hipEvent_t *ev = nullptr;  // 2 * kMaxPairs
    const char **names = nullptr;
    int used = 0;
    bool overflow = false;
};

struct Level {
    int dims[3];
    int64_t offset;  // element offset into occ_hi / vis_hi (levels >= 4)
};

// The level table, passed to kernels by value.
struct LevelChain {
    int n;
    Level lv[kMaxLevels];
};

}  // namespace vrt

struct vrt_ctx {
    vrt_desc desc;
    int64_t max_bricks;
    int64_t max_supers;
    int64_t hi_elems;  // capacity of occ_hi / vis_hi
    int64_t walk_entries;  // capacity of walk, shared by the queued rays of a trace
    vrt::Arenas a;
    // frame state
    bool voxelized = false, culled = false, shaded = false;
    int dims[3] = {0, 0, 0};
    int n_levels = 0;
    vrt::Level levels[vrt::kMaxLevels];
    int64_t n_vertices = 0;
    int64_t rq = 0;
    int voxelizer = VRT_VOX_CAPSULE;    // membership of the current frame
    const float *seg_rgba = nullptr;     // per-segment colour and opacity of the current frame, or null
    float alpha_default = 0.0f;          // opacity of segments without their own colour (0: the camera's)
    float origin[3] = {0, 0, 0};
    float voxel_size = 1;
    hipStream_t last_stream = nullptr;
    vrt::Profiler prof;
    vrt_tune tune[2] = {{256, 16, 2, 4, 4096, {0, 0, 0}}, {256, 16, 2, 4, 4096, {0, 0, 0}}};  // per trace mode
};

namespace vrt {
// Elements of occ_hi / vis_hi that the current grid's levels >= 4 use.
inline int64_t hi_used(const vrt_ctx *c) {
    if (c->n_levels <= 4) return 0;
    const Level &l = c->levels[c->n_levels - 1];
    return l.offset + (int64_t)l.dims[0] * l.dims[1] * l.dims[2];
}
}  // namespace vrt

namespace vrt {

// ------------------------------------------------------------------------
// kernel timing brackets (no-ops unless profiling is enabled)

inline void prof_begin(vrt_ctx *c, const char *name, hipStream_t st) {
    Profiler &p = c->prof;
    if (!p.enabled) return;
    if (p.used >= Profiler::kMaxPairs) {
        p.overflow = true;
        return;
    }
    p.names[p.used] = name;
    (void)hipEventRecord(p.ev[2 * p.used], st);
}
inline void prof_end(vrt_ctx *c, hipStream_t st) {
    Profiler &p = c->prof;
    if (!p.enabled || p.used >= Profiler::kMaxPairs) return;
    (void)hipEventRecord(p.ev[2 * p.used + 1], st);
    ++p.used;
}

#define VRT_LAUNCH(ctx, name, stream, ...)  \
    do {                                     \
        ::vrt::prof_begin(ctx, name, stream); \
        __VA_ARGS__;                         \
        ::vrt::prof_end(ctx, stream);        \
    } while (0)

// ------------------------------------------------------------------------
// launchers (each file owns its kernels)

hipError_t launch_voxelize(vrt_ctx *c, const vrt_lines *lines, float s_q, hipStream_t st);
hipError_t launch_cull(vrt_ctx *c, const int64_t eye_q[3], int64_t limit, hipStream_t st);
hipError_t launch_sort_lists(vrt_ctx *c, hipStream_t st);
vrt_status shade_params(const vrt_ctx *c, const vrt_shading *s, int *U, int *L);
hipError_t launch_shade(vrt_ctx *c, const vrt_shading *s, const int *U, const int *L, hipStream_t st);
struct TraceParams {
    float F[3], R[3], U[3];  // camera basis: forward, right*tan*aspect, up*tan
    float O[3];              // eye in voxel units (exact)
    int W, H;
    int mode;
    float alpha, tau;
    float radius;            // voxel units
    float voxel_size;
    const float4 *seg_rgba;  // per-segment colour and opacity, or null (colour = |unit tangent|, opacity alpha)
    const float *lit;        // voxel-space shading of the hit's voxel (brick-major), or null (unshaded)
};
hipError_t launch_trace(vrt_ctx *c, const TraceParams &p, const vrt_image *img, hipStream_t st);
hipError_t launch_trace_stats(vrt_ctx *c, const TraceParams &p, const vrt_image *img, hipStream_t st);
bool tune_valid(const vrt_tune &t);
hipError_t launch_debug_rays(const TraceParams &p, const int64_t *pix, int64_t n, float *dirs, hipStream_t st);

// ------------------------------------------------------------------------
// device helpers

__device__ __forceinline__ int64_t brick_index_of(int x, int y, int z, int nbx, int nby) {
    return ((int64_t)(z >> 3) * nby + (y >> 3)) * nbx + (x >> 3);
}
__device__ __forceinline__ int local_of(int x, int y, int z) { return ((z & 7) << 6) | ((y & 7) << 3) | (x & 7); }

// floor(n / m) for 0 < m, |n| + m < 2^52 and |n / m| < 2^20 (voxel indices),
// exact, with no binary64 arithmetic: the binary32 estimate from n, m and the
// hardware reciprocal has a relative error below 2^-21, hence an absolute
// error below one half at these quotients, and is corrected by one exact
// 64-bit integer comparison each way (|q m| stays below |n| + 2m < 2^53).
__device__ __forceinline__ long long floor_div(long long n, long long m) {
    long long q = (long long)floorf((float)n * __builtin_amdgcn_rcpf((float)m));
    if (q * m > n) q -= 1;
    else if ((q + 1) * m <= n) q += 1;
    return q;
}

// smallest w >= 0 with w*w >= n (n < 2^62), exact: a binary32 square root
// estimate corrected by exact 64-bit integer comparisons
__device__ __forceinline__ long long ceil_isqrt(long long n) {
    if (n <= 0) return 0;
    long long w = (long long)__builtin_amdgcn_sqrtf((float)n);
    while (w * w < n) ++w;
    while (w > 0 && (w - 1) * (w - 1) >= n) --w;
    return w;
}

__device__ __forceinline__ void set_err(DevStatus *s, unsigned bit) { atomicOr(&s->err, bit); }

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Capsule voxel set of one segment (Section 3.1, Alg. 1 with the projected
// radius that is conservative in 3D): per major-axis slab, a 2D box on the
// minor axes.  Calls f(x, y, z) for every voxel, each exactly once.  The span
// is kept in axis-permuted scalars (index 0 = major axis a0, 1 and 2 = the
// minor axes a1 < a2): runtime-indexed arrays would live in per-lane scratch.
struct SlabSpan {
    int mode;  // VRT_VOX_*: the capsule set, or a comparison voxelizer's
    int a0, a1, a2;
    long long A0, A1, A2;  // start point on (a0, a1, a2) after the swap
    long long D, d1, d2;   // direction on (a0, a1, a2), D >= 0
    long long lo0, hi0;    // closed capsule extent along a0
    int vlo0, vhi0, vlo1, vhi1, vlo2, vhi2;  // voxel ranges
    long long W1, W2;      // half-widths scaled by D
    bool empty;
};

__device__ __forceinline__ long long sel3(long long x, long long y, long long z, int k) {
    return k == 0 ? x : (k == 1 ? y : z);
}

__device__ __forceinline__ SlabSpan make_span(int3 a, int3 b, long long rq, const int *G, int mode) {
    SlabSpan s;
    s.mode = mode;
    const long long dx = (long long)b.x - a.x, dy = (long long)b.y - a.y, dz = (long long)b.z - a.z;
    const long long ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy, az = dz < 0 ? -dz : dz;
    int a0 = 0;
    long long am = ax;
    if (ay > am) {
        a0 = 1;
        am = ay;
    }
    if (az > am) a0 = 2;
    s.a0 = a0;
    s.a1 = a0 == 0 ? 1 : 0;
    s.a2 = a0 == 2 ? 1 : 2;
    const bool swap = sel3(dx, dy, dz, a0) < 0;
    const long long sx = swap ? b.x : a.x, sy = swap ? b.y : a.y, sz = swap ? b.z : a.z;
    const long long ex = swap ? -dx : dx, ey = swap ? -dy : dy, ez = swap ? -dz : dz;
    s.A0 = sel3(sx, sy, sz, s.a0);
    s.A1 = sel3(sx, sy, sz, s.a1);
    s.A2 = sel3(sx, sy, sz, s.a2);
    s.D = sel3(ex, ey, ez, s.a0);
    s.d1 = sel3(ex, ey, ez, s.a1);
    s.d2 = sel3(ex, ey, ez, s.a2);
    // closed capsule AABB and the voxel range touching it, per original axis
    const long long lox = (a.x < b.x ? a.x : b.x) - rq, hix = (a.x < b.x ? b.x : a.x) + rq;
    const long long loy = (a.y < b.y ? a.y : b.y) - rq, hiy = (a.y < b.y ? b.y : a.y) + rq;
    const long long loz = (a.z < b.z ? a.z : b.z) - rq, hiz = (a.z < b.z ? b.z : a.z) + rq;
    long long vlx = (lox - 1) >> 8, vhx = hix >> 8;  // floor division by kQ = 256
    long long vly = (loy - 1) >> 8, vhy = hiy >> 8;
    long long vlz = (loz - 1) >> 8, vhz = hiz >> 8;
    vlx = vlx < 0 ? 0 : vlx;
    vly = vly < 0 ? 0 : vly;
    vlz = vlz < 0 ? 0 : vlz;
    vhx = vhx > G[0] - 1 ? G[0] - 1 : vhx;
    vhy = vhy > G[1] - 1 ? G[1] - 1 : vhy;
    vhz = vhz > G[2] - 1 ? G[2] - 1 : vhz;
    s.empty = vlx > vhx || vly > vhy || vlz > vhz;
    s.lo0 = sel3(lox, loy, loz, s.a0);
    s.hi0 = sel3(hix, hiy, hiz, s.a0);
    s.vlo0 = (int)sel3(vlx, vly, vlz, s.a0);
    s.vhi0 = (int)sel3(vhx, vhy, vhz, s.a0);
    s.vlo1 = (int)sel3(vlx, vly, vlz, s.a1);
    s.vhi1 = (int)sel3(vhx, vhy, vhz, s.a1);
    s.vlo2 = (int)sel3(vlx, vly, vlz, s.a2);
    s.vhi2 = (int)sel3(vhx, vhy, vhz, s.a2);
    s.W1 = s.W2 = 0;
    if (s.D > 0) {
        s.W1 = ceil_isqrt(rq * rq * (s.D * s.D + s.d1 * s.d1));
        s.W2 = ceil_isqrt(rq * rq * (s.D * s.D + s.d2 * s.d2));
    }
    return s;
}

// Minor-axis voxel range of slab x: the segment's line at the slab's ends
// (ta, tb), widened by W (numerators scaled by D), clipped to [vlo, vhi].
__device__ __forceinline__ void slab_range(const SlabSpan &s, int x, long long A, long long d, long long W, int vlo,
                                           int vhi, int &rl, int &rh) {
    if (s.D == 0) {
        rl = vlo;
        rh = vhi;
        return;
    }
    const long long ta = s.lo0 > (long long)x * kQ ? s.lo0 : (long long)x * kQ;
    const long long tb = s.hi0 < (long long)(x + 1) * kQ ? s.hi0 : (long long)(x + 1) * kQ;
    const long long ca = A * s.D + d * (ta - s.A0);
    const long long cb = A * s.D + d * (tb - s.A0);
    const long long nlo = (ca < cb ? ca : cb) - W, nhi = (ca < cb ? cb : ca) + W;
    const long long m = s.D * kQ;
    const long long l = floor_div(nlo - 1, m), h = floor_div(nhi, m);
    rl = (int)(l > vlo ? l : vlo);
    rh = (int)(h < vhi ? h : vhi);
}

// Thin-line comparison voxelizer (Section 4.1, the "DDA" of Table 2): the
// voxels whose open interior the open segment meets, plus the cells of its
// endpoints, inside the box given on the span's axes.  An exact integer walk
// from the start cell: the next crossing on each axis is the fraction
// num/den of the segment (den = |d|), the smallest one is taken next, tied
// axes step together (voxels touched only along an edge or at a corner are
// not entered), and the walk ends before a crossing at or past the far end,
// whose cell is added when it differs.  A segment lying in a voxel face
// plane meets no open interior: only its endpoint cells.
template <class F>
__device__ __forceinline__ int for_each_thin_voxel(const SlabSpan &s, int lo0, int hi0, int lo1, int hi1, int lo2,
                                                   int hi2, F &&f) {
    const long long A0 = s.A0, A1 = s.A1, A2 = s.A2;
    const long long d0 = s.D, d1 = s.d1, d2 = s.d2;
    long long c0 = A0 >> 8, c1 = A1 >> 8, c2 = A2 >> 8;  // floor division by kQ = 256
    const long long e0 = (A0 + d0) >> 8, e1 = (A1 + d1) >> 8, e2 = (A2 + d2) >> 8;
    int n = 0;
    auto emit = [&](long long x, long long j, long long k) {
        if (x < lo0 || x > hi0 || j < lo1 || j > hi1 || k < lo2 || k > hi2) return;
        const int vx = s.a0 == 0 ? (int)x : (s.a1 == 0 ? (int)j : (int)k);
        const int vy = s.a0 == 1 ? (int)x : (s.a1 == 1 ? (int)j : (int)k);
        const int vz = s.a0 == 2 ? (int)x : (s.a1 == 2 ? (int)j : (int)k);
        f(vx, vy, vz);
        ++n;
    };
    emit(c0, c1, c2);
    const bool flat = (d0 == 0 && (A0 & 255) == 0) || (d1 == 0 && (A1 & 255) == 0) || (d2 == 0 && (A2 & 255) == 0);
    if (d0 != 0 && !flat) {  // d0 = |major component| > 0: not a point
        // distance (numerator) to the next plane on each axis; den = |d|, 0 when the axis never steps
        long long n0 = (c0 + 1) * kQ - A0;  // d0 > 0
        long long n1 = d1 > 0 ? (c1 + 1) * kQ - A1 : A1 - c1 * kQ;
        long long n2 = d2 > 0 ? (c2 + 1) * kQ - A2 : A2 - c2 * kQ;
        const long long g1 = d1 < 0 ? -d1 : d1, g2 = d2 < 0 ? -d2 : d2;
        const int s1 = d1 > 0 ? 1 : -1, s2 = d2 > 0 ? 1 : -1;
        for (;;) {
            // smallest crossing fraction among the stepping axes (axis 0 always steps)
            long long bn = n0, bd = d0;
            if (g1 && n1 * bd < bn * g1) bn = n1, bd = g1;
            if (g2 && n2 * bd < bn * g2) bn = n2, bd = g2;
            if (!(bn < bd)) break;  // at or past the far end
            const bool t0 = n0 * bd == bn * d0, t1 = g1 && n1 * bd == bn * g1, t2 = g2 && n2 * bd == bn * g2;
            if (t0) c0 += 1, n0 += kQ;
            if (t1) c1 += s1, n1 += kQ;
            if (t2) c2 += s2, n2 += kQ;
            emit(c0, c1, c2);
        }
    }
    if (c0 != e0 || c1 != e1 || c2 != e2) emit(e0, e1, e2);
    return n;
}

// The voxels of the set inside the box [lo0, hi0] x [lo1, hi1] x [lo2, hi2]
// given on the span's axes (a0, a1, a2); each exactly once.  kMode: the
// membership mode when known at compile time (the per-brick kernels are
// instantiated per mode), -1 to read it from the span.
template <int kMode = -1, class F>
__device__ __forceinline__ int for_each_voxel_clip(const SlabSpan &s, int lo0, int hi0, int lo1, int hi1, int lo2,
                                                   int hi2, F &&f) {
    const int mode = kMode >= 0 ? kMode : s.mode;
    if (s.empty) return 0;
    if (mode == VRT_VOX_THIN) {
        const int b0 = s.vlo0 > lo0 ? s.vlo0 : lo0, b1 = s.vlo1 > lo1 ? s.vlo1 : lo1, b2 = s.vlo2 > lo2 ? s.vlo2 : lo2;
        const int u0 = s.vhi0 < hi0 ? s.vhi0 : hi0, u1 = s.vhi1 < hi1 ? s.vhi1 : hi1, u2 = s.vhi2 < hi2 ? s.vhi2 : hi2;
        return for_each_thin_voxel(s, b0, u0, b1, u1, b2, u2, f);
    }
    int n = 0;
    const int x0 = s.vlo0 > lo0 ? s.vlo0 : lo0, x1 = s.vhi0 < hi0 ? s.vhi0 : hi0;
    for (int x = x0; x <= x1; ++x) {
        int l1 = s.vlo1, h1 = s.vhi1, l2 = s.vlo2, h2 = s.vhi2;  // the capsule AABB voxelizer: the whole box
        if (mode == VRT_VOX_CAPSULE) {
            slab_range(s, x, s.A1, s.d1, s.W1, s.vlo1, s.vhi1, l1, h1);
            slab_range(s, x, s.A2, s.d2, s.W2, s.vlo2, s.vhi2, l2, h2);
        }
        l1 = l1 > lo1 ? l1 : lo1;
        h1 = h1 < hi1 ? h1 : hi1;
        l2 = l2 > lo2 ? l2 : lo2;
        h2 = h2 < hi2 ? h2 : hi2;
        for (int j = l1; j <= h1; ++j)
            for (int k = l2; k <= h2; ++k) {
                // (x, j, k) on axes (a0, a1, a2) back to (x, y, z)
                const int vx = s.a0 == 0 ? x : (s.a1 == 0 ? j : k);
                const int vy = s.a0 == 1 ? x : (s.a1 == 1 ? j : k);
                const int vz = s.a0 == 2 ? x : (s.a1 == 2 ? j : k);
                f(vx, vy, vz);
                ++n;
            }
    }
    return n;
}

template <int kMode = -1, class F>
__device__ __forceinline__ int for_each_voxel(const SlabSpan &s, F &&f) {
    return for_each_voxel_clip<kMode>(s, s.vlo0, s.vhi0, s.vlo1, s.vhi1, s.vlo2, s.vhi2, f);
}

// The voxels of the set inside brick (bx, by, bz).
template <int kMode = -1, class F>
__device__ __forceinline__ int for_each_voxel_in_brick(const SlabSpan &s, int bx, int by, int bz, F &&f) {
    const int l0 = 8 * (int)sel3(bx, by, bz, s.a0), l1 = 8 * (int)sel3(bx, by, bz, s.a1);
    const int l2 = 8 * (int)sel3(bx, by, bz, s.a2);
    return for_each_voxel_clip<kMode>(s, l0, l0 + 7, l1, l1 + 7, l2, l2 + 7, f);
}

// Voxel box of the set on the original axes.
__device__ __forceinline__ void span_box(const SlabSpan &s, int &lx, int &hx, int &ly, int &hy, int &lz, int &hz) {
    lx = s.a0 == 0 ? s.vlo0 : (s.a1 == 0 ? s.vlo1 : s.vlo2);
    hx = s.a0 == 0 ? s.vhi0 : (s.a1 == 0 ? s.vhi1 : s.vhi2);
    ly = s.a0 == 1 ? s.vlo0 : (s.a1 == 1 ? s.vlo1 : s.vlo2);
    hy = s.a0 == 1 ? s.vhi0 : (s.a1 == 1 ? s.vhi1 : s.vhi2);
    lz = s.a0 == 2 ? s.vlo0 : (s.a1 == 2 ? s.vlo1 : s.vlo2);
    hz = s.a0 == 2 ? s.vhi0 : (s.a1 == 2 ? s.vhi1 : s.vhi2);
}

// Appends `val` to list[] for every lane with p set, one counter update per
// wave.  Called by all lanes of the wave together.
template <class T>
__device__ __forceinline__ void wave_append(bool p, T val, unsigned *counter, T *list) {
    const unsigned long long m = __ballot(p);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(counter, (unsigned)__popcll(m));
    base = __shfl(base, leader, 64);
    if (p) list[base + (unsigned)__popcll(m & ((1ull << lane) - 1ull))] = val;
}
}  // namespace vrt
