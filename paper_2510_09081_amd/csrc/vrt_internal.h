// vrt_internal.h -- shared declarations of the HIP implementation (not part of the ABI).
#pragma once

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

struct DevStatus {
    unsigned int err;
    unsigned int n_bricks;
    unsigned long long n_fragments;
    unsigned long long n_listed;
    int bbox[6];  // blocking-voxel bounds: min x,y,z then max x,y,z (voxels)
    unsigned int pad[4];
};

struct Arenas {
    VRec *vrec = nullptr;
    uint32_t *words = nullptr;      // [max_bricks * 512]
    uint16_t *occ0 = nullptr;       // [max_bricks * 512]
    uint16_t *occ1 = nullptr;       // [max_bricks * 64]
    uint16_t *occ2 = nullptr;       // [max_bricks * 8]
    uint16_t *occ3 = nullptr;       // [max_bricks]
    uint16_t *occ_hi = nullptr;     // levels >= 4
    uint8_t *blk = nullptr;         // [max_bricks * 512]
    uint8_t *brick_blk = nullptr;   // [max_bricks]
    uint8_t *vis0 = nullptr;        // [max_bricks * 512]
    uint8_t *vis1 = nullptr;        // [max_bricks * 64]
    uint8_t *vis2 = nullptr;        // [max_bricks * 8]
    uint8_t *vis3 = nullptr;        // [max_bricks]
    uint8_t *vis_hi = nullptr;      // levels >= 4
    uint32_t *cursor = nullptr;     // [max_bricks * 512] list start, then end after pass 2
    uint32_t *ids = nullptr;        // [max_fragments]
    uint8_t *brick_flag = nullptr;  // [max_bricks]
    int32_t *brick_list = nullptr;  // [max_bricks]
    int32_t *brick_slot = nullptr;  // [max_bricks] slot in brick_list or -1
    uint32_t *brick_total = nullptr;// [max_bricks] visible fragments per occupied brick (by slot)
    uint32_t *brick_base = nullptr; // [max_bricks] exclusive scan of brick_total
    DevStatus *status = nullptr;
};

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

}  // namespace vrt

struct vrt_ctx {
    vrt_desc desc;
    int64_t max_bricks;
    int64_t hi_elems;  // capacity of occ_hi / vis_hi
    vrt::Arenas a;
    // frame state
    bool voxelized = false, culled = false;
    int dims[3] = {0, 0, 0};
    int n_levels = 0;
    vrt::Level levels[vrt::kMaxLevels];
    int64_t n_vertices = 0;
    int64_t rq = 0;
    float origin[3] = {0, 0, 0};
    float voxel_size = 1;
    hipStream_t last_stream = nullptr;
    vrt::Profiler prof;
};

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
struct TraceParams {
    float F[3], R[3], U[3];  // camera basis: forward, right*tan*aspect, up*tan
    float O[3];              // eye in voxel units (exact)
    int W, H;
    int mode;
    float alpha, tau;
    float radius;            // voxel units
    float voxel_size;
};
hipError_t launch_trace(vrt_ctx *c, const TraceParams &p, const vrt_image *img, hipStream_t st);
hipError_t launch_debug_rays(const TraceParams &p, const int64_t *pix, int64_t n, float *dirs, hipStream_t st);

// ------------------------------------------------------------------------
// device helpers

__device__ __forceinline__ int64_t brick_index_of(int x, int y, int z, int nbx, int nby) {
    return ((int64_t)(z >> 3) * nby + (y >> 3)) * nbx + (x >> 3);
}
__device__ __forceinline__ int local_of(int x, int y, int z) { return ((z & 7) << 6) | ((y & 7) << 3) | (x & 7); }

// floor(n / m) for m > 0, exact: a binary64 estimate corrected in integers.
__device__ __forceinline__ long long floor_div(long long n, long long m) {
    long long q = (long long)floor((double)n / (double)m);
    while (q * m > n) --q;
    while ((q + 1) * m <= n) ++q;
    return q;
}

// smallest w >= 0 with w*w >= n
__device__ __forceinline__ long long ceil_isqrt(long long n) {
    if (n <= 0) return 0;
    long long w = (long long)sqrt((double)n);
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
// minor axes.  Calls f(x, y, z) for every voxel, each exactly once.
struct SlabSpan {
    int a0, a1, a2;
    long long A[3], d[3], D;
    long long lo[3], hi[3];
    int vlo[3], vhi[3];
    long long W1, W2;
    bool empty;
};

__device__ __forceinline__ SlabSpan make_span(int3 a, int3 b, long long rq, const int *G) {
    SlabSpan s;
    long long A[3] = {a.x, a.y, a.z}, B[3] = {b.x, b.y, b.z};
    long long d[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    long long ad[3] = {d[0] < 0 ? -d[0] : d[0], d[1] < 0 ? -d[1] : d[1], d[2] < 0 ? -d[2] : d[2]};
    int a0 = 0;
    if (ad[1] > ad[a0]) a0 = 1;
    if (ad[2] > ad[a0]) a0 = 2;
    bool swap = d[a0] < 0;
    for (int c = 0; c < 3; ++c) {
        s.A[c] = swap ? B[c] : A[c];
        s.d[c] = swap ? -d[c] : d[c];
    }
    s.a0 = a0;
    s.a1 = a0 == 0 ? 1 : 0;
    s.a2 = a0 == 2 ? 1 : 2;
    s.D = s.d[a0];
    s.empty = false;
    for (int c = 0; c < 3; ++c) {
        long long mn = A[c] < B[c] ? A[c] : B[c], mx = A[c] < B[c] ? B[c] : A[c];
        s.lo[c] = mn - rq;
        s.hi[c] = mx + rq;
        long long vl = floor_div(s.lo[c] - 1, kQ), vh = floor_div(s.hi[c], kQ);
        if (vl < 0) vl = 0;
        if (vh > G[c] - 1) vh = G[c] - 1;
        s.vlo[c] = (int)vl;
        s.vhi[c] = (int)vh;
        if (vl > vh) s.empty = true;
    }
    s.W1 = s.W2 = 0;
    if (s.D > 0) {
        s.W1 = ceil_isqrt(rq * rq * (s.D * s.D + s.d[s.a1] * s.d[s.a1]));
        s.W2 = ceil_isqrt(rq * rq * (s.D * s.D + s.d[s.a2] * s.d[s.a2]));
    }
    return s;
}

// minor-axis voxel range of slab x on axis i with half-width W
__device__ __forceinline__ void slab_range(const SlabSpan &s, int x, int i, long long W, int &rl, int &rh) {
    if (s.D == 0) {
        rl = s.vlo[i];
        rh = s.vhi[i];
        return;
    }
    long long ta = s.lo[s.a0] > (long long)x * kQ ? s.lo[s.a0] : (long long)x * kQ;
    long long tb = s.hi[s.a0] < (long long)(x + 1) * kQ ? s.hi[s.a0] : (long long)(x + 1) * kQ;
    long long ca = s.A[i] * s.D + s.d[i] * (ta - s.A[s.a0]);
    long long cb = s.A[i] * s.D + s.d[i] * (tb - s.A[s.a0]);
    long long nlo = (ca < cb ? ca : cb) - W, nhi = (ca < cb ? cb : ca) + W;
    long long m = s.D * kQ;
    long long l = floor_div(nlo - 1, m), h = floor_div(nhi, m);
    rl = (int)(l > s.vlo[i] ? l : s.vlo[i]);
    rh = (int)(h < s.vhi[i] ? h : s.vhi[i]);
}

template <class F>
__device__ __forceinline__ int for_each_voxel(const SlabSpan &s, F &&f) {
    if (s.empty) return 0;
    int n = 0;
    for (int x = s.vlo[s.a0]; x <= s.vhi[s.a0]; ++x) {
        int l1, h1, l2, h2;
        slab_range(s, x, s.a1, s.W1, l1, h1);
        slab_range(s, x, s.a2, s.W2, l2, h2);
        for (int j = l1; j <= h1; ++j)
            for (int k = l2; k <= h2; ++k) {
                int C[3];
                C[s.a0] = x;
                C[s.a1] = j;
                C[s.a2] = k;
                f(C[0], C[1], C[2]);
                ++n;
            }
    }
    return n;
}

}  // namespace vrt
