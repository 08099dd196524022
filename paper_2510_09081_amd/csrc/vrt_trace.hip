// vrt_trace.hip -- Section 3.5: voxel ray tracing through the per-voxel lists.
#include <climits>

#include "vrt_internal.h"

namespace vrt {
namespace {

// Shade-phase launch shape (all points give identical images):
//   G  lanes that share one ray (8, 16 or 32),
//   B  list entries per lane whose vertex records are fetched together (2 or 4),
//   K  accepted (t, id) keys a lane keeps per pass in transparent mode (4 or 8).
template <int G, int B, int K>
struct ShadeCfg {
    static constexpr int kGroup = G, kBatch = B, kLaneKeys = K;
    static_assert(G == 8 || G == 16 || G == 32, "group");
};
using DefaultShade = ShadeCfg<16, 2, 4>;
constexpr int kMaxShadeGroups = 64;  // groups per block: at most 512 threads of 8-lane groups

// Primary ray through the centre of pixel (px, py), row 0 at the top, as a
// fixed binary32 sequence (no contraction): u = 2(x + .5)/W - 1,
// v = 1 - 2(y + .5)/H, d = (F + u R) + v U, D = d / |d|.
__device__ __forceinline__ float3 primary_dir(const TraceParams &p, int px, int py) {
    float u = (2.0f * ((float)px + 0.5f)) / (float)p.W - 1.0f;
    float v = 1.0f - (2.0f * ((float)py + 0.5f)) / (float)p.H;
    float d0 = (p.F[0] + u * p.R[0]) + v * p.U[0];
    float d1 = (p.F[1] + u * p.R[1]) + v * p.U[1];
    float d2 = (p.F[2] + u * p.R[2]) + v * p.U[2];
    float ss = d0 * d0;
    ss = ss + d1 * d1;
    ss = ss + d2 * d2;
    float len = sqrtf(ss);
    return make_float3(d0 / len, d1 / len, d2 / len);
}

__device__ __forceinline__ float dot3(float3 a, float3 b) {
    float s = a.x * b.x;
    s = fmaf(a.y, b.y, s);
    return fmaf(a.z, b.z, s);
}
__device__ __forceinline__ float3 sub3(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }

// Hit geometry uses the hardware reciprocal and square root (about one ulp
// each): hit parameters only need to stay within the binary32 error margins
// that decide which pixels are compared exactly, while the primary rays keep
// the correctly rounded sequence.
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float fsqrt(float a) { return __builtin_amdgcn_sqrtf(a); }

// Entry root of |oc + t D| = r (unit D): smaller root, stable form.
__device__ __forceinline__ float sphere_entry(float3 oc, float3 D, float r2) {
    float b = dot3(oc, D);
    float c = dot3(oc, oc) - r2;
    float h = b * b - c;
    if (h < 0.0f) return -INFINITY;
    float sq = fsqrt(h);
    float q = b >= 0.0f ? -(b + sq) : (sq - b);
    return b >= 0.0f ? q : fdiv(c, q);
}

__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Ray-capsule entry after Quilez's capsule intersector: the infinite
// cylinder's entry root if it falls on the body, else the end sphere on that
// side; -inf on a miss.  The quadratic's terms are taken from cross products
// (Lagrange's identity) instead of differences of dot products, which keeps
// the hit/miss decision accurate to binary32 rounding for thin capsules:
//   w = D x ba, u = oa x ba,
//   a = |w|^2, b = w.u, c = |u|^2 - r^2 |ba|^2,
//   b^2 - a c = |ba|^2 (r^2 |w|^2 - (oa.w)^2).
// A capsule of radius 0 has no interior and is never hit.
__device__ __forceinline__ float capsule_entry(float3 ro, float3 D, float3 pa, float3 pb, float r) {
    if (!(r > 0.0f)) return -INFINITY;
    const float3 ba = sub3(pb, pa), oa = sub3(ro, pa);
    const float baba = dot3(ba, ba);
    const float r2 = r * r;
    // The three ways to an end sphere (a point segment, a ray parallel to the
    // axis, an entry beyond an end) share one sphere test, so that lanes of a
    // wave taking different ways run it together.
    float3 oc = oa;
    if (baba != 0.0f) {
        const float3 w = cross3(D, ba), u = cross3(oa, ba);
        const float ww = dot3(w, w);
        const float bard = dot3(ba, D), baoa = dot3(ba, oa);
        const float c = dot3(u, u) - r2 * baba;
        if (ww == 0.0f) {  // parallel to the axis: inside the cylinder or a miss
            if (c > 0.0f) return -INFINITY;
            if (!(bard > 0.0f)) oc = sub3(ro, pb);
        } else {
            const float ow = dot3(oa, w);
            const float g = r2 * ww - ow * ow;
            if (g < 0.0f) return -INFINITY;  // misses the infinite cylinder, hence the capsule
            const float b = dot3(w, u);
            const float sq = fsqrt(baba * g);
            const float t = fdiv(b >= 0.0f ? -(b + sq) : c, b >= 0.0f ? ww : sq - b);  // the stable root
            const float y = baoa + t * bard;
            if (y > 0.0f && y < baba) return t;
            if (!(y <= 0.0f)) oc = sub3(ro, pb);
        }
    }
    return sphere_entry(oc, D, r2);
}

struct TraceArgs {
    TraceParams p;
    int G[3];
    int nb[3];
    int n4[3], n5[3], n6[3];  // 16^3, 32^3 and 64^3 cells per axis (culling levels 4, 5, 6)
    const uint8_t *vis4, *vis5, *vis6;  // culling levels 4..6, each null when the grid has no such level
    const uint8_t *vis3;      // culling level 3 (bricks)
    uint8_t *bskip;           // per brick: 0 if visible, else log2 of the largest invisible cell holding it
    const uint64_t *cell;     // per voxel: list start | visible count << 32
    const uint64_t *lmask;    // per brick: voxels with a non-empty list (8 words, z-slice w in word w)
    const uint64_t *lmask2;   // per brick: 2^3 cells holding such a voxel
    DevStatus *st;            // visible-brick box, ray-queue length
    const uint32_t *ids;
    const VRec *vrec;
    const SRec16 *srec16;     // FP16 form only
    int64_t nv;               // vertices of the frame (ids must be < nv - 1)
    int64_t capacity;         // entries of ids
    uint4 *queue;             // rays that reached a list: pixel, packed voxel (after the walk phase: walked
                              // entries | more << 31), entry t, exit t of the visible box
    uint2 *walk;              // walk_capacity(walk_entries, n_queue) entries per queued ray: packed voxel, entry t
    int64_t walk_entries;
    uint32_t *cont;           // queued rays whose walk stopped at the limit unfinished, resumed by a later launch
    float *rgba;
    float *depth;
    int *first_id;
    uint8_t *stat_vox;        // statistics variant only
    uint8_t *stat_seg;
    unsigned long long *stat_acc;
};

struct Counters {
    unsigned long long skip64 = 0, skip8 = 0, vox = 0, list = 0, test = 0, pass = 0;
};

// A segment in the frame of voxel (cx, cy, cz): endpoints relative to the
// voxel corner (voxel units), clip normals, and which ends are clipped.
struct LocalSeg {
    float3 pa, pb, n0, n1;
    bool ia, ib;
};

__device__ __forceinline__ float3 rel(const VRec &v, int cx, int cy, int cz) {
    return make_float3((float)(v.x - cx * kQ) * (1.0f / kQ), (float)(v.y - cy * kQ) * (1.0f / kQ),
                       (float)(v.z - cz * kQ) * (1.0f / kQ));
}

// Plain form: from the two int32 vertex records (exact).
__device__ __forceinline__ LocalSeg local_seg(const VRec &A, const VRec &B, int cx, int cy, int cz) {
    LocalSeg s;
    s.pa = rel(A, cx, cy, cz);
    s.pb = rel(B, cx, cy, cz);
    s.n0 = make_float3(A.nx, A.ny, A.nz);
    s.n1 = make_float3(B.nx, B.ny, B.nz);
    s.ia = (A.flags & kInterior) != 0;
    s.ib = (B.flags & kInterior) != 0;
    return s;
}

// FP16 form: brick centre minus voxel corner (an exact small integer plus one
// half) plus the binary16 offset; the sum is exact in binary32.
__device__ __forceinline__ LocalSeg local_seg(const SRec16 &r, int cx, int cy, int cz) {
    LocalSeg s;
    const float ox = (float)(8 * (int)r.bx + 4 - cx), oy = (float)(8 * (int)r.by + 4 - cy),
                oz = (float)(8 * (int)r.bz + 4 - cz);
    s.pa = make_float3(ox + __half2float(r.a[0]), oy + __half2float(r.a[1]), oz + __half2float(r.a[2]));
    s.pb = make_float3(ox + __half2float(r.b[0]), oy + __half2float(r.b[1]), oz + __half2float(r.b[2]));
    constexpr float kSn = 1.0f / 32767.0f;
    s.n0 = make_float3((float)r.n0[0] * kSn, (float)r.n0[1] * kSn, (float)r.n0[2] * kSn);
    s.n1 = make_float3((float)r.n1[0] * kSn, (float)r.n1[1] * kSn, (float)r.n1[2] * kSn);
    s.ia = (r.flags & 1u) != 0;
    s.ib = (r.flags & 2u) != 0;
    return s;
}

// Accepted hit of a segment inside the current voxel: entry parameter s in
// [0, tl) from the voxel-local origin ro, and on the kept side of both clip
// planes ((P - A).n0 >= 0 at an interior A, (P - B).n1 < 0 at an interior B).
__device__ __forceinline__ bool voxel_hit(const LocalSeg &g, float radius, float3 ro, float3 D, float tl, float &s) {
    s = capsule_entry(ro, D, g.pa, g.pb, radius);
    if (!(s >= 0.0f && s < tl)) return false;
    const float3 P = make_float3(fmaf(s, D.x, ro.x), fmaf(s, D.y, ro.y), fmaf(s, D.z, ro.z));
    if (g.ia && !(dot3(sub3(P, g.pa), g.n0) >= 0.0f)) return false;
    if (g.ib && !(dot3(sub3(P, g.pb), g.n1) < 0.0f)) return false;
    return true;
}

// Colour = |unit tangent|, from the endpoints (identical in both forms while
// the FP16 offsets are exact).
__device__ __forceinline__ float3 seg_colour(float3 pa, float3 pb) {
    const float dx = pb.x - pa.x, dy = pb.y - pa.y, dz = pb.z - pa.z;
    const float len = fsqrt(dx * dx + dy * dy + dz * dz);
    if (len == 0.0f) return make_float3(0.0f, 0.0f, 0.0f);
    const float il = __builtin_amdgcn_rcpf(len);
    return make_float3(fabsf(dx) * il, fabsf(dy) * il, fabsf(dz) * il);
}

__device__ __forceinline__ bool key_less(float s0, uint32_t i0, float s1, uint32_t i1) {
    return s0 < s1 || (s0 == s1 && i0 < i1);
}

// Parameter of the crossing with plane `bnd` on one axis: (bnd - O) * (1/D).
// bnd - O is exact in binary32 (both are multiples of 1/256 below 2^16), and
// every boundary is computed by this one expression, so neighbouring cells
// share their boundary parameters exactly.
__device__ __forceinline__ float tcross(int bnd, float o, float inv) { return ((float)bnd - o) * inv; }

struct Ray {
    float O[3], D[3], inv[3];
    int step[3];
};

// Element m of a 3-array without a runtime-indexed access (which would place
// the array in per-lane scratch memory).
template <class T>
__device__ __forceinline__ T pick3(const T *a, int m) {
    return m == 0 ? a[0] : (m == 1 ? a[1] : a[2]);
}
template <class T>
__device__ __forceinline__ void put3(T *a, int m, T v) {
    if (m == 0) a[0] = v;
    else if (m == 1) a[1] = v;
    else a[2] = v;
}

__device__ __forceinline__ Ray make_ray(const TraceParams &p, float3 D) {
    Ray r;
    r.O[0] = p.O[0];
    r.O[1] = p.O[1];
    r.O[2] = p.O[2];
    r.D[0] = D.x;
    r.D[1] = D.y;
    r.D[2] = D.z;
    for (int k = 0; k < 3; ++k) {
        r.step[k] = r.D[k] > 0.0f ? 1 : (r.D[k] < 0.0f ? -1 : 0);
        r.inv[k] = r.step[k] == 0 ? 0.0f : 1.0f / r.D[k];
    }
    return r;
}

// Parameter interval of the ray inside the box of visible bricks.
__device__ __forceinline__ bool clip_visible(const TraceArgs &a, const Ray &r, float &tin, float &tout, int *vb) {
    for (int k = 0; k < 6; ++k) vb[k] = a.st->vbox[k];
    tin = 0.0f;
    tout = INFINITY;
    if (!(vb[0] <= vb[3] && vb[1] <= vb[4] && vb[2] <= vb[5])) return false;
    for (int k = 0; k < 3; ++k) {
        const int lo = 8 * vb[k], hi = 8 * (vb[3 + k] + 1);
        if (r.step[k] == 0) {
            if (r.O[k] < (float)lo || r.O[k] > (float)hi) return false;
            continue;
        }
        float t1 = tcross(lo, r.O[k], r.inv[k]), t2 = tcross(hi, r.O[k], r.inv[k]);
        if (t1 > t2) {
            const float tt = t1;
            t1 = t2;
            t2 = tt;
        }
        tin = fmaxf(tin, t1);
        tout = fminf(tout, t2);
    }
    return tin < tout;
}

// Index of the cell of culling level L (2^L voxels a side, n cells per axis)
// holding voxel v.
__device__ __forceinline__ int64_t coarse_index(const int *v, int L, const int *n) {
    return ((int64_t)(v[2] >> L) * n[1] + (v[1] >> L)) * n[0] + (v[0] >> L);
}

// Crosses the empty S^3 cell (S = 2^sh) holding voxel v: returns false when
// the ray leaves the grid; else v becomes the voxel entered after the cell's
// exit face (monotone in the direction of travel, clamped to the cell on the
// other axes) and tcur the exit parameter.
__device__ __forceinline__ bool skip_cell(const Ray &r, const int *G, int sh, int *v, float &tcur) {
    const int S = 1 << sh;
    int cellk[3];
    float tb[3];
    for (int k = 0; k < 3; ++k) {
        cellk[k] = v[k] >> sh;  // v >= 0
        tb[k] = r.step[k] == 0 ? INFINITY : tcross(S * (cellk[k] + (r.step[k] > 0)), r.O[k], r.inv[k]);
    }
    int m = 0;
    float tm = tb[0];
    if (tb[1] < tm) {
        m = 1;
        tm = tb[1];
    }
    if (tb[2] < tm) {
        m = 2;
        tm = tb[2];
    }
    const float te = fmaxf(tm, tcur);
    for (int k = 0; k < 3; ++k) {
        int nv;
        if (k == m) {
            nv = r.step[k] > 0 ? S * (cellk[k] + 1) : S * cellk[k] - 1;
            if (nv < 0 || nv >= G[k]) return false;
        } else {
            nv = (int)floorf(fmaf(te, r.D[k], r.O[k]));
            if (r.step[k] > 0) nv = nv < v[k] ? v[k] : nv;
            if (r.step[k] < 0) nv = nv > v[k] ? v[k] : nv;
            const int lo = S * cellk[k];
            const int hi = min(S * cellk[k] + S - 1, G[k] - 1);
            nv = nv < lo ? lo : (nv > hi ? hi : nv);
        }
        v[k] = nv;
    }
    tcur = te;
    return true;
}

// DDA state of one ray: current voxel, its entry parameter, the next boundary
// parameter on each axis (valid unless `fresh`), and the end of the walk.
struct Walk {
    int v[3];
    float tcur, tout;
    float tnext[3];
    bool fresh;
    int m;          // axis of the current voxel's exit
    float texit;    // exit parameter of the current voxel
    int64_t vi;     // brick-major index of the current voxel
    uint64_t cd;    // its list descriptor
    int64_t bvis = -1;  // a brick already found visible (its culling flags need no second look)
};

// Steps past the current voxel along its exit axis; false when the ray leaves the grid.
__device__ __forceinline__ bool step_voxel(const TraceArgs &a, const Ray &r, Walk &w) {
    const int m = w.m;
    const int st = pick3(r.step, m);
    const int nv = pick3(w.v, m) + st;
    if (nv < 0 || nv >= pick3(a.G, m)) return false;
    put3(w.v, m, nv);
    w.tcur = w.texit;
    put3(w.tnext, m, tcross(nv + (st > 0), pick3(r.O, m), pick3(r.inv, m)));
    return true;
}

// The list mask of the brick a walk is in (its z-slice words) and the mask of
// its 2^3 cells holding a list voxel, held by the walker: in registers (one
// ray per lane), or the voxel words in LDS (one ray per group of lanes, which
// all hold the same values).
struct MaskRegs {
    static constexpr bool kEarly = false;  // many rays meet invisible bricks: load only for visible ones
    static constexpr bool kCells = true;   // crosses list-free 2^3 and 4^3 cells in one jump
    uint64_t m[8];
    uint64_t c2;  // the brick's 2^3 cells holding a list voxel
    __device__ void set(const uint64_t *src, const uint64_t *cells) {
#pragma unroll
        for (int k = 0; k < 8; ++k) m[k] = src[k];
        c2 = *cells;
    }
    __device__ void put(const uint64_t *v) {
#pragma unroll
        for (int k = 0; k < 8; ++k) m[k] = v[k];
    }
    __device__ uint64_t slice(int z) const {  // selects, not an indexed register read
        const uint64_t a0 = (z & 1) ? m[1] : m[0], a1 = (z & 1) ? m[3] : m[2];
        const uint64_t a2 = (z & 1) ? m[5] : m[4], a3 = (z & 1) ? m[7] : m[6];
        const uint64_t b0 = (z & 2) ? a1 : a0, b1 = (z & 2) ? a3 : a2;
        return (z & 4) ? b1 : b0;
    }
};
// Registers, read beside the culling flags (one round trip per brick entered).
struct MaskRegsEarly : MaskRegs {
    static constexpr bool kEarly = true;
};
struct MaskLds {
    static constexpr bool kEarly = true;  // read beside the culling flags, before they are known
    static constexpr bool kCells = true;  // crosses list-free 2^3 and 4^3 cells in one jump
    uint64_t *p;  // word k at p[k * stride]
    int stride;
    uint64_t c2 = 0;  // the brick's 2^3 cells holding a list voxel (in registers)
    __device__ void set(const uint64_t *src, const uint64_t *) {
        uint64_t m[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) m[k] = src[k];
        put(m);
    }
    __device__ void put(const uint64_t *v) {
#pragma unroll
        for (int k = 0; k < 8; ++k) p[k * stride] = v[k];
    }
    __device__ uint64_t slice(int z) const { return p[(z & 7) * stride]; }
};

// Exit axis and exit parameter of the current voxel from its boundary
// parameters (the lowest axis wins a tie).
__device__ __forceinline__ void voxel_exit(Walk &w) {
    float tm = w.tnext[0];
    w.m = 0;
    if (w.tnext[1] < tm) {
        w.m = 1;
        tm = w.tnext[1];
    }
    if (w.tnext[2] < tm) {
        w.m = 2;
        tm = w.tnext[2];
    }
    w.texit = fmaxf(tm, w.tcur);
}

// Boundary parameters of voxel v's exit planes; every walk computes them with
// this one expression, so a voxel entered by a step, after a jump or from a
// stored walk entry has the same exit parameter.
__device__ __forceinline__ void voxel_bounds(const Ray &r, Walk &w) {
    for (int k = 0; k < 3; ++k)
        w.tnext[k] = r.step[k] == 0 ? INFINITY : tcross(w.v[k] + (r.step[k] > 0), r.O[k], r.inv[k]);
}

__device__ __forceinline__ uint32_t pack_voxel(const int *v) {
    return (uint32_t)v[0] | ((uint32_t)v[1] << 10) | ((uint32_t)v[2] << 20);
}
__device__ __forceinline__ void unpack_voxel(uint32_t p, int *v) {
    v[0] = (int)(p & 1023u);
    v[1] = (int)((p >> 10) & 1023u);
    v[2] = (int)((p >> 20) & 1023u);
}
// Brick-major index of voxel v.
__device__ __forceinline__ int64_t voxel_index(const TraceArgs &a, const int *v) {
    const int64_t b = ((int64_t)(v[2] >> 3) * a.nb[1] + (v[1] >> 3)) * a.nb[0] + (v[0] >> 3);
    return b * kBrickVox + local_of(v[0], v[1], v[2]);
}

// One step of the march from the current voxel (included) towards the first
// visible voxel with a non-empty list: an invisible cell of 8^3 to 64^3
// voxels is crossed in one jump; in a visible brick, a list-free 4^3 or 2^3
// cell is crossed in one jump and a single voxel without a list is stepped
// past on the brick's list mask (both loaded once when the walk enters the
// brick).  Returns 1 when the current voxel is such a voxel, -1 when the ray
// has left the box or the grid, 0 after a jump or step.  Every step advances
// the walk by at least one voxel.
template <bool kStats, class Mask, bool kLoadCd>
__device__ __forceinline__ int march_step(const TraceArgs &a, const Ray &r, Walk &w, Counters &cn, Mask &mk) {
    if (!(w.tcur < w.tout)) return -1;
    const int64_t b = ((int64_t)(w.v[2] >> 3) * a.nb[1] + (w.v[1] >> 3)) * a.nb[0] + (w.v[0] >> 3);
    if (b != w.bvis) {  // a new brick: its own culling flag, and its 64^3 cell's
        // both read at once; a 64^3 cell is visible iff one of its bricks is
        uint64_t m[8];  // the brick's list mask, read early by walkers that keep it
        uint64_t c2 = 0;
        if (Mask::kEarly) {
#pragma unroll
            for (int k = 0; k < 8; ++k) m[k] = a.lmask[b * 8 + k];
            c2 = a.lmask2[b];
        }
        const uint8_t v3 = a.vis3[b];
        const uint8_t v4 = a.vis4 ? a.vis4[coarse_index(w.v, 4, a.n4)] : 1;
        const uint8_t v5 = a.vis5 ? a.vis5[coarse_index(w.v, 5, a.n5)] : 1;
        const uint8_t v6 = a.vis6 ? a.vis6[coarse_index(w.v, 6, a.n6)] : 1;
        if (!v3) {  // the largest invisible cell holding the brick is crossed in one jump
            const int sh = !v6 ? 6 : (!v5 ? 5 : (!v4 ? 4 : 3));
            if (kStats) {
                if (sh == 6) ++cn.skip64;
                else ++cn.skip8;
            }
            if (!skip_cell(r, a.G, sh, w.v, w.tcur)) return -1;
            w.fresh = true;
            return 0;
        }
        if (Mask::kEarly) {
            mk.put(m);
            mk.c2 = c2;
        } else {
            mk.set(a.lmask + b * 8, a.lmask2 + b);
        }
        w.bvis = b;
    }
    if (Mask::kCells) {  // a 2^3 or 4^3 cell of the brick without list voxels is crossed in one jump
        const int xl = w.v[0] & 7, yl = w.v[1] & 7, zl = w.v[2] & 7;
        if (!((mk.c2 >> (((zl >> 1) << 4) | ((yl >> 1) << 2) | (xl >> 1))) & 1ull)) {
            const bool e4 = !(mk.c2 & (0x00330033ull << (((zl >> 2) << 5) | ((yl >> 2) << 3) | ((xl >> 2) << 1))));
            if (kStats) ++cn.skip8;
            if (!skip_cell(r, a.G, e4 ? 2 : 1, w.v, w.tcur)) return -1;
            w.fresh = true;
            return 0;
        }
    }
    if (w.fresh) {
        voxel_bounds(r, w);
        w.fresh = false;
    }
    voxel_exit(w);
    if (kStats) ++cn.vox;
    const int l = local_of(w.v[0], w.v[1], w.v[2]);
    if ((mk.slice(w.v[2]) >> (l & 63)) & 1ull) {
        w.vi = b * kBrickVox + l;
        if (kLoadCd) w.cd = a.cell[w.vi];
        return 1;
    }
    return step_voxel(a, r, w) ? 0 : -1;
}

// Steps a walk bounded by every grid dimension three times over (each step
// advances it by a voxel at least).
__device__ __forceinline__ int march_limit(const TraceArgs &a) { return 3 * (a.G[0] + a.G[1] + a.G[2]) + 16; }

// Advances from the current voxel (included) to the first visible voxel with
// a non-empty list; false if none.  kLoadCd: also read its list descriptor.
template <bool kStats, class Mask, bool kLoadCd = true>
__device__ __forceinline__ bool march(const TraceArgs &a, const Ray &r, Walk &w, Counters &cn, Mask &mk) {
    const int max_iter = march_limit(a);
    for (int it = 0; it < max_iter; ++it) {
        const int st = march_step<kStats, Mask, kLoadCd>(a, r, w, cn, mk);
        if (st != 0) return st > 0;
    }
    return false;
}

// Segment id in the frame of voxel (cx, cy, cz), read in the context's form.
template <int kForm>
__device__ __forceinline__ LocalSeg load_seg(const TraceArgs &a, uint32_t id, int cx, int cy, int cz) {
    if (kForm == VRT_FORM_FP16) {
        const SRec16 r = a.srec16[id];
        if (!(r.flags & kSRecPlain)) return local_seg(r, cx, cy, cz);
    }
    return local_seg(a.vrec[id], a.vrec[id + 1], cx, cy, cz);
}

// Colour and opacity of a hit on segment id: the caller's per-segment RGBA
// (opacity clamped to [0, 1]) when given, else |unit tangent| and the
// default opacity.
template <int kForm>
__device__ __forceinline__ float3 hit_colour(const TraceArgs &a, uint32_t id, int cx, int cy, int cz, float &alpha) {
    if (a.p.seg_rgba) {
        const float4 q = a.p.seg_rgba[id];
        alpha = fminf(fmaxf(q.w, 0.0f), 1.0f);
        return make_float3(q.x, q.y, q.z);
    }
    alpha = a.p.alpha;
    const LocalSeg g = load_seg<kForm>(a, id, cx, cy, cz);
    return seg_colour(g.pa, g.pb);
}

// hit_colour with the opacity in w.
template <int kForm>
__device__ __forceinline__ float4 hit_rgba(const TraceArgs &a, uint32_t id, int cx, int cy, int cz) {
    float alpha;
    const float3 c = hit_colour<kForm>(a, id, cx, cy, cz, alpha);
    return make_float4(c.x, c.y, c.z, alpha);
}

// Calls f(id, seg) for the entries of the current voxel's list that belong to
// lane `gl` of a kGroup-lane group (entries gl, gl + kGroup, ...).  The
// records of kBatch entries are fetched before any of them is tested, so each
// lane keeps several independent loads in flight.
template <bool kStats, int kForm, class Cfg, class F>
__device__ __forceinline__ void for_each_entry(const TraceArgs &a, const Walk &w, int gl, Counters &cn, F &&f) {
    // after a capacity overflow the lists are undefined but reads stay inside ids
    const uint32_t start = (uint32_t)w.cd, cnt = (uint32_t)(w.cd >> 32);
    const uint32_t end = (int64_t)start + cnt <= a.capacity ? start + cnt : start;
    const int cx = w.v[0], cy = w.v[1], cz = w.v[2];
    constexpr int kGroup = Cfg::kGroup, kBatch = Cfg::kBatch;
    for (uint32_t k = start + gl; k < end; k += kGroup * kBatch) {
        uint32_t id[kBatch];
        LocalSeg g[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) id[j] = k + j * kGroup < end ? a.ids[k + j * kGroup] : 0xFFFFFFFFu;
#pragma unroll
        for (int j = 0; j < kBatch; ++j) g[j] = load_seg<kForm>(a, (int64_t)id[j] + 1 < a.nv ? id[j] : 0u, cx, cy, cz);
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            if (!((int64_t)id[j] + 1 < a.nv)) continue;
            if (kStats) {
                ++cn.test;
                a.stat_seg[id[j]] = 1;
            }
            f(id[j], g[j]);
        }
    }
}

// (t, id) order as one integer: t >= 0, so its binary32 bits order like t.
__device__ __forceinline__ unsigned long long hit_key(float s, uint32_t id) {
    return ((unsigned long long)__float_as_uint(s) << 32) | id;
}
constexpr unsigned long long kNoKey = ~0ull;

// Minimum over the kGroup lanes of this lane's group (xor offsets stay inside
// an aligned group).
template <int kGroup>
__device__ __forceinline__ unsigned long long group_min(unsigned long long k) {
    for (int o = kGroup / 2; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(k, o, 64);
        k = y < k ? y : k;
    }
    return k;
}
// The kGroup bits of this lane's group in a wave-wide ballot (bit j = lane j of the group).
template <int kGroup>
__device__ __forceinline__ unsigned long long group_ballot(bool p, int lane) {
    const unsigned long long m = __ballot(p);
    return (m >> (lane & ~(kGroup - 1))) & (kGroup == 64 ? ~0ull : ((1ull << kGroup) - 1ull));
}
template <int kGroup>
__device__ __forceinline__ bool group_any(bool p, int lane) {
    return group_ballot<kGroup>(p, lane) != 0ull;
}

// Result of one ray.
struct Shade {
    float3 col = make_float3(0.0f, 0.0f, 0.0f);
    float T = 1.0f;
    float first_t = INFINITY;
    int first = -1;
};

// Processes the current voxel's list with the kGroup lanes of the ray's group;
// true when the ray is finished (opaque: a hit in this voxel; transparent:
// transmittance below tau).  Every lane of the group returns the same result.
template <bool kStats, int kForm, class Cfg>
__device__ __forceinline__ bool shade_voxel(const TraceArgs &a, const Ray &r, const Walk &w, Shade &sh, Counters &cn,
                                            int lane) {
    constexpr int kGroup = Cfg::kGroup, kLaneKeys = Cfg::kLaneKeys;
    const int gl = lane & (kGroup - 1);
    const float3 D = make_float3(r.D[0], r.D[1], r.D[2]);
    const float3 ro = make_float3(fmaf(w.tcur, D.x, r.O[0] - (float)w.v[0]), fmaf(w.tcur, D.y, r.O[1] - (float)w.v[1]),
                                  fmaf(w.tcur, D.z, r.O[2] - (float)w.v[2]));
    const float tl = w.texit - w.tcur;
    const int cx = w.v[0], cy = w.v[1], cz = w.v[2];
    const float radius = a.p.radius;
    if (kStats && gl == 0) {
        ++cn.list;
        a.stat_vox[w.vi] = 1;
    }
    if (a.p.mode == VRT_TRACE_OPAQUE) {
        unsigned long long best = kNoKey;
        for_each_entry<kStats, kForm, Cfg>(a, w, gl, cn, [&](uint32_t id, const LocalSeg &g) {
            float s;
            if (voxel_hit(g, radius, ro, D, tl, s)) {
                const unsigned long long key = hit_key(s, id);
                best = key < best ? key : best;
            }
        });
        if (!group_any<kGroup>(best != kNoKey, lane)) return false;  // no hit: skip the reduction
        best = group_min<kGroup>(best);
        const uint32_t id = (uint32_t)best;
        sh.first = (int)id;
        sh.first_t = w.tcur + __uint_as_float((uint32_t)(best >> 32));
        float unused_alpha;
        sh.col = hit_colour<kForm>(a, id, cx, cy, cz, unused_alpha);
        if (a.p.lit) {  // voxel-space shading of the voxel holding the hit (Section 3.4)
            const float l = a.p.lit[w.vi];
            sh.col = make_float3(sh.col.x * l, sh.col.y * l, sh.col.z * l);
        }
        sh.T = 0.0f;
        return true;
    }
    // Transparent: each lane keeps its kLaneKeys smallest accepted keys above
    // the threshold; the group composites the smallest head key of all lanes
    // while it is safe, i.e. while no lane that dropped keys has run dry;
    // otherwise it rescans above the last composited key.
    unsigned long long thr = 0ull;
    bool have_thr = false;
    const float lit = a.p.lit ? a.p.lit[w.vi] : 1.0f;  // voxel-space shading of this voxel (Section 3.4)
    for (;;) {
        unsigned long long kk[kLaneKeys];
#pragma unroll
        for (int j = 0; j < kLaneKeys; ++j) kk[j] = kNoKey;
        int nacc = 0;
        if (kStats && gl == 0) ++cn.pass;
        for_each_entry<kStats, kForm, Cfg>(a, w, gl, cn, [&](uint32_t id, const LocalSeg &g) {
            float s;
            if (!voxel_hit(g, radius, ro, D, tl, s)) return;
            unsigned long long key = hit_key(s, id);
            if (have_thr && !(key > thr)) return;
            ++nacc;
#pragma unroll
            for (int j = 0; j < kLaneKeys; ++j) {  // sorted insert, the largest falls off the end
                const bool less = key < kk[j];
                const unsigned long long lo = less ? key : kk[j];
                key = less ? kk[j] : key;
                kk[j] = lo;
            }
        });
        const bool dropped = nacc > kLaneKeys;
        bool rescan = false;
        // each lane holds the colour and opacity of its smallest key, read as
        // soon as that key is at the head, so a pop takes them from the owner
        // lane instead of reading them after the group has found the minimum
        float4 hc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (kk[0] != kNoKey) hc = hit_rgba<kForm>(a, (uint32_t)kk[0], cx, cy, cz);
        for (;;) {
            if (group_any<kGroup>(dropped && kk[0] == kNoKey, lane)) {
                rescan = true;
                break;
            }
            if (!group_any<kGroup>(kk[0] != kNoKey, lane)) break;  // nothing left: skip the reduction
            const unsigned long long m = group_min<kGroup>(kk[0]);
            // keys are unique (one per segment), so exactly one lane holds m: it pops, and its colour is used
            const bool own = kk[0] == m;
            const int src = (lane & ~(kGroup - 1)) + __ffsll((long long)group_ballot<kGroup>(own, lane)) - 1;
            float3 c = make_float3(__shfl(hc.x, src, 64), __shfl(hc.y, src, 64), __shfl(hc.z, src, 64));
            const float alpha = __shfl(hc.w, src, 64);
            if (own) {
#pragma unroll
                for (int j = 0; j + 1 < kLaneKeys; ++j) kk[j] = kk[j + 1];
                kk[kLaneKeys - 1] = kNoKey;
                if (kk[0] != kNoKey) hc = hit_rgba<kForm>(a, (uint32_t)kk[0], cx, cy, cz);
            }
            c = make_float3(c.x * lit, c.y * lit, c.z * lit);
            const uint32_t id = (uint32_t)m;
            if (sh.first < 0) {
                sh.first = (int)id;
                sh.first_t = w.tcur + __uint_as_float((uint32_t)(m >> 32));
            }
            const float wgt = sh.T * alpha;
            sh.col.x += wgt * c.x;
            sh.col.y += wgt * c.y;
            sh.col.z += wgt * c.z;
            sh.T *= (1.0f - alpha);
            thr = m;
            have_thr = true;
            if (sh.T < a.p.tau) return true;
        }
        if (!rescan) return false;
    }
}

__device__ __forceinline__ void write_pixel(const TraceArgs &a, int64_t pixel, const Shade &sh) {
    float4 out;
    if (a.p.mode == VRT_TRACE_OPAQUE)
        out = sh.first >= 0 ? make_float4(sh.col.x, sh.col.y, sh.col.z, 1.0f) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    else
        out = make_float4(sh.col.x, sh.col.y, sh.col.z, 1.0f - sh.T);
    reinterpret_cast<float4 *>(a.rgba)[pixel] = out;
    if (a.depth) a.depth[pixel] = sh.first >= 0 ? sh.first_t * a.p.voxel_size : INFINITY;
    if (a.first_id) a.first_id[pixel] = sh.first;
}

// Adds the wave's counters to the statistics (per-ray test counts are summed
// over the ray's group before the maximum is taken).
template <bool kStats>
__device__ __forceinline__ void flush_counters(const TraceArgs &a, const Counters &cn, bool hit, int lane, int group) {
    if (!kStats) return;
    unsigned long long v[7] = {hit ? 1ull : 0ull, cn.skip64, cn.skip8, cn.vox, cn.list, cn.test, cn.pass};
    for (int k = 0; k < 7; ++k) {
        unsigned long long x = v[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0 && x) atomicAdd(&a.stat_acc[k], x);
    }
    unsigned long long mx = cn.test;
    for (int o = group / 2; o > 0; o >>= 1) mx += __shfl_xor(mx, o, 64);
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(mx, o, 64);
        mx = y > mx ? y : mx;
    }
    if (lane == 0 && mx) atomicMax(&a.stat_acc[7], mx);
}

// Per brick of the grid: 0 when the brick is visible, else the shift (3..6)
// of the largest invisible cell of 8^3 .. 64^3 voxels holding it (a 64^3
// cell is visible iff one of its bricks is), so the walk phase reads one byte
// per brick it enters.
__device__ __forceinline__ void b_brick_skip(TraceArgs a, unsigned bid_, unsigned nblk_) {
    const uint32_t nb = (uint32_t)a.nb[0] * a.nb[1] * a.nb[2];
    for (uint32_t b = bid_ * blockDim.x + threadIdx.x; b < nb; b += nblk_ * blockDim.x) {
        uint8_t sh = 0;
        if (!a.vis3[b]) {
            const int v[3] = {(int)(b % (uint32_t)a.nb[0]) * 8, (int)((b / (uint32_t)a.nb[0]) % (uint32_t)a.nb[1]) * 8,
                              (int)(b / ((uint32_t)a.nb[0] * a.nb[1])) * 8};
            const uint8_t v4 = a.vis4 ? a.vis4[coarse_index(v, 4, a.n4)] : 1;
            const uint8_t v5 = a.vis5 ? a.vis5[coarse_index(v, 5, a.n5)] : 1;
            const uint8_t v6 = a.vis6 ? a.vis6[coarse_index(v, 6, a.n6)] : 1;
            sh = !v6 ? 6 : (!v5 ? 5 : (!v4 ? 4 : 3));
        }
        a.bskip[b] = sh;
    }
}
__global__ void __launch_bounds__(256) k_brick_skip(TraceArgs a) { b_brick_skip(a, blockIdx.x, gridDim.x); }

// One step of the walk phase (the march's step with one jump site, so that
// the lanes of a wave in different states run fewer distinct paths): -1 when
// the ray has left the box or the grid, 0 after a jump over an invisible cell
// or a list-free 2^3 / 4^3 cell, 1 on a voxel without a list, 2 on a visible
// voxel with a list (the caller steps past both).
template <bool kStats>
__device__ __forceinline__ int walk_step(const TraceArgs &a, const Ray &r, Walk &w, MaskRegs &mk, Counters &cn) {
    if (!(w.tcur < w.tout)) return -1;
    const uint32_t b = ((uint32_t)(w.v[2] >> 3) * (uint32_t)a.nb[1] + (uint32_t)(w.v[1] >> 3)) * (uint32_t)a.nb[0] +
                       (uint32_t)(w.v[0] >> 3);
    int sh = 0;
    if ((int64_t)b != w.bvis) {
        sh = a.bskip[b];
        if (sh == 0) {
            mk.set(a.lmask + (size_t)b * 8, a.lmask2 + b);
            w.bvis = b;
        }
    }
    const int xl = w.v[0] & 7, yl = w.v[1] & 7, zl = w.v[2] & 7;
    if (sh == 0 && !((mk.c2 >> (((zl >> 1) << 4) | ((yl >> 1) << 2) | (xl >> 1))) & 1ull))
        sh = (mk.c2 & (0x00330033ull << (((zl >> 2) << 5) | ((yl >> 2) << 3) | ((xl >> 2) << 1)))) ? 1 : 2;
    if (sh) {
        if (kStats) {
            if (sh == 6) ++cn.skip64;
            else ++cn.skip8;
        }
        if (!skip_cell(r, a.G, sh, w.v, w.tcur)) return -1;
        w.fresh = true;
        return 0;
    }
    if (w.fresh) {
        voxel_bounds(r, w);
        w.fresh = false;
    }
    voxel_exit(w);
    if (kStats) ++cn.vox;
    return ((mk.slice(w.v[2]) >> (local_of(xl, yl, zl) & 63)) & 1ull) ? 2 : 1;
}

// Steps of the march phase: a ray that has not reached a list voxel after
// them is queued where it stands and the walk phase goes on from there, so a
// few long marches do not hold the march launch (the walk phase records list
// voxels wherever it starts; a ray that meets none is written as a miss).
constexpr int kMarchSteps = 64;

// Advances from the current voxel (included) to the first visible voxel with
// a list in walk-phase steps: true when it is there or after kMarchSteps
// steps (the ray is queued either way), false when the ray meets none.
// Leaves the list descriptor unread.
template <bool kStats>
__device__ __forceinline__ bool first_list_voxel(const TraceArgs &a, const Ray &r, Walk &w, Counters &cn, MaskRegs &mk) {
    const int limit = march_limit(a);
    const int max_iter = limit < kMarchSteps ? limit : kMarchSteps;
    for (int it = 0; it < max_iter; ++it) {
        const int st = walk_step<kStats>(a, r, w, mk, cn);
        if (st < 0) return false;
        if (st == 2) return true;
        if (st == 1 && !step_voxel(a, r, w)) return false;
    }
    return max_iter < limit;
}

// Clears the ray queue and combines the stripes of the visible-brick box.
__device__ __forceinline__ void b_trace_begin(DevStatus *st, unsigned bid_, unsigned nblk_) {
    const int k = threadIdx.x;
    if (k == 0) {
        st->n_queue = 0;
        st->n_cont = 0;
    }
    if (k < 6) {
        int v = k < 3 ? INT_MAX : INT_MIN;
        for (int s = 0; s < kStripes; ++s) {
            const int u = st->stripe[s].vbox[k];
            v = k < 3 ? (u < v ? u : v) : (u > v ? u : v);
        }
        st->vbox[k] = v;
    }
}

__global__ void k_trace_begin(DevStatus *st) { b_trace_begin(st, blockIdx.x, gridDim.x); }

// Phase 1, one thread per pixel (a 64-lane wavefront covers an 8x8 tile):
// primary ray, clip to the box of visible bricks, march through empty cells to
// the first visible voxel with a list (at most kMarchSteps steps).  Rays that
// reach one, or are still marching after those steps, are appended to the
// queue (wave-aggregated) where they stand; the others are written as misses.
// Block tile of the march phase: 16 pixels wide, 8 rows per pair of wavefronts.
__device__ __host__ inline int march_tile_rows(int threads) { return (threads / 128) * 8; }

template <bool kStats>
__device__ __forceinline__ void b_trace_march(TraceArgs a, unsigned bid_, unsigned nblk_) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tiles_x = (a.p.W + 15) / 16;
    const int bx = (int)(bid_ % (unsigned)tiles_x), by = (int)(bid_ / (unsigned)tiles_x);
    const int px = bx * 16 + (wv & 1) * 8 + (lane & 7);
    const int py = by * march_tile_rows(blockDim.x) + (wv >> 1) * 8 + (lane >> 3);
    const bool live = px < a.p.W && py < a.p.H;
    const float3 D = primary_dir(a.p, live ? px : 0, live ? py : 0);
    const Ray r = make_ray(a.p, D);
    Counters cn;
    Walk w;
    int vb[6];
    bool found = false;
    if (live && clip_visible(a, r, w.tcur, w.tout, vb)) {
        for (int k = 0; k < 3; ++k) {
            const int vk = (int)floorf(fmaf(w.tcur, r.D[k], r.O[k]));
            const int lo = 8 * vb[k], hi = 8 * vb[3 + k] + 7;
            w.v[k] = vk < lo ? lo : (vk > hi ? hi : vk);
        }
        w.fresh = true;
        MaskRegs mk;
        found = first_list_voxel<kStats>(a, r, w, cn, mk);
    }
    // one queue append per block (same-address atomics serialize)
    __shared__ unsigned s_wcnt[16];
    __shared__ unsigned s_base;
    const unsigned long long mask = __ballot(found);
    if (lane == 0) s_wcnt[wv] = (unsigned)__popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned tot = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) tot += s_wcnt[k];
        s_base = tot ? atomicAdd(&a.st->n_queue, tot) : 0u;
    }
    __syncthreads();
    if (found) {
        unsigned pos = s_base + (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
        for (int k = 0; k < wv; ++k) pos += s_wcnt[k];
        const uint32_t pix = (uint32_t)(py * a.p.W + px);
        a.queue[pos] = make_uint4(pix, pack_voxel(w.v), __float_as_uint(w.tcur), __float_as_uint(w.tout));
    }
    flush_counters<kStats>(a, cn, false, lane, 1);
    if (live && !found) write_pixel(a, (int64_t)py * a.p.W + px, Shade());
}

template <bool kStats>
__global__ void __launch_bounds__(512) k_trace_march(TraceArgs a) { b_trace_march<kStats>(a, blockIdx.x, gridDim.x); }

// Walk entries per queued ray (0: no walk phase; the shade phase walks).
__device__ __forceinline__ int64_t walk_capacity(int64_t entries, unsigned n) {
    if (n == 0) return 0;
    const int64_t k = entries / (int64_t)n;
    return k < kWalkMax ? k : kWalkMax;
}

// Walk phase, one thread per queued ray: continues the march from where the
// march phase left the ray (its first list voxel, or where its march steps
// ran out) and records every visible voxel with a list it passes, in order,
// with its entry parameter (at most walk_capacity entries).  The ray's queue
// entry then holds the count and whether the walk stopped at the limit with
// list voxels left.  The walk needs no list data, so the shade phase's
// lanes find the voxels of a ray without walking them one after another.
__device__ __forceinline__ void b_trace_walk(TraceArgs a, unsigned bid_, unsigned nblk_) {
    const unsigned n = a.st->n_queue;
    const int64_t K = walk_capacity(a.walk_entries, n);
    for (unsigned i = bid_ * blockDim.x + threadIdx.x; i < n; i += nblk_ * blockDim.x) {
        const uint4 q = a.queue[i];
        const float3 D = primary_dir(a.p, (int)(q.x % (uint32_t)a.p.W), (int)(q.x / (uint32_t)a.p.W));
        const Ray r = make_ray(a.p, D);
        Walk w;
        unpack_voxel(q.y, w.v);
        w.tcur = __uint_as_float(q.z);
        w.tout = __uint_as_float(q.w);
        w.fresh = true;
        MaskRegs mk;
        Counters cn;
        uint2 *out = a.walk + (int64_t)i * K;
        uint32_t cnt = 0;
        bool more = false;
        // one loop of single steps: a lane that finds a list voxel records it
        // and steps on while the other lanes of the wave are still marching
        const int max_iter = march_limit(a);
        for (int it = 0; it < max_iter; ++it) {
            const int st = walk_step<false>(a, r, w, mk, cn);
            if (st < 0) break;
            if (st == 2) {
                if (cnt == (uint64_t)K) {
                    more = true;
                    break;
                }
                out[cnt++] = make_uint2(pack_voxel(w.v), __float_as_uint(w.tcur));
            }
            if (st > 0 && !step_voxel(a, r, w)) break;
        }
        a.queue[i].y = cnt | (more ? 0x80000000u : 0u);
    }
}

__global__ void __launch_bounds__(64) k_trace_walk(TraceArgs a) { b_trace_walk(a, blockIdx.x, gridDim.x); }

// Phase 2, one kGroup-lane group per queued ray: lists, capsule tests and
// compositing, continuing the walk until the ray is finished.  All lanes of a
// group follow the same walk; list entries are split across them.
// Work unit bid_ of nblk_, each of unit_threads threads (this thread is
// unit_tid of its unit): the whole workgroup, or one wave of it when the
// waves of a workgroup take work on their own.
// The walked voxels of queued ray i (K entries per ray).  The lanes of the
// group read kGroup entries and their list descriptors at once and take the
// voxels in order from them.  A ray whose walk stopped at the limit and that
// is not finished after its entries is left to the resume launch.
// Returns false when the ray went to the resume list (its pixel is written there).
template <int kForm, class Cfg>
__device__ __forceinline__ bool shade_walked(const TraceArgs &a, const Ray &r, const uint4 &q, unsigned i, int64_t K,
                                             Shade &sh, Counters &cn, int lane) {
    constexpr int kGroup = Cfg::kGroup;
    const int gl = lane & (kGroup - 1), gbase = lane & ~(kGroup - 1);
    const uint32_t cnt = q.y & 0x7FFFFFFFu;
    const uint2 *ent = a.walk + (int64_t)i * K;
    Walk w;
    w.tout = __uint_as_float(q.w);
    uint2 cur = make_uint2(0u, 0u);
    for (uint32_t base = 0; base < cnt; base += kGroup) {
        uint2 e = make_uint2(0u, 0u);
        uint64_t cd = 0;
        if (base + gl < cnt) {
            e = ent[base + gl];
            int v[3];
            unpack_voxel(e.x, v);
            cd = a.cell[voxel_index(a, v)];
        }
        const uint32_t m = cnt - base < (uint32_t)kGroup ? cnt - base : (uint32_t)kGroup;
        for (uint32_t j = 0; j < m; ++j) {
            const int src = gbase + (int)j;
            cur.x = (uint32_t)__shfl((int)e.x, src, 64);
            cur.y = (uint32_t)__shfl((int)e.y, src, 64);
            w.cd = __shfl(cd, src, 64);
            unpack_voxel(cur.x, w.v);
            w.tcur = __uint_as_float(cur.y);
            voxel_bounds(r, w);
            voxel_exit(w);
            w.vi = voxel_index(a, w.v);
            if (shade_voxel<false, kForm, Cfg>(a, r, w, sh, cn, lane)) return true;
        }
    }
    if (!(q.y >> 31)) return true;
    // the walk stopped at the limit: the ray's state goes to its walk slot (whose
    // entries are all read) and the ray to the resume list
    if (gl == 0) {
        uint32_t *slot = reinterpret_cast<uint32_t *>(a.walk + (int64_t)i * K);
        const uint32_t vals[8] = {cur.x, cur.y, __float_as_uint(sh.col.x), __float_as_uint(sh.col.y),
                                  __float_as_uint(sh.col.z), __float_as_uint(sh.T), (uint32_t)sh.first,
                                  __float_as_uint(sh.first_t)};
#pragma unroll
        for (int k = 0; k < 8; ++k) slot[k] = vals[k];
        a.cont[atomicAdd(&a.st->n_cont, 1u)] = i;
    }
    return false;
}

// kWalked: the walk phase has run (plain launches); the statistics variant
// and the batched form walk in this phase.
template <bool kStats, int kForm, class Cfg = DefaultShade, bool kWalked = false>
__device__ __forceinline__ void b_trace_shade(TraceArgs a, unsigned bid_, unsigned nblk_, unsigned unit_threads,
                                              unsigned unit_tid) {
    constexpr int kGroup = Cfg::kGroup;
    const int lane = threadIdx.x & 63;
    const unsigned n = a.st->n_queue;
    const unsigned ngroups = nblk_ * (unit_threads / kGroup);
    const unsigned grp = bid_ * (unit_threads / kGroup) + unit_tid / kGroup;
    __shared__ uint64_t s_mask[8 * kMaxShadeGroups];  // the list mask of each group's brick
    MaskLds mk{s_mask + threadIdx.x / kGroup, (int)(blockDim.x / kGroup)};
    // every group runs the same number of rounds so counters can be reduced per wave
    const unsigned rounds = (n + ngroups - 1) / ngroups;
    const int64_t K = kWalked ? walk_capacity(a.walk_entries, n) : 0;
    for (unsigned rd = 0; rd < rounds; ++rd) {
        const unsigned i = rd * ngroups + grp;
        Counters cn;
        Shade sh;
        if (kWalked && i < n) {  // K >= 1: walk_entries >= max_pixels >= n
            const uint4 q = a.queue[i];
            const float3 D = primary_dir(a.p, (int)(q.x % (uint32_t)a.p.W), (int)(q.x / (uint32_t)a.p.W));
            const Ray r = make_ray(a.p, D);
            if (shade_walked<kForm, Cfg>(a, r, q, i, K, sh, cn, lane) && (lane & (kGroup - 1)) == 0)
                write_pixel(a, (int64_t)q.x, sh);
        } else if (!kWalked && i < n) {
            const uint4 q = a.queue[i];
            const int px = (int)(q.x % (uint32_t)a.p.W), py = (int)(q.x / (uint32_t)a.p.W);
            const float3 D = primary_dir(a.p, px, py);
            const Ray r = make_ray(a.p, D);
            Walk w;
            unpack_voxel(q.y, w.v);
            w.tcur = __uint_as_float(q.z);
            w.tout = __uint_as_float(q.w);
            w.fresh = true;
            Counters walk_cn;  // walk counters once per ray
            // recomputes the exit data of the queued voxel
            bool have = march<kStats>(a, r, w, walk_cn, mk);
            while (have) {
                if (shade_voxel<kStats, kForm, Cfg>(a, r, w, sh, cn, lane)) break;
                if (!step_voxel(a, r, w)) break;
                have = march<kStats>(a, r, w, walk_cn, mk);
            }
            if ((lane & (kGroup - 1)) == 0) {
                write_pixel(a, (int64_t)q.x, sh);
                cn.skip64 += walk_cn.skip64;
                cn.skip8 += walk_cn.skip8;
                cn.vox += walk_cn.vox;
            }
        }
        flush_counters<kStats>(a, cn, sh.first >= 0 && (lane & (kGroup - 1)) == 0, lane, kGroup);
    }
}

// Resume launch, one kGroup-lane group per ray of the resume list: the
// saved state, then the walk from the last walked voxel on, as the shade
// phase does without a walk phase.
template <int kForm, class Cfg = DefaultShade>
__device__ __forceinline__ void b_trace_resume(TraceArgs a, unsigned bid_, unsigned nblk_, unsigned unit_threads,
                                               unsigned unit_tid) {
    constexpr int kGroup = Cfg::kGroup;
    const int lane = threadIdx.x & 63;
    const unsigned n = a.st->n_cont;
    const int64_t K = walk_capacity(a.walk_entries, a.st->n_queue);
    const unsigned ngroups = nblk_ * (unit_threads / kGroup);
    __shared__ uint64_t s_mask[8 * kMaxShadeGroups];
    MaskLds mk{s_mask + threadIdx.x / kGroup, (int)(blockDim.x / kGroup)};
    for (unsigned k = bid_ * (unit_threads / kGroup) + unit_tid / kGroup; k < n; k += ngroups) {
        const unsigned i = a.cont[k];
        const uint4 q = a.queue[i];
        const uint32_t *slot = reinterpret_cast<const uint32_t *>(a.walk + (int64_t)i * K);
        Shade sh;
        sh.col = make_float3(__uint_as_float(slot[2]), __uint_as_float(slot[3]), __uint_as_float(slot[4]));
        sh.T = __uint_as_float(slot[5]);
        sh.first = (int)slot[6];
        sh.first_t = __uint_as_float(slot[7]);
        const float3 D = primary_dir(a.p, (int)(q.x % (uint32_t)a.p.W), (int)(q.x / (uint32_t)a.p.W));
        const Ray r = make_ray(a.p, D);
        Walk w;
        unpack_voxel(slot[0], w.v);
        w.tcur = __uint_as_float(slot[1]);
        w.tout = __uint_as_float(q.w);
        w.fresh = true;
        Counters cn;
        // re-enter the last walked voxel, step past it and go on
        bool have = march<false>(a, r, w, cn, mk) && step_voxel(a, r, w) && march<false>(a, r, w, cn, mk);
        while (have) {
            if (shade_voxel<false, kForm, Cfg>(a, r, w, sh, cn, lane)) break;
            if (!step_voxel(a, r, w)) break;
            have = march<false>(a, r, w, cn, mk);
        }
        if ((lane & (kGroup - 1)) == 0) write_pixel(a, (int64_t)q.x, sh);
    }
}

template <int kForm>
__global__ void __launch_bounds__(64) k_trace_resume(TraceArgs a) {
    b_trace_resume<kForm>(a, blockIdx.x, gridDim.x, blockDim.x, threadIdx.x);
}

__device__ __forceinline__ void b_debug_rays(TraceParams p, const int64_t *__restrict__ pix, int64_t n, float *__restrict__ dirs, unsigned bid_, unsigned nblk_) {
    int64_t i = (int64_t)bid_ * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t q = pix[i];
    int px = (int)(q % p.W), py = (int)(q / p.W);
    float3 d = primary_dir(p, px, py);
    dirs[3 * i] = d.x;
    dirs[3 * i + 1] = d.y;
    dirs[3 * i + 2] = d.z;
}

// Four waves per SIMD (at most 128 registers): the fourth wave hides more
// latency than the few spilled registers cost.  Rays are taken in xcd_order
// (neighbouring rays test the same segments).
template <bool kStats, int kForm, class Cfg, bool kWalked>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) k_trace_shade(TraceArgs a) { b_trace_shade<kStats, kForm, Cfg, kWalked>(a, xcd_order(blockIdx.x, gridDim.x), gridDim.x, blockDim.x, threadIdx.x); }

__global__ void k_debug_rays(TraceParams p, const int64_t *__restrict__ pix, int64_t n, float *__restrict__ dirs) { b_debug_rays(p, pix, n, dirs, blockIdx.x, gridDim.x); }

// Clears the statistics marks of the occupied bricks, the segments and the counters.
__device__ __forceinline__ void b_stat_clear(const int32_t *__restrict__ list, const DevStatus *__restrict__ st, int64_t nv,
                             uint8_t *__restrict__ vox, uint8_t *__restrict__ seg, unsigned long long *__restrict__ acc, unsigned bid_, unsigned nblk_) {
    const unsigned nb = st->n_bricks;
    for (unsigned sl = bid_; sl < nb; sl += nblk_) {
        const int64_t b = list[sl];
        for (int t = threadIdx.x; t < kBrickVox; t += blockDim.x) vox[b * kBrickVox + t] = 0;
    }
    for (int64_t i = (int64_t)bid_ * blockDim.x + threadIdx.x; i < nv; i += (int64_t)nblk_ * blockDim.x)
        seg[i] = 0;
    if (bid_ == 0 && threadIdx.x < 16) acc[threadIdx.x] = 0;
}

__global__ void k_stat_clear(const int32_t *__restrict__ list, const DevStatus *__restrict__ st, int64_t nv,
                             uint8_t *__restrict__ vox, uint8_t *__restrict__ seg, unsigned long long *__restrict__ acc) { b_stat_clear(list, st, nv, vox, seg, acc, blockIdx.x, gridDim.x); }

// Distinct voxels read, their list lengths, and distinct segments tested.
__device__ __forceinline__ void b_stat_reduce(const int32_t *__restrict__ list, const DevStatus *__restrict__ st, int64_t nv,
                              const uint8_t *__restrict__ vox, const uint64_t *__restrict__ cell,
                              const uint8_t *__restrict__ seg, unsigned long long *__restrict__ acc, unsigned bid_, unsigned nblk_) {
    unsigned long long nvx = 0, nent = 0, nseg = 0;
    const unsigned nb = st->n_bricks;
    for (unsigned sl = bid_; sl < nb; sl += nblk_) {
        const int64_t b = list[sl];
        for (int t = threadIdx.x; t < kBrickVox; t += blockDim.x)
            if (vox[b * kBrickVox + t]) {
                ++nvx;
                nent += cell[b * kBrickVox + t] >> 32;
            }
    }
    for (int64_t i = (int64_t)bid_ * blockDim.x + threadIdx.x; i < nv; i += (int64_t)nblk_ * blockDim.x)
        nseg += seg[i];
    unsigned long long v[3] = {nvx, nent, nseg};
    for (int k = 0; k < 3; ++k) {
        unsigned long long x = v[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if ((threadIdx.x & 63) == 0 && x) atomicAdd(&acc[8 + k], x);
    }
}

__global__ void k_stat_reduce(const int32_t *__restrict__ list, const DevStatus *__restrict__ st, int64_t nv,
                              const uint8_t *__restrict__ vox, const uint64_t *__restrict__ cell,
                              const uint8_t *__restrict__ seg, unsigned long long *__restrict__ acc) { b_stat_reduce(list, st, nv, vox, cell, seg, acc, blockIdx.x, gridDim.x); }

}  // namespace

static TraceArgs trace_args(vrt_ctx *c, const TraceParams &p, const vrt_image *img) {
    TraceArgs a;
    a.p = p;
    for (int k = 0; k < 3; ++k) {
        a.G[k] = c->dims[k];
        a.nb[k] = c->dims[k] / 8;
    }
    a.vis3 = c->a.vis3;
    a.bskip = c->a.bskip;
    const uint8_t **hv[3] = {&a.vis4, &a.vis5, &a.vis6};
    int *hn[3] = {a.n4, a.n5, a.n6};
    for (int L = 4; L <= 6; ++L) {
        *hv[L - 4] = nullptr;
        for (int k = 0; k < 3; ++k) hn[L - 4][k] = 0;
        if (c->n_levels > L) {
            const Level &l = c->levels[L];
            *hv[L - 4] = c->a.vis_hi + l.offset;
            for (int k = 0; k < 3; ++k) hn[L - 4][k] = l.dims[k];
        }
    }
    a.cell = c->a.cell;
    a.lmask = c->a.lmask;
    a.lmask2 = c->a.lmask2;
    a.st = c->a.status;
    a.ids = c->a.ids;
    a.vrec = c->a.vrec;
    a.srec16 = c->a.srec16;
    a.nv = c->n_vertices;
    a.capacity = c->desc.max_fragments;
    a.queue = c->a.queue;
    a.walk = c->a.walk;
    a.cont = c->a.cont;
    a.walk_entries = c->walk_entries;
    a.rgba = img->rgba;
    a.depth = img->depth;
    a.first_id = img->first_id;
    a.stat_vox = c->a.stat_vox;
    a.stat_seg = c->a.stat_seg;
    a.stat_acc = c->a.stat_acc;
    return a;
}

bool tune_valid(const vrt_tune &t) {
    const bool mt = t.march_threads == 128 || t.march_threads == 256 || t.march_threads == 512;
    const bool g = t.shade_group == 8 || t.shade_group == 16 || t.shade_group == 32;
    const bool b = t.shade_batch == 2 || t.shade_batch == 4;
    const bool k = t.lane_keys == 4 || t.lane_keys == 8;
    const bool nb = t.shade_blocks >= 256 && t.shade_blocks <= 65535;
    return mt && g && b && k && nb && t.reserved[0] == 0 && t.reserved[1] == 0 && t.reserved[2] == 0;
}

static unsigned march_grid(const TraceParams &p, int threads) {
    const int rows = march_tile_rows(threads);
    return (unsigned)(((p.W + 15) / 16) * ((p.H + rows - 1) / rows));
}

// Walk phase grid: one thread per pixel that could be queued, one wave per
// block (the queued rays' waves then spread evenly over the compute units:
// 2.5% faster than four-wave blocks), at most 8192 blocks (grid-stride beyond).
constexpr int kWalkThreads = 64;
static unsigned walk_grid(const TraceParams &p) {
    const int64_t b = ((int64_t)p.W * p.H + kWalkThreads - 1) / kWalkThreads;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

// Resume launch: rays past the walk limit are rare (they need more than
// kWalkPerPixel * max_pixels / n_queue list voxels).
constexpr unsigned kResumeBlocks = 256;

static unsigned skip_grid(const vrt_ctx *c) {
    const int64_t b = ((int64_t)(c->dims[0] / 8) * (c->dims[1] / 8) * (c->dims[2] / 8) + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

// Launches the shade kernel instance of shape (group, batch, keys).
template <bool kStats, int kForm>
static void launch_shade(const vrt_tune &t, const TraceArgs &a, hipStream_t st) {
    // single-wave workgroups (shade_blocks counts 256 threads): a wave's slot is
    // free as soon as the wave is done, not when the slowest wave of its block is
    const unsigned blocks = (unsigned)t.shade_blocks * 4u;
#define VRT_SHADE_CASE(G, B, K)                                                                  \
    case G * 100 + B * 10 + K:                                                                   \
        k_trace_shade<kStats, kForm, ShadeCfg<G, B, K>, !kStats><<<blocks, 64, 0, st>>>(a);     \
        break;
    switch (t.shade_group * 100 + t.shade_batch * 10 + t.lane_keys) {
        VRT_SHADE_CASE(8, 2, 4) VRT_SHADE_CASE(8, 2, 8) VRT_SHADE_CASE(8, 4, 4) VRT_SHADE_CASE(8, 4, 8)
        VRT_SHADE_CASE(16, 2, 4) VRT_SHADE_CASE(16, 2, 8) VRT_SHADE_CASE(16, 4, 4) VRT_SHADE_CASE(16, 4, 8)
        VRT_SHADE_CASE(32, 2, 4) VRT_SHADE_CASE(32, 2, 8) VRT_SHADE_CASE(32, 4, 4) VRT_SHADE_CASE(32, 4, 8)
        default: break;  // unreachable: the shape is validated when it is set
    }
#undef VRT_SHADE_CASE
}

hipError_t launch_trace(vrt_ctx *c, const TraceParams &p, const vrt_image *img, hipStream_t st) {
    TraceArgs a = trace_args(c, p, img);
    const vrt_tune &t = c->tune[p.mode == VRT_TRACE_OPAQUE ? 0 : 1];
    VRT_LAUNCH(c, "k_trace_begin", st, k_trace_begin<<<1, 64, 0, st>>>(a.st));
    VRT_LAUNCH(c, "k_brick_skip", st, k_brick_skip<<<skip_grid(c), 256, 0, st>>>(a));
    VRT_LAUNCH(c, "k_trace_march", st, k_trace_march<false><<<march_grid(p, t.march_threads), t.march_threads, 0, st>>>(a));
    VRT_LAUNCH(c, "k_trace_walk", st, k_trace_walk<<<walk_grid(p), kWalkThreads, 0, st>>>(a));
    if (c->desc.form == VRT_FORM_FP16) {
        VRT_LAUNCH(c, "k_trace_shade", st, (launch_shade<false, VRT_FORM_FP16>(t, a, st)));
        VRT_LAUNCH(c, "k_trace_resume", st, k_trace_resume<VRT_FORM_FP16><<<kResumeBlocks, 64, 0, st>>>(a));
    } else {
        VRT_LAUNCH(c, "k_trace_shade", st, (launch_shade<false, VRT_FORM_PLAIN>(t, a, st)));
        VRT_LAUNCH(c, "k_trace_resume", st, k_trace_resume<VRT_FORM_PLAIN><<<kResumeBlocks, 64, 0, st>>>(a));
    }
    return hipGetLastError();
}

// The counters are gathered with the default shape (kbuffer_passes depends on
// the group and lane_keys; every other counter does not).
hipError_t launch_trace_stats(vrt_ctx *c, const TraceParams &p, const vrt_image *img, hipStream_t st) {
    TraceArgs a = trace_args(c, p, img);
    k_stat_clear<<<1024, 256, 0, st>>>(c->a.brick_list, c->a.status, c->n_vertices, a.stat_vox, a.stat_seg, a.stat_acc);
    k_trace_begin<<<1, 64, 0, st>>>(a.st);
    k_brick_skip<<<skip_grid(c), 256, 0, st>>>(a);
    k_trace_march<true><<<march_grid(p, 256), 256, 0, st>>>(a);
    if (c->desc.form == VRT_FORM_FP16) k_trace_shade<true, VRT_FORM_FP16, DefaultShade, false><<<16384, 64, 0, st>>>(a);
    else k_trace_shade<true, VRT_FORM_PLAIN, DefaultShade, false><<<16384, 64, 0, st>>>(a);
    k_stat_reduce<<<1024, 256, 0, st>>>(c->a.brick_list, c->a.status, c->n_vertices, a.stat_vox, a.cell, a.stat_seg,
                                        a.stat_acc);
    return hipGetLastError();
}

hipError_t launch_debug_rays(const TraceParams &p, const int64_t *pix, int64_t n, float *dirs, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_debug_rays<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, pix, n, dirs);
    return hipGetLastError();
}

}  // namespace vrt
