// vrt_trace.hip -- Section 3.5: voxel ray tracing through the per-voxel lists.
#include "vrt_internal.h"

namespace vrt {
namespace {

constexpr int kKeys = 8;  // k-buffer entries per pass (transparent)

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

// Entry root of |oc + t D| = r (unit D): smaller root, stable form.
__device__ __forceinline__ float sphere_entry(float3 oc, float3 D, float r2) {
    float b = dot3(oc, D);
    float c = dot3(oc, oc) - r2;
    float h = b * b - c;
    if (h < 0.0f) return -INFINITY;
    float sq = sqrtf(h);
    float q = b >= 0.0f ? -(b + sq) : (sq - b);
    return b >= 0.0f ? q : c / q;
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
    if (baba == 0.0f) return sphere_entry(oa, D, r2);
    const float3 w = cross3(D, ba), u = cross3(oa, ba);
    const float ww = dot3(w, w);
    const float bard = dot3(ba, D), baoa = dot3(ba, oa);
    const float c = dot3(u, u) - r2 * baba;
    if (ww == 0.0f) {  // parallel to the axis: inside the cylinder or a miss
        if (c > 0.0f) return -INFINITY;
        return sphere_entry(bard > 0.0f ? oa : sub3(ro, pb), D, r2);
    }
    const float ow = dot3(oa, w);
    const float g = r2 * ww - ow * ow;
    if (g < 0.0f) return -INFINITY;  // misses the infinite cylinder, hence the capsule
    const float b = dot3(w, u);
    const float sq = sqrtf(baba * g);
    const float t = b >= 0.0f ? -(b + sq) / ww : c / (sq - b);
    const float y = baoa + t * bard;
    if (y > 0.0f && y < baba) return t;
    return sphere_entry(y <= 0.0f ? oa : sub3(ro, pb), D, r2);
}

struct TraceArgs {
    TraceParams p;
    int G[3];
    int nb[3];
    const uint8_t *vis0;
    const uint8_t *vis3;
    const uint32_t *words;
    const uint32_t *cursor;
    const uint32_t *ids;
    const VRec *vrec;
    int64_t nv;        // vertices of the frame (ids must be < nv - 1)
    int64_t capacity;  // entries of ids
    float *rgba;
    float *depth;
    int *first_id;
};

__device__ __forceinline__ float3 rel(const VRec &v, int cx, int cy, int cz) {
    return make_float3((float)(v.x - cx * kQ) * (1.0f / kQ), (float)(v.y - cy * kQ) * (1.0f / kQ),
                       (float)(v.z - cz * kQ) * (1.0f / kQ));
}

// Accepted hit of segment id inside the current voxel: entry parameter s in
// [0, tl) from the voxel-local origin ro, and on the kept side of both clip
// planes ((P - A).n0 >= 0 at an interior A, (P - B).n1 < 0 at an interior B).
__device__ __forceinline__ bool voxel_hit(const TraceArgs &a, uint32_t id, float3 ro, float3 D, int cx, int cy, int cz,
                                          float tl, float &s) {
    if ((int64_t)id + 1 >= a.nv) return false;
    VRec A = a.vrec[id], B = a.vrec[id + 1];
    float3 pa = rel(A, cx, cy, cz), pb = rel(B, cx, cy, cz);
    s = capsule_entry(ro, D, pa, pb, a.p.radius);
    if (!(s >= 0.0f && s < tl)) return false;
    float3 P = make_float3(fmaf(s, D.x, ro.x), fmaf(s, D.y, ro.y), fmaf(s, D.z, ro.z));
    if (A.flags & kInterior) {
        if (!(dot3(sub3(P, pa), make_float3(A.nx, A.ny, A.nz)) >= 0.0f)) return false;
    }
    if (B.flags & kInterior) {
        if (!(dot3(sub3(P, pb), make_float3(B.nx, B.ny, B.nz)) < 0.0f)) return false;
    }
    return true;
}

__device__ __forceinline__ float3 seg_colour(const TraceArgs &a, uint32_t id) {
    VRec A = a.vrec[id], B = a.vrec[id + 1];
    float dx = (float)(B.x - A.x), dy = (float)(B.y - A.y), dz = (float)(B.z - A.z);
    float len = sqrtf(dx * dx + dy * dy + dz * dz);
    if (len == 0.0f) return make_float3(0.0f, 0.0f, 0.0f);
    return make_float3(fabsf(dx) / len, fabsf(dy) / len, fabsf(dz) / len);
}

__device__ __forceinline__ bool key_less(float s0, uint32_t i0, float s1, uint32_t i1) {
    return s0 < s1 || (s0 == s1 && i0 < i1);
}

__device__ __forceinline__ float tcross(int bnd, float o, float d) { return ((float)bnd - o) / d; }

// One thread per pixel; a 64-lane wavefront covers an 8x8 pixel tile.
__global__ void __launch_bounds__(256) k_trace(TraceArgs a) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int px = blockIdx.x * 16 + (w & 1) * 8 + (lane & 7);
    const int py = blockIdx.y * 16 + (w >> 1) * 8 + (lane >> 3);
    if (px >= a.p.W || py >= a.p.H) return;
    const float3 D = primary_dir(a.p, px, py);
    const float O[3] = {a.p.O[0], a.p.O[1], a.p.O[2]};
    const float Dv[3] = {D.x, D.y, D.z};
    float tin = 0.0f, tout = INFINITY;
    bool inside = true;
    for (int k = 0; k < 3; ++k) {
        if (Dv[k] == 0.0f) {
            if (O[k] < 0.0f || O[k] > (float)a.G[k]) inside = false;
            continue;
        }
        float t1 = tcross(0, O[k], Dv[k]), t2 = tcross(a.G[k], O[k], Dv[k]);
        if (t1 > t2) {
            float tt = t1;
            t1 = t2;
            t2 = tt;
        }
        tin = fmaxf(tin, t1);
        tout = fminf(tout, t2);
    }
    const int64_t pixel = (int64_t)py * a.p.W + px;
    float3 col = make_float3(0.0f, 0.0f, 0.0f);
    float T = 1.0f, first_t = INFINITY;
    int first = -1;
    const bool opaque = a.p.mode == VRT_TRACE_OPAQUE;
    if (inside && tin < tout) {
        int v[3], step[3];
        float tnext[3];
        for (int k = 0; k < 3; ++k) {
            float pk = fmaf(tin, Dv[k], O[k]);
            int vk = (int)floorf(pk);
            vk = vk < 0 ? 0 : (vk >= a.G[k] ? a.G[k] - 1 : vk);
            v[k] = vk;
            step[k] = Dv[k] > 0.0f ? 1 : (Dv[k] < 0.0f ? -1 : 0);
            tnext[k] = step[k] == 0 ? INFINITY : tcross(v[k] + (step[k] > 0), O[k], Dv[k]);
        }
        float tcur = tin;
        const int max_iter = 3 * (a.G[0] + a.G[1] + a.G[2]) + 16;
        for (int it = 0; it < max_iter; ++it) {
            const int bx = v[0] >> 3, by = v[1] >> 3, bz = v[2] >> 3;
            const int64_t b = ((int64_t)bz * a.nb[1] + by) * a.nb[0] + bx;
            if (!a.vis3[b]) {
                // skip the whole brick: exit through its nearest face
                const int bb[3] = {bx, by, bz};
                float tb[3];
                int m = 0;
                for (int k = 0; k < 3; ++k) {
                    tb[k] = step[k] == 0 ? INFINITY : tcross(8 * (bb[k] + (step[k] > 0)), O[k], Dv[k]);
                    if (tb[k] < tb[m]) m = k;
                }
                float te = fmaxf(tb[m], tcur);
                bool out = false;
                for (int k = 0; k < 3; ++k) {
                    int nv;
                    if (k == m) {
                        nv = step[k] > 0 ? 8 * (bb[k] + 1) : 8 * bb[k] - 1;
                        if (nv < 0 || nv >= a.G[k]) out = true;
                    } else {
                        nv = (int)floorf(fmaf(te, Dv[k], O[k]));
                        if (step[k] > 0) nv = nv < v[k] ? v[k] : nv;
                        if (step[k] < 0) nv = nv > v[k] ? v[k] : nv;
                        int lo = 8 * bb[k], hi = 8 * bb[k] + 7;
                        nv = nv < lo ? lo : (nv > hi ? hi : nv);
                    }
                    v[k] = nv;
                }
                if (out) break;
                tcur = te;
                for (int k = 0; k < 3; ++k)
                    tnext[k] = step[k] == 0 ? INFINITY : tcross(v[k] + (step[k] > 0), O[k], Dv[k]);
                if (!(tcur < tout)) break;
                continue;
            }
            int m = 0;
            if (tnext[1] < tnext[m]) m = 1;
            if (tnext[2] < tnext[m]) m = 2;
            const float texit = fmaxf(tnext[m], tcur);
            const int64_t vi = b * kBrickVox + local_of(v[0], v[1], v[2]);
            const uint32_t cnt = a.vis0[vi] ? (a.words[vi] & 0xFFFFu) : 0u;
            if (cnt) {
                // after a capacity overflow the lists are undefined but reads stay inside ids
                const uint32_t cend = a.cursor[vi];
                const uint32_t end = (int64_t)cend < a.capacity ? cend : (uint32_t)a.capacity;
                const uint32_t start = end >= cnt ? end - cnt : 0u;
                const float3 ro = make_float3(fmaf(tcur, D.x, O[0] - (float)v[0]), fmaf(tcur, D.y, O[1] - (float)v[1]),
                                              fmaf(tcur, D.z, O[2] - (float)v[2]));
                const float tl = texit - tcur;
                if (opaque) {
                    float best = INFINITY;
                    uint32_t bid = 0xFFFFFFFFu;
                    for (uint32_t k = start; k < end; ++k) {
                        uint32_t id = a.ids[k];
                        float s;
                        if (voxel_hit(a, id, ro, D, v[0], v[1], v[2], tl, s) && key_less(s, id, best, bid)) {
                            best = s;
                            bid = id;
                        }
                    }
                    if (bid != 0xFFFFFFFFu) {
                        first = (int)bid;
                        first_t = tcur + best;
                        col = seg_colour(a, bid);
                        T = 0.0f;
                        break;
                    }
                } else {
                    // k-buffer passes: the kKeys smallest (s, id) keys above the last composited key
                    float ls = -INFINITY;
                    uint32_t lid = 0;
                    bool first_pass = true;
                    for (;;) {
                        float ks[kKeys];
                        uint32_t ki[kKeys];
                        int nk = 0, above = 0;
                        for (uint32_t k = start; k < end; ++k) {
                            uint32_t id = a.ids[k];
                            float s;
                            if (!voxel_hit(a, id, ro, D, v[0], v[1], v[2], tl, s)) continue;
                            if (!first_pass && !key_less(ls, lid, s, id)) continue;
                            ++above;
                            if (nk == kKeys && !key_less(s, id, ks[kKeys - 1], ki[kKeys - 1])) continue;
                            int j = nk < kKeys ? nk++ : kKeys - 1;
                            while (j > 0 && key_less(s, id, ks[j - 1], ki[j - 1])) {
                                ks[j] = ks[j - 1];
                                ki[j] = ki[j - 1];
                                --j;
                            }
                            ks[j] = s;
                            ki[j] = id;
                        }
                        for (int j = 0; j < nk && !(T < a.p.tau); ++j) {
                            if (first < 0) {
                                first = (int)ki[j];
                                first_t = tcur + ks[j];
                            }
                            float3 c = seg_colour(a, ki[j]);
                            float wgt = T * a.p.alpha;
                            col.x += wgt * c.x;
                            col.y += wgt * c.y;
                            col.z += wgt * c.z;
                            T *= (1.0f - a.p.alpha);
                        }
                        if (above <= kKeys || T < a.p.tau || nk == 0) break;
                        ls = ks[kKeys - 1];
                        lid = ki[kKeys - 1];
                        first_pass = false;
                    }
                    if (T < a.p.tau) break;
                }
            }
            // step to the next voxel
            v[m] += step[m];
            if (v[m] < 0 || v[m] >= a.G[m]) break;
            tcur = texit;
            tnext[m] = tcross(v[m] + (step[m] > 0), O[m], Dv[m]);
            if (!(tcur < tout)) break;
        }
    }
    float4 out;
    if (opaque) out = first >= 0 ? make_float4(col.x, col.y, col.z, 1.0f) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    else out = make_float4(col.x, col.y, col.z, 1.0f - T);
    reinterpret_cast<float4 *>(a.rgba)[pixel] = out;
    if (a.depth) a.depth[pixel] = first >= 0 ? first_t * a.p.voxel_size : INFINITY;
    if (a.first_id) a.first_id[pixel] = first;
}

__global__ void k_debug_rays(TraceParams p, const int64_t *__restrict__ pix, int64_t n, float *__restrict__ dirs) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t q = pix[i];
    int px = (int)(q % p.W), py = (int)(q / p.W);
    float3 d = primary_dir(p, px, py);
    dirs[3 * i] = d.x;
    dirs[3 * i + 1] = d.y;
    dirs[3 * i + 2] = d.z;
}

}  // namespace

hipError_t launch_trace(vrt_ctx *c, const TraceParams &p, const vrt_image *img, hipStream_t st) {
    TraceArgs a;
    a.p = p;
    for (int k = 0; k < 3; ++k) {
        a.G[k] = c->dims[k];
        a.nb[k] = c->dims[k] / 8;
    }
    a.vis0 = c->a.vis0;
    a.vis3 = c->a.vis3;
    a.words = c->a.words;
    a.cursor = c->a.cursor;
    a.ids = c->a.ids;
    a.vrec = c->a.vrec;
    a.nv = c->n_vertices;
    a.capacity = c->desc.max_fragments;
    a.rgba = img->rgba;
    a.depth = img->depth;
    a.first_id = img->first_id;
    dim3 grid((p.W + 15) / 16, (p.H + 15) / 16);
    VRT_LAUNCH(c, "k_trace", st, k_trace<<<grid, 256, 0, st>>>(a));
    return hipGetLastError();
}

hipError_t launch_debug_rays(const TraceParams &p, const int64_t *pix, int64_t n, float *dirs, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_debug_rays<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, pix, n, dirs);
    return hipGetLastError();
}

}  // namespace vrt
