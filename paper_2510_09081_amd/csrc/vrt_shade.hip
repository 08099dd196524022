// vrt_shade.hip -- Section 3.4: voxel-space shading.  Ambient occlusion from
// cones traced through the occupancy pyramid and a directional shadow ray,
// evaluated once per visible voxel before ray tracing; the tracer then scales
// each hit's colour by the value of the voxel holding the hit point (one
// sample per ray-capsule hit).
#include <cmath>

#include "vrt_internal.h"

namespace vrt {
namespace {

constexpr int kShadeMaxCones = 64;
constexpr int kShadeMaxSamples = 6;

struct ShadeArgs {
    GridArgs g;
    const int32_t *slot;    // brick -> slot in the occupied-brick list, or -1
    const int32_t *list;    // occupied bricks
    const DevStatus *st;
    const uint8_t *vis0;
    const uint16_t *occ0, *occ1, *occ2, *occ3, *occ_hi;
    Level lv[kShadeMaxSamples + 1];  // levels 0..J (dims; offsets into occ_hi from level 4)
    int K, J;
    int U[3 * kShadeMaxCones];  // cone directions, 1/256 units
    int L[3];                   // light direction, 1/256 units
    float ambient;
    float *lit;                 // per voxel, brick-major
};

// Occupancy (fraction) of cell (x, y, z) of pyramid level L; 0 outside the
// level's grid and in unoccupied bricks.
__device__ __forceinline__ float occ_cell(const ShadeArgs &a, int L, int x, int y, int z) {
    const Level &lv = a.lv[L];
    if (x < 0 || y < 0 || z < 0 || x >= lv.dims[0] || y >= lv.dims[1] || z >= lv.dims[2]) return 0.0f;
    unsigned o;
    if (L >= 4) {
        o = a.occ_hi[lv.offset + ((int64_t)z * lv.dims[1] + y) * lv.dims[0] + x];
    } else if (L == 3) {  // one entry per brick, dense (zero in unoccupied bricks)
        o = a.occ3[((int64_t)z * a.g.nb[1] + y) * a.g.nb[0] + x];
    } else {  // per-brick blocks of (8 >> L)^3 cells, defined in occupied bricks only
        const int sh = 3 - L, m = (1 << sh) - 1;
        const int64_t b = ((int64_t)(z >> sh) * a.g.nb[1] + (y >> sh)) * a.g.nb[0] + (x >> sh);
        if (a.slot[b] < 0) return 0.0f;
        const int local = ((((z & m) << sh) | (y & m)) << sh) | (x & m);
        o = L == 0 ? a.occ0[b * kBrickVox + local] : (L == 1 ? a.occ1[b * 64 + local] : a.occ2[b * 8 + local]);
    }
    return (float)o * (1.0f / 256.0f);
}

// Transmittance toward the light from the centre of voxel p: the product of
// 1 - occupancy over the voxels the ray enters until it leaves the grid.  The
// walk is exact in 32-bit integers: the next crossing on axis k is the
// fraction n_k / d_k of the ray's unit step (d_k = |L_k|, n_k grows by one
// voxel per plane; every value stays below 2^27 on grids up to 1024^3), the
// smallest is taken, tied axes step together.  An unoccupied brick holds no
// occupancy, so the walk jumps to its exit: the axis whose far face comes
// first, and on every axis the planes crossed at or before that parameter.
// The walk stops once the transmittance is below kShadowEps, which moves the
// result by less than kShadowEps.
constexpr float kShadowEps = 1.0f / 65536.0f;

__device__ __forceinline__ float shadow_walk(const ShadeArgs &a, int p0, int p1, int p2) {
    int u[3] = {p0, p1, p2};
    int n[3] = {kQ / 2, kQ / 2, kQ / 2};
    int d[3], s[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d[k] = a.L[k] < 0 ? -a.L[k] : a.L[k];
        s[k] = a.L[k] > 0 ? 1 : -1;
    }
    float T = 1.0f;
    for (int guard = 0; guard < 4 * (a.g.G[0] + a.g.G[1] + a.g.G[2]); ++guard) {
        // one crossing: the smallest n/d over the stepping axes, ties together
        int bn = 0, bd = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (d[k] && (!bd || n[k] * bd < bn * d[k])) bn = n[k], bd = d[k];
        if (!bd) break;
        bool out = false;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (d[k] && n[k] * bd == bn * d[k]) {
                u[k] += s[k];
                n[k] += kQ;
                out |= u[k] < 0 || u[k] >= a.g.G[k];
            }
        if (out) break;
        const int64_t b = ((int64_t)(u[2] >> 3) * a.g.nb[1] + (u[1] >> 3)) * a.g.nb[0] + (u[0] >> 3);
        if (a.slot[b] >= 0) {
            const int local = ((u[2] & 7) << 6) | ((u[1] & 7) << 3) | (u[0] & 7);
            T = T * (1.0f - (float)a.occ0[b * kBrickVox + local] * (1.0f / 256.0f));
            if (T < kShadowEps) break;
            continue;
        }
        // an unoccupied brick: its exit parameter N/D is the first far-face crossing
        int N = 0, D = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (!d[k]) continue;
            const int lo = u[k] & ~7;
            const int cross = s[k] > 0 ? lo + 8 - u[k] : u[k] - lo + 1;  // planes to the far face, that one included
            const int e = n[k] + (cross - 1) * kQ;
            if (!D || e * D < N * d[k]) N = e, D = d[k];
        }
        // every plane crossed at or before N/D is passed: the walk resumes in the voxel after the exit
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (!d[k] || n[k] * D > N * d[k]) continue;
            const int c = (N * d[k] - n[k] * D) / (kQ * D) + 1;
            u[k] += s[k] * c;
            n[k] += c * kQ;
            out |= u[k] < 0 || u[k] >= a.g.G[k];
        }
        if (out) break;
        const int64_t b2 = ((int64_t)(u[2] >> 3) * a.g.nb[1] + (u[1] >> 3)) * a.g.nb[0] + (u[0] >> 3);
        if (a.slot[b2] >= 0) {
            const int local = ((u[2] & 7) << 6) | ((u[1] & 7) << 3) | (u[0] & 7);
            T = T * (1.0f - (float)a.occ0[b2 * kBrickVox + local] * (1.0f / 256.0f));
            if (T < kShadowEps) break;
        }
    }
    return T;
}

// One workgroup (512 threads, one voxel each) per occupied brick.
__global__ void __launch_bounds__(512) k_shade(ShadeArgs a) {
    const unsigned nbk = a.st->n_bricks;
    const int t = threadIdx.x;
    for (unsigned sl = blockIdx.x; sl < nbk; sl += gridDim.x) {
        const int64_t b = a.list[sl];
        const int64_t vi = b * kBrickVox + t;
        if (!a.vis0[vi]) continue;
        int bx, by, bz;
        brick_xyz((uint32_t)b, a.g.nb, bx, by, bz);
        const int p0 = 8 * bx + (t & 7), p1 = 8 * by + ((t >> 3) & 7), p2 = 8 * bz + (t >> 6);
        // voxel centre in 1/256 units (below 2^18 on grids up to 1024^3: 32-bit arithmetic is exact)
        const int C0 = p0 * kQ + kQ / 2, C1 = p1 * kQ + kQ / 2, C2 = p2 * kQ + kQ / 2;
        // ambient occlusion: sample j of cone k at 2^j voxels, in the level-j cell holding it
        float sum = 0.0f;
        for (int k = 0; k < a.K; ++k) {
            float acc = 0.0f;
            for (int j = 1; j <= a.J; ++j) {
                const int step = 1 << j;  // 2^j voxels; the arithmetic shift below is a floor division
                const int x = (C0 + a.U[3 * k] * step) >> (8 + j);
                const int y = (C1 + a.U[3 * k + 1] * step) >> (8 + j);
                const int z = (C2 + a.U[3 * k + 2] * step) >> (8 + j);
                acc = acc + (1.0f - acc) * occ_cell(a, j, x, y, z);
            }
            sum = sum + (1.0f - acc);
        }
        const float ao = sum / (float)a.K;
        // shadow: integer walk from the voxel centre along L to the grid edge (tied axes step together)
        const float T = shadow_walk(a, p0, p1, p2);
        a.lit[vi] = ao * (a.ambient + (1.0f - a.ambient) * T);
    }
}

}  // namespace

// Host side of vrt_shade: cone and light directions in binary64, rounded to
// integers in 1/256 units.
vrt_status shade_params(const vrt_ctx *c, const vrt_shading *s, int *U, int *L) {
    if (s->n_cones < 1 || s->n_cones > kShadeMaxCones || s->n_samples < 1 || s->n_samples > kShadeMaxSamples ||
        s->n_samples >= c->n_levels || !(s->ambient >= 0.0f && s->ambient <= 1.0f))
        return VRT_ERR_INVALID_ARG;
    const double lx = s->light_dir[0], ly = s->light_dir[1], lz = s->light_dir[2];
    const double ln = std::sqrt(lx * lx + ly * ly + lz * lz);
    if (!(ln > 0.0) || !std::isfinite(ln)) return VRT_ERR_INVALID_ARG;
    L[0] = (int)std::rint(256.0 * lx / ln);
    L[1] = (int)std::rint(256.0 * ly / ln);
    L[2] = (int)std::rint(256.0 * lz / ln);
    const double golden = M_PI * (3.0 - std::sqrt(5.0));
    for (int k = 0; k < s->n_cones; ++k) {
        const double z = 1.0 - (2.0 * k + 1.0) / (double)s->n_cones;
        const double r = std::sqrt(1.0 - z * z), phi = golden * (double)k;
        U[3 * k] = (int)std::rint(256.0 * r * std::cos(phi));
        U[3 * k + 1] = (int)std::rint(256.0 * r * std::sin(phi));
        U[3 * k + 2] = (int)std::rint(256.0 * z);
    }
    return VRT_OK;
}

hipError_t launch_shade(vrt_ctx *c, const vrt_shading *s, const int *U, const int *L, hipStream_t st) {
    ShadeArgs a;
    for (int k = 0; k < 3; ++k) {
        a.g.G[k] = c->dims[k];
        a.g.nb[k] = c->dims[k] / 8;
        a.g.ns[k] = (c->dims[k] + 63) / 64;
        a.L[k] = L[k];
    }
    a.slot = c->a.brick_slot;
    a.list = c->a.brick_list;
    a.st = c->a.status;
    a.vis0 = c->a.vis0;
    a.occ0 = c->a.occ0;
    a.occ1 = c->a.occ1;
    a.occ2 = c->a.occ2;
    a.occ3 = c->a.occ3;
    a.occ_hi = c->a.occ_hi;
    for (int j = 0; j <= kShadeMaxSamples; ++j) a.lv[j] = j < c->n_levels ? c->levels[j] : Level{};
    a.K = s->n_cones;
    a.J = s->n_samples;
    for (int k = 0; k < 3 * s->n_cones; ++k) a.U[k] = U[k];
    a.ambient = s->ambient;
    a.lit = c->a.lit;
    VRT_LAUNCH(c, "k_shade", st, k_shade<<<4096, 512, 0, st>>>(a));
    return hipGetLastError();
}

}  // namespace vrt
