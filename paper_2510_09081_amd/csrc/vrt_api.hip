// vrt_api.hip -- context, argument validation and the C ABI entry points.
#include <cmath>
#include <cstring>
#include <new>

#include "vrt_internal.h"

using namespace vrt;

namespace {

thread_local int32_t g_last_hip = 0;

vrt_status hip_fail(hipError_t e) {
    g_last_hip = (int32_t)e;
    return VRT_ERR_HIP;
}

#define VRT_HIP(call)                              \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_fail(e_); \
    } while (0)

template <class T>
hipError_t alloc(T *&p, int64_t n) {
    return hipMalloc((void **)&p, (size_t)(n > 0 ? n : 1) * sizeof(T));
}

void free_all(Arenas &a) {
    void *ptrs[] = {a.vrec, a.words, a.occ0, a.occ1, a.occ2, a.occ3, a.occ_hi, a.blk, a.blk_bits, a.brick_bits, a.super_blk,
                    a.occ_list, a.vis0,
                    a.vis1, a.vis2,  a.vis3, a.bskip, a.vis_hi, a.cursor, a.cell, a.lmask, a.lmask2, a.queue, a.walk, a.cont, a.srec16, a.ids, a.brick_flag, a.bin_count, a.bin_range, a.cand, a.bins, a.long_ids, a.items, a.chunk_cnt, a.brick_list, a.brick_slot,
                    a.brick_total, a.brick_base, a.status, a.lit, a.stat_vox, a.stat_seg, a.stat_acc};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    a = Arenas();
}

// Pyramid level dims: level L = ceil(dims / 2^L) down to 1^3.
int level_dims(const int dims[3], Level *lv) {
    int n = 0;
    int d[3] = {dims[0], dims[1], dims[2]};
    int64_t off = 0;
    for (;;) {
        for (int k = 0; k < 3; ++k) lv[n].dims[k] = d[k];
        lv[n].offset = 0;
        if (n >= 4) {
            lv[n].offset = off;
            off += (int64_t)d[0] * d[1] * d[2];
        }
        ++n;
        if (d[0] == 1 && d[1] == 1 && d[2] == 1) break;
        for (int k = 0; k < 3; ++k) d[k] = (d[k] + 1) / 2;
    }
    return n;
}

int64_t hi_elems_for(int max_dim) {
    Level lv[kMaxLevels + 1];
    int dims[3] = {max_dim, max_dim, max_dim};
    int n = level_dims(dims, lv);
    int64_t s = 0;
    for (int L = 4; L < n; ++L) s += (int64_t)lv[L].dims[0] * lv[L].dims[1] * lv[L].dims[2];
    return s;
}

// Capacities of a context derived from its description.
void ctx_sizes(vrt_ctx *c, const vrt_desc &d) {
    c->desc = d;
    const int64_t nbd = d.max_dim / 8;
    c->max_bricks = nbd * nbd * nbd;
    const int64_t nsd = (d.max_dim + 63) / 64;
    c->max_supers = nsd * nsd * nsd;
    c->hi_elems = hi_elems_for(d.max_dim);
    c->walk_entries = d.max_pixels * kWalkPerPixel;
}

// Every arena of a context with its element count: f(pointer, count) is called
// once per array, in one fixed order (allocation by vrt_create, placement in a
// fixed buffer by the no-allocation frame).
template <class F>
void arena_fields(Arenas &a, const vrt_desc &d, int64_t mb, int64_t hi_elems, int64_t walk_entries, F &&f) {
    f(a.vrec, d.max_vertices);
    f(a.words, mb * kBrickVox);
    f(a.occ0, mb * kBrickVox);
    f(a.occ1, mb * 64);
    f(a.occ2, mb * 8);
    f(a.occ3, mb);
    f(a.occ_hi, hi_elems);
    f(a.blk, mb * kBrickVox);
    f(a.blk_bits, mb * 16);
    {
        const int nbd = d.max_dim / 8;
        const int nbm[3] = {nbd, nbd, nbd};
        const CellFlagLayout cl = cell_flag_layout(nbm);
        f(a.brick_bits, cl.words);
        f(a.super_blk, cl.bytes);
    }
    f(a.occ_list, mb * kBrickVox);
    f(a.vis0, mb * kBrickVox);
    f(a.vis1, mb * 64);
    f(a.vis2, mb * 8);
    f(a.vis3, mb);
    f(a.bskip, mb);
    f(a.vis_hi, hi_elems);
    f(a.cursor, mb * kBrickVox);
    f(a.cell, mb * kBrickVox);
    f(a.lmask, mb * 8);
    f(a.lmask2, mb);
    f(a.queue, d.max_pixels);
    f(a.walk, walk_entries);
    f(a.cont, d.max_pixels);
    if (d.form == VRT_FORM_FP16) f(a.srec16, d.max_vertices);
    f(a.ids, d.max_fragments);
    f(a.brick_flag, mb);
    f(a.bin_count, mb * kBinStride);
    f(a.bin_range, mb);
    f(a.cand, mb);
    f(a.bins, (int64_t)kMaxBinBricks * d.max_vertices);
    f(a.long_ids, d.max_vertices);
    f(a.items, mb + (int64_t)kMaxBinBricks * d.max_vertices / kBinChunk + 1);
    f(a.chunk_cnt, mb / (1024 * 16) + 1);
    f(a.brick_list, mb);
    f(a.brick_slot, mb);
    f(a.brick_total, mb);
    f(a.brick_base, mb);
    f(a.status, 1);
    f(a.lit, mb * kBrickVox);
    f(a.stat_vox, mb * kBrickVox);
    f(a.stat_seg, d.max_vertices);
    f(a.stat_acc, 16);
}

bool finite3(const float *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Eye in 1/256 voxel, rounded in binary64; |E| < 2^22 keeps every later
// difference exact in binary32 and every culling product inside int64.
vrt_status quantize_eye(const vrt_ctx *c, const float *eye, int64_t E[3]) {
    if (!finite3(eye)) return VRT_ERR_INVALID_ARG;
    double s = 256.0 / (double)c->voxel_size;
    for (int k = 0; k < 3; ++k) {
        double q = std::rint(((double)eye[k] - (double)c->origin[k]) * s);
        if (!(std::fabs(q) < 4194304.0)) return VRT_ERR_RANGE;
        E[k] = (int64_t)q;
    }
    return VRT_OK;
}

}  // namespace

extern "C" {

vrt_status vrt_create(const vrt_desc *desc, vrt_ctx **out) {
    if (!desc || !out) return VRT_ERR_INVALID_ARG;
    *out = nullptr;
    if (desc->max_vertices < 2 || desc->max_fragments < 1 || desc->max_dim < 8 || desc->max_dim > 1024 ||
        desc->max_dim % 8 != 0 || desc->max_vertices > ((int64_t)1 << 31) || desc->max_fragments > 0xFFFFFFFFll ||
        desc->max_pixels < 1 || desc->max_pixels > ((int64_t)1 << 31) ||
        (desc->form != VRT_FORM_PLAIN && desc->form != VRT_FORM_FP16))
        return VRT_ERR_INVALID_ARG;
    int ndev = 0;
    VRT_HIP(hipGetDeviceCount(&ndev));
    if (desc->device < 0 || desc->device >= ndev) return VRT_ERR_INVALID_ARG;
    VRT_HIP(hipSetDevice(desc->device));
    vrt_ctx *c = new (std::nothrow) vrt_ctx();
    if (!c) return VRT_ERR_INVALID_ARG;
    ctx_sizes(c, *desc);
    Arenas &a = c->a;
    const int64_t mb = c->max_bricks;
    hipError_t e = hipSuccess;
    arena_fields(a, *desc, mb, c->hi_elems, c->walk_entries, [&](auto *&p, int64_t n) {
        if (e == hipSuccess) e = alloc(p, n);
    });
    if (e == hipSuccess) e = hipMemset(a.words, 0, (size_t)mb * kBrickVox * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(a.brick_flag, 0, (size_t)mb);
    if (e == hipSuccess) e = hipMemset(a.bin_count, 0, (size_t)mb * kBinStride * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(a.brick_slot, 0xFF, (size_t)mb * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(a.status, 0, sizeof(DevStatus));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_all(a);
        delete c;
        return hip_fail(e);
    }
    *out = c;
    return VRT_OK;
}

static void profiler_free(Profiler &p) {
    if (p.ev) {
        for (int i = 0; i < 2 * Profiler::kMaxPairs; ++i) (void)hipEventDestroy(p.ev[i]);
        delete[] p.ev;
        delete[] p.names;
    }
    p = Profiler();
}

vrt_status vrt_destroy(vrt_ctx *c) {
    if (!c) return VRT_ERR_INVALID_ARG;
    (void)hipSetDevice(c->desc.device);
    (void)hipDeviceSynchronize();
    profiler_free(c->prof);
    free_all(c->a);
    delete c;
    return VRT_OK;
}

// Validation and context state of one voxelization (shared by the plain and
// the batched paths); on success *s_q is the binary32 fixed-point scale.
static vrt_status prepare_voxelize(vrt_ctx *c, const vrt_lines *L, const vrt_grid *g, float *s_q) {
    if (!c || !L || !g) return VRT_ERR_INVALID_ARG;
    if (!L->xyz || !L->poly_offsets || L->n_polylines < 1 || L->n_vertices < 1 ||
        L->n_vertices > c->desc.max_vertices || L->n_polylines > L->n_vertices)
        return VRT_ERR_INVALID_ARG;
    if (!(L->radius >= 0.0f) || !std::isfinite(L->radius)) return VRT_ERR_INVALID_ARG;
    if (L->voxelizer != VRT_VOX_CAPSULE && L->voxelizer != VRT_VOX_THIN && L->voxelizer != VRT_VOX_AABB)
        return VRT_ERR_INVALID_ARG;
    if (!(L->alpha_default >= 0.0f && L->alpha_default <= 1.0f) || L->reserved != 0) return VRT_ERR_INVALID_ARG;
    if (L->rgba && ((uintptr_t)L->rgba % 16) != 0) return VRT_ERR_INVALID_ARG;
    if (!(g->voxel_size > 0.0f) || !std::isfinite(g->voxel_size) || !finite3(g->origin)) return VRT_ERR_INVALID_ARG;
    for (int k = 0; k < 3; ++k)
        if (g->dims[k] < 8 || g->dims[k] % 8 != 0 || g->dims[k] > c->desc.max_dim) return VRT_ERR_INVALID_ARG;
    const double rq = std::rint((double)L->radius * 256.0 / (double)g->voxel_size);
    if (!(rq <= 16384.0)) return VRT_ERR_RANGE;
    for (int k = 0; k < 3; ++k) {
        c->dims[k] = g->dims[k];
        c->origin[k] = g->origin[k];
    }
    c->voxel_size = g->voxel_size;
    c->rq = (int64_t)rq;
    c->n_vertices = L->n_vertices;
    c->voxelizer = L->voxelizer;
    c->seg_rgba = L->rgba;
    c->alpha_default = L->alpha_default;
    c->n_levels = level_dims(c->dims, c->levels);
    c->voxelized = false;
    c->culled = false;
    *s_q = (float)(256.0 / (double)g->voxel_size);
    return VRT_OK;
}

vrt_status vrt_voxelize(vrt_ctx *c, const vrt_lines *L, const vrt_grid *g, void *stream) {
    float s_q;
    const vrt_status s = prepare_voxelize(c, L, g, &s_q);
    if (s != VRT_OK) return s;
    VRT_HIP(hipSetDevice(c->desc.device));
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    VRT_HIP(launch_voxelize(c, L, s_q, st));
    c->voxelized = true;
    return VRT_OK;
}

// Validation of one view: the eye in 1/256 voxel and the blocking limit
// (-1: no culling; 1: opaque; else the alpha layers until transmittance < tau).
static vrt_status prepare_cull(const vrt_ctx *c, const vrt_view *v, int64_t E[3], int64_t *limit) {
    if (!c || !v) return VRT_ERR_INVALID_ARG;
    if (!c->voxelized) return VRT_ERR_NOT_BUILT;
    if (v->cull_mode == VRT_CULL_NONE) {
        *limit = -1;
    } else if (v->cull_mode == VRT_CULL_OPAQUE) {
        *limit = 1;
    } else if (v->cull_mode == VRT_CULL_ALPHA) {
        if (!(v->alpha > 0.0f && v->alpha <= 1.0f) || !(v->tau > 0.0f && v->tau < 1.0f)) return VRT_ERR_INVALID_ARG;
        double T = 1.0;
        int64_t k = 0;
        while (!(T < (double)v->tau)) {
            T *= 1.0 - (double)v->alpha;
            ++k;
        }
        *limit = k < 1 ? 1 : k;
    } else {
        return VRT_ERR_INVALID_ARG;
    }
    return quantize_eye(c, v->eye, E);
}

vrt_status vrt_cull(vrt_ctx *c, const vrt_view *v, void *stream) {
    int64_t E[3], limit;
    const vrt_status s = prepare_cull(c, v, E, &limit);
    if (s != VRT_OK) return s;
    VRT_HIP(hipSetDevice(c->desc.device));
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    c->culled = false;
    c->shaded = false;
    VRT_HIP(launch_cull(c, E, limit, st));
    c->culled = true;
    return VRT_OK;
}

vrt_status vrt_shade(vrt_ctx *c, const vrt_shading *sh, void *stream) {
    if (!c || !sh || sh->reserved != 0) return VRT_ERR_INVALID_ARG;
    if (!c->culled) return VRT_ERR_NOT_BUILT;
    if (!sh->enable) {
        c->shaded = false;
        return VRT_OK;
    }
    int U[3 * 64], L[3];
    const vrt_status s = shade_params(c, sh, U, L);
    if (s != VRT_OK) return s;
    VRT_HIP(hipSetDevice(c->desc.device));
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    VRT_HIP(launch_shade(c, sh, U, L, st));
    c->shaded = true;
    return VRT_OK;
}

vrt_status vrt_sort_lists(vrt_ctx *c, void *stream) {
    if (!c) return VRT_ERR_INVALID_ARG;
    if (!c->culled) return VRT_ERR_NOT_BUILT;
    VRT_HIP(hipSetDevice(c->desc.device));
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    VRT_HIP(launch_sort_lists(c, st));
    return VRT_OK;
}

static vrt_status camera_params(const vrt_ctx *c, const vrt_camera *cam, TraceParams &p) {
    if (!finite3(cam->eye) || !finite3(cam->target) || !finite3(cam->up)) return VRT_ERR_INVALID_ARG;
    if (cam->width < 1 || cam->height < 1 || cam->width > 65536 || cam->height > 65536 ||
        (int64_t)cam->width * cam->height > c->desc.max_pixels)
        return VRT_ERR_INVALID_ARG;
    if (!(cam->fovy_deg > 0.0f && cam->fovy_deg < 180.0f)) return VRT_ERR_INVALID_ARG;
    if (cam->mode != VRT_TRACE_OPAQUE && cam->mode != VRT_TRACE_TRANSPARENT) return VRT_ERR_INVALID_ARG;
    if (cam->mode == VRT_TRACE_TRANSPARENT &&
        (!(cam->alpha > 0.0f && cam->alpha <= 1.0f) || !(cam->tau > 0.0f && cam->tau < 1.0f)))
        return VRT_ERR_INVALID_ARG;
    // camera basis in binary64, rounded once to binary32
    double f[3], r[3], u[3];
    for (int k = 0; k < 3; ++k) f[k] = (double)cam->target[k] - (double)cam->eye[k];
    double nf = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(nf > 0.0)) return VRT_ERR_INVALID_ARG;
    for (int k = 0; k < 3; ++k) f[k] = f[k] / nf;
    const double up0 = cam->up[0], up1 = cam->up[1], up2 = cam->up[2];
    r[0] = f[1] * up2 - f[2] * up1;
    r[1] = f[2] * up0 - f[0] * up2;
    r[2] = f[0] * up1 - f[1] * up0;
    double nr = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(nr > 0.0)) return VRT_ERR_INVALID_ARG;
    for (int k = 0; k < 3; ++k) r[k] = r[k] / nr;
    u[0] = r[1] * f[2] - r[2] * f[1];
    u[1] = r[2] * f[0] - r[0] * f[2];
    u[2] = r[0] * f[1] - r[1] * f[0];
    const double th = std::tan((double)cam->fovy_deg * M_PI / 360.0);
    const double aspect = (double)cam->width / (double)cam->height;
    for (int k = 0; k < 3; ++k) {
        p.F[k] = (float)f[k];
        p.R[k] = (float)(r[k] * (th * aspect));
        p.U[k] = (float)(u[k] * th);
    }
    int64_t E[3];
    vrt_status s = quantize_eye(c, cam->eye, E);
    if (s != VRT_OK) return s;
    for (int k = 0; k < 3; ++k) p.O[k] = (float)E[k] / 256.0f;
    p.W = cam->width;
    p.H = cam->height;
    p.mode = cam->mode;
    p.alpha = cam->mode == VRT_TRACE_TRANSPARENT ? (c->alpha_default > 0.0f ? c->alpha_default : cam->alpha) : 1.0f;
    p.seg_rgba = reinterpret_cast<const float4 *>(c->seg_rgba);
    p.lit = c->shaded ? c->a.lit : nullptr;
    p.tau = cam->mode == VRT_TRACE_TRANSPARENT ? cam->tau : 0.5f;
    p.radius = (float)c->rq / 256.0f;
    p.voxel_size = c->voxel_size;
    return VRT_OK;
}

vrt_status vrt_trace(vrt_ctx *c, const vrt_camera *cam, const vrt_image *img, void *stream) {
    if (!c || !cam || !img || !img->rgba) return VRT_ERR_INVALID_ARG;
    if (!c->culled) return VRT_ERR_NOT_BUILT;
    TraceParams p;
    vrt_status s = camera_params(c, cam, p);
    if (s != VRT_OK) return s;
    VRT_HIP(hipSetDevice(c->desc.device));
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    VRT_HIP(launch_trace(c, p, img, st));
    return VRT_OK;
}

vrt_status vrt_trace_stats_run(vrt_ctx *c, const vrt_camera *cam, const vrt_image *img, vrt_trace_stats *out,
                               void *stream) {
    if (!c || !cam || !img || !img->rgba || !out) return VRT_ERR_INVALID_ARG;
    if (!c->culled) return VRT_ERR_NOT_BUILT;
    TraceParams p;
    vrt_status s = camera_params(c, cam, p);
    if (s != VRT_OK) return s;
    VRT_HIP(hipSetDevice(c->desc.device));
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    VRT_HIP(launch_trace_stats(c, p, img, st));
    VRT_HIP(hipStreamSynchronize(st));
    unsigned long long acc[16];
    VRT_HIP(hipMemcpy(acc, c->a.stat_acc, sizeof(acc), hipMemcpyDeviceToHost));
    out->rays = (int64_t)cam->width * cam->height;
    out->rays_hit = (int64_t)acc[0];
    out->cell_skips_64 = (int64_t)acc[1];
    out->cell_skips_8 = (int64_t)acc[2];
    out->voxel_steps = (int64_t)acc[3];
    out->list_visits = (int64_t)acc[4];
    out->capsule_tests = (int64_t)acc[5];
    out->kbuffer_passes = (int64_t)acc[6];
    out->max_tests_per_ray = (int64_t)acc[7];
    out->distinct_list_voxels = (int64_t)acc[8];
    out->distinct_list_entries = (int64_t)acc[9];
    out->distinct_segments = (int64_t)acc[10];
    return VRT_OK;
}

vrt_status vrt_debug_rays(vrt_ctx *c, const vrt_camera *cam, const int64_t *pixels, int64_t n, float *dirs,
                          void *stream) {
    if (!c || !cam || (n > 0 && (!pixels || !dirs)) || n < 0) return VRT_ERR_INVALID_ARG;
    if (!c->voxelized) return VRT_ERR_NOT_BUILT;
    TraceParams p;
    vrt_status s = camera_params(c, cam, p);
    if (s != VRT_OK) return s;
    VRT_HIP(hipSetDevice(c->desc.device));
    VRT_HIP(launch_debug_rays(p, pixels, n, dirs, (hipStream_t)stream));
    return VRT_OK;
}

vrt_status vrt_frame_status(vrt_ctx *c, vrt_frame_info *out) {
    if (!c || !out) return VRT_ERR_INVALID_ARG;
    VRT_HIP(hipSetDevice(c->desc.device));
    VRT_HIP(hipStreamSynchronize(c->last_stream));
    DevStatus h;
    VRT_HIP(hipMemcpy(&h, c->a.status, sizeof(DevStatus), hipMemcpyDeviceToHost));
    vrt_status ds = VRT_OK;
    if (h.err & kErrInvalid) ds = VRT_ERR_INVALID_ARG;
    else if (h.err & kErrRange) ds = VRT_ERR_RANGE;
    else if (h.err & kErrCount) ds = VRT_ERR_COUNT_OVERFLOW;
    else if (h.err & kErrCapacity) ds = VRT_ERR_CAPACITY;
    unsigned zero = 0;
    VRT_HIP(hipMemcpy(&c->a.status->err, &zero, sizeof(unsigned), hipMemcpyHostToDevice));
    out->device_status = ds;
    out->n_fragments = (int64_t)h.n_fragments;
    out->n_listed = (int64_t)h.n_listed;
    out->n_bricks = (int64_t)h.n_bricks;
    out->required_fragments = (int64_t)h.n_listed;
    out->n_occupied = (int64_t)h.n_occ;
    unsigned long long nvis = 0;
    for (int k = 0; k < kStripes; ++k) nvis += h.stripe[k].vvis;
    out->n_visible = (int64_t)nvis;
    return VRT_OK;
}

vrt_status vrt_query_as(vrt_ctx *c, vrt_as_view *o) {
    if (!c || !o) return VRT_ERR_INVALID_ARG;
    if (!c->voxelized) return VRT_ERR_NOT_BUILT;
    VRT_HIP(hipSetDevice(c->desc.device));
    VRT_HIP(hipStreamSynchronize(c->last_stream));
    unsigned nb = 0;
    VRT_HIP(hipMemcpy(&nb, &c->a.status->n_bricks, sizeof(unsigned), hipMemcpyDeviceToHost));
    std::memset(o, 0, sizeof(*o));
    for (int k = 0; k < 3; ++k) o->dims[k] = c->dims[k];
    o->n_levels = c->n_levels;
    o->n_bricks = (int32_t)nb;
    const Arenas &a = c->a;
    o->brick_list = a.brick_list;
    o->words = a.words;
    o->occ[0] = a.occ0;
    o->occ[1] = a.occ1;
    o->occ[2] = a.occ2;
    o->occ[3] = a.occ3;
    o->occ_hi = a.occ_hi;
    o->blocking = a.blk;
    o->vis[0] = a.vis0;
    o->vis[1] = a.vis1;
    o->vis[2] = a.vis2;
    o->vis[3] = a.vis3;
    o->vis_hi = a.vis_hi;
    o->list_end = a.cursor;
    o->ids = a.ids;
    o->lit = a.lit;
    return VRT_OK;
}

vrt_status vrt_copy_to_host(void *dst, const void *src, int64_t bytes) {
    if (bytes < 0 || (bytes > 0 && (!dst || !src))) return VRT_ERR_INVALID_ARG;
    if (bytes == 0) return VRT_OK;
    VRT_HIP(hipMemcpy(dst, src, (size_t)bytes, hipMemcpyDeviceToHost));
    return VRT_OK;
}

vrt_status vrt_profile_enable(vrt_ctx *c, int32_t enable) {
    if (!c) return VRT_ERR_INVALID_ARG;
    VRT_HIP(hipSetDevice(c->desc.device));
    Profiler &p = c->prof;
    if (enable && !p.ev) {
        p.ev = new (std::nothrow) hipEvent_t[2 * Profiler::kMaxPairs];
        p.names = new (std::nothrow) const char *[Profiler::kMaxPairs];
        if (!p.ev || !p.names) {
            delete[] p.ev;
            delete[] p.names;
            p = Profiler();
            return VRT_ERR_INVALID_ARG;
        }
        for (int i = 0; i < 2 * Profiler::kMaxPairs; ++i) {
            hipError_t e = hipEventCreate(&p.ev[i]);
            if (e != hipSuccess) {
                for (int k = 0; k < i; ++k) (void)hipEventDestroy(p.ev[k]);
                delete[] p.ev;
                delete[] p.names;
                p = Profiler();
                return hip_fail(e);
            }
        }
    }
    p.enabled = enable != 0 && p.ev != nullptr;
    p.used = 0;
    p.overflow = false;
    return VRT_OK;
}

vrt_status vrt_profile_read(vrt_ctx *c, vrt_kernel_time *out, int32_t max_records, int32_t *n_records) {
    if (!c || !n_records || max_records < 0 || (max_records > 0 && !out)) return VRT_ERR_INVALID_ARG;
    VRT_HIP(hipSetDevice(c->desc.device));
    Profiler &p = c->prof;
    *n_records = 0;
    if (p.used > 0) VRT_HIP(hipEventSynchronize(p.ev[2 * p.used - 1]));
    for (int i = 0; i < p.used; ++i) {
        float ms = 0.0f;
        VRT_HIP(hipEventElapsedTime(&ms, p.ev[2 * i], p.ev[2 * i + 1]));
        int k = 0;
        for (; k < *n_records; ++k)
            if (std::strncmp(out[k].name, p.names[i], sizeof(out[k].name)) == 0) break;
        if (k == *n_records) {
            if (k >= max_records) continue;
            std::memset(out[k].name, 0, sizeof(out[k].name));
            std::strncpy(out[k].name, p.names[i], sizeof(out[k].name) - 1);
            out[k].launches = 0;
            out[k].total_ms = 0.0;
            ++*n_records;
        }
        out[k].launches += 1;
        out[k].total_ms += ms;
    }
    const bool over = p.overflow;
    p.used = 0;
    p.overflow = false;
    return over ? VRT_ERR_CAPACITY : VRT_OK;
}

struct vrt_graph {
    vrt_ctx *ctx;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

vrt_status vrt_graph_create(vrt_ctx *c, const vrt_lines *lines, const vrt_grid *grid, const vrt_view *views,
                            const vrt_camera *cams, const vrt_image *imgs, int32_t n_passes, vrt_graph **out) {
    if (!c || !lines || !grid || !out || n_passes < 0 || (n_passes > 0 && (!views || !cams || !imgs)))
        return VRT_ERR_INVALID_ARG;
    *out = nullptr;
    VRT_HIP(hipSetDevice(c->desc.device));
    const bool prof = c->prof.enabled;
    c->prof.enabled = false;  // no event records inside the graph
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        c->prof.enabled = prof;
        return hip_fail(e);
    }
    hipGraph_t graph = nullptr;
    vrt_status st = VRT_OK;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = vrt_voxelize(c, lines, grid, cap);
        for (int32_t i = 0; st == VRT_OK && i < n_passes; ++i) {
            st = vrt_cull(c, &views[i], cap);
            if (st == VRT_OK) st = vrt_trace(c, &cams[i], &imgs[i], cap);
        }
        hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (e2 != hipSuccess && st == VRT_OK) st = hip_fail(e2);
    } else {
        st = hip_fail(e);
    }
    hipGraphExec_t exec = nullptr;
    if (st == VRT_OK) {
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) st = hip_fail(e);
    }
    (void)hipStreamDestroy(cap);
    c->prof.enabled = prof;
    c->last_stream = nullptr;
    if (st != VRT_OK) {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    vrt_graph *g = new (std::nothrow) vrt_graph{c, graph, exec};
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return VRT_ERR_INVALID_ARG;
    }
    *out = g;
    return VRT_OK;
}

vrt_status vrt_graph_launch(vrt_graph *g, void *stream) {
    if (!g) return VRT_ERR_INVALID_ARG;
    VRT_HIP(hipSetDevice(g->ctx->desc.device));
    VRT_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    g->ctx->last_stream = (hipStream_t)stream;
    return VRT_OK;
}

vrt_status vrt_graph_destroy(vrt_graph *g) {
    if (!g) return VRT_ERR_INVALID_ARG;
    (void)hipSetDevice(g->ctx->desc.device);
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
    return VRT_OK;
}

int32_t vrt_last_hip_error(void) { return g_last_hip; }

const char *vrt_status_string(vrt_status s) {
    switch (s) {
    case VRT_OK: return "ok";
    case VRT_ERR_INVALID_ARG: return "invalid argument";
    case VRT_ERR_RANGE: return "coordinate or length outside the fixed-point range";
    case VRT_ERR_NOT_BUILT: return "acceleration structure not built for this call";
    case VRT_ERR_CAPACITY: return "listed fragments exceed the context capacity";
    case VRT_ERR_COUNT_OVERFLOW: return "more than 65535 fragments in one voxel";
    case VRT_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// One frame without allocation, for callers that cannot allocate device
// memory.  The acceleration structure lives in `scratch`, one fixed array per
// device; host code reaches it only through the address hipGetSymbolAddress
// returns for that device (the array's name is a host-side stand-in).

#include <mutex>
#include <type_traits>

static __device__ __align__(256) unsigned char scratch[VRT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoAllocDevices = 64;

struct NoAllocSlot {
    bool ready = false;
    unsigned char *ptr = nullptr;  // this device's copy of scratch
    vrt_ctx ctx;                   // host state of the frame; its arenas are placed in ptr
};
NoAllocSlot g_noalloc[kNoAllocDevices];
std::mutex g_noalloc_mu;

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void fill_u32(void *p, int64_t n, uint32_t v, hipStream_t st) {
    if (n <= 0) return;
    const int64_t blocks = (n + 255) / 256;
    k_fill_u32<<<(unsigned)(blocks < 1024 ? blocks : 1024), 256, 0, st>>>((uint32_t *)p, n, v);
}

// The current device's slot; on its first use looks up the device address of
// scratch and places every arena in it.
vrt_status noalloc_slot(NoAllocSlot **out) {
    int dev = 0;
    VRT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocDevices) return VRT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    NoAllocSlot &s = g_noalloc[dev];
    if (!s.ready) {
        void *p = nullptr;
        VRT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        vrt_desc d = {VRT_NOALLOC_MAX_VERTICES, VRT_NOALLOC_MAX_FRAGMENTS, VRT_NOALLOC_MAX_DIM, dev,
                      VRT_NOALLOC_MAX_PIXELS, VRT_FORM_PLAIN, 0};
        vrt_ctx &c = s.ctx;
        ctx_sizes(&c, d);
        c.walk_entries = (int64_t)VRT_NOALLOC_MAX_PIXELS * 4;  // half the usual walk budget: rays past it march on
        unsigned char *base = static_cast<unsigned char *>(p);
        size_t off = 0;
        arena_fields(c.a, d, c.max_bricks, c.hi_elems, c.walk_entries, [&](auto *&q, int64_t n) {
            using T = std::remove_reference_t<decltype(*q)>;
            off = (off + 255) & ~(size_t)255;
            q = reinterpret_cast<T *>(base + off);
            off += (size_t)(n > 0 ? n : 1) * sizeof(T);
        });
        if (off > (size_t)VRT_NOALLOC_SCRATCH_BYTES) {  // the limits above do not fit the array
            c = vrt_ctx();
            return VRT_ERR_CAPACITY;
        }
        s.ptr = base;
        s.ready = true;
    }
    *out = &s;
    return VRT_OK;
}

}  // namespace

extern "C" vrt_status vrt_frame_noalloc(const vrt_lines *lines, const vrt_grid *grid, const vrt_view *view,
                                        const vrt_camera *cam, const vrt_image *img, vrt_frame_info *info,
                                        void *stream) {
    if (!lines || !grid || !view || !cam || !img || !img->rgba) return VRT_ERR_INVALID_ARG;
    if (lines->n_vertices > VRT_NOALLOC_MAX_VERTICES || grid->dims[0] > VRT_NOALLOC_MAX_DIM ||
        grid->dims[1] > VRT_NOALLOC_MAX_DIM || grid->dims[2] > VRT_NOALLOC_MAX_DIM ||
        (int64_t)cam->width * (int64_t)cam->height > VRT_NOALLOC_MAX_PIXELS)
        return VRT_ERR_CAPACITY;
    NoAllocSlot *s = nullptr;
    vrt_status r = noalloc_slot(&s);
    if (r != VRT_OK) return r;
    vrt_ctx *c = &s->ctx;
    // every argument is validated before anything is enqueued
    float s_q;
    r = prepare_voxelize(c, lines, grid, &s_q);
    if (r != VRT_OK) return r;
    c->voxelized = true;
    int64_t E[3], limit;
    r = prepare_cull(c, view, E, &limit);
    if (r != VRT_OK) return r;
    TraceParams p;
    r = camera_params(c, cam, p);
    if (r != VRT_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    // the previous call's contents: clear what the frame expects at zero
    // (words, brick flags, bin counters, status) and the brick-slot map
    const Arenas &A = c->a;
    const int64_t nb = (int64_t)(c->dims[0] / 8) * (c->dims[1] / 8) * (c->dims[2] / 8);
    fill_u32(A.words, nb * kBrickVox, 0u, st);
    fill_u32(A.brick_flag, (nb + 3) / 4, 0u, st);
    fill_u32(A.bin_count, nb * kBinStride, 0u, st);
    fill_u32(A.brick_slot, nb, 0xFFFFFFFFu, st);
    fill_u32(A.status, (int64_t)(sizeof(DevStatus) / 4), 0u, st);
    VRT_HIP(hipGetLastError());
    VRT_HIP(launch_voxelize(c, lines, s_q, st));
    VRT_HIP(launch_cull(c, E, limit, st));
    c->culled = true;
    VRT_HIP(launch_trace(c, p, img, st));
    if (info) return vrt_frame_status(c, info);
    return VRT_OK;
}
