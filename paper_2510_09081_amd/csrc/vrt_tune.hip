// vrt_tune.hip -- launch-shape setting and the host-timed autotuners.
//
// The tracer's launch shape (march block size, lanes per ray, records fetched
// together, keys per lane, shade grid) changes only the time of a trace, not
// its image: every shape computes the same (t, id) keys and composites them in
// the same order.  The shape autotuner times shapes on the caller's own frame
// and keeps the fastest; results can be kept in a small JSON cache file.
//
// The grid resolution is the other free parameter: the grid only narrows the
// search for hits (voxelization and culling are conservative), so every grid
// yields the same hits up to binary32 rounding of the hit parameters, while
// list lengths, fragment counts and walk lengths change.  The grid autotuner
// times whole frames for caller-given candidate grids.
#include <unistd.h>

#include <cstdio>
#include <map>
#include <string>

using namespace vrt;

namespace {

const char *kTuneFormat =
    "{\"march_threads\": %d, \"shade_group\": %d, \"shade_batch\": %d, \"lane_keys\": %d, \"shade_blocks\": %d, "
    "\"ms\": %f}";

struct TuneEntry {
    vrt_tune t;
    float ms;
};

// Cache key: device architecture, form, mode, grid, image, vertex count and the caller's name.
std::string tune_key(const vrt_ctx *c, const TraceParams &p, const char *user) {
    hipDeviceProp_t prop;
    std::string arch = hipGetDeviceProperties(&prop, c->desc.device) == hipSuccess ? prop.gcnArchName : "unknown";
    char buf[256];
    std::snprintf(buf, sizeof(buf), "|%s|%s|%dx%dx%d|%dx%d|%lld|", c->desc.form == VRT_FORM_FP16 ? "fp16" : "plain",
                  p.mode == VRT_TRACE_OPAQUE ? "opaque" : "transparent", c->dims[0], c->dims[1], c->dims[2], p.W, p.H,
                  (long long)c->n_vertices);
    std::string k = arch + buf + (user ? user : "");
    for (char &ch : k)  // keep the key a plain JSON string
        if (ch == '"' || ch == '\\' || (unsigned char)ch < 0x20) ch = '_';
    return k;
}

// Reads the entries of a cache file written by tune_store; lines that do not
// parse are skipped.
std::map<std::string, TuneEntry> tune_load(const char *path) {
    std::map<std::string, TuneEntry> m;
    FILE *f = std::fopen(path, "r");
    if (!f) return m;
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        const char *q0 = std::strchr(line, '"');
        if (!q0) continue;
        const char *q1 = std::strchr(q0 + 1, '"');
        if (!q1) continue;
        const char *colon = std::strchr(q1, ':');
        if (!colon) continue;
        TuneEntry e;
        std::memset(&e, 0, sizeof(e));
        const char *body = colon + 1;
        while (*body == ' ') ++body;
        if (std::sscanf(body, kTuneFormat, &e.t.march_threads, &e.t.shade_group, &e.t.shade_batch, &e.t.lane_keys,
                        &e.t.shade_blocks, &e.ms) != 6)
            continue;
        if (!tune_valid(e.t)) continue;
        m[std::string(q0 + 1, q1)] = e;
    }
    std::fclose(f);
    return m;
}

// Rewrites the cache file through a temporary file in the same directory.
void tune_store(const char *path, const std::map<std::string, TuneEntry> &m) {
    const std::string tmp = std::string(path) + ".tmp." + std::to_string((long long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fputs("{\n", f);
    size_t i = 0;
    for (const auto &kv : m) {
        std::fprintf(f, "\"%s\": ", kv.first.c_str());
        std::fprintf(f, kTuneFormat, kv.second.t.march_threads, kv.second.t.shade_group, kv.second.t.shade_batch,
                     kv.second.t.lane_keys, kv.second.t.shade_blocks, (double)kv.second.ms);
        std::fputs(++i < m.size() ? ",\n" : "\n", f);
    }
    std::fputs("}\n", f);
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), path);
    else std::remove(tmp.c_str());
}

// Mean time of `reps` traces with shape t, after `warmup` untimed ones.
vrt_status time_shape(vrt_ctx *c, const TraceParams &p, const vrt_image *img, hipStream_t st, const vrt_tune &t,
                      int warmup, int reps, hipEvent_t e0, hipEvent_t e1, float &ms) {
    c->tune[p.mode == VRT_TRACE_OPAQUE ? 0 : 1] = t;
    for (int i = 0; i < warmup; ++i) VRT_HIP(launch_trace(c, p, img, st));
    VRT_HIP(hipEventRecord(e0, st));
    for (int i = 0; i < reps; ++i) VRT_HIP(launch_trace(c, p, img, st));
    VRT_HIP(hipEventRecord(e1, st));
    VRT_HIP(hipEventSynchronize(e1));
    float total = 0.0f;
    VRT_HIP(hipEventElapsedTime(&total, e0, e1));
    ms = total / (float)reps;
    return VRT_OK;
}

int32_t *tune_field(vrt_tune &t, int k) {
    switch (k) {
        case 0: return &t.march_threads;
        case 1: return &t.shade_group;
        case 2: return &t.shade_batch;
        case 3: return &t.lane_keys;
        default: return &t.shade_blocks;
    }
}

vrt_status search(vrt_ctx *c, const TraceParams &p, const vrt_tune_space *sp, hipStream_t st, hipEvent_t e0,
                  hipEvent_t e1, vrt_tune_result *out) {
    static const int32_t kValues[5][5] = {
        {128, 256, 512, 0, 0}, {8, 16, 32, 0, 0}, {2, 4, 0, 0, 0}, {4, 8, 0, 0, 0}, {1024, 2048, 4096, 8192, 16384}};
    const int mi = p.mode == VRT_TRACE_OPAQUE ? 0 : 1;
    vrt_tune cur = c->tune[mi];
    float cur_ms = 0.0f;
    vrt_status s = time_shape(c, p, sp->image, st, cur, sp->warmup, sp->reps, e0, e1, cur_ms);
    if (s != VRT_OK) return s;
    out->start_ms = cur_ms;
    out->evaluated = 1;
    for (int sweep = 0; sweep < sp->sweeps; ++sweep) {
        bool changed = false;
        for (int k = 0; k < 5; ++k) {
            if (k == 3 && p.mode == VRT_TRACE_OPAQUE) continue;  // keys per lane: transparent only
            const int32_t timed = *tune_field(cur, k);  // the value cur_ms was measured with
            for (int j = 0; j < 5 && kValues[k][j]; ++j) {
                if (kValues[k][j] == timed) continue;
                vrt_tune cand = cur;
                *tune_field(cand, k) = kValues[k][j];
                float ms = 0.0f;
                s = time_shape(c, p, sp->image, st, cand, sp->warmup, sp->reps, e0, e1, ms);
                if (s != VRT_OK) return s;
                ++out->evaluated;
                if (ms < 0.99f * cur_ms) {  // 1% hysteresis against timing noise
                    cur = cand;
                    cur_ms = ms;
                    changed = true;
                }
            }
        }
        if (!changed) break;
    }
    c->tune[mi] = cur;
    out->best = cur;
    out->best_ms = cur_ms;
    return VRT_OK;
}

// One frame: voxelize, then cull and trace every pass.
vrt_status grid_frame(vrt_ctx *c, const vrt_lines *L, const vrt_grid *g, const vrt_view *views,
                      const vrt_camera *cams, const vrt_image *imgs, int n_passes, void *stream) {
    vrt_status s = vrt_voxelize(c, L, g, stream);
    for (int i = 0; s == VRT_OK && i < n_passes; ++i) {
        s = vrt_cull(c, &views[i], stream);
        if (s == VRT_OK) s = vrt_trace(c, &cams[i], &imgs[i], stream);
    }
    return s;
}

vrt_status grid_search(vrt_ctx *c, const vrt_lines *L, const vrt_grid *grids, int n, const vrt_view *views,
                       const vrt_camera *cams, const vrt_image *imgs, int n_passes, int reps, int warmup,
                       hipEvent_t e0, hipEvent_t e1, int32_t *best, float *ms, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    float best_ms = INFINITY;
    vrt_status unfit = VRT_ERR_CAPACITY;  // returned when no candidate fits
    *best = -1;
    for (int i = 0; i < n; ++i) {
        ms[i] = INFINITY;
        vrt_status s = grid_frame(c, L, &grids[i], views, cams, imgs, n_passes, stream);
        if (s != VRT_OK) return s;
        vrt_frame_info info;
        s = vrt_frame_status(c, &info);
        if (s != VRT_OK) return s;
        if (info.device_status != VRT_OK) {  // does not fit the context's capacities
            unfit = info.device_status;
            continue;
        }
        for (int k = 0; k < warmup; ++k) {
            s = grid_frame(c, L, &grids[i], views, cams, imgs, n_passes, stream);
            if (s != VRT_OK) return s;
        }
        VRT_HIP(hipEventRecord(e0, st));
        for (int k = 0; k < reps; ++k) {
            s = grid_frame(c, L, &grids[i], views, cams, imgs, n_passes, stream);
            if (s != VRT_OK) return s;
        }
        VRT_HIP(hipEventRecord(e1, st));
        VRT_HIP(hipEventSynchronize(e1));
        float total = 0.0f;
        VRT_HIP(hipEventElapsedTime(&total, e0, e1));
        s = vrt_frame_status(c, &info);
        if (s != VRT_OK) return s;
        if (info.device_status != VRT_OK) {
            unfit = info.device_status;
            continue;
        }
        ms[i] = total / (float)reps;
        if (ms[i] < best_ms) {
            best_ms = ms[i];
            *best = i;
        }
    }
    return *best >= 0 ? VRT_OK : unfit;
}

}  // namespace

extern "C" {

vrt_status vrt_autotune_grid(vrt_ctx *c, const vrt_lines *lines, const vrt_grid *grids, int32_t n_grids,
                             const vrt_view *views, const vrt_camera *cams, const vrt_image *imgs, int32_t n_passes,
                             int32_t reps, int32_t warmup, int32_t *best, float *ms, void *stream) {
    if (!c || !lines || !grids || n_grids < 1 || !views || !cams || !imgs || n_passes < 1 || reps < 1 ||
        warmup < 0 || !best || !ms)
        return VRT_ERR_INVALID_ARG;
    VRT_HIP(hipSetDevice(c->desc.device));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    VRT_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he);
    }
    const bool prof = c->prof.enabled;
    c->prof.enabled = false;
    const vrt_status s =
        grid_search(c, lines, grids, n_grids, views, cams, imgs, n_passes, reps, warmup, e0, e1, best, ms, stream);
    c->prof.enabled = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return s;
}


vrt_status vrt_set_tune(vrt_ctx *c, int32_t mode, const vrt_tune *t) {
    if (!c || !t || (mode != VRT_TRACE_OPAQUE && mode != VRT_TRACE_TRANSPARENT) || !tune_valid(*t))
        return VRT_ERR_INVALID_ARG;
    c->tune[mode == VRT_TRACE_OPAQUE ? 0 : 1] = *t;
    return VRT_OK;
}

vrt_status vrt_get_tune(vrt_ctx *c, int32_t mode, vrt_tune *t) {
    if (!c || !t || (mode != VRT_TRACE_OPAQUE && mode != VRT_TRACE_TRANSPARENT)) return VRT_ERR_INVALID_ARG;
    *t = c->tune[mode == VRT_TRACE_OPAQUE ? 0 : 1];
    return VRT_OK;
}

vrt_status vrt_autotune(vrt_ctx *c, const vrt_tune_space *sp, vrt_tune_result *out, void *stream) {
    if (!c || !sp || !out || !sp->cam || !sp->image || !sp->image->rgba) return VRT_ERR_INVALID_ARG;
    if (sp->reps < 1 || sp->warmup < 0 || sp->sweeps < 1) return VRT_ERR_INVALID_ARG;
    if (!c->culled) return VRT_ERR_NOT_BUILT;
    TraceParams p;
    vrt_status s = camera_params(c, sp->cam, p);
    if (s != VRT_OK) return s;
    VRT_HIP(hipSetDevice(c->desc.device));
    std::memset(out, 0, sizeof(*out));
    const int mi = p.mode == VRT_TRACE_OPAQUE ? 0 : 1;
    const std::string key = tune_key(c, p, sp->key);
    std::map<std::string, TuneEntry> cache;
    if (sp->cache_path) {
        cache = tune_load(sp->cache_path);
        auto it = cache.find(key);
        if (it != cache.end()) {
            c->tune[mi] = it->second.t;
            out->best = it->second.t;
            out->best_ms = it->second.ms;
            out->start_ms = it->second.ms;
            out->from_cache = 1;
            return VRT_OK;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    VRT_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he);
    }
    const bool prof = c->prof.enabled;  // tuning launches are not profiled
    c->prof.enabled = false;
    const vrt_tune start = c->tune[mi];
    s = search(c, p, sp, st, e0, e1, out);
    c->prof.enabled = prof;
    if (s != VRT_OK) c->tune[mi] = start;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != VRT_OK) return s;
    if (sp->cache_path) {
        cache[key] = TuneEntry{out->best, out->best_ms};
        tune_store(sp->cache_path, cache);
    }
    return VRT_OK;
}

}  // extern "C"
