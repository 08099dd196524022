// vrt_batch.hip -- batched form: many line sets, each with its own grid, view
// and camera, voxelized, culled, listed and traced in one persistent launch.
//
// The launch is cooperative (every block resident) and walks the frame's
// stages as phases separated by grid barriers.  Inside a phase every (set,
// stage) pair contributes a number of virtual blocks -- the grid the plain
// launch of that stage would use, counted from the device-side sizes the
// previous phases produced -- and the resident blocks take them from a ticket
// counter, the sets in decreasing size order so the largest start first.
// Each virtual block runs the same kernel body as the plain launch.  The
// same phases also run as one launch each (staged form), or the view-
// independent build (up to the erosion) in one cooperative launch and every
// later phase as a launch of its own (split form).
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "vrt_internal.h"

namespace vrt {
namespace {

constexpr int kBatchThreads = 512;
constexpr int kMaxBatch = 1024;
constexpr int kParts = 3;  // stages sharing one phase
// Work per virtual block of the per-brick phases (their bodies loop over
// slots with the virtual block's stride): fewer tickets and barriers.
constexpr unsigned kBricksPerVB = 8;  // occupied bricks
constexpr unsigned kItemsPerVB = 4;   // binned (brick, chunk) items or candidate bricks
enum : int {
    P_CLEAR, P_INGEST, P_BIN_COUNT, P_BIN_ALLOC, P_BIN_FILL, P_ACCUM, P_LONG, P_COMPACT, P_OCC, P_ERODE, P_WALK,
    P_CBRICK, P_SCAN, P_OFFSETS, P_SCATTER, P_SCATTER_LONG, P_MARCH, P_RAYWALK, P_SHADE8, P_SHADE16, P_SHADE32,
    P_RESUME, kPhases
};
// The shade phase is split by the sets' group size, so that each staged
// kernel holds the tracer body of one group size only (and keeps its
// register budget).
__host__ __device__ constexpr int shade_phase_group(int ph) { return ph == P_SHADE8 ? 8 : (ph == P_SHADE16 ? 16 : 32); }

struct SetDesc {
    Arenas a;
    VoxPlan vp;
    CullPlan cp;
    TraceArgs ta;
    int64_t capacity;
    int n_levels;
    Level levels[kMaxLevels];
    int64_t n_hi;  // elements of the levels >= 4
    unsigned march_blocks;
    int fp16;
    int shade_group;  // lanes per ray in the shade phase: the set's tuned value (8, 16 or 32)
};

__device__ __forceinline__ unsigned cdiv(uint64_t n, unsigned d) { return (unsigned)((n + d - 1) / d); }

// Virtual blocks of stage `part` of phase `ph` for one set.
__device__ unsigned part_blocks(int ph, int part, const SetDesc &d) {
    const DevStatus *st = d.a.status;
    const unsigned T = kBatchThreads;
    switch (ph) {
    case P_CLEAR:
        return part == 0 ? cdiv(st->n_bricks, kBricksPerVB)
                         : (part == 1 ? cdiv(reset_items(d.vp.nb, d.vp.nw, d.vp.nf), T) : 0u);
    case P_INGEST: return part == 0 ? cdiv(d.vp.nv, T) : 0u;
    case P_BIN_COUNT: return part == 0 ? (d.fp16 ? cdiv(d.vp.nv, T) : 0u) : (part == 1 ? cdiv(d.vp.nv, T) : 0u);
    case P_BIN_ALLOC: return part == 0 ? cdiv(st->n_cand, T) : 0u;
    case P_BIN_FILL: return part == 0 ? cdiv(d.vp.nv, T) : 0u;
    case P_ACCUM: return part == 0 ? cdiv(st->n_items, kItemsPerVB) : 0u;
    case P_LONG: return part == 0 ? cdiv(st->n_long, T) : 0u;
    case P_COMPACT: return part == 0 ? 1u : 0u;
    case P_OCC: return part == 0 ? cdiv(st->n_bricks, kBricksPerVB) : 0u;
    case P_ERODE:
        if (part == 0) return cdiv(st->n_bricks, kBricksPerVB);
        if (part == 1) return d.n_levels > 4 ? mip_tree_regions(d.levels) : 0u;
        return cdiv(d.cp.nb > d.n_hi ? d.cp.nb : d.n_hi, T);
    case P_WALK: return part == 0 ? (d.cp.limit >= 0 ? cdiv(st->n_occ, T) : 0u) : (part == 1 && d.n_levels > 8 ? 1u : 0u);
    case P_CBRICK: return part == 0 ? cdiv(st->n_bricks, kBricksPerVB) : 0u;
    case P_SCAN: return part == 0 ? 1u : 0u;
    case P_OFFSETS: return part == 0 ? cdiv(st->n_bricks, kBricksPerVB) : 0u;
    case P_SCATTER: return part == 0 ? cdiv(st->n_cand, kItemsPerVB) : (part == 1 ? cdiv(d.cp.nb, T) : 0u);
    case P_SCATTER_LONG: return part == 0 ? cdiv(st->n_long, T) : (part == 1 ? 1u : 0u);
    case P_MARCH: return part == 0 ? d.march_blocks : 0u;
    case P_RAYWALK: return part == 0 ? cdiv(st->n_queue, T) : 0u;
    case P_SHADE8:
    case P_SHADE16:
    case P_SHADE32:  // one-wave units, in the phase of the set's group size
        return part == 0 && d.shade_group == shade_phase_group(ph) ? cdiv(st->n_queue, 64u / (unsigned)d.shade_group)
                                                                    : 0u;
    case P_RESUME: return part == 0 ? cdiv(st->n_cont, 64u / 16u) : 0u;
    default: return 0u;
    }
}



// Virtual block vb of nvb of stage `part` of phase `ph` for set d.
__device__ __forceinline__ void run_part(int ph, int part, const SetDesc &d, unsigned vb, unsigned nvb) {
    const Arenas &A = d.a;
    switch (ph) {
    case P_CLEAR:
        if (part == 0) b_clear_prev(A.words, A.brick_list, A.status, vb, nvb);
        else b_reset(A.occ3, A.bin_count, A.brick_bits, d.vp.nb, d.vp.nw, A.super_blk, d.vp.nf, A.status, vb, nvb);
        break;
    case P_INGEST: b_ingest(d.vp.ia, A.vrec, A.status, vb, nvb); break;
    case P_BIN_COUNT:
        if (part == 0) b_pack16(A.vrec, d.vp.nv, A.srec16, vb, nvb);
        else b_bin_count(d.vp.ba, A.status, vb, nvb);
        break;
    case P_BIN_ALLOC: b_bin_alloc(d.vp.ba, A.status, vb, nvb); break;
    case P_BIN_FILL: b_bin_fill(d.vp.ba, A.status, vb, nvb); break;
    case P_ACCUM: b_brick_accum<-1>(d.vp.aa, A.status, vb, nvb); break;
    case P_LONG: b_vox_long(d.vp.ca, A.long_ids, A.status, vb, nvb); break;
    case P_COMPACT: b_brick_compact(A.brick_flag, d.vp.nb, A.brick_list, A.brick_slot, A.status, 0u, 1u); break;
    case P_OCC: b_occ_brick(A.words, A.brick_list, A.status, A.occ0, A.occ1, A.occ2, A.occ3, A.occ_list, vb, nvb); break;
    case P_ERODE:
        if (part == 0)
            b_erode(d.vp.g, A.occ0, A.brick_list, A.brick_slot, A.status, A.blk, A.blk_bits, A.brick_bits, A.super_blk,
                    vb, nvb);
        else if (part == 1) b_mip_avg_tree(A.occ3, d.vp.g.nb, A.occ_hi, d.levels, d.n_levels, vb);
        else b_cull_reset(A.vis3, d.cp.nb, A.vis_hi, d.n_hi, A.status, vb, nvb);
        break;
    case P_WALK:
        if (part == 0) b_cull_walk<false>(d.cp.ca, d.cp.cells, A.occ_list, A.status, A.vis0, vb, nvb);
        else b_mip_avg_top(A.occ_hi, d.levels, d.n_levels);
        break;
    case P_CBRICK:
        b_cull_brick(d.cp.limit, d.cp.g, A.words, A.brick_list, A.status, A.vis0, A.vis1, A.vis2, A.vis3, A.vis_hi,
                     d.levels, d.n_levels, A.brick_total, vb, nvb);
        break;
    case P_SCAN: b_scan_bricks(A.brick_total, A.brick_base, A.status, d.capacity, A.vis_hi, d.levels, d.n_levels, 0u, 1u); break;
    case P_OFFSETS: b_list_offsets(A.words, A.vis0, A.brick_list, A.brick_base, A.status, A.cursor, A.cell, A.lmask, A.lmask2, vb, nvb); break;
    case P_SCATTER:  // the lists, and the trace's per-brick skip bytes (the culling levels are final)
        if (part == 0) b_scatter_brick<-1>(d.cp.sb, A.status, vb, nvb);
        else b_brick_skip(d.ta, vb, nvb);
        break;
    case P_SCATTER_LONG:
        if (part == 0) b_scatter_long(d.cp.sb, A.status, vb, nvb);
        else b_trace_begin(A.status, 0u, 1u);
        break;
    case P_MARCH: b_trace_march<false>(d.ta, vb, nvb); break;
    case P_RAYWALK: b_trace_walk(d.ta, vb, nvb); break;
    case P_SHADE8:  // one wave per unit; the set's tuned group size, default batch and keys
        if (d.fp16) b_trace_shade<false, VRT_FORM_FP16, ShadeCfg<8, 2, 4>, true>(d.ta, vb, nvb, 64u, threadIdx.x & 63u);
        else b_trace_shade<false, VRT_FORM_PLAIN, ShadeCfg<8, 2, 4>, true>(d.ta, vb, nvb, 64u, threadIdx.x & 63u);
        break;
    case P_SHADE16:
        if (d.fp16) b_trace_shade<false, VRT_FORM_FP16, ShadeCfg<16, 2, 4>, true>(d.ta, vb, nvb, 64u, threadIdx.x & 63u);
        else b_trace_shade<false, VRT_FORM_PLAIN, ShadeCfg<16, 2, 4>, true>(d.ta, vb, nvb, 64u, threadIdx.x & 63u);
        break;
    case P_SHADE32:
        if (d.fp16) b_trace_shade<false, VRT_FORM_FP16, ShadeCfg<32, 2, 4>, true>(d.ta, vb, nvb, 64u, threadIdx.x & 63u);
        else b_trace_shade<false, VRT_FORM_PLAIN, ShadeCfg<32, 2, 4>, true>(d.ta, vb, nvb, 64u, threadIdx.x & 63u);
        break;
    case P_RESUME:  // rays past the walk limit, default group size
        if (d.fp16) b_trace_resume<VRT_FORM_FP16>(d.ta, vb, nvb, 64u, threadIdx.x & 63u);
        else b_trace_resume<VRT_FORM_PLAIN>(d.ta, vb, nvb, 64u, threadIdx.x & 63u);
        break;
    default: break;
    }
}

// Runs ticket t of a phase: the (set, stage) whose range of pre[] holds it.
// The ticket is uniform over the wave, and so are the set index and the
// virtual block derived from it (made explicit with readfirstlane), so the
// set's arguments are read with scalar loads into scalar registers, as a
// kernel's own arguments are.
__device__ __forceinline__ void run_ticket(int ph, const SetDesc *__restrict__ sets, int nk, const unsigned *pre,
                                           unsigned t) {
    int lo = 0, hi = nk - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const unsigned b0 = (unsigned)__builtin_amdgcn_readfirstlane((int)pre[lo]);
    const unsigned b1 = (unsigned)__builtin_amdgcn_readfirstlane((int)pre[lo + 1]);
    run_part(ph, lo % kParts, sets[lo / kParts], t - b0, b1 - b0);
}

// One phase of the batch: the resident blocks take the phase's virtual blocks
// of every set from the ticket counter tickets[ph]; block 0 clears the next
// phase's counter (it is not read before this phase has ended), so the
// counters are zero at every launch.
__device__ __forceinline__ void batch_phase(int ph, const SetDesc *__restrict__ sets, int nsets,
                                            unsigned *__restrict__ tickets, unsigned *pre, unsigned &ticket) {
    const int nk = nsets * kParts;
    if (blockIdx.x == 0 && threadIdx.x == 0) tickets[(ph + 1) % kPhases] = 0u;
    for (int k = threadIdx.x; k < nk; k += blockDim.x) pre[k + 1] = part_blocks(ph, k % kParts, sets[k / kParts]);
    __syncthreads();
    if (threadIdx.x == 0) {
        pre[0] = 0u;
        for (int k = 1; k <= nk; ++k) pre[k] += pre[k - 1];
    }
    __syncthreads();
    const unsigned total = pre[nk];
    if (ph >= P_SHADE8) {  // the waves take one-wave units on their own: a long ray holds only its wave
        const unsigned lane = threadIdx.x & 63u;
        for (;;) {
            unsigned t = 0;
            if (lane == 0) t = atomicAdd(&tickets[ph], 1u);
            t = (unsigned)__builtin_amdgcn_readfirstlane((int)t);  // wave-uniform: scalar from here on
            if (t >= total) break;
            run_ticket(ph, sets, nk, pre, t);
        }
        __syncthreads();  // pre[] is rewritten by the next phase
        return;
    }
    for (;;) {
        if (threadIdx.x == 0) ticket = atomicAdd(&tickets[ph], 1u);
        __syncthreads();
        const unsigned t = (unsigned)__builtin_amdgcn_readfirstlane((int)ticket);
        __syncthreads();
        if (t >= total) break;
        run_ticket(ph, sets, nk, pre, t);
        __syncthreads();
    }
}

// The persistent batch kernel: phases [0, kEnd), separated by grid barriers
// (kEnd = kPhases: every phase).  As one function holding every phase it
// would take about 240 registers (one 512-thread block per compute unit,
// two waves per SIMD); it is capped at four waves per SIMD, which costs
// 416 bytes of spills per lane and is still 1.27x faster on the
// 64-set batch.  kEnd = P_WALK holds the build phases only (the cooperative
// launch of the split form, 240 bytes of spills).  Its occupancy is set by
// its heaviest phase, so every phase runs with fewer resident waves than its
// own phase kernel: on the 64-set batch each phase moved from the
// cooperative launch to a launch of its own saves 0.15-0.3 ms, the culling
// phases most.
template <int kEnd>
__global__ void __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_batch(const SetDesc *__restrict__ sets, int nsets, unsigned *__restrict__ tickets) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    __shared__ unsigned pre[kMaxBatch * kParts + 1];
    __shared__ unsigned ticket;
    for (int ph = 0; ph < kEnd; ++ph) {
        batch_phase(ph, sets, nsets, tickets, pre, ticket);
        grid.sync();
    }
}

// The staged form: one launch per phase (kernel boundaries instead of grid
// barriers), each compiled for its own phase only, so it keeps the register
// budget of that phase's bodies.
template <int kPh>
__global__ void __launch_bounds__(kBatchThreads) k_batch_phase(const SetDesc *__restrict__ sets, int nsets,
                                                               unsigned *__restrict__ tickets) {
    __shared__ unsigned pre[kMaxBatch * kParts + 1];
    __shared__ unsigned ticket;
    batch_phase(kPh, sets, nsets, tickets, pre, ticket);
}

// The staged shade phases, at the tracer kernel's four waves per SIMD.
template <int kPh>
__global__ void __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_batch_shade_phase(const SetDesc *__restrict__ sets, int nsets, unsigned *__restrict__ tickets) {
    __shared__ unsigned pre[kMaxBatch * kParts + 1];
    __shared__ unsigned ticket;
    batch_phase(kPh, sets, nsets, tickets, pre, ticket);
}

// Host handle of the staged kernel of phase ph.
const void *phase_kernel(int ph) {
    switch (ph) {
    case P_CLEAR: return (const void *)k_batch_phase<P_CLEAR>;
    case P_INGEST: return (const void *)k_batch_phase<P_INGEST>;
    case P_BIN_COUNT: return (const void *)k_batch_phase<P_BIN_COUNT>;
    case P_BIN_ALLOC: return (const void *)k_batch_phase<P_BIN_ALLOC>;
    case P_BIN_FILL: return (const void *)k_batch_phase<P_BIN_FILL>;
    case P_ACCUM: return (const void *)k_batch_phase<P_ACCUM>;
    case P_LONG: return (const void *)k_batch_phase<P_LONG>;
    case P_COMPACT: return (const void *)k_batch_phase<P_COMPACT>;
    case P_OCC: return (const void *)k_batch_phase<P_OCC>;
    case P_ERODE: return (const void *)k_batch_phase<P_ERODE>;
    case P_WALK: return (const void *)k_batch_phase<P_WALK>;
    case P_CBRICK: return (const void *)k_batch_phase<P_CBRICK>;
    case P_SCAN: return (const void *)k_batch_phase<P_SCAN>;
    case P_OFFSETS: return (const void *)k_batch_phase<P_OFFSETS>;
    case P_SCATTER: return (const void *)k_batch_phase<P_SCATTER>;
    case P_SCATTER_LONG: return (const void *)k_batch_phase<P_SCATTER_LONG>;
    case P_MARCH: return (const void *)k_batch_phase<P_MARCH>;
    case P_RAYWALK: return (const void *)k_batch_phase<P_RAYWALK>;
    case P_SHADE8: return (const void *)k_batch_shade_phase<P_SHADE8>;
    case P_SHADE16: return (const void *)k_batch_shade_phase<P_SHADE16>;
    case P_SHADE32: return (const void *)k_batch_shade_phase<P_SHADE32>;
    default: return (const void *)k_batch_shade_phase<P_RESUME>;
    }
}

}  // namespace
}  // namespace vrt

struct vrt_batch {
    int n = 0;
    int device = 0;
    std::vector<vrt_ctx *> ctx;
    vrt::SetDesc *d_sets = nullptr;
    vrt::SetDesc *h_sets = nullptr;  // pinned staging
    unsigned *d_tickets = nullptr;
    hipEvent_t copied = nullptr;
    bool copy_pending = false;
    unsigned grid = 0;                     // resident blocks of the persistent kernel
    unsigned grid_split = 0;               // resident blocks of the split form's build kernel
    unsigned phase_grid[vrt::kPhases] = {}; // resident blocks of each staged phase kernel
};

extern "C" {

vrt_status vrt_batch_create(const vrt_desc *descs, int32_t n, vrt_batch **out) {
    using namespace vrt;
    if (!descs || !out || n < 1 || n > kMaxBatch) return VRT_ERR_INVALID_ARG;
    *out = nullptr;
    for (int i = 1; i < n; ++i)
        if (descs[i].device != descs[0].device) return VRT_ERR_INVALID_ARG;
    VRT_HIP(hipSetDevice(descs[0].device));
    int coop = 0;
    VRT_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, descs[0].device));
    if (!coop) return VRT_ERR_INVALID_ARG;
    vrt_batch *b = new (std::nothrow) vrt_batch();
    if (!b) return VRT_ERR_INVALID_ARG;
    b->n = n;
    b->device = descs[0].device;
    vrt_status st = VRT_OK;
    for (int i = 0; i < n && st == VRT_OK; ++i) {
        vrt_ctx *c = nullptr;
        st = vrt_create(&descs[i], &c);
        if (st == VRT_OK) b->ctx.push_back(c);
    }
    hipError_t e = hipSuccess;
    if (st == VRT_OK) e = hipMalloc((void **)&b->d_sets, sizeof(SetDesc) * n);
    if (st == VRT_OK && e == hipSuccess) e = hipHostMalloc((void **)&b->h_sets, sizeof(SetDesc) * n);
    if (st == VRT_OK && e == hipSuccess) e = hipMalloc((void **)&b->d_tickets, sizeof(unsigned) * kPhases);
    if (st == VRT_OK && e == hipSuccess) e = hipMemset(b->d_tickets, 0, sizeof(unsigned) * kPhases);
    if (st == VRT_OK && e == hipSuccess) e = hipEventCreateWithFlags(&b->copied, hipEventDisableTiming);
    int per_cu = 0, per_cu_split = 0, ncu = 0;
    if (st == VRT_OK && e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<kPhases>, kBatchThreads, 0);
    if (st == VRT_OK && e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_split, k_batch<P_WALK>, kBatchThreads, 0);
    if (st == VRT_OK && e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device);
    for (int ph = 0; ph < kPhases && st == VRT_OK && e == hipSuccess; ++ph) {
        int pc = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, phase_kernel(ph), kBatchThreads, 0);
        b->phase_grid[ph] = (unsigned)((pc > 0 ? pc : 1) * ncu);
    }
    if (st == VRT_OK && e == hipSuccess) e = hipDeviceSynchronize();
    if (st == VRT_OK && e != hipSuccess) st = hip_fail(e);
    if (st == VRT_OK && (per_cu < 1 || per_cu_split < 1)) st = VRT_ERR_INVALID_ARG;
    b->grid = (unsigned)(per_cu * ncu);
    b->grid_split = (unsigned)(per_cu_split * ncu);
    if (st != VRT_OK) {
        vrt_batch_destroy(b);
        return st;
    }
    *out = b;
    return VRT_OK;
}

vrt_status vrt_batch_run(vrt_batch *b, const vrt_batch_item *items, int32_t n, int32_t mode, void *stream) {
    using namespace vrt;
    if (!b || !items || n != b->n) return VRT_ERR_INVALID_ARG;
    if (mode != VRT_BATCH_PERSISTENT && mode != VRT_BATCH_SEQUENTIAL && mode != VRT_BATCH_STAGED &&
        mode != VRT_BATCH_SPLIT)
        return VRT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    VRT_HIP(hipSetDevice(b->device));
    if (mode == VRT_BATCH_SEQUENTIAL) {
        for (int i = 0; i < n; ++i) {
            vrt_status s = vrt_voxelize(b->ctx[i], &items[i].lines, &items[i].grid, stream);
            if (s == VRT_OK) s = vrt_cull(b->ctx[i], &items[i].view, stream);
            if (s == VRT_OK) s = vrt_trace(b->ctx[i], &items[i].cam, &items[i].image, stream);
            if (s != VRT_OK) return s;
        }
        return VRT_OK;
    }
    // validate every set and compute its arguments exactly as the plain calls do
    std::vector<float> sq(n);
    std::vector<int64_t> E(3 * n), lim(n);
    std::vector<TraceParams> tp(n);
    for (int i = 0; i < n; ++i) {
        vrt_ctx *c = b->ctx[i];
        vrt_status s = prepare_voxelize(c, &items[i].lines, &items[i].grid, &sq[i]);
        if (s != VRT_OK) return s;
        c->voxelized = true;
        s = prepare_cull(c, &items[i].view, &E[3 * i], &lim[i]);
        if (s != VRT_OK) return s;
        c->culled = true;
        c->shaded = false;  // the batched forms trace unshaded
        if (!items[i].image.rgba) return VRT_ERR_INVALID_ARG;
        s = camera_params(c, &items[i].cam, tp[i]);
        if (s != VRT_OK) return s;
    }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return items[x].lines.n_vertices > items[y].lines.n_vertices; });
    if (b->copy_pending) VRT_HIP(hipEventSynchronize(b->copied));  // the staging buffer is free again
    for (int k = 0; k < n; ++k) {
        const int i = order[k];
        vrt_ctx *c = b->ctx[i];
        SetDesc &d = b->h_sets[k];
        d.a = c->a;
        d.vp = make_vox_plan(c, &items[i].lines, sq[i]);
        d.cp = make_cull_plan(c, &E[3 * i], lim[i]);
        d.ta = trace_args(c, tp[i], &items[i].image);
        d.capacity = c->desc.max_fragments;
        d.n_levels = c->n_levels;
        for (int L = 0; L < kMaxLevels; ++L) d.levels[L] = c->levels[L];
        d.n_hi = hi_used(c);
        d.march_blocks = (unsigned)(((tp[i].W + 15) / 16) *
                                    ((tp[i].H + march_tile_rows(kBatchThreads) - 1) / march_tile_rows(kBatchThreads)));
        d.fp16 = c->desc.form == VRT_FORM_FP16;
        d.shade_group = c->tune[tp[i].mode == VRT_TRACE_OPAQUE ? 0 : 1].shade_group;
        c->last_stream = st;
    }
    VRT_HIP(hipMemcpyAsync(b->d_sets, b->h_sets, sizeof(SetDesc) * n, hipMemcpyHostToDevice, st));
    VRT_HIP(hipEventRecord(b->copied, st));
    b->copy_pending = true;
    const SetDesc *sets = b->d_sets;
    int nsets = n;
    unsigned *tickets = b->d_tickets;
    void *args[] = {(void *)&sets, (void *)&nsets, (void *)&tickets};
    if (mode == VRT_BATCH_STAGED) {
        for (int ph = 0; ph < kPhases; ++ph)
            VRT_HIP(hipLaunchKernel(phase_kernel(ph), dim3(b->phase_grid[ph]), dim3(kBatchThreads), args, 0, st));
        return VRT_OK;
    }
    if (mode == VRT_BATCH_SPLIT) {  // the build phases in one cooperative launch, then one launch per phase
        VRT_HIP(hipLaunchCooperativeKernel((const void *)k_batch<P_WALK>, dim3(b->grid_split), dim3(kBatchThreads),
                                           args, 0, st));
        for (int ph = P_WALK; ph < kPhases; ++ph)
            VRT_HIP(hipLaunchKernel(phase_kernel(ph), dim3(b->phase_grid[ph]), dim3(kBatchThreads), args, 0, st));
        return VRT_OK;
    }
    VRT_HIP(hipLaunchCooperativeKernel((const void *)k_batch<kPhases>, dim3(b->grid), dim3(kBatchThreads), args, 0,
                                       st));
    return VRT_OK;
}

vrt_status vrt_batch_context(vrt_batch *b, int32_t i, vrt_ctx **out) {
    if (!b || !out || i < 0 || i >= b->n) return VRT_ERR_INVALID_ARG;
    *out = b->ctx[i];
    return VRT_OK;
}

vrt_status vrt_batch_destroy(vrt_batch *b) {
    if (!b) return VRT_ERR_INVALID_ARG;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    for (vrt_ctx *c : b->ctx) vrt_destroy(c);
    if (b->d_sets) (void)hipFree(b->d_sets);
    if (b->h_sets) (void)hipHostFree(b->h_sets);
    if (b->d_tickets) (void)hipFree(b->d_tickets);
    if (b->copied) (void)hipEventDestroy(b->copied);
    delete b;
    return VRT_OK;
}

}  // extern "C"
