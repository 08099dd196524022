// vrt_microbench.hip -- memory-system ceilings on the device the frame runs on:
// a streaming copy (the practical HBM bandwidth) and 32-bit device atomics on
// random words and on words confined to 2 KiB regions (the locality of one
// brick's packed count/occupancy words).  Measurement only; no frame state.
#include "vrt_internal.h"

namespace vrt {
namespace {

// splitmix64 finalizer (Steele, Lea and Flood, 2014): a well-mixed 64-bit
// value per operation index.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void __launch_bounds__(256) k_mb_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Operation i adds 1 to word mix(i) mod nwords.
__global__ void __launch_bounds__(256) k_mb_atomic_random(uint32_t *__restrict__ a, int64_t nwords, int64_t ops,
                                                          uint64_t seed) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ops; i += stride)
        atomicAdd(&a[mix64(seed + (uint64_t)i) % (uint64_t)nwords], 1u);
}

// The 64 operations of one wave step fall in one 2 KiB region (512 words)
// chosen from the wave's step index; inside it each lane takes a random word.
__global__ void __launch_bounds__(256) k_mb_atomic_brick(uint32_t *__restrict__ a, int64_t nwords, int64_t ops,
                                                         uint64_t seed) {
    const int64_t nreg = nwords / 512;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ops; i += stride) {
        const uint64_t reg = mix64(seed ^ (uint64_t)(i >> 6)) % (uint64_t)nreg;
        const uint64_t w = mix64(seed + (uint64_t)i) & 511u;
        atomicAdd(&a[reg * 512 + w], 1u);
    }
}

}  // namespace
}  // namespace vrt

extern "C" vrt_status vrt_microbench(int32_t kind, void *buf, int64_t bytes, int64_t ops, float *ms, void *stream) {
    using namespace vrt;
    if (!buf || !ms || bytes < 4096 || bytes % 4096 != 0 || (kind != VRT_MB_COPY && ops < 1) ||
        (kind != VRT_MB_COPY && kind != VRT_MB_ATOMIC_RANDOM && kind != VRT_MB_ATOMIC_BRICK))
        return VRT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) {
        if (kind == VRT_MB_COPY) {
            const int64_t n = bytes / 2 / sizeof(uint4);
            uint4 *p = static_cast<uint4 *>(buf);
            k_mb_copy<<<8192, 256, 0, st>>>(p, p + n, n);
        } else if (kind == VRT_MB_ATOMIC_RANDOM) {
            k_mb_atomic_random<<<8192, 256, 0, st>>>(static_cast<uint32_t *>(buf), bytes / 4, ops, 12345u);
        } else {
            k_mb_atomic_brick<<<8192, 256, 0, st>>>(static_cast<uint32_t *>(buf), bytes / 4, ops, 12345u);
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e);
    return VRT_OK;
}
