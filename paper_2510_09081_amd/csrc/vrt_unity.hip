// vrt_unity.hip -- the library as one translation unit, so that the batched
// persistent kernel can run the same device bodies as the per-stage kernels.
#include "vrt_voxelize.hip"
#include "vrt_cull.hip"
#include "vrt_trace.hip"
#include "vrt_shade.hip"
#include "vrt_api.hip"
#include "vrt_tune.hip"
#include "vrt_batch.hip"
#include "vrt_microbench.hip"
