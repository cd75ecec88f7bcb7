// Stage 3: key emission (Speedy-Splat Sec. 3.2 "duplicateWithKeys"; the
// "Process" step of Alg. 1).
//
// Gaussian i re-walks its tile spans with the same FP64 function the
// preprocess stage counted with and writes key = tile_id << 32 | bits(depth),
// value = i, at [offsets[i] - counts[i], offsets[i]).
#include "ss_internal.h"

namespace ss {
namespace {

__global__ __launch_bounds__(256) void k_emit(int tx_n, int ty_n, int64_t n, int mode,
                                              uint32_t limit,
                                              const float4* __restrict__ geom,
                                              const float4* __restrict__ conic,
                                              const uint32_t* __restrict__ counts,
                                              const uint32_t* __restrict__ offsets,
                                              uint64_t* __restrict__ keys,
                                              uint32_t* __restrict__ values) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t cnt = counts[i];
    if (cnt == 0u) return;
    const uint32_t end = offsets[i] < limit ? offsets[i] : limit;
    uint32_t pos = end - cnt;
    const float4 g = geom[i], q = conic[i];
    Ellipse e;
    if (!ellipse_setup(g, q, mode, tx_n, ty_n, e)) return;
    const uint64_t dbits = (uint64_t)__float_as_uint(g.z);
    const bool cols = (mode == SS_TILE_ACCUTILE) && (e.y1 - e.y0 > e.x1 - e.x0);
    const uint32_t vi = (uint32_t)i;
    for_each_span(e, mode, tx_n, ty_n, [&](int major, int lo, int hi) {
        for (int k = lo; k <= hi; ++k) {
            const uint32_t tile = cols ? (uint32_t)(k * tx_n + major) : (uint32_t)(major * tx_n + k);
            if (pos < end) {
                keys[pos] = ((uint64_t)tile << 32) | dbits;
                values[pos] = vi;
            }
            ++pos;
        }
    });
}

}  // namespace

hipError_t launch_emit(int tx_n, int ty_n, int64_t n, int mode, const ss_frame& f, uint64_t* keys,
                       uint32_t* values, uint64_t n_pairs, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int block = 256;
    const int64_t grid = (n + block - 1) / block;
    hipLaunchKernelGGL(k_emit, dim3((unsigned)grid), dim3(block), 0, s, tx_n, ty_n, n, mode,
                       (uint32_t)n_pairs,
                       reinterpret_cast<const float4*>(f.geom),
                       reinterpret_cast<const float4*>(f.conic), f.counts, f.offsets, keys,
                       values);
    return hipGetLastError();
}

}  // namespace ss
