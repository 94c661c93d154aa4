// HIP kernel of libteuk for gfx950 (MI355X): a streaming copy that measures
// what HBM delivers to a plain read-and-write kernel (teuk_stream_copy), the
// practical ceiling beside the step kernel's bandwidth, and the kernel of
// known traffic against which hardware byte counters are calibrated.
#include <algorithm>

#include "teuk_internal.h"

namespace teuk {

// Each thread moves UNROLL 16-byte vectors per trip, a block's accesses in
// each trip being contiguous 4 KiB spans; the loads of a trip are issued
// before its stores, so UNROLL x 16 B per lane are in flight.
constexpr int COPY_UNROLL = 4;
constexpr int COPY_THREADS = 256;

__global__ __launch_bounds__(COPY_THREADS) void stream_copy_kernel(const uint4* __restrict__ src,
                                                                   uint4* __restrict__ dst, int64_t n) {
    const int64_t span = (int64_t)COPY_THREADS * COPY_UNROLL;
    const int64_t step = (int64_t)gridDim.x * span;
    for (int64_t base = (int64_t)blockIdx.x * span + threadIdx.x; base < n; base += step) {
        uint4 v[COPY_UNROLL];
#pragma unroll
        for (int u = 0; u < COPY_UNROLL; ++u) {
            const int64_t i = base + (int64_t)u * COPY_THREADS;
            if (i < n) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < COPY_UNROLL; ++u) {
            const int64_t i = base + (int64_t)u * COPY_THREADS;
            if (i < n) dst[i] = v[u];
        }
    }
}

}  // namespace teuk

extern "C" int teuk_stream_copy(const void* src, void* dst, int64_t bytes, void* hip_stream) {
    using namespace teuk;
    if (!src || !dst || bytes < 0 || bytes % 16 != 0) return TEUK_EINVAL;
    if ((uintptr_t)src % 16 != 0 || (uintptr_t)dst % 16 != 0) return TEUK_EINVAL;
    const char* s = (const char*)src;
    const char* d = (const char*)dst;
    if (s < d + bytes && d < s + bytes) return TEUK_EINVAL;   // overlapping buffers
    const int64_t n = bytes / 16;
    if (n == 0) return TEUK_OK;
    const int64_t span = (int64_t)COPY_THREADS * COPY_UNROLL;
    // 8192 blocks (32 per CU) cover the GPU; small copies take fewer
    const int64_t blocks = std::min<int64_t>(8192, (n + span - 1) / span);
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(COPY_THREADS), 0,
                       (hipStream_t)hip_stream, (const uint4*)src, (uint4*)dst, n);
    return hipGetLastError() == hipSuccess ? TEUK_OK : TEUK_EDEVICE;
}
