// HIP kernel of libteuk for gfx950 (MI355X): the watchdog's scan of the
// state (teuk_set_watchdog), kept apart from the step kernels.
#include "teuk_internal.h"

namespace teuk {

// Watchdog scan of one state field: a value whose magnitude is not below
// lim (lim = +Inf: non-finite values only; NaN fails every comparison) marks
// the state.  The first scan that finds one keeps tag + 1 in *found (the
// caller's label of the scan: its step, and for a batch the instance): every
// lane that writes in one launch writes the same value, and later launches,
// ordered on the stream, see it and leave it.
template <typename R>
__global__ void watch_kernel(const R* __restrict__ x, int64_t n, R lim, int64_t tag,
                             unsigned long long* found) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (; i < n; i += stride) bad |= !(fabs(x[i]) < lim);
    if (bad && *found == 0ull) *found = (unsigned long long)(tag + 1);
}
void launch_watch_fp64(const double* x, int64_t n, double lim, int64_t tag, unsigned long long* found,
                       hipStream_t s) {
    hipLaunchKernelGGL(watch_kernel<double>, dim3(1024), dim3(256), 0, s, x, n, lim, tag, found);
}
void launch_watch_fp32(const float* x, int64_t n, float lim, int64_t tag, unsigned long long* found,
                       hipStream_t s) {
    hipLaunchKernelGGL(watch_kernel<float>, dim3(1024), dim3(256), 0, s, x, n, lim, tag, found);
}

}  // namespace teuk
