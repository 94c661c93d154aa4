// The reverse sweep of teuk_adjoint for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc): its workspace -- the adjoint's ping-pong partner pair,
// the source-gradient partial sums and the result words -- lives in one
// file-scope device array of fixed size instead of a caller's buffer.
//
// Each GPU that runs this entry point holds its own copy of the array until
// the process ends.  Host code never uses the array's name as an address:
// the device address of each GPU's copy is looked up once, with that GPU
// current, and kept per device.  Every call on one GPU shares that copy, so
// calls that overlap on one GPU (two streams, two threads) race; the sweep
// itself writes every word it reads before reading it (the partner pair is
// written by the first reverse step, the partial sums are zero-filled by a
// kernel), so what an earlier call left behind does not matter.
#include <cstdio>
#include <mutex>

#include "teuk_internal.h"

namespace {

// 40 MiB: the reverse sweep of a 4096 x 256 grid needs 35.4 MB.
constexpr int64_t kScratchBytes = int64_t(40) << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `dev`'s copy of the array (looked up on first use, with
// that device current).
int scratch_address(teuk_ctx* c, int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return teuk::ctx_fail(c, TEUK_ENOTSUP, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return teuk::ctx_fail(c, TEUK_EDEVICE, "hipGetDevice failed");
        if (cur != dev && hipSetDevice(dev) != hipSuccess)
            return teuk::ctx_fail(c, TEUK_EDEVICE, "hipSetDevice to the context's device failed");
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || p == nullptr) {
            char msg[256];
            std::snprintf(msg, sizeof(msg), "hipGetSymbolAddress of the scratch array: %s", hipGetErrorString(e));
            return teuk::ctx_fail(c, TEUK_EDEVICE, msg);
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TEUK_OK;
}

}  // namespace

extern "C" int64_t teuk_adjoint_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" int teuk_adjoint_noalloc(teuk_ctx* c, double rstar_obs, const void* dL_dwave, int64_t n_steps,
                                    double t_start, void* dL_dphi0, void* dL_dpi0, double* dL_dr0,
                                    double* dL_damp) {
    if (!c) return TEUK_EINVAL;
    const int64_t need = teuk_adjoint_workspace_bytes(c);
    if (need < 0) return teuk::ctx_fail(c, (int)need, "the reverse sweep is FP64 only");
    if (need > kScratchBytes) {
        char msg[256];
        std::snprintf(msg, sizeof(msg),
                      "the reverse sweep of this grid needs %lld B of workspace; the fixed scratch array holds "
                      "%lld B (use teuk_adjoint with a workspace)",
                      (long long)need, (long long)kScratchBytes);
        return teuk::ctx_fail(c, TEUK_EINVAL, msg);
    }
    void* ws = nullptr;
    const int rc = scratch_address(c, teuk::ctx_device(c), &ws);
    if (rc != TEUK_OK) return rc;
    return teuk_adjoint(c, rstar_obs, dL_dwave, n_steps, t_start, ws, kScratchBytes, dL_dphi0, dL_dpi0, dL_dr0,
                        dL_damp);
}
