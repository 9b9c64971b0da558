// kmvp_gauss_noalloc: the Gaussian kernel product for callers that cannot
// allocate device memory (code under graph capture, tight serving loops).  The
// product's scratch (prepared points, sort buffers, partial sums) lives in a
// fixed static device array, one per device, instead of a caller workspace.
#include <mutex>

#include "solvers.h"

// kmvp_gauss on the given scratch without tuning (api.hip).
int kmvp_gauss_on_scratch(const krr_points *pts, double sigma, double shift, int32_t prec, const void *q, void *y,
                          void *scratch, size_t scratch_bytes, krr_stream_t stream);

namespace {

constexpr size_t kScratchBytes = static_cast<size_t>(128) << 20;  // 128 MiB

// Held by every device the library runs on until the process ends.  Host code
// never uses this name as an address (it is a host-side stand-in): it takes the
// device address from hipGetSymbolAddress, once per device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// The current device's address of `scratch` (looked up on the first call on
// that device, with that device current).
int scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KRR_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return KRR_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return KRR_EHIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return KRR_OK;
}

}  // namespace

extern "C" {

size_t krr_noalloc_scratch_bytes(void) { return kScratchBytes; }

int kmvp_gauss_noalloc(const krr_points *pts, double sigma, double shift, int32_t prec, const void *q, void *y,
                       krr_stream_t stream) {
    if (pts == nullptr) return KRR_EINVAL;
    const size_t need = krr_workspace_size(KRR_WS_KMVP, pts, 1, 1, nullptr);
    if (need == 0) return KRR_EINVAL;
    if (need > kScratchBytes) return KRR_EUNSUPPORTED;
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != KRR_OK) return rc;
    return kmvp_gauss_on_scratch(pts, sigma, shift, prec, q, y, ws, kScratchBytes, stream);
}

}  // extern "C"
