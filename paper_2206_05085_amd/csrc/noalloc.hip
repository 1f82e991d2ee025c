// dvgo_distortion_loss for callers that cannot allocate: the per-chunk checkpoints of the
// backward sweep live in a fixed file-scope device array instead of a caller workspace.
//
// Each GPU holds its own copy of `scratch` at its own address.  Host code never uses the
// array's name as a device address: the address is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept.  The kernel writes every checkpoint
// it reads within the same call (forward sweep first, then the reverse sweep of the same ray),
// so nothing needs clearing between calls.  Calls that overlap on one GPU share the array and
// race.
#include <mutex>

#include "dvgo_internal.h"

using namespace dvgo;

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)1 << 21;  // 2 MiB: 262144 checkpoints of 8 bytes
constexpr int MAX_DEV = 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
void *g_scratch[MAX_DEV];

// The device address of this device's copy of `scratch` (looked up on the first call per device).
int scratch_ptr(void **out) {
    int dev = 0;
    int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= MAX_DEV) return set_error(DVGO_ERR_RANGE, "device index %d beyond %d", dev, MAX_DEV);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (rc) return rc;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return DVGO_OK;
}

}  // namespace

extern "C" int dvgo_distortion_loss_noalloc(int32_t n_rays, const int32_t *ray_offsets, int64_t n_samples,
                                            const float *w, const float *s_mid, const float *s_len, float *loss,
                                            const float *grad_loss, float *grad_w, void *stream) {
    int rc = distortion_check(n_rays, ray_offsets, n_samples, w, s_mid, s_len, loss, grad_loss, grad_w);
    if (rc || n_rays == 0) return rc;
    const size_t need = distortion_scratch_bytes(n_rays, n_samples);
    if (need > SCRATCH_BYTES)
        return set_error(DVGO_ERR_RANGE,
                         "batch needs %zu bytes of checkpoints (n_samples/64 + n_rays + 1 = %zu), more than the "
                         "fixed %zu", need, need / 8, SCRATCH_BYTES);
    void *p = nullptr;
    rc = scratch_ptr(&p);
    if (rc) return rc;
    return launch_distortion(n_rays, ray_offsets, n_samples, w, s_mid, s_len, loss, grad_loss, grad_w, p,
                             (hipStream_t)stream);
}
