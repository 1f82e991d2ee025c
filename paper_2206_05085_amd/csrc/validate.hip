// Host-side constants of the method and the debug-mode validation of ragged batches.
//
// The activation shift b of sigma = softplus(raw + b) follows from the initial alpha the paper
// fixes (section 5.4: alpha_init at a step of delta_ref voxels): alpha(raw = 0, delta_ref) =
// 1 - (1 + e^b)^(-delta_ref) = alpha_init gives b = ln((1 - alpha_init)^(-1/delta_ref) - 1).
//
// Validation reads the batch on the device: ray_offsets must start at 0, never decrease and end
// at n_samples, and s_mid must not decrease within a ray (Eq. 2 assumes sorted midpoints; ties
// are harmless).  One thread per ray checks its own offsets before it reads any sample, so a
// broken batch is reported without an out-of-bounds access.  The verdict lands in a small
// file-scope device word, read back synchronously.
#include <math.h>
#include <stdlib.h>

#include <mutex>

#include "dvgo_internal.h"

using namespace dvgo;

namespace {

enum { BAD_OFFSETS = 1, BAD_ORDER = 2 };

__device__ int g_verdict;  // addressed from the host only through hipGetSymbolAddress

__global__ void verdict_clear_kernel(int *v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) v[0] = 0;
}

__global__ __launch_bounds__(256) void validate_kernel(int R, int64_t S, const int *__restrict__ offs,
                                                       const float *__restrict__ s_mid, int *verdict) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r > R) return;
    const int64_t a = offs[r];
    int bad = 0;
    if (r == 0 && a != 0) bad |= BAD_OFFSETS;
    if (r == R) {
        if (a != S) bad |= BAD_OFFSETS;
    } else {
        const int64_t b = offs[r + 1];
        if (a < 0 || b < a || b > S) {
            bad |= BAD_OFFSETS;
        } else if (s_mid) {
            for (int64_t k = a + 1; k < b; ++k)
                if (!(s_mid[k] >= s_mid[k - 1])) {  // a NaN midpoint is not ordered either
                    bad |= BAD_ORDER;
                    break;
                }
        }
    }
    if (bad) atomicOr(verdict, bad);
}

constexpr int MAX_DEV = 64;
std::mutex g_mu;          // one validation at a time (they share the device word)
int *g_verdict_ptr[MAX_DEV];
int g_debug = -1;          // -1: not yet read from the environment

int verdict_ptr(int **out) {
    int dev = 0;
    int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= MAX_DEV) return set_error(DVGO_ERR_RANGE, "device index %d beyond %d", dev, MAX_DEV);
    if (!g_verdict_ptr[dev]) {
        void *p = nullptr;
        rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(g_verdict)), "hipGetSymbolAddress(verdict)");
        if (rc) return rc;
        g_verdict_ptr[dev] = static_cast<int *>(p);
    }
    *out = g_verdict_ptr[dev];
    return DVGO_OK;
}

}  // namespace

namespace dvgo {

bool debug_mode() {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_debug < 0) {
        const char *e = getenv("DVGO_DEBUG");
        g_debug = (e && e[0] && e[0] != '0') ? 1 : 0;
    }
    return g_debug != 0;
}

int validate_batch(int32_t n_rays, int64_t n_samples, const int32_t *ray_offsets, const float *s_mid,
                   hipStream_t st) {
    if (n_rays < 0 || n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays or n_samples");
    if (!ray_offsets) return set_error(DVGO_ERR_NULL, "ray_offsets is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    int *v = nullptr;
    int rc = verdict_ptr(&v);
    if (rc) return rc;
    hipLaunchKernelGGL(verdict_clear_kernel, dim3(1), dim3(64), 0, st, v);
    hipLaunchKernelGGL(validate_kernel, dim3((unsigned)((n_rays + 1 + 255) / 256)), dim3(256), 0, st, n_rays,
                       n_samples, ray_offsets, s_mid, v);
    rc = check_hip(hipGetLastError(), "validate_kernel launch");
    if (rc) return rc;
    int host = 0;
    rc = check_hip(hipMemcpyAsync(&host, v, sizeof(int), hipMemcpyDeviceToHost, st), "verdict read-back");
    if (!rc) rc = check_hip(hipStreamSynchronize(st), "verdict wait");
    if (rc) return rc;
    if (host & BAD_OFFSETS)
        return set_error(DVGO_ERR_SHAPE, "ray_offsets must start at 0, never decrease and end at n_samples (%lld)",
                         (long long)n_samples);
    if (host & BAD_ORDER) return set_error(DVGO_ERR_UNSORTED, "s_mid decreases within a ray");
    return DVGO_OK;
}

}  // namespace dvgo

extern "C" int dvgo_act_shift(double alpha_init, double delta_ref, double *shift) {
    if (!shift) return set_error(DVGO_ERR_NULL, "shift is NULL");
    if (!(alpha_init > 0.0 && alpha_init < 1.0)) return set_error(DVGO_ERR_RANGE, "alpha_init must be in (0, 1)");
    if (!(delta_ref > 0.0 && delta_ref < 1e30)) return set_error(DVGO_ERR_RANGE, "delta_ref must be positive");
    // (1 - a)^(-1/d) - 1 = expm1(-log1p(-a)/d): no cancellation for small alpha_init
    *shift = log(expm1(-log1p(-alpha_init) / delta_ref));
    return DVGO_OK;
}

extern "C" int dvgo_set_debug(int32_t on) {
    (void)debug_mode();  // the environment's setting is read first, so this call overrides it
    std::lock_guard<std::mutex> lk(g_mu);
    const int prev = g_debug;
    g_debug = on ? 1 : 0;
    return prev;
}

extern "C" int dvgo_validate_samples(const dvgo_samples *s, void *stream) {
    if (!s) return set_error(DVGO_ERR_NULL, "samples is NULL");
    if (s->struct_size != sizeof(dvgo_samples)) return set_error(DVGO_ERR_ABI, "dvgo_samples.struct_size mismatch");
    if (s->n_samples > 0 && !s->s_mid) return set_error(DVGO_ERR_NULL, "s_mid is NULL");
    return validate_batch(s->n_rays, s->n_samples, s->ray_offsets, s->s_mid, (hipStream_t)stream);
}
