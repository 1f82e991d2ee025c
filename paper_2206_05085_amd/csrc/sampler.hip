// Sample producer: parsimonious sampling inside the scene box (section 3, re-implemented
// rendering utilities) or along forward-facing rays warped to normalised device coordinates
// (section 5.3), with occupancy compaction (section 1), and the occupancy mask update.
//
// The producer runs in two passes over the same per-ray arithmetic: a count pass (one wave
// per ray, candidates in chunks of 64 lanes, a ballot per chunk), a one-block prefix sum that
// turns the counts into ray_offsets, and an emit pass that recomputes every candidate and
// writes the kept ones at offset + (live lanes below it).  Both passes call the same device
// functions, whose float32 operations are each rounded on their own (no contraction), so
// the two passes and any other IEEE float32 evaluation of the same steps take identical
// decisions.
#include <cfloat>
#include <cmath>

#include "dvgo_internal.h"

using namespace dvgo;

namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kMaxPerRay = 1 << 20;

struct SamplerArgs {
    float bmin[3], bmax[3];
    float near, step;
    float delta;       // every sample's alpha interval: step / voxel (box), step (NDC planes)
    int max_per_ray;
    int mn[3];         // mask vertex grid
    const uint8_t *mask;
    float fx, fy;      // NDC: 2 focal / W, 2 focal / H
    float span;        // NDC: planes - 1
    int n_ndc;         // NDC: candidates per ray, min(floor(span / step) + 1, max_per_ray)
};

// Per-ray plan: the number of candidates and what places them.
struct RayPlan {
    int n;
    float tn, te;            // box mode: interval along t
    float on[3], dn[3];      // NDC mode: origin and direction of the warped ray
};

// Box interval of one ray by the slab method; returns the number of candidates.
__device__ __forceinline__ int clip_ray(const SamplerArgs &a, const float (&o)[3], const float (&d)[3], float &tn,
                                        float &te) {
#pragma clang fp contract(off)
    float enter = -INFINITY, leave = INFINITY;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        float lo, hi;
        if (d[ax] != 0.0f) {
            const float t0 = (a.bmin[ax] - o[ax]) / d[ax];
            const float t1 = (a.bmax[ax] - o[ax]) / d[ax];
            lo = t0 < t1 ? t0 : t1;
            hi = t0 < t1 ? t1 : t0;
        } else if (a.bmin[ax] <= o[ax] && o[ax] <= a.bmax[ax]) {
            lo = -INFINITY;
            hi = INFINITY;
        } else {
            lo = INFINITY;
            hi = -INFINITY;
        }
        enter = lo > enter ? lo : enter;
        leave = hi < leave ? hi : leave;
    }
    tn = enter > a.near ? enter : a.near;
    te = leave;
    if (!(leave > tn)) return 0;
    // candidates at t_k = t_near + (k + 1/2) step while t_k < t_exit
    const float c = (leave - tn) / a.step - 0.5f;
    if (!(c > 0.0f)) return 0;
    if (c > (float)a.max_per_ray) return a.max_per_ray;
    return (int)__builtin_ceilf(c);
}

// Whether the mask keeps point x (nearest vertex, clamped to the grid).
__device__ __forceinline__ bool mask_keeps(const SamplerArgs &a, const float (&x)[3]) {
#pragma clang fp contract(off)
    if (!a.mask) return true;
    int idx[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const float sc = (float)(a.mn[ax] - 1) / (a.bmax[ax] - a.bmin[ax]);
        const float u = (x[ax] - a.bmin[ax]) * sc;
        if (!(u >= 0.0f)) idx[ax] = 0;
        else if (u >= (float)(a.mn[ax] - 1)) idx[ax] = a.mn[ax] - 1;
        else idx[ax] = (int)__builtin_rintf(u);
    }
    return a.mask[((int64_t)idx[0] * a.mn[1] + idx[1]) * a.mn[2] + idx[2]] != 0;
}

// NeRF's normalised device coordinates of a forward-facing ray (camera looking down -z):
// the origin moves to the near plane, then origin and direction are warped so that NDC
// depth runs from -1 (near plane) to 1 (infinity) over t' in [0, 1].
__device__ __forceinline__ bool ndc_ray(const SamplerArgs &a, const float (&o)[3], const float (&d)[3],
                                        float (&on)[3], float (&dn)[3]) {
#pragma clang fp contract(off)
    if (!(d[2] < 0.0f)) return false;  // never crosses the near plane in front of the camera
    const float t0 = -(a.near + o[2]) / d[2];
    float p[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) p[ax] = __builtin_fmaf(t0, d[ax], o[ax]);
    const float qx = p[0] / p[2], qy = p[1] / p[2];
    const float nz = (2.0f * a.near) / p[2];
    on[0] = -(a.fx * qx);
    on[1] = -(a.fy * qy);
    on[2] = 1.0f + nz;
    dn[0] = -(a.fx * (d[0] / d[2] - qx));
    dn[1] = -(a.fy * (d[1] / d[2] - qy));
    dn[2] = -nz;
    return true;
}

template <int MODE>
__device__ __forceinline__ RayPlan plan_ray(const SamplerArgs &a, const float (&o)[3], const float (&d)[3]) {
    RayPlan p;
    if (MODE == DVGO_SAMPLE_BOX) {
        p.n = clip_ray(a, o, d, p.tn, p.te);
    } else {
        p.tn = 0.0f;
        p.te = ndc_ray(a, o, d, p.on, p.dn) ? 1.0f : 0.0f;
        p.n = p.te > 0.0f ? a.n_ndc : 0;
    }
    return p;
}

// Point of candidate k of a ray and whether it is kept.
template <int MODE>
__device__ __forceinline__ bool candidate(const SamplerArgs &a, const RayPlan &p, const float (&o)[3],
                                          const float (&d)[3], int k, float (&x)[3]) {
#pragma clang fp contract(off)
    if (MODE == DVGO_SAMPLE_BOX) {
        // the midpoint of the k-th step after t_near
        const float t = __builtin_fmaf((float)k + 0.5f, a.step, p.tn);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) x[ax] = __builtin_fmaf(t, d[ax], o[ax]);
    } else {
        // plane coordinate k step; dropped outside the box across the image axes
        const float t = ((float)k * a.step) / a.span;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) x[ax] = __builtin_fmaf(t, p.dn[ax], p.on[ax]);
        if (!(a.bmin[0] <= x[0] && x[0] <= a.bmax[0] && a.bmin[1] <= x[1] && x[1] <= a.bmax[1])) return false;
    }
    return mask_keeps(a, x);
}

__device__ __forceinline__ int wave_ray() {
    return blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ void load_ray(const float *org, const float *dir, int r, float (&o)[3], float (&d)[3]) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        o[ax] = org[3 * (int64_t)r + ax];
        d[ax] = dir[3 * (int64_t)r + ax];
    }
}

// kept candidates per ray -> offs[r + 1]; the ray's parameter interval -> t_near / t_far
// (0, 0 when it has none)
template <int MODE>
__global__ __launch_bounds__(256) void sample_count_kernel(SamplerArgs a, int R, const float *org, const float *dir,
                                                           int *offs, float *t_near, float *t_far) {
    const int r = wave_ray();
    if (r >= R) return;
    float o[3], d[3];
    load_ray(org, dir, r, o, d);
    const RayPlan p = plan_ray<MODE>(a, o, d);
    int cnt = p.n;
    if (a.mask || MODE == DVGO_SAMPLE_NDC) {
        cnt = 0;
        for (int k0 = 0; k0 < p.n; k0 += 64) {
            const int k = k0 + lane();
            float x[3];
            const bool live = k < p.n && candidate<MODE>(a, p, o, d, k, x);
            cnt += __popcll(__ballot(live));
        }
    }
    if (lane() == 0) {
        offs[r + 1] = cnt;
        const bool hit = p.te > p.tn;
        if (t_near) t_near[r] = hit ? p.tn : 0.0f;
        if (t_far) t_far[r] = hit ? p.te : 0.0f;
    }
}

// offs[1..R] (counts) -> inclusive prefix sums in place; offs[0] = 0.  One block; each pass
// covers SCAN_E consecutive entries per thread (all loads issued before the block scan).
constexpr int SCAN_E = 8;

__global__ __launch_bounds__(1024) void offsets_scan_kernel(int R, int *offs) {
    __shared__ int wsum[16];
    __shared__ int carry;
    if (threadIdx.x == 0) {
        carry = 0;
        offs[0] = 0;
    }
    __syncthreads();
    for (int base = 0; base < R; base += 1024 * SCAN_E) {
        const int r0 = base + threadIdx.x * SCAN_E;
        int v[SCAN_E];
#pragma unroll
        for (int e = 0; e < SCAN_E; ++e) v[e] = r0 + e < R ? offs[r0 + e + 1] : 0;
#pragma unroll
        for (int e = 1; e < SCAN_E; ++e) v[e] += v[e - 1];
        int t = v[SCAN_E - 1];
#pragma unroll
        for (int s = 1; s < 64; s <<= 1) {
            const int u = __shfl_up(t, s, 64);
            if (lane() >= s) t += u;
        }
        if (lane() == 63) wsum[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x < 16) {
            int w = wsum[threadIdx.x];
#pragma unroll
            for (int s = 1; s < 16; s <<= 1) {
                const int u = __shfl_up(w, s, 16);
                if ((int)threadIdx.x >= s) w += u;
            }
            wsum[threadIdx.x] = w;
        }
        __syncthreads();
        // entries before this thread's run: carry + earlier waves + earlier lanes of this wave
        const int before = carry + ((threadIdx.x >> 6) ? wsum[(threadIdx.x >> 6) - 1] : 0) + t - v[SCAN_E - 1];
#pragma unroll
        for (int e = 0; e < SCAN_E; ++e)
            if (r0 + e < R) offs[r0 + e + 1] = before + v[e];
        __syncthreads();
        if (threadIdx.x == 0) carry += wsum[15];
        __syncthreads();
    }
}

// kept candidates of ray r at offs[r] + (kept candidates before them); indices outside
// [0, capacity) are not written
template <int MODE>
__global__ __launch_bounds__(256) void sample_emit_kernel(SamplerArgs a, int R, const float *org, const float *dir,
                                                          const int *offs, int64_t capacity, float *xyz,
                                                          float *delta, float *s_mid, float *s_len) {
    const int r = wave_ray();
    if (r >= R) return;
    float o[3], d[3];
    load_ray(org, dir, r, o, d);
    const RayPlan p = plan_ray<MODE>(a, o, d);
    const int n = p.n;
    if (n == 0) return;
    const float fn = (float)n;
    const float sl = 1.0f / fn;
    int64_t pos = offs[r];
    for (int k0 = 0; k0 < n; k0 += 64) {
        const int k = k0 + lane();
        float x[3];
        const bool live = k < n && candidate<MODE>(a, p, o, d, k, x);
        const uint64_t b = __ballot(live);
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0));
        const int64_t i = pos + below;
        if (live && i >= 0 && i < capacity) {
            xyz[3 * i + 0] = x[0];
            xyz[3 * i + 1] = x[1];
            xyz[3 * i + 2] = x[2];
            delta[i] = a.delta;
            s_mid[i] = ((float)k + 0.5f) / fn;
            s_len[i] = sl;
        }
        pos += __popcll(b);
    }
}

// mask[v] = mask[v] && (some vertex of the 3x3x3 neighbourhood has raw >= thr); thr is the
// smallest float32 logit whose alpha at the sampling step reaches the alpha threshold.  A
// thread owns OCC_Z consecutive z vertices of one (x, y) column: it ORs the dense test over
// the 3x3 (x, y) neighbours for z0-1 .. z0+OCC_Z, then each output ORs three of those.
constexpr int OCC_Z = 4;

__global__ __launch_bounds__(256) void occupancy_kernel(const float *raw, int cs, int nx, int ny, int nz, float thr,
                                                        uint8_t *mask) {
    const int nq = (nz + OCC_Z - 1) / OCC_Z;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nx * ny * nq) return;
    const int q = t % nq;
    const int y = (t / nq) % ny;
    const int x = t / (nq * ny);
    const int z0 = q * OCC_Z;
    const int64_t row = ((int64_t)x * ny + y) * nz;
    uint8_t m[OCC_Z];
    bool any = false;
#pragma unroll
    for (int j = 0; j < OCC_Z; ++j) {
        m[j] = z0 + j < nz ? mask[row + z0 + j] : 0;
        any |= m[j] != 0;
    }
    if (!any) return;  // already 0 everywhere: nothing to switch off
    bool col[OCC_Z + 2] = {};
    for (int a = x > 0 ? x - 1 : 0; a <= (x + 1 < nx ? x + 1 : nx - 1); ++a)
        for (int b = y > 0 ? y - 1 : 0; b <= (y + 1 < ny ? y + 1 : ny - 1); ++b) {
            const float *p = raw + ((int64_t)a * ny + b) * nz * cs;
#pragma unroll
            for (int i = 0; i < OCC_Z + 2; ++i) {
                const int z = z0 - 1 + i;
                if (z >= 0 && z < nz) col[i] |= p[(int64_t)z * cs] >= thr;
            }
        }
#pragma unroll
    for (int j = 0; j < OCC_Z; ++j)
        if (z0 + j < nz) mask[row + z0 + j] = (m[j] != 0 && (col[j] || col[j + 1] || col[j + 2])) ? 1 : 0;
}

int make_sampler(const dvgo_sampler *sp, int32_t n_rays, const float *org, const float *dir, SamplerArgs &a) {
    if (!sp) return set_error(DVGO_ERR_NULL, "sampler is NULL");
    if (sp->struct_size != sizeof(dvgo_sampler)) return set_error(DVGO_ERR_ABI, "dvgo_sampler.struct_size mismatch");
    if (n_rays < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays");
    if (n_rays > 0 && (!org || !dir)) return set_error(DVGO_ERR_NULL, "origins or dirs is NULL");
    for (int ax = 0; ax < 3; ++ax) {
        if (!(sp->xyz_max[ax] > sp->xyz_min[ax]) || !std::isfinite(sp->xyz_min[ax]) || !std::isfinite(sp->xyz_max[ax]))
            return set_error(DVGO_ERR_SHAPE, "sampler box: need finite xyz_min < xyz_max");
        a.bmin[ax] = sp->xyz_min[ax];
        a.bmax[ax] = sp->xyz_max[ax];
    }
    if (!(sp->step > 0.f) || !std::isfinite(sp->step) || !(sp->voxel > 0.f) || !std::isfinite(sp->voxel))
        return set_error(DVGO_ERR_RANGE, "step and voxel must be positive and finite");
    if (!std::isfinite(sp->near)) return set_error(DVGO_ERR_RANGE, "near must be finite");
    if (sp->max_per_ray < 1 || sp->max_per_ray > kMaxPerRay)
        return set_error(DVGO_ERR_RANGE, "max_per_ray must be in [1, 2^20]");
    if ((int64_t)sp->max_per_ray * n_rays > INT32_MAX)
        return set_error(DVGO_ERR_RANGE, "max_per_ray * n_rays must stay below 2^31 (int32 offsets)");
    a.mask = sp->mask;
    if (sp->mask) {
        int64_t cells = 1;
        for (int ax = 0; ax < 3; ++ax) {
            if (sp->mask_shape[ax] < 1) return set_error(DVGO_ERR_SHAPE, "mask_shape entries must be >= 1");
            cells *= sp->mask_shape[ax];
        }
        if (cells >= ((int64_t)1 << 31)) return set_error(DVGO_ERR_RANGE, "mask has >= 2^31 vertices");
    }
    for (int ax = 0; ax < 3; ++ax) a.mn[ax] = sp->mask ? sp->mask_shape[ax] : 1;
    a.near = sp->near;
    a.step = sp->step;
    a.delta = sp->step / sp->voxel;
    a.max_per_ray = sp->max_per_ray;
    a.fx = a.fy = a.span = 0.0f;
    a.n_ndc = 0;
    if (sp->mode == DVGO_SAMPLE_NDC) {
        if (!(sp->near > 0.f)) return set_error(DVGO_ERR_RANGE, "NDC sampling needs near > 0");
        if (!(sp->ndc_fx > 0.f) || !(sp->ndc_fy > 0.f) || !std::isfinite(sp->ndc_fx) || !std::isfinite(sp->ndc_fy))
            return set_error(DVGO_ERR_RANGE, "NDC sampling needs positive finite ndc_fx, ndc_fy");
        if (sp->ndc_planes < 2) return set_error(DVGO_ERR_SHAPE, "NDC sampling needs ndc_planes >= 2");
        a.fx = sp->ndc_fx;
        a.fy = sp->ndc_fy;
        a.span = (float)(sp->ndc_planes - 1);
        const float jmax = std::floor(a.span / sp->step);
        a.n_ndc = jmax + 1.0f > (float)sp->max_per_ray ? sp->max_per_ray : (int)jmax + 1;
        a.delta = sp->step;
    } else if (sp->mode != DVGO_SAMPLE_BOX) {
        return set_error(DVGO_ERR_UNSUPPORTED, "unknown sampler mode %d", sp->mode);
    }
    return DVGO_OK;
}

int ray_blocks(int R) { return (R + kWavesPerBlock - 1) / kWavesPerBlock; }

// Smallest float32 logit raw with 1 - exp(-softplus(raw + b) delta) >= alpha_thr.
float logit_threshold(double b, double delta, double alpha_thr) {
    const double sigma = -std::log1p(-alpha_thr) / delta;                            // alpha_thr -> sigma
    const double z = sigma > 30.0 ? sigma + std::log1p(-std::exp(-sigma)) : std::log(std::expm1(sigma));  // softplus^-1
    const double t = z - b;
    if (t > (double)FLT_MAX) return INFINITY;
    float f = (float)t;
    if ((double)f < t) f = std::nextafter(f, INFINITY);
    return f;
}

}  // namespace

extern "C" int dvgo_sample_count(const dvgo_sampler *sp, int32_t n_rays, const float *origins, const float *dirs,
                                 int32_t *ray_offsets, float *t_near, float *t_far, void *stream) {
    SamplerArgs a;
    int rc = make_sampler(sp, n_rays, origins, dirs, a);
    if (rc) return rc;
    if (!ray_offsets) return set_error(DVGO_ERR_NULL, "ray_offsets is NULL");
    if (n_rays > 0) {
        if (sp->mode == DVGO_SAMPLE_NDC)
            hipLaunchKernelGGL(sample_count_kernel<DVGO_SAMPLE_NDC>, dim3(ray_blocks(n_rays)),
                               dim3(64 * kWavesPerBlock), 0, (hipStream_t)stream, a, n_rays, origins, dirs,
                               ray_offsets, t_near, t_far);
        else
            hipLaunchKernelGGL(sample_count_kernel<DVGO_SAMPLE_BOX>, dim3(ray_blocks(n_rays)),
                               dim3(64 * kWavesPerBlock), 0, (hipStream_t)stream, a, n_rays, origins, dirs,
                               ray_offsets, t_near, t_far);
        rc = check_hip(hipGetLastError(), "sample_count_kernel launch");
        if (rc) return rc;
    }
    hipLaunchKernelGGL(offsets_scan_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, n_rays, ray_offsets);
    return check_hip(hipGetLastError(), "offsets_scan_kernel launch");
}

extern "C" int dvgo_sample_emit(const dvgo_sampler *sp, int32_t n_rays, const float *origins, const float *dirs,
                                const int32_t *ray_offsets, int64_t capacity, float *xyz, float *delta, float *s_mid,
                                float *s_len, void *stream) {
    SamplerArgs a;
    int rc = make_sampler(sp, n_rays, origins, dirs, a);
    if (rc) return rc;
    if (capacity < 0) return set_error(DVGO_ERR_SHAPE, "negative capacity");
    if (n_rays == 0 || capacity == 0) return DVGO_OK;
    if (!ray_offsets || !xyz || !delta || !s_mid || !s_len)
        return set_error(DVGO_ERR_NULL, "ray_offsets or an output array is NULL");
    if (sp->mode == DVGO_SAMPLE_NDC)
        hipLaunchKernelGGL(sample_emit_kernel<DVGO_SAMPLE_NDC>, dim3(ray_blocks(n_rays)), dim3(64 * kWavesPerBlock),
                           0, (hipStream_t)stream, a, n_rays, origins, dirs, ray_offsets, capacity, xyz, delta, s_mid,
                           s_len);
    else
        hipLaunchKernelGGL(sample_emit_kernel<DVGO_SAMPLE_BOX>, dim3(ray_blocks(n_rays)), dim3(64 * kWavesPerBlock),
                           0, (hipStream_t)stream, a, n_rays, origins, dirs, ray_offsets, capacity, xyz, delta, s_mid,
                           s_len);
    return check_hip(hipGetLastError(), "sample_emit_kernel launch");
}

extern "C" int dvgo_occupancy_update(const dvgo_grid *density, float act_shift, float delta, float alpha_thr,
                                     uint8_t *mask, void *stream) {
    DevGrid dg;
    int rc = make_dev_grid(density, "density", &dg, false);
    if (rc) return rc;
    if (!mask) return set_error(DVGO_ERR_NULL, "mask is NULL");
    if (!(delta > 0.f) || !std::isfinite(delta)) return set_error(DVGO_ERR_RANGE, "delta must be positive and finite");
    if (!(alpha_thr >= 0.f && alpha_thr < 1.f)) return set_error(DVGO_ERR_RANGE, "alpha_thr must be in [0, 1)");
    if (!std::isfinite(act_shift)) return set_error(DVGO_ERR_RANGE, "act_shift must be finite");
    const float thr = logit_threshold(act_shift, delta, alpha_thr);
    const int64_t threads = (int64_t)dg.n[0] * dg.n[1] * ((dg.n[2] + OCC_Z - 1) / OCC_Z);
    hipLaunchKernelGGL(occupancy_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       dg.data, dg.cs, dg.n[0], dg.n[1], dg.n[2], thr, mask);
    return check_hip(hipGetLastError(), "occupancy_kernel launch");
}
