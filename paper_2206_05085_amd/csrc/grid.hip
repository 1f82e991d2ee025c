// Grid gather/scatter, alpha, fused Adam, loss head and the host-side plumbing of libdvgo.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "dvgo_internal.h"

namespace dvgo {

static thread_local char g_err[512] = "";

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return DVGO_OK;
    return set_error(DVGO_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int make_dev_grid(const dvgo_grid *g, const char *name, DevGrid *out, bool need_grad) {
    if (!g) return set_error(DVGO_ERR_NULL, "%s grid is NULL", name);
    if (g->struct_size != sizeof(dvgo_grid)) return set_error(DVGO_ERR_ABI, "%s: dvgo_grid.struct_size mismatch", name);
    if (g->nx < 2 || g->ny < 2 || g->nz < 2) return set_error(DVGO_ERR_SHAPE, "%s: every grid dimension must be >= 2", name);
    if (g->channels < 1 || g->ch_stride < g->channels || g->ch_stride > 16)
        return set_error(DVGO_ERR_SHAPE, "%s: need 1 <= channels <= ch_stride <= 16", name);
    const int64_t total = (int64_t)g->nx * g->ny * g->nz * g->ch_stride;
    if (total >= ((int64_t)1 << 31)) return set_error(DVGO_ERR_RANGE, "%s: grid has >= 2^31 floats", name);
    if (!g->data) return set_error(DVGO_ERR_NULL, "%s: data is NULL", name);
    if (need_grad && !g->grad) return set_error(DVGO_ERR_NULL, "%s: grad is NULL", name);
    out->data = g->data;
    out->grad = g->grad;
    out->n[0] = g->nx;
    out->n[1] = g->ny;
    out->n[2] = g->nz;
    out->cs = g->ch_stride;
    out->C = g->channels;
    out->sy = g->nz * g->ch_stride;
    out->sx = g->ny * out->sy;
    for (int a = 0; a < 3; ++a) {
        const double lo = g->xyz_min[a], hi = g->xyz_max[a];
        if (!(hi > lo)) return set_error(DVGO_ERR_SHAPE, "%s: xyz_max must exceed xyz_min", name);
        const double s = (double)(out->n[a] - 1) / (hi - lo);
        const double o = -lo * s;
        out->s_hi[a] = (float)s;
        out->s_lo[a] = (float)(s - (double)out->s_hi[a]);
        out->o_hi[a] = (float)o;
        out->o_lo[a] = (float)(o - (double)out->o_hi[a]);
        out->s_d[a] = s;
        out->o_d[a] = o;
    }
    if (g->warp != DVGO_WARP_NONE && g->warp != DVGO_WARP_CONTRACT_INF && g->warp != DVGO_WARP_CONTRACT_L2)
        return set_error(DVGO_ERR_UNSUPPORTED, "%s: unknown warp %d", name, g->warp);
    if (g->warp != DVGO_WARP_NONE && !(g->warp_b > 0.f && g->warp_b < 1e30f))
        return set_error(DVGO_ERR_RANGE, "%s: the contraction's b must be positive and finite", name);
    out->warp = g->warp;
    out->wb = g->warp_b;
    return DVGO_OK;
}

}  // namespace dvgo

using namespace dvgo;

namespace {

constexpr int kBlock = 256;

int grid_blocks(int64_t work, int per_block = kBlock) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b > 65535 * 16) b = 65535 * 16;
    return (int)(b < 1 ? 1 : b);
}

template <bool W>
__global__ __launch_bounds__(kBlock) void gather_kernel(DevGrid g, int64_t S, const float *__restrict__ xyz,
                                                        float *__restrict__ out, int vec_out) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < S; k += (int64_t)gridDim.x * kBlock) {
        const Tri t = trilinear<W>(g, xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2]);
        float acc[16];
#pragma unroll
        for (int ch = 0; ch < 16; ++ch) acc[ch] = 0.f;
        if ((g.cs & 3) == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (4 * q < g.C) {
                    const float4 v = interp4(g, t, 4 * q);
                    acc[4 * q] = v.x;
                    acc[4 * q + 1] = v.y;
                    acc[4 * q + 2] = v.z;
                    acc[4 * q + 3] = v.w;
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const float *p = g.data + t.base + corner_off(g, c);
#pragma unroll
                for (int ch = 0; ch < 16; ++ch)
                    if (ch < g.C) acc[ch] += t.w[c] * p[ch];
            }
        }
        if (vec_out) {
            // C % 4 == 0 and out 16-byte aligned: the row leaves as C / 4 float4 stores
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (4 * q < g.C)
                    *reinterpret_cast<float4 *>(out + k * g.C + 4 * q) =
                        make_float4(acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]);
        } else {
#pragma unroll
            for (int ch = 0; ch < 16; ++ch)
                if (ch < g.C) out[k * g.C + ch] = acc[ch];
        }
    }
}

// Rows made of whole float4 groups (ch_stride % 4 == 0): G adjacent lanes share a sample, lane
// r of them taking channels 4r..4r+3 (G = ceil(C / 4)), 64 / G consecutive samples per wave.  The
// G lanes of a sample read each corner's row as one contiguous span in the same instruction, so a
// corner costs one or two lines per load rather than G loads spread over G instructions, and the
// wave's working set stays small enough for the cache to keep the rows its neighbours reuse.
// Same helper (interp4) as the one-lane-per-sample path and the colour head's fused lookup: the
// same bits.
template <int G, bool W>
__global__ __launch_bounds__(kBlock) void gather_groups_kernel(DevGrid g, int64_t S, const float *__restrict__ xyz,
                                                               float *__restrict__ out, int vec_out) {
    constexpr int SPW = 64 / G;  // samples per wave
    const int ln = lane(), sl = ln / G, r = ln - sl * G;
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t base = ((blockIdx.x * (int64_t)kBlock + threadIdx.x) >> 6) * SPW; base < S; base += nwaves * SPW) {
        const int64_t k = base + sl;
        if (sl >= SPW || k >= S) continue;
        const Tri t = trilinear<W>(g, xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2]);
        const float4 v = interp4(g, t, 4 * r);
        if (vec_out) {
            *reinterpret_cast<float4 *>(out + k * g.C + 4 * r) = v;
        } else {
            const float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (4 * r + i < g.C) out[k * g.C + 4 * r + i] = e[i];
        }
    }
}

template <int G>
void launch_gather_groups(const DevGrid &dg, int64_t S, const float *xyz, float *out, int vec_out, hipStream_t st) {
    const int64_t waves = (S + 64 / G - 1) / (64 / G);
    int64_t blocks = (waves + kBlock / 64 - 1) / (kBlock / 64);
    if (blocks > 65535 * 16) blocks = 65535 * 16;
    if (dg.warp)
        hipLaunchKernelGGL((gather_groups_kernel<G, true>), dim3((unsigned)blocks), dim3(kBlock), 0, st, dg, S, xyz, out,
                           vec_out);
    else
        hipLaunchKernelGGL((gather_groups_kernel<G, false>), dim3((unsigned)blocks), dim3(kBlock), 0, st, dg, S, xyz,
                           out, vec_out);
}

// One lane per sample, 64 consecutive samples per wave: consecutive samples lie along a
// ray, so contributions to shared vertices are summed in the wave before the atomics.
template <int NC, bool W>
__global__ __launch_bounds__(kBlock) void scatter_kernel(DevGrid g, int64_t S, const float *__restrict__ xyz,
                                                         const float *__restrict__ gout, int vec_in) {
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    const int64_t wave = (blockIdx.x * (int64_t)kBlock + threadIdx.x) >> 6;
    for (int64_t base = wave * 64; base < S; base += nwaves * 64) {
        const int64_t k = base + lane();
        const bool valid = k < S;
        Cell cl{0, 0, 0, 0.f, 0.f, 0.f};
        float v[NC];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) v[ch] = 0.f;
        if (valid) {
            cl = cell_of<W>(g, xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2]);
            if (NC % 4 == 0 && vec_in) {
                // C % 4 == 0 and gout 16-byte aligned: the row arrives as C / 4 float4 loads
#pragma unroll
                for (int q = 0; q < NC / 4; ++q)
                    if (4 * q < g.C) {
                        const float4 t = *reinterpret_cast<const float4 *>(gout + k * g.C + 4 * q);
                        v[4 * q] = t.x;
                        v[4 * q + 1] = t.y;
                        v[4 * q + 2] = t.z;
                        v[4 * q + 3] = t.w;
                    }
            } else {
#pragma unroll
                for (int ch = 0; ch < NC; ++ch)
                    if (ch < g.C) v[ch] = gout[k * g.C + ch];
            }
        }
        scatter_wave<NC>(g, valid, cl, v, g.C);
    }
}

// rows of C floats can move as float4: C % 4 == 0 and the array 16-byte aligned
inline int vec_rows(const float *p, int C) { return (C & 3) == 0 && ((uintptr_t)p & 15) == 0 ? 1 : 0; }

template <int NC>
void launch_scatter(const DevGrid &dg, int64_t S, const float *xyz, const float *gout, hipStream_t st) {
    int64_t waves = (S + 63) / 64;
    int64_t blocks = (waves + 3) / 4;
    if (blocks > 256 * 16) blocks = 256 * 16;
    if (dg.warp)
        hipLaunchKernelGGL((scatter_kernel<NC, true>), dim3((unsigned)blocks), dim3(kBlock),
                           scatter_lds_bytes(NC, kBlock), st, dg, S, xyz, gout, vec_rows(gout, dg.C));
    else
        hipLaunchKernelGGL((scatter_kernel<NC, false>), dim3((unsigned)blocks), dim3(kBlock),
                           scatter_lds_bytes(NC, kBlock), st, dg, S, xyz, gout, vec_rows(gout, dg.C));
}

template <bool W>
__global__ __launch_bounds__(kBlock) void alpha_kernel(DevGrid g, int64_t S, const float *__restrict__ xyz,
                                                       const float *__restrict__ delta, float shift,
                                                       float *__restrict__ alpha) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < S; k += (int64_t)gridDim.x * kBlock) {
        const Tri t = trilinear<W>(g, xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2]);
        const float raw = interp_ch(g, t, 0);
        alpha[k] = -expm1f(-softplusf(raw + shift) * delta[k]);
    }
}

// Streams the four arrays as float4 (the 16-byte-aligned body) with a scalar head/tail.
// With skip, a float4 group whose four gradients are all zero is not read further and
// nothing is written; within a partly non-zero group the zero-gradient lanes keep their
// values bit for bit.  Each thread takes ADAM_U groups a stride apart per pass and issues
// all their gradient loads, then all parameter / moment loads, before it computes, so a
// wave keeps several independent loads in flight instead of one dependent chain.  The skip
// is decided per 128-byte line (the 8 lanes holding 8 consecutive groups): a line with any
// non-zero gradient is read and written whole, its zero-gradient elements written back
// unchanged, so the memory sees full-line writes instead of masked partial ones.  Gradients and
// moments are read and written with the nontemporal (streaming) cache hint, since nothing else in a
// step reads them again soon; the parameters keep the default policy, since the next step's lookups
// read them back.
constexpr int ADAM_U = 4;

__global__ __launch_bounds__(kBlock) void adam_kernel(AdamArgs a, int64_t head, int64_t n4) {
    adam_bias(a);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t tid = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    float4 *P = reinterpret_cast<float4 *>(a.p + head), *G = reinterpret_cast<float4 *>(a.g + head);
    float4 *M = reinterpret_cast<float4 *>(a.m + head), *V = reinterpret_cast<float4 *>(a.v + head);
    for (int64_t i0 = tid; i0 < n4; i0 += ADAM_U * stride) {
        float4 g[ADAM_U], p[ADAM_U], m[ADAM_U], v[ADAM_U];
        bool live[ADAM_U];
#pragma unroll
        for (int u = 0; u < ADAM_U; ++u) {
            const int64_t i = i0 + u * stride;
            g[u] = i < n4 ? ld_nt(G + i) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < ADAM_U; ++u) {
            const int64_t i = i0 + u * stride;
            const bool any = g[u].x != 0.f || g[u].y != 0.f || g[u].z != 0.f || g[u].w != 0.f;
            // any non-zero gradient among the 8 lanes of this lane's line (groups i & ~7 .. i | 7)
            const unsigned long long b = __ballot(any);
            const bool line = ((b >> (lane() & ~7)) & 0xFFull) != 0;
            live[u] = i < n4 && (!a.skip || line);
            if (live[u]) {
                p[u] = P[i];
                m[u] = ld_nt(M + i);
                v[u] = ld_nt(V + i);
            }
        }
#pragma unroll
        for (int u = 0; u < ADAM_U; ++u) {
            if (!live[u]) continue;
            const int64_t i = i0 + u * stride;
            if (!a.skip || g[u].x != 0.f) adam_one(a, g[u].x, p[u].x, m[u].x, v[u].x);
            if (!a.skip || g[u].y != 0.f) adam_one(a, g[u].y, p[u].y, m[u].y, v[u].y);
            if (!a.skip || g[u].z != 0.f) adam_one(a, g[u].z, p[u].z, m[u].z, v[u].z);
            if (!a.skip || g[u].w != 0.f) adam_one(a, g[u].w, p[u].w, m[u].w, v[u].w);
            P[i] = p[u];
            st_nt(M + i, m[u]);
            st_nt(V + i, v[u]);
            if (a.zero) st_nt(G + i, make_float4(0.f, 0.f, 0.f, 0.f));
        }
    }
    // scalar head [0, head) and tail [head + 4 n4, n)
    const int64_t tail0 = head + 4 * n4;
    const int64_t nscalar = head + (a.n - tail0);
    for (int64_t j = tid; j < nscalar; j += stride) {
        const int64_t i = j < head ? j : tail0 + (j - head);
        const float g = a.g[i];
        if (a.skip && g == 0.f) continue;
        adam_one(a, g, a.p[i], a.m[i], a.v[i]);
        if (a.zero) a.g[i] = 0.f;
    }
}

// gradients only (thread per ray): the same expressions as loss_head_kernel's
__global__ __launch_bounds__(256) void loss_grad_kernel(int R, const float *__restrict__ rgb,
                                                        const float *__restrict__ tgt, float lam, float *grad_rgb,
                                                        float *grad_dist) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= R) return;
    const float inv3R = 1.f / (3.f * (float)R), invR = 1.f / (float)R;
    if (grad_rgb) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) grad_rgb[3 * r + ch] = 2.f * (rgb[3 * r + ch] - tgt[3 * r + ch]) * inv3R;
    }
    if (grad_dist) grad_dist[r] = lam * invR;
}

// single block: the loss is written (not accumulated), so no pre-zeroed scalar is needed
__global__ __launch_bounds__(1024) void loss_head_kernel(int R, const float *__restrict__ rgb,
                                                         const float *__restrict__ tgt, const float *__restrict__ dist,
                                                         float lam, float *loss, float *grad_rgb, float *grad_dist) {
    __shared__ float red[16];
    float acc = 0.f;
    const float inv3R = 1.f / (3.f * (float)R), invR = 1.f / (float)R;
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        float e2 = 0.f;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float e = rgb[3 * r + ch] - tgt[3 * r + ch];
            e2 += e * e;
            if (grad_rgb) grad_rgb[3 * r + ch] = 2.f * e * inv3R;
        }
        acc += e2 * inv3R;
        if (dist) acc += lam * dist[r] * invR;
        if (grad_dist) grad_dist[r] = lam * invR;
    }
    acc = wave_sum(acc);
    if (lane() == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x < 64) {
        float v = threadIdx.x < (blockDim.x >> 6) ? red[threadIdx.x] : 0.f;
        v = wave_sum(v);
        if (threadIdx.x == 0 && loss) loss[0] = v;
    }
}

}  // namespace

extern "C" int dvgo_abi_version(void) { return DVGO_ABI_VERSION; }

extern "C" const char *dvgo_last_error(void) { return g_err; }

extern "C" int dvgo_grid_gather(const dvgo_grid *g, int64_t n_samples, const float *xyz, float *out, void *stream) {
    DevGrid dg;
    int rc = make_dev_grid(g, "grid", &dg, false);
    if (rc) return rc;
    if (n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative n_samples");
    if (n_samples == 0) return DVGO_OK;
    if (!xyz || !out) return set_error(DVGO_ERR_NULL, "xyz or out is NULL");
    if ((g->ch_stride & 3) == 0 && ((uintptr_t)g->data & 15))
        return set_error(DVGO_ERR_SHAPE, "grid data must be 16-byte aligned when ch_stride is a multiple of 4");
    const hipStream_t st = (hipStream_t)stream;
    const int vec_out = vec_rows(out, dg.C);
    if ((dg.cs & 3) == 0) {
        switch ((dg.C + 3) / 4) {
            case 1: launch_gather_groups<1>(dg, n_samples, xyz, out, vec_out, st); break;
            case 2: launch_gather_groups<2>(dg, n_samples, xyz, out, vec_out, st); break;
            case 3: launch_gather_groups<3>(dg, n_samples, xyz, out, vec_out, st); break;
            default: launch_gather_groups<4>(dg, n_samples, xyz, out, vec_out, st); break;
        }
        return check_hip(hipGetLastError(), "gather_groups_kernel launch");
    }
    if (dg.warp)
        hipLaunchKernelGGL(gather_kernel<true>, dim3(grid_blocks(n_samples)), dim3(kBlock), 0, st, dg, n_samples, xyz,
                           out, vec_out);
    else
        hipLaunchKernelGGL(gather_kernel<false>, dim3(grid_blocks(n_samples)), dim3(kBlock), 0, st, dg, n_samples, xyz,
                           out, vec_out);
    return check_hip(hipGetLastError(), "gather_kernel launch");
}

extern "C" int dvgo_grid_scatter(const dvgo_grid *g, int64_t n_samples, const float *xyz, const float *grad_out,
                                 void *stream) {
    DevGrid dg;
    int rc = make_dev_grid(g, "grid", &dg, true);
    if (rc) return rc;
    if (n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative n_samples");
    if (n_samples == 0) return DVGO_OK;
    if (!xyz || !grad_out) return set_error(DVGO_ERR_NULL, "xyz or grad_out is NULL");
    const hipStream_t st = (hipStream_t)stream;
    const int C = g->channels;
    if (C == 1) launch_scatter<1>(dg, n_samples, xyz, grad_out, st);
    else if (C <= 3) launch_scatter<3>(dg, n_samples, xyz, grad_out, st);
    else if (C <= 4) launch_scatter<4>(dg, n_samples, xyz, grad_out, st);
    else if (C <= 8) launch_scatter<8>(dg, n_samples, xyz, grad_out, st);
    else if (C <= 12) launch_scatter<12>(dg, n_samples, xyz, grad_out, st);
    else launch_scatter<16>(dg, n_samples, xyz, grad_out, st);
    return check_hip(hipGetLastError(), "scatter_kernel launch");
}

extern "C" int dvgo_alpha(const dvgo_grid *density, int64_t n_samples, const float *xyz, const float *delta,
                          float act_shift, float *alpha, void *stream) {
    DevGrid dg;
    int rc = make_dev_grid(density, "density", &dg, false);
    if (rc) return rc;
    if (n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative n_samples");
    if (n_samples == 0) return DVGO_OK;
    if (!xyz || !delta || !alpha) return set_error(DVGO_ERR_NULL, "xyz, delta or alpha is NULL");
    if (dg.warp)
        hipLaunchKernelGGL(alpha_kernel<true>, dim3(grid_blocks(n_samples)), dim3(kBlock), 0, (hipStream_t)stream, dg,
                           n_samples, xyz, delta, act_shift, alpha);
    else
        hipLaunchKernelGGL(alpha_kernel<false>, dim3(grid_blocks(n_samples)), dim3(kBlock), 0, (hipStream_t)stream,
                           dg, n_samples, xyz, delta, act_shift, alpha);
    return check_hip(hipGetLastError(), "alpha_kernel launch");
}

__global__ void counter_add_kernel(int *c, int d) {
    if (threadIdx.x == 0 && blockIdx.x == 0) c[0] += d;
}

extern "C" int dvgo_counter_add(int32_t *counter, int32_t delta, void *stream) {
    if (!counter) return set_error(DVGO_ERR_NULL, "counter is NULL");
    hipLaunchKernelGGL(counter_add_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, counter, delta);
    return check_hip(hipGetLastError(), "counter_add_kernel launch");
}

extern "C" int dvgo_grid_adam_step(float *param, float *grad, float *exp_avg, float *exp_avg_sq, int64_t n,
                                   float lr, float beta1, float beta2, float eps, int32_t step,
                                   const int32_t *step_dev, int32_t skip_zero_grad, int32_t zero_grad_after,
                                   void *stream) {
    if (n < 0) return set_error(DVGO_ERR_SHAPE, "negative n");
    if (n == 0) return DVGO_OK;
    if (!param || !grad || !exp_avg || !exp_avg_sq) return set_error(DVGO_ERR_NULL, "an Adam array is NULL");
    if (!step_dev && step < 1) return set_error(DVGO_ERR_RANGE, "step is 1-based");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f))
        return set_error(DVGO_ERR_RANGE, "betas must be in [0, 1)");
    const uintptr_t al = (uintptr_t)param & 15;
    if (((uintptr_t)grad & 15) != al || ((uintptr_t)exp_avg & 15) != al || ((uintptr_t)exp_avg_sq & 15) != al ||
        (al & 3))
        return set_error(DVGO_ERR_SHAPE, "param, grad and moments must share their 16-byte alignment");
    AdamArgs a;
    a.p = param;
    a.g = grad;
    a.m = exp_avg;
    a.v = exp_avg_sq;
    a.n = n;
    const int t = step_dev ? 1 : step;
    const double bc1 = 1.0 - pow((double)beta1, t), bc2 = 1.0 - pow((double)beta2, t);
    a.lr_t = (float)((double)lr / bc1);
    a.inv_sqrt_bc2 = (float)(1.0 / sqrt(bc2));
    a.lr = lr;
    a.step_dev = step_dev;
    a.b1 = beta1;
    a.b2 = beta2;
    a.eps = eps;
    a.skip = skip_zero_grad != 0;
    a.zero = zero_grad_after != 0;
    int64_t head = al ? (int64_t)((16 - al) / 4) : 0;
    if (head > n) head = n;
    const int64_t n4 = (n - head) / 4;
    const int blocks = grid_blocks(n4 > 0 ? n4 : n, kBlock);
    const int cap = 256 * 8;  // a few waves per CU; each thread streams many float4 groups
    hipLaunchKernelGGL(adam_kernel, dim3(blocks < cap ? blocks : cap), dim3(kBlock), 0, (hipStream_t)stream, a, head,
                       n4);
    return check_hip(hipGetLastError(), "adam_kernel launch");
}

extern "C" int dvgo_loss_head(int32_t n_rays, const float *rgb, const float *target, const float *dist,
                              float dist_weight, float *loss, float *grad_rgb, float *grad_dist, void *stream) {
    if (n_rays < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays");
    if (n_rays == 0) return DVGO_OK;
    if (!rgb || !target) return set_error(DVGO_ERR_NULL, "rgb or target is NULL");
    if (!loss && !grad_rgb && !grad_dist) return set_error(DVGO_ERR_NULL, "no output requested");
    if (!loss) {
        hipLaunchKernelGGL(loss_grad_kernel, dim3((unsigned)((n_rays + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                           n_rays, rgb, target, dist_weight, grad_rgb, grad_dist);
        return check_hip(hipGetLastError(), "loss_grad_kernel launch");
    }
    hipLaunchKernelGGL(loss_head_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, n_rays, rgb, target, dist,
                       dist_weight, loss, grad_rgb, grad_dist);
    return check_hip(hipGetLastError(), "loss_head_kernel launch");
}

// ------------------------------------------------------------------ total variation
//
// Gradient of the grid's total-variation regulariser (section 2, efficient TV loss), added
// straight into the gradient: for vertex p and channel c,
//     grad[p][c] += coef * sum over the (up to six) axis neighbours n of clamp(v[p][c] - v[n][c], -delta, delta)
// with coef = 2 weight / (N C).  Vector path (channels == ch_stride, a multiple of 4): G =
// channels / 4 lanes per vertex, each owning one float4 of the row, so every load of a wave
// is contiguous; floor(64 / G) vertices per wave.  Scalar path: one lane per vertex, channel
// loop.  Blocks are renumbered so that each XCD (blocks are dealt to the 8 XCDs round-robin)
// walks one contiguous slab of the grid and finds the x and y neighbour planes in its own L2.
// In sparse mode a vertex is updated only if some channel of its incoming gradient is
// non-zero; a lane reads and writes only its own vertex's gradient, so the test never sees
// another lane's update.
namespace {

constexpr int TV_BLOCK = 256, N_XCD = 8;

__device__ __forceinline__ int64_t xcd_block(int nblocks) {
    // hardware block b runs on XCD b % 8; give XCD k the logical range [k q, (k+1) q)
    const int q = (nblocks + N_XCD - 1) / N_XCD;
    return (int64_t)(blockIdx.x % N_XCD) * q + blockIdx.x / N_XCD;
}

template <bool VEC>
__global__ __launch_bounds__(TV_BLOCK) void tv_kernel(DevGrid g, float coef, float delta, int dense, int64_t nvert,
                                                     int nblocks) {
    const int64_t lb = xcd_block(nblocks);
    if (lb >= nblocks) return;  // whole block: padding of the renumbering
    const int G = VEC ? g.C / 4 : 1;            // lanes per vertex
    const int vpw = 64 / G;                     // vertices per wave
    const int ln = lane(), vl = ln / G, grp = ln - vl * G;
    const int64_t wave = lb * (TV_BLOCK / 64) + (threadIdx.x >> 6);
    const int64_t i = wave * vpw + vl;
    const bool live = vl < vpw && i < nvert;
    const int nz = g.n[2], ny = g.n[1], nx = g.n[0];
    const int z = live ? (int)(i % nz) : 0;
    const int64_t t = live ? i / nz : 0;
    const int y = (int)(t % ny), x = (int)(t / ny);
    const int64_t base = i * g.cs + 4 * grp;
    if (VEC) {
        float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
        if (live) q = *reinterpret_cast<const float4 *>(g.grad + base);
        if (!dense) {
            const bool nonzero = live && ((q.x != 0.f) | (q.y != 0.f) | (q.z != 0.f) | (q.w != 0.f));
            const unsigned long long b = __ballot(nonzero);  // every lane takes part
            const unsigned long long mine = ((1ull << G) - 1) << (vl * G);
            if (!(b & mine)) return;
        }
        if (!live) return;
        const float4 v = *reinterpret_cast<const float4 *>(g.data + base);
        const int64_t off[6] = {-(int64_t)g.sx, (int64_t)g.sx, -(int64_t)g.sy, (int64_t)g.sy, -(int64_t)g.cs,
                                (int64_t)g.cs};
        const bool ok[6] = {x > 0, x < nx - 1, y > 0, y < ny - 1, z > 0, z < nz - 1};
        float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            if (!ok[k]) continue;
            const float4 u = *reinterpret_cast<const float4 *>(g.data + base + off[k]);
            sum.x += fminf(fmaxf(v.x - u.x, -delta), delta);
            sum.y += fminf(fmaxf(v.y - u.y, -delta), delta);
            sum.z += fminf(fmaxf(v.z - u.z, -delta), delta);
            sum.w += fminf(fmaxf(v.w - u.w, -delta), delta);
        }
        q.x += coef * sum.x;
        q.y += coef * sum.y;
        q.z += coef * sum.z;
        q.w += coef * sum.w;
        *reinterpret_cast<float4 *>(g.grad + base) = q;
    } else {
        if (!live) return;
        float *gp = g.grad + i * g.cs;
        const float *vp = g.data + i * g.cs;
        if (!dense) {
            bool any = false;
            for (int c = 0; c < g.C; ++c) any |= gp[c] != 0.f;
            if (!any) return;
        }
        const int64_t off[6] = {-(int64_t)g.sx, (int64_t)g.sx, -(int64_t)g.sy, (int64_t)g.sy, -(int64_t)g.cs,
                                (int64_t)g.cs};
        const bool ok[6] = {x > 0, x < nx - 1, y > 0, y < ny - 1, z > 0, z < nz - 1};
        for (int c = 0; c < g.C; ++c) {
            const float v = vp[c];
            float sum = 0.f;
#pragma unroll
            for (int k = 0; k < 6; ++k)
                if (ok[k]) sum += fminf(fmaxf(v - vp[off[k] + c], -delta), delta);
            gp[c] += coef * sum;
        }
    }
}

}  // namespace

extern "C" int dvgo_tv_add_grad(const dvgo_grid *g, float weight, float delta, int32_t dense, void *stream) {
    DevGrid dg;
    int rc = make_dev_grid(g, "grid", &dg, true);
    if (rc) return rc;
    if (!(delta > 0.f)) return set_error(DVGO_ERR_RANGE, "delta must be > 0");
    const int64_t nvert = (int64_t)g->nx * g->ny * g->nz;
    const bool vec = g->channels == g->ch_stride && (g->ch_stride & 3) == 0;
    if (vec && (((uintptr_t)g->data | (uintptr_t)g->grad) & 15))
        return set_error(DVGO_ERR_SHAPE, "grid data and grad must be 16-byte aligned when ch_stride is a multiple of 4");
    const float coef = (float)(2.0 * (double)weight / ((double)nvert * g->channels));
    const int vpw = vec ? 64 / (g->ch_stride / 4) : 64;
    const int64_t waves = (nvert + vpw - 1) / vpw;
    const int nblocks = (int)((waves + TV_BLOCK / 64 - 1) / (TV_BLOCK / 64));
    const int launched = (nblocks + N_XCD - 1) / N_XCD * N_XCD;
    if (vec)
        hipLaunchKernelGGL(tv_kernel<true>, dim3(launched), dim3(TV_BLOCK), 0, (hipStream_t)stream, dg, coef, delta,
                           dense ? 1 : 0, nvert, nblocks);
    else
        hipLaunchKernelGGL(tv_kernel<false>, dim3(launched), dim3(TV_BLOCK), 0, (hipStream_t)stream, dg, coef, delta,
                           dense ? 1 : 0, nvert, nblocks);
    return check_hip(hipGetLastError(), "tv_kernel launch");
}

// ------------------------------------------------------------------ brick-binned scatter
//
// The scatter of per-sample values into a grid, re-organised so that the global atomics are
// few and coalesced.  Samples are binned by the 8^3-cell brick that holds their cell (a
// counting sort: counts, an exclusive prefix, placement); then one block per brick adds its
// samples' trilinear contributions into a 9^3-vertex LDS tile with LDS atomics and flushes the
// tile with one global atomic per touched vertex channel, consecutive lanes on consecutive
// addresses.  Consecutive samples lie along one ray and share a brick, so the counting passes
// aggregate each run of equal bricks in the wave into one atomic.

namespace {

constexpr int BRICK = 8;            // cells per brick edge
constexpr int BV = BRICK + 1;       // vertices per brick edge
constexpr int BIN_WAVES = 4;

struct BinGeom {
    int nb[3];  // bricks per axis
    int n;      // bricks
};

BinGeom bin_geom(const DevGrid &g) {
    BinGeom b;
    b.n = 1;
    for (int a = 0; a < 3; ++a) {
        b.nb[a] = (g.n[a] - 1 + BRICK - 1) / BRICK;
        b.n *= b.nb[a];
    }
    return b;
}

__device__ __forceinline__ int brick_of(const BinGeom &b, const Cell &c) {
    return ((c.ix / BRICK) * b.nb[1] + c.iy / BRICK) * b.nb[2] + c.iz / BRICK;
}

struct BinWs {
    int *offs;    // [n + 1] first slot of each brick in perm
    int *cursor;  // [n] counts, then placement cursors
    int *perm;    // [S] sample indices grouped by brick
};

size_t bin_bytes(int nb, int64_t S, size_t *o_cursor, size_t *o_perm) {
    size_t o = align_up((size_t)(nb + 1) * 4, 256);
    *o_cursor = o;
    o += align_up((size_t)nb * 4, 256);
    *o_perm = o;
    o += (size_t)S * 4;
    return o;
}

__global__ __launch_bounds__(256) void bin_zero_kernel(int *p, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}

template <bool W>
__global__ __launch_bounds__(64 * BIN_WAVES) void bin_count_kernel(DevGrid g, BinGeom bg, int64_t S,
                                                                 const float *__restrict__ xyz, int *cnt) {
    const int64_t nwaves = (int64_t)gridDim.x * BIN_WAVES;
    for (int64_t base = (int64_t)(blockIdx.x * BIN_WAVES + (threadIdx.x >> 6)) * 64; base < S; base += nwaves * 64) {
        const int64_t k = base + lane();
        int key = -1;
        if (k < S) key = brick_of(bg, cell_of<W>(g, xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2]));
        const Run run = wave_runs(key);
        if (run.head) atomicAdd(&cnt[key], run.len);
    }
}

// offs = exclusive prefix of cnt (one block); cnt is reset to zero for the placement cursors
__global__ __launch_bounds__(1024) void bin_scan_kernel(int n, int *cnt, int *offs) {
    __shared__ int wsum[16];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int i = base + threadIdx.x;
        const int c = i < n ? cnt[i] : 0;
        int v = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(v, d, 64);
            if (lane() >= d) v += t;
        }
        if (lane() == 63) wsum[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x < 16) {
            int w = wsum[threadIdx.x];
#pragma unroll
            for (int d = 1; d < 16; d <<= 1) {
                const int t = __shfl_up(w, d, 16);
                if ((int)threadIdx.x >= d) w += t;
            }
            wsum[threadIdx.x] = w;
        }
        __syncthreads();
        const int below = (threadIdx.x >> 6) ? wsum[(threadIdx.x >> 6) - 1] : 0;
        if (i < n) {
            offs[i] = carry + below + v - c;
            cnt[i] = 0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            carry += wsum[15];
            if (base + 1024 >= n) offs[n] = carry;
        }
        __syncthreads();
    }
    if (n == 0 && threadIdx.x == 0) offs[0] = 0;
}

template <bool W>
__global__ __launch_bounds__(64 * BIN_WAVES) void bin_place_kernel(DevGrid g, BinGeom bg, int64_t S,
                                                                 const float *__restrict__ xyz, const int *offs,
                                                                 int *cursor, int *perm) {
    const int64_t nwaves = (int64_t)gridDim.x * BIN_WAVES;
    for (int64_t base = (int64_t)(blockIdx.x * BIN_WAVES + (threadIdx.x >> 6)) * 64; base < S; base += nwaves * 64) {
        const int64_t k = base + lane();
        int key = -1;
        if (k < S) key = brick_of(bg, cell_of<W>(g, xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2]));
        const Run run = wave_runs(key);
        int start = 0;
        if (run.head) start = atomicAdd(&cursor[key], run.len);
        start = __shfl(start, run.head_lane, 64);
        if (key >= 0) perm[offs[key] + start + (lane() - run.head_lane)] = (int)k;
    }
}

// One block per brick: LDS tile of BV^3 vertices x NC channels, channel-major with a padded
// plane (TPL floats) so that the lanes of one LDS atomic, which hold different vertices of
// one channel, spread over the banks.  Thread = (sample, corner).
constexpr int TPL = BV * BV * BV + 8;  // 737: odd stride between channel planes

template <int NC, bool W>
__global__ __launch_bounds__(256) void brick_scatter_kernel(DevGrid g, BinGeom bg, const float *__restrict__ xyz,
                                                            const float *__restrict__ vals, const int *offs,
                                                            const int *perm) {
    __shared__ float tile[TPL * NC];
    const int b = blockIdx.x;
    const int beg = offs[b], end = offs[b + 1];
    if (beg == end) return;
    const int bz = b % bg.nb[2], by = (b / bg.nb[2]) % bg.nb[1], bx = b / (bg.nb[2] * bg.nb[1]);
    const int x0 = bx * BRICK, y0 = by * BRICK, z0 = bz * BRICK;
    for (int i = threadIdx.x; i < TPL * NC; i += 256) tile[i] = 0.f;
    __syncthreads();
    // thread = sample: every sample of the brick has its loads in flight at once
    for (int i = beg + threadIdx.x; i < end; i += 256) {
        const int s = perm[i];
        const Cell c = cell_of<W>(g, xyz[3 * (int64_t)s], xyz[3 * (int64_t)s + 1], xyz[3 * (int64_t)s + 2]);
        const float *src = vals + (int64_t)s * g.C;
        float val[NC];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) val[ch] = ch < g.C ? src[ch] : 0.f;
        const int v0 = ((c.ix - x0) * BV + (c.iy - y0)) * BV + (c.iz - z0);
#pragma unroll
        for (int corner = 0; corner < 8; ++corner) {
            const int dx = (corner >> 2) & 1, dy = (corner >> 1) & 1, dz = corner & 1;
            const float w = corner_weight(c, dx, dy, dz);
            const int v = v0 + (dx * BV + dy) * BV + dz;
#pragma unroll
            for (int ch = 0; ch < NC; ++ch)
                if (ch < g.C) atomicAdd(&tile[ch * TPL + v], w * val[ch]);
        }
    }
    __syncthreads();
    // flush in memory order (channel fastest) so consecutive lanes hit consecutive addresses
    for (int i = threadIdx.x; i < BV * BV * BV * NC; i += 256) {
        const int v = i / NC, ch = i - v * NC;
        const float t = tile[ch * TPL + v];
        if (t == 0.f) continue;
        const int lz = v % BV, ly = (v / BV) % BV, lx = v / (BV * BV);
        const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        if (gx < g.n[0] && gy < g.n[1] && gz < g.n[2])
            unsafeAtomicAdd(g.grad + (int64_t)gx * g.sx + (int64_t)gy * g.sy + (int64_t)gz * g.cs + ch, t);
    }
}

template <int NC>
void launch_brick_scatter(const DevGrid &dg, const BinGeom &bg, const float *xyz, const float *vals, const BinWs &w,
                          hipStream_t st) {
    if (dg.warp)
        hipLaunchKernelGGL((brick_scatter_kernel<NC, true>), dim3(bg.n), dim3(256), 0, st, dg, bg, xyz, vals, w.offs,
                           w.perm);
    else
        hipLaunchKernelGGL((brick_scatter_kernel<NC, false>), dim3(bg.n), dim3(256), 0, st, dg, bg, xyz, vals,
                           w.offs, w.perm);
}

int bin_setup(const dvgo_grid *g, int64_t S, const void *ws, size_t ws_bytes, DevGrid &dg, BinGeom &bg, BinWs &w,
              bool need_grad) {
    int rc = make_dev_grid(g, "grid", &dg, need_grad);
    if (rc) return rc;
    if (S < 0) return set_error(DVGO_ERR_SHAPE, "negative n_samples");
    if (S >= ((int64_t)1 << 31)) return set_error(DVGO_ERR_RANGE, "n_samples must be below 2^31");
    bg = bin_geom(dg);
    size_t oc, op;
    const size_t need = bin_bytes(bg.n, S, &oc, &op);
    if (!ws || ws_bytes < need) return set_error(DVGO_ERR_WORKSPACE, "bin workspace too small (%zu < %zu)", ws_bytes, need);
    if (((uintptr_t)ws & 255) != 0) return set_error(DVGO_ERR_SHAPE, "bin workspace must be 256-byte aligned");
    w.offs = (int *)ws;
    w.cursor = (int *)((char *)ws + oc);
    w.perm = (int *)((char *)ws + op);
    return DVGO_OK;
}

int bin_blocks(int64_t S) {
    const int64_t b = (S + 64 * BIN_WAVES - 1) / (64 * BIN_WAVES);
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

extern "C" int dvgo_bin_workspace_size(const dvgo_grid *g, int64_t n_samples, size_t *bytes) {
    DevGrid dg;
    int rc = make_dev_grid(g, "grid", &dg, false);
    if (rc) return rc;
    if (!bytes) return set_error(DVGO_ERR_NULL, "bytes is NULL");
    if (n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative n_samples");
    size_t a, b;
    *bytes = bin_bytes(bin_geom(dg).n, n_samples, &a, &b);
    return DVGO_OK;
}

extern "C" int dvgo_bin_samples(const dvgo_grid *g, int64_t n_samples, const float *xyz, void *ws, size_t ws_bytes,
                                void *stream) {
    DevGrid dg;
    BinGeom bg;
    BinWs w;
    int rc = bin_setup(g, n_samples, ws, ws_bytes, dg, bg, w, false);
    if (rc) return rc;
    if (n_samples > 0 && !xyz) return set_error(DVGO_ERR_NULL, "xyz is NULL");
    const hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(bin_zero_kernel, dim3((bg.n + 255) / 256 < 1024 ? (bg.n + 255) / 256 : 1024), dim3(256), 0, st,
                       w.cursor, bg.n);
    const int nb = bin_blocks(n_samples);
    if (n_samples > 0) {
        if (dg.warp)
            hipLaunchKernelGGL(bin_count_kernel<true>, dim3(nb), dim3(64 * BIN_WAVES), 0, st, dg, bg, n_samples, xyz,
                               w.cursor);
        else
            hipLaunchKernelGGL(bin_count_kernel<false>, dim3(nb), dim3(64 * BIN_WAVES), 0, st, dg, bg, n_samples, xyz,
                               w.cursor);
    }
    hipLaunchKernelGGL(bin_scan_kernel, dim3(1), dim3(1024), 0, st, bg.n, w.cursor, w.offs);
    if (n_samples > 0) {
        if (dg.warp)
            hipLaunchKernelGGL(bin_place_kernel<true>, dim3(nb), dim3(64 * BIN_WAVES), 0, st, dg, bg, n_samples, xyz,
                               w.offs, w.cursor, w.perm);
        else
            hipLaunchKernelGGL(bin_place_kernel<false>, dim3(nb), dim3(64 * BIN_WAVES), 0, st, dg, bg, n_samples, xyz,
                               w.offs, w.cursor, w.perm);
    }
    return check_hip(hipGetLastError(), "bin kernels launch");
}

extern "C" int dvgo_grid_scatter_binned(const dvgo_grid *g, int64_t n_samples, const float *xyz, const float *grad_out,
                                        const void *ws, size_t ws_bytes, void *stream) {
    DevGrid dg;
    BinGeom bg;
    BinWs w;
    int rc = bin_setup(g, n_samples, ws, ws_bytes, dg, bg, w, true);
    if (rc) return rc;
    if (n_samples == 0) return DVGO_OK;
    if (!xyz || !grad_out) return set_error(DVGO_ERR_NULL, "xyz or grad_out is NULL");
    const hipStream_t st = (hipStream_t)stream;
    const int C = g->channels;
    if (C == 1) launch_brick_scatter<1>(dg, bg, xyz, grad_out, w, st);
    else if (C <= 3) launch_brick_scatter<3>(dg, bg, xyz, grad_out, w, st);
    else if (C <= 4) launch_brick_scatter<4>(dg, bg, xyz, grad_out, w, st);
    else if (C <= 8) launch_brick_scatter<8>(dg, bg, xyz, grad_out, w, st);
    else if (C <= 12) launch_brick_scatter<12>(dg, bg, xyz, grad_out, w, st);
    else launch_brick_scatter<16>(dg, bg, xyz, grad_out, w, st);
    return check_hip(hipGetLastError(), "brick_scatter_kernel launch");
}

// ------------------------------------------------------------------ grid resampling

namespace {

// out vertex (i, j, k) of an (mx, my, mz) grid over the same box = trilinear value of the
// source at that vertex's position; positions in double, rounded to float32 like any point
__global__ __launch_bounds__(256) void resample_kernel(DevGrid g, int mx, int my, int mz, double lo0, double lo1,
                                                       double lo2, double st0, double st1, double st2,
                                                       float *__restrict__ out) {
    const int64_t n = (int64_t)mx * my * mz;
    for (int64_t v = blockIdx.x * (int64_t)256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
        const int k = (int)(v % mz), j = (int)((v / mz) % my), i = (int)(v / ((int64_t)my * mz));
        const float x = (float)(lo0 + (double)i * st0), y = (float)(lo1 + (double)j * st1),
                    z = (float)(lo2 + (double)k * st2);
        const Tri t = trilinear<false>(g, x, y, z);
        for (int ch = 0; ch < g.cs; ++ch) out[v * g.cs + ch] = ch < g.C ? interp_ch(g, t, ch) : 0.f;
    }
}

}  // namespace

extern "C" int dvgo_grid_resample(const dvgo_grid *src, int32_t nx, int32_t ny, int32_t nz, float *out,
                                  void *stream) {
    DevGrid dg;
    int rc = make_dev_grid(src, "source grid", &dg, false);
    if (rc) return rc;
    if (nx < 2 || ny < 2 || nz < 2) return set_error(DVGO_ERR_SHAPE, "every output dimension must be >= 2");
    if ((int64_t)nx * ny * nz * src->ch_stride >= ((int64_t)1 << 31))
        return set_error(DVGO_ERR_RANGE, "output grid has >= 2^31 floats");
    if (!out) return set_error(DVGO_ERR_NULL, "out is NULL");
    dg.warp = DVGO_WARP_NONE;  // vertices are addressed in the grid's own box
    const double lo[3] = {src->xyz_min[0], src->xyz_min[1], src->xyz_min[2]};
    const double hi[3] = {src->xyz_max[0], src->xyz_max[1], src->xyz_max[2]};
    const int m[3] = {nx, ny, nz};
    double st[3];
    for (int a = 0; a < 3; ++a) st[a] = (hi[a] - lo[a]) / (double)(m[a] - 1);
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t blocks = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
    hipLaunchKernelGGL(resample_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, dg, nx, ny, nz,
                       lo[0], lo[1], lo[2], st[0], st[1], st[2], out);
    return check_hip(hipGetLastError(), "resample_kernel launch");
}
