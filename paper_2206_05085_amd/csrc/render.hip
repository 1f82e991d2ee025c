// Volume rendering forward/backward and the O(N) distortion loss on ragged rays (gfx950).
//
// One wavefront owns one ray and walks it in chunks of 64 samples (one sample per lane).
// Within a chunk every prefix quantity is a wave64 scan; across chunks a carry is kept.
//   forward : log-transmittance L (exclusive scan of sigma*delta), the weight prefix W,
//             and the distortion prefix Q; colour and distortion are reduced per lane.
//   backward: chunks are visited last-to-first.  Prefix state is restored from a per-chunk
//             checkpoint (L, W, Q) written by the forward, suffix state (sum of later
//             weights, Q', and the sum of later g*w) is carried from the chunk after.
//
// Distortion (section 2).  Eq. 1's first term equals 2 sum_i w_i Q_i with
//   Q_i = sum_{j<i} w_j (m_i - m_j),  Q_{i+1} = Q_i + W_{<=i} (m_{i+1} - m_i),
// which is Eq. 2's prefix-sum rewrite arranged so that every added term is non-negative
// (midpoints are sorted), i.e. free of the cancellation between m_i P_i and PM_i that the
// literal form of Eq. 2 suffers in float32.  Its derivative (Eq. 3, plus the derivative of
// the second term of Eq. 1) is
//   dD/dw_k = 2 (Q_k + Q'_k) + (2/3) w_k l_k,   Q'_k = sum_{i>k} w_i (m_i - m_k),
// with the suffix recurrence Q'_k = Q'_{k+1} + (m_{k+1} - m_k) W_{>k}.
//
// Compositing backward.  With g_k = dL/dC . c_k + dL/dD dD/dw_k:
//   dL/dx_k = T_{k+1} g_k - S_k,   S_k = sum_{i>k} g_i w_i + (dL/dC . bg + dL/dT_N) T_N,
//   dL/draw_k = dL/dx_k * delta_k * sigmoid(raw_k + b),   dL/dc_k = w_k dL/dC.
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <tuple>

#include "dvgo_internal.h"

using namespace dvgo;

namespace {

struct RenderArgs {
    int n_rays;
    const int *offs;
    const float *xyz, *delta, *s_mid, *s_len;
    DevGrid dens, col;
    const float *srgb;
    float act_shift, halt_T, bg0, bg1, bg2;
    int want_dist;
    // forward outputs / saved state
    float *rgb, *T_final, *dist, *sample_w;
    int *halt_idx;
    float4 *ckpt;
    float *raw_saved;  // each sample's interpolated density logit, written by the forward
    // backward
    const float *T_in, *grad_rgb, *grad_dist, *grad_T;
    const float *target;  // fused forward + loss + backward: per-ray target colours and the
    float lam;            // distortion weight of the loss
    float *grad_srgb;
    float *grad_raw;  // per-sample density-logit gradient (written instead of the density scatter)
    // schedule: rays ray_list[0..n_list) (identity when NULL), taken by the waves of the grid
    // in turn (wave i handles entries i, i + n_waves, ...)
    const int *ray_list;
    int n_list;
};

// the wave's share of the ray list; every lane of a wave sees the same sequence
#define FOR_EACH_RAY(a, r)                                                                              \
    for (int _i = blockIdx.x * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6),                        \
             _nw = (int)gridDim.x * (int)(blockDim.x >> 6);                                               \
         _i < (a).n_list; _i += _nw)                                                                      \
        for (int r = (a).ray_list ? (a).ray_list[_i] : _i, _once = 1; _once; _once = 0)

struct SampleIn {
    float raw, c0, c1, c2, x, alpha, m, mn, l, delta;
    Cell cd, cc;  // cells of the density and colour grids
};

__device__ __forceinline__ void zero_sample(SampleIn &s) {
    s.x = s.alpha = s.m = s.mn = s.l = s.c0 = s.c1 = s.c2 = s.delta = s.raw = 0.f;
    s.cd = Cell{0, 0, 0, 0.f, 0.f, 0.f};
    s.cc = s.cd;
}

template <int MODE, bool WARP>
__device__ __forceinline__ void load_sample(const RenderArgs &a, int k, bool has_next, SampleIn &s) {
    const float px = a.xyz[3 * k], py = a.xyz[3 * k + 1], pz = a.xyz[3 * k + 2];
    s.cd = cell_of<WARP>(a.dens, px, py, pz);
    s.raw = interp_ch(a.dens, tri_from_cell(a.dens, s.cd), 0);
    if (MODE == DVGO_COLOR_GRID) {
        s.cc = cell_of<WARP>(a.col, px, py, pz);
        const Tri tc = tri_from_cell(a.col, s.cc);
        s.c0 = interp_ch(a.col, tc, 0);
        s.c1 = interp_ch(a.col, tc, 1);
        s.c2 = interp_ch(a.col, tc, 2);
    } else if (MODE == DVGO_COLOR_SAMPLES) {
        s.c0 = a.srgb[3 * k];
        s.c1 = a.srgb[3 * k + 1];
        s.c2 = a.srgb[3 * k + 2];
    } else {
        s.c0 = s.c1 = s.c2 = 0.f;
    }
    s.delta = a.delta[k];
    s.x = softplusf(s.raw + a.act_shift) * s.delta;
    s.alpha = -expm1f(-s.x);
    s.m = a.s_mid[k];
    s.l = a.s_len[k];
    s.mn = has_next ? a.s_mid[k + 1] : 0.f;
}

// The backward's loader: the density logit comes from the forward's saved copy (no density
// lookup), and the optical depth and alpha follow from it exactly as in the forward.  The
// points are read only where a cell is still needed: the colour grid's lookup and scatter, or
// the density scatter inside the kernel.
template <int MODE, bool WARP>
__device__ __forceinline__ void load_sample_bwd(const RenderArgs &a, int k, bool has_next, SampleIn &s) {
    s.raw = a.raw_saved[k];
    if (MODE == DVGO_COLOR_GRID || !a.grad_raw) {
        const float px = a.xyz[3 * k], py = a.xyz[3 * k + 1], pz = a.xyz[3 * k + 2];
        if (!a.grad_raw) s.cd = cell_of<WARP>(a.dens, px, py, pz);
        if (MODE == DVGO_COLOR_GRID) {
            s.cc = cell_of<WARP>(a.col, px, py, pz);
            const Tri tc = tri_from_cell(a.col, s.cc);
            s.c0 = interp_ch(a.col, tc, 0);
            s.c1 = interp_ch(a.col, tc, 1);
            s.c2 = interp_ch(a.col, tc, 2);
        }
    }
    if (MODE == DVGO_COLOR_SAMPLES) {
        s.c0 = a.srgb[3 * k];
        s.c1 = a.srgb[3 * k + 1];
        s.c2 = a.srgb[3 * k + 2];
    } else if (MODE != DVGO_COLOR_GRID) {
        s.c0 = s.c1 = s.c2 = 0.f;
    }
    s.delta = a.delta[k];
    s.x = softplusf(s.raw + a.act_shift) * s.delta;
    s.alpha = -expm1f(-s.x);
    s.m = a.s_mid[k];
    s.l = a.s_len[k];
    s.mn = has_next ? a.s_mid[k + 1] : 0.f;
}

// What the forward of one ray leaves in registers (the same in every lane, and the values it
// stores): colour, final transmittance, halt index.
struct RayFwd {
    float c0, c1, c2, TN;
    int halt;
};

// The backward's per-ray inputs: upstream gradients of colour, distortion and final
// transmittance, the forward's final transmittance and halt index.
struct RayGrad {
    float g0, g1, g2, gD, gT, T_in;
    int hend;
};

template <int MODE, bool WARP>
__device__ __forceinline__ RayFwd render_fwd_ray(const RenderArgs &a, int r) {
    const int ln = lane();
    const int beg = a.offs[r], end = a.offs[r + 1];
    float L = 0.f, W = 0.f, Q = 0.f;
    float accC0 = 0.f, accC1 = 0.f, accC2 = 0.f, accD = 0.f;
    int halt = end;
    float T_halt = 1.f;
    int64_t ck = ckpt_slot(beg, r, beg);
    for (int c0 = beg; c0 < end; c0 += 64, ++ck) {
        if (ln == 0) a.ckpt[ck] = make_float4(L, W, Q, 0.f);
        const int k = c0 + ln;
        const bool valid = k < end;
        const bool has_next = k + 1 < end;
        SampleIn s;
        if (valid) {
            load_sample<MODE, WARP>(a, k, has_next, s);
            a.raw_saved[k] = s.raw;
        } else {
            zero_sample(s);
        }
        const float xi = wave_incl(s.x);
        const float T = expf(-(L + wave_excl(xi)));
        if (a.halt_T > 0.f) {
            const unsigned long long hm = __ballot(valid && T < a.halt_T);
            if (hm) {
                const int f = __ffsll(hm) - 1;
                halt = c0 + f;
                T_halt = bcast(T, f);
            }
        }
        const bool live = valid && k < halt;
        const float w = live ? T * s.alpha : 0.f;
        if (a.sample_w && valid) a.sample_w[k] = w;
        const float wi = wave_incl(w);
        const float u = (live && has_next) ? (W + wi) * (s.mn - s.m) : 0.f;
        const float ui = wave_incl(u);
        const float Qk = Q + wave_excl(ui);
        accD += w * (2.f * Qk + w * s.l * (1.f / 3.f));
        accC0 += w * s.c0;
        accC1 += w * s.c1;
        accC2 += w * s.c2;
        L += bcast(xi, 63);
        W += bcast(wi, 63);
        Q += bcast(ui, 63);
        if (halt < end) {
            if (a.sample_w)
                for (int kk = c0 + 64 + ln; kk < end; kk += 64) a.sample_w[kk] = 0.f;
            break;
        }
    }
    // the butterfly sums may differ in the last bit between lanes: lane 0's are the results
    const float TN = halt < end ? T_halt : expf(-L);
    RayFwd f;
    f.c0 = bcast(wave_sum(accC0), 0) + TN * a.bg0;
    f.c1 = bcast(wave_sum(accC1), 0) + TN * a.bg1;
    f.c2 = bcast(wave_sum(accC2), 0) + TN * a.bg2;
    f.TN = TN;
    f.halt = halt;
    accD = wave_sum(accD);
    if (ln == 0) {
        a.rgb[3 * r] = f.c0;
        a.rgb[3 * r + 1] = f.c1;
        a.rgb[3 * r + 2] = f.c2;
        a.T_final[r] = TN;
        if (a.want_dist) a.dist[r] = accD;
        a.halt_idx[r] = halt;
    }
    return f;
}

template <int MODE, bool WARP>
__global__ __launch_bounds__(1024) void render_fwd_kernel(RenderArgs a) {
    FOR_EACH_RAY(a, r) render_fwd_ray<MODE, WARP>(a, r);
}

template <int MODE, bool WARP>
__device__ __forceinline__ void render_bwd_ray(const RenderArgs &a, int r, const RayGrad &in) {
    const int ln = lane();
    const int beg = a.offs[r], end = a.offs[r + 1];
    const int hend = in.hend;
    const float g0 = in.g0, g1 = in.g1, g2 = in.g2, gD = in.gD;
    float Scar = (g0 * a.bg0 + g1 * a.bg1 + g2 * a.bg2 + in.gT) * in.T_in;
    float Wgt = 0.f, Qp = 0.f;
    if (MODE == DVGO_COLOR_SAMPLES) {
        for (int k = hend + ln; k < end; k += 64) {
            a.grad_srgb[3 * k] = 0.f;
            a.grad_srgb[3 * k + 1] = 0.f;
            a.grad_srgb[3 * k + 2] = 0.f;
        }
    }
    if (a.grad_raw)
        for (int k = hend + ln; k < end; k += 64) a.grad_raw[k] = 0.f;
    if (hend <= beg) return;
    const int nch = (hend - beg + 63) / 64;
    const float b = a.act_shift;
    for (int ci = nch - 1; ci >= 0; --ci) {
        const int c0 = beg + ci * 64;
        const float4 cp = a.ckpt[ckpt_slot(beg, r, c0)];
        const int k = c0 + ln;
        const bool valid = k < hend;
        const bool has_next = k + 1 < hend;
        SampleIn s;
        zero_sample(s);
        if (valid) load_sample_bwd<MODE, WARP>(a, k, has_next, s);
        const float xi = wave_incl(s.x);
        const float T = expf(-(cp.x + wave_excl(xi)));
        const float Tn = expf(-(cp.x + xi));
        const float w = valid ? T * s.alpha : 0.f;
        const float wi = wave_incl(w);
        const float u = (valid && has_next) ? (cp.y + wi) * (s.mn - s.m) : 0.f;
        const float Qk = cp.z + wave_excl(wave_incl(u));
        const float wr = wave_incl_rev(w);
        const float wgt = Wgt + wave_excl_rev(wr);
        const float v = (valid && has_next) ? (s.mn - s.m) * wgt : 0.f;
        const float Qpk = Qp + wave_incl_rev(v);
        float g = g0 * s.c0 + g1 * s.c1 + g2 * s.c2;
        if (gD != 0.f) g += gD * (2.f * (Qk + Qpk) + (2.f / 3.f) * w * s.l);
        const float gwr = wave_incl_rev(g * w);
        const float Sk = Scar + wave_excl_rev(gwr);
        const float draw = valid ? (Tn * g - Sk) * s.delta * sigmoidf(s.raw + b) : 0.f;
        if (a.grad_raw) {
            if (valid) a.grad_raw[k] = draw;
        } else {
            const float dd[1] = {draw};
            scatter_wave<1>(a.dens, valid, s.cd, dd);
        }
        if (MODE == DVGO_COLOR_GRID) {
            const float dc[3] = {w * g0, w * g1, w * g2};
            scatter_wave<3>(a.col, valid, s.cc, dc);
        } else if (valid) {
            a.grad_srgb[3 * k] = w * g0;
            a.grad_srgb[3 * k + 1] = w * g1;
            a.grad_srgb[3 * k + 2] = w * g2;
        }
        Wgt += bcast(wr, 0);
        Qp = bcast(Qpk, 0);
        Scar += bcast(gwr, 0);
    }
}

template <int MODE, bool WARP>
__global__ __launch_bounds__(1024) void render_bwd_kernel(RenderArgs a) {
    FOR_EACH_RAY(a, r) {
        RayGrad in;
        in.hend = a.halt_idx[r];
        in.g0 = a.grad_rgb[3 * r];
        in.g1 = a.grad_rgb[3 * r + 1];
        in.g2 = a.grad_rgb[3 * r + 2];
        in.gD = a.grad_dist ? a.grad_dist[r] : 0.f;
        in.gT = a.grad_T ? a.grad_T[r] : 0.f;
        in.T_in = a.T_in[r];
        render_bwd_ray<MODE, WARP>(a, r, in);
    }
}

// Forward, loss gradient and backward of each ray in one pass of its wave.  The loss is the
// training loss of the step, L = sum_r |rgb_r - target_r|^2 / (3 R) + lam sum_r dist_r / R
// (photometric MSE plus the weighted distortion of section 2), whose gradient for ray r needs
// only that ray's colour: dL/drgb_r = 2 (rgb_r - target_r) / (3 R), dL/ddist_r = lam / R.
// The backward then reads the checkpoints and density logits this wave has just stored.
template <int MODE, bool WARP>
__global__ __launch_bounds__(1024) void render_train_kernel(RenderArgs a) {
    const float inv3R = 1.f / (3.f * (float)a.n_rays), invR = 1.f / (float)a.n_rays;
    FOR_EACH_RAY(a, r) {
        const RayFwd f = render_fwd_ray<MODE, WARP>(a, r);
        RayGrad in;
        in.g0 = 2.f * (f.c0 - a.target[3 * r]) * inv3R;
        in.g1 = 2.f * (f.c1 - a.target[3 * r + 1]) * inv3R;
        in.g2 = 2.f * (f.c2 - a.target[3 * r + 2]) * inv3R;
        in.gD = a.want_dist ? a.lam * invR : 0.f;
        in.gT = 0.f;
        in.T_in = f.TN;
        in.hend = f.halt;
        // the other lanes' stores of this wave (checkpoints, logits) complete before the reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        render_bwd_ray<MODE, WARP>(a, r, in);
    }
}

// Standalone distortion loss on given weights; forward sweep, then (if requested) a
// reverse sweep that reads the chunk checkpoints this same wave wrote.
__global__ __launch_bounds__(256) void distortion_kernel(int n_rays, const int *offs, const float *wv,
                                                         const float *mv, const float *lv, float *loss,
                                                         const float *gl, float *gw, float2 *ckpt) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n_rays) return;
    const int ln = lane();
    const int beg = offs[r], end = offs[r + 1];
    const bool bwd = gw != nullptr;
    float W = 0.f, Q = 0.f, accD = 0.f;
    int64_t ck = ckpt_slot(beg, r, beg);
    for (int c0 = beg; c0 < end; c0 += 64, ++ck) {
        if (bwd && ln == 0) ckpt[ck] = make_float2(W, Q);
        const int k = c0 + ln;
        const bool valid = k < end, has_next = k + 1 < end;
        const float w = valid ? wv[k] : 0.f;
        const float m = valid ? mv[k] : 0.f;
        const float mn = has_next ? mv[k + 1] : 0.f;
        const float l = valid ? lv[k] : 0.f;
        const float wi = wave_incl(w);
        const float u = has_next ? (W + wi) * (mn - m) : 0.f;
        const float ui = wave_incl(u);
        const float Qk = Q + wave_excl(ui);
        accD += w * (2.f * Qk + w * l * (1.f / 3.f));
        W += bcast(wi, 63);
        Q += bcast(ui, 63);
    }
    accD = wave_sum(accD);
    if (loss && ln == 0) loss[r] = accD;
    if (!bwd || end <= beg) return;
    __threadfence_block();
    const float gD = gl[r];
    float Wgt = 0.f, Qp = 0.f;
    const int nch = (end - beg + 63) / 64;
    for (int ci = nch - 1; ci >= 0; --ci) {
        const int c0 = beg + ci * 64;
        const float2 cp = ckpt[ckpt_slot(beg, r, c0)];
        const int k = c0 + ln;
        const bool valid = k < end, has_next = k + 1 < end;
        const float w = valid ? wv[k] : 0.f;
        const float m = valid ? mv[k] : 0.f;
        const float mn = has_next ? mv[k + 1] : 0.f;
        const float l = valid ? lv[k] : 0.f;
        const float wi = wave_incl(w);
        const float u = has_next ? (cp.x + wi) * (mn - m) : 0.f;
        const float Qk = cp.y + wave_excl(wave_incl(u));
        const float wr = wave_incl_rev(w);
        const float wgt = Wgt + wave_excl_rev(wr);  // every lane must join the shuffle
        const float v = has_next ? (mn - m) * wgt : 0.f;
        const float Qpk = Qp + wave_incl_rev(v);
        if (valid) gw[k] += gD * (2.f * (Qk + Qpk) + (2.f / 3.f) * w * l);
        Wgt += bcast(wr, 0);
        Qp = bcast(Qpk, 0);
    }
}

int check_samples(const dvgo_samples *s) {
    if (!s) return set_error(DVGO_ERR_NULL, "samples is NULL");
    if (s->struct_size != sizeof(dvgo_samples)) return set_error(DVGO_ERR_ABI, "dvgo_samples.struct_size mismatch");
    if (s->n_rays < 0 || s->n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays or n_samples");
    if (s->n_samples > MAX_SAMPLES)
        return set_error(DVGO_ERR_RANGE, "n_samples must be at most %lld", (long long)MAX_SAMPLES);
    if (!s->ray_offsets) return set_error(DVGO_ERR_NULL, "ray_offsets is NULL");
    if (s->n_samples > 0 && (!s->xyz || !s->delta || !s->s_mid || !s->s_len))
        return set_error(DVGO_ERR_NULL, "a per-sample array is NULL");
    return DVGO_OK;
}

int fill_render_args(const dvgo_render_params *p, const dvgo_samples *s, const dvgo_grid *density,
                     const dvgo_grid *color, const float *sample_rgb, bool bwd, RenderArgs &a,
                     bool density_grad = true) {
    if (!p) return set_error(DVGO_ERR_NULL, "params is NULL");
    if (p->struct_size != sizeof(dvgo_render_params))
        return set_error(DVGO_ERR_ABI, "dvgo_render_params.struct_size mismatch");
    int rc = check_samples(s);
    if (rc) return rc;
    if (p->color_mode != DVGO_COLOR_GRID && p->color_mode != DVGO_COLOR_SAMPLES && p->color_mode != DVGO_COLOR_NONE)
        return set_error(DVGO_ERR_UNSUPPORTED, "unknown color_mode %d", p->color_mode);
    if (bwd && p->color_mode == DVGO_COLOR_NONE)
        return set_error(DVGO_ERR_UNSUPPORTED, "DVGO_COLOR_NONE is forward only");
    if (!(p->halt_T >= 0.f && p->halt_T < 1.f)) return set_error(DVGO_ERR_RANGE, "halt_T must be in [0, 1)");
    memset(&a, 0, sizeof(a));
    rc = make_dev_grid(density, "density", &a.dens, bwd && density_grad);
    if (rc) return rc;
    if (p->color_mode == DVGO_COLOR_GRID) {
        if (!color) return set_error(DVGO_ERR_NULL, "color grid is NULL in DVGO_COLOR_GRID mode");
        rc = make_dev_grid(color, "color", &a.col, bwd);
        if (rc) return rc;
        if (color->channels < 3) return set_error(DVGO_ERR_SHAPE, "color grid needs 3 channels");
    } else if (p->color_mode == DVGO_COLOR_SAMPLES && s->n_samples > 0 && !sample_rgb) {
        return set_error(DVGO_ERR_NULL, "sample_rgb is NULL in DVGO_COLOR_SAMPLES mode");
    }
    a.n_rays = s->n_rays;
    a.offs = s->ray_offsets;
    a.xyz = s->xyz;
    a.delta = s->delta;
    a.s_mid = s->s_mid;
    a.s_len = s->s_len;
    a.srgb = sample_rgb;
    a.act_shift = p->act_shift;
    a.halt_T = p->halt_T;
    a.bg0 = p->bg[0];
    a.bg1 = p->bg[1];
    a.bg2 = p->bg[2];
    a.want_dist = p->want_dist != 0;
    if (p->ray_list) {
        if (p->n_list < 0 || p->n_list > s->n_rays) return set_error(DVGO_ERR_RANGE, "n_list must be in [0, n_rays]");
        a.ray_list = p->ray_list;
        a.n_list = p->n_list;
    } else {
        a.ray_list = nullptr;
        a.n_list = s->n_rays;
    }
    if (p->waves_per_block < 0 || p->waves_per_block > 16) return set_error(DVGO_ERR_RANGE, "waves_per_block in 0..16");
    if (p->grid_waves < 0) return set_error(DVGO_ERR_RANGE, "grid_waves must be >= 0");
    return DVGO_OK;
}

struct Launch {
    dim3 grid, block;
};

Launch launch_shape(const dvgo_render_params *p, int n_list) {
    const int wpb = p->waves_per_block ? p->waves_per_block : 4;
    int waves = p->grid_waves ? (p->grid_waves < n_list ? p->grid_waves : n_list) : n_list;
    if (waves < 1) waves = 1;
    return Launch{dim3((waves + wpb - 1) / wpb), dim3(64 * wpb)};
}

// kernels with the contraction path only where a grid of the call has a warp
bool any_warp(const dvgo_render_params *p, const RenderArgs &a) {
    return a.dens.warp || (p->color_mode == DVGO_COLOR_GRID && a.col.warp);
}

template <bool W>
void launch_fwd_w(const dvgo_render_params *p, const Launch &L, const RenderArgs &a, hipStream_t st) {
    if (p->color_mode == DVGO_COLOR_GRID)
        hipLaunchKernelGGL((render_fwd_kernel<DVGO_COLOR_GRID, W>), L.grid, L.block, 0, st, a);
    else if (p->color_mode == DVGO_COLOR_SAMPLES)
        hipLaunchKernelGGL((render_fwd_kernel<DVGO_COLOR_SAMPLES, W>), L.grid, L.block, 0, st, a);
    else
        hipLaunchKernelGGL((render_fwd_kernel<DVGO_COLOR_NONE, W>), L.grid, L.block, 0, st, a);
}

template <bool W>
void launch_bwd_w(const dvgo_render_params *p, const Launch &L, const RenderArgs &a, hipStream_t st) {
    if (p->color_mode == DVGO_COLOR_GRID)
        hipLaunchKernelGGL((render_bwd_kernel<DVGO_COLOR_GRID, W>), L.grid, L.block, scatter_lds_bytes(3, L.block.x),
                           st, a);
    else
        hipLaunchKernelGGL((render_bwd_kernel<DVGO_COLOR_SAMPLES, W>), L.grid, L.block, 0, st, a);
}

template <bool W>
void launch_train_w(const dvgo_render_params *p, const Launch &L, const RenderArgs &a, hipStream_t st) {
    if (p->color_mode == DVGO_COLOR_GRID)
        hipLaunchKernelGGL((render_train_kernel<DVGO_COLOR_GRID, W>), L.grid, L.block,
                           scatter_lds_bytes(3, L.block.x), st, a);
    else
        hipLaunchKernelGGL((render_train_kernel<DVGO_COLOR_SAMPLES, W>), L.grid, L.block, 0, st, a);
}

int launch_train(const dvgo_render_params *p, const RenderArgs &a, hipStream_t st) {
    const Launch L = launch_shape(p, a.n_list);
    if (any_warp(p, a)) launch_train_w<true>(p, L, a, st);
    else launch_train_w<false>(p, L, a, st);
    return check_hip(hipGetLastError(), "render_train_kernel launch");
}

int launch_fwd(const dvgo_render_params *p, const RenderArgs &a, hipStream_t st) {
    const Launch L = launch_shape(p, a.n_list);
    if (any_warp(p, a)) launch_fwd_w<true>(p, L, a, st);
    else launch_fwd_w<false>(p, L, a, st);
    return check_hip(hipGetLastError(), "render_fwd_kernel launch");
}

int launch_bwd(const dvgo_render_params *p, const RenderArgs &a, hipStream_t st) {
    const Launch L = launch_shape(p, a.n_list);
    if (any_warp(p, a)) launch_bwd_w<true>(p, L, a, st);
    else launch_bwd_w<false>(p, L, a, st);
    return check_hip(hipGetLastError(), "render_bwd_kernel launch");
}

// state: halt index [R] | chunk checkpoints [ckpt_count] | density logits [S], each part
// 256-byte aligned
size_t state_bytes(int32_t n_rays, int64_t n_samples) {
    return align_up((size_t)n_rays * 4, 256) + align_up((size_t)ckpt_count(n_rays, n_samples) * sizeof(float4), 256) +
           (size_t)n_samples * 4;
}

void split_state(void *state, int32_t n_rays, int64_t n_samples, int **halt, float4 **ck, float **raw) {
    *halt = (int *)state;
    *ck = (float4 *)((char *)state + align_up((size_t)n_rays * 4, 256));
    *raw = (float *)((char *)*ck + align_up((size_t)ckpt_count(n_rays, n_samples) * sizeof(float4), 256));
}

}  // namespace

extern "C" int dvgo_render_state_size(int32_t n_rays, int64_t n_samples, size_t *bytes) {
    if (!bytes) return set_error(DVGO_ERR_NULL, "bytes is NULL");
    if (n_rays < 0 || n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative size");
    *bytes = state_bytes(n_rays, n_samples);
    return DVGO_OK;
}

extern "C" int dvgo_render_forward(const dvgo_render_params *p, const dvgo_samples *s, const dvgo_grid *density,
                                   const dvgo_grid *color, const float *sample_rgb, float *rgb, float *T_final,
                                   float *dist, float *sample_w, void *state, size_t state_bytes_, void *stream) {
    RenderArgs a;
    int rc = fill_render_args(p, s, density, color, sample_rgb, false, a);
    if (rc) return rc;
    if (s->n_rays == 0) return DVGO_OK;
    if (!rgb || !T_final || !state) return set_error(DVGO_ERR_NULL, "rgb, T_final or state is NULL");
    if (p->want_dist && !dist) return set_error(DVGO_ERR_NULL, "dist is NULL with want_dist");
    if (state_bytes_ < state_bytes(s->n_rays, s->n_samples))
        return set_error(DVGO_ERR_WORKSPACE, "state buffer too small (%zu < %zu)", state_bytes_,
                         state_bytes(s->n_rays, s->n_samples));
    a.rgb = rgb;
    a.T_final = T_final;
    a.dist = dist;
    a.sample_w = sample_w;
    split_state(state, s->n_rays, s->n_samples, &a.halt_idx, &a.ckpt, &a.raw_saved);
    if (debug_mode()) {
        rc = validate_batch(s->n_rays, s->n_samples, s->ray_offsets, s->s_mid, (hipStream_t)stream);
        if (rc) return rc;
    }
    if (a.n_list == 0) return DVGO_OK;
    return launch_fwd(p, a, (hipStream_t)stream);
}

extern "C" int dvgo_render_backward(const dvgo_render_params *p, const dvgo_samples *s, const dvgo_grid *density,
                                    const dvgo_grid *color, const float *sample_rgb, const float *T_final,
                                    const void *state, size_t state_bytes_, const float *grad_rgb,
                                    const float *grad_dist, const float *grad_T, float *grad_sample_rgb,
                                    float *grad_sample_density, void *stream) {
    RenderArgs a;
    int rc = fill_render_args(p, s, density, color, sample_rgb, true, a, grad_sample_density == nullptr);
    if (rc) return rc;
    if (s->n_rays == 0) return DVGO_OK;
    if (!T_final || !state || !grad_rgb) return set_error(DVGO_ERR_NULL, "T_final, state or grad_rgb is NULL");
    if (p->color_mode == DVGO_COLOR_SAMPLES && s->n_samples > 0 && !grad_sample_rgb)
        return set_error(DVGO_ERR_NULL, "grad_sample_rgb is NULL in DVGO_COLOR_SAMPLES mode");
    if (state_bytes_ < state_bytes(s->n_rays, s->n_samples))
        return set_error(DVGO_ERR_WORKSPACE, "state buffer too small");
    a.T_in = T_final;
    a.grad_rgb = grad_rgb;
    a.grad_dist = p->want_dist ? grad_dist : nullptr;
    a.grad_T = grad_T;
    a.grad_srgb = grad_sample_rgb;
    a.grad_raw = grad_sample_density;
    split_state(const_cast<void *>(state), s->n_rays, s->n_samples, &a.halt_idx, &a.ckpt, &a.raw_saved);
    if (debug_mode()) {
        rc = validate_batch(s->n_rays, s->n_samples, s->ray_offsets, s->s_mid, (hipStream_t)stream);
        if (rc) return rc;
    }
    if (a.n_list == 0) return DVGO_OK;
    return launch_bwd(p, a, (hipStream_t)stream);
}

extern "C" int dvgo_render_train(const dvgo_render_params *p, const dvgo_samples *s, const dvgo_grid *density,
                                 const dvgo_grid *color, const float *sample_rgb, const float *target,
                                 float dist_weight, float *rgb, float *T_final, float *dist, void *state,
                                 size_t state_bytes_, float *grad_sample_rgb, float *grad_sample_density,
                                 void *stream) {
    RenderArgs a;
    int rc = fill_render_args(p, s, density, color, sample_rgb, true, a, grad_sample_density == nullptr);
    if (rc) return rc;
    if (s->n_rays == 0) return DVGO_OK;
    if (!rgb || !T_final || !state || !target) return set_error(DVGO_ERR_NULL, "rgb, T_final, state or target is NULL");
    if (p->want_dist && !dist) return set_error(DVGO_ERR_NULL, "dist is NULL with want_dist");
    if (p->color_mode == DVGO_COLOR_SAMPLES && s->n_samples > 0 && !grad_sample_rgb)
        return set_error(DVGO_ERR_NULL, "grad_sample_rgb is NULL in DVGO_COLOR_SAMPLES mode");
    if (!(dist_weight >= 0.f && dist_weight <= 3.4e38f))
        return set_error(DVGO_ERR_RANGE, "dist_weight must be finite and >= 0");
    if (state_bytes_ < state_bytes(s->n_rays, s->n_samples))
        return set_error(DVGO_ERR_WORKSPACE, "state buffer too small (%zu < %zu)", state_bytes_,
                         state_bytes(s->n_rays, s->n_samples));
    a.rgb = rgb;
    a.T_final = T_final;
    a.dist = dist;
    a.sample_w = nullptr;
    a.target = target;
    a.lam = dist_weight;
    a.grad_srgb = grad_sample_rgb;
    a.grad_raw = grad_sample_density;
    split_state(state, s->n_rays, s->n_samples, &a.halt_idx, &a.ckpt, &a.raw_saved);
    if (debug_mode()) {
        rc = validate_batch(s->n_rays, s->n_samples, s->ray_offsets, s->s_mid, (hipStream_t)stream);
        if (rc) return rc;
    }
    if (a.n_list == 0) return DVGO_OK;
    return launch_train(p, a, (hipStream_t)stream);
}

// ------------------------------------------------------------------- scheduling

namespace {

constexpr int NCLASS = 64;

__global__ __launch_bounds__(1024) void schedule_kernel(int R, const int *offs, int *order, int *class_offsets) {
    __shared__ int hist[NCLASS], start[NCLASS], cursor[NCLASS];
    for (int c = threadIdx.x; c < NCLASS; c += blockDim.x) {
        hist[c] = 0;
        cursor[c] = 0;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        const int ch = (offs[r + 1] - offs[r] + 63) / 64;
        atomicAdd(&hist[ch < NCLASS - 1 ? ch : NCLASS - 1], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int pos = 0;
        for (int k = 0; k < NCLASS; ++k) {  // class k holds rays with 63 - k chunks
            const int c = NCLASS - 1 - k;
            start[c] = pos;
            class_offsets[k] = pos;
            pos += hist[c];
        }
        class_offsets[NCLASS] = pos;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        int ch = (offs[r + 1] - offs[r] + 63) / 64;
        ch = ch < NCLASS - 1 ? ch : NCLASS - 1;
        order[start[ch] + atomicAdd(&cursor[ch], 1)] = r;
    }
}

struct TuneKey {
    int mode, want_dist;
    int n_rays;
    long long n_samples;
    const void *list;
    int n_list;
    float halt_T;
    int dens_warp, col_warp;
    int sample_grad;  // the backward writes per-sample density gradients (no in-kernel scatter)
    bool operator<(const TuneKey &o) const {
        return std::tie(mode, want_dist, n_rays, n_samples, list, n_list, halt_T, dens_warp, col_warp, sample_grad) <
               std::tie(o.mode, o.want_dist, o.n_rays, o.n_samples, o.list, o.n_list, o.halt_T, o.dens_warp,
                        o.col_warp, o.sample_grad);
    }
};
struct TuneVal {
    int wpb, grid_waves;
    float ms;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

}  // namespace

extern "C" int dvgo_ray_schedule(int32_t n_rays, const int32_t *ray_offsets, int32_t *order, int32_t *class_offsets,
                                 void *stream) {
    if (n_rays < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays");
    if (!ray_offsets || !order || !class_offsets) return set_error(DVGO_ERR_NULL, "an argument is NULL");
    hipLaunchKernelGGL(schedule_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, n_rays, ray_offsets, order,
                       class_offsets);
    return check_hip(hipGetLastError(), "schedule_kernel launch");
}

extern "C" int dvgo_render_autotune(const dvgo_render_params *p, const dvgo_samples *s, const dvgo_grid *density,
                                    const dvgo_grid *color, const float *sample_rgb, int32_t sample_density_grad,
                                    int32_t *waves_per_block, int32_t *grid_waves, float *ms, void *stream) {
    RenderArgs a;
    int rc = fill_render_args(p, s, density, color, sample_rgb, false, a);
    if (rc) return rc;
    if (p->color_mode == DVGO_COLOR_NONE) return set_error(DVGO_ERR_UNSUPPORTED, "autotune needs a colour mode");
    if (!waves_per_block || !grid_waves) return set_error(DVGO_ERR_NULL, "output pointers are NULL");
    const int sg = sample_density_grad ? 1 : 0;
    const TuneKey key{p->color_mode, p->want_dist, s->n_rays, (long long)s->n_samples, p->ray_list, a.n_list,
                      p->halt_T, a.dens.warp, p->color_mode == DVGO_COLOR_GRID ? a.col.warp : 0, sg};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *waves_per_block = it->second.wpb;
            *grid_waves = it->second.grid_waves;
            if (ms) *ms = it->second.ms;
            return DVGO_OK;
        }
    }
    const int R = s->n_rays;
    const int64_t S = s->n_samples;
    const hipStream_t st = (hipStream_t)stream;
    // scratch outputs; gradients go to scratch grids so the caller's buffers are untouched
    const size_t n_dens = (size_t)density->nx * density->ny * density->nz * density->ch_stride;
    const size_t n_col = color ? (size_t)color->nx * color->ny * color->nz * color->ch_stride : 0;
    float *buf = nullptr;
    const size_t nf = (size_t)R * 3 + 2 * (size_t)R + (size_t)R * 3 + 2 * (size_t)R + n_dens + n_col + (size_t)S * 3 +
                      (sg ? (size_t)S : 0);
    void *state = nullptr;
    const size_t sb = state_bytes(R, S);
    if (hipMalloc(&buf, nf * sizeof(float)) != hipSuccess || hipMalloc(&state, sb) != hipSuccess) {
        if (buf) (void)hipFree(buf);
        return set_error(DVGO_ERR_HIP, "autotune scratch allocation failed");
    }
    float *rgb = buf, *T = rgb + 3 * (size_t)R, *dist = T + R, *grgb = dist + R, *gdist = grgb + 3 * (size_t)R,
          *gT = gdist + R, *gden = gT + R, *gcol = gden + n_dens, *gs = gcol + n_col, *graw = gs + (size_t)S * 3;
    // the first HIP failure below is kept in rc; later steps are skipped, the scratch is freed
    auto ck = [&rc](hipError_t e, const char *what) {
        if (!rc && e != hipSuccess) rc = check_hip(e, what);
    };
    ck(hipMemsetD32Async((hipDeviceptr_t)grgb, 0x3f800000, 3 * (size_t)R + 2 * (size_t)R, st), "autotune fill");  // ones
    dvgo_grid dg = *density, cg;
    dg.grad = gden;
    if (color) {
        cg = *color;
        cg.grad = gcol;
    }
    RenderArgs fa = a, ba;
    fa.rgb = rgb;
    fa.T_final = T;
    fa.dist = dist;
    fa.sample_w = nullptr;
    split_state(state, R, S, &fa.halt_idx, &fa.ckpt, &fa.raw_saved);
    if (!rc) rc = fill_render_args(p, s, &dg, color ? &cg : nullptr, sample_rgb, true, ba);
    ba.grad_raw = sg ? graw : nullptr;  // the caller's backward variant: per-sample gradients or in-kernel scatter
    ba.T_in = T;
    ba.grad_rgb = grgb;
    ba.grad_dist = p->want_dist ? gdist : nullptr;
    ba.grad_T = gT;
    ba.grad_srgb = gs;
    ba.halt_idx = fa.halt_idx;
    ba.ckpt = fa.ckpt;
    ba.raw_saved = fa.raw_saved;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ck(hipEventCreate(&e0), "autotune event");
    ck(hipEventCreate(&e1), "autotune event");
    TuneVal best{4, 0, 1e30f};
    const int wpbs[] = {2, 4, 8, 16};
    const int grids[] = {0, 1024, 2048, 4096, 8192, 16384};
    for (int wi = 0; wi < 4 && !rc; ++wi) {
        for (int gi = 0; gi < 6 && !rc; ++gi) {
            if (grids[gi] >= a.n_list && grids[gi] != 0) continue;
            dvgo_render_params q = *p;
            q.waves_per_block = wpbs[wi];
            q.grid_waves = grids[gi];
            rc = launch_fwd(&q, fa, st);  // warm-up
            if (!rc) rc = launch_bwd(&q, ba, st);
            ck(hipEventRecord(e0, st), "autotune event record");
            for (int rep = 0; rep < 3 && !rc; ++rep) {
                rc = launch_fwd(&q, fa, st);
                if (!rc) rc = launch_bwd(&q, ba, st);
            }
            ck(hipEventRecord(e1, st), "autotune event record");
            ck(hipEventSynchronize(e1), "autotune event wait");
            float t = 0.f;
            ck(hipEventElapsedTime(&t, e0, e1), "autotune event time");
            t /= 3.f;
            if (!rc && t < best.ms) best = TuneVal{wpbs[wi], grids[gi], t};
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    ck(hipStreamSynchronize(st), "autotune stream wait");  // the scratch is idle before it is freed
    (void)hipFree(buf);
    (void)hipFree(state);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = best;
    }
    *waves_per_block = best.wpb;
    *grid_waves = best.grid_waves;
    if (ms) *ms = best.ms;
    return DVGO_OK;
}

extern "C" int dvgo_distortion_workspace_size(int32_t n_rays, int64_t n_samples, size_t *bytes) {
    if (!bytes) return set_error(DVGO_ERR_NULL, "bytes is NULL");
    if (n_rays < 0 || n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative size");
    *bytes = (size_t)ckpt_count(n_rays, n_samples) * sizeof(float2);
    return DVGO_OK;
}

namespace dvgo {

int distortion_check(int32_t n_rays, const int32_t *ray_offsets, int64_t n_samples, const float *w, const float *s_mid,
                     const float *s_len, const float *loss, const float *grad_loss, const float *grad_w) {
    if (n_rays < 0 || n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays or n_samples");
    if (n_samples > MAX_SAMPLES) return set_error(DVGO_ERR_RANGE, "n_samples must be at most %lld", (long long)MAX_SAMPLES);
    if (n_rays == 0) return DVGO_OK;
    if (!ray_offsets) return set_error(DVGO_ERR_NULL, "ray_offsets is NULL");
    if (n_samples > 0 && (!w || !s_mid || !s_len)) return set_error(DVGO_ERR_NULL, "w, s_mid or s_len is NULL");
    const bool bwd = grad_loss && grad_w;
    if (!loss && !bwd) return set_error(DVGO_ERR_NULL, "nothing to compute: loss and grad_w are NULL");
    if ((grad_loss == nullptr) != (grad_w == nullptr))
        return set_error(DVGO_ERR_NULL, "grad_loss and grad_w must both be given for the backward");
    return DVGO_OK;
}

size_t distortion_scratch_bytes(int32_t n_rays, int64_t n_samples) {
    return (size_t)ckpt_count(n_rays, n_samples) * sizeof(float2);
}

int launch_distortion(int32_t n_rays, const int32_t *ray_offsets, int64_t n_samples, const float *w, const float *s_mid,
                      const float *s_len, float *loss, const float *grad_loss, float *grad_w, void *ckpt,
                      hipStream_t st) {
    if (debug_mode()) {
        const int rc = validate_batch(n_rays, n_samples, ray_offsets, s_mid, st);
        if (rc) return rc;
    }
    const bool bwd = grad_loss && grad_w;
    const dim3 grid((n_rays + 3) / 4), block(256);
    hipLaunchKernelGGL(distortion_kernel, grid, block, 0, st, n_rays, ray_offsets, w, s_mid, s_len, loss,
                       bwd ? grad_loss : nullptr, bwd ? grad_w : nullptr, (float2 *)ckpt);
    return check_hip(hipGetLastError(), "distortion_kernel launch");
}

}  // namespace dvgo

extern "C" int dvgo_distortion_loss(int32_t n_rays, const int32_t *ray_offsets, int64_t n_samples, const float *w,
                                    const float *s_mid, const float *s_len, float *loss, const float *grad_loss,
                                    float *grad_w, void *ws, size_t ws_bytes, void *stream) {
    int rc = distortion_check(n_rays, ray_offsets, n_samples, w, s_mid, s_len, loss, grad_loss, grad_w);
    if (rc || n_rays == 0) return rc;
    const size_t need = distortion_scratch_bytes(n_rays, n_samples);
    if (grad_loss && grad_w && (!ws || ws_bytes < need))
        return set_error(DVGO_ERR_WORKSPACE, "workspace too small (%zu < %zu)", ws_bytes, need);
    return launch_distortion(n_rays, ray_offsets, n_samples, w, s_mid, s_len, loss, grad_loss, grad_w, ws,
                             (hipStream_t)stream);
}
