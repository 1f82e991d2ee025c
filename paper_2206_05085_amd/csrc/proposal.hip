// Learned proposal stage on gfx950: a coarse density-only pass, a 64-64-64-64-64 MLP on
// BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation, FP32 master weights)
// that predicts a 64-bin weight histogram per ray, its cross-entropy training backward,
// the rendered-weight histograms it is trained on, and inverse-CDF resampling of a fine
// ragged batch with an entropy fallback to plain uniform sampling.
//
// MFMA tiling follows the colour MLP: activations stay "hidden-major" in registers
// (lane (q = lane/16, j = lane%16) owns rows 4q..4q+3 of ray j of each 16-row tile), and a
// K-step of 32 consumes two consecutive row tiles by ordering the reduction index as
// k(kk, q, e) = 32 kk + 4 q + e (e < 4) or 32 kk + 16 + 4 q + (e - 4) (e >= 4); the matching
// weight operand is two 8-byte runs of one LDS row.
#include <string.h>

#include "dvgo_internal.h"

using namespace dvgo;

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int NB = 64;   // bins = input = hidden = output width
constexpr int NL = 4;    // linear layers (three hidden ReLU layers)
constexpr int WS = 72;   // LDS row stride (bf16) of weight and staging tiles
constexpr int THREADS = 256, TILE = 64;
constexpr int MAX_BLOCKS = 128;
constexpr int NPARAM = NL * (NB * NB + NB);

__device__ __forceinline__ v4f mfma_bf16(bf16x8 a, bf16x8 b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int kidx(int kk, int q, int e) {
    return 32 * kk + (e < 4 ? 4 * q + e : 16 + 4 * q + (e - 4));
}

// A operand of K-step kk from one LDS row (entries k(kk, q, 0..7))
__device__ __forceinline__ bf16x8 load_a(const __bf16 *row, int kk, int q) {
    const bf16x4 lo = *reinterpret_cast<const bf16x4 *>(row + 32 * kk + 4 * q);
    const bf16x4 hi = *reinterpret_cast<const bf16x4 *>(row + 32 * kk + 16 + 4 * q);
    return bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// B operand of K-step kk from a C-layout activation (tiles 2kk and 2kk+1)
__device__ __forceinline__ bf16x8 pack_b(const v4f &t0, const v4f &t1) {
    return bf16x8{(__bf16)t0[0], (__bf16)t0[1], (__bf16)t0[2], (__bf16)t0[3],
                  (__bf16)t1[0], (__bf16)t1[1], (__bf16)t1[2], (__bf16)t1[3]};
}

struct PropArgs {
    const float *W[NL], *b[NL];
    float *gW[NL], *gb[NL];
    int R;
    const float *x;
    float *logits, *prob, *entropy;
    const float *target;
    float *loss, *partial;
    int nblocks;
};

// fp32 master weights -> bf16 (round to nearest even) in LDS: W rows [out][in]; WT rows [in][out]
__device__ void stage_weights(const PropArgs &a, __bf16 *Wl, __bf16 *WT) {
    for (int i = threadIdx.x; i < NL * NB * NB; i += blockDim.x) {
        const int l = i / (NB * NB), o = (i / NB) % NB, c = i % NB;
        const __bf16 v = (__bf16)a.W[l][o * NB + c];
        Wl[(l * NB + o) * WS + c] = v;
        if (WT) WT[(l * NB + c) * WS + o] = v;
    }
}

// forward of 16 rays; act[l][kk] = bf16 input operand of layer l; z = logits (fp32, C-layout)
__device__ __forceinline__ void forward_tile(const PropArgs &a, const __bf16 *Wl, int ray, bool rv, int q, int j,
                                             bf16x8 act[NL][2], v4f z[4]) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
        float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
        if (rv) {
            lo = *reinterpret_cast<const float4 *>(a.x + (int64_t)ray * NB + 32 * kk + 4 * q);
            hi = *reinterpret_cast<const float4 *>(a.x + (int64_t)ray * NB + 32 * kk + 16 + 4 * q);
        }
        act[0][kk] = bf16x8{(__bf16)lo.x, (__bf16)lo.y, (__bf16)lo.z, (__bf16)lo.w,
                            (__bf16)hi.x, (__bf16)hi.y, (__bf16)hi.z, (__bf16)hi.w};
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        v4f acc[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            acc[m] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) acc[m] = mfma_bf16(load_a(Wl + (l * NB + 16 * m + j) * WS, kk, q), act[l][kk], acc[m]);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[m][r] += a.b[l][16 * m + 4 * q + r];
        }
        if (l + 1 < NL) {
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[m][r] = fmaxf(acc[m][r], 0.f);
            act[l + 1][0] = pack_b(acc[0], acc[1]);
            act[l + 1][1] = pack_b(acc[2], acc[3]);
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) z[m] = acc[m];
        }
    }
}

// per-ray softmax over the 64 logits held by the 4 lanes (q = 0..3) of column j
__device__ __forceinline__ void softmax_tile(const v4f z[4], v4f p[4], float &mx, float &lse, float &ent) {
    mx = -INFINITY;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) mx = fmaxf(mx, z[m][r]);
    mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    float s = 0.f;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            p[m][r] = expf(z[m][r] - mx);
            s += p[m][r];
        }
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    const float inv = 1.f / s;
    float pz = 0.f;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            p[m][r] *= inv;
            pz += p[m][r] * (z[m][r] - mx);
        }
    pz += __shfl_xor(pz, 16, 64);
    pz += __shfl_xor(pz, 32, 64);
    lse = logf(s);
    ent = lse - pz;
}

__global__ __launch_bounds__(THREADS) void prop_fwd_kernel(PropArgs a) {
    __shared__ __bf16 Wl[NL * NB * WS];
    stage_weights(a, Wl, nullptr);
    __syncthreads();
    const int wv = threadIdx.x >> 6, ln = lane(), j = ln & 15, q = ln >> 4;
    const int ntiles = (a.R + TILE - 1) / TILE;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int ray = tile * TILE + wv * 16 + j;
        const bool rv = ray < a.R;
        bf16x8 act[NL][2];
        v4f z[4], p[4];
        forward_tile(a, Wl, ray, rv, q, j, act, z);
        float mx, lse, ent;
        softmax_tile(z, p, mx, lse, ent);
        if (rv) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int o = ray * NB + 16 * m + 4 * q;
                if (a.logits) *reinterpret_cast<float4 *>(a.logits + o) = make_float4(z[m][0], z[m][1], z[m][2], z[m][3]);
                if (a.prob) *reinterpret_cast<float4 *>(a.prob + o) = make_float4(p[m][0], p[m][1], p[m][2], p[m][3]);
            }
            if (a.entropy && q == 0) a.entropy[ray] = ent;
        }
    }
}

// Cross-entropy backward.  dL/dz = (softmax - target)/R; every gradient that enters a
// product is rounded to bf16 like the weights and activations.
__global__ __launch_bounds__(THREADS) void prop_bwd_kernel(PropArgs a) {
    __shared__ __bf16 Wl[NL * NB * WS];
    __shared__ __bf16 WT[NL * NB * WS];
    __shared__ __bf16 sdz[TILE * WS];
    __shared__ __bf16 sact[TILE * WS];
    __shared__ float sloss[THREADS / 64];
    stage_weights(a, Wl, WT);
    __syncthreads();
    const int tid = threadIdx.x, wv = tid >> 6, ln = lane(), j = ln & 15, q = ln >> 4;
    const int row = wv * 16 + j;
    v4f dW[NL][4];
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int t = 0; t < 4; ++t) dW[l][t] = v4f{0.f, 0.f, 0.f, 0.f};
    float db[NL] = {0.f, 0.f, 0.f, 0.f};
    float loss_acc = 0.f;
    const float invR = 1.f / (float)a.R;
    const int ntiles = (a.R + TILE - 1) / TILE;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int ray = tile * TILE + row;
        const bool rv = ray < a.R;
        bf16x8 act[NL][2];
        v4f z[4], p[4];
        forward_tile(a, Wl, ray, rv, q, j, act, z);
        float mx, lse, ent;
        softmax_tile(z, p, mx, lse, ent);
        v4f dz[4];
        float ce = 0.f;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            float4 tg = make_float4(0.f, 0.f, 0.f, 0.f);
            if (rv) tg = *reinterpret_cast<const float4 *>(a.target + (int64_t)ray * NB + 16 * m + 4 * q);
            const float t4[4] = {tg.x, tg.y, tg.z, tg.w};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ce -= t4[r] * (z[m][r] - mx - lse);
                dz[m][r] = rv ? (float)(__bf16)((p[m][r] - t4[r]) * invR) : 0.f;
            }
        }
        loss_acc += rv ? ce : 0.f;
#pragma unroll
        for (int l = NL - 1; l >= 0; --l) {
            // stage dz_l [ray][out] and the layer input a_l [ray][in] for the weight gradient
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) sdz[row * WS + 16 * m + 4 * q + r] = (__bf16)dz[m][r];
#pragma unroll
            for (int kk = 0; kk < 2; ++kk)
#pragma unroll
                for (int e = 0; e < 8; ++e) sact[row * WS + kidx(kk, q, e)] = act[l][kk][e];
            __syncthreads();
            // dW_l[out 16 wv + .., in 16 t + ..] += sum over the 64 rays of the tile
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                bf16x8 A;
#pragma unroll
                for (int e = 0; e < 8; ++e) A[e] = sdz[(32 * kk + 8 * q + e) * WS + 16 * wv + j];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    bf16x8 B;
#pragma unroll
                    for (int e = 0; e < 8; ++e) B[e] = sact[(32 * kk + 8 * q + e) * WS + 16 * t + j];
                    dW[l][t] = mfma_bf16(A, B, dW[l][t]);
                }
            }
            if (tid < NB) {
                float s = 0.f;
                for (int r2 = 0; r2 < TILE; ++r2) s += (float)sdz[r2 * WS + tid];
                db[l] += s;
            }
            __syncthreads();
            if (l > 0) {
                // d a_l = W_l^T dz_l, then the ReLU mask of a_l (a_l > 0 <=> its pre-activation > 0)
                const bf16x8 B0 = pack_b(dz[0], dz[1]), B1 = pack_b(dz[2], dz[3]);
                v4f da[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    da[m] = mfma_bf16(load_a(WT + (l * NB + 16 * m + j) * WS, 0, q), B0, v4f{0.f, 0.f, 0.f, 0.f});
                    da[m] = mfma_bf16(load_a(WT + (l * NB + 16 * m + j) * WS, 1, q), B1, da[m]);
                }
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float av = (float)act[l][m >> 1][(m & 1) * 4 + r];
                        dz[m][r] = av > 0.f ? (float)(__bf16)da[m][r] : 0.f;
                    }
            }
        }
    }
    // this block's partial gradients, layer by layer: W_l [out][in] then b_l
    float *P = a.partial + (int64_t)blockIdx.x * (NPARAM + 1);
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        float *pw = P + l * (NB * NB + NB), *pb = pw + NB * NB;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) pw[(16 * wv + 4 * q + r) * NB + 16 * t + j] = dW[l][t][r];
        if (tid < NB) pb[tid] = db[l];
    }
    loss_acc = wave_sum(loss_acc);
    if (ln == 0) sloss[wv] = loss_acc;
    __syncthreads();
    if (tid == 0) P[NPARAM] = (sloss[0] + sloss[1] + sloss[2] + sloss[3]) * invR;
}

__global__ void prop_reduce_kernel(PropArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > NPARAM) return;
    float s = 0.f;
    for (int b = 0; b < a.nblocks; ++b) s += a.partial[(int64_t)b * (NPARAM + 1) + i];
    if (i == NPARAM) {
        if (a.loss) a.loss[0] = s;
        return;
    }
    const int l = i / (NB * NB + NB), k = i % (NB * NB + NB);
    if (k < NB * NB) a.gW[l][k] += s;
    else a.gb[l][k - NB * NB] += s;
}

// ------------------------------------------------------------------- coarse pass

struct RayArgs {
    int R;
    const float *o, *d, *tn, *tf;
};

// one wave per ray, lane = coarse sample / bin; positions are formed in double so that
// they equal the float32 rounding of the exact point
__global__ __launch_bounds__(256) void coarse_kernel(RayArgs ra, DevGrid g, float shift, float voxel, float eps,
                                                     float *feat, float *wout) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= ra.R) return;
    const int k = lane();
    const float a = ra.tn[r], b = ra.tf[r];
    const bool hit = b > a;
    float x = 0.f, alpha = 0.f;
    if (hit) {
        const double t = (double)a + ((double)k + 0.5) / NB * ((double)b - (double)a);
        const float px = (float)((double)ra.o[3 * r] + t * (double)ra.d[3 * r]);
        const float py = (float)((double)ra.o[3 * r + 1] + t * (double)ra.d[3 * r + 1]);
        const float pz = (float)((double)ra.o[3 * r + 2] + t * (double)ra.d[3 * r + 2]);
        const float raw = interp_ch(g, trilinear<true>(g, px, py, pz), 0);
        const float delta = (float)(((double)b - (double)a) / NB / (double)voxel);
        x = softplusf(raw + shift) * delta;
        alpha = -expm1f(-x);
    }
    const float T = expf(-wave_excl(wave_incl(x)));
    const float w = T * alpha;
    feat[(int64_t)r * NB + k] = log1pf(w / eps);
    if (wout) wout[(int64_t)r * NB + k] = w;
}

// target histogram of rendered weights: bin = floor(s_mid * B); normalised when the total
// reaches min_mass, else uniform.  One wave per ray, bins accumulated in LDS.
__global__ __launch_bounds__(256) void histogram_kernel(int R, const int *offs, const float *w, const float *s_mid,
                                                        float min_mass, float *hist) {
    __shared__ float bins[4][NB];
    const int wv = threadIdx.x >> 6, r = blockIdx.x * 4 + wv, ln = lane();
    if (r >= R) return;
    bins[wv][ln] = 0.f;
    __threadfence_block();
    float tot = 0.f;
    for (int k = offs[r] + ln; k < offs[r + 1]; k += 64) {
        int bi = (int)floorf(s_mid[k] * (float)NB);
        bi = bi < 0 ? 0 : (bi > NB - 1 ? NB - 1 : bi);
        atomicAdd(&bins[wv][bi], w[k]);
        tot += w[k];
    }
    tot = wave_sum(tot);
    __threadfence_block();
    const float v = bins[wv][ln];
    hist[(int64_t)r * NB + ln] = tot >= min_mass ? v / tot : 1.f / NB;
}

// ----------------------------------------------------------------- resampling

// counts (0 for rays that miss, n_plain above the entropy threshold, else n_fine) and
// their exclusive prefix sum, in one block
__global__ __launch_bounds__(1024) void resample_offsets_kernel(int R, const float *tn, const float *tf,
                                                                const float *H, float tau, int n_fine, int n_plain,
                                                                int *offs) {
    __shared__ int wsum[16];
    __shared__ int carry;
    if (threadIdx.x == 0) {
        carry = 0;
        offs[0] = 0;
    }
    __syncthreads();
    for (int base = 0; base < R; base += 1024) {
        const int r = base + threadIdx.x;
        int c = 0;
        if (r < R) c = !(tf[r] > tn[r]) ? 0 : (H[r] > tau ? n_plain : n_fine);
        // inclusive scan of c across the block
        int v = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(v, d, 64);
            if (lane() >= d) v += t;
        }
        if (lane() == 63) wsum[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x < 16) {
            int s = wsum[threadIdx.x];
#pragma unroll
            for (int d = 1; d < 16; d <<= 1) {
                const int t = __shfl_up(s, d, 16);
                if ((int)threadIdx.x >= d) s += t;
            }
            wsum[threadIdx.x] = s;
        }
        __syncthreads();
        const int wave_off = (threadIdx.x >> 6) ? wsum[(threadIdx.x >> 6) - 1] : 0;
        if (r < R) offs[r + 1] = carry + wave_off + v;
        __syncthreads();
        if (threadIdx.x == 0) carry += wsum[15];
        __syncthreads();
    }
}

// one wave per ray: plain uniform samples for fallback rays, else interval resampling:
// n+1 interval ends at the inverse CDF of u_j = j/n of the 64-bin piecewise-constant
// density (lane = bin for the CDF scan), each sample the midpoint of two consecutive ends
// The mass test and the in-bin slope use the bin masses themselves, not differences of
// the float32 CDF (a tiny mass next to a large prefix would vanish in the difference).
__device__ __forceinline__ float inv_cdf(const float *cdf, const float *pm, float u, float total) {
    if (!(u < total)) {
        int b = NB - 1;
        while (b > 0 && !(pm[b] > 0.f)) --b;
        return (float)(b + 1) / (float)NB;
    }
    int b = 0;
    while (b < NB - 1 && !(cdf[b + 1] > u)) ++b;
    const float pb = pm[b];
    float frac = pb > 0.f ? (u - cdf[b]) / pb : 0.f;
    frac = fminf(fmaxf(frac, 0.f), 1.f);
    return ((float)b + frac) / (float)NB;
}

__global__ __launch_bounds__(256) void resample_fill_kernel(RayArgs ra, const float *prob, const float *H, float tau,
                                                            const int *offs, int n_fine, int n_plain, float voxel,
                                                            float *xyz, float *delta, float *s_mid, float *s_len) {
    __shared__ float cdf_s[4][NB + 1];
    __shared__ float pm_s[4][NB];
    __shared__ float ends[4][257];
    const int wv = threadIdx.x >> 6, r = blockIdx.x * 4 + wv, ln = lane();
    if (r >= ra.R) return;
    const int beg = offs[r], n = offs[r + 1] - beg;
    if (n == 0) return;
    const double a = ra.tn[r], len = (double)ra.tf[r] - (double)ra.tn[r];
    const bool plain = H[r] > tau;
    float *e = ends[wv];
    if (!plain) {
        const float pb = prob[(int64_t)r * NB + ln];
        const float c = wave_incl(pb);
        pm_s[wv][ln] = pb;
        cdf_s[wv][ln + 1] = c;
        if (ln == 0) cdf_s[wv][0] = 0.f;
        __threadfence_block();
        const float total = cdf_s[wv][NB];
        for (int jj = ln; jj <= n; jj += 64) e[jj] = inv_cdf(cdf_s[wv], pm_s[wv], (float)jj / (float)n * total, total);
        __threadfence_block();
    }
    for (int jj = ln; jj < n; jj += 64) {
        float sm, sl;
        if (plain) {
            sm = ((float)jj + 0.5f) / (float)n;
            sl = 1.f / (float)n;
        } else {
            sm = 0.5f * (e[jj] + e[jj + 1]);
            sl = e[jj + 1] - e[jj];
        }
        const int64_t k = beg + jj;
        const double t = a + (double)sm * len;
        xyz[3 * k] = (float)((double)ra.o[3 * r] + t * (double)ra.d[3 * r]);
        xyz[3 * k + 1] = (float)((double)ra.o[3 * r + 1] + t * (double)ra.d[3 * r + 1]);
        xyz[3 * k + 2] = (float)((double)ra.o[3 * r + 2] + t * (double)ra.d[3 * r + 2]);
        s_mid[k] = sm;
        s_len[k] = sl;
        delta[k] = (float)((double)sl * len / (double)voxel);
    }
}

// Guarded resampling: the coarse bins the coarse pass found occupied (its weight, or a
// neighbour's, at least w_min) are cut into n_base sub-intervals plus a share of n_extra allotted
// by the predicted probabilities; unoccupied bins get none.  One wave per ray, lane = bin for the
// occupancy test; lane 0 then allots the extras in bin order with a running double sum, so the
// integers equal those of a sequential evaluation (round(x) = floor(x + 1/2) of n_extra S_b/S_tot,
// differenced).  counts [R,64] is written; offs[r+1] receives the ray's total for the scan below.
constexpr int MAX_PER_BIN = 1 << 14;

__global__ __launch_bounds__(256) void guard_count_kernel(RayArgs ra, const float *prob, const float *wc,
                                                          const float *H, float tau, int n_base, int n_extra,
                                                          float w_min, int *counts, int *offs) {
    __shared__ int occ_s[4][NB];
    __shared__ float p_s[4][NB];
    const int wv = threadIdx.x >> 6, r = blockIdx.x * 4 + wv, ln = lane();
    if (r >= ra.R) return;
    int m = 0;
    if (ra.tf[r] > ra.tn[r]) {
        if (H[r] > tau) {
            m = n_base;
        } else {
            const float w = wc[(int64_t)r * NB + ln];
            const float wl = __shfl_up(w, 1, 64), wr = __shfl_down(w, 1, 64);
            float mx = w;
            if (ln > 0 && wl > mx) mx = wl;
            if (ln < NB - 1 && wr > mx) mx = wr;
            occ_s[wv][ln] = mx >= w_min ? 1 : 0;
            p_s[wv][ln] = prob[(int64_t)r * NB + ln];
            __threadfence_block();
            if (ln == 0) {
                double S_tot = 0.0;
                int n_occ = 0;
                for (int b = 0; b < NB; ++b)
                    if (occ_s[wv][b]) {
                        S_tot += (double)p_s[wv][b];
                        ++n_occ;
                    }
                const bool uniform = !(S_tot > 0.0);
                if (uniform) S_tot = (double)n_occ;
                double S = 0.0;
                for (int b = 0; b < NB; ++b) {
                    int mb = 0;
                    if (occ_s[wv][b]) {
                        const double lo = floor((double)n_extra * (S / S_tot) + 0.5);
                        S += uniform ? 1.0 : (double)p_s[wv][b];
                        const double hi = floor((double)n_extra * (S / S_tot) + 0.5);
                        mb = n_base + (int)(hi - lo);
                    }
                    occ_s[wv][b] = mb;  // the bin's count, read back by its lane below
                }
            }
            __threadfence_block();
            m = occ_s[wv][ln];
        }
    }
    counts[(int64_t)r * NB + ln] = m;
    int tot = m;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) tot += __shfl_xor(tot, d, 64);
    if (ln == 0) offs[r + 1] = tot;
}

// offs[0] = 0, offs[1..R] = inclusive prefix of the per-ray totals left there (one block)
__global__ __launch_bounds__(1024) void guard_scan_kernel(int R, int *offs) {
    __shared__ int wsum[16];
    __shared__ int carry;
    if (threadIdx.x == 0) {
        carry = 0;
        offs[0] = 0;
    }
    __syncthreads();
    for (int base = 0; base < R; base += 1024) {
        const int r = base + threadIdx.x;
        int v = r < R ? offs[r + 1] : 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(v, d, 64);
            if (lane() >= d) v += t;
        }
        if (lane() == 63) wsum[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x < 16) {
            int t = wsum[threadIdx.x];
#pragma unroll
            for (int d = 1; d < 16; d <<= 1) {
                const int u = __shfl_up(t, d, 16);
                if ((int)threadIdx.x >= d) t += u;
            }
            wsum[threadIdx.x] = t;
        }
        __syncthreads();
        const int wave_off = (threadIdx.x >> 6) ? wsum[(threadIdx.x >> 6) - 1] : 0;
        if (r < R) offs[r + 1] = carry + wave_off + v;
        __syncthreads();
        if (threadIdx.x == 0) carry += wsum[15];
        __syncthreads();
    }
}

// one wave per ray, lane = bin: sub-interval i of bin b cut into m sits at
// s = (b + (i + 1/2)/m)/64, length 1/(64 m); positions formed in double
__global__ __launch_bounds__(256) void guard_fill_kernel(RayArgs ra, const int *offs, const int *counts, float voxel,
                                                         float *xyz, float *delta, float *s_mid, float *s_len) {
    const int wv = threadIdx.x >> 6, r = blockIdx.x * 4 + wv, ln = lane();
    if (r >= ra.R) return;
    const int m = counts[(int64_t)r * NB + ln];
    const int incl = [&] {
        int v = m;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(v, d, 64);
            if (ln >= d) v += t;
        }
        return v;
    }();
    const int64_t k0 = (int64_t)offs[r] + (incl - m);
    const double a = ra.tn[r], len = (double)ra.tf[r] - (double)ra.tn[r];
    for (int i = 0; i < m; ++i) {
        const int64_t k = k0 + i;
        const double sm = ((double)ln + ((double)i + 0.5) / (double)m) / (double)NB;
        const double sl = 1.0 / ((double)NB * (double)m);
        const double t = a + sm * len;
        xyz[3 * k] = (float)((double)ra.o[3 * r] + t * (double)ra.d[3 * r]);
        xyz[3 * k + 1] = (float)((double)ra.o[3 * r + 1] + t * (double)ra.d[3 * r + 1]);
        xyz[3 * k + 2] = (float)((double)ra.o[3 * r + 2] + t * (double)ra.d[3 * r + 2]);
        s_mid[k] = (float)sm;
        s_len[k] = (float)sl;
        delta[k] = (float)(sl * len / (double)voxel);
    }
}

// ------------------------------------------------------------------- host side

int check_prop(const dvgo_proposal *p, bool bwd) {
    if (!p) return set_error(DVGO_ERR_NULL, "proposal is NULL");
    if (p->struct_size != sizeof(dvgo_proposal)) return set_error(DVGO_ERR_ABI, "dvgo_proposal.struct_size mismatch");
    if (p->n_bins != NB || p->hidden != NB || p->n_layers != NL)
        return set_error(DVGO_ERR_UNSUPPORTED, "proposal must be 64 bins, 64 hidden, 4 linear layers");
    for (int l = 0; l < NL; ++l) {
        if (!p->W[l] || !p->b[l]) return set_error(DVGO_ERR_NULL, "proposal weight %d is NULL", l);
        if (bwd && (!p->gW[l] || !p->gb[l])) return set_error(DVGO_ERR_NULL, "proposal gradient %d is NULL", l);
    }
    return DVGO_OK;
}

void fill_prop(const dvgo_proposal *p, PropArgs &a) {
    memset(&a, 0, sizeof(a));
    for (int l = 0; l < NL; ++l) {
        a.W[l] = p->W[l];
        a.b[l] = p->b[l];
        a.gW[l] = p->gW[l];
        a.gb[l] = p->gb[l];
    }
}

int prop_blocks(int R) {
    const int t = (R + TILE - 1) / TILE;
    return t < 1 ? 1 : (t < MAX_BLOCKS ? t : MAX_BLOCKS);
}

int check_rays(const dvgo_rays *rays) {
    if (!rays) return set_error(DVGO_ERR_NULL, "rays is NULL");
    if (rays->struct_size != sizeof(dvgo_rays)) return set_error(DVGO_ERR_ABI, "dvgo_rays.struct_size mismatch");
    if (rays->n_rays < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays");
    if (rays->n_rays > 0 && (!rays->origins || !rays->dirs || !rays->t_near || !rays->t_far))
        return set_error(DVGO_ERR_NULL, "a ray array is NULL");
    return DVGO_OK;
}

RayArgs ray_args(const dvgo_rays *rays) {
    return RayArgs{rays->n_rays, rays->origins, rays->dirs, rays->t_near, rays->t_far};
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

extern "C" int dvgo_proposal_coarse(const dvgo_rays *rays, const dvgo_grid *density, float act_shift, float voxel,
                                    float eps, float *feat, float *w_coarse, void *stream) {
    int rc = check_rays(rays);
    if (rc) return rc;
    DevGrid dg;
    rc = make_dev_grid(density, "density", &dg, false);
    if (rc) return rc;
    if (rays->n_rays == 0) return DVGO_OK;
    if (!feat) return set_error(DVGO_ERR_NULL, "feat is NULL");
    if (!(voxel > 0.f) || !(eps > 0.f)) return set_error(DVGO_ERR_RANGE, "voxel and eps must be positive");
    hipLaunchKernelGGL(coarse_kernel, dim3((rays->n_rays + 3) / 4), dim3(256), 0, (hipStream_t)stream, ray_args(rays),
                       dg, act_shift, voxel, eps, feat, w_coarse);
    return check_hip(hipGetLastError(), "coarse_kernel launch");
}

extern "C" int dvgo_proposal_forward(const dvgo_proposal *p, int32_t n_rays, const float *feat, float *logits,
                                     float *prob, float *entropy, void *stream) {
    int rc = check_prop(p, false);
    if (rc) return rc;
    if (n_rays < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays");
    if (n_rays == 0) return DVGO_OK;
    if (!feat || (!logits && !prob && !entropy)) return set_error(DVGO_ERR_NULL, "feat or every output is NULL");
    if (!aligned16(feat) || (logits && !aligned16(logits)) || (prob && !aligned16(prob)))
        return set_error(DVGO_ERR_SHAPE, "feat, logits and prob must be 16-byte aligned");
    PropArgs a;
    fill_prop(p, a);
    a.R = n_rays;
    a.x = feat;
    a.logits = logits;
    a.prob = prob;
    a.entropy = entropy;
    hipLaunchKernelGGL(prop_fwd_kernel, dim3(prop_blocks(n_rays)), dim3(THREADS), 0, (hipStream_t)stream, a);
    return check_hip(hipGetLastError(), "prop_fwd_kernel launch");
}

extern "C" int dvgo_proposal_workspace_size(const dvgo_proposal *p, int32_t n_rays, size_t *bytes) {
    int rc = check_prop(p, false);
    if (rc) return rc;
    if (!bytes) return set_error(DVGO_ERR_NULL, "bytes is NULL");
    if (n_rays < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays");
    *bytes = (size_t)prop_blocks(n_rays) * (NPARAM + 1) * sizeof(float);
    return DVGO_OK;
}

extern "C" int dvgo_proposal_backward(const dvgo_proposal *p, int32_t n_rays, const float *feat, const float *target,
                                      float *loss, void *ws, size_t ws_bytes, void *stream) {
    int rc = check_prop(p, true);
    if (rc) return rc;
    if (n_rays < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays");
    if (n_rays == 0) return DVGO_OK;
    if (!feat || !target) return set_error(DVGO_ERR_NULL, "feat or target is NULL");
    if (!aligned16(feat) || !aligned16(target)) return set_error(DVGO_ERR_SHAPE, "feat and target must be 16-byte aligned");
    const size_t need = (size_t)prop_blocks(n_rays) * (NPARAM + 1) * sizeof(float);
    if (!ws || ws_bytes < need) return set_error(DVGO_ERR_WORKSPACE, "workspace too small (%zu < %zu)", ws_bytes, need);
    PropArgs a;
    fill_prop(p, a);
    a.R = n_rays;
    a.x = feat;
    a.target = target;
    a.loss = loss;
    a.partial = (float *)ws;
    a.nblocks = prop_blocks(n_rays);
    hipLaunchKernelGGL(prop_bwd_kernel, dim3(a.nblocks), dim3(THREADS), 0, (hipStream_t)stream, a);
    rc = check_hip(hipGetLastError(), "prop_bwd_kernel launch");
    if (rc) return rc;
    hipLaunchKernelGGL(prop_reduce_kernel, dim3((NPARAM + 1 + 255) / 256), dim3(256), 0, (hipStream_t)stream, a);
    return check_hip(hipGetLastError(), "prop_reduce_kernel launch");
}

extern "C" int dvgo_histogram(int32_t n_rays, const int32_t *ray_offsets, const float *w, const float *s_mid,
                              int32_t n_bins, float min_mass, float *hist, void *stream) {
    if (n_bins != NB) return set_error(DVGO_ERR_UNSUPPORTED, "n_bins must be %d", NB);
    if (n_rays < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays");
    if (n_rays == 0) return DVGO_OK;
    if (!ray_offsets || !hist) return set_error(DVGO_ERR_NULL, "ray_offsets or hist is NULL");
    hipLaunchKernelGGL(histogram_kernel, dim3((n_rays + 3) / 4), dim3(256), 0, (hipStream_t)stream, n_rays, ray_offsets,
                       w, s_mid, min_mass, hist);
    return check_hip(hipGetLastError(), "histogram_kernel launch");
}

extern "C" int dvgo_resample_offsets(const dvgo_rays *rays, const float *entropy, float tau, int32_t n_fine,
                                     int32_t n_plain, int32_t *ray_offsets, void *stream) {
    int rc = check_rays(rays);
    if (rc) return rc;
    if (n_fine < 1 || n_fine > 256 || n_plain < 1) return set_error(DVGO_ERR_RANGE, "need 1 <= n_fine <= 256, n_plain >= 1");
    if (!ray_offsets || (rays->n_rays > 0 && !entropy)) return set_error(DVGO_ERR_NULL, "entropy or ray_offsets is NULL");
    if ((int64_t)rays->n_rays * (n_fine > n_plain ? n_fine : n_plain) >= ((int64_t)1 << 31))
        return set_error(DVGO_ERR_RANGE, "batch would exceed 2^31 samples");
    hipLaunchKernelGGL(resample_offsets_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, rays->n_rays,
                       rays->t_near, rays->t_far, entropy, tau, n_fine, n_plain, ray_offsets);
    return check_hip(hipGetLastError(), "resample_offsets_kernel launch");
}

extern "C" int dvgo_resample(const dvgo_rays *rays, const float *prob, const float *entropy, float tau,
                             const int32_t *ray_offsets, int32_t n_fine, int32_t n_plain, float voxel, float *xyz,
                             float *delta, float *s_mid, float *s_len, void *stream) {
    int rc = check_rays(rays);
    if (rc) return rc;
    if (n_fine < 1 || n_fine > 256 || n_plain < 1) return set_error(DVGO_ERR_RANGE, "need 1 <= n_fine <= 256, n_plain >= 1");
    if (rays->n_rays == 0) return DVGO_OK;
    if (!prob || !entropy || !ray_offsets || !xyz || !delta || !s_mid || !s_len)
        return set_error(DVGO_ERR_NULL, "an argument array is NULL");
    if (!(voxel > 0.f)) return set_error(DVGO_ERR_RANGE, "voxel must be positive");
    hipLaunchKernelGGL(resample_fill_kernel, dim3((rays->n_rays + 3) / 4), dim3(256), 0, (hipStream_t)stream,
                       ray_args(rays), prob, entropy, tau, ray_offsets, n_fine, n_plain, voxel, xyz, delta, s_mid, s_len);
    return check_hip(hipGetLastError(), "resample_fill_kernel launch");
}

extern "C" int dvgo_resample_guarded_offsets(const dvgo_rays *rays, const float *prob, const float *w_coarse,
                                             const float *entropy, float tau, int32_t n_base, int32_t n_extra,
                                             float w_min, int32_t *ray_offsets, int32_t *counts, void *stream) {
    int rc = check_rays(rays);
    if (rc) return rc;
    if (n_base < 1 || n_extra < 0 || n_base + n_extra > MAX_PER_BIN)
        return set_error(DVGO_ERR_RANGE, "need n_base >= 1, n_extra >= 0, n_base + n_extra <= %d", MAX_PER_BIN);
    if ((int64_t)rays->n_rays * (NB * (int64_t)n_base + n_extra) >= ((int64_t)1 << 31))
        return set_error(DVGO_ERR_RANGE, "batch could exceed 2^31 samples");
    if (!ray_offsets) return set_error(DVGO_ERR_NULL, "ray_offsets is NULL");
    if (rays->n_rays > 0 && (!prob || !w_coarse || !entropy || !counts))
        return set_error(DVGO_ERR_NULL, "prob, w_coarse, entropy or counts is NULL");
    const hipStream_t st = (hipStream_t)stream;
    if (rays->n_rays > 0)
        hipLaunchKernelGGL(guard_count_kernel, dim3((rays->n_rays + 3) / 4), dim3(256), 0, st, ray_args(rays), prob,
                           w_coarse, entropy, tau, n_base, n_extra, w_min, counts, ray_offsets);
    hipLaunchKernelGGL(guard_scan_kernel, dim3(1), dim3(1024), 0, st, rays->n_rays, ray_offsets);
    return check_hip(hipGetLastError(), "guarded resampling offsets launch");
}

extern "C" int dvgo_resample_guarded(const dvgo_rays *rays, const int32_t *ray_offsets, const int32_t *counts,
                                     float voxel, float *xyz, float *delta, float *s_mid, float *s_len,
                                     void *stream) {
    int rc = check_rays(rays);
    if (rc) return rc;
    if (rays->n_rays == 0) return DVGO_OK;
    if (!ray_offsets || !counts || !xyz || !delta || !s_mid || !s_len)
        return set_error(DVGO_ERR_NULL, "an argument array is NULL");
    if (!(voxel > 0.f)) return set_error(DVGO_ERR_RANGE, "voxel must be positive");
    hipLaunchKernelGGL(guard_fill_kernel, dim3((rays->n_rays + 3) / 4), dim3(256), 0, (hipStream_t)stream,
                       ray_args(rays), ray_offsets, counts, voxel, xyz, delta, s_mid, s_len);
    return check_hip(hipGetLastError(), "guard_fill_kernel launch");
}
