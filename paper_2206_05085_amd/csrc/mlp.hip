// Colour MLP of the hybrid representation (Table 1): [features, view encoding] -> 128 ->
// 128 -> RGB, forward and backward on gfx950 FP16 matrix cores with FP32-grade products.
//
// Split precision.  Every matrix operand v is held as two FP16 parts scaled by a power of
// two, v 2^e = hi + lo with hi = fp16(v 2^e) and lo = fp16(v 2^e - hi), and a product is
// taken as hi*hi' + hi*lo' + lo*hi' (three v_mfma_f32_16x16x32_f16 into one FP32
// accumulator).  The dropped lo*lo' term and the rounding of lo leave a relative error near
// 2^-22 per product.  The power of two keeps operands inside the FP16 normal range: weight
// matrices use one exponent each (largest entry just under 2^14); an activation column (one
// sample) uses an exponent from a bound on its magnitude that every wave can evaluate on
// its own (infinity norms of the weights times the sample's input or upstream gradient).
// Accumulators are brought back to true scale with v_ldexp, which is exact.
//
// Layout.  A 16x16 accumulator tile holds 16 hidden units (rows) x 16 samples (columns);
// lane (q = lane/16, j = lane%16) owns rows 4q..4q+3 of column j.  A K-step of 32 reads
// the lane's 8 operand slots (q, e) as logical index k(kk, q, e) = 32 kk + 4 q + e (e < 4)
// or 32 kk + 16 + 4 q + (e - 4) (e >= 4), so two consecutive row tiles of one layer's
// output are the next layer's B operand without any data movement.  Weight rows are
// stored with their columns in that slot order ("phys" order), so an A operand is one
// 16-byte read per part.
//
// Forward: each wave owns 16 NC samples and all 128 hidden units; W1 and W2 (both parts)
// sit in LDS.  Backward: a block's waves own slices of 16 BWD_MP hidden units for the block's
// 32-sample tiles and keep their rows of W1, W2 or W2^T in registers (two roles, see the
// backward section); activations are exchanged through sample-major LDS planes.  The weight
// gradients reduce over samples, so their unit-major operands are read from those planes with
// transposing LDS reads; their accumulators carry a power-of-two frame that only ever decreases
// (rescaled when a tile needs it), and a sample's operands are scaled so that the product lands
// in that frame.
#include <string.h>

#include "dvgo_internal.h"

using namespace dvgo;

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));

constexpr int H = 128;      // hidden width
constexpr int KX = 64;      // padded input width: features 0..11, view encoding 12..47, zeros 48..63
constexpr int PEW = 36;     // per-ray encoding row (input columns 12..47)
constexpr int RS1 = 72;     // row stride (halves) of a 64-wide operand row
constexpr int RS2 = 136;    // row stride (halves) of a 128-wide operand row
constexpr int MAXE = 100;   // clamp of scaling exponents
constexpr int FRAME_NONE = 1 << 20;
constexpr int MAX_BLOCKS = 256;

// ---- weight image (written by mlp_prep_kernel into the workspace) ----
// W2 comes first so that every W2 read of the forward kernel reaches its LDS copy with one
// base register and a 16-bit immediate offset.
constexpr int IMG_W2H = 0;
constexpr int IMG_W2L = IMG_W2H + H * RS2 * 2;
constexpr int IMG_W1H = IMG_W2L + H * RS2 * 2;   // start of the part the backward kernel stages
constexpr int IMG_W1L = IMG_W1H + H * RS1 * 2;
constexpr int IMG_B1 = IMG_W1L + H * RS1 * 2;
constexpr int IMG_B2 = IMG_B1 + H * 4;
constexpr int IMG_W3 = IMG_B2 + H * 4;
constexpr int IMG_B3 = IMG_W3 + 3 * H * 4;
constexpr int IMG_META = IMG_B3 + 16;
constexpr int IMG_FWD_END = IMG_META + 48;  // end of the forward kernel's LDS image
constexpr int IMG_W2TH = IMG_FWD_END;
constexpr int IMG_W2TL = IMG_W2TH + H * RS2 * 2;
constexpr int IMG_W1FH = IMG_W2TL + H * RS2 * 2;
constexpr int IMG_W1FL = IMG_W1FH + 16 * RS2 * 2;
constexpr int IMG_BYTES = IMG_W1FL + 16 * RS2 * 2;
static_assert(IMG_W1H % 16 == 0 && IMG_FWD_END % 16 == 0 && IMG_BYTES % 16 == 0, "image alignment");

struct Meta {
    int sw1, sw2;           // weight exponents of W1 and W2 (W2^T shares sw2, W1F shares sw1)
    float n1, b1max;        // max_i sum_k |W1[i][k]|, max |b1|
    float n2t, n3t;         // max_in sum_out |W2[out][in]|, max_h sum_o |W3[o][h]|
    int pad[6];
};
static_assert(sizeof(Meta) == 48, "meta size");

__host__ __device__ constexpr int kidx(int kk, int q, int e) {
    return 32 * kk + (e < 4 ? 4 * q + e : 16 + 4 * q + (e - 4));
}

__device__ __forceinline__ v4f mfma16(h8 a, h8 b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// exponent e with |v| 2^e < 2^14 for every |v| <= m
__device__ __forceinline__ int scale_exp(float m) {
    int k;
    frexpf(m, &k);
    const int e = 14 - k;
    return e < -MAXE ? -MAXE : (e > MAXE ? MAXE : e);
}

// exponent k with m < 2^k (FRAME_NONE - style "no constraint" handled by callers for m == 0)
__device__ __forceinline__ int ceil_exp(float m) {
    int k;
    frexpf(m, &k);
    return k;
}

// hi and lo parts of two values in packed halves: hi = fp16(t0), fp16(t1) from one packed
// conversion (round to nearest even, as every float -> half conversion here), lo = fp16(t - hi)
// of each from one mixed-precision FMA that writes its half of the register directly (t - hi is
// exact in FP32, so each equals (_Float16)(t - (float)hi)).  The compiler's hazard tracking does
// not see these as vector-ALU writes, and a matrix instruction may read a vector register only two
// wait states after a vector-ALU instruction wrote it: with MM (the results feed a product
// directly) the block ends with those two (s_nop 1); results that only go to LDS stores need none.
template <bool MM>
__device__ __forceinline__ void split2(float t0, float t1, unsigned &hi, unsigned &lo) {
    if (MM)
        asm("v_cvt_pk_f16_f32 %0, %2, %3\n\t"
            "v_fma_mixlo_f16 %1, %2, 1.0, -%0 op_sel_hi:[0,0,1]\n\t"
            "v_fma_mixhi_f16 %1, %3, 1.0, -%0 op_sel:[0,0,1] op_sel_hi:[0,0,1]\n\t"
            "s_nop 1"
            : "=&v"(hi), "=&v"(lo)
            : "v"(t0), "v"(t1));
    else
        asm("v_cvt_pk_f16_f32 %0, %2, %3\n\t"
            "v_fma_mixlo_f16 %1, %2, 1.0, -%0 op_sel_hi:[0,0,1]\n\t"
            "v_fma_mixhi_f16 %1, %3, 1.0, -%0 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
            : "=&v"(hi), "=&v"(lo)
            : "v"(t0), "v"(t1));
}

// MM: the parts feed a matrix product directly (see split2)
template <bool MM>
__device__ __forceinline__ void split4(const float v[4], float sc, h4 &hi, h4 &lo) {
    uint2 h, l;
    split2<MM>(v[0] * sc, v[1] * sc, h.x, l.x);
    split2<MM>(v[2] * sc, v[3] * sc, h.y, l.y);
    hi = __builtin_bit_cast(h4, h);
    lo = __builtin_bit_cast(h4, l);
}

__device__ __forceinline__ h8 cat(h4 a, h4 b) { return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7); }

// logistic function with the hardware exponential and reciprocal (about 1e-7 relative; the
// limits are exact: 1/(1 + inf) = 0 and 1/(1 + 0) = 1)
__device__ __forceinline__ float fast_sigmoid(float z) { return __builtin_amdgcn_rcpf(1.f + __expf(-z)); }

// Reductions over aligned lane groups with DPP moves (no LDS round trip).  quad_perm [1,0,3,2]
// and [2,3,0,1] reduce each quad; row_half_mirror (lane i of an 8-lane half-row reads lane
// 7 - i) joins the two quads of a half-row; row_mirror (15 - i) joins the halves of a row.
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_movf(float v) {
    return __builtin_bit_cast(float, dpp_mov<CTRL>(__builtin_bit_cast(int, v)));
}
// min over the 16 lanes of each row
__device__ __forceinline__ int row16_min(int v) {
    v = min(v, dpp_mov<0xB1>(v));
    v = min(v, dpp_mov<0x4E>(v));
    v = min(v, dpp_mov<0x141>(v));
    return min(v, dpp_mov<0x140>(v));
}
// max over each aligned group of 8 lanes
__device__ __forceinline__ float group8_max(float v) {
    v = fmaxf(v, dpp_movf<0xB1>(v));
    v = fmaxf(v, dpp_movf<0x4E>(v));
    return fmaxf(v, dpp_movf<0x141>(v));
}

__device__ __forceinline__ float pow2(int e) { return __builtin_amdgcn_ldexpf(1.f, e); }
__device__ __forceinline__ float ldx(float v, int e) { return __builtin_amdgcn_ldexpf(v, e); }

struct MlpArgs {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    int in_feat, n_in;  // n_in = in_feat + 3 + 6 F (columns of W1)
    int n_freq;
    int n_rays;
    const int *offs;
    const float *dirs;
    int S;
    const float *feat;
    int feat_vec;        // in_feat == 12 and feat 16-byte aligned: rows load as float4
    float *rgb;
    unsigned char *img;  // weight image (workspace)
    float *pe;           // [R][PEW] view encodings (workspace)
    int *tile_ray;       // [ceil(S/32)] ray of the first sample of each 32-sample tile (workspace)
    int n_tiles;         // ceil(S/32)
    const float *grad_rgb;
    float *grad_feat;
    float *partial;  // [blocks][n_params] (workspace)
    int n_params;
    float *gW1, *gb1, *gW2, *gb2, *gW3, *gb3;
    int nblocks;
    // fused feature gather: the feature grid the forward looks the features up in, and the
    // sample points
    DevGrid fg;
    const float *xyz;
    float *feat_out;  // forward with the gather: the features it used, [S][in_feat] (may be NULL)
};

// padded input column k -> column of W1 (or -1 for padding)
__host__ __device__ __forceinline__ int w1_col(int in_feat, int n_freq, int k) {
    if (k < 12) return k < in_feat ? k : -1;
    const int p = k - 12;
    return p < 3 + 6 * n_freq ? in_feat + p : -1;
}

// ------------------------------------------------------------------ preparation

constexpr int TILE = 32;   // samples per wave tile (forward) and per block tile (backward)

// ray of sample s: the last r with offs[r] <= s (rays may be empty)
__device__ __forceinline__ int find_ray(const int *offs, int R, int s) {
    int lo = 0, hi = R - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= s) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The same search for a sample of the 32-sample tile whose first sample lies on ray r0:
// every lane of the wave holds w = offs[min(r0 + lane, R)] and the search runs over the
// 64-entry window with shuffles; a sample beyond the window falls back to find_ray.  All
// 64 lanes must call it (the shuffles read every lane).
__device__ __forceinline__ int ray_in_window(const int *offs, int R, int r0, int w, int s) {
    int lo = 0, hi = 63;
#pragma unroll
    for (int it = 0; it < 6; ++it) {
        const int mid = (lo + hi + 1) >> 1;
        const int v = __shfl(w, mid, 64);
        if (v <= s) lo = mid; else hi = mid - 1;
    }
    if (lo == 63 && r0 + 64 <= R && offs[r0 + 64] <= s) return find_ray(offs, R, s);
    return r0 + lo;
}

// The same ray for the 8 consecutive samples sbase + (lane >> 3) of a wave (sbase wave-uniform
// and at or after offs[r0]): per sample, a ballot counts the window entries at or before it
// (a prefix, as offs is non-decreasing), so no lane-to-lane round trips are needed.  All 64
// lanes must call it.
__device__ __forceinline__ int ray_of_group8(const int *offs, int R, int r0, int w, int sbase) {
    const int k = lane() >> 3;
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int c = __popcll(__ballot(w <= sbase + i));
        cnt = k == i ? c : cnt;
    }
    const int s = sbase + k;
    if (cnt == 64 && r0 + 64 <= R && offs[r0 + 64] <= s) return find_ray(offs, R, s);
    return r0 + cnt - 1;
}

__device__ __forceinline__ int window_entry(const int *offs, int R, int r0) {
    const int i = r0 + lane();
    return offs[i < R ? i : R];
}

__device__ float block_max(float v, float *red) {
    // blockDim.x is a multiple of 64 and at most 1024
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if (lane() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float m = 0.f;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) m = fmaxf(m, red[i]);
    return m;
}

__device__ __forceinline__ void put_split(unsigned char *img, int off_h, int off_l, int idx, float v, float sc) {
    const float t = v * sc;
    const _Float16 h = (_Float16)t;
    reinterpret_cast<_Float16 *>(img + off_h)[idx] = h;
    reinterpret_cast<_Float16 *>(img + off_l)[idx] = (_Float16)(t - (float)h);
}

// logical index of phys slot p of a 128- or 64-wide operand row
__device__ __forceinline__ int phys_to_k(int p) { return kidx(p >> 5, (p >> 3) & 3, p & 7); }

constexpr int PREP_THREADS = 512;
constexpr int PREP_W2_BLOCKS = 16;  // 8 rows of W2 and of W2^T each
constexpr int PREP_W1_BLOCKS = 4;   // 32 rows of W1 each (block 0 of them also W1F, b1, b3)
constexpr int PREP_FIXED_BLOCKS = PREP_W2_BLOCKS + PREP_W1_BLOCKS + 1;

// blocks [0, 16): W2 and W2^T planes; every one of them also reduces max|W2| and the column
// sums of |W2| from the same loads (block 0 stores sw2 and n2t).  Blocks [16, 20): W1 planes,
// max|W1| and the row sums of |W1| (block 16 stores sw1, n1, b1max and writes W1F, b1, b3).
// Block 20: W3, b2, n3t.  Then view encodings (one ray per thread) and tile start rays.
__global__ __launch_bounds__(PREP_THREADS) void mlp_prep_kernel(MlpArgs a) {
    __shared__ float red[PREP_THREADS / 64];
    __shared__ float sums[PREP_THREADS];
    unsigned char *img = a.img;
    Meta *meta = reinterpret_cast<Meta *>(img + IMG_META);
    const int tid = threadIdx.x, b = blockIdx.x;
    const int pe_blocks = (a.n_rays + PREP_THREADS - 1) / PREP_THREADS;
    if (b < PREP_W2_BLOCKS) {
        // element i = tid + 512 k sits in column tid % 128 (512 is a multiple of H)
        float m = 0.f, cs = 0.f;
#pragma unroll 8
        for (int i = tid; i < H * H; i += PREP_THREADS) {
            const float v = fabsf(a.W2[i]);
            m = fmaxf(m, v);
            cs += v;
        }
        sums[tid] = cs;
        const int sw = scale_exp(block_max(m, red));  // its barriers also order the sums
        float n2t = 0.f;
        if (b == 0) {
            const float col = tid < H ? sums[tid] + sums[tid + H] + sums[tid + 2 * H] + sums[tid + 3 * H] : 0.f;
            n2t = block_max(col, red);
        }
        const float sc = pow2(sw);
        for (int i = tid; i < 8 * RS2; i += PREP_THREADS) {
            const int row = 8 * b + i / RS2, p = i % RS2;
            const int k = p < H ? phys_to_k(p) : -1;
            put_split(img, IMG_W2H, IMG_W2L, row * RS2 + p, k >= 0 ? a.W2[row * H + k] : 0.f, sc);
            put_split(img, IMG_W2TH, IMG_W2TL, row * RS2 + p, k >= 0 ? a.W2[k * H + row] : 0.f, sc);
        }
        if (b == 0 && tid == 0) {
            meta->sw2 = sw;
            meta->n2t = n2t;
        }
    } else if (b < PREP_W2_BLOCKS + PREP_W1_BLOCKS) {
        const int wb = b - PREP_W2_BLOCKS;
        if (tid < H) sums[tid] = 0.f;
        __syncthreads();
        float m = 0.f;
        for (int i = tid; i < H * a.n_in; i += PREP_THREADS) {
            const float v = fabsf(a.W1[i]);
            m = fmaxf(m, v);
            atomicAdd(&sums[i / a.n_in], v);
        }
        const int sw = scale_exp(block_max(m, red));
        const float sc = pow2(sw);
        for (int i = tid; i < 32 * RS1; i += PREP_THREADS) {
            const int row = 32 * wb + i / RS1, p = i % RS1;
            const int c = p < KX ? w1_col(a.in_feat, a.n_freq, phys_to_k(p)) : -1;
            put_split(img, IMG_W1H, IMG_W1L, row * RS1 + p, c >= 0 ? a.W1[row * a.n_in + c] : 0.f, sc);
        }
        if (wb == 0) {
            const float n1 = block_max(tid < H ? sums[tid] : 0.f, red);
            const float b1max = block_max(tid < H ? fabsf(a.b1[tid]) : 0.f, red);
            // W1F[c][phys over hidden] = W1[hidden][c] for the feature columns c < in_feat
            for (int i = tid; i < 16 * RS2; i += PREP_THREADS) {
                const int c = i / RS2, p = i % RS2;
                const int h = p < H ? phys_to_k(p) : -1;
                put_split(img, IMG_W1FH, IMG_W1FL, i, (h >= 0 && c < a.in_feat) ? a.W1[h * a.n_in + c] : 0.f, sc);
            }
            float *b1 = reinterpret_cast<float *>(img + IMG_B1);
            float *b3 = reinterpret_cast<float *>(img + IMG_B3);
            if (tid < H) b1[tid] = a.b1[tid];
            if (tid < 4) b3[tid] = tid < 3 ? a.b3[tid] : 0.f;
            if (tid == 0) {
                meta->sw1 = sw;
                meta->n1 = n1;
                meta->b1max = b1max;
            }
        }
    } else if (b == PREP_FIXED_BLOCKS - 1) {
        float *w3 = reinterpret_cast<float *>(img + IMG_W3);
        float *b2 = reinterpret_cast<float *>(img + IMG_B2);
        float cs = 0.f;
        for (int i = tid; i < 3 * H; i += PREP_THREADS) w3[i] = a.W3[i];
        if (tid < H) {
            b2[tid] = a.b2[tid];
            cs = fabsf(a.W3[tid]) + fabsf(a.W3[H + tid]) + fabsf(a.W3[2 * H + tid]);
        }
        const float n3t = block_max(cs, red);
        if (tid == 0) meta->n3t = n3t;
    } else if (b >= PREP_FIXED_BLOCKS + pe_blocks) {
        const int t = (b - PREP_FIXED_BLOCKS - pe_blocks) * PREP_THREADS + tid;
        if (t < a.n_tiles) a.tile_ray[t] = find_ray(a.offs, a.n_rays, TILE * t);
    } else {
        const int r = (b - PREP_FIXED_BLOCKS) * PREP_THREADS + tid;
        if (r < a.n_rays) {
            const float d[3] = {a.dirs[3 * r], a.dirs[3 * r + 1], a.dirs[3 * r + 2]};
            float *row = a.pe + (int64_t)r * PEW;
            for (int i = 0; i < PEW; ++i) row[i] = 0.f;
            for (int ax = 0; ax < 3; ++ax) row[ax] = d[ax];
            for (int f = 0; f < a.n_freq; ++f)
                for (int ax = 0; ax < 3; ++ax) {
                    const float v = ldexpf(d[ax], f);
                    row[3 + 3 * f + ax] = sinf(v);
                    row[3 + 3 * a.n_freq + 3 * f + ax] = cosf(v);
                }
        }
    }
}

// Pointer into a kernel's LDS block at byte offset `off`, with the offset hidden from the
// optimiser: accesses then share one base register and use the 16-bit immediate offset of
// ds_read/ds_write instead of one materialised address per constant offset above 64 KB.
__device__ __forceinline__ unsigned char *lds_region(unsigned char *sm, int off) {
    asm volatile("" : "+s"(off));
    return sm + off;
}

// A lane index the optimiser must treat as new in every loop iteration, so that address
// arithmetic built from it is recomputed next to its use (and folded into instruction
// offsets) instead of being hoisted out of the loop into long-lived registers.
__device__ __forceinline__ int fresh(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ float4 feat4(const MlpArgs &a, int s, int c0) {
    const float *fp = a.feat + (int64_t)s * a.in_feat;
    if (a.feat_vec) return *reinterpret_cast<const float4 *>(fp + c0);
    return make_float4(c0 < a.in_feat ? fp[c0] : 0.f, c0 + 1 < a.in_feat ? fp[c0 + 1] : 0.f,
                       c0 + 2 < a.in_feat ? fp[c0 + 2] : 0.f, c0 + 3 < a.in_feat ? fp[c0 + 3] : 0.f);
}

// The 8 inputs of operand slot group (kk, q) of a valid sample s on ray `ray`, features read
// from a.feat: logical columns k(kk, q, 0..7).  For kk = 0 these are features 4q..4q+3 (view
// encoding 0..3 when q = 3) and view encoding 4+4q..7+4q; for kk = 1 view encoding 20+4q..23+4q
// and padding.  (The kernels use it only for feature rows that cannot be read as float4.)
__device__ __forceinline__ void load_x8(const MlpArgs &a, int s, int ray, int kk, int q, float v[8]) {
    const float *pe = a.pe + (int64_t)ray * PEW;
    float4 lo, hi;
    if (kk == 0) {
        lo = q < 3 ? feat4(a, s, 4 * q) : *reinterpret_cast<const float4 *>(pe);
        hi = *reinterpret_cast<const float4 *>(pe + 4 + 4 * q);
    } else {
        lo = *reinterpret_cast<const float4 *>(pe + 20 + 4 * q);
        hi = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    v[0] = lo.x; v[1] = lo.y; v[2] = lo.z; v[3] = lo.w;
    v[4] = hi.x; v[5] = hi.y; v[6] = hi.z; v[7] = hi.w;
}

__device__ __forceinline__ void copy_to_lds(unsigned char *dst, const unsigned char *src, int bytes) {
    for (int i = threadIdx.x * 16; i < bytes; i += blockDim.x * 16)
        *reinterpret_cast<uint4 *>(dst + i) = *reinterpret_cast<const uint4 *>(src + i);
}

// ------------------------------------------------------------------ forward
//
// The forward's LDS copy of the weight image re-strides the FP16 weight rows.  On gfx950 the
// operand reads of a row tile (lane j reads row j, lane group q the 16 bytes at 16 q) run without
// bank conflicts when the row stride is 32 bytes more than a multiple of 64; the image's strides
// (272 and 144 bytes, which the backward's planes share) are 16 bytes more and read about 1.7x
// slower (measured with this read pattern in isolation: ~120 against ~205 bytes per clock per CU).
constexpr int FRS2 = 144;  // halves per W2 row in the forward's LDS (128 used)
constexpr int FRS1 = 80;   // halves per W1 row in the forward's LDS (64 used)
constexpr int F_W2H = 0;
constexpr int F_W2L = F_W2H + H * FRS2 * 2;
constexpr int F_W1H = F_W2L + H * FRS2 * 2;
constexpr int F_W1L = F_W1H + H * FRS1 * 2;
constexpr int F_SMALL = F_W1L + H * FRS1 * 2;          // b1, b2, W3, b3, meta, laid out as in the image
constexpr int F_END = F_SMALL + (IMG_FWD_END - IMG_B1);
static_assert((FRS2 * 2) % 64 == 32 && (FRS1 * 2) % 64 == 32 && F_SMALL % 16 == 0, "forward LDS strides");
static_assert(F_END <= 160 * 1024, "forward LDS block");

// rows of row_bytes (a multiple of 16) from src with stride sstride to dst with stride dstride
__device__ __forceinline__ void copy_rows_to_lds(unsigned char *dst, int dstride, const unsigned char *src,
                                                 int sstride, int rows, int row_bytes) {
    const int chunks = row_bytes / 16;
    for (int i = threadIdx.x; i < rows * chunks; i += blockDim.x) {
        const int r = i / chunks, c = i - r * chunks;
        *reinterpret_cast<uint4 *>(dst + r * dstride + 16 * c) =
            *reinterpret_cast<const uint4 *>(src + r * sstride + 16 * c);
    }
}

// Wave tiles of the forward: with the feature lookup inside (GM > 0) 16 samples per wave and 16
// waves per block, so four waves share each SIMD and hide the lookups' latency behind each other's
// products; with the features read from memory 32 samples per wave and 8 waves, which reuses each
// weight operand for two column tiles.
template <int GM>
struct FwdShape {
    static constexpr int NC = GM ? 1 : 2;       // 16-sample column tiles per wave tile
    static constexpr int WAVES = GM ? 16 : 8;   // waves per block
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int WTILE = 16 * NC;       // samples per wave tile
    static_assert(TILE % WTILE == 0, "forward wave tiles split the 32-sample tiles of tile_ray");
};

template <bool SPLIT, int GM>
__global__ __launch_bounds__(FwdShape<GM>::THREADS) void mlp_fwd_kernel(MlpArgs a) {
    constexpr int FWD_NC = FwdShape<GM>::NC, FWD_WAVES = FwdShape<GM>::WAVES, FWD_WTILE = FwdShape<GM>::WTILE;
    __shared__ __attribute__((aligned(16))) unsigned char sm[F_END];
    copy_rows_to_lds(sm + F_W2H, FRS2 * 2, a.img + IMG_W2H, RS2 * 2, H, H * 2);
    copy_rows_to_lds(sm + F_W2L, FRS2 * 2, a.img + IMG_W2L, RS2 * 2, H, H * 2);
    copy_rows_to_lds(sm + F_W1H, FRS1 * 2, a.img + IMG_W1H, RS1 * 2, H, 64 * 2);
    copy_rows_to_lds(sm + F_W1L, FRS1 * 2, a.img + IMG_W1L, RS1 * 2, H, 64 * 2);
    copy_to_lds(sm + F_SMALL, a.img + IMG_B1, IMG_FWD_END - IMG_B1);
    __syncthreads();
    const _Float16 *W2h = reinterpret_cast<const _Float16 *>(sm + F_W2H);
    const _Float16 *W2l = reinterpret_cast<const _Float16 *>(sm + F_W2L);
    const unsigned char *r1 = lds_region(sm, F_W1H);
    const _Float16 *W1h = reinterpret_cast<const _Float16 *>(r1);
    const _Float16 *W1l = reinterpret_cast<const _Float16 *>(r1 + (F_W1L - F_W1H));
    const unsigned char *rs = r1 + (F_SMALL - F_W1H);
    const float *b1 = reinterpret_cast<const float *>(rs);
    const float *b2 = reinterpret_cast<const float *>(rs + (IMG_B2 - IMG_B1));
    const float *W3 = reinterpret_cast<const float *>(rs + (IMG_W3 - IMG_B1));
    const float *b3 = reinterpret_cast<const float *>(rs + (IMG_B3 - IMG_B1));
    const Meta meta = *reinterpret_cast<const Meta *>(rs + (IMG_META - IMG_B1));
    const int ln = lane(), j = ln & 15, q = ln >> 4;
    const int nwt = (a.S + FWD_WTILE - 1) / FWD_WTILE;
    const int wt0 = blockIdx.x * FWD_WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wstep = gridDim.x * FWD_WAVES;
    if (wt0 >= nwt) return;
    // First ray of a wave tile's enclosing tile (past the last tile, the last tile's ray), read
    // through the scalar cache: the index is wave-uniform and the table is read-only here.
    const __attribute__((address_space(4))) int *tray = (const __attribute__((address_space(4))) int *)a.tile_ray;
    auto first_ray = [&](int wt) { return tray[(wt < nwt ? wt : nwt - 1) / (TILE / FWD_WTILE)]; };
    // sample points of a wave tile's feature lookups (the last sample's past the end)
    auto points = [&](int wt, float (&p)[FWD_NC][3]) {
#pragma unroll
        for (int c = 0; c < FWD_NC; ++c) {
            const int sp = min(wt * FWD_WTILE + 16 * c + j, a.S - 1);
#pragma unroll
            for (int d = 0; d < 3; ++d) p[c][d] = a.xyz[3 * (int64_t)sp + d];
        }
    };
    // The ray window entry and the sample points of the next tile are loaded one tile ahead,
    // so their latency runs behind the products of the tile before.
    // The output of a tile is stored at the head of the next one (after that tile's wait for its
    // prefetched values), so that the wait does not include the store.
    int r0 = first_ray(wt0);
    int win = window_entry(a.offs, a.n_rays, r0);
    int r0n = first_ray(wt0 + wstep);
    float pt[FWD_NC][3];
    if (GM) points(wt0, pt);
    float zout[FWD_NC];
    int sout[FWD_NC];
#pragma unroll
    for (int c = 0; c < FWD_NC; ++c) sout[c] = -1;
    auto store_out = [&]() {
#pragma unroll
        for (int c = 0; c < FWD_NC; ++c)
            if (q < 3 && sout[c] >= 0) a.rgb[(int64_t)sout[c] * 3 + q] = zout[c];
    };
    for (int wt = wt0; wt < nwt; wt += wstep) {
        int s[FWD_NC], ex[FWD_NC], e1[FWD_NC];
        bool sv[FWD_NC];
        h8 xh[FWD_NC][2], xl[FWD_NC][2];
        // this tile's inputs: every lane issues the same loads, with no divergent branch around them
        // (divergent branches would make one lane group's loads wait for another's).  Slot group
        // (kk, q): kk = 0 features 4q..4q+3 (view encoding 0..3 when q = 3) and view encoding
        // 4+4q..7+4q; kk = 1 view encoding 20+4q..23+4q and padding.
        float4 lo0[FWD_NC], hi0[FWD_NC], lo1[FWD_NC];
        int ray[FWD_NC];
#pragma unroll
        for (int c = 0; c < FWD_NC; ++c) {
            s[c] = wt * FWD_WTILE + 16 * c + j;
            sv[c] = s[c] < a.S;
            ray[c] = min(ray_in_window(a.offs, a.n_rays, r0, win, s[c]), a.n_rays - 1);
        }
        store_out();  // the previous tile's output
        // scalar load of a later tile's first ray, issued after the ray search so that the search's
        // LDS waits do not wait for it (used one tile later)
        const int r0f = first_ray(wt + 2 * wstep);
#pragma unroll
        for (int c = 0; c < FWD_NC; ++c) {
            const int sc = sv[c] ? s[c] : a.S - 1;
            const float *pe = a.pe + (int64_t)ray[c] * PEW;
            const float4 v0 = *reinterpret_cast<const float4 *>(pe);
            hi0[c] = *reinterpret_cast<const float4 *>(pe + 4 + 4 * q);
            lo1[c] = *reinterpret_cast<const float4 *>(pe + 20 + 4 * q);
            const bool fq = 4 * q < a.in_feat;  // never for q = 3 (at most 12 features)
            float4 f;
            if (GM) {
                const Tri t = trilinear<GM == 2>(a.fg, pt[c][0], pt[c][1], pt[c][2]);
                f = interp4(a.fg, t, fq ? 4 * q : 0);
                if (a.feat_out && fq && sv[c])
                    *reinterpret_cast<float4 *>(a.feat_out + (int64_t)s[c] * a.in_feat + 4 * q) = f;
            } else if (a.feat_vec) {
                f = *reinterpret_cast<const float4 *>(a.feat + (int64_t)sc * 12 + (fq ? 4 * q : 0));
            } else {
                f = fq ? feat4(a, sc, 4 * q) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
            lo0[c] = q == 3 ? v0 : (fq ? f : make_float4(0.f, 0.f, 0.f, 0.f));
        }
        // the next tile's ray window entry and sample points
        r0 = r0n;
        r0n = r0f;
        win = window_entry(a.offs, a.n_rays, r0);
        if (GM) points(wt + wstep, pt);
#pragma unroll
        for (int c = 0; c < FWD_NC; ++c) {
            const bool v = sv[c];
            const float xv[2][8] = {{v ? lo0[c].x : 0.f, v ? lo0[c].y : 0.f, v ? lo0[c].z : 0.f, v ? lo0[c].w : 0.f,
                                     v ? hi0[c].x : 0.f, v ? hi0[c].y : 0.f, v ? hi0[c].z : 0.f, v ? hi0[c].w : 0.f},
                                    {v ? lo1[c].x : 0.f, v ? lo1[c].y : 0.f, v ? lo1[c].z : 0.f, v ? lo1[c].w : 0.f,
                                     0.f, 0.f, 0.f, 0.f}};
            float m = 0.f;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk)
#pragma unroll
                for (int e = 0; e < 8; ++e) m = fmaxf(m, fabsf(xv[kk][e]));
            m = fmaxf(m, __shfl_xor(m, 16, 64));
            m = fmaxf(m, __shfl_xor(m, 32, 64));
            ex[c] = scale_exp(m);
            e1[c] = scale_exp(meta.n1 * m + meta.b1max);
            const float sc = pow2(ex[c]);
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                h4 h0, l0, h1, l1;
                split4<true>(&xv[kk][0], sc, h0, l0);
                split4<true>(&xv[kk][4], sc, h1, l1);
                xh[c][kk] = cat(h0, h1);
                xl[c][kk] = cat(l0, l1);
            }
        }
        // layer 1: h1 = relu(W1 x + b1), kept as the split B operand of layer 2
        h4 hh[FWD_NC][8], hl[FWD_NC][8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            v4f acc[FWD_NC];
#pragma unroll
            for (int c = 0; c < FWD_NC; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int o = (16 * m + j) * FRS1 + 32 * kk + 8 * q;
                const h8 ah = *reinterpret_cast<const h8 *>(W1h + o);
                const h8 al = *reinterpret_cast<const h8 *>(W1l + o);
                if (SPLIT) {
#pragma unroll
                    for (int c = 0; c < FWD_NC; ++c) acc[c] = mfma16(al, xh[c][kk], acc[c]);
#pragma unroll
                    for (int c = 0; c < FWD_NC; ++c) acc[c] = mfma16(ah, xl[c][kk], acc[c]);
                }
#pragma unroll
                for (int c = 0; c < FWD_NC; ++c) acc[c] = mfma16(ah, xh[c][kk], acc[c]);
            }
            const float4 bb = *reinterpret_cast<const float4 *>(b1 + 16 * m + 4 * q);
#pragma unroll
            for (int c = 0; c < FWD_NC; ++c) {
                const float un = pow2(-(meta.sw1 + ex[c]));
                float v[4] = {fmaxf(fmaf(acc[c][0], un, bb.x), 0.f), fmaxf(fmaf(acc[c][1], un, bb.y), 0.f),
                              fmaxf(fmaf(acc[c][2], un, bb.z), 0.f), fmaxf(fmaf(acc[c][3], un, bb.w), 0.f)};
                split4<true>(v, pow2(e1[c]), hh[c][m], hl[c][m]);
            }
            // keep the scheduler from hoisting every weight load of the layer (spills)
            __builtin_amdgcn_sched_barrier(0);
        }
        // layer 2 and the output layer: z3 = W3 relu(W2 h1 + b2) (+ b3), output rows on VALU
        float z[FWD_NC][3];
#pragma unroll
        for (int c = 0; c < FWD_NC; ++c) z[c][0] = z[c][1] = z[c][2] = 0.f;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            v4f acc[FWD_NC];
#pragma unroll
            for (int c = 0; c < FWD_NC; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int o = (16 * m + j) * FRS2 + 32 * kk + 8 * q;
                const h8 ah = *reinterpret_cast<const h8 *>(W2h + o);
                const h8 al = *reinterpret_cast<const h8 *>(W2l + o);
                if (SPLIT) {
#pragma unroll
                    for (int c = 0; c < FWD_NC; ++c) {
                        const h8 bh = cat(hh[c][2 * kk], hh[c][2 * kk + 1]);
                        acc[c] = mfma16(al, bh, acc[c]);
                    }
#pragma unroll
                    for (int c = 0; c < FWD_NC; ++c)
                        acc[c] = mfma16(ah, cat(hl[c][2 * kk], hl[c][2 * kk + 1]), acc[c]);
                }
#pragma unroll
                for (int c = 0; c < FWD_NC; ++c) acc[c] = mfma16(ah, cat(hh[c][2 * kk], hh[c][2 * kk + 1]), acc[c]);
            }
            const float4 bb = *reinterpret_cast<const float4 *>(b2 + 16 * m + 4 * q);
            const float4 w0 = *reinterpret_cast<const float4 *>(W3 + 16 * m + 4 * q);
            const float4 w1 = *reinterpret_cast<const float4 *>(W3 + H + 16 * m + 4 * q);
            const float4 w2 = *reinterpret_cast<const float4 *>(W3 + 2 * H + 16 * m + 4 * q);
            const float bv[4] = {bb.x, bb.y, bb.z, bb.w};
            const float wv[3][4] = {{w0.x, w0.y, w0.z, w0.w}, {w1.x, w1.y, w1.z, w1.w}, {w2.x, w2.y, w2.z, w2.w}};
#pragma unroll
            for (int c = 0; c < FWD_NC; ++c) {
                const float un = pow2(-(meta.sw2 + e1[c]));
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float h2 = fmaxf(fmaf(acc[c][r], un, bv[r]), 0.f);
#pragma unroll
                    for (int o = 0; o < 3; ++o) z[c][o] += wv[o][r] * h2;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int c = 0; c < FWD_NC; ++c) {
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                z[c][o] += __shfl_xor(z[c][o], 16, 64);
                z[c][o] += __shfl_xor(z[c][o], 32, 64);
            }
            const float zq = q == 0 ? z[c][0] : (q == 1 ? z[c][1] : z[c][2]);
            zout[c] = fast_sigmoid(zq + b3[q < 3 ? q : 0]);
            sout[c] = sv[c] ? s[c] : -1;
        }
    }
    store_out();
}

// ------------------------------------------------------------------ backward
//
// Block = 2 BWD_RW waves in two roles (8 waves of 32 units each with BWD_MP = 2).  P waves
// (0..RW-1) own units 16 BWD_MP p .. of both hidden layers for the forward recompute and hold
// those rows of W1 and W2 in registers; C waves (RW..2RW-1) own the same units for the backward
// chain and hold those rows of W2^T.  The C waves run one tile behind, so every phase pairs P
// and C work on the same SIMDs.  Phases
// of iteration t (block-wide barriers between them; the inputs of t are already staged):
//   A  P: layer 1 of t -> h1 plane, mask bits;              C: dz1 of t-1 (frame plane)
//         dW2 += dz2^T h1 of t-1
//   B  P: layer 2 of t -> h2, logit partials                C: dW1 += dz1^T x of t-1, dfeat partials
//                                                              of t-1; loads of t+1
//   C  P: dz3, dz2 of t -> its frame plane, half of         C: dz3, exponents, b2 b3 sums, the other
//         the dz2 plane                                        half of the dz2 plane (the same values)
//   D  P: feature gradient of t-1                           C: stage t+1; dW3 of t; the first dz2
//                                                              operands of dz1 of t
// (dW2 of a tile waits for the next phase A, where the P waves would otherwise idle beside the
// longer dz1 of the C waves; h1 is double-buffered for it, and the dz2 frame plane and the dW2
// frame stay put until the next phase C.  The feature partials and half of the dz2 plane sit with
// the C waves for the same balance: phase A is theirs to lengthen, phase C the P waves'.)
// After the last tile one more A/B pair finishes the C side.  Both roles run the same
// number of barriers, so s_barrier stays matched.

constexpr int BWD_MP = 2;                   // 16-unit row tiles of one layer per wave
constexpr int BWD_RW = 8 / BWD_MP;          // waves per role: BWD_RW x 16 BWD_MP = 128 units
constexpr int BWD_RT = 64 * BWD_RW;         // threads per role
constexpr int BWD_WAVES = 2 * BWD_RW, BWD_THREADS = 64 * BWD_WAVES;
// row tiles mp < DB_SPLIT of the dz2 plane are written by the P waves, the rest by the C waves
// (both form the same dz2 values; the split balances phase C between the roles)
constexpr int DB_SPLIT = BWD_MP / 2;
static_assert(BWD_MP == 1 || BWD_MP == 2, "one or two row tiles per wave");
constexpr int NT = TILE;  // samples per block tile (two 16-sample column tiles)

// LDS of the backward kernel (bytes); the small image part is staged at offset 0
constexpr int BS = IMG_FWD_END - IMG_B1;             // b1, b2, W3, b3, meta
constexpr int BSL(int img_off) { return img_off - IMG_B1; }
// Every activation plane is sample-major ([NT samples][row stride] hi, then lo), written with 8-byte
// stores of a lane's four units; the weight-gradient products read their unit-major operands from
// the same planes with transposing LDS reads (see tr_operand).
constexpr int XB_BYTES = 2 * NT * RS1 * 2;           // x B operand [NT][RS1] hi, lo
constexpr int HB_BYTES = 2 * NT * RS2 * 2;           // one [NT][RS2] hi, lo plane
constexpr int B_XB0 = BS;                            // x: two buffers (tile parity)
constexpr int B_HB = B_XB0 + 2 * XB_BYTES;           // h1: layer-2 and dW2 B operand, two (parity)
constexpr int B_DB = B_HB + 2 * HB_BYTES;            // dz2: dz1 B operand (per-sample scale)
constexpr int B_D2S = B_DB + HB_BYTES;               // dz2 in the dW2 frame: dW2 A operand
constexpr int B_D1S = B_D2S + HB_BYTES;              // dz1 in the dW1 frame: dW1 A operand
constexpr int B_Z3P = B_D1S + HB_BYTES;              // logit partials [RW][NT][4] f32
constexpr int DFS = 12;                              // row of dfeat partials (features)
constexpr int B_DFP = B_Z3P + BWD_RW * NT * 4 * 4;   // dfeat partials [RW][NT][DFS] f32
constexpr int H2S = 36;                              // row stride (floats) of the h2 plane
constexpr int B_H2 = B_DFP + BWD_RW * NT * DFS * 4;  // h2 [H][H2S] f32, written by P, read by C
constexpr int B_MASK = B_H2 + H * H2S * 4;           // h1 > 0 bits per lane [2][RW waves][64 lanes] u16
constexpr int B_XMAX = B_MASK + 2 * BWD_RW * 64 * 2; // max |x| per sample [2][NT]
constexpr int B_GR = B_XMAX + 2 * NT * 4;            // grad_rgb [2][NT][4]
constexpr int B_END = B_GR + 2 * NT * 16;
static_assert(B_END <= 160 * 1024, "backward LDS");
static_assert(B_XB0 % 16 == 0 && B_HB % 16 == 0 && B_DB % 16 == 0 && B_D2S % 16 == 0 && B_D1S % 16 == 0 &&
                  B_Z3P % 16 == 0 && B_DFP % 16 == 0 && B_MASK % 8 == 0,
              "LDS alignment");

// exponent that moves a gradient column into the accumulator frame F (operand scale e of
// the other factor); a zero column stays zero for any shift, so the clamp only guards range
__device__ __forceinline__ int frame_shift(int F, int e) {
    const int d = F - e;
    return d < -300 ? -300 : (d > 300 ? 300 : d);
}

__device__ __forceinline__ h8 lds_h8(const unsigned char *base, int off, int idx) {
    return *reinterpret_cast<const h8 *>(reinterpret_cast<const _Float16 *>(base + off) + idx);
}

__device__ __forceinline__ h8 glb_h8(const unsigned char *img, int off, int idx) {
    return *reinterpret_cast<const h8 *>(reinterpret_cast<const _Float16 *>(img + off) + idx);
}

// four values of one sample (a lane's units u0..u0+3), each moved by 2^e (exact; a zero stays zero
// for any e), split and stored at element idx of a sample-major plane (lo plane only in split mode)
template <bool SPLIT>
__device__ __forceinline__ void put_split4(unsigned char *plane, int idx, const float v[4], int e) {
    uint2 hi, lo;
    split2<false>(ldx(v[0], e), ldx(v[1], e), hi.x, lo.x);
    split2<false>(ldx(v[2], e), ldx(v[3], e), hi.y, lo.y);
    *reinterpret_cast<uint2 *>(reinterpret_cast<_Float16 *>(plane) + idx) = hi;
    if (SPLIT) *reinterpret_cast<uint2 *>(reinterpret_cast<_Float16 *>(plane) + NT * RS2 + idx) = lo;
}

// 64 bits per lane through the transposing LDS read: within each group of 16 lanes, the four
// 16-bit elements that lane t' addresses go to lanes 4 (t' mod 4) .. 4 (t' mod 4) + 3, each into
// element slot t' / 4.
__device__ __forceinline__ h4 lds_tr4(const unsigned char *p) {
    typedef short s4 __attribute__((ext_vector_type(4)));
    const s4 r = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s4 *)(p));
    return __builtin_bit_cast(h4, r);
}

// Unit-major MFMA operand (16 units U0..U0+15 as rows, the tile's 32 samples as K) from a
// sample-major plane [NT][RS] in which unit U0 + 4a + r sits at column cb + 8a + r (cb = the
// column of U0; phys slot order, U0 a multiple of 16): lane (q, j) gets unit U0 + j, its K slot
// 4h + e (h = read, e = element) holding sample 16h + 4e + q.  (The weight-gradient products sum
// over K, so any slot order serves as long as both operands use this one.)  Lane j of group q
// addresses the four units U0 + 4 (j mod 4) .. + 3 of sample 4 (j / 4) + q (+16 in the second
// read), so the four rows one 16-lane group reads lie 4 rows apart: with the 136-half row stride
// they start 16 banks apart and the group's 8-byte reads hit distinct banks.  The lane offset, in
// halves, is tr_lane<RS>(), taken once by the caller so that every read of a phase shares one
// address register.
template <int RS>
__device__ __forceinline__ int tr_lane(int j, int q) { return (4 * (j >> 2) + q) * RS + 8 * (j & 3); }
template <int RS>
__device__ __forceinline__ h8 tr_operand(const unsigned char *plane, int tl, int cb) {
    const _Float16 *p = reinterpret_cast<const _Float16 *>(plane) + tl + cb;
    return cat(lds_tr4(reinterpret_cast<const unsigned char *>(p)),
               lds_tr4(reinterpret_cast<const unsigned char *>(p + 16 * RS)));
}
// column of unit (or logical input) 16 n in the phys slot order of a 128- or 64-wide row
__device__ __forceinline__ int unit_col(int n) { return 32 * (n >> 1) + 4 * (n & 1); }

__device__ __forceinline__ void store_h4(unsigned char *base, int off, int idx, h4 v) {
    *reinterpret_cast<h4 *>(reinterpret_cast<_Float16 *>(base + off) + idx) = v;
}

// Block barrier that orders LDS only: the waves' outstanding global stores (the feature
// gradient rows) stay in flight across it instead of being drained at every phase.
// No global memory is exchanged between the waves of a block inside the backward kernel.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Feature gradient of a finished tile: the partials of the C waves, summed in a fixed order; t =
// the calling thread's index within its role.
__device__ __forceinline__ void feat_grad_out(const MlpArgs &a, const float *dfp, int pbase, int t) {
    for (int i = t; i < NT * a.in_feat; i += BWD_RT) {
        const int sl = i / a.in_feat, c = i % a.in_feat;
        const int s = pbase + sl;
        if (s < a.S) {
            float g = dfp[sl * DFS + c];
#pragma unroll
            for (int ww = 1; ww < BWD_RW; ++ww) g += dfp[(ww * NT + sl) * DFS + c];
            a.grad_feat[(int64_t)s * a.in_feat + c] = g;
        }
    }
}

// Per-sample quantities every wave derives identically from LDS (columns c: sample 16c + j)
struct SampleExp {
    int ex[2], e1[2];
};

__device__ __forceinline__ SampleExp sample_exp(const float *xmax_s, const Meta &meta, int j) {
    SampleExp r;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const float xm = xmax_s[16 * c + j];
        r.ex[c] = scale_exp(xm);
        r.e1[c] = scale_exp(meta.n1 * xm + meta.b1max);
    }
    return r;
}

// Output-layer gradient of this lane's two samples and the exponents that follow from it.
struct GradExp {
    float dz3[2][3];
    int g2[2], g1[2], k2[2], k1[2];
};

__device__ __forceinline__ GradExp grad_exp(const float *z3p, const float *gr_s, const float *b3, const Meta &meta,
                                            int j) {
    GradExp g;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int sl = 16 * c + j;
        float mx = 0.f;
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            float z = b3[o];
#pragma unroll
            for (int ww = 0; ww < BWD_RW; ++ww) z += z3p[(ww * NT + sl) * 4 + o];
            const float y = fast_sigmoid(z);
            g.dz3[c][o] = gr_s[sl * 4 + o] * y * (1.f - y);
            mx = fmaxf(mx, fabsf(g.dz3[c][o]));
        }
        // |dz2| <= n3t max|dz3| and |dz1| <= n2t |dz2| (infinity norms of W3^T and W2^T)
        const float bnd2 = meta.n3t * mx, bnd1 = meta.n2t * bnd2;
        g.g2[c] = scale_exp(bnd2);
        g.g1[c] = scale_exp(bnd1);
        g.k2[c] = bnd2 > 0.f ? ceil_exp(bnd2) : -FRAME_NONE;
        g.k1[c] = bnd1 > 0.f ? ceil_exp(bnd1) : -FRAME_NONE;
    }
    return g;
}

// (W3^T dz3) for unit row r of a lane's 4: one fixed sequence of FMAs, so both roles that form
// it get the same value bit for bit
__device__ __forceinline__ float w3t_dz3(const float (&wv)[3][4], const float (&dz3)[3], int r) {
    return __builtin_fmaf(wv[2][r], dz3[2], __builtin_fmaf(wv[1][r], dz3[1], wv[0][r] * dz3[0]));
}

// smallest frame the tile allows: F <= 14 + (other operand's exponent) - ceil_exp(bound)
__device__ __forceinline__ int tile_frame(const int other_e[2], const int k[2]) {
    int f = FRAME_NONE;
#pragma unroll
    for (int c = 0; c < 2; ++c) f = min(f, 14 + other_e[c] - k[c]);
    f = row16_min(f);  // over the 16 sample lanes j of the row
    // every lane holds the same value: make it scalar so the (rare) rescale is a real branch
    return __builtin_amdgcn_readfirstlane(f);
}

template <int M, int N>
__device__ __forceinline__ void rescale(v4f (&acc)[M][N], int &F, int f) {
    if (f < F) {
        const int d = max(f - F, -300);
#pragma unroll
        for (int mp = 0; mp < M; ++mp)
#pragma unroll
            for (int n = 0; n < N; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[mp][n][r] = ldx(acc[mp][n][r], d);
        F = f;
    }
}

template <bool SPLIT>
__global__ __launch_bounds__(BWD_THREADS) void mlp_bwd_kernel(MlpArgs a) {
    __shared__ __attribute__((aligned(16))) unsigned char sm[B_END];
    copy_to_lds(sm, a.img + IMG_B1, BS);
    const int tid = threadIdx.x, ln = lane(), j = ln & 15, q = ln >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const Meta meta = *reinterpret_cast<const Meta *>(a.img + IMG_META);
    const float *b1 = reinterpret_cast<const float *>(sm + BSL(IMG_B1));
    const float *b2 = reinterpret_cast<const float *>(sm + BSL(IMG_B2));
    const float *W3 = reinterpret_cast<const float *>(sm + BSL(IMG_W3));
    const float *b3 = reinterpret_cast<const float *>(sm + BSL(IMG_B3));
    unsigned char *db = lds_region(sm, B_DB);    // dz2 (per-sample scale)
    unsigned char *d2s = lds_region(sm, B_D2S);  // dz2 in the dW2 frame
    unsigned char *d1s = lds_region(sm, B_D1S);  // dz1 in the dW1 frame
    unsigned char *rB = lds_region(sm, B_Z3P);   // partials, h2, masks, per-sample values
    float *z3p = reinterpret_cast<float *>(rB);
    float *dfp = reinterpret_cast<float *>(rB + (B_DFP - B_Z3P));
    float *h2s = reinterpret_cast<float *>(rB + (B_H2 - B_Z3P));
    // bit (c MP + mp) 4 + r of lane (j, q) of wave w: h1 > 0 for unit 16 (MP w + mp) + 4q + r,
    // sample 16c + j; the P wave and the C wave of the same w use the same lane -> (unit, sample) map
    uint16_t *mask_b = reinterpret_cast<uint16_t *>(rB + (B_MASK - B_Z3P));
    float *xmax_b = reinterpret_cast<float *>(rB + (B_XMAX - B_Z3P));
    float *gr_b = reinterpret_cast<float *>(rB + (B_GR - B_Z3P));
    const int ntiles = a.n_tiles;
    float *P = a.partial + (int64_t)blockIdx.x * a.n_params;
    float *pW1 = P, *pb1 = pW1 + H * a.n_in, *pW2 = pb1 + H, *pb2 = pW2 + H * H, *pW3 = pb2 + H, *pb3 = pW3 + 3 * H;

    if (wave < BWD_RW) {
        // ================================================================ P waves
        const int w = wave;
        h8 w2h[BWD_MP][4], w2l[BWD_MP][4], w1h[BWD_MP][2], w1l[BWD_MP][2];
#pragma unroll
        for (int mp = 0; mp < BWD_MP; ++mp) {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int o = (16 * (BWD_MP * w + mp) + j) * RS2 + 32 * kk + 8 * q;
                w2h[mp][kk] = glb_h8(a.img, IMG_W2H, o);
                w2l[mp][kk] = glb_h8(a.img, IMG_W2L, o);
            }
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int o = (16 * (BWD_MP * w + mp) + j) * RS1 + 32 * kk + 8 * q;
                w1h[mp][kk] = glb_h8(a.img, IMG_W1H, o);
                w1l[mp][kk] = glb_h8(a.img, IMG_W1L, o);
            }
        }
        v4f dW2[BWD_MP][8];
#pragma unroll
        for (int mp = 0; mp < BWD_MP; ++mp)
#pragma unroll
            for (int n = 0; n < 8; ++n) dW2[mp][n] = v4f{0.f, 0.f, 0.f, 0.f};
        int F2 = FRAME_NONE;
        // dW2 += dz2^T h1 of a finished tile (K = its 32 samples; both operands read transposed from
        // the sample-major planes: the dz2 frame plane and that tile's h1 plane)
        auto dw2_step = [&](const unsigned char *h1p) {
            const int ln = fresh(lane()), j = ln & 15, q = ln >> 4;
            const int tl = tr_lane<RS2>(j, q);
#pragma unroll
            for (int mp = 0; mp < BWD_MP; ++mp) {
                const int cb = unit_col(BWD_MP * w + mp);
                const h8 ah = tr_operand<RS2>(d2s, tl, cb);
                const h8 al = SPLIT ? tr_operand<RS2>(d2s + NT * RS2 * 2, tl, cb) : ah;
#pragma unroll
                for (int n = 0; n < 8; ++n) {
                    const h8 bh = tr_operand<RS2>(h1p, tl, unit_col(n));
                    const h8 bl = SPLIT ? tr_operand<RS2>(h1p + NT * RS2 * 2, tl, unit_col(n)) : bh;
                    if (SPLIT) {
                        dW2[mp][n] = mfma16(al, bh, dW2[mp][n]);
                        dW2[mp][n] = mfma16(ah, bl, dW2[mp][n]);
                    }
                    dW2[mp][n] = mfma16(ah, bh, dW2[mp][n]);
                }
            }
        };
        lds_barrier();  // staged image and the first tile's inputs
        int it = 0;
        for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x, ++it) {
            const int ln = fresh(lane()), j = ln & 15, q = ln >> 4;
            const int pb = it & 1;
            unsigned char *hb = lds_region(sm, B_HB + pb * HB_BYTES);
            const float *xmax_s = xmax_b + pb * NT;
            const float *gr_s = gr_b + pb * NT * 4;
            const int xb = B_XB0 + pb * XB_BYTES;
            uint16_t *mask1 = mask_b + pb * (BWD_RW * 64);
            // ---- A: layer 1 for this wave's units; h1 -> the h1 plane, mask bits
            {
                const SampleExp se = sample_exp(xmax_s, meta, j);
                v4f acc[2][BWD_MP];  // [c][mp]
                unsigned mbits = 0;
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int mp = 0; mp < BWD_MP; ++mp) acc[c][mp] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kk = 0; kk < 2; ++kk) {
                    h8 bh[2], bl[2];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        bh[c] = lds_h8(sm, xb, (16 * c + j) * RS1 + 32 * kk + 8 * q);
                        bl[c] = lds_h8(sm, xb + NT * RS1 * 2, (16 * c + j) * RS1 + 32 * kk + 8 * q);
                    }
                    if (SPLIT) {
#pragma unroll
                        for (int c = 0; c < 2; ++c)
#pragma unroll
                            for (int mp = 0; mp < BWD_MP; ++mp) acc[c][mp] = mfma16(w1l[mp][kk], bh[c], acc[c][mp]);
#pragma unroll
                        for (int c = 0; c < 2; ++c)
#pragma unroll
                            for (int mp = 0; mp < BWD_MP; ++mp) acc[c][mp] = mfma16(w1h[mp][kk], bl[c], acc[c][mp]);
                    }
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int mp = 0; mp < BWD_MP; ++mp) acc[c][mp] = mfma16(w1h[mp][kk], bh[c], acc[c][mp]);
                }
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const float un = pow2(-(meta.sw1 + se.ex[c]));
                    const float sc = pow2(se.e1[c]);
#pragma unroll
                    for (int mp = 0; mp < BWD_MP; ++mp) {
                        const float4 bb = *reinterpret_cast<const float4 *>(b1 + 16 * (BWD_MP * w + mp) + 4 * q);
                        const float bv[4] = {bb.x, bb.y, bb.z, bb.w};
                        float h1[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            h1[r] = fmaxf(fmaf(acc[c][mp][r], un, bv[r]), 0.f);
                            mbits |= (h1[r] > 0.f ? 1u : 0u) << ((c * BWD_MP + mp) * 4 + r);
                        }
                        h4 hi, lo;
                        split4<false>(h1, sc, hi, lo);
                        const int ob = (16 * c + j) * RS2 + unit_col(BWD_MP * w + mp) + 8 * q;
                        store_h4(hb, 0, ob, hi);
                        if (SPLIT) store_h4(hb, NT * RS2 * 2, ob, lo);
                    }
                }
                mask1[w * 64 + ln] = (uint16_t)mbits;
            }
            if (it > 0) dw2_step(lds_region(sm, B_HB + (pb ^ 1) * HB_BYTES));
            lds_barrier();
            // ---- B: layer 2 for this wave's units, logit partials
            {
                const SampleExp se = sample_exp(xmax_s, meta, j);
                v4f acc[2][BWD_MP];  // [c][mp]
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int mp = 0; mp < BWD_MP; ++mp) acc[c][mp] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    h8 bh[2], bl[2];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        bh[c] = lds_h8(hb, 0, (16 * c + j) * RS2 + 32 * kk + 8 * q);
                        bl[c] = lds_h8(hb, NT * RS2 * 2, (16 * c + j) * RS2 + 32 * kk + 8 * q);
                    }
                    if (SPLIT) {
#pragma unroll
                        for (int c = 0; c < 2; ++c)
#pragma unroll
                            for (int mp = 0; mp < BWD_MP; ++mp) acc[c][mp] = mfma16(w2l[mp][kk], bh[c], acc[c][mp]);
#pragma unroll
                        for (int c = 0; c < 2; ++c)
#pragma unroll
                            for (int mp = 0; mp < BWD_MP; ++mp) acc[c][mp] = mfma16(w2h[mp][kk], bl[c], acc[c][mp]);
                    }
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int mp = 0; mp < BWD_MP; ++mp) acc[c][mp] = mfma16(w2h[mp][kk], bh[c], acc[c][mp]);
                }
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const float un = pow2(-(meta.sw2 + se.e1[c]));
                    float zp[3] = {0.f, 0.f, 0.f};
#pragma unroll
                    for (int mp = 0; mp < BWD_MP; ++mp) {
                        const int u0 = 16 * (BWD_MP * w + mp) + 4 * q;
                        const float4 bb = *reinterpret_cast<const float4 *>(b2 + u0);
                        const float4 x0 = *reinterpret_cast<const float4 *>(W3 + u0);
                        const float4 x1 = *reinterpret_cast<const float4 *>(W3 + H + u0);
                        const float4 x2 = *reinterpret_cast<const float4 *>(W3 + 2 * H + u0);
                        const float bv[4] = {bb.x, bb.y, bb.z, bb.w};
                        const float wv[3][4] = {{x0.x, x0.y, x0.z, x0.w}, {x1.x, x1.y, x1.z, x1.w}, {x2.x, x2.y, x2.z, x2.w}};
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float h2 = fmaxf(fmaf(acc[c][mp][r], un, bv[r]), 0.f);
                            h2s[(u0 + r) * H2S + 16 * c + j] = h2;
#pragma unroll
                            for (int o = 0; o < 3; ++o) zp[o] += wv[o][r] * h2;
                        }
                    }
#pragma unroll
                    for (int o = 0; o < 3; ++o) {
                        zp[o] += __shfl_xor(zp[o], 16, 64);
                        zp[o] += __shfl_xor(zp[o], 32, 64);
                    }
                    const float zq = q == 0 ? zp[0] : (q == 1 ? zp[1] : zp[2]);
                    if (q < 3) z3p[(w * NT + 16 * c + j) * 4 + q] = zq;
                }
            }
            lds_barrier();
            // ---- C: dz3, dz2 = mask(h2) W3^T dz3 (VALU): the dz2 plane and the dz2 frame plane
            {
                const SampleExp se = sample_exp(xmax_s, meta, j);
                const GradExp ge = grad_exp(z3p, gr_s, b3, meta, j);
                rescale(dW2, F2, tile_frame(se.e1, ge.k2));
#pragma unroll
                for (int mp = 0; mp < BWD_MP; ++mp) {
                    const int u0 = 16 * (BWD_MP * w + mp) + 4 * q;
                    const float4 x0 = *reinterpret_cast<const float4 *>(W3 + u0);
                    const float4 x1 = *reinterpret_cast<const float4 *>(W3 + H + u0);
                    const float4 x2 = *reinterpret_cast<const float4 *>(W3 + 2 * H + u0);
                    const float wv[3][4] = {{x0.x, x0.y, x0.z, x0.w}, {x1.x, x1.y, x1.z, x1.w}, {x2.x, x2.y, x2.z, x2.w}};
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        float dz2[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float d = w3t_dz3(wv, ge.dz3[c], r);
                            dz2[r] = h2s[(u0 + r) * H2S + 16 * c + j] > 0.f ? d : 0.f;
                        }
                        const int ob = (16 * c + j) * RS2 + unit_col(BWD_MP * w + mp) + 8 * q;
                        if (mp < DB_SPLIT) {
                            // dz2 at its per-sample scale: the dz1 operand plane (row tiles mp >=
                            // DB_SPLIT are the C waves' share of it)
                            h4 hi, lo;
                            split4<false>(dz2, pow2(ge.g2[c]), hi, lo);
                            store_h4(db, 0, ob, hi);
                            if (SPLIT) store_h4(db, NT * RS2 * 2, ob, lo);
                        }
                        put_split4<SPLIT>(d2s, ob, dz2, frame_shift(F2, se.e1[c]));  // exact for any shift
                    }
                }
            }
            lds_barrier();
            // ---- D: feature gradient of the previous tile (its partials came from the C waves' phase A)
            if (it > 0) feat_grad_out(a, dfp, (tile - (int)gridDim.x) * NT, tid);
            lds_barrier();
        }
        // dW2 of the last tile; the C side's last A/B pair
        if (it > 0) dw2_step(lds_region(sm, B_HB + ((it - 1) & 1) * HB_BYTES));
        lds_barrier();
        lds_barrier();
        // ---- partial gradient of the P role: W2
        const int u2 = F2 == FRAME_NONE ? 0 : -F2;
#pragma unroll
        for (int mp = 0; mp < BWD_MP; ++mp)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int hrow = 16 * (BWD_MP * w + mp) + 4 * q + r;
#pragma unroll
                for (int n = 0; n < 8; ++n) pW2[hrow * H + 16 * n + j] = ldx(dW2[mp][n][r], u2);
            }
    } else {
        // ================================================================ C waves
        const int w = wave - BWD_RW;
        const int ct = tid - BWD_RT;           // index within the C role
        // input staging: the first 256 threads of the role (waves 0..3), sample xsl, slot group xg
        const bool stager = BWD_RW <= 4 || w < 4;
        const int xsl = ct >> 3, xg = ct & 7;
        h8 w2th[BWD_MP][4], w2tl[BWD_MP][4];
#pragma unroll
        for (int mp = 0; mp < BWD_MP; ++mp)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int o = (16 * (BWD_MP * w + mp) + j) * RS2 + 32 * kk + 8 * q;
                w2th[mp][kk] = glb_h8(a.img, IMG_W2TH, o);
                w2tl[mp][kk] = glb_h8(a.img, IMG_W2TL, o);
            }
        // W1's feature columns, transposed (rows = features), over this wave's units as K: 32 units
        // (two row tiles) in one 16x16x32 product, or 16 units in one 16x16x16 product
        const int ofF = j * RS2 + unit_col(BWD_MP * w) + 8 * q;
        const h8 w1fh = glb_h8(a.img, IMG_W1FH, ofF), w1fl = glb_h8(a.img, IMG_W1FL, ofF);
        v4f dW1[BWD_MP][3];
#pragma unroll
        for (int mp = 0; mp < BWD_MP; ++mp)
#pragma unroll
            for (int n = 0; n < 3; ++n) dW1[mp][n] = v4f{0.f, 0.f, 0.f, 0.f};
        // lane-local sums over this lane's samples; reduced over the 16 sample lanes at the end
        float db1[BWD_MP][4], db2[BWD_MP][4], dw3[3][BWD_MP][4], db3[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int mp = 0; mp < BWD_MP; ++mp)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                db1[mp][r] = db2[mp][r] = 0.f;
#pragma unroll
                for (int o = 0; o < 3; ++o) dw3[o][mp][r] = 0.f;
            }
        int F1 = FRAME_NONE;
        // inputs of a tile: global loads, in three steps spread over phases so that their
        // latency overlaps other work (ray window; ray search and feature loads; staging)
        // The loaded values stay raw until stage_tile (phase D), where lanes past the last sample
        // and the padding columns are zeroed, so that nothing consumes the loads before then.
        float4 xlo = make_float4(0.f, 0.f, 0.f, 0.f), xhi = xlo;
        float grv = 0.f;
        unsigned xok = 0;  // bit 0: xlo is real, bit 1: xhi is real, bit 2: grv is real
        auto load_tile = [&](int t, int r0, int win) {
            const int s = t * NT + xsl;
            const bool sv = s < a.S;
            // all lanes take part; this wave's samples are t NT + 8 w + (lane >> 3).  Lanes past the
            // last sample load from the last sample and its ray (kept in range).
            const int ray = min(ray_of_group8(a.offs, a.n_rays, r0, win, t * NT + 8 * w), a.n_rays - 1);
            const int sc = sv ? s : a.S - 1;
            const int kk = xg >> 2, q = xg & 3;
            if (a.feat_vec) {
                // every lane issues the same two 16-byte loads and one 4-byte load, with no divergent
                // branch around them (divergent branches would make one group's loads wait for the
                // other's, as both write the same registers)
                const float *pe = a.pe + (int64_t)ray * PEW;
                const float *pl = kk == 0 && q < 3 ? a.feat + (int64_t)sc * 12 + 4 * q : pe + (kk == 0 ? 0 : 20 + 4 * q);
                xlo = *reinterpret_cast<const float4 *>(pl);
                xhi = *reinterpret_cast<const float4 *>(pe + 4 + 4 * q);
                grv = a.grad_rgb[(int64_t)sc * 3 + (xg < 3 ? xg : 2)];
                xok = (sv ? 1u : 0u) | (sv && kk == 0 ? 2u : 0u) | (sv && xg < 3 ? 4u : 0u);
            } else {
                float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                float g = 0.f;
                if (sv) {
                    load_x8(a, s, ray, kk, q, v);
                    if (xg < 3) g = a.grad_rgb[(int64_t)s * 3 + xg];
                }
                xlo = make_float4(v[0], v[1], v[2], v[3]);
                xhi = make_float4(v[4], v[5], v[6], v[7]);
                grv = g;
                xok = 7u;
            }
        };
        // ... and their split into the x plane of buffer pb (layer-1 B operand, read transposed by
        // dW1), max |x| and grad_rgb
        auto stage_tile = [&](int pb) {
            const bool l = xok & 1u, h = xok & 2u;
            const float xv[8] = {l ? xlo.x : 0.f, l ? xlo.y : 0.f, l ? xlo.z : 0.f, l ? xlo.w : 0.f,
                                 h ? xhi.x : 0.f, h ? xhi.y : 0.f, h ? xhi.z : 0.f, h ? xhi.w : 0.f};
            float m = 0.f;
#pragma unroll
            for (int e = 0; e < 8; ++e) m = fmaxf(m, fabsf(xv[e]));
            m = group8_max(m);  // over the 8 slot groups xg of this sample
            const float sc = pow2(scale_exp(m));
            h4 h0, l0, h1, l1;
            split4<false>(&xv[0], sc, h0, l0);
            split4<false>(&xv[4], sc, h1, l1);
            const int xb = B_XB0 + pb * XB_BYTES;
            *reinterpret_cast<h8 *>(reinterpret_cast<_Float16 *>(sm + xb) + xsl * RS1 + 8 * xg) = cat(h0, h1);
            if (SPLIT)
                *reinterpret_cast<h8 *>(reinterpret_cast<_Float16 *>(sm + xb + NT * RS1 * 2) + xsl * RS1 + 8 * xg) =
                    cat(l0, l1);
            if (xg == 0) xmax_b[pb * NT + xsl] = m;
            if (xg < 4) gr_b[(pb * NT + xsl) * 4 + xg] = (xok & 4u) ? grv : 0.f;
        };
        // dW1 += dz1^T x of a finished tile (its x buffer pb; both operands read transposed from the
        // sample-major planes; logical inputs 0..47 in the three 16-column blocks)
        auto dw1_step = [&](int pb) {
            const int ln = fresh(lane()), j = ln & 15, q = ln >> 4;
            const int t2 = tr_lane<RS2>(j, q), t1 = tr_lane<RS1>(j, q);
            const unsigned char *xp = lds_region(sm, B_XB0 + pb * XB_BYTES);
#pragma unroll
            for (int mp = 0; mp < BWD_MP; ++mp) {
                const int cb = unit_col(BWD_MP * w + mp);
                const h8 dh = tr_operand<RS2>(d1s, t2, cb);
                const h8 dl = SPLIT ? tr_operand<RS2>(d1s + NT * RS2 * 2, t2, cb) : dh;
#pragma unroll
                for (int n = 0; n < 3; ++n) {
                    const h8 bh = tr_operand<RS1>(xp, t1, unit_col(n));
                    const h8 bl = SPLIT ? tr_operand<RS1>(xp + NT * RS1 * 2, t1, unit_col(n)) : bh;
                    if (SPLIT) {
                        dW1[mp][n] = mfma16(dl, bh, dW1[mp][n]);
                        dW1[mp][n] = mfma16(dh, bl, dW1[mp][n]);
                    }
                    dW1[mp][n] = mfma16(dh, bh, dW1[mp][n]);
                }
            }
        };
        // dW3 += dz3 h2^T over this lane's units and samples (h2 of the current tile)
        auto dw3_step = [&](const float (&dz3)[2][3], int j, int q) {
#pragma unroll
            for (int mp = 0; mp < BWD_MP; ++mp)
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float h2 = h2s[(16 * (BWD_MP * w + mp) + 4 * q + r) * H2S + 16 * c + j];
#pragma unroll
                        for (int o = 0; o < 3; ++o) dw3[o][mp][r] += dz3[c][o] * h2;
                    }
        };
        // dz1 = mask(h1) W2^T dz2 of a tile (mask bits of parity pb, exponents g2/g1/ex of that
        // tile), dfeat partials, dz1 in the dW1 frame
        float kdz1[BWD_MP][2][4];  // dz1 of the last dz1_step, for its feature partials
        // The first K-step's dz2 operands and the mask bits of the next dz1_step, read at the end of
        // phase D (the dz2 plane and the mask of that tile are complete there and stay put until the
        // next phase C / A), so that dz1's first products do not wait for LDS at the head of phase A.
        h8 pf_bh[2], pf_bl[2];
        unsigned pf_mbits = 0;
        auto dz1_prefetch = [&](int pb) {
            const int ln = fresh(lane()), j = ln & 15, q = ln >> 4;
            pf_mbits = mask_b[pb * (BWD_RW * 64) + w * 64 + ln];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                pf_bh[c] = lds_h8(db, 0, (16 * c + j) * RS2 + 8 * q);
                pf_bl[c] = lds_h8(db, NT * RS2 * 2, (16 * c + j) * RS2 + 8 * q);
            }
        };
        auto dz1_step = [&](const int g2[2], const int g1[2], const int ex[2]) {
            const int ln = fresh(lane()), j = ln & 15, q = ln >> 4;
            const unsigned mbits = pf_mbits;  // this lane's h1 > 0 bits (prefetched)
            float dz1[BWD_MP][2][4];
            v4f acc[2][BWD_MP];  // [c][mp]
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int mp = 0; mp < BWD_MP; ++mp) acc[c][mp] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                h8 bh[2], bl[2];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    bh[c] = kk == 0 ? pf_bh[c] : lds_h8(db, 0, (16 * c + j) * RS2 + 32 * kk + 8 * q);
                    bl[c] = kk == 0 ? pf_bl[c] : lds_h8(db, NT * RS2 * 2, (16 * c + j) * RS2 + 32 * kk + 8 * q);
                }
                if (SPLIT) {
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int mp = 0; mp < BWD_MP; ++mp) acc[c][mp] = mfma16(w2tl[mp][kk], bh[c], acc[c][mp]);
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int mp = 0; mp < BWD_MP; ++mp) acc[c][mp] = mfma16(w2th[mp][kk], bl[c], acc[c][mp]);
                }
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int mp = 0; mp < BWD_MP; ++mp) acc[c][mp] = mfma16(w2th[mp][kk], bh[c], acc[c][mp]);
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float un = pow2(-(meta.sw2 + g2[c]));
                const int fs = frame_shift(F1, ex[c]);  // exact for any shift; 0 stays 0
#pragma unroll
                for (int mp = 0; mp < BWD_MP; ++mp) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const bool on = (mbits >> ((c * BWD_MP + mp) * 4 + r)) & 1u;
                        dz1[mp][c][r] = on ? acc[c][mp][r] * un : 0.f;
                        db1[mp][r] += dz1[mp][c][r];
                    }
                    put_split4<SPLIT>(d1s, (16 * c + j) * RS2 + unit_col(BWD_MP * w + mp) + 8 * q, dz1[mp][c], fs);
                }
            }
#pragma unroll
            for (int mp = 0; mp < BWD_MP; ++mp)
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r) kdz1[mp][c][r] = dz1[mp][c][r];
        };
        // dfeat partial of the tile whose dz1 the last dz1_step computed (kdz1; exponents g1 of that
        // tile) over this wave's units: rows = feature 4q + r, column = sample.  It runs in phase B,
        // where the C waves wait for the P waves' layer 2, instead of lengthening phase A.
        auto dfeat_step = [&](const int g1[2]) {
            const int ln = fresh(lane()), j = ln & 15, q = ln >> 4;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float sc = pow2(g1[c]);
                v4f df = v4f{0.f, 0.f, 0.f, 0.f};
                if constexpr (BWD_MP == 2) {
                    h4 h0, l0, h1v, l1v;
                    split4<true>(kdz1[0][c], sc, h0, l0);
                    split4<true>(kdz1[1][c], sc, h1v, l1v);
                    const h8 bh = cat(h0, h1v), bl = cat(l0, l1v);
                    if (SPLIT) {
                        df = mfma16(w1fl, bh, df);
                        df = mfma16(w1fh, bl, df);
                    }
                    df = mfma16(w1fh, bh, df);
                } else {
                    // K = this wave's 16 units: slots 4q..4q+3 of the 16x16x16 product
                    h4 h0, l0;
                    split4<true>(kdz1[0][c], sc, h0, l0);
                    const h4 ah = __builtin_shufflevector(w1fh, w1fh, 0, 1, 2, 3);
                    const h4 al = __builtin_shufflevector(w1fl, w1fl, 0, 1, 2, 3);
                    if (SPLIT) {
                        df = __builtin_amdgcn_mfma_f32_16x16x16f16(al, h0, df, 0, 0, 0);
                        df = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, l0, df, 0, 0, 0);
                    }
                    df = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, h0, df, 0, 0, 0);
                }
                const float un = pow2(-(meta.sw1 + g1[c]));
                if (q < DFS / 4)
                    *reinterpret_cast<float4 *>(dfp + (w * NT + 16 * c + j) * DFS + 4 * q) =
                        make_float4(df[0] * un, df[1] * un, df[2] * un, df[3] * un);
            }
        };
        // First rays of this block's tiles, 64 iterations at a time: lane l holds that of iteration
        // wb + l (wb a multiple of 64; indices past the last tile repeat the last tile's ray, a
        // valid ray).  One load per 64 tiles instead of a dependent load at the head of every tile.
        auto ray_window = [&](int wb) {
            const int t = (int)blockIdx.x + (wb + lane()) * (int)gridDim.x;
            return a.tile_ray[t < ntiles ? t : ntiles - 1];
        };
        int trw = 0;
        if ((int)blockIdx.x < ntiles) {
            trw = ray_window(0);
            if (stager) {
                const int r0 = __builtin_amdgcn_readlane(trw, 0);
                load_tile(blockIdx.x, r0, window_entry(a.offs, a.n_rays, r0));
                stage_tile(0);
            }
        }
        lds_barrier();  // staged image and the first tile's inputs
        int it = 0, pbase = -1;
        int pg2[2] = {0, 0}, pg1[2] = {0, 0}, pex[2] = {0, 0};  // exponents of the previous tile
        float tdz3[2][3];                                         // this tile's dz3 (for dW3 in D)
        for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x, ++it) {
            const int ln = fresh(lane()), j = ln & 15, q = ln >> 4;
            const int pb = it & 1;
            const bool next = tile + (int)gridDim.x < ntiles;
            // ---- A: ray window of the next tile (its loads are issued first and consumed in B);
            //      dz1 of the previous tile
            if (((it + 1) & 63) == 0) trw = ray_window(it + 1);
            const int r0n = __builtin_amdgcn_readlane(trw, (it + 1) & 63);
            const int winn = window_entry(a.offs, a.n_rays, r0n);
            if (pbase >= 0) dz1_step(pg2, pg1, pex);
            lds_barrier();
            // ---- B: dW1 of the previous tile; then the loads of the next tile's inputs, whose
            //      latency runs through phase C (they are staged in D)
            if (pbase >= 0) {
                dw1_step(pb ^ 1);
                dfeat_step(pg1);
            }
            if (stager) load_tile(tile + gridDim.x, r0n, winn);  // past the last tile: zeroed, not staged
            lds_barrier();
            // ---- C: output gradient and exponents of this tile; the frame of dW1; db2 += dz2,
            //      db3 += dz3 (VALU, h2 from the P waves)
            {
                const SampleExp se = sample_exp(xmax_b + pb * NT, meta, j);
                const GradExp ge = grad_exp(z3p, gr_b + pb * NT * 4, b3, meta, j);
                rescale(dW1, F1, tile_frame(se.ex, ge.k1));
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    pg2[c] = ge.g2[c];
                    pg1[c] = ge.g1[c];
                    pex[c] = se.ex[c];
#pragma unroll
                    for (int o = 0; o < 3; ++o) tdz3[c][o] = ge.dz3[c][o];
                }
                if (w == 0 && q == 0) {
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int o = 0; o < 3; ++o) db3[o] += ge.dz3[c][o];
                }
#pragma unroll
                for (int mp = 0; mp < BWD_MP; ++mp) {
                    const int u0 = 16 * (BWD_MP * w + mp) + 4 * q;
                    const float4 x0 = *reinterpret_cast<const float4 *>(W3 + u0);
                    const float4 x1 = *reinterpret_cast<const float4 *>(W3 + H + u0);
                    const float4 x2 = *reinterpret_cast<const float4 *>(W3 + 2 * H + u0);
                    const float wv[3][4] = {{x0.x, x0.y, x0.z, x0.w}, {x1.x, x1.y, x1.z, x1.w}, {x2.x, x2.y, x2.z, x2.w}};
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        float dz2[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float h2 = h2s[(u0 + r) * H2S + 16 * c + j];
                            const float d = w3t_dz3(wv, ge.dz3[c], r);
                            dz2[r] = h2 > 0.f ? d : 0.f;  // the P waves' dz2, bit for bit
                            db2[mp][r] += dz2[r];
                        }
                        // dz2 at its per-sample scale, the B operand of the next phase A's dz1: row
                        // tiles mp >= DB_SPLIT (the P waves write the others)
                        if (mp >= DB_SPLIT) {
                            h4 hi, lo;
                            split4<false>(dz2, pow2(ge.g2[c]), hi, lo);
                            const int ob = (16 * c + j) * RS2 + unit_col(BWD_MP * w + mp) + 8 * q;
                            store_h4(db, 0, ob, hi);
                            if (SPLIT) store_h4(db, NT * RS2 * 2, ob, lo);
                        }
                    }
                }
            }
            lds_barrier();
            // ---- D: the next tile's inputs -> x planes (the P waves write the previous tile's
            //      feature gradient meanwhile); dW3 += dz3 h2^T of this tile (h2 stays until the
            //      P waves' next layer 2)
            if (next && stager) stage_tile(pb ^ 1);
            dw3_step(tdz3, j, q);
            dz1_prefetch(pb);  // for the next phase A's dz1 of this tile
            lds_barrier();
            pbase = tile * NT;
        }
        // ---- the last tile: A (dz1), B (dW1 and the feature gradient)
        if (pbase >= 0) {
            dz1_step(pg2, pg1, pex);  // operands prefetched in the last phase D
            dfeat_step(pg1);  // before the barrier: feat_grad_out below reads every wave's partials
        }
        lds_barrier();
        if (pbase >= 0) {
            dw1_step((it - 1) & 1);
            feat_grad_out(a, dfp, pbase, ct);
        }
        lds_barrier();
        // ---- partial gradients of the C role: W1, b1, b2, W3, b3
        const int u1 = F1 == FRAME_NONE ? 0 : -F1;
#pragma unroll
        for (int mp = 0; mp < BWD_MP; ++mp)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int hrow = 16 * (BWD_MP * w + mp) + 4 * q + r;
#pragma unroll
                for (int n = 0; n < 3; ++n) {
                    const int c = w1_col(a.in_feat, a.n_freq, 16 * n + j);
                    if (c >= 0) pW1[hrow * a.n_in + c] = ldx(dW1[mp][n][r], u1);
                }
                float s1 = db1[mp][r], s2 = db2[mp][r], s3[3] = {dw3[0][mp][r], dw3[1][mp][r], dw3[2][mp][r]};
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) {
                    s1 += __shfl_xor(s1, o, 64);
                    s2 += __shfl_xor(s2, o, 64);
#pragma unroll
                    for (int t = 0; t < 3; ++t) s3[t] += __shfl_xor(s3[t], o, 64);
                }
                if (j == 0) {
                    pb1[hrow] = s1;
                    pb2[hrow] = s2;
#pragma unroll
                    for (int t = 0; t < 3; ++t) pW3[t * H + hrow] = s3[t];
                }
            }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1)
#pragma unroll
            for (int t = 0; t < 3; ++t) db3[t] += __shfl_xor(db3[t], o, 64);
        if (ct < 3) pb3[ct] = db3[ct];
    }
}

// gradient += sum of the per-block partials: 64 parameters per block, the four waves sum
// interleaved quarters of the partials and are combined in a fixed order
constexpr int RED_THREADS = 256;

__global__ __launch_bounds__(RED_THREADS) void mlp_reduce_kernel(MlpArgs a) {
    __shared__ float part[RED_THREADS / 64][64];
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int i = blockIdx.x * 64 + l;
    float acc = 0.f;
    if (i < a.n_params) {
#pragma unroll 8
        for (int b = wv; b < a.nblocks; b += RED_THREADS / 64) acc += a.partial[(int64_t)b * a.n_params + i];
    }
    part[wv][l] = acc;
    __syncthreads();
    if (wv != 0 || i >= a.n_params) return;
    acc = (part[0][l] + part[1][l]) + (part[2][l] + part[3][l]);
    const int nW1 = H * a.n_in;
    int k = i;
    if (k < nW1) { a.gW1[k] += acc; return; }
    k -= nW1;
    if (k < H) { a.gb1[k] += acc; return; }
    k -= H;
    if (k < H * H) { a.gW2[k] += acc; return; }
    k -= H * H;
    if (k < H) { a.gb2[k] += acc; return; }
    k -= H;
    if (k < 3 * H) { a.gW3[k] += acc; return; }
    k -= 3 * H;
    a.gb3[k] += acc;
}

int check_mlp(const dvgo_color_mlp *m, bool bwd) {
    if (!m) return set_error(DVGO_ERR_NULL, "mlp is NULL");
    if (m->struct_size != sizeof(dvgo_color_mlp)) return set_error(DVGO_ERR_ABI, "dvgo_color_mlp.struct_size mismatch");
    if (m->hidden != H) return set_error(DVGO_ERR_UNSUPPORTED, "hidden must be %d", H);
    if (m->in_feat < 1 || m->in_feat > 12) return set_error(DVGO_ERR_UNSUPPORTED, "in_feat must be in [1, 12]");
    if (m->precision != DVGO_MLP_SPLIT_F16 && m->precision != DVGO_MLP_F16)
        return set_error(DVGO_ERR_UNSUPPORTED, "unknown precision %d", m->precision);
    if (m->n_freq < 0 || m->n_freq > 4) return set_error(DVGO_ERR_UNSUPPORTED, "n_freq must be in [0, 4]");
    if (!m->W1 || !m->b1 || !m->W2 || !m->b2 || !m->W3 || !m->b3) return set_error(DVGO_ERR_NULL, "a weight is NULL");
    if (bwd && (!m->gW1 || !m->gb1 || !m->gW2 || !m->gb2 || !m->gW3 || !m->gb3))
        return set_error(DVGO_ERR_NULL, "a weight gradient is NULL");
    return DVGO_OK;
}

int n_in_of(const dvgo_color_mlp *m) { return m->in_feat + 3 + 6 * m->n_freq; }
int n_params_of(const dvgo_color_mlp *m) { return H * n_in_of(m) + H + H * H + H + 3 * H + 3; }
int bwd_blocks(int64_t S) {
    int64_t t = (S + NT - 1) / NT;
    return (int)(t < MAX_BLOCKS ? (t < 1 ? 1 : t) : MAX_BLOCKS);
}

size_t ws_layout(const dvgo_color_mlp *m, int32_t R, int64_t S, size_t *off_pe, size_t *off_tr, size_t *off_part) {
    size_t o = align_up((size_t)IMG_BYTES, 256);
    *off_pe = o;
    o += align_up((size_t)R * PEW * 4, 256);
    *off_tr = o;
    o += align_up((size_t)((S + TILE - 1) / TILE) * 4, 256);
    *off_part = o;
    o += (size_t)bwd_blocks(S) * n_params_of(m) * 4;
    return o;
}

int setup(const dvgo_color_mlp *m, int32_t R, const int32_t *offs, const float *dirs, int64_t S, const float *feat,
          void *ws, size_t ws_bytes, bool bwd, MlpArgs &a, bool need_feat = true) {
    int rc = check_mlp(m, bwd);
    if (rc) return rc;
    if (R < 0 || S < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays or n_samples");
    if (S >= ((int64_t)1 << 31) / 16) return set_error(DVGO_ERR_RANGE, "n_samples too large");
    if (S > 0 && (R == 0 || !offs || !dirs || (need_feat && !feat)))
        return set_error(DVGO_ERR_NULL, "ray_offsets, dirs or feat is NULL");
    size_t off_pe, off_tr, off_part;
    const size_t need = ws_layout(m, R, S, &off_pe, &off_tr, &off_part);
    if (!ws || ws_bytes < need) return set_error(DVGO_ERR_WORKSPACE, "workspace too small (%zu < %zu)", ws_bytes, need);
    if (((uintptr_t)ws & 255) != 0) return set_error(DVGO_ERR_SHAPE, "workspace must be 256-byte aligned");
    memset(&a, 0, sizeof(a));
    a.W1 = m->W1; a.b1 = m->b1; a.W2 = m->W2; a.b2 = m->b2; a.W3 = m->W3; a.b3 = m->b3;
    a.gW1 = m->gW1; a.gb1 = m->gb1; a.gW2 = m->gW2; a.gb2 = m->gb2; a.gW3 = m->gW3; a.gb3 = m->gb3;
    a.in_feat = m->in_feat;
    a.n_freq = m->n_freq;
    a.n_in = n_in_of(m);
    a.n_params = n_params_of(m);
    a.n_rays = R;
    a.offs = offs;
    a.dirs = dirs;
    a.S = (int)S;
    a.feat = feat;
    a.feat_vec = m->in_feat == 12 && ((uintptr_t)feat & 15) == 0;
    a.img = (unsigned char *)ws;
    a.pe = (float *)((char *)ws + off_pe);
    a.tile_ray = (int *)((char *)ws + off_tr);
    a.n_tiles = (int)((S + TILE - 1) / TILE);
    a.partial = (float *)((char *)ws + off_part);
    a.nblocks = bwd_blocks(S);
    return DVGO_OK;
}

template <int GM>
int launch_fwd(const MlpArgs &a, const dvgo_color_mlp *m, hipStream_t st) {
    using F = FwdShape<GM>;
    const int64_t nwt = (a.S + F::WTILE - 1) / F::WTILE;
    const int64_t nb = (nwt + F::WAVES - 1) / F::WAVES;
    const dim3 grid((int)(nb < MAX_BLOCKS ? nb : MAX_BLOCKS));
    if (m->precision == DVGO_MLP_F16)
        hipLaunchKernelGGL((mlp_fwd_kernel<false, GM>), grid, dim3(F::THREADS), 0, st, a);
    else
        hipLaunchKernelGGL((mlp_fwd_kernel<true, GM>), grid, dim3(F::THREADS), 0, st, a);
    return check_hip(hipGetLastError(), "mlp_fwd_kernel launch");
}

int launch_prep(const MlpArgs &a, hipStream_t st) {
    const int n = PREP_FIXED_BLOCKS + (a.n_rays + PREP_THREADS - 1) / PREP_THREADS +
                  (a.n_tiles + PREP_THREADS - 1) / PREP_THREADS;
    hipLaunchKernelGGL(mlp_prep_kernel, dim3(n), dim3(PREP_THREADS), 0, st, a);
    return check_hip(hipGetLastError(), "mlp_prep_kernel launch");
}

}  // namespace

extern "C" int dvgo_mlp_workspace_size(const dvgo_color_mlp *m, int32_t n_rays, int64_t n_samples, size_t *bytes) {
    int rc = check_mlp(m, false);
    if (rc) return rc;
    if (!bytes) return set_error(DVGO_ERR_NULL, "bytes is NULL");
    if (n_rays < 0 || n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative size");
    size_t a, b, c;
    *bytes = ws_layout(m, n_rays, n_samples, &a, &b, &c);
    return DVGO_OK;
}

extern "C" int dvgo_mlp_prepare(const dvgo_color_mlp *m, int32_t n_rays, const int32_t *ray_offsets,
                                const float *dirs, int64_t n_samples, void *ws, size_t ws_bytes, void *stream) {
    MlpArgs a;
    int rc = setup(m, n_rays, ray_offsets, dirs, n_samples, nullptr, ws, ws_bytes, false, a, false);
    if (rc) return rc;
    if (n_samples == 0) return DVGO_OK;
    return launch_prep(a, (hipStream_t)stream);
}

extern "C" int dvgo_mlp_forward(const dvgo_color_mlp *m, int32_t n_rays, const int32_t *ray_offsets,
                                const float *dirs, int64_t n_samples, const float *feat, float *rgb, void *ws,
                                size_t ws_bytes, void *stream) {
    MlpArgs a;
    int rc = setup(m, n_rays, ray_offsets, dirs, n_samples, feat, ws, ws_bytes, false, a);
    if (rc) return rc;
    if (n_samples == 0) return DVGO_OK;
    if (!rgb) return set_error(DVGO_ERR_NULL, "rgb is NULL");
    a.rgb = rgb;
    hipStream_t st = (hipStream_t)stream;
    if (!m->prepared) {
        rc = launch_prep(a, st);
        if (rc) return rc;
    }
    return launch_fwd<0>(a, m, st);
}

extern "C" int dvgo_mlp_forward_gather(const dvgo_color_mlp *m, int32_t n_rays, const int32_t *ray_offsets,
                                       const float *dirs, int64_t n_samples, const dvgo_grid *feat_grid,
                                       const float *xyz, float *feat_out, float *rgb, void *ws, size_t ws_bytes,
                                       void *stream) {
    MlpArgs a;
    int rc = setup(m, n_rays, ray_offsets, dirs, n_samples, nullptr, ws, ws_bytes, false, a, false);
    if (rc) return rc;
    rc = make_dev_grid(feat_grid, "feature grid", &a.fg, false);
    if (rc) return rc;
    if (feat_grid->channels != m->in_feat)
        return set_error(DVGO_ERR_SHAPE, "feature grid channels (%d) != in_feat (%d)", feat_grid->channels, m->in_feat);
    if ((m->in_feat & 3) || (feat_grid->ch_stride & 3) || ((uintptr_t)feat_grid->data & 15) ||
        ((uintptr_t)feat_out & 15))
        return set_error(DVGO_ERR_UNSUPPORTED,
                         "the fused gather needs in_feat and ch_stride multiples of 4 and 16-byte aligned data and "
                         "feat_out");
    if (n_samples == 0) return DVGO_OK;
    if (!rgb || !xyz) return set_error(DVGO_ERR_NULL, "rgb or xyz is NULL");
    a.rgb = rgb;
    a.xyz = xyz;
    a.feat_out = feat_out;
    hipStream_t st = (hipStream_t)stream;
    if (!m->prepared) {
        rc = launch_prep(a, st);
        if (rc) return rc;
    }
    return a.fg.warp ? launch_fwd<2>(a, m, st) : launch_fwd<1>(a, m, st);
}

namespace {

int launch_reduce(const MlpArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((a.n_params + 63) / 64), dim3(RED_THREADS), 0, st, a);
    return check_hip(hipGetLastError(), "mlp_reduce_kernel launch");
}

int mlp_backward_impl(const dvgo_color_mlp *m, int32_t n_rays, const int32_t *ray_offsets, const float *dirs,
                      int64_t n_samples, const float *feat, const float *grad_rgb, float *grad_feat, void *ws,
                      size_t ws_bytes, void *stream, bool reduce) {
    MlpArgs a;
    int rc = setup(m, n_rays, ray_offsets, dirs, n_samples, feat, ws, ws_bytes, true, a);
    if (rc) return rc;
    if (n_samples == 0) return DVGO_OK;
    if (!grad_rgb || !grad_feat) return set_error(DVGO_ERR_NULL, "grad_rgb or grad_feat is NULL");
    a.grad_rgb = grad_rgb;
    a.grad_feat = grad_feat;
    hipStream_t st = (hipStream_t)stream;
    if (!m->prepared) {
        rc = launch_prep(a, st);
        if (rc) return rc;
    }
    if (m->precision == DVGO_MLP_F16)
        hipLaunchKernelGGL((mlp_bwd_kernel<false>), dim3(a.nblocks), dim3(BWD_THREADS), 0, st, a);
    else
        hipLaunchKernelGGL((mlp_bwd_kernel<true>), dim3(a.nblocks), dim3(BWD_THREADS), 0, st, a);
    rc = check_hip(hipGetLastError(), "mlp_bwd_kernel launch");
    if (rc || !reduce) return rc;
    return launch_reduce(a, st);
}

}  // namespace

extern "C" int dvgo_mlp_backward(const dvgo_color_mlp *m, int32_t n_rays, const int32_t *ray_offsets,
                                 const float *dirs, int64_t n_samples, const float *feat, const float *grad_rgb,
                                 float *grad_feat, void *ws, size_t ws_bytes, void *stream) {
    return mlp_backward_impl(m, n_rays, ray_offsets, dirs, n_samples, feat, grad_rgb, grad_feat, ws, ws_bytes,
                             stream, true);
}

extern "C" int dvgo_mlp_backward_partials(const dvgo_color_mlp *m, int32_t n_rays, const int32_t *ray_offsets,
                                          const float *dirs, int64_t n_samples, const float *feat,
                                          const float *grad_rgb, float *grad_feat, void *ws, size_t ws_bytes,
                                          void *stream) {
    return mlp_backward_impl(m, n_rays, ray_offsets, dirs, n_samples, feat, grad_rgb, grad_feat, ws, ws_bytes,
                             stream, false);
}

extern "C" int dvgo_mlp_reduce_grads(const dvgo_color_mlp *m, int32_t n_rays, int64_t n_samples, void *ws,
                                     size_t ws_bytes, void *stream) {
    int rc = check_mlp(m, true);
    if (rc) return rc;
    if (n_rays < 0 || n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays or n_samples");
    if (n_samples >= ((int64_t)1 << 31) / 16) return set_error(DVGO_ERR_RANGE, "n_samples too large");
    size_t off_pe, off_tr, off_part;
    const size_t need = ws_layout(m, n_rays, n_samples, &off_pe, &off_tr, &off_part);
    if (!ws || ws_bytes < need) return set_error(DVGO_ERR_WORKSPACE, "workspace too small (%zu < %zu)", ws_bytes, need);
    if (((uintptr_t)ws & 255) != 0) return set_error(DVGO_ERR_SHAPE, "workspace must be 256-byte aligned");
    if (n_samples == 0) return DVGO_OK;
    MlpArgs a;
    memset(&a, 0, sizeof(a));
    a.gW1 = m->gW1; a.gb1 = m->gb1; a.gW2 = m->gW2; a.gb2 = m->gb2; a.gW3 = m->gW3; a.gb3 = m->gb3;
    a.in_feat = m->in_feat;
    a.n_freq = m->n_freq;
    a.n_in = n_in_of(m);
    a.n_params = n_params_of(m);
    a.partial = (float *)((char *)ws + off_part);
    a.nblocks = bwd_blocks(n_samples);
    return launch_reduce(a, (hipStream_t)stream);
}
