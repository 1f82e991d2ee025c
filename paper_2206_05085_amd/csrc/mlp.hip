// Colour MLP of the hybrid representation (Table 1): [features, view encoding] -> 128 ->
// 128 -> RGB, forward and backward on gfx950 FP32 matrix cores (v_mfma_f32_16x16x4_f32).
//
// Layout.  Activations are kept "hidden-major": a 16x16 MFMA tile holds 16 hidden units
// (rows) x 16 samples (columns), and lane (q = lane/16, j = lane%16) owns rows 4q..4q+3
// of column j.  The next layer consumes a tile in place by ordering its reduction index
// as k = 16*tile + 4q + r: the B operand of K-step (tile, r) is the lane's own r-th
// accumulator element, and the matching A operand W[out][16*tile + 4q + r] is four
// consecutive floats of one weight row (one 16-byte LDS read for four K-steps).
// Weight gradients reduce over samples, so their operands are staged through LDS with
// samples as rows and each block accumulates a private partial that a second kernel sums.
#include <string.h>

#include "dvgo_internal.h"

using namespace dvgo;

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int H = 128;      // hidden width
constexpr int KX = 48;      // padded input width: features in columns 0..11, encoding in 12..47
constexpr int PEW = 36;     // per-ray encoding row (input columns 12..47)
constexpr int W2S = 132;    // LDS row stride of W2 (floats)
constexpr int W1S = 52;     // LDS row stride of W1 (forward)
constexpr int SH = 144;     // LDS row stride of staged [sample][hidden] tiles
constexpr int XS = 52;      // LDS row stride of staged inputs
constexpr int FWD_THREADS = 512, FWD_TILE = 128;
constexpr int BWD_THREADS = 256, BWD_TILE = 64;
constexpr int MAX_BLOCKS = 256;

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

struct MlpArgs {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    int in_feat, n_in;  // n_in = in_feat + 3 + 6 F (columns of W1)
    int n_freq;
    int n_rays;
    const int *offs;
    const float *dirs;
    int S;
    const float *feat;
    float *rgb;
    float *W1p;   // [H][KX] W1 with columns moved to the padded input layout (workspace)
    float *pe;    // [R][PEW] view encodings (workspace)
    const float *grad_rgb;
    float *grad_feat;
    float *partial;  // [blocks][n_params] (workspace)
    int n_params;
    float *gW1, *gb1, *gW2, *gb2, *gW3, *gb3;
    int nblocks;
};

// padded input column k of W1p -> column of W1 (or -1 for padding)
__device__ __forceinline__ int w1_col(const MlpArgs &a, int k) {
    if (k < 12) return k < a.in_feat ? k : -1;
    const int p = k - 12;
    return p < 3 + 6 * a.n_freq ? a.in_feat + p : -1;
}

__global__ void mlp_prep_kernel(MlpArgs a) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < H * KX) {
        const int h = tid / KX, k = tid % KX;
        const int c = w1_col(a, k);
        a.W1p[tid] = c >= 0 ? a.W1[h * a.n_in + c] : 0.f;
    }
    const int r = tid - H * KX;
    if (r >= 0 && r < a.n_rays) {
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

__device__ __forceinline__ int find_ray(const int *offs, int R, int s) {
    int lo = 0, hi = R - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= s) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// input element x[s][16 kb + 4 q + r] of this lane's sample
__device__ __forceinline__ void load_inputs(const MlpArgs &a, int s, bool sv, int q, float xin[3][4]) {
    int ray = sv ? find_ray(a.offs, a.n_rays, s) : 0;
    const float *pe = a.pe + (int64_t)ray * PEW;
#pragma unroll
    for (int kb = 0; kb < 3; ++kb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = 16 * kb + 4 * q + r;
            float v = 0.f;
            if (sv) {
                if (k < 12) v = k < a.in_feat ? a.feat[(int64_t)s * a.in_feat + k] : 0.f;
                else v = pe[k - 12];
            }
            xin[kb][r] = v;
        }
}

// Forward of the three layers for the 16 samples of this wave; returns h1, h2 (post-ReLU)
// and the pre-sigmoid output z3 (rows 0..2 of acc3 in lanes q == 0).
template <bool W1_IN_LDS>
__device__ __forceinline__ void mlp_forward_tile(const MlpArgs &a, const float *W1src, int w1s, const float *W2s,
                                                 const float xin[3][4], int q, int j, v4f acc1[8], v4f acc2[8],
                                                 v4f &acc3) {
#pragma unroll
    for (int m = 0; m < 8; ++m) acc1[m] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 3; ++kb) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const float4 w = *reinterpret_cast<const float4 *>(W1src + (16 * m + j) * w1s + 16 * kb + 4 * q);
            acc1[m] = mfma4(w.x, xin[kb][0], acc1[m]);
            acc1[m] = mfma4(w.y, xin[kb][1], acc1[m]);
            acc1[m] = mfma4(w.z, xin[kb][2], acc1[m]);
            acc1[m] = mfma4(w.w, xin[kb][3], acc1[m]);
        }
    }
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc1[m][r] = fmaxf(acc1[m][r] + a.b1[16 * m + 4 * q + r], 0.f);
#pragma unroll
    for (int m = 0; m < 8; ++m) acc2[m] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 8; ++t) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const float4 w = *reinterpret_cast<const float4 *>(W2s + (16 * m + j) * W2S + 16 * t + 4 * q);
            acc2[m] = mfma4(w.x, acc1[t][0], acc2[m]);
            acc2[m] = mfma4(w.y, acc1[t][1], acc2[m]);
            acc2[m] = mfma4(w.z, acc1[t][2], acc2[m]);
            acc2[m] = mfma4(w.w, acc1[t][3], acc2[m]);
        }
        // keep the scheduler from hoisting every weight load of the layer (register spills)
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc2[m][r] = fmaxf(acc2[m][r] + a.b2[16 * m + 4 * q + r], 0.f);
    acc3 = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 8; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float w = j < 3 ? a.W3[j * H + 16 * t + 4 * q + r] : 0.f;
            acc3 = mfma4(w, acc2[t][r], acc3);
        }
    }
}

__global__ __launch_bounds__(FWD_THREADS) void mlp_fwd_kernel(MlpArgs a) {
    __shared__ float W2s[H * W2S];
    __shared__ float W1s[H * W1S];
    for (int i = threadIdx.x; i < H * H; i += FWD_THREADS) W2s[(i / H) * W2S + (i % H)] = a.W2[i];
    for (int i = threadIdx.x; i < H * KX; i += FWD_THREADS) W1s[(i / KX) * W1S + (i % KX)] = a.W1p[i];
    __syncthreads();
    const int wv = threadIdx.x >> 6, ln = lane(), j = ln & 15, q = ln >> 4;
    const int ntiles = (a.S + FWD_TILE - 1) / FWD_TILE;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int s = tile * FWD_TILE + wv * 16 + j;
        const bool sv = s < a.S;
        float xin[3][4];
        load_inputs(a, s, sv, q, xin);
        v4f acc1[8], acc2[8], acc3;
        mlp_forward_tile<true>(a, W1s, W1S, W2s, xin, q, j, acc1, acc2, acc3);
        if (q == 0 && sv) {
#pragma unroll
            for (int r = 0; r < 3; ++r) a.rgb[(int64_t)s * 3 + r] = sigmoidf(acc3[r] + a.b3[r]);
        }
    }
}

__global__ __launch_bounds__(BWD_THREADS) void mlp_bwd_kernel(MlpArgs a) {
    __shared__ float W2s[H * W2S];
    __shared__ float bufA[BWD_TILE * SH];
    __shared__ float bufB[BWD_TILE * SH];
    __shared__ float xs[BWD_TILE * XS];
    __shared__ float dz3s[BWD_TILE * 4];
    for (int i = threadIdx.x; i < H * H; i += BWD_THREADS) W2s[(i / H) * W2S + (i % H)] = a.W2[i];
    __syncthreads();
    const int tid = threadIdx.x;
    const int wv = tid >> 6, ln = lane(), j = ln & 15, q = ln >> 4;
    v4f dW2acc[2][8], dW1acc[2][3], dW3acc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int t = 0; t < 8; ++t) dW2acc[i][t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 3; ++t) dW1acc[i][t] = v4f{0.f, 0.f, 0.f, 0.f};
        dW3acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    float db_acc = 0.f;   // threads 0..127: b2[tid] (phase 1) and b1[tid] (phase 2) share nothing
    float db1_acc = 0.f;
    float db3_acc = 0.f;  // threads 128..130
    const int ntiles = (a.S + BWD_TILE - 1) / BWD_TILE;
    const int row = wv * 16 + j;  // this lane's sample row inside the tile
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int s = tile * BWD_TILE + row;
        const bool sv = s < a.S;
        float xin[3][4];
        load_inputs(a, s, sv, q, xin);
#pragma unroll
        for (int kb = 0; kb < 3; ++kb)
            *reinterpret_cast<float4 *>(&xs[row * XS + 16 * kb + 4 * q]) =
                make_float4(xin[kb][0], xin[kb][1], xin[kb][2], xin[kb][3]);
        v4f acc1[8], acc2[8], acc3;
        mlp_forward_tile<false>(a, a.W1p, KX, W2s, xin, q, j, acc1, acc2, acc3);
        // output layer: dz3 = dL/drgb * y (1 - y) (lanes q == 0 hold rows o = 0..3)
        float dz3v[4] = {0.f, 0.f, 0.f, 0.f};
        if (q == 0 && sv) {
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const float y = sigmoidf(acc3[r] + a.b3[r]);
                dz3v[r] = a.grad_rgb[(int64_t)s * 3 + r] * y * (1.f - y);
            }
        }
        if (q == 0) *reinterpret_cast<float4 *>(&dz3s[row * 4]) = make_float4(dz3v[0], dz3v[1], dz3v[2], dz3v[3]);
        // B operand dz3[o = q][s_j] lives in lane (0, j), element q
        float bq = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float t = __shfl(dz3v[r], j, 64);
            if (q == r) bq = t;
        }
        // dh2 = W3^T dz3 (one K-step over o), then ReLU mask of layer 2
        v4f dz2[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const float w = q < 3 ? a.W3[q * H + 16 * m + j] : 0.f;
            dz2[m] = mfma4(w, bq, v4f{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int r = 0; r < 4; ++r) dz2[m][r] = acc2[m][r] > 0.f ? dz2[m][r] : 0.f;
        }
        // dh1 = W2^T dz2: reduction over h' = 16 t + 4 q + r, A = W2[h'][16 m + j]
        v4f dz1[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) dz1[m] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 8; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float *wrow = W2s + (16 * t + 4 * q + r) * W2S + j;
#pragma unroll
                for (int m = 0; m < 8; ++m) dz1[m] = mfma4(wrow[16 * m], dz2[t][r], dz1[m]);
            }
        }
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) dz1[m][r] = acc1[m][r] > 0.f ? dz1[m][r] : 0.f;
        // dfeat = W1f^T dz1: rows = feature column c = j (< 12), reduction over h
        v4f df = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float w = j < 12 ? a.W1p[(16 * m + 4 * q + r) * KX + j] : 0.f;
                df = mfma4(w, dz1[m][r], df);
            }
        if (sv) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = 4 * q + r;
                if (c < a.in_feat) a.grad_feat[(int64_t)s * a.in_feat + c] = df[r];
            }
        }
        // ---- phase 1: dW2 = sum_s dz2 h1^T, db2 = sum_s dz2
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            *reinterpret_cast<float4 *>(&bufA[row * SH + 16 * m + 4 * q]) =
                make_float4(dz2[m][0], dz2[m][1], dz2[m][2], dz2[m][3]);
            *reinterpret_cast<float4 *>(&bufB[row * SH + 16 * m + 4 * q]) =
                make_float4(acc1[m][0], acc1[m][1], acc1[m][2], acc1[m][3]);
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < BWD_TILE / 4; ++ks) {
            const float *ra = bufA + (4 * ks + q) * SH + j;
            const float *rb = bufB + (4 * ks + q) * SH + j;
            const float a0 = ra[16 * (2 * wv)], a1 = ra[16 * (2 * wv + 1)];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float bv = rb[16 * t];
                dW2acc[0][t] = mfma4(a0, bv, dW2acc[0][t]);
                dW2acc[1][t] = mfma4(a1, bv, dW2acc[1][t]);
            }
        }
        if (tid < H) {
            float sacc = 0.f;
            for (int r = 0; r < BWD_TILE; ++r) sacc += bufA[r * SH + tid];
            db_acc += sacc;
        }
        __syncthreads();
        // ---- phase 2: dW1 = sum_s dz1 x^T, dW3 = sum_s dz3 h2^T, db1, db3
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            *reinterpret_cast<float4 *>(&bufA[row * SH + 16 * m + 4 * q]) =
                make_float4(dz1[m][0], dz1[m][1], dz1[m][2], dz1[m][3]);
            *reinterpret_cast<float4 *>(&bufB[row * SH + 16 * m + 4 * q]) =
                make_float4(acc2[m][0], acc2[m][1], acc2[m][2], acc2[m][3]);
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < BWD_TILE / 4; ++ks) {
            const int sr = 4 * ks + q;
            const float a0 = bufA[sr * SH + 16 * (2 * wv) + j], a1 = bufA[sr * SH + 16 * (2 * wv + 1) + j];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const float bv = xs[sr * XS + 16 * t + j];
                dW1acc[0][t] = mfma4(a0, bv, dW1acc[0][t]);
                dW1acc[1][t] = mfma4(a1, bv, dW1acc[1][t]);
            }
            const float a3 = j < 3 ? dz3s[sr * 4 + j] : 0.f;
            dW3acc[0] = mfma4(a3, bufB[sr * SH + 16 * (2 * wv) + j], dW3acc[0]);
            dW3acc[1] = mfma4(a3, bufB[sr * SH + 16 * (2 * wv + 1) + j], dW3acc[1]);
        }
        if (tid < H) {
            float sacc = 0.f;
            for (int r = 0; r < BWD_TILE; ++r) sacc += bufA[r * SH + tid];
            db1_acc += sacc;
        } else if (tid < H + 3) {
            float sacc = 0.f;
            for (int r = 0; r < BWD_TILE; ++r) sacc += dz3s[r * 4 + (tid - H)];
            db3_acc += sacc;
        }
        __syncthreads();
    }
    // ---- write this block's partial gradients in parameter order W1, b1, W2, b2, W3, b3
    float *P = a.partial + (int64_t)blockIdx.x * a.n_params;
    float *pW1 = P, *pb1 = pW1 + H * a.n_in, *pW2 = pb1 + H, *pb2 = pW2 + H * H, *pW3 = pb2 + H, *pb3 = pW3 + 3 * H;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int m = 2 * wv + i;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int hrow = 16 * m + 4 * q + r;
#pragma unroll
            for (int t = 0; t < 8; ++t) pW2[hrow * H + 16 * t + j] = dW2acc[i][t][r];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const int c = w1_col(a, 16 * t + j);
                if (c >= 0) pW1[hrow * a.n_in + c] = dW1acc[i][t][r];
            }
            if (q == 0 && r < 3) pW3[r * H + 16 * (2 * wv + i) + j] = dW3acc[i][r];
        }
    }
    if (tid < H) {
        pb2[tid] = db_acc;
        pb1[tid] = db1_acc;
    } else if (tid < H + 3) {
        pb3[tid - H] = db3_acc;
    }
}

// gradient += sum of the per-block partials
__global__ void mlp_reduce_kernel(MlpArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_params) return;
    float acc = 0.f;
    for (int b = 0; b < a.nblocks; ++b) acc += a.partial[(int64_t)b * a.n_params + i];
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
    if (m->n_freq < 0 || m->n_freq > 4) return set_error(DVGO_ERR_UNSUPPORTED, "n_freq must be in [0, 4]");
    if (!m->W1 || !m->b1 || !m->W2 || !m->b2 || !m->W3 || !m->b3) return set_error(DVGO_ERR_NULL, "a weight is NULL");
    if (bwd && (!m->gW1 || !m->gb1 || !m->gW2 || !m->gb2 || !m->gW3 || !m->gb3))
        return set_error(DVGO_ERR_NULL, "a weight gradient is NULL");
    return DVGO_OK;
}

int n_in_of(const dvgo_color_mlp *m) { return m->in_feat + 3 + 6 * m->n_freq; }
int n_params_of(const dvgo_color_mlp *m) { return H * n_in_of(m) + H + H * H + H + 3 * H + 3; }
int bwd_blocks(int64_t S) {
    int64_t t = (S + BWD_TILE - 1) / BWD_TILE;
    return (int)(t < MAX_BLOCKS ? (t < 1 ? 1 : t) : MAX_BLOCKS);
}

size_t ws_layout(const dvgo_color_mlp *m, int32_t R, int64_t S, size_t *off_pe, size_t *off_part) {
    size_t o = align_up((size_t)H * KX * 4, 256);
    *off_pe = o;
    o += align_up((size_t)R * PEW * 4, 256);
    *off_part = o;
    o += (size_t)bwd_blocks(S) * n_params_of(m) * 4;
    return o;
}

int setup(const dvgo_color_mlp *m, int32_t R, const int32_t *offs, const float *dirs, int64_t S, const float *feat,
          void *ws, size_t ws_bytes, bool bwd, MlpArgs &a) {
    int rc = check_mlp(m, bwd);
    if (rc) return rc;
    if (R < 0 || S < 0) return set_error(DVGO_ERR_SHAPE, "negative n_rays or n_samples");
    if (S >= ((int64_t)1 << 31) / 16) return set_error(DVGO_ERR_RANGE, "n_samples too large");
    if (S > 0 && (R == 0 || !offs || !dirs || !feat)) return set_error(DVGO_ERR_NULL, "ray_offsets, dirs or feat is NULL");
    size_t off_pe, off_part;
    const size_t need = ws_layout(m, R, S, &off_pe, &off_part);
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
    a.W1p = (float *)ws;
    a.pe = (float *)((char *)ws + off_pe);
    a.partial = (float *)((char *)ws + off_part);
    a.nblocks = bwd_blocks(S);
    return DVGO_OK;
}

int launch_prep(const MlpArgs &a, hipStream_t st) {
    const int n = H * KX + a.n_rays;
    hipLaunchKernelGGL(mlp_prep_kernel, dim3((n + 255) / 256), dim3(256), 0, st, a);
    return check_hip(hipGetLastError(), "mlp_prep_kernel launch");
}

}  // namespace

extern "C" int dvgo_mlp_workspace_size(const dvgo_color_mlp *m, int32_t n_rays, int64_t n_samples, size_t *bytes) {
    int rc = check_mlp(m, false);
    if (rc) return rc;
    if (!bytes) return set_error(DVGO_ERR_NULL, "bytes is NULL");
    if (n_rays < 0 || n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative size");
    size_t a, b;
    *bytes = ws_layout(m, n_rays, n_samples, &a, &b);
    return DVGO_OK;
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
    rc = launch_prep(a, st);
    if (rc) return rc;
    const int ntiles = (int)((n_samples + FWD_TILE - 1) / FWD_TILE);
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(ntiles < MAX_BLOCKS ? ntiles : MAX_BLOCKS), dim3(FWD_THREADS), 0, st, a);
    return check_hip(hipGetLastError(), "mlp_fwd_kernel launch");
}

extern "C" int dvgo_mlp_backward(const dvgo_color_mlp *m, int32_t n_rays, const int32_t *ray_offsets,
                                 const float *dirs, int64_t n_samples, const float *feat, const float *grad_rgb,
                                 float *grad_feat, void *ws, size_t ws_bytes, void *stream) {
    MlpArgs a;
    int rc = setup(m, n_rays, ray_offsets, dirs, n_samples, feat, ws, ws_bytes, true, a);
    if (rc) return rc;
    if (n_samples == 0) return DVGO_OK;
    if (!grad_rgb || !grad_feat) return set_error(DVGO_ERR_NULL, "grad_rgb or grad_feat is NULL");
    a.grad_rgb = grad_rgb;
    a.grad_feat = grad_feat;
    hipStream_t st = (hipStream_t)stream;
    rc = launch_prep(a, st);
    if (rc) return rc;
    hipLaunchKernelGGL(mlp_bwd_kernel, dim3(a.nblocks), dim3(BWD_THREADS), 0, st, a);
    rc = check_hip(hipGetLastError(), "mlp_bwd_kernel launch");
    if (rc) return rc;
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((a.n_params + 255) / 256), dim3(256), 0, st, a);
    return check_hip(hipGetLastError(), "mlp_reduce_kernel launch");
}
