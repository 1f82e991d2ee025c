// Owner-computes scatter of per-sample values into a grid (the adjoint of the trilinear lookup,
// section 3's interpolation), optionally fused with the zero-gradient-skipping Adam update of
// section 3.
//
// The grid's vertices are cut into bricks of 4 x 4 x 32 (x, y, z) and every vertex belongs to
// exactly one brick.  The long edge runs along z, the fastest axis of the grid's layout, so that a
// one-channel brick row is one full 128-byte line: the write-back of a brick then touches no line
// that another brick also owns.  A sample's cell touches the bricks that own its eight corners: one, or two along each
// axis where the cell sits on a brick's upper face, so up to eight (sample, brick) pairs.  The
// pairs are counting-sorted by brick (count, one-block prefix, place; runs of equal bricks among
// the consecutive samples of a wave take one atomic).  Then one block per brick sums its pairs'
// contributions to the vertices it owns in LDS and writes every touched vertex once: either
// grad += sum (plain read-modify-write, no global atomics: no other block owns the vertex), or
// the Adam update of the vertex straight from the sum, so the dense gradient is never written to
// or read from memory.  Elements whose summed gradient is exactly zero are skipped, as the
// fused Adam of section 3 skips grid points without gradient.
#include <math.h>
#include <string.h>

#include "dvgo_internal.h"

using namespace dvgo;

namespace {

constexpr int OBX = 4, OBY = 4, OBZ = 32;  // owned vertices per brick edge
constexpr int OWN_BIN_WAVES = 4;

struct OwnGeom {
    int nb[3];  // bricks per axis
    int n;      // bricks
};

OwnGeom own_geom(const DevGrid &g) {
    OwnGeom o;
    o.n = 1;
    const int e[3] = {OBX, OBY, OBZ};
    for (int a = 0; a < 3; ++a) {
        o.nb[a] = (g.n[a] + e[a] - 1) / e[a];
        o.n *= o.nb[a];
    }
    return o;
}

// The j-th owner brick of a cell (j = 4 ex + 2 ey + ez: the upper neighbour along an axis where
// the cell's upper corners fall into the next brick), or -1.  Consecutive samples in one cell
// get the same keys in the same slots.
__device__ __forceinline__ int owner_key(const OwnGeom &o, const Cell &c, int j) {
    const int ex = (j >> 2) & 1, ey = (j >> 1) & 1, ez = j & 1;
    const int bx0 = c.ix / OBX, by0 = c.iy / OBY, bz0 = c.iz / OBZ;
    const int bx1 = (c.ix + 1) / OBX, by1 = (c.iy + 1) / OBY, bz1 = (c.iz + 1) / OBZ;
    if ((ex && bx1 == bx0) || (ey && by1 == by0) || (ez && bz1 == bz0)) return -1;
    return ((ex ? bx1 : bx0) * o.nb[1] + (ey ? by1 : by0)) * o.nb[2] + (ez ? bz1 : bz0);
}

struct OwnWs {
    int *offs;    // [n + 1] first pair of each brick in perm
    int *cursor;  // [n] counts, then placement cursors
    int *perm;    // [8 S] sample index of every pair, grouped by brick
};

size_t own_bytes(int nb, int64_t S, size_t *o_cursor, size_t *o_perm) {
    size_t o = align_up((size_t)(nb + 1) * 4, 256);
    *o_cursor = o;
    o += align_up((size_t)nb * 4, 256);
    *o_perm = o;
    o += (size_t)S * 8 * 4;
    return o;
}

__global__ __launch_bounds__(256) void own_zero_kernel(int *p, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}

template <bool W>
__global__ __launch_bounds__(64 * OWN_BIN_WAVES) void own_count_kernel(DevGrid g, OwnGeom o, int64_t S,
                                                                     const float *__restrict__ xyz, int *cnt) {
    const int64_t nwaves = (int64_t)gridDim.x * OWN_BIN_WAVES;
    for (int64_t base = (int64_t)(blockIdx.x * OWN_BIN_WAVES + (threadIdx.x >> 6)) * 64; base < S;
         base += nwaves * 64) {
        const int64_t k = base + lane();
        Cell c{0, 0, 0, 0.f, 0.f, 0.f};
        const bool valid = k < S;
        if (valid) c = cell_of<W>(g, xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2]);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int key = valid ? owner_key(o, c, j) : -1;
            if (__ballot(key >= 0) == 0ull) continue;
            const Run run = wave_runs(key);
            if (run.head) atomicAdd(&cnt[key], run.len);
        }
    }
}

// offs = exclusive prefix of cnt, offs[n] = total (one block, each thread one contiguous chunk);
// cnt is reset to zero for the placement cursors
__global__ __launch_bounds__(1024) void own_scan_kernel(int n, int *cnt, int *offs) {
    __shared__ int wsum[16];
    const int per = (n + 1023) / 1024;
    const int b = threadIdx.x * per, e = min(b + per, n);
    int sum = 0;
    for (int i = b; i < e; ++i) sum += cnt[i];
    int v = sum;  // inclusive scan of the chunk sums across the block
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(v, d, 64);
        if (lane() >= d) v += t;
    }
    if (lane() == 63) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x < 64) {
        int w = threadIdx.x < 16 ? wsum[threadIdx.x] : 0;
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) {
            const int t = __shfl_up(w, d, 64);
            if ((int)threadIdx.x >= d) w += t;
        }
        if (threadIdx.x < 16) wsum[threadIdx.x] = w;
    }
    __syncthreads();
    int run = v - sum + ((threadIdx.x >> 6) ? wsum[(threadIdx.x >> 6) - 1] : 0);
    for (int i = b; i < e; ++i) {
        const int c = cnt[i];
        offs[i] = run;
        run += c;
        cnt[i] = 0;
    }
    if (threadIdx.x == 0) offs[n] = wsum[15];
}

template <bool W>
__global__ __launch_bounds__(64 * OWN_BIN_WAVES) void own_place_kernel(DevGrid g, OwnGeom o, int64_t S,
                                                                     const float *__restrict__ xyz, const int *offs,
                                                                     int *cursor, int *perm) {
    const int64_t nwaves = (int64_t)gridDim.x * OWN_BIN_WAVES;
    for (int64_t base = (int64_t)(blockIdx.x * OWN_BIN_WAVES + (threadIdx.x >> 6)) * 64; base < S;
         base += nwaves * 64) {
        const int64_t k = base + lane();
        Cell c{0, 0, 0, 0.f, 0.f, 0.f};
        const bool valid = k < S;
        if (valid) c = cell_of<W>(g, xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2]);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int key = valid ? owner_key(o, c, j) : -1;
            if (__ballot(key >= 0) == 0ull) continue;
            const Run run = wave_runs(key);
            int start = 0;
            if (run.head) start = atomicAdd(&cursor[key], run.len);
            start = __shfl(start, run.head_lane, 64);
            if (key >= 0) perm[offs[key] + start + (lane() - run.head_lane)] = (int)k;
        }
    }
}

constexpr int OWN_THREADS = 256;
constexpr int OV = OBX * OBY * OBZ;  // owned vertices per brick

// LDS row of one owned vertex: NC channels, padded to an odd stride so that the lanes of one LDS
// atomic, which hold different vertices, spread over the banks
constexpr int tile_stride(int NC) { return NC == 1 ? 1 : (NC | 1); }

struct OwnArgs {
    DevGrid g;          // geometry (and warp) of the grid; grad: target of MODE 0
    OwnGeom o;
    const float *xyz;   // [S,3]
    const float *vals;  // [S, g.C]
    const int *offs, *perm;
    int vec_in;         // vals rows move as float4 (C % 4 == 0, 16-byte aligned)
    AdamArgs adam;      // MODE 1: p, m, v over the grid's layout; g unused
};

// MODE 0: g.grad += scatter.  MODE 1: Adam update of every element with a non-zero gradient.
// One block per brick: its pairs add their contributions to the corners the brick owns in an LDS
// tile (thread = pair; LDS atomics, corners visited in a lane-rotated order so that neighbouring
// lanes holding samples of one cell add to different vertices in the same instruction); then every
// touched vertex is written once.  The LDS atomics cost grows with the channel count: this is the
// density's scatter (one channel); the 12-channel features keep the in-wave aggregated global
// atomics of dvgo_grid_scatter.
template <int NC, bool W, int MODE>
__global__ __launch_bounds__(OWN_THREADS) void own_scatter_kernel(OwnArgs A) {
    constexpr int TS = tile_stride(NC);
    __shared__ float tile[OV * TS];
    const int b = blockIdx.x;
    const int beg = A.offs[b], end = A.offs[b + 1];
    if (beg == end) return;
    const DevGrid &g = A.g;
    const int C = g.C;
    const int bz = b % A.o.nb[2], by = (b / A.o.nb[2]) % A.o.nb[1], bx = b / (A.o.nb[2] * A.o.nb[1]);
    const int x0 = bx * OBX, y0 = by * OBY, z0 = bz * OBZ;
    for (int i = threadIdx.x; i < OV * TS; i += OWN_THREADS) tile[i] = 0.f;
    __syncthreads();
    const int rot = lane() & 7;
    for (int i = beg + threadIdx.x; i < end; i += OWN_THREADS) {
        const int64_t s = A.perm[i];
        const Cell c = cell_of<W>(g, A.xyz[3 * s], A.xyz[3 * s + 1], A.xyz[3 * s + 2]);
        float val[NC];
        if (NC % 4 == 0 && A.vec_in) {
#pragma unroll
            for (int q = 0; q < NC / 4; ++q) {
                const float4 t = 4 * q < C ? *reinterpret_cast<const float4 *>(A.vals + s * C + 4 * q)
                                           : make_float4(0.f, 0.f, 0.f, 0.f);
                val[4 * q] = t.x;
                val[4 * q + 1] = t.y;
                val[4 * q + 2] = t.z;
                val[4 * q + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) val[ch] = ch < C ? A.vals[s * C + ch] : 0.f;
        }
        const int lx = c.ix - x0, ly = c.iy - y0, lz = c.iz - z0;  // from -1 to the brick edge - 1
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int corner = (k + rot) & 7;
            const int dx = (corner >> 2) & 1, dy = (corner >> 1) & 1, dz = corner & 1;
            const int vx = lx + dx, vy = ly + dy, vz = lz + dz;
            if ((unsigned)vx >= (unsigned)OBX || (unsigned)vy >= (unsigned)OBY || (unsigned)vz >= (unsigned)OBZ) continue;
            const float w = corner_weight(c, dx, dy, dz);
            float *t = tile + ((vx * OBY + vy) * OBZ + vz) * TS;
#pragma unroll
            for (int ch = 0; ch < NC; ++ch)
                if (ch < C) atomicAdd(t + ch, w * val[ch]);
        }
    }
    __syncthreads();
    // write: element e = (row (vx, vy), f = vz C + ch), f fastest, so consecutive lanes cover
    // consecutive addresses of one brick row
    const int rowlen = OBZ * C;
    AdamArgs ad = A.adam;
    if (MODE == 1) adam_bias(ad);
    for (int e = threadIdx.x; e < OBX * OBY * rowlen; e += OWN_THREADS) {
        const int row = e / rowlen, f = e - row * rowlen;
        const int vz = f / C, ch = f - vz * C, vx = row / OBY, vy = row - vx * OBY;
        const int gx = x0 + vx, gy = y0 + vy, gz = z0 + vz;
        const float t = tile[((vx * OBY + vy) * OBZ + vz) * TS + ch];
        if (t == 0.f || gx >= g.n[0] || gy >= g.n[1] || gz >= g.n[2]) continue;
        const int64_t off = (int64_t)gx * g.sx + (int64_t)gy * g.sy + (int64_t)gz * g.cs + ch;
        if (MODE == 0) {
            g.grad[off] += t;
        } else {
            float p = ad.p[off];
            float m = __builtin_nontemporal_load(ad.m + off);
            float v = __builtin_nontemporal_load(ad.v + off);
            adam_one(ad, t, p, m, v);
            ad.p[off] = p;
            __builtin_nontemporal_store(m, ad.m + off);
            __builtin_nontemporal_store(v, ad.v + off);
        }
    }
}

template <int NC, int MODE>
void launch_own(const OwnArgs &A, hipStream_t st) {
    if (A.g.warp)
        hipLaunchKernelGGL((own_scatter_kernel<NC, true, MODE>), dim3(A.o.n), dim3(OWN_THREADS), 0, st, A);
    else
        hipLaunchKernelGGL((own_scatter_kernel<NC, false, MODE>), dim3(A.o.n), dim3(OWN_THREADS), 0, st, A);
}

template <int MODE>
void launch_own_c(const OwnArgs &A, hipStream_t st) {
    const int C = A.g.C;
    if (C == 1) launch_own<1, MODE>(A, st);
    else if (C <= 3) launch_own<3, MODE>(A, st);
    else if (C <= 4) launch_own<4, MODE>(A, st);
    else if (C <= 8) launch_own<8, MODE>(A, st);
    else if (C <= 12) launch_own<12, MODE>(A, st);
    else launch_own<16, MODE>(A, st);
}

int own_setup(const dvgo_grid *g, int64_t S, const void *ws, size_t ws_bytes, DevGrid &dg, OwnGeom &o, OwnWs &w,
              bool need_grad) {
    int rc = make_dev_grid(g, "grid", &dg, need_grad);
    if (rc) return rc;
    if (S < 0) return set_error(DVGO_ERR_SHAPE, "negative n_samples");
    if (S > MAX_SAMPLES / 8) return set_error(DVGO_ERR_RANGE, "n_samples must be at most %lld", (long long)(MAX_SAMPLES / 8));
    o = own_geom(dg);
    size_t oc, op;
    const size_t need = own_bytes(o.n, S, &oc, &op);
    if (!ws || ws_bytes < need) return set_error(DVGO_ERR_WORKSPACE, "owner workspace too small (%zu < %zu)", ws_bytes, need);
    if (((uintptr_t)ws & 255) != 0) return set_error(DVGO_ERR_SHAPE, "owner workspace must be 256-byte aligned");
    w.offs = (int *)ws;
    w.cursor = (int *)((char *)ws + oc);
    w.perm = (int *)((char *)ws + op);
    return DVGO_OK;
}

int own_blocks(int64_t S) {
    const int64_t b = (S + 64 * OWN_BIN_WAVES - 1) / (64 * OWN_BIN_WAVES);
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

int fill_own_args(const dvgo_grid *g, int64_t S, const float *xyz, const float *vals, const void *ws, size_t ws_bytes,
                  bool need_grad, OwnArgs &A) {
    memset(&A, 0, sizeof(A));
    OwnWs w;
    int rc = own_setup(g, S, ws, ws_bytes, A.g, A.o, w, need_grad);
    if (rc) return rc;
    if (S > 0 && (!xyz || !vals)) return set_error(DVGO_ERR_NULL, "xyz or grad_out is NULL");
    A.xyz = xyz;
    A.vals = vals;
    A.offs = w.offs;
    A.perm = w.perm;
    A.vec_in = (A.g.C % 4 == 0 && ((uintptr_t)vals & 15) == 0) ? 1 : 0;
    return DVGO_OK;
}

}  // namespace

extern "C" int dvgo_owner_workspace_size(const dvgo_grid *g, int64_t n_samples, size_t *bytes) {
    DevGrid dg;
    int rc = make_dev_grid(g, "grid", &dg, false);
    if (rc) return rc;
    if (!bytes) return set_error(DVGO_ERR_NULL, "bytes is NULL");
    if (n_samples < 0) return set_error(DVGO_ERR_SHAPE, "negative n_samples");
    size_t a, b;
    *bytes = own_bytes(own_geom(dg).n, n_samples, &a, &b);
    return DVGO_OK;
}

extern "C" int dvgo_owner_bin(const dvgo_grid *g, int64_t n_samples, const float *xyz, void *ws, size_t ws_bytes,
                              void *stream) {
    DevGrid dg;
    OwnGeom o;
    OwnWs w;
    int rc = own_setup(g, n_samples, ws, ws_bytes, dg, o, w, false);
    if (rc) return rc;
    if (n_samples > 0 && !xyz) return set_error(DVGO_ERR_NULL, "xyz is NULL");
    const hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(own_zero_kernel, dim3((o.n + 255) / 256 < 1024 ? (o.n + 255) / 256 : 1024), dim3(256), 0, st,
                       w.cursor, o.n);
    const int nb = own_blocks(n_samples);
    if (n_samples > 0) {
        if (dg.warp)
            hipLaunchKernelGGL(own_count_kernel<true>, dim3(nb), dim3(64 * OWN_BIN_WAVES), 0, st, dg, o, n_samples, xyz,
                               w.cursor);
        else
            hipLaunchKernelGGL(own_count_kernel<false>, dim3(nb), dim3(64 * OWN_BIN_WAVES), 0, st, dg, o, n_samples,
                               xyz, w.cursor);
    }
    hipLaunchKernelGGL(own_scan_kernel, dim3(1), dim3(1024), 0, st, o.n, w.cursor, w.offs);
    if (n_samples > 0) {
        if (dg.warp)
            hipLaunchKernelGGL(own_place_kernel<true>, dim3(nb), dim3(64 * OWN_BIN_WAVES), 0, st, dg, o, n_samples, xyz,
                               w.offs, w.cursor, w.perm);
        else
            hipLaunchKernelGGL(own_place_kernel<false>, dim3(nb), dim3(64 * OWN_BIN_WAVES), 0, st, dg, o, n_samples,
                               xyz, w.offs, w.cursor, w.perm);
    }
    return check_hip(hipGetLastError(), "owner binning launch");
}

extern "C" int dvgo_grid_scatter_owned(const dvgo_grid *g, int64_t n_samples, const float *xyz, const float *grad_out,
                                       const void *ws, size_t ws_bytes, void *stream) {
    OwnArgs A;
    int rc = fill_own_args(g, n_samples, xyz, grad_out, ws, ws_bytes, true, A);
    if (rc) return rc;
    if (n_samples == 0) return DVGO_OK;
    launch_own_c<0>(A, (hipStream_t)stream);
    return check_hip(hipGetLastError(), "own_scatter_kernel launch");
}

extern "C" int dvgo_grid_scatter_adam(const dvgo_grid *g, int64_t n_samples, const float *xyz, const float *grad_out,
                                      const void *ws, size_t ws_bytes, float *param, float *exp_avg, float *exp_avg_sq,
                                      float lr, float beta1, float beta2, float eps, int32_t step,
                                      const int32_t *step_dev, void *stream) {
    OwnArgs A;
    int rc = fill_own_args(g, n_samples, xyz, grad_out, ws, ws_bytes, false, A);
    if (rc) return rc;
    if (!param || !exp_avg || !exp_avg_sq) return set_error(DVGO_ERR_NULL, "param or a moment is NULL");
    if (!step_dev && step < 1) return set_error(DVGO_ERR_RANGE, "step is 1-based");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f))
        return set_error(DVGO_ERR_RANGE, "betas must be in [0, 1)");
    if (n_samples == 0) return DVGO_OK;
    AdamArgs &a = A.adam;
    a.p = param;
    a.g = nullptr;
    a.m = exp_avg;
    a.v = exp_avg_sq;
    a.n = (int64_t)g->nx * g->ny * g->nz * g->ch_stride;
    const int t = step_dev ? 1 : step;
    const double bc1 = 1.0 - pow((double)beta1, t), bc2 = 1.0 - pow((double)beta2, t);
    a.lr_t = (float)((double)lr / bc1);
    a.inv_sqrt_bc2 = (float)(1.0 / sqrt(bc2));
    a.lr = lr;
    a.step_dev = step_dev;
    a.b1 = beta1;
    a.b2 = beta2;
    a.eps = eps;
    a.skip = 1;
    a.zero = 0;
    launch_own_c<1>(A, (hipStream_t)stream);
    return check_hip(hipGetLastError(), "own_scatter_kernel launch");
}
