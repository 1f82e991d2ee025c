// Internal helpers shared by the gfx950 kernels of libdvgo (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dvgo.h"

namespace dvgo {

// ----------------------------------------------------------------------------- wave64

// All scans run across the 64 lanes of one wavefront (CDNA wave64).
__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// inclusive prefix sum: lane l gets sum of lanes 0..l
__device__ __forceinline__ float wave_incl(float v) {
    const int l = lane();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        float t = __shfl_up(v, d, 64);
        if (l >= d) v += t;
    }
    return v;
}

// exclusive prefix from an inclusive one (lane 0 gets 0); exact, no subtraction
__device__ __forceinline__ float wave_excl(float incl) {
    float t = __shfl_up(incl, 1, 64);
    return lane() == 0 ? 0.f : t;
}

// inclusive suffix sum: lane l gets sum of lanes l..63
__device__ __forceinline__ float wave_incl_rev(float v) {
    const int l = lane();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        float t = __shfl_down(v, d, 64);
        if (l + d < 64) v += t;
    }
    return v;
}

// exclusive suffix from an inclusive suffix (lane 63 gets 0)
__device__ __forceinline__ float wave_excl_rev(float incl_rev) {
    float t = __shfl_down(incl_rev, 1, 64);
    return lane() == 63 ? 0.f : t;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ float bcast(float v, int src) { return __shfl(v, src, 64); }

// --------------------------------------------------------------------------- math

__device__ __forceinline__ float softplusf(float z) {
    return z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z));
}

__device__ __forceinline__ float sigmoidf(float z) {
    if (z >= 0.f) return 1.f / (1.f + expf(-z));
    float e = expf(z);
    return e / (1.f + e);
}

// --------------------------------------------------------------------------- grids

// Device view of a dvgo_grid.  The world->index map u = x*s + o per axis is carried as
// double-float pairs (hi + lo) so the cell index and the fractional position are exact to
// float32 precision of the fraction itself, not of u (u reaches 319 on a 320^3 grid).
struct DevGrid {
    const float *data;
    float *grad;
    int n[3];
    int cs;  // floats per vertex
    int C;   // channels used
    int sx, sy;  // strides (floats) of x and y; z stride is cs
    float s_hi[3], s_lo[3], o_hi[3], o_lo[3];
    int warp;              // DVGO_WARP_*: 0 = points index the box directly
    double wb;             // b of Eq. 4
    double s_d[3], o_d[3]; // the index map u = x*s + o in double, for warped points
};

struct Tri {
    int base;     // float offset of corner (0,0,0)
    float w[8];   // corner c = 4dx + 2dy + dz
};

// Cell index i0 in [0, n-2] and fraction f in [0, 1] of coordinate x on one axis.
__device__ __forceinline__ void axis_coord(float x, float shi, float slo, float ohi, float olo, int n, int &i0,
                                           float &f) {
    // The error-free transforms below need each operation rounded on its own: an FMA
    // formed from x*shi + ohi would break the two-sum.
#pragma clang fp contract(off)
    // x*shi exactly as p + pe (FMA), then p + ohi exactly as u + e (two-sum)
    float p = x * shi;
    float pe = fmaf(x, shi, -p);
    float u = p + ohi;
    float bb = u - p;
    float e = (p - (u - bb)) + (ohi - bb);
    float lo = e + pe + fmaf(x, slo, olo);
    float fl = floorf(u);
    float fr = (u - fl) + lo;  // u - fl is exact
    if (fr < 0.f) { fl -= 1.f; fr += 1.f; }
    else if (fr >= 1.f) { fl += 1.f; fr -= 1.f; }
    const float top = (float)(n - 2);
    if (!(fl >= 0.f)) { i0 = 0; f = 0.f; }               // below the box (or NaN)
    else if (fl > top) { i0 = n - 2; f = 1.f; }          // on or above the upper face
    else { i0 = (int)fl; f = fr; }
}

// Cell index and fraction of a point addressed through the unbounded-scene contraction
// (Eq. 4, p = inf or 2).  The contraction and the index map run in double, so the fraction
// is accurate to float32 although the contracted point is a derived value; the clamping
// matches axis_coord.
__device__ __forceinline__ void warped_coords(const DevGrid &g, float x, float y, float z, int (&i)[3],
                                              float (&f)[3]) {
    double p[3] = {(double)x, (double)y, (double)z};
    double n;
    if (g.warp == DVGO_WARP_CONTRACT_INF) {
        n = fabs(p[0]);
        n = fabs(p[1]) > n ? fabs(p[1]) : n;
        n = fabs(p[2]) > n ? fabs(p[2]) : n;
    } else {
        n = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    }
    const double s = n > 1.0 ? (1.0 + g.wb - g.wb / n) / n : 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = p[a] * s * g.s_d[a] + g.o_d[a];
        const double fl = floor(u);
        if (!(fl >= 0.0)) { i[a] = 0; f[a] = 0.f; }              // below the box (or NaN)
        else if (fl > (double)(g.n[a] - 2)) { i[a] = g.n[a] - 2; f[a] = 1.f; }
        else { i[a] = (int)fl; f[a] = (float)(u - fl); }
    }
}

// W: the kernel was built for grids with a warp (the double-precision contraction path costs
// registers, so kernels for plain grids leave it out).
template <bool W>
__device__ __forceinline__ void grid_coords(const DevGrid &g, float x, float y, float z, int (&i)[3], float (&f)[3]) {
    if (W && g.warp) {
        warped_coords(g, x, y, z, i, f);
        return;
    }
    axis_coord(x, g.s_hi[0], g.s_lo[0], g.o_hi[0], g.o_lo[0], g.n[0], i[0], f[0]);
    axis_coord(y, g.s_hi[1], g.s_lo[1], g.o_hi[1], g.o_lo[1], g.n[1], i[1], f[1]);
    axis_coord(z, g.s_hi[2], g.s_lo[2], g.o_hi[2], g.o_lo[2], g.n[2], i[2], f[2]);
}

template <bool W = false>
__device__ __forceinline__ Tri trilinear(const DevGrid &g, float x, float y, float z) {
    int i[3];
    float fr[3];
    grid_coords<W>(g, x, y, z, i, fr);
    const int ix = i[0], iy = i[1], iz = i[2];
    const float fx = fr[0], fy = fr[1], fz = fr[2];
    Tri t;
    t.base = ix * g.sx + iy * g.sy + iz * g.cs;
    const float wx[2] = {1.f - fx, fx}, wy[2] = {1.f - fy, fy}, wz[2] = {1.f - fz, fz};
#pragma unroll
    for (int c = 0; c < 8; ++c) t.w[c] = (wx[(c >> 2) & 1] * wy[(c >> 1) & 1]) * wz[c & 1];
    return t;
}

// Cell and fractions of a point (the inputs of the trilinear weights), kept for the
// aggregated scatter below.
struct Cell {
    int ix, iy, iz;
    float fx, fy, fz;
};

template <bool W = false>
__device__ __forceinline__ Cell cell_of(const DevGrid &g, float x, float y, float z) {
    int i[3];
    float fr[3];
    grid_coords<W>(g, x, y, z, i, fr);
    return Cell{i[0], i[1], i[2], fr[0], fr[1], fr[2]};
}

__device__ __forceinline__ float corner_weight(const Cell &c, int dx, int dy, int dz) {
    return ((dx ? c.fx : 1.f - c.fx) * (dy ? c.fy : 1.f - c.fy)) * (dz ? c.fz : 1.f - c.fz);
}

// Orders the calling wave's LDS accesses (for the compiler and the hardware) without waiting
// for its outstanding global stores and atomics, which stay in flight.
__device__ __forceinline__ void lds_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup", "local"); }

// Adjoint of trilinear interpolation for the 64 points held by the lanes of a wave, with
// the contributions that land on the same vertex summed inside the wave before the atomic.
//
// Points come from consecutive samples along rays, so the lanes that touch one vertex form
// runs of neighbouring lanes.  A (lane, corner) pair is the head of its run when the lane
// before does not touch that vertex; the head walks forward over the following lanes while
// they still touch the vertex, adds their weighted values (each lane's corner for that
// vertex follows from its own cell), and alone issues the atomics.  Every contribution is
// counted once: a non-head belongs to exactly one run, whose head reaches it.  All lanes
// must call this (it shuffles); lanes with valid == false contribute nothing.
// Whole-wave DPP shifts by one lane with zero fill (vector-ALU moves, no LDS round trip):
// from_next: lane l takes lane l + 1's value (lane 63 takes 0); from_prev: lane l takes lane
// l - 1's (lane 0 takes 0).  The empty asm keeps each shift a move of its own: the compiler
// would otherwise fold it into the instruction that uses it.
__device__ __forceinline__ int from_next(int x) {
    int y = __builtin_amdgcn_update_dpp(0, x, 0x130, 0xF, 0xF, true);
    asm volatile("" : "+v"(y));
    return y;
}
__device__ __forceinline__ int from_prev(int x) {
    int y = __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, true);
    asm volatile("" : "+v"(y));
    return y;
}
__device__ __forceinline__ float from_next(float x) { return __builtin_bit_cast(float, from_next(__builtin_bit_cast(int, x))); }

template <int NC>
__device__ __forceinline__ void scatter_wave(const DevGrid &g, bool valid, const Cell &cl, const float (&v)[NC],
                                             int nch = NC) {
    const int ln = lane();
    const int px = from_prev(cl.ix), py = from_prev(cl.iy), pz = from_prev(cl.iz);
    const bool pvalid = from_prev(valid ? 1 : 0) != 0;  // lane 0 has no predecessor
    const int base = cl.ix * g.sx + cl.iy * g.sy + cl.iz * g.cs;
    // The corners go in groups: with many channels four at a time, since their accumulators are the
    // largest register set of the scatter and halving them lets more waves share a SIMD (the walk
    // then runs once per group).
    constexpr int CG = NC > 4 ? 4 : 8;
#pragma unroll
    for (int c0 = 0; c0 < 8; c0 += CG) {
        float acc[CG][NC];
        unsigned head = 0;  // bit cc: corner c0 + cc heads its run
#pragma unroll
        for (int cc = 0; cc < CG; ++cc) {
            const int c = c0 + cc;
            const int dx = (c >> 2) & 1, dy = (c >> 1) & 1, dz = c & 1;
            const int ax = cl.ix + dx - px, ay = cl.iy + dy - py, az = cl.iz + dz - pz;
            const bool prev_touches = pvalid && (unsigned)ax <= 1u && (unsigned)ay <= 1u && (unsigned)az <= 1u;
            if (valid && !prev_touches) head |= 1u << cc;
            const float w = corner_weight(cl, dx, dy, dz);
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) acc[cc][ch] = w * v[ch];
        }
        unsigned active = head;
        // the values of lane ln + k, moved one lane further each step (zeros past lane 63, so the
        // validity flag of a lane beyond the wave reads as false)
        int nx = cl.ix, ny = cl.iy, nz = cl.iz, nval = valid ? 1 : 0;
        Cell nc = cl;
        float nv[NC];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) nv[ch] = v[ch];
        for (int k = 1; k < 64; ++k) {
            if (__ballot(active != 0) == 0ull) break;
            nx = from_next(nx);
            ny = from_next(ny);
            nz = from_next(nz);
            nval = from_next(nval);
            nc.fx = from_next(nc.fx);
            nc.fy = from_next(nc.fy);
            nc.fz = from_next(nc.fz);
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) nv[ch] = from_next(nv[ch]);
            const bool nvalid = nval != 0;
#pragma unroll
            for (int cc = 0; cc < CG; ++cc) {
                if (!(active & (1u << cc))) continue;
                const int c = c0 + cc;
                const int ax = cl.ix + ((c >> 2) & 1) - nx, ay = cl.iy + ((c >> 1) & 1) - ny,
                          az = cl.iz + (c & 1) - nz;
                if (nvalid && (unsigned)ax <= 1u && (unsigned)ay <= 1u && (unsigned)az <= 1u) {
                    const float w = corner_weight(nc, ax, ay, az);
#pragma unroll
                    for (int ch = 0; ch < NC; ++ch) acc[cc][ch] += w * nv[ch];
                } else {
                    active &= ~(1u << cc);
                }
            }
        }
        if (NC == 1) {
#pragma unroll
            for (int cc = 0; cc < CG; ++cc) {
                const int c = c0 + cc;
                if (head & (1u << cc))
                    unsafeAtomicAdd(g.grad + base + ((c >> 2) & 1) * g.sx + ((c >> 1) & 1) * g.sy + (c & 1) * g.cs,
                                    acc[cc][0]);
            }
            continue;
        }
        // Multi-channel: compact the heads through this wave's LDS slice and issue the atomics with
        // consecutive lanes on consecutive channels of one vertex, so one instruction covers a few
        // whole vertex rows instead of one float of 64 vertices.  The two corners of a cell that
        // differ only in z (2p, 2p + 1) are adjacent rows of the z-fastest layout: a lane puts both
        // of its records next to each other, so a pair that both lanes' runs start on leaves as one
        // contiguous 2C-float span (fewer memory packets per vertex than two separate rows).
        extern __shared__ float scatter_lds[];
        float *vals = scatter_lds + (threadIdx.x >> 6) * (128 * (NC + 1));
        int *keys = reinterpret_cast<int *>(vals + 128 * NC);
#pragma unroll
        for (int pp = 0; pp < CG / 2; ++pp) {
            const int p = c0 / 2 + pp;  // corners 2p, 2p + 1 (bits 2pp, 2pp + 1 of head)
            const bool h0 = (head >> (2 * pp)) & 1u, h1 = (head >> (2 * pp + 1)) & 1u;
            const unsigned long long m0 = __ballot(h0), m1 = __ballot(h1);
            if ((m0 | m1) == 0ull) continue;
            const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m0 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m0, 0u)) +
                             __builtin_amdgcn_mbcnt_hi((unsigned)(m1 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m1, 0u));
            const int nh = __popcll(m0) + __popcll(m1);
            const int k0 = base + ((p >> 1) & 1) * g.sx + (p & 1) * g.sy;  // corner 2p (dz = 0)
            if (h0) {
                keys[rank] = k0;
#pragma unroll
                for (int ch = 0; ch < NC; ++ch) vals[rank * NC + ch] = acc[2 * pp][ch];
            }
            if (h1) {
                const int r1 = rank + (h0 ? 1 : 0);
                keys[r1] = k0 + g.cs;
#pragma unroll
                for (int ch = 0; ch < NC; ++ch) vals[r1 * NC + ch] = acc[2 * pp + 1][ch];
            }
            lds_fence();  // the slice is this wave's own: LDS order only, the atomics stay in flight
            for (int i = ln; i < nh * NC; i += 64) {
                const int e = i / NC, ch = i - e * NC;
                if (ch < nch) unsafeAtomicAdd(g.grad + keys[e] + ch, vals[i]);
            }
            lds_fence();
        }
    }
}

// bytes of dynamic LDS a block of `threads` needs for scatter_wave<NC>
__host__ __device__ constexpr int scatter_lds_bytes(int NC, int threads) {
    return NC == 1 ? 0 : (threads / 64) * 128 * (NC + 1) * 4;
}

__device__ __forceinline__ Tri tri_from_cell(const DevGrid &g, const Cell &c) {
    Tri t;
    t.base = c.ix * g.sx + c.iy * g.sy + c.iz * g.cs;
#pragma unroll
    for (int k = 0; k < 8; ++k) t.w[k] = corner_weight(c, (k >> 2) & 1, (k >> 1) & 1, k & 1);
    return t;
}

__device__ __forceinline__ int corner_off(const DevGrid &g, int c) {
    return ((c >> 2) & 1) * g.sx + ((c >> 1) & 1) * g.sy + (c & 1) * g.cs;
}

// Channels c0..c0+3 of a trilinear lookup (rows 16-byte aligned, c0 % 4 == 0): corners in the
// order 0..7, one FMA each, so every kernel that interpolates this way gets the same bits.
__device__ __forceinline__ float4 interp4(const DevGrid &g, const Tri &t, int c0) {
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float4 v = *reinterpret_cast<const float4 *>(g.data + t.base + corner_off(g, c) + c0);
        acc.x = __builtin_fmaf(t.w[c], v.x, acc.x);
        acc.y = __builtin_fmaf(t.w[c], v.y, acc.y);
        acc.z = __builtin_fmaf(t.w[c], v.z, acc.z);
        acc.w = __builtin_fmaf(t.w[c], v.w, acc.w);
    }
    return acc;
}

__device__ __forceinline__ float interp_ch(const DevGrid &g, const Tri &t, int ch) {
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) acc += t.w[c] * g.data[t.base + corner_off(g, c) + ch];
    return acc;
}

__device__ __forceinline__ void scatter_ch(const DevGrid &g, const Tri &t, int ch, float v) {
#pragma unroll
    for (int c = 0; c < 8; ++c) unsafeAtomicAdd(&g.grad[t.base + corner_off(g, c) + ch], t.w[c] * v);
}

// ------------------------------------------------------------------------------ Adam

// The update of one element (section 3's fused Adam): every kernel that applies Adam uses these
// expressions, so they agree bit for bit on the same gradient.
struct AdamArgs {
    float *p, *g, *m, *v;
    int64_t n;
    float lr_t;          // lr / (1 - beta1^t)
    float inv_sqrt_bc2;  // 1 / sqrt(1 - beta2^t)
    float b1, b2, eps, lr;
    const int *step_dev;  // when set, t is read here and lr_t / inv_sqrt_bc2 are recomputed
    int skip, zero;
};

__device__ __forceinline__ void adam_bias(AdamArgs &a) {
    if (a.step_dev) {
        const int t = *a.step_dev;
        const double bc1 = 1.0 - pow((double)a.b1, t), bc2 = 1.0 - pow((double)a.b2, t);
        a.lr_t = (float)((double)a.lr / bc1);
        a.inv_sqrt_bc2 = (float)(1.0 / sqrt(bc2));
    }
}

// Each operation rounded as written (explicit FMAs, no contraction), so every kernel that inlines
// this gets the same bits whatever code surrounds it.
__device__ __forceinline__ void adam_one(const AdamArgs &a, float g, float &p, float &m, float &v) {
#pragma clang fp contract(off)
    m = __builtin_fmaf(a.b1, m, (1.f - a.b1) * g);
    v = __builtin_fmaf(a.b2, v, (1.f - a.b2) * (g * g));
    p = p - (a.lr_t * m) / __builtin_fmaf(sqrtf(v), a.inv_sqrt_bc2, a.eps);
}

typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_nt(const float4 *p) {
    const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_nt(float4 *p, float4 a) {
    const nt_f4 v = {a.x, a.y, a.z, a.w};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_f4 *>(p));
}


// ------------------------------------------------------------------------ wave runs

// Runs of equal keys among the lanes of a wave: the head of each run (key >= 0) learns the run
// length; every lane learns its run's head.
struct Run {
    bool head;
    int len, head_lane;
};

__device__ __forceinline__ Run wave_runs(int key) {
    const int ln = lane();
    const int prev = __shfl_up(key, 1, 64);
    const bool head = key >= 0 && (ln == 0 || prev != key);
    const bool start = ln == 0 || prev != key;  // a run boundary (invalid lanes start runs too)
    const unsigned long long starts = __ballot(start);
    const unsigned long long after = ln == 63 ? 0ull : starts & (~0ull << (ln + 1));
    const int next = after ? __ffsll((long long)after) - 1 : 64;
    const unsigned long long upto = starts & (ln == 63 ? ~0ull : ((2ull << ln) - 1));
    Run r;
    r.head = head;
    r.len = next - ln;
    r.head_lane = 63 - __clzll((long long)upto);
    return r;
}

// ------------------------------------------------------------------------- host side

int set_error(int code, const char *fmt, ...);
int check_hip(hipError_t e, const char *what);
int make_dev_grid(const dvgo_grid *g, const char *name, DevGrid *out, bool need_grad);

// Debug mode (dvgo_set_debug, or DVGO_DEBUG=1 in the environment): the entry points that take a
// ragged batch first check it on the device with validate_batch (synchronous).
bool debug_mode();
int validate_batch(int32_t n_rays, int64_t n_samples, const int32_t *ray_offsets, const float *s_mid, hipStream_t st);

// The distortion loss on given weights (render.hip): argument checks, the bytes of its per-chunk
// checkpoint scratch, and the launch with a caller-chosen scratch pointer.
int distortion_check(int32_t n_rays, const int32_t *ray_offsets, int64_t n_samples, const float *w, const float *s_mid,
                     const float *s_len, const float *loss, const float *grad_loss, const float *grad_w);
size_t distortion_scratch_bytes(int32_t n_rays, int64_t n_samples);
int launch_distortion(int32_t n_rays, const int32_t *ray_offsets, int64_t n_samples, const float *w, const float *s_mid,
                      const float *s_len, float *loss, const float *grad_loss, float *grad_w, void *ckpt,
                      hipStream_t st);

// Largest batch the per-sample kernels address: 3 * n_samples (the xyz and colour rows) stays
// below 2^31 in their int32 indices.
constexpr int64_t MAX_SAMPLES = ((int64_t)1 << 31) / 3 - 1;

// checkpoint slot of the chunk starting at sample c0 of ray r (rays own disjoint slot ranges)
__host__ __device__ __forceinline__ int64_t ckpt_slot(int64_t beg, int r, int64_t c0) {
    return beg / 64 + r + (c0 - beg) / 64;
}
__host__ __device__ __forceinline__ int64_t ckpt_count(int32_t n_rays, int64_t n_samples) {
    return n_samples / 64 + n_rays + 1;
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace dvgo
