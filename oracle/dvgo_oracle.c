/*
 * FP64 CPU oracle for the per-ray training step of direct voxel-grid radiance fields
 * (Sun, Sun & Chen, "Improved Direct Voxel Grid Optimization for Radiance Fields
 * Reconstruction", arXiv 2206.05085).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct reference
 * that the HIP path is checked against.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header or constant with
 * the HIP library.
 *
 * Conventions.  Every floating-point input arrives as the same float32 buffer the GPU
 * receives and is widened to double at its point of use; every result is double.  All
 * per-ray work is independent and runs under OpenMP; scatters into grids run serially in
 * (ray, sample, corner) order so results are deterministic.
 *
 * Where the paper leaves a detail open, the reading taken here is stated at the function
 * that uses it.  Functions that follow an exact definition implement that definition
 * directly (for instance the double sum of Eq. 1, not its O(N) rewrite), so that a reader
 * can check each line against the paper.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_VERSION 1

typedef struct {
    const float *data;   /* [nx][ny][nz][cs] channel-last */
    int32_t n[3];
    int32_t cs;          /* floats per vertex */
    int32_t C;           /* channels used */
    float bmin[3], bmax[3];
    int32_t warp;        /* 0: points index the box directly; 1, 2: Eq. 4 contraction, p = inf, 2 */
    double wb;           /* b of Eq. 4 */
} orc_grid;

int orc_version(void) { return ORC_VERSION; }

/* Threads the OpenMP loops use (for timing the oracle on one core and on all of them). */
int orc_threads(void) { return omp_get_max_threads(); }
int orc_set_threads(int32_t n)
{
    const int prev = omp_get_max_threads();
    omp_set_num_threads(n > 0 ? n : 1);
    return prev;
}

/* Shift b of the density activation.  Section 5.4 fixes the initial alpha (1e-4) at a
 * 0.5-voxel step but does not write the activation out.  Reading: sigma =
 * softplus(raw + b), alpha = 1 - exp(-sigma * delta), with b chosen so that raw = 0 at
 * delta = delta_ref gives alpha_init:  (1 + e^b)^(-delta_ref) = 1 - alpha_init. */
double orc_act_shift(double alpha_init, double delta_ref)
{
    return log(pow(1.0 - alpha_init, -1.0 / delta_ref) - 1.0);
}

static double softplus(double z) { return z > 0 ? z + log1p(exp(-z)) : log1p(exp(z)); }
static double sigmoid(double z)
{
    if (z >= 0) return 1.0 / (1.0 + exp(-z));
    double e = exp(z);
    return e / (1.0 + e);
}

/* ------------------------------------------------------------------ interpolation */

/* Eq. 4, the parameterisation of unbounded scenes (section 5.4): a point inside the unit
 * p-ball is kept; a point outside is moved along its own direction to the radius
 * 1 + b - b/||x||_p, so all of space lands inside the p-ball of radius 1 + b, which the
 * grid's box [-1-b, 1+b]^3 covers.  p = inf (warp 1) or p = 2 (warp 2). */
static void contract(int32_t warp, double b, const double x[3], double out[3])
{
    double n;
    if (warp == 1) {
        n = fabs(x[0]);
        if (fabs(x[1]) > n) n = fabs(x[1]);
        if (fabs(x[2]) > n) n = fabs(x[2]);
    } else {
        n = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    }
    const double s = n <= 1.0 ? 1.0 : (1.0 + b - b / n) / n;
    for (int a = 0; a < 3; ++a) out[a] = x[a] * s;
}

/* Trilinear interpolation on a vertex grid whose corner vertices sit on the box corners
 * (the paper queries its grids through a library routine, section 4; reading: vertex i is
 * at bmin + i (bmax - bmin)/(n - 1)).  A coordinate is clamped to the box, and a point on
 * the upper face uses the last cell with fraction 1.  Corner c = 4 dx + 2 dy + dz.  A grid
 * with a warp is addressed at the contracted point (Eq. 4) instead of the point itself. */
static void corners(const orc_grid *g, const float *p, int64_t idx[8], double wt[8])
{
    int64_t i0[3];
    double f[3];
    double x[3] = {p[0], p[1], p[2]};
    if (g->warp) contract(g->warp, g->wb, x, x);
    for (int a = 0; a < 3; ++a) {
        double lo = g->bmin[a], hi = g->bmax[a];
        double u = (x[a] - lo) / (hi - lo) * (double)(g->n[a] - 1);
        if (!(u > 0.0)) u = 0.0; /* also maps NaN to 0 */
        if (u > g->n[a] - 1) u = g->n[a] - 1;
        int64_t i = (int64_t)floor(u);
        if (i > g->n[a] - 2) i = g->n[a] - 2;
        i0[a] = i;
        f[a] = u - (double)i;
    }
    for (int c = 0; c < 8; ++c) {
        int dx = (c >> 2) & 1, dy = (c >> 1) & 1, dz = c & 1;
        idx[c] = (((i0[0] + dx) * g->n[1] + (i0[1] + dy)) * g->n[2] + (i0[2] + dz)) * g->cs;
        wt[c] = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
    }
}

static void interp(const orc_grid *g, const float *p, double *out)
{
    int64_t idx[8];
    double wt[8];
    corners(g, p, idx, wt);
    for (int ch = 0; ch < g->C; ++ch) out[ch] = 0.0;
    for (int c = 0; c < 8; ++c)
        for (int ch = 0; ch < g->C; ++ch) out[ch] += wt[c] * (double)g->data[idx[c] + ch];
}

/* Adjoint of interp: grad[vertex] += weight * g.  grad has the grid's [..][cs] layout. */
static void interp_adjoint(const orc_grid *g, const float *p, const double *gv, double *grad)
{
    int64_t idx[8];
    double wt[8];
    corners(g, p, idx, wt);
    for (int c = 0; c < 8; ++c)
        for (int ch = 0; ch < g->C; ++ch) grad[idx[c] + ch] += wt[c] * gv[ch];
}

void orc_gather(const orc_grid *g, int64_t S, const float *xyz, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < S; ++k) interp(g, xyz + 3 * k, out + k * g->C);
}

void orc_scatter(const orc_grid *g, int64_t S, const float *xyz, const double *gv, double *grad)
{
    for (int64_t k = 0; k < S; ++k) interp_adjoint(g, xyz + 3 * k, gv + k * g->C, grad);
}

/* ---------------------------------------------------------------- distortion loss */

/* Eq. 1 written out: for one ray with weights w, interval midpoints m and lengths l,
 *   D = sum_i sum_j w_i w_j |m_i - m_j| + (1/3) sum_i w_i^2 l_i.                     */
static double dist_ray(int n, const double *w, const float *m, const float *l)
{
    double a = 0.0, b = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) a += w[i] * w[j] * fabs((double)m[i] - (double)m[j]);
        b += w[i] * w[i] * (double)l[i];
    }
    return a + b / 3.0;
}

/* Derivative of Eq. 1 by w_k, written out (Eq. 3 plus the derivative of the second term,
 * which Eq. 3 leaves out; Eq. 3's third sum should read w_i m_i):
 *   dD/dw_k = 2 sum_j w_j |m_k - m_j| + (2/3) w_k l_k.                                 */
static void dist_ray_grad(int n, const double *w, const float *m, const float *l, double *g)
{
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += w[j] * fabs((double)m[k] - (double)m[j]);
        g[k] = 2.0 * s + 2.0 / 3.0 * w[k] * (double)l[k];
    }
}

void orc_distortion(int32_t R, const int32_t *offs, const double *w, const float *m, const float *l, double *D)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t r = 0; r < R; ++r) {
        int64_t o = offs[r];
        D[r] = dist_ray(offs[r + 1] - offs[r], w + o, m + o, l + o);
    }
}

void orc_distortion_grad(int32_t R, const int32_t *offs, const double *w, const float *m, const float *l,
                         const double *gD, double *gw)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t r = 0; r < R; ++r) {
        int64_t o = offs[r];
        int n = offs[r + 1] - offs[r];
        dist_ray_grad(n, w + o, m + o, l + o, gw + o);
        for (int k = 0; k < n; ++k) gw[o + k] *= gD[r];
    }
}

/* The O(N) rewrite of Eq. 2 exactly as the paper states it: with sorted midpoints the
 * first term equals 2 sum_i w_i (m_i P_i - PM_i), where P_i and PM_i are the exclusive
 * prefix sums of w and w*m.  Kept as a second form so tests can confirm the rewrite. */
void orc_distortion_prefix(int32_t R, const int32_t *offs, const double *w, const float *m, const float *l, double *D)
{
    for (int32_t r = 0; r < R; ++r) {
        int64_t o = offs[r];
        int n = offs[r + 1] - offs[r];
        double P = 0.0, PM = 0.0, first = 0.0, second = 0.0;
        for (int i = 0; i < n; ++i) {
            double wi = w[o + i], mi = m[o + i];
            first += 2.0 * wi * (mi * P - PM);
            second += wi * wi * (double)l[o + i];
            P += wi;
            PM += wi * mi;
        }
        D[r] = first + second / 3.0;
    }
}

/* Eq. 3 (third sum corrected to w_i m_i) plus (2/3) w_k l_k, with prefix and suffix sums. */
void orc_distortion_prefix_grad(int32_t R, const int32_t *offs, const double *w, const float *m, const float *l,
                                double *gw)
{
    for (int32_t r = 0; r < R; ++r) {
        int64_t o = offs[r];
        int n = offs[r + 1] - offs[r];
        double totW = 0.0, totWM = 0.0;
        for (int i = 0; i < n; ++i) { totW += w[o + i]; totWM += w[o + i] * m[o + i]; }
        double P = 0.0, PM = 0.0;
        for (int k = 0; k < n; ++k) {
            double wk = w[o + k], mk = m[o + k];
            double SW = totW - P - wk, SWM = totWM - PM - wk * mk;
            gw[o + k] = 2.0 * mk * P - 2.0 * PM + 2.0 * SWM - 2.0 * mk * SW + 2.0 / 3.0 * wk * (double)l[o + k];
            P += wk;
            PM += wk * mk;
        }
    }
}

/* -------------------------------------------------------------------- rendering */

/* Per-ray forward quantities for one ray.  Colour is either interpolated from a colour
 * grid (identity activation; reading for the grid-colour mode) or given per sample.
 *
 * Density to alpha (section 3): sigma = softplus(raw + b), alpha = 1 - exp(-sigma delta).
 * Front-to-back accumulation: T_0 = 1, T_{k+1} = T_k (1 - alpha_k), w_k = T_k alpha_k,
 * C = sum_k w_k c_k + T_N bg.  Halting (section 3): once the accumulated transmittance
 * T_k drops below halt_T (> 0), sample k and all later samples are skipped (w = 0) and
 * T_N is that T_k.  halt_T = 0 disables it. */
typedef struct {
    int n, halt;        /* halt = index of the first skipped sample, n if none */
    double *raw, *c, *x, *alpha, *T, *w;  /* T has n+1 entries */
} ray_fwd;

static void ray_forward(ray_fwd *rf, int n, const float *xyz, const float *delta, const orc_grid *dens,
                        const orc_grid *col, const double *srgb, double act_shift, double halt_T)
{
    rf->n = n;
    rf->T[0] = 1.0;
    rf->halt = n;
    for (int k = 0; k < n; ++k) {
        interp(dens, xyz + 3 * k, &rf->raw[k]);
        if (col) interp(col, xyz + 3 * k, rf->c + 3 * k);
        else for (int ch = 0; ch < 3; ++ch) rf->c[3 * k + ch] = srgb[3 * k + ch];
        double sigma = softplus(rf->raw[k] + act_shift);
        rf->x[k] = sigma * (double)delta[k];
        rf->alpha[k] = -expm1(-rf->x[k]);
    }
    for (int k = 0; k < n; ++k) {
        if (rf->halt == n && halt_T > 0.0 && rf->T[k] < halt_T) rf->halt = k;
        if (rf->halt <= k) {
            rf->w[k] = 0.0;
            rf->T[k + 1] = rf->T[k];
            continue;
        }
        rf->w[k] = rf->T[k] * rf->alpha[k];
        rf->T[k + 1] = rf->T[k] * exp(-rf->x[k]);
    }
}

static ray_fwd alloc_ray(int n)
{
    ray_fwd rf;
    size_t m = (size_t)(n > 0 ? n : 1);
    rf.raw = malloc(m * sizeof(double));
    rf.c = malloc(3 * m * sizeof(double));
    rf.x = malloc(m * sizeof(double));
    rf.alpha = malloc(m * sizeof(double));
    rf.T = malloc((m + 1) * sizeof(double));
    rf.w = malloc(m * sizeof(double));
    return rf;
}

static void free_ray(ray_fwd *rf)
{
    free(rf->raw); free(rf->c); free(rf->x); free(rf->alpha); free(rf->T); free(rf->w);
}

/* Forward render of a ragged batch.  Outputs per ray: rgb[R,3], T_N[R], D[R] (Eq. 1 on
 * the ray's weights with the caller's normalised midpoints and lengths); optionally the
 * per-sample weights w[S] and alphas. */
void orc_render_forward(int32_t R, const int32_t *offs, const float *xyz, const float *delta, const float *s_mid,
                        const float *s_len, const orc_grid *dens, const orc_grid *col, const double *srgb,
                        double act_shift, double halt_T, const double *bg,
                        double *rgb, double *T_N, double *D, double *w_out, double *alpha_out)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int32_t r = 0; r < R; ++r) {
        int64_t o = offs[r];
        int n = offs[r + 1] - offs[r];
        ray_fwd rf = alloc_ray(n);
        ray_forward(&rf, n, xyz + 3 * o, delta + o, dens, col, srgb ? srgb + 3 * o : NULL, act_shift, halt_T);
        double TN = rf.T[n];
        for (int ch = 0; ch < 3; ++ch) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += rf.w[k] * rf.c[3 * k + ch];
            rgb[3 * r + ch] = acc + TN * bg[ch];
        }
        T_N[r] = TN;
        if (D) D[r] = dist_ray(n, rf.w, s_mid + o, s_len + o);
        if (w_out) for (int k = 0; k < n; ++k) w_out[o + k] = rf.w[k];
        if (alpha_out) for (int k = 0; k < n; ++k) alpha_out[o + k] = rf.alpha[k];
        free_ray(&rf);
    }
}

/* Backward of the forward render by the chain rule, for upstream gradients
 * G_C = dL/dC [R,3], G_D = dL/dD [R] (or NULL) and G_T = dL/dT_N [R] (or NULL).
 *
 * With g_k = G_C . c_k + G_D dD/dw_k (the direct dependence of L on w_k):
 *   dw_i/dx_k = T_{k+1} if i = k,  -w_i if i > k,  0 if i < k;  dT_N/dx_k = -T_N,
 * so dL/dx_k = T_{k+1} g_k - sum_{i>k} g_i w_i - (G_C . bg + G_T) T_N, and
 * dL/draw_k = dL/dx_k * delta_k * sigmoid(raw_k + b);  dL/dc_k = w_k G_C.
 * Skipped (halted) samples receive no gradient.  The inner sum is evaluated directly,
 * O(N^2) per ray, on purpose.
 *
 * Outputs (accumulated, +=): grad_dens (density grid layout), grad_col (colour grid
 * layout, grid-colour mode) or grad_srgb [S,3] (per-sample colour mode). */
void orc_render_backward(int32_t R, const int32_t *offs, const float *xyz, const float *delta, const float *s_mid,
                         const float *s_len, const orc_grid *dens, const orc_grid *col, const double *srgb,
                         double act_shift, double halt_T, const double *bg,
                         const double *G_C, const double *G_D, const double *G_T,
                         double *grad_dens, double *grad_col, double *grad_srgb)
{
    int64_t S = offs[R];
    double *draw = calloc((size_t)(S > 0 ? S : 1), sizeof(double));
    double *dc = calloc((size_t)(S > 0 ? 3 * S : 1), sizeof(double));
#pragma omp parallel for schedule(dynamic, 8)
    for (int32_t r = 0; r < R; ++r) {
        int64_t o = offs[r];
        int n = offs[r + 1] - offs[r];
        ray_fwd rf = alloc_ray(n);
        ray_forward(&rf, n, xyz + 3 * o, delta + o, dens, col, srgb ? srgb + 3 * o : NULL, act_shift, halt_T);
        double *g = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double *dDdw = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double gd = G_D ? G_D[r] : 0.0;
        if (G_D) dist_ray_grad(n, rf.w, s_mid + o, s_len + o, dDdw);
        for (int k = 0; k < n; ++k) {
            double gc = 0.0;
            for (int ch = 0; ch < 3; ++ch) gc += G_C[3 * r + ch] * rf.c[3 * k + ch];
            g[k] = gc + (G_D ? gd * dDdw[k] : 0.0);
        }
        double tail = (G_T ? G_T[r] : 0.0);
        for (int ch = 0; ch < 3; ++ch) tail += G_C[3 * r + ch] * bg[ch];
        tail *= rf.T[n];
        for (int k = 0; k < n; ++k) {
            if (k >= rf.halt) { draw[o + k] = 0.0; continue; }
            double later = 0.0;
            for (int i = k + 1; i < n; ++i) later += g[i] * rf.w[i];
            double dx = rf.T[k + 1] * g[k] - later - tail;
            draw[o + k] = dx * (double)delta[k + o] * sigmoid(rf.raw[k] + act_shift);
            for (int ch = 0; ch < 3; ++ch) dc[3 * (o + k) + ch] = rf.w[k] * G_C[3 * r + ch];
        }
        free(g);
        free(dDdw);
        free_ray(&rf);
    }
    for (int64_t k = 0; k < S; ++k) {
        interp_adjoint(dens, xyz + 3 * k, draw + k, grad_dens);
        if (col && grad_col) interp_adjoint(col, xyz + 3 * k, dc + 3 * k, grad_col);
    }
    if (grad_srgb) for (int64_t k = 0; k < 3 * S; ++k) grad_srgb[k] += dc[k];
    free(draw);
    free(dc);
}

/* Per-sample alpha only (density path of the forward); used for the coarse proposal pass. */
void orc_alpha(int64_t S, const float *xyz, const float *delta, const orc_grid *dens, double act_shift, double *alpha)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < S; ++k) {
        double raw;
        interp(dens, xyz + 3 * k, &raw);
        alpha[k] = -expm1(-softplus(raw + act_shift) * (double)delta[k]);
    }
}

/* Photometric + distortion loss: L = (1/(3R)) sum ||C_r - target_r||^2 + lambda (1/R) sum D_r
 * (reading: both terms are means over rays).  Returns L; writes G_C and G_D. */
double orc_loss_head(int32_t R, const double *rgb, const float *target, const double *D, double lambda,
                     double *G_C, double *G_D)
{
    double L = 0.0;
    for (int32_t r = 0; r < R; ++r) {
        for (int ch = 0; ch < 3; ++ch) {
            double e = rgb[3 * r + ch] - (double)target[3 * r + ch];
            L += e * e / (3.0 * R);
            if (G_C) G_C[3 * r + ch] = 2.0 * e / (3.0 * R);
        }
        if (D) L += lambda * D[r] / R;
        if (G_D) G_D[r] = lambda / R;
    }
    return L;
}

/* ------------------------------------------------------------------- colour MLP */

/* View-direction encoding: [d, sin(2^0 d), ..., sin(2^{F-1} d), cos(2^0 d), ..., cos(2^{F-1} d)],
 * each block xyz in order: 3 + 6F values. */
static void view_pe(const float *d, int F, double *pe)
{
    for (int a = 0; a < 3; ++a) pe[a] = d[a];
    for (int q = 0; q < F; ++q)
        for (int a = 0; a < 3; ++a) {
            double v = ldexp((double)d[a], q);
            pe[3 + 3 * q + a] = sin(v);
            pe[3 + 3 * F + 3 * q + a] = cos(v);
        }
}

/* Hybrid colour head: input [feat(C), PE(d)], two hidden ReLU layers of H, sigmoid RGB.
 * half != 0: the cheaper colour head, whose matrix products take each operand rounded to an
 * FP16 significand (see r16); exact double otherwise. */
typedef struct {
    const float *W1, *b1, *W2, *b2, *W3, *b3;  /* [H][C+3+6F], [H], [H][H], [H], [3][H], [3] */
    int32_t C, F, H;
    int32_t half;
} orc_mlp;

/* v rounded to 11 significant bits, to nearest even: the value an FP16 operand carries after
 * an exact power-of-two scaling into the FP16 normal range (the range itself is not modelled). */
static double r16(double v)
{
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    const double m = frexp(v, &e);  /* v = m 2^e, 1/2 <= |m| < 1 */
    return ldexp(nearbyint(ldexp(m, 11)), e - 11);
}

/* An operand of one of the head's matrix products (layers 1 and 2, the back-propagation
 * through W2 and W1, the gradients of W2 and W1). */
static double opnd(const orc_mlp *P, double v) { return P->half ? r16(v) : v; }

static int64_t find_ray(int32_t R, const int32_t *offs, int64_t k)
{
    int64_t lo = 0, hi = R - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (offs[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

static void mlp_fwd_one(const orc_mlp *P, const double *x, double *z1, double *h1, double *z2, double *h2, double *rgb)
{
    int I = P->C + 3 + 6 * P->F, H = P->H;
    for (int i = 0; i < H; ++i) {
        double s = P->b1[i];
        for (int j = 0; j < I; ++j) s += opnd(P, P->W1[i * I + j]) * opnd(P, x[j]);
        z1[i] = s;
        h1[i] = s > 0 ? s : 0.0;
    }
    for (int i = 0; i < H; ++i) {
        double s = P->b2[i];
        for (int j = 0; j < H; ++j) s += opnd(P, P->W2[i * H + j]) * opnd(P, h1[j]);
        z2[i] = s;
        h2[i] = s > 0 ? s : 0.0;
    }
    for (int i = 0; i < 3; ++i) {
        double s = P->b3[i];
        for (int j = 0; j < H; ++j) s += (double)P->W3[i * H + j] * h2[j];
        rgb[i] = sigmoid(s);
    }
}

void orc_mlp_forward(const orc_mlp *P, int32_t R, const int32_t *offs, const float *dirs, const double *feat,
                     double *rgb)
{
    int64_t S = offs[R];
    int I = P->C + 3 + 6 * P->F, H = P->H;
#pragma omp parallel
    {
        double *x = malloc(sizeof(double) * I), *buf = malloc(sizeof(double) * 4 * H);
#pragma omp for schedule(static)
        for (int64_t k = 0; k < S; ++k) {
            int64_t r = find_ray(R, offs, k);
            for (int c = 0; c < P->C; ++c) x[c] = feat[k * P->C + c];
            view_pe(dirs + 3 * r, P->F, x + P->C);
            mlp_fwd_one(P, x, buf, buf + H, buf + 2 * H, buf + 3 * H, rgb + 3 * k);
        }
        free(x);
        free(buf);
    }
}

/* Backward of the colour head for upstream grad_rgb [S,3]: writes grad_feat [S,C] and
 * accumulates (+=) the parameter gradients, serially in sample order. */
static void mlp_backward_range(const orc_mlp *P, int32_t R, const int32_t *offs, const float *dirs,
                               const double *feat, const double *grad_rgb, double *grad_feat, int64_t k0, int64_t k1,
                               double *gW1, double *gb1, double *gW2, double *gb2, double *gW3, double *gb3)
{
    int I = P->C + 3 + 6 * P->F, H = P->H;
    double *x = malloc(sizeof(double) * I);
    double *z1 = malloc(sizeof(double) * H), *h1 = malloc(sizeof(double) * H);
    double *z2 = malloc(sizeof(double) * H), *h2 = malloc(sizeof(double) * H);
    double *d2 = malloc(sizeof(double) * H), *d1 = malloc(sizeof(double) * H);
    double rgb[3], d3[3];
    for (int64_t k = k0; k < k1; ++k) {
        int64_t r = find_ray(R, offs, k);
        for (int c = 0; c < P->C; ++c) x[c] = feat[k * P->C + c];
        view_pe(dirs + 3 * r, P->F, x + P->C);
        mlp_fwd_one(P, x, z1, h1, z2, h2, rgb);
        for (int i = 0; i < 3; ++i) {
            d3[i] = grad_rgb[3 * k + i] * rgb[i] * (1.0 - rgb[i]);
            gb3[i] += d3[i];
            for (int j = 0; j < H; ++j) gW3[i * H + j] += d3[i] * h2[j];
        }
        for (int j = 0; j < H; ++j) {
            double s = 0.0;
            for (int i = 0; i < 3; ++i) s += (double)P->W3[i * H + j] * d3[i];
            d2[j] = z2[j] > 0 ? s : 0.0;
        }
        for (int i = 0; i < H; ++i) {
            gb2[i] += d2[i];
            for (int j = 0; j < H; ++j) gW2[i * H + j] += opnd(P, d2[i]) * opnd(P, h1[j]);
        }
        for (int j = 0; j < H; ++j) {
            double s = 0.0;
            for (int i = 0; i < H; ++i) s += opnd(P, P->W2[i * H + j]) * opnd(P, d2[i]);
            d1[j] = z1[j] > 0 ? s : 0.0;
        }
        for (int i = 0; i < H; ++i) {
            gb1[i] += d1[i];
            for (int j = 0; j < I; ++j) gW1[i * I + j] += opnd(P, d1[i]) * opnd(P, x[j]);
        }
        for (int c = 0; c < P->C; ++c) {
            double s = 0.0;
            for (int i = 0; i < H; ++i) s += opnd(P, P->W1[i * I + c]) * opnd(P, d1[i]);
            grad_feat[k * P->C + c] = s;
        }
    }
    free(x); free(z1); free(h1); free(z2); free(h2); free(d2); free(d1);
}

/* One sample's contribution to every colour-head gradient, with the ReLU mask of one
 * hidden unit optionally inverted (flip_layer 1 or 2, unit flip_unit; 0 = none).
 * out = [dfeat (C) | dW1 | db1 | dW2 | db2 | dW3 | db3]. */
static void mlp_sample_grads(const orc_mlp *P, const double *x, const double *g, int flip_layer, int flip_unit,
                             double *out)
{
    int I = P->C + 3 + 6 * P->F, H = P->H;
    double *z1 = malloc(sizeof(double) * H), *h1 = malloc(sizeof(double) * H);
    double *z2 = malloc(sizeof(double) * H), *h2 = malloc(sizeof(double) * H);
    double *d2 = malloc(sizeof(double) * H), *d1 = malloc(sizeof(double) * H), rgb[3], d3[3];
    mlp_fwd_one(P, x, z1, h1, z2, h2, rgb);
    double *df = out, *W1 = df + P->C, *b1 = W1 + (int64_t)H * I, *W2 = b1 + H, *b2 = W2 + (int64_t)H * H,
           *W3 = b2 + H, *b3 = W3 + 3 * H;
    for (int i = 0; i < 3; ++i) {
        d3[i] = g[i] * rgb[i] * (1.0 - rgb[i]);
        b3[i] = d3[i];
        for (int j = 0; j < H; ++j) W3[i * H + j] = d3[i] * h2[j];
    }
    for (int j = 0; j < H; ++j) {
        double t = 0.0;
        for (int i = 0; i < 3; ++i) t += (double)P->W3[i * H + j] * d3[i];
        int on = z2[j] > 0;
        if (flip_layer == 2 && flip_unit == j) on = !on;
        d2[j] = on ? t : 0.0;
    }
    for (int i = 0; i < H; ++i) {
        b2[i] = d2[i];
        for (int j = 0; j < H; ++j) W2[i * H + j] = d2[i] * h1[j];
    }
    for (int j = 0; j < H; ++j) {
        double t = 0.0;
        for (int i = 0; i < H; ++i) t += (double)P->W2[i * H + j] * d2[i];
        int on = z1[j] > 0;
        if (flip_layer == 1 && flip_unit == j) on = !on;
        d1[j] = on ? t : 0.0;
    }
    for (int i = 0; i < H; ++i) {
        b1[i] = d1[i];
        for (int j = 0; j < I; ++j) W1[i * I + j] = d1[i] * x[j];
    }
    for (int c = 0; c < P->C; ++c) {
        double t = 0.0;
        for (int i = 0; i < H; ++i) t += (double)P->W1[i * I + c] * d1[i];
        df[c] = t;
    }
    free(z1); free(h1); free(z2); free(h2); free(d2); free(d1);
}

/* Slack of the colour-head gradients at non-differentiable points: for every hidden unit
 * whose pre-activation is within thr (relative to |b| + sum |W x|) of its ReLU kink, the
 * absolute change of each gradient when that unit's mask is inverted, summed over such
 * units.  Either mask is a valid (sub)gradient there, so a float32 evaluation may land on
 * either side.  slack_feat [S,C] and slack_par [n_params] (W1, b1, W2, b2, W3, b3) are
 * accumulated (+=).  With P->half the pre-activations are those of the cheaper head. */
void orc_mlp_kink_slack(const orc_mlp *P, int32_t R, const int32_t *offs, const float *dirs, const double *feat,
                        const double *grad_rgb, double thr, double *slack_feat, double *slack_par)
{
    int64_t S = offs[R];
    int I = P->C + 3 + 6 * P->F, H = P->H;
    int64_t np = (int64_t)H * I + H + (int64_t)H * H + H + 3 * H + 3, nout = P->C + np;
    int nt = 1;
#pragma omp parallel
    {
#pragma omp single
        nt = omp_get_num_threads();
    }
    /* one parameter-slack buffer per thread, added in thread order at the end */
    double *par = calloc((size_t)nt * (size_t)np, sizeof(double));
#pragma omp parallel
    {
        double *x = malloc(sizeof(double) * I), *a = malloc(sizeof(double) * nout), *b = malloc(sizeof(double) * nout);
        double *z1 = malloc(sizeof(double) * H), *h1 = malloc(sizeof(double) * H);
        double *mine = par + (size_t)omp_get_thread_num() * (size_t)np;
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < S; ++k) {
            int64_t r = find_ray(R, offs, k);
            for (int c = 0; c < P->C; ++c) x[c] = feat[k * P->C + c];
            view_pe(dirs + 3 * r, P->F, x + P->C);
            int computed = 0;
            for (int layer = 1; layer <= 2; ++layer)
                for (int i = 0; i < H; ++i) {
                    double z, mag;
                    if (layer == 1) {
                        z = P->b1[i];
                        mag = fabs((double)P->b1[i]);
                        for (int j = 0; j < I; ++j) {
                            const double t = opnd(P, P->W1[i * I + j]) * opnd(P, x[j]);
                            z += t;
                            mag += fabs(t);
                        }
                        z1[i] = z;
                        h1[i] = z > 0 ? z : 0.0;
                    } else {
                        z = P->b2[i];
                        mag = fabs((double)P->b2[i]);
                        for (int j = 0; j < H; ++j) {
                            const double t = opnd(P, P->W2[i * H + j]) * opnd(P, h1[j]);
                            z += t;
                            mag += fabs(t);
                        }
                    }
                    if (!(mag > 0 && fabs(z) < thr * mag)) continue;
                    if (!computed) { mlp_sample_grads(P, x, grad_rgb + 3 * k, 0, 0, a); computed = 1; }
                    mlp_sample_grads(P, x, grad_rgb + 3 * k, layer, i, b);
                    for (int c = 0; c < P->C; ++c) slack_feat[k * P->C + c] += fabs(b[c] - a[c]);
                    for (int64_t q = 0; q < np; ++q) mine[q] += fabs(b[P->C + q] - a[P->C + q]);
                }
        }
        free(x); free(a); free(b); free(z1); free(h1);
    }
    for (int t = 0; t < nt; ++t)
        for (int64_t q = 0; q < np; ++q) slack_par[q] += par[(size_t)t * (size_t)np + q];
    free(par);
}

/* Magnitudes the colour head's outputs are conditioned on: the forward and backward passes
 * re-run with every weight, activation and gradient replaced by its absolute value (ReLU masks
 * and the sigmoid slope taken from the true evaluation).  A relative perturbation e of every
 * matrix operand moves each output by at most a small multiple of e times its magnitude, to
 * first order; a cancelling output (|y| much smaller than its magnitude) is sensitive in
 * proportion.  Writes mag_rgb [S,3] and mag_feat [S,C]; accumulates mag_par [n_params] (W1,
 * b1, W2, b2, W3, b3 order) with += .  Operands are those of P (P->half rounds them). */
void orc_mlp_magnitudes(const orc_mlp *P, int32_t R, const int32_t *offs, const float *dirs, const double *feat,
                        const double *grad_rgb, double *mag_rgb, double *mag_feat, double *mag_par)
{
    int64_t S = offs[R];
    int I = P->C + 3 + 6 * P->F, H = P->H;
    double *gW1 = mag_par, *gb1 = gW1 + (int64_t)H * I, *gW2 = gb1 + H, *gb2 = gW2 + (int64_t)H * H, *gW3 = gb2 + H,
           *gb3 = gW3 + 3 * H;
    double *x = malloc(sizeof(double) * I), *ax = malloc(sizeof(double) * I);
    double *z1 = malloc(sizeof(double) * H), *h1 = malloc(sizeof(double) * H);
    double *z2 = malloc(sizeof(double) * H), *h2 = malloc(sizeof(double) * H);
    double *A1 = malloc(sizeof(double) * H), *A2 = malloc(sizeof(double) * H);
    double *D1 = malloc(sizeof(double) * H), *D2 = malloc(sizeof(double) * H);
    double rgb[3], D3[3];
    for (int64_t k = 0; k < S; ++k) {
        int64_t r = find_ray(R, offs, k);
        for (int c = 0; c < P->C; ++c) x[c] = feat[k * P->C + c];
        view_pe(dirs + 3 * r, P->F, x + P->C);
        mlp_fwd_one(P, x, z1, h1, z2, h2, rgb);
        for (int j = 0; j < I; ++j) ax[j] = fabs(opnd(P, x[j]));
        for (int i = 0; i < H; ++i) {
            double a = fabs((double)P->b1[i]);
            for (int j = 0; j < I; ++j) a += fabs(opnd(P, P->W1[i * I + j])) * ax[j];
            A1[i] = z1[i] > 0 ? a : 0.0;
        }
        for (int i = 0; i < H; ++i) {
            double a = fabs((double)P->b2[i]);
            for (int j = 0; j < H; ++j) a += fabs(opnd(P, P->W2[i * H + j])) * A1[j];
            A2[i] = z2[i] > 0 ? a : 0.0;
        }
        for (int o = 0; o < 3; ++o) {
            double a = fabs((double)P->b3[o]);
            for (int j = 0; j < H; ++j) a += fabs((double)P->W3[o * H + j]) * A2[j];
            const double slope = rgb[o] * (1.0 - rgb[o]);
            mag_rgb[3 * k + o] = slope * a;
            D3[o] = fabs(grad_rgb[3 * k + o]) * slope;
            gb3[o] += D3[o];
            for (int j = 0; j < H; ++j) gW3[o * H + j] += D3[o] * A2[j];
        }
        for (int j = 0; j < H; ++j) {
            double t = 0.0;
            for (int o = 0; o < 3; ++o) t += fabs((double)P->W3[o * H + j]) * D3[o];
            D2[j] = z2[j] > 0 ? t : 0.0;
            gb2[j] += D2[j];
        }
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < H; ++j) gW2[i * H + j] += D2[i] * A1[j];
        for (int j = 0; j < H; ++j) {
            double t = 0.0;
            for (int i = 0; i < H; ++i) t += fabs(opnd(P, P->W2[i * H + j])) * D2[i];
            D1[j] = z1[j] > 0 ? t : 0.0;
            gb1[j] += D1[j];
        }
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < I; ++j) gW1[i * I + j] += D1[i] * ax[j];
        for (int c = 0; c < P->C; ++c) {
            double t = 0.0;
            for (int i = 0; i < H; ++i) t += fabs(opnd(P, P->W1[i * I + c])) * D1[i];
            mag_feat[k * P->C + c] = t;
        }
    }
    free(x); free(ax); free(z1); free(h1); free(z2); free(h2); free(A1); free(A2); free(D1); free(D2);
}

/* Backward of the colour head for upstream grad_rgb [S,3]: writes grad_feat [S,C] and
 * accumulates (+=) the parameter gradients.  Samples are split into fixed contiguous
 * blocks whose partial sums are added in block order, so the result does not depend on
 * the number of threads. */
void orc_mlp_backward(const orc_mlp *P, int32_t R, const int32_t *offs, const float *dirs, const double *feat,
                      const double *grad_rgb, double *grad_feat,
                      double *gW1, double *gb1, double *gW2, double *gb2, double *gW3, double *gb3)
{
    int64_t S = offs[R];
    int I = P->C + 3 + 6 * P->F, H = P->H;
    const int64_t BLK = 4096;
    int64_t nb = (S + BLK - 1) / BLK;
    int64_t np = (int64_t)H * I + H + (int64_t)H * H + H + 3 * H + 3;
    double *part = calloc((size_t)(nb > 0 ? nb : 1) * np, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nb; ++b) {
        double *q = part + b * np;
        double *qW1 = q, *qb1 = qW1 + (int64_t)H * I, *qW2 = qb1 + H, *qb2 = qW2 + (int64_t)H * H, *qW3 = qb2 + H,
               *qb3 = qW3 + 3 * H;
        int64_t k1 = (b + 1) * BLK < S ? (b + 1) * BLK : S;
        mlp_backward_range(P, R, offs, dirs, feat, grad_rgb, grad_feat, b * BLK, k1, qW1, qb1, qW2, qb2, qW3, qb3);
    }
    for (int64_t b = 0; b < nb; ++b) {
        const double *q = part + b * np;
        int64_t o = 0;
        for (int64_t i = 0; i < (int64_t)H * I; ++i) gW1[i] += q[o++];
        for (int i = 0; i < H; ++i) gb1[i] += q[o++];
        for (int64_t i = 0; i < (int64_t)H * H; ++i) gW2[i] += q[o++];
        for (int i = 0; i < H; ++i) gb2[i] += q[o++];
        for (int i = 0; i < 3 * H; ++i) gW3[i] += q[o++];
        for (int i = 0; i < 3; ++i) gb3[i] += q[o++];
    }
    free(part);
}

/* ------------------------------------------------------------------------- Adam */

/* Adam with bias correction and 1-based step t; elements whose gradient is exactly zero
 * (either sign) are skipped, leaving parameter and both moments untouched (section 3,
 * fused Adam that does not update grid points with zero gradient). */
void orc_adam(int64_t n, double *p, const double *g, double *m, double *v, double lr, double beta1,
              double beta2, double eps, int32_t t, int32_t skip_zero)
{
    double bc1 = 1.0 - pow(beta1, t), bc2 = 1.0 - pow(beta2, t);
    for (int64_t i = 0; i < n; ++i) {
        if (skip_zero && g[i] == 0.0) continue;
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / bc1, vh = v[i] / bc2;
        p[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* -------------------------------------------------------------- proposal network */

/* Round to bfloat16 with round-to-nearest-even, via float32 (the kernel's own operand
 * precision is float32 before it narrows to bfloat16). */
static double bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan */
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

void orc_r16_round(int64_t n, const double *in, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = r16(in[i]);
}

void orc_bf16_round(int64_t n, const double *in, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = bf16(in[i]);
}

/* Proposal MLP: L linear layers with ReLU between them, sizes[0] -> ... -> sizes[L].
 * Each layer's weights and inputs are rounded to bfloat16 before the product; products
 * accumulate in double; biases stay in full precision.  Output: logits [R, sizes[L]]. */
typedef struct {
    int32_t L;
    int32_t sizes[8];
    const float *W[8], *b[8];
} orc_prop;

static void prop_fwd_one(const orc_prop *P, const double *x0, double *acts /* sum of sizes */, double *z /* per layer */)
{
    /* acts holds the bf16-rounded input of every layer; z the pre-activation of every layer */
    int off = 0, zoff = 0;
    for (int i = 0; i < P->sizes[0]; ++i) acts[i] = bf16(x0[i]);
    for (int l = 0; l < P->L; ++l) {
        int I = P->sizes[l], O = P->sizes[l + 1];
        const double *in = acts + off;
        for (int o = 0; o < O; ++o) {
            double s = 0.0;
            for (int i = 0; i < I; ++i) s += bf16((double)P->W[l][o * I + i]) * in[i];
            s += (double)P->b[l][o];
            z[zoff + o] = s;
            if (l + 1 < P->L) acts[off + I + o] = bf16(s > 0 ? s : 0.0);
        }
        off += I;
        zoff += O;
    }
}

static int prop_total(const orc_prop *P, int upto)
{
    int t = 0;
    for (int l = 0; l < upto; ++l) t += P->sizes[l];
    return t;
}

/* Logits, softmax probabilities and the entropy -sum p ln p of every ray. */
void orc_prop_forward(const orc_prop *P, int32_t R, const double *x, double *logits, double *prob, double *entropy)
{
    int B = P->sizes[P->L], I0 = P->sizes[0];
    int na = prop_total(P, P->L), nz = prop_total(P, P->L + 1) - I0;
#pragma omp parallel
    {
        double *acts = malloc(sizeof(double) * na), *z = malloc(sizeof(double) * nz);
#pragma omp for schedule(static)
        for (int32_t r = 0; r < R; ++r) {
            prop_fwd_one(P, x + (int64_t)r * I0, acts, z);
            const double *lg = z + nz - B;
            double mx = lg[0];
            for (int b = 1; b < B; ++b) mx = lg[b] > mx ? lg[b] : mx;
            double s = 0.0;
            for (int b = 0; b < B; ++b) s += exp(lg[b] - mx);
            double H = 0.0;
            for (int b = 0; b < B; ++b) {
                double p = exp(lg[b] - mx) / s;
                if (logits) logits[(int64_t)r * B + b] = lg[b];
                if (prob) prob[(int64_t)r * B + b] = p;
                if (p > 0) H -= p * log(p);
            }
            if (entropy) entropy[r] = H;
        }
        free(acts);
        free(z);
    }
}

/* Cross-entropy -(1/R) sum_r sum_b p_rb ln softmax(z_r)_b against target histograms p,
 * and its backward through the network.  The gradient at the logits is
 * (softmax(z) - p)/R.  In the backward, every gradient that enters a product (the
 * gradient at a layer's output) is rounded to bfloat16 like the weights and inputs.
 * Parameter gradients are accumulated (+=); returns the loss. */
double orc_prop_backward(const orc_prop *P, int32_t R, const double *x, const double *target,
                         double **gW, double **gb)
{
    int B = P->sizes[P->L], I0 = P->sizes[0];
    int na = prop_total(P, P->L), nz = prop_total(P, P->L + 1) - I0;
    double *acts = malloc(sizeof(double) * na), *z = malloc(sizeof(double) * nz);
    double *dz = malloc(sizeof(double) * 1024), *din = malloc(sizeof(double) * 1024);
    double loss = 0.0;
    for (int32_t r = 0; r < R; ++r) {
        prop_fwd_one(P, x + (int64_t)r * I0, acts, z);
        const double *lg = z + nz - B;
        double mx = lg[0];
        for (int b = 1; b < B; ++b) mx = lg[b] > mx ? lg[b] : mx;
        double s = 0.0;
        for (int b = 0; b < B; ++b) s += exp(lg[b] - mx);
        const double *tg = target + (int64_t)r * B;
        for (int b = 0; b < B; ++b) {
            double lp = lg[b] - mx - log(s);
            loss -= tg[b] * lp / R;
            dz[b] = (exp(lp) - tg[b]) / R;
        }
        /* walk layers backwards; dz holds dL/dz of layer l (size O) */
        int zoff = nz, aoff = na;
        for (int l = P->L - 1; l >= 0; --l) {
            int I = P->sizes[l], O = P->sizes[l + 1];
            zoff -= O;
            aoff -= I;
            const double *in = acts + aoff;
            for (int o = 0; o < O; ++o) dz[o] = bf16(dz[o]);
            for (int o = 0; o < O; ++o) {
                gb[l][o] += dz[o];
                for (int i = 0; i < I; ++i) gW[l][o * I + i] += dz[o] * in[i];
            }
            if (l == 0) break;
            for (int i = 0; i < I; ++i) {
                double t = 0.0;
                for (int o = 0; o < O; ++o) t += bf16((double)P->W[l][o * I + i]) * dz[o];
                din[i] = z[zoff - I + i] > 0 ? t : 0.0; /* ReLU of the previous layer */
            }
            for (int i = 0; i < I; ++i) dz[i] = din[i];
        }
    }
    free(acts); free(z); free(dz); free(din);
    return loss;
}

/* Target histogram of a rendered ray: h_b = sum of the weights of samples whose
 * normalised midpoint falls into bin b of B equal bins on [0,1]; normalised to sum 1
 * when the total is at least min_mass, otherwise uniform. */
void orc_histogram(int32_t R, const int32_t *offs, const double *w, const float *s_mid, int32_t B, double min_mass,
                   double *hist)
{
    for (int32_t r = 0; r < R; ++r) {
        double *h = hist + (int64_t)r * B, tot = 0.0;
        for (int b = 0; b < B; ++b) h[b] = 0.0;
        for (int64_t k = offs[r]; k < offs[r + 1]; ++k) {
            int b = (int)floor((double)s_mid[k] * B);
            if (b < 0) b = 0;
            if (b > B - 1) b = B - 1;
            h[b] += w[k];
            tot += w[k];
        }
        for (int b = 0; b < B; ++b) h[b] = tot >= min_mass ? h[b] / tot : 1.0 / B;
    }
}

/* Inverse CDF of a piecewise-constant density of B equal bins on s in [0,1] with bin
 * masses p (cdf[b] = sum of the first b masses): the point where the CDF reaches u.
 * For 0 <= u < cdf[B] it lies in the first bin whose right CDF value exceeds u (zero-mass
 * bins are never chosen), linearly inside the bin; u >= cdf[B] maps to the right edge of
 * the last bin with mass. */
static double inv_cdf(int B, const double *p, const double *cdf, double u)
{
    if (!(u < cdf[B])) {
        int b = B - 1;
        while (b > 0 && !(p[b] > 0)) --b;
        return (b + 1.0) / B;
    }
    int b = 0;
    while (b < B - 1 && !(cdf[b + 1] > u)) ++b;
    double frac = p[b] > 0 ? (u - cdf[b]) / p[b] : 0.0;
    if (frac < 0) frac = 0;
    if (frac > 1) frac = 1;
    return (b + frac) / B;
}

/* Interval resampling of n fine samples per ray: n + 1 interval ends e_j = F^{-1}(u_j) at
 * u_j = (j/n) * cdf[B] (F the piecewise-constant CDF above), sample j = the interval
 * [e_j, e_{j+1}] represented by its midpoint: s_mid = (e_j + e_{j+1})/2, s_len = e_{j+1} - e_j.
 * Stretches of zero mass outside [e_0, e_n] carry no sample.  Bounded rays map s linearly to
 * t in [t_near, t_far]: x = o + t d; delta is the interval's t-length over the voxel size. */
static void resample_ray(int B, const double *pr, double *cdf, double *e, int n, const float *o, const float *d,
                         double tn, double tf, double voxel, double *xyz, double *delta, double *s_mid, double *s_len)
{
    cdf[0] = 0.0;
    for (int b = 0; b < B; ++b) cdf[b + 1] = cdf[b] + pr[b];
    for (int j = 0; j <= n; ++j) e[j] = inv_cdf(B, pr, cdf, (double)j / n * cdf[B]);
    double len = tf - tn;
    for (int j = 0; j < n; ++j) {
        double sm = 0.5 * (e[j] + e[j + 1]), t = tn + sm * len;
        for (int a = 0; a < 3; ++a) xyz[3 * j + a] = (double)o[a] + t * (double)d[a];
        s_mid[j] = sm;
        s_len[j] = e[j + 1] - e[j];
        delta[j] = s_len[j] * len / voxel;
    }
}

void orc_resample(int32_t R, int32_t B, const double *p, int32_t n, const float *o, const float *d, const float *tn,
                  const float *tf, double voxel, double *xyz, double *delta, double *s_mid, double *s_len)
{
    double *cdf = malloc(sizeof(double) * (B + 1)), *e = malloc(sizeof(double) * (n + 1));
    for (int32_t r = 0; r < R; ++r) {
        int64_t k = (int64_t)r * n;
        resample_ray(B, p + (int64_t)r * B, cdf, e, n, o + 3 * r, d + 3 * r, tn[r], tf[r], voxel, xyz + 3 * k,
                     delta + k, s_mid + k, s_len + k);
    }
    free(cdf);
    free(e);
}

/* Coarse pass of the proposal stage (learned sample placement; not part of the paper,
 * which relies on its occupancy mask, section 1): B uniform samples per ray at
 * s = (k + 1/2)/B between t_near and t_far, density-only alpha (the same activation as
 * the render), front-to-back weights w_k = T_k alpha_k, and the network input
 * feat_k = ln(1 + w_k / eps).  Rays with t_far <= t_near get zeros. */
void orc_proposal_coarse(int32_t R, const float *o, const float *d, const float *tn, const float *tf,
                         const orc_grid *dens, double act_shift, double voxel, int32_t B, double eps, double *w_out,
                         double *feat_out)
{
#pragma omp parallel for schedule(static)
    for (int32_t r = 0; r < R; ++r) {
        double *w = w_out + (int64_t)r * B, *f = feat_out + (int64_t)r * B;
        double a = tn[r], b = tf[r];
        if (!(b > a)) {
            for (int k = 0; k < B; ++k) w[k] = f[k] = 0.0;
            continue;
        }
        double delta = (b - a) / B / voxel, T = 1.0;
        for (int k = 0; k < B; ++k) {
            double t = a + (k + 0.5) / B * (b - a);
            float p[3];
            for (int ax = 0; ax < 3; ++ax) p[ax] = (float)((double)o[3 * r + ax] + t * (double)d[3 * r + ax]);
            double raw;
            interp(dens, p, &raw);
            double x = softplus(raw + act_shift) * delta;
            double alpha = -expm1(-x);
            w[k] = T * alpha;
            T *= exp(-x);
            f[k] = log1p(w[k] / eps);
        }
    }
}

/* Ragged fine batch from proposal probabilities p [R,B] and entropies H [R]:
 * rays with t_far <= t_near get no samples; rays with H > tau fall back to n_plain
 * uniform samples (s_mid = (k + 1/2)/n_plain, s_len = 1/n_plain); the others get n_fine
 * samples by interval resampling as in orc_resample.  Points: x = o + t d with t linear
 * in s on [t_near, t_far]; delta = s_len (t_far - t_near) / voxel.  offs [R+1] is written;
 * the per-sample outputs must hold offs[R] entries. */
void orc_resample_batch(int32_t R, int32_t B, const double *p, const double *H, double tau, int32_t n_fine,
                        int32_t n_plain, const float *o, const float *d, const float *tn, const float *tf, double voxel,
                        int32_t *offs, double *xyz, double *delta, double *s_mid, double *s_len)
{
    offs[0] = 0;
    for (int32_t r = 0; r < R; ++r) {
        int n = !(tf[r] > tn[r]) ? 0 : (H[r] > tau ? n_plain : n_fine);
        offs[r + 1] = offs[r] + n;
    }
    double *cdf = malloc(sizeof(double) * (B + 1)), *s = malloc(sizeof(double) * (n_fine + 1));
    for (int32_t r = 0; r < R; ++r) {
        int n = offs[r + 1] - offs[r];
        if (n == 0) continue;
        double len = (double)tf[r] - (double)tn[r];
        int64_t base = offs[r];
        if (n == n_plain && H[r] > tau) {
            for (int k = 0; k < n; ++k) {
                double sm = (k + 0.5) / n, t = (double)tn[r] + sm * len;
                for (int a = 0; a < 3; ++a) xyz[3 * (base + k) + a] = (double)o[3 * r + a] + t * (double)d[3 * r + a];
                s_mid[base + k] = sm;
                s_len[base + k] = 1.0 / n;
                delta[base + k] = len / n / voxel;
            }
            continue;
        }
        resample_ray(B, p + (int64_t)r * B, cdf, s, n, o + 3 * r, d + 3 * r, tn[r], tf[r], voxel, xyz + 3 * base,
                     delta + base, s_mid + base, s_len + base);
    }
    free(cdf);
    free(s);
}

/* Guarded resampling (a reading of the learned proposal, which the paper does not have; it
 * combines section 1's idea of skipping empty space with placement by the proposal):
 * the 64 coarse bins of a ray are cut into equal sub-intervals, each sample the midpoint of one.
 *   - Bin b is occupied when its coarse weight or a neighbour's, max(w[b-1], w[b], w[b+1]), is at
 *     least w_min; unoccupied bins get no sample (space the coarse pass found empty or occluded).
 *   - An occupied bin gets n_base sub-intervals (n_base = 4 gives plain 256-sample spacing) plus
 *     its share of n_extra extra ones, allotted by the predicted probabilities over the occupied
 *     bins: with S_b the running sum (double, bin order) of prob over the occupied bins before b
 *     and S_tot the total, bin b gets round(n_extra S_{b+1}/S_tot) - round(n_extra S_b/S_tot) with
 *     round(x) = floor(x + 1/2), so the shares sum to n_extra; if S_tot = 0 every occupied bin
 *     counts 1 instead of its probability.
 *   - Fallback rays (H > tau): every bin occupied with n_base sub-intervals and no extras, i.e.
 *     plain uniform sampling at B n_base samples.  Rays with t_far <= t_near get no samples.
 * Sample i of a bin b cut into m: s_mid = (b + (i + 1/2)/m)/B, s_len = 1/(B m); x = o + t d,
 * t = t_near + s_mid (t_far - t_near); delta = s_len (t_far - t_near)/voxel.  Inputs are the
 * float32 arrays the GPU works on (prob and w_coarse [R,B], H [R]); offs [R+1] is written and
 * counts [R,B] (may be NULL) receives the sub-interval count of every bin. */
void orc_resample_guarded(int32_t R, int32_t B, const float *prob, const float *w_coarse, const float *H, float tau,
                          int32_t n_base, int32_t n_extra, float w_min, const float *o, const float *d, const float *tn,
                          const float *tf, double voxel, int32_t *offs, int32_t *counts, double *xyz, double *delta,
                          double *s_mid, double *s_len)
{
    int32_t *m = malloc(sizeof(int32_t) * (size_t)R * B);
    offs[0] = 0;
    for (int32_t r = 0; r < R; ++r) {
        int32_t *mr = m + (int64_t)r * B;
        const float *w = w_coarse + (int64_t)r * B, *p = prob + (int64_t)r * B;
        int total = 0;
        if (!(tf[r] > tn[r])) {
            for (int b = 0; b < B; ++b) mr[b] = 0;
        } else if (H[r] > tau) {
            for (int b = 0; b < B; ++b) mr[b] = n_base;
        } else {
            int occ[256];
            double S_tot = 0.0;
            int n_occ = 0;
            for (int b = 0; b < B; ++b) {
                float mx = w[b];
                if (b > 0 && w[b - 1] > mx) mx = w[b - 1];
                if (b + 1 < B && w[b + 1] > mx) mx = w[b + 1];
                occ[b] = mx >= w_min;
                if (occ[b]) {
                    S_tot += (double)p[b];
                    ++n_occ;
                }
            }
            const int uniform = !(S_tot > 0.0);
            if (uniform) S_tot = (double)n_occ;
            double S = 0.0;
            for (int b = 0; b < B; ++b) {
                if (!occ[b]) {
                    mr[b] = 0;
                    continue;
                }
                const double lo = floor((double)n_extra * (S / S_tot) + 0.5);
                S += uniform ? 1.0 : (double)p[b];
                const double hi = floor((double)n_extra * (S / S_tot) + 0.5);
                mr[b] = n_base + (int)(hi - lo);
            }
        }
        for (int b = 0; b < B; ++b) total += mr[b];
        offs[r + 1] = offs[r] + total;
        if (counts) for (int b = 0; b < B; ++b) counts[(int64_t)r * B + b] = mr[b];
    }
    if (xyz) {
        for (int32_t r = 0; r < R; ++r) {
            const int32_t *mr = m + (int64_t)r * B;
            const double len = (double)tf[r] - (double)tn[r];
            int64_t k = offs[r];
            for (int b = 0; b < B; ++b)
                for (int i = 0; i < mr[b]; ++i, ++k) {
                    const double sm = (b + (i + 0.5) / mr[b]) / B, t = (double)tn[r] + sm * len;
                    for (int a = 0; a < 3; ++a) xyz[3 * k + a] = (double)o[3 * r + a] + t * (double)d[3 * r + a];
                    s_mid[k] = sm;
                    s_len[k] = 1.0 / ((double)B * mr[b]);
                    delta[k] = s_len[k] * len / voxel;
                }
        }
    }
    free(m);
}

/* Softmax probabilities and entropy -sum p ln p of given logits [R,B] (per row). */
void orc_softmax_entropy(int32_t R, int32_t B, const double *logits, double *prob, double *H)
{
    for (int32_t r = 0; r < R; ++r) {
        const double *z = logits + (int64_t)r * B;
        double mx = z[0];
        for (int b = 1; b < B; ++b) mx = z[b] > mx ? z[b] : mx;
        double s = 0.0;
        for (int b = 0; b < B; ++b) s += exp(z[b] - mx);
        double h = 0.0;
        for (int b = 0; b < B; ++b) {
            double p = exp(z[b] - mx) / s;
            prob[(int64_t)r * B + b] = p;
            if (p > 0) h -= p * log(p);
        }
        H[r] = h;
    }
}

/* -------------------------------------------------------------- total variation */

/* Total-variation regulariser of a grid (section 2, efficient TV loss): for every vertex p
 * and channel c, the Huber penalty of the difference to each of its (up to six) axis
 * neighbours n,
 *     L = weight / (N C) * sum_p sum_c sum_n huber(v[p][c] - v[n][c]),
 * N = number of vertices, C = channels, huber(x) = x^2/2 for |x| <= delta, else
 * delta (|x| - delta/2).  Every neighbour pair appears from both of its ends, so
 *     dL/dv[p][c] = 2 weight / (N C) * sum_n clamp(v[p][c] - v[n][c], -delta, delta).
 * grad ([N][cs], FP64) receives += dL/dv at every vertex (dense != 0) or only at the
 * vertices where some channel of the incoming grad is non-zero (sparse).  mag (optional,
 * [N][cs]) receives 2 weight / (N C) * sum_n |clamp(...)|, the magnitude a float evaluation
 * of the sum is conditioned on.  Returns L. */
double orc_tv(const orc_grid *g, double weight, double delta, int32_t dense, double *grad, double *mag)
{
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2], N = nx * ny * nz;
    const double scale = weight / ((double)N * g->C);
    double loss = 0.0;
    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t z = 0; z < nz; ++z) {
                const int64_t i = (x * ny + y) * nz + z;
                int touched = dense;
                if (grad)
                    for (int c = 0; c < g->C && !touched; ++c) touched = grad[i * g->cs + c] != 0.0;
                const int64_t nb[6][3] = {{x - 1, y, z}, {x + 1, y, z}, {x, y - 1, z},
                                          {x, y + 1, z}, {x, y, z - 1}, {x, y, z + 1}};
                for (int c = 0; c < g->C; ++c) {
                    const double v = g->data[i * g->cs + c];
                    double d_sum = 0.0, d_abs = 0.0;
                    for (int k = 0; k < 6; ++k) {
                        if (nb[k][0] < 0 || nb[k][0] >= nx || nb[k][1] < 0 || nb[k][1] >= ny || nb[k][2] < 0 ||
                            nb[k][2] >= nz)
                            continue;
                        const int64_t j = (nb[k][0] * ny + nb[k][1]) * nz + nb[k][2];
                        const double d = v - (double)g->data[j * g->cs + c];
                        loss += fabs(d) <= delta ? 0.5 * d * d : delta * (fabs(d) - 0.5 * delta);
                        const double cl = d < -delta ? -delta : (d > delta ? delta : d);
                        d_sum += cl;
                        d_abs += fabs(cl);
                    }
                    if (grad && touched) grad[i * g->cs + c] += 2.0 * scale * d_sum;
                    if (mag) mag[i * g->cs + c] = 2.0 * scale * d_abs;
                }
            }
    return scale * loss;
}

/* ------------------------------------------------------------------ sample producer */

/* Occupancy mask update.  Section 1: as training goes on, a mask gradually switches off
 * space of low density so that most point queries can be skipped.  Readings: a vertex is
 * dense when the alpha of its own density logit at the sampling step reaches alpha_thr
 * (alpha = 1 - exp(-softplus(raw + b) delta), the activation of section 5.4); a vertex stays
 * active only if it was active and some vertex of its 3x3x3 neighbourhood (clipped at the
 * grid faces) is dense.  The active set therefore only shrinks, and because of the one-vertex
 * dilation every cell that touches a dense vertex has all its eight vertices active.
 * mask: [nx][ny][nz] bytes, non-zero = active; rewritten as 0/1.  Double precision, straight
 * from the definition (expm1 keeps small alphas exact). */
void orc_occupancy_update(const orc_grid *dens, double act_shift, double delta, double alpha_thr, uint8_t *mask)
{
    const int64_t nx = dens->n[0], ny = dens->n[1], nz = dens->n[2], N = nx * ny * nz;
    uint8_t *is_dense = (uint8_t *)malloc((size_t)N);
    for (int64_t i = 0; i < N; ++i) {
        const double sigma = softplus((double)dens->data[i * dens->cs] + act_shift);
        const double alpha = -expm1(-sigma * delta);
        is_dense[i] = alpha >= alpha_thr;
    }
    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t z = 0; z < nz; ++z) {
                const int64_t i = (x * ny + y) * nz + z;
                int near_dense = 0;
                for (int64_t a = x - 1; a <= x + 1; ++a)
                    for (int64_t b = y - 1; b <= y + 1; ++b)
                        for (int64_t c = z - 1; c <= z + 1; ++c)
                            if (a >= 0 && a < nx && b >= 0 && b < ny && c >= 0 && c < nz)
                                near_dense |= is_dense[(a * ny + b) * nz + c];
                mask[i] = (mask[i] != 0) && near_dense;
            }
    free(is_dense);
}

/* Ray/box clip of one ray by the slab method; returns the number of candidate samples.
 * Every step is one float32 operation rounded on its own (see orc_sample_rays). */
static int32_t clip_and_count(const float *o, const float *d, const float *bmin, const float *bmax, float near,
                              float step, int32_t max_per_ray, float *t_near, float *t_exit)
{
    float enter = -INFINITY, leave = INFINITY;
    for (int a = 0; a < 3; ++a) {
        float lo, hi;
        if (d[a] != 0.0f) {
            const float t0 = (bmin[a] - o[a]) / d[a];
            const float t1 = (bmax[a] - o[a]) / d[a];
            lo = t0 < t1 ? t0 : t1;
            hi = t0 < t1 ? t1 : t0;
        } else if (bmin[a] <= o[a] && o[a] <= bmax[a]) {
            lo = -INFINITY;
            hi = INFINITY;
        } else {
            lo = INFINITY;
            hi = -INFINITY;
        }
        if (lo > enter) enter = lo;
        if (hi < leave) leave = hi;
    }
    const float tn = enter > near ? enter : near;
    *t_near = tn;
    *t_exit = leave;
    if (!(leave > tn)) return 0;
    /* samples at t_k = t_near + (k + 1/2) step for every k >= 0 with t_k < t_exit */
    const float c = (leave - tn) / step - 0.5f;
    if (!(c > 0.0f)) return 0;
    if (c > (float)max_per_ray) return max_per_ray;
    return (int32_t)ceilf(c);
}

/* Nearest vertex of point x on the occupancy grid (clamped to the grid). */
static int64_t nearest_vertex(const float *x, const float *bmin, const float *bmax, const int32_t *n)
{
    int64_t idx[3];
    for (int a = 0; a < 3; ++a) {
        const float sc = (float)(n[a] - 1) / (bmax[a] - bmin[a]);
        const float u = (x[a] - bmin[a]) * sc;
        if (!(u >= 0.0f)) idx[a] = 0;
        else if (u >= (float)(n[a] - 1)) idx[a] = n[a] - 1;
        else idx[a] = (int64_t)rintf(u);
    }
    return (idx[0] * n[1] + idx[1]) * n[2] + idx[2];
}

/* Parsimonious sampling with occupancy compaction.  Section 3 (re-implemented rendering
 * utilities): points are placed only where the ray crosses the scene box (bounded scenes);
 * section 1: points in switched-off space are skipped.  Readings, all taken in float32 with
 * each operation rounded on its own (round to nearest even), because these decisions produce
 * integers (sample counts, offsets):
 *   - the ray's box interval by the slab method, per axis (bmin - o)/d and (bmax - o)/d
 *     (an axis with d = 0 is unbounded if o lies within its slab, else empty); t_near is the
 *     larger of the entry and `near`; the ray misses when the exit is not beyond t_near;
 *   - candidate k (k = 0, 1, ...) is the interval [t_near + k step, t_near + (k+1) step] at its
 *     midpoint t_k = fma(k + 1/2, step, t_near); candidates run while t_k < t_exit, i.e.
 *     n = ceil((t_exit - t_near)/step - 1/2), capped at max_per_ray;
 *   - its point is x = fma(t_k, d, o) per axis; it is kept when the occupancy mask is set at
 *     the nearest vertex, u = (x - bmin) (n_a - 1)/(bmax - bmin) rounded to nearest even and
 *     clamped to the grid (mask NULL keeps every candidate);
 *   - a kept candidate carries delta = step / voxel, s_mid = (k + 1/2)/n, s_len = 1/n: s is
 *     linear in t over the n candidate intervals of the unmasked ray.
 * Rays are laid out in order, each ray's samples in increasing k.  Writes ray_offsets [R+1],
 * t_near and t_far [R] (the box interval; both 0 for a ray that misses), and, when xyz is not
 * NULL, the samples (arrays sized by the return value, the total).  Returns the total. */
int64_t orc_sample_rays(int32_t R, const float *o, const float *d, const float *bmin, const float *bmax, float near,
                        float step, float voxel, int32_t max_per_ray, const uint8_t *mask, const int32_t *mshape,
                        int32_t *offs, float *t_near, float *t_far, float *xyz, float *delta, float *s_mid,
                        float *s_len)
{
    int64_t total = 0;
    offs[0] = 0;
    for (int32_t r = 0; r < R; ++r) {
        float tn, te;
        const int32_t n = clip_and_count(o + 3 * r, d + 3 * r, bmin, bmax, near, step, max_per_ray, &tn, &te);
        t_near[r] = te > tn ? tn : 0.0f;
        t_far[r] = te > tn ? te : 0.0f;
        for (int32_t k = 0; k < n; ++k) {
            const float t = fmaf((float)k + 0.5f, step, tn);
            float x[3];
            for (int a = 0; a < 3; ++a) x[a] = fmaf(t, d[3 * r + a], o[3 * r + a]);
            if (mask && !mask[nearest_vertex(x, bmin, bmax, mshape)]) continue;
            if (xyz) {
                for (int a = 0; a < 3; ++a) xyz[3 * total + a] = x[a];
                delta[total] = step / voxel;
                s_mid[total] = ((float)k + 0.5f) / (float)n;
                s_len[total] = 1.0f / (float)n;
            }
            ++total;
        }
        offs[r + 1] = (int32_t)total;
    }
    return total;
}

/* Forward-facing sampling (section 5.3): rays of a forward-facing capture are warped with
 * NeRF's normalised device coordinates to a bounded volume holding D planes at fixed depths
 * (a multiplane-image-like grid), and every ray is traced from the first plane to the last
 * with a step of s planes, which gives 2D - 1 points at s = 0.5.  Readings, all decided in
 * float32 with each operation rounded on its own:
 *   - camera space looks down -z; fx = 2 focal / W, fy = 2 focal / H, near = the near plane;
 *     a ray with d_z >= 0 never crosses it and gets no samples;
 *   - the origin moves to the near plane, t0 = -(near + o_z)/d_z, o <- fma(t0, d, o); the NDC
 *     origin is (-fx (o_x/o_z), -fy (o_y/o_z), 1 + (2 near)/o_z) and the NDC direction
 *     (-fx (d_x/d_z - o_x/o_z), -fy (d_y/d_z - o_y/o_z), -(2 near)/o_z), so NDC depth runs
 *     from -1 (near plane) to 1 (infinity) over t' in [0, 1];
 *   - the planes sit at NDC depth -1 + 2 p/(D - 1), p = 0 .. D - 1; sample j (j = 0 .. J,
 *     J = floor((D - 1)/s), capped at max_per_ray candidates) is at plane coordinate j s,
 *     t' = (j s)/(D - 1), point fma(t', d', o') per axis; it owns the interval of one step
 *     around it: delta = s (planes are one voxel apart along depth), s_mid = (j + 1/2)/(J + 1),
 *     s_len = 1/(J + 1);
 *   - a sample is kept when its point lies in the box across the image axes (bmin <= x' <= bmax
 *     for x and y; depth is inside by construction, and the first and last planes sit on the
 *     box faces, where a rounding must not drop them) and the mask (if any) is set at its
 *     nearest vertex, as in orc_sample_rays.
 * Writes ray_offsets [R+1] and, when xyz is not NULL, the samples.  Returns the total. */
int64_t orc_sample_ndc(int32_t R, const float *o, const float *d, const float *bmin, const float *bmax, float fx,
                       float fy, float near, int32_t planes, float step, int32_t max_per_ray, const uint8_t *mask,
                       const int32_t *mshape, int32_t *offs, float *xyz, float *delta, float *s_mid, float *s_len)
{
    int64_t total = 0;
    offs[0] = 0;
    const float span = (float)(planes - 1);
    const float jmax = floorf(span / step);
    const int32_t n = jmax + 1.0f > (float)max_per_ray ? max_per_ray : (int32_t)jmax + 1;
    for (int32_t r = 0; r < R; ++r) {
        const float *ro = o + 3 * r, *rd = d + 3 * r;
        if (rd[2] < 0.0f) {
            const float t0 = -(near + ro[2]) / rd[2];
            float p[3];
            for (int a = 0; a < 3; ++a) p[a] = fmaf(t0, rd[a], ro[a]);
            const float qx = p[0] / p[2], qy = p[1] / p[2];
            const float on[3] = {-(fx * qx), -(fy * qy), 1.0f + (2.0f * near) / p[2]};
            const float dn[3] = {-(fx * (rd[0] / rd[2] - qx)), -(fy * (rd[1] / rd[2] - qy)), -((2.0f * near) / p[2])};
            for (int32_t j = 0; j < n; ++j) {
                const float t = ((float)j * step) / span;
                float x[3];
                int inside = 1;
                for (int a = 0; a < 3; ++a) x[a] = fmaf(t, dn[a], on[a]);
                for (int a = 0; a < 2; ++a) inside &= bmin[a] <= x[a] && x[a] <= bmax[a];
                if (!inside) continue;
                if (mask && !mask[nearest_vertex(x, bmin, bmax, mshape)]) continue;
                if (xyz) {
                    for (int a = 0; a < 3; ++a) xyz[3 * total + a] = x[a];
                    delta[total] = step;
                    s_mid[total] = ((float)j + 0.5f) / (float)n;
                    s_len[total] = 1.0f / (float)n;
                }
                ++total;
            }
        }
        offs[r + 1] = (int32_t)total;
    }
    return total;
}
