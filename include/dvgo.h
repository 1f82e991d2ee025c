/*
 * dvgo.h -- C-ABI of libdvgo.so, the MI355X (gfx950) kernels of the per-ray training step
 * of direct voxel-grid radiance fields (Sun, Sun & Chen, arXiv 2206.05085).
 *
 * General conventions (apply to every entry point below)
 * ------------------------------------------------------
 * Return value:  DVGO_OK (0) or a negative DVGO_ERR_* code.  A human-readable detail of the
 *   last failure on the calling thread is returned by dvgo_last_error().  No C++ exception
 *   crosses this interface.  On an error nothing has been enqueued.
 * Memory:  every array pointer is a DEVICE pointer owned by the caller (hipMalloc'd or
 *   torch-allocated on the current device), unless stated otherwise.  The library never
 *   allocates in these calls.  Where scratch memory is needed the caller passes a workspace
 *   whose minimum size is returned by the matching *_size query.
 * Streams:  `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls are
 *   asynchronous on that stream; argument validation is synchronous and host-side only (it
 *   never reads device memory), except in debug mode (below).
 * Gradients:  gradients into parameter grids and weights are ACCUMULATED (+=), never
 *   overwritten: the caller zeroes them (or lets dvgo_grid_adam_step zero them).  This is the
 *   paper's convention of adding gradients into the tensor between backward and the
 *   optimiser step (section 2, efficient TV loss).  Per-sample and per-ray gradient outputs
 *   are written (overwritten).
 * Floating point:  float32 everywhere.  NaN/Inf propagate; nothing traps.  Gradient
 *   accumulation uses atomics, so summation order (and the last bits) may vary run to run.
 * Ragged batches:  ray r owns samples ray_offsets[r] .. ray_offsets[r+1]-1 of every
 *   per-sample array; ray_offsets has n_rays+1 non-decreasing entries with ray_offsets[0] = 0
 *   and ray_offsets[n_rays] = n_samples (section 2, uneven numbers of points per ray).
 *   Within a ray s_mid must be non-decreasing (section 2 assumes sorted midpoints).
 *   These two device-side properties are the caller's contract.  They are checked on the
 *   device only in debug mode (dvgo_set_debug, or DVGO_DEBUG=1 in the environment), where
 *   dvgo_render_forward, dvgo_render_backward and dvgo_distortion_loss first run
 *   dvgo_validate_samples (synchronously) and return its error; dvgo_validate_samples can also
 *   be called on its own.  n_samples is at most 715827881 ((2^31)/3 - 1), so that the
 *   kernels' 32-bit element indices of [S,3] rows cannot overflow; larger batches return
 *   DVGO_ERR_RANGE.
 * Structs carry `struct_size` = sizeof(struct) for ABI evolution; a mismatch is DVGO_ERR_ABI.
 */
#ifndef DVGO_H
#define DVGO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DVGO_ABI_VERSION 6

enum {
    DVGO_OK = 0,
    DVGO_ERR_NULL = -1,        /* a required pointer is NULL */
    DVGO_ERR_SHAPE = -2,       /* inconsistent or unsupported sizes */
    DVGO_ERR_RANGE = -3,       /* a size or index exceeds what the kernels address */
    DVGO_ERR_UNSORTED = -4,    /* debug validation: s_mid decreases within a ray */
    DVGO_ERR_WORKSPACE = -5,   /* workspace / state buffer smaller than its query says */
    DVGO_ERR_HIP = -6,         /* a HIP runtime call (launch) failed */
    DVGO_ERR_UNSUPPORTED = -7, /* a mode or parameter value that is not implemented */
    DVGO_ERR_ABI = -8          /* struct_size mismatch */
};

enum { DVGO_COLOR_GRID = 0, DVGO_COLOR_SAMPLES = 1, DVGO_COLOR_NONE = 2 };

/* How points address a grid's box (dvgo_grid.warp).  NONE: directly.  CONTRACT_INF /
 * CONTRACT_L2: through the unbounded-scene contraction of Eq. 4 (section 5.4), p = inf / 2. */
enum { DVGO_WARP_NONE = 0, DVGO_WARP_CONTRACT_INF = 1, DVGO_WARP_CONTRACT_L2 = 2 };

/* Dense vertex grid, channel-last: value (i,j,k,c) at data[((i*ny + j)*nz + k)*ch_stride + c].
 * Vertex i along x sits at xyz_min[0] + i*(xyz_max[0]-xyz_min[0])/(nx-1) (vertices on the box
 * corners).  A query point is clamped to the box; trilinear weights use the enclosing cell.
 * Requirements: nx,ny,nz >= 2; 1 <= channels <= ch_stride <= 16; xyz_max > xyz_min;
 * nx*ny*nz*ch_stride < 2^31.  `grad` (same layout) receives += in backward calls; it may be
 * NULL where a call does not write it.
 * warp (DVGO_WARP_*) and warp_b: with a contraction, every lookup of this grid (gather,
 * scatter, the renderer's density and colour lookups, alpha, the proposal's coarse pass)
 * addresses the box at x' = x if ||x||_p <= 1, else (1 + b - b/||x||_p) x/||x||_p (Eq. 4,
 * b = warp_b > 0), computed in double; the paper's box for it is [-1-b, 1+b]^3 (any box is
 * accepted; points outside it clamp as usual).  Points (xyz) stay in world coordinates. */
typedef struct dvgo_grid {
    uint32_t struct_size;
    int32_t nx, ny, nz;
    int32_t channels;
    int32_t ch_stride;
    float xyz_min[3];
    float xyz_max[3];
    const float *data;
    float *grad;
    int32_t warp;
    float warp_b;
} dvgo_grid;

/* Flattened ragged batch of samples (point queries) along rays.
 * xyz [S,3]: query points in grid coordinates' world frame.
 * delta [S]: length of the sample's interval in voxel units (the alpha step, section 5.4).
 * s_mid [S], s_len [S]: midpoint and length of the sample's interval in the per-ray
 *   normalised coordinate s in [0,1] that the distortion loss uses (Eq. 1). */
typedef struct dvgo_samples {
    uint32_t struct_size;
    int32_t n_rays;
    int64_t n_samples;
    const int32_t *ray_offsets;
    const float *xyz;
    const float *delta;
    const float *s_mid;
    const float *s_len;
} dvgo_samples;

/* act_shift: b in sigma = softplus(raw + b) (section 3 density-to-alpha; b sets the initial
 *   alpha, section 5.4).  halt_T: stop a ray once its accumulated transmittance falls below
 *   this value (section 3; the paper uses 1e-3); 0 disables halting.  bg: background colour
 *   composited with the final transmittance.  color_mode: DVGO_COLOR_GRID (colour =
 *   trilinear value of a 3-channel colour grid), DVGO_COLOR_SAMPLES (colour given per
 *   sample, e.g. by the colour MLP) or DVGO_COLOR_NONE (density only: every sample colour is
 *   0, forward only).  want_dist: also compute the distortion loss (Eq. 1). */
typedef struct dvgo_render_params {
    uint32_t struct_size;
    float act_shift;
    float halt_T;
    float bg[3];
    int32_t color_mode;
    int32_t want_dist;
    /* Schedule (all zero = one wave per ray, 4 waves per block).  ray_list (device, may be
     * NULL): the rays to process, in this order, each listed at most once; rays not listed
     * are left untouched.  n_list: entries of ray_list.  waves_per_block: 1..16 (0 = 4).
     * grid_waves: 0 = one wave per listed ray; > 0 = a persistent grid of that many waves,
     * wave i taking list entries i, i + grid_waves, ... (longest-first lists balance it). */
    const int32_t *ray_list;
    int32_t n_list;
    int32_t waves_per_block;
    int32_t grid_waves;
} dvgo_render_params;

/* Colour MLP: input [features(in_feat), view-direction encoding(3 + 6*n_freq)] -> hidden ->
 * hidden -> 3 with ReLU, ReLU, sigmoid (the hybrid colour of Table 1).  View encoding of a
 * unit direction d: [d, sin(2^0 d) .. sin(2^(F-1) d), cos(2^0 d) .. cos(2^(F-1) d)], each block
 * in x,y,z order.  Weights are row-major [out][in] (W1 [H][in_feat+3+6F], W2 [H][H],
 * W3 [3][H]); the g* pointers receive += in dvgo_mlp_backward.
 * Supported: in_feat <= 12, n_freq <= 4 (so the input fits 48 columns), hidden = 128.
 * precision: DVGO_MLP_SPLIT_F16 (default, FP32-grade: every matrix-core operand is split into two
 * FP16 parts and a product takes three FP16 products) or DVGO_MLP_F16 (the cheaper colour head:
 * every matrix-core operand is one FP16 value after the same power-of-two scaling, i.e. rounded
 * to 11 significant bits, products accumulated in FP32).  In both modes the layer-1/2 products,
 * the weight gradients of W1/W2 and the back-propagation through W2 and W1 run on matrix cores;
 * biases, the output layer, its gradients and all activations stay in FP32.
 * prepared: 0 = every call first writes its preparation into the workspace (the weights as
 * scaled FP16 planes, the view encodings of the rays, the first ray of every 32-sample tile).
 * Nonzero = the workspace already holds that preparation and the call skips it: allowed only
 * when the last call on this workspace was a dvgo_mlp_prepare / dvgo_mlp_forward /
 * dvgo_mlp_backward with the same weights (unchanged since), n_rays,
 * ray_offsets, dirs and n_samples, e.g. the backward that follows the forward of one step.
 * The library cannot check this; a stale workspace gives wrong results, not an error. */
enum { DVGO_MLP_SPLIT_F16 = 0, DVGO_MLP_F16 = 1 };

typedef struct dvgo_color_mlp {
    uint32_t struct_size;
    int32_t in_feat;
    int32_t n_freq;
    int32_t hidden;
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    float *gW1, *gb1, *gW2, *gb2, *gW3, *gb3;
    int32_t precision;
    int32_t prepared;
} dvgo_color_mlp;

int dvgo_abi_version(void);
const char *dvgo_last_error(void);

/* Shift b of the density activation sigma = softplus(raw + b) (section 3's density-to-alpha
 * step): the value for which raw = 0 gives alpha = 1 - exp(-sigma delta_ref) = alpha_init, i.e.
 * b = ln((1 - alpha_init)^(-1/delta_ref) - 1) (section 5.4 sets alpha_init = 1e-4 at a
 * 0.5-voxel step, b = -8.517).  Host-only, in double.  Errors: DVGO_ERR_NULL (shift),
 * DVGO_ERR_RANGE (alpha_init outside (0, 1), delta_ref not positive). */
int dvgo_act_shift(double alpha_init, double delta_ref, double *shift);

/* Debug mode: on != 0 makes dvgo_render_forward, dvgo_render_backward and dvgo_distortion_loss
 * validate their batch on the device first (dvgo_validate_samples: synchronous, not for graph
 * capture).  The initial setting comes from the environment variable DVGO_DEBUG (non-zero =
 * on).  Returns the previous setting (0 or 1). */
int dvgo_set_debug(int32_t on);

/* Checks a ragged batch on the device (its ray_offsets and s_mid; the other arrays are not
 * read): ray_offsets[0] == 0, ray_offsets never decreases and ray_offsets[n_rays] ==
 * n_samples (else DVGO_ERR_SHAPE), and s_mid is non-decreasing within every ray (section 2's
 * sorted midpoints; else DVGO_ERR_UNSORTED; a NaN midpoint counts as out of order).  Each ray's
 * samples are read only after its own offsets were found in range.  Synchronises `stream` to
 * read the verdict; concurrent calls in one process take turns.  Other errors: DVGO_ERR_NULL,
 * DVGO_ERR_ABI, DVGO_ERR_HIP. */
int dvgo_validate_samples(const dvgo_samples *s, void *stream);

/* Size in bytes of the per-batch state that dvgo_render_forward saves for
 * dvgo_render_backward (per-ray halt index, per-64-sample chunk checkpoints and each sample's
 * interpolated density logit raw_k: 4 bytes per sample plus ~20 bytes per ray). */
int dvgo_render_state_size(int32_t n_rays, int64_t n_samples, size_t *bytes);

/* Forward volume rendering of a ragged batch (section 3 rendering utilities, section 2 Eq. 1).
 * Per sample k: raw_k = trilinear(density, x_k); sigma_k = softplus(raw_k + act_shift);
 * alpha_k = 1 - exp(-sigma_k delta_k); T_0 = 1, T_{k+1} = T_k (1 - alpha_k); w_k = T_k alpha_k.
 * Per ray: rgb = sum_k w_k c_k + T_N bg; T_final = T_N; dist = Eq. 1 on (w, s_mid, s_len)
 * computed in O(N) by prefix scans.
 * color: the 3-channel colour grid (DVGO_COLOR_GRID) or NULL; sample_rgb [S,3] for
 * DVGO_COLOR_SAMPLES, else NULL.  Outputs rgb [R,3], T_final [R], dist [R] (NULL allowed
 * when want_dist = 0), and optionally the per-sample weights sample_w [S] (NULL: not
 * written; halted samples get 0).  state: device buffer of dvgo_render_state_size bytes,
 * written here and read by the backward; it must stay unchanged in between. */
int dvgo_render_forward(const dvgo_render_params *p, const dvgo_samples *s, const dvgo_grid *density,
                        const dvgo_grid *color, const float *sample_rgb, float *rgb, float *T_final, float *dist,
                        float *sample_w, void *state, size_t state_bytes, void *stream);

/* Backward of dvgo_render_forward (recomputes each ray's transmittance, weights and
 * distortion prefixes from the saved chunk checkpoints and the saved density logits raw_k:
 * the density grid is not read again, so it must not change between the two calls; the
 * colour grid, in grid mode, is looked up again).  Upstream gradients: grad_rgb [R,3] (required),
 * grad_dist [R] and grad_T [R] (NULL = zero).  T_final must be the forward's output.
 * Writes: density->grad += dL/d(density values); in grid mode color->grad += dL/d(colour
 * values); in sample mode grad_sample_rgb [S,3] = dL/dc (overwritten; zero for halted
 * samples).  The derivative of the distortion term follows Eq. 3 (its third sum read as
 * w_i m_i) plus the derivative of Eq. 1's second term, (2/3) w_k s_len_k.
 * grad_sample_density [S] (may be NULL): when given, the kernel writes dL/d(raw_k), the
 * gradient with respect to each sample's interpolated density logit (zero for halted
 * samples), INSTEAD of adding into density->grad (which may then be NULL); the caller
 * scatters it, e.g. with dvgo_grid_scatter_binned. */
int dvgo_render_backward(const dvgo_render_params *p, const dvgo_samples *s, const dvgo_grid *density,
                         const dvgo_grid *color, const float *sample_rgb, const float *T_final, const void *state,
                         size_t state_bytes, const float *grad_rgb, const float *grad_dist, const float *grad_T,
                         float *grad_sample_rgb, float *grad_sample_density, void *stream);

/* Forward, loss gradient and backward of a training step's rendering in one launch (each ray's
 * wave runs dvgo_render_forward's walk, forms its own loss gradient, then
 * dvgo_render_backward's walk).  The loss is the one dvgo_loss_head computes:
 * L = sum_r |rgb_r - target_r|^2 / (3 R) + dist_weight sum_r dist_r / R (the photometric MSE
 * plus the weighted distortion term of section 2; its dist term only with want_dist), so ray r's
 * upstream gradients are dL/drgb_r = 2 (rgb_r - target_r) / (3 R) and dL/ddist_r =
 * dist_weight / R, and dL/dT_final = 0.  target [R,3] (device), dist_weight >= 0.
 * Outputs, bit for bit as dvgo_render_forward, then dvgo_loss_head without the loss value,
 * then dvgo_render_backward would give them: rgb [R,3], T_final [R], dist [R] (want_dist),
 * state (as the forward leaves it), grad_sample_rgb [S,3] (sample mode, overwritten) and
 * either grad_sample_density [S] (overwritten) or density->grad += (when it is NULL); in grid
 * mode color->grad +=.  The loss value itself is not computed (dvgo_loss_head gives it from
 * rgb and dist).  Errors as for the two calls; DVGO_COLOR_NONE is not accepted. */
int dvgo_render_train(const dvgo_render_params *p, const dvgo_samples *s, const dvgo_grid *density,
                      const dvgo_grid *color, const float *sample_rgb, const float *target, float dist_weight,
                      float *rgb, float *T_final, float *dist, void *state, size_t state_bytes,
                      float *grad_sample_rgb, float *grad_sample_density, void *stream);

/* Schedule of a ragged batch: order [R] = the rays sorted by decreasing number of 64-sample
 * chunks (ceil(length/64), lengths above 63 chunks share the last class; order within a
 * class is unspecified), and class_offsets [65]: order[class_offsets[k] .. class_offsets[k+1])
 * are the rays with 63 - k chunks (k = 63: empty rays).  One block; stream-ordered. */
int dvgo_ray_schedule(int32_t n_rays, const int32_t *ray_offsets, int32_t *order, int32_t *class_offsets,
                      void *stream);

/* Project autotuner for the render kernels: times forward + backward of this batch for a set
 * of launch shapes (waves per block x persistent grid sizes, honouring p->ray_list) with HIP
 * events on `stream` and returns the fastest in *waves_per_block, *grid_waves (and its time
 * in *ms, may be NULL).  sample_density_grad != 0 times the backward variant that writes
 * per-sample density gradients (grad_sample_density of dvgo_render_backward, for a caller that
 * scatters them itself); 0 times the variant that scatters into the density grid in the kernel.
 * Results are cached per (colour mode, distortion, rays, samples, ray list, halt_T, warps of
 * the grids, backward variant) in the process; a cached shape returns without timing.
 * Synchronises the stream and allocates scratch outputs: not for use inside graph capture.
 * Parameter gradients are untouched. */
int dvgo_render_autotune(const dvgo_render_params *p, const dvgo_samples *s, const dvgo_grid *density,
                         const dvgo_grid *color, const float *sample_rgb, int32_t sample_density_grad,
                         int32_t *waves_per_block, int32_t *grid_waves, float *ms, void *stream);

/* Size of the workspace dvgo_distortion_loss needs when grad_w is requested. */
int dvgo_distortion_workspace_size(int32_t n_rays, int64_t n_samples, size_t *bytes);

/* Distortion loss of section 2 on given weights (Eq. 1, computed in O(N) per ray by the
 * prefix-sum rewrite of Eq. 2 and the prefix/suffix form of Eq. 3).  Inputs w, s_mid, s_len
 * [S] on the ray_offsets layout.  loss [R] (may be NULL) receives D_r.  If grad_loss [R] and
 * grad_w [S] are both non-NULL, grad_w += grad_loss[r] * dD_r/dw_k; this needs `ws` of
 * dvgo_distortion_workspace_size bytes (else ws may be NULL). */
int dvgo_distortion_loss(int32_t n_rays, const int32_t *ray_offsets, int64_t n_samples, const float *w,
                         const float *s_mid, const float *s_len, float *loss, const float *grad_loss, float *grad_w,
                         void *ws, size_t ws_bytes, void *stream);

/* dvgo_distortion_loss for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same computation and
 * arguments, minus the workspace.  The backward's per-chunk checkpoints live in a fixed 2 MiB
 * device array inside the library (one per GPU, held until the process ends), so a call
 * allocates nothing; it accepts batches with n_samples/64 + n_rays + 1 <= 262144 checkpoints
 * (e.g. 8192 rays of up to about 16.2 M samples in all) and returns DVGO_ERR_RANGE beyond.  Calls
 * that overlap on one GPU share that array and race: serialise them (one stream, or events).
 * Results equal dvgo_distortion_loss's bit for bit. */
int dvgo_distortion_loss_noalloc(int32_t n_rays, const int32_t *ray_offsets, int64_t n_samples, const float *w,
                                 const float *s_mid, const float *s_len, float *loss, const float *grad_loss,
                                 float *grad_w, void *stream);

/* Total-variation regulariser of a grid, gradient only (section 2, efficient TV loss: the
 * loss itself is not formed; its gradient is added into the grid gradient between the
 * backward pass and the optimiser step).  Loss read as
 *     L = weight / (N C) * sum_p sum_c sum_n huber_delta(v[p][c] - v[n][c])
 * over vertices p (N of them), channels c < channels (C) and the up to six axis neighbours
 * n of p; so g->grad[p][c] += 2 weight / (N C) * sum_n clamp(v[p][c] - v[n][c], -delta, delta).
 * dense != 0: every vertex; dense == 0 (the paper's mode after its first 10k iterations):
 * only vertices where some channel of the incoming g->grad is non-zero.  g->data is read,
 * g->grad is read and updated in place (padding channels untouched).  The Huber threshold
 * is not given in the paper: delta > 0 is an argument.  Errors: DVGO_ERR_NULL,
 * DVGO_ERR_SHAPE (dimensions < 2, bad channels, misaligned float4 rows), DVGO_ERR_RANGE
 * (delta <= 0). */
int dvgo_tv_add_grad(const dvgo_grid *g, float weight, float delta, int32_t dense, void *stream);

/* Fused Adam over n float32 elements (section 3, re-implemented Adam): with 1-based step t,
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr * (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps).
 * t is `step`, or, when step_dev is not NULL, the int32 at step_dev read by the kernel (so a
 * captured HIP graph can advance it between replays with dvgo_counter_add); t must be >= 1.
 * skip_zero_grad != 0: elements whose gradient is exactly zero are skipped entirely (p, m,
 * v untouched), as the paper does for grid points without gradient.  zero_grad_after != 0:
 * the gradient is reset to zero for the next step. */
int dvgo_grid_adam_step(float *param, float *grad, float *exp_avg, float *exp_avg_sq, int64_t n, float lr,
                        float beta1, float beta2, float eps, int32_t step, const int32_t *step_dev,
                        int32_t skip_zero_grad, int32_t zero_grad_after, void *stream);

/* counter[0] += delta on the device (one thread); used to advance the Adam step counter
 * inside captured graphs. */
int dvgo_counter_add(int32_t *counter, int32_t delta, void *stream);

/* Trilinear gather of every channel at n_samples points: out [S, channels] row-major. */
int dvgo_grid_gather(const dvgo_grid *g, int64_t n_samples, const float *xyz, float *out, void *stream);

/* Adjoint of dvgo_grid_gather: g->grad += scatter of grad_out [S, channels]. */
int dvgo_grid_scatter(const dvgo_grid *g, int64_t n_samples, const float *xyz, const float *grad_out,
                      void *stream);

/* Brick-binned scatter (the same sum as dvgo_grid_scatter, organised for few, coalesced global
 * atomics).  dvgo_bin_samples sorts the samples by the 8^3-cell brick of the grid that holds
 * their cell (a counting sort into the caller's workspace of dvgo_bin_workspace_size bytes,
 * 256-byte aligned); dvgo_grid_scatter_binned then adds grad->g += trilinear^T(grad_out) brick
 * by brick, accumulating each brick in on-chip memory first.  The workspace must hold the bins
 * of the same grid geometry (shape, box, warp) and the same xyz; grids with equal geometry can
 * share one binning.  Bins depend only on the points, so one binning serves every scatter of a
 * step. */
int dvgo_bin_workspace_size(const dvgo_grid *g, int64_t n_samples, size_t *bytes);
int dvgo_bin_samples(const dvgo_grid *g, int64_t n_samples, const float *xyz, void *ws, size_t ws_bytes,
                     void *stream);
int dvgo_grid_scatter_binned(const dvgo_grid *g, int64_t n_samples, const float *xyz, const float *grad_out,
                             const void *ws, size_t ws_bytes, void *stream);

/* Owner-computes scatter (the same sum as dvgo_grid_scatter, with no global atomics).  The
 * grid's vertices are cut into bricks of 4 x 4 x 32 (z longest) and each vertex belongs to one brick;
 * dvgo_owner_bin counting-sorts the (sample, brick) pairs of every sample whose cell has corners
 * in that brick (1 to 8 bricks per sample) into the caller's workspace of
 * dvgo_owner_workspace_size bytes (256-byte aligned; about 32 bytes per sample).  Bins depend only
 * on the points and the grid geometry (shape, box, warp): one binning serves every grid of the
 * same geometry and xyz.  dvgo_grid_scatter_owned then adds g->grad += trilinear^T(grad_out)
 * (grad_out [S, channels]): one block per brick sums its pairs' contributions to the vertices it
 * owns on chip and updates each touched vertex once, with a plain read-modify-write (no other
 * kernel may write g->grad meanwhile; elements whose sum is exactly zero are not written).
 * n_samples is at most 89478485 (8 pairs per sample must index in int32). */
int dvgo_owner_workspace_size(const dvgo_grid *g, int64_t n_samples, size_t *bytes);
int dvgo_owner_bin(const dvgo_grid *g, int64_t n_samples, const float *xyz, void *ws, size_t ws_bytes,
                   void *stream);
int dvgo_grid_scatter_owned(const dvgo_grid *g, int64_t n_samples, const float *xyz, const float *grad_out,
                            const void *ws, size_t ws_bytes, void *stream);

/* dvgo_grid_scatter_owned fused with dvgo_grid_adam_step(skip_zero_grad = 1): the gradient of
 * each grid element is the scatter of grad_out alone (no other gradient term: the dense gradient
 * is never formed, g->grad is ignored and may be NULL), and every element whose gradient is not
 * exactly zero takes section 3's Adam update with the same arithmetic as dvgo_grid_adam_step;
 * elements with a zero gradient (untouched vertices, padding channels) keep p, m and v bit for
 * bit.  param, exp_avg, exp_avg_sq: the grid's layout [nx][ny][nz][ch_stride]; g->data must be
 * non-NULL (e.g. param) and is not read.  lr, betas, eps, step and step_dev as in
 * dvgo_grid_adam_step.  The result equals scatter into a zeroed gradient followed by the skipping
 * Adam step, up to the order in which each element's terms are summed.  Use the two calls
 * instead when another term (e.g. dvgo_tv_add_grad) must join the gradient first. */
int dvgo_grid_scatter_adam(const dvgo_grid *g, int64_t n_samples, const float *xyz, const float *grad_out,
                           const void *ws, size_t ws_bytes, float *param, float *exp_avg, float *exp_avg_sq, float lr,
                           float beta1, float beta2, float eps, int32_t step, const int32_t *step_dev,
                           void *stream);

/* Resampling of a grid to another resolution over the same box (progressive grid scaling, the
 * "grid scaling schedule" of Table 7's footnote): out [nx][ny][nz][src->ch_stride] (written)
 * holds at vertex (i, j, k) the trilinear value of src at xyz_min + (i, j, k) (xyz_max -
 * xyz_min)/(n - 1), each coordinate formed in double and rounded to float32; padding channels
 * are written as 0.  The lookup is in the grid's own box (a warp of src is not applied). */
int dvgo_grid_resample(const dvgo_grid *src, int32_t nx, int32_t ny, int32_t nz, float *out, void *stream);

/* Per-sample alpha of the density path only (trilinear, softplus shift, 1 - exp(-sigma delta)):
 * alpha [S].  Used for the coarse samples of the proposal stage. */
int dvgo_alpha(const dvgo_grid *density, int64_t n_samples, const float *xyz, const float *delta, float act_shift,
               float *alpha, void *stream);

/* Workspace for the colour MLP (split weight image, per-ray direction encodings, tile
 * start rays and per-block weight-gradient partials). */
int dvgo_mlp_workspace_size(const dvgo_color_mlp *m, int32_t n_rays, int64_t n_samples, size_t *bytes);

/* The preparation every colour-MLP call starts with, alone: writes into ws the weights as scaled
 * FP16 planes, the view encodings of the rays and the first ray of each 32-sample tile, so that
 * following calls on ws with the same weights and batch can set m->prepared (e.g. on another
 * stream, ahead of the feature gather).  Same arguments and workspace as dvgo_mlp_forward, minus
 * the features; m->prepared is ignored. */
int dvgo_mlp_prepare(const dvgo_color_mlp *m, int32_t n_rays, const int32_t *ray_offsets, const float *dirs,
                     int64_t n_samples, void *ws, size_t ws_bytes, void *stream);

/* Colour MLP forward: rgb [S,3] from feat [S, in_feat] and the direction dirs [R,3] of each
 * sample's ray.  Products run on FP16 matrix cores with every operand split into two FP16
 * parts under a power-of-two scale (hi*hi + hi*lo + lo*hi, FP32 accumulation), which keeps
 * them within about 2^-22 relative; results match an FP32 evaluation to rounding.  Inputs
 * and hidden activations are supported up to about 2^30 in magnitude. */
int dvgo_mlp_forward(const dvgo_color_mlp *m, int32_t n_rays, const int32_t *ray_offsets, const float *dirs,
                     int64_t n_samples, const float *feat, float *rgb, void *ws, size_t ws_bytes, void *stream);

/* dvgo_mlp_forward with the feature gather fused in: the features of sample k are the
 * trilinear lookup of feat_grid at xyz[k] (section 3's interpolation; the grid's warp applied),
 * computed inside the kernel with the same operations as dvgo_grid_gather, so they equal its
 * output bit for bit, and written to feat_out [S, in_feat] when feat_out is not NULL (the input
 * dvgo_mlp_backward recomputes from).  Needs feat_grid->channels == in_feat, in_feat and
 * ch_stride multiples of 4, and feat_grid->data and feat_out 16-byte aligned
 * (DVGO_ERR_UNSUPPORTED otherwise).  Same workspace, preparation and rgb output as
 * dvgo_mlp_forward. */
int dvgo_mlp_forward_gather(const dvgo_color_mlp *m, int32_t n_rays, const int32_t *ray_offsets, const float *dirs,
                            int64_t n_samples, const dvgo_grid *feat_grid, const float *xyz, float *feat_out,
                            float *rgb, void *ws, size_t ws_bytes, void *stream);

/* Colour MLP backward (recomputes the forward, same split-FP16 arithmetic): grad_feat
 * [S, in_feat] written; weight and bias gradients accumulated into m->g*.  A hidden unit whose
 * pre-activation lies within rounding of its ReLU kink may take either side, as in any
 * floating-point evaluation. */
int dvgo_mlp_backward(const dvgo_color_mlp *m, int32_t n_rays, const int32_t *ray_offsets, const float *dirs,
                      int64_t n_samples, const float *feat, const float *grad_rgb, float *grad_feat, void *ws,
                      size_t ws_bytes, void *stream);

/* dvgo_mlp_backward in two parts, so that a caller can take the weight-gradient reduction off
 * the path of the work that needs only grad_feat (e.g. onto another stream, beside the feature
 * scatter).  dvgo_mlp_backward_partials: same arguments and outputs as dvgo_mlp_backward except
 * that the weight and bias gradients stay in ws as one partial sum per block.
 * dvgo_mlp_reduce_grads: adds those partials into m->g* in the same fixed order as
 * dvgo_mlp_backward (the two calls together give its gradients bit for bit); m, n_rays,
 * n_samples and ws as in the partials call.  The partials live in their own part of ws, which
 * dvgo_mlp_prepare and the forward calls do not touch; the next backward call on ws overwrites
 * them, so it must follow the reduction. */
int dvgo_mlp_backward_partials(const dvgo_color_mlp *m, int32_t n_rays, const int32_t *ray_offsets, const float *dirs,
                               int64_t n_samples, const float *feat, const float *grad_rgb, float *grad_feat, void *ws,
                               size_t ws_bytes, void *stream);
int dvgo_mlp_reduce_grads(const dvgo_color_mlp *m, int32_t n_rays, int64_t n_samples, void *ws, size_t ws_bytes,
                          void *stream);

/* Loss head: loss[0] = (1/(3R)) sum ||rgb_r - target_r||^2 + dist_weight (1/R) sum dist_r
 * (dist may be NULL: no distortion term); grad_rgb [R,3] and grad_dist [R] (may be NULL)
 * receive dloss/drgb and dloss/ddist.  The paper weights the distortion term by 1e-2
 * (sections 5.3, 5.4).  Any of loss, grad_rgb, grad_dist may be NULL (not all three).  With
 * loss NULL the gradients come from a launch over all rays with no reduction; the loss value
 * needs a one-block reduction, so a caller can take it on another stream, off the path of the
 * backward. */
int dvgo_loss_head(int32_t n_rays, const float *rgb, const float *target, const float *dist, float dist_weight,
                   float *loss, float *grad_rgb, float *grad_dist, void *stream);

/* ------------------------------------------------------------------ proposal stage
 * Learned sample placement (not part of the paper, which relies on its occupancy mask,
 * section 1): a coarse density-only pass feeds a small MLP that predicts where a ray's
 * weight lies; fine samples are drawn there, with plain uniform sampling as fallback. */

/* Rays of a bounded scene: origins [R,3], unit directions [R,3], and the clipped interval
 * [t_near, t_far] [R] (t_far <= t_near marks a ray that misses the scene box). */
typedef struct dvgo_rays {
    uint32_t struct_size;
    int32_t n_rays;
    const float *origins;
    const float *dirs;
    const float *t_near;
    const float *t_far;
} dvgo_rays;

/* Proposal MLP: n_layers linear layers n_bins -> hidden -> ... -> n_bins with ReLU between,
 * float32 master weights W[l] [out][in] and b[l] [out]; the kernels round weights,
 * activations and back-propagated gradients to bfloat16 (round to nearest even) and
 * accumulate products in float32.  gW/gb receive += in dvgo_proposal_backward.
 * Supported: n_bins = 64, hidden = 64, n_layers = 4. */
typedef struct dvgo_proposal {
    uint32_t struct_size;
    int32_t n_bins;
    int32_t hidden;
    int32_t n_layers;
    const float *W[4];
    const float *b[4];
    float *gW[4];
    float *gb[4];
} dvgo_proposal;

/* Coarse pass: 64 uniform samples per ray at s = (k+1/2)/64 of [t_near, t_far], density-
 * only alpha (same activation as dvgo_render_forward, delta = (t_far-t_near)/64/voxel),
 * front-to-back weights w_k, network input feat_k = ln(1 + w_k/eps) [R,64]; w_coarse [R,64]
 * (may be NULL) receives the weights. */
int dvgo_proposal_coarse(const dvgo_rays *rays, const dvgo_grid *density, float act_shift, float voxel, float eps,
                         float *feat, float *w_coarse, void *stream);

/* Proposal forward: logits [R,64], softmax probabilities prob [R,64] and entropy
 * -sum p ln p [R] (each output may be NULL, not all).  feat/logits/prob 16-byte aligned. */
int dvgo_proposal_forward(const dvgo_proposal *p, int32_t n_rays, const float *feat, float *logits, float *prob,
                          float *entropy, void *stream);

int dvgo_proposal_workspace_size(const dvgo_proposal *p, int32_t n_rays, size_t *bytes);

/* Proposal training backward: cross-entropy -(1/R) sum_r sum_b target_rb ln softmax(z_r)_b
 * against target histograms [R,64] (rows sum to 1); loss[0] (may be NULL) receives the loss,
 * p->gW / p->gb receive += the gradients.  ws: dvgo_proposal_workspace_size bytes. */
int dvgo_proposal_backward(const dvgo_proposal *p, int32_t n_rays, const float *feat, const float *target,
                           float *loss, void *ws, size_t ws_bytes, void *stream);

/* Training target: histogram of rendered weights w [S] over n_bins equal bins of s_mid,
 * normalised to sum 1 when the ray's total weight is at least min_mass, else uniform:
 * hist [R, n_bins].  Supported: n_bins = 64. */
int dvgo_histogram(int32_t n_rays, const int32_t *ray_offsets, const float *w, const float *s_mid, int32_t n_bins,
                   float min_mass, float *hist, void *stream);

/* Offsets of the fine batch: rays that miss get 0 samples, rays with entropy > tau get
 * n_plain (fallback to plain uniform sampling), the others n_fine; writes the exclusive
 * prefix ray_offsets [R+1].  Needs 1 <= n_fine <= 256. */
int dvgo_resample_offsets(const dvgo_rays *rays, const float *entropy, float tau, int32_t n_fine, int32_t n_plain,
                          int32_t *ray_offsets, void *stream);

/* Fills the fine batch laid out by dvgo_resample_offsets.  Fallback rays: s_mid =
 * (k+1/2)/n_plain, s_len = 1/n_plain.  Others (interval resampling): n_fine+1 interval ends
 * e_j = F^{-1}(j/n_fine) of the 64-bin piecewise-constant density prob [R,64] (first bin whose
 * right CDF exceeds u, linear inside the bin; u = 1 maps to the right edge of the last bin
 * with mass); sample j is the interval [e_j, e_{j+1}] at its midpoint: s_mid = (e_j+e_{j+1})/2,
 * s_len = e_{j+1} - e_j.  Points x = o + t d, t = t_near + s (t_far - t_near); delta = s_len
 * (t_far - t_near)/voxel.  Outputs hold ray_offsets[R] samples. */
int dvgo_resample(const dvgo_rays *rays, const float *prob, const float *entropy, float tau,
                  const int32_t *ray_offsets, int32_t n_fine, int32_t n_plain, float voxel, float *xyz, float *delta,
                  float *s_mid, float *s_len, void *stream);

/* Guarded resampling (a reading of the learned proposal that combines section 1's skipping of
 * empty space with placement by the network): coarse bin b of a ray is occupied when
 * max(w_coarse[b-1], w_coarse[b], w_coarse[b+1]) >= w_min (weights of dvgo_proposal_coarse);
 * an occupied bin is cut into n_base equal sub-intervals (n_base = 4: the spacing of plain
 * 256-sample rendering) plus its share of n_extra more, allotted by prob over the occupied bins:
 * with S_b the running sum (double, bin order) of prob over the occupied bins before b and S_tot
 * the total, bin b gets floor(n_extra S_{b+1}/S_tot + 1/2) - floor(n_extra S_b/S_tot + 1/2) (every
 * occupied bin counts 1 instead when S_tot = 0); unoccupied bins get no sample.  Rays with
 * entropy > tau take every bin at n_base (plain uniform sampling); rays with t_far <= t_near
 * take none.  dvgo_resample_guarded_offsets writes counts [R,64] (sub-intervals per bin) and
 * ray_offsets [R+1]; needs n_base >= 1, n_extra >= 0, n_base + n_extra <= 16384.
 * dvgo_resample_guarded fills the batch: sub-interval i of bin b cut into m is the sample
 * s_mid = (b + (i + 1/2)/m)/64, s_len = 1/(64 m), x = o + t d with t = t_near + s_mid (t_far -
 * t_near), delta = s_len (t_far - t_near)/voxel; outputs hold ray_offsets[R] samples. */
int dvgo_resample_guarded_offsets(const dvgo_rays *rays, const float *prob, const float *w_coarse,
                                  const float *entropy, float tau, int32_t n_base, int32_t n_extra, float w_min,
                                  int32_t *ray_offsets, int32_t *counts, void *stream);
int dvgo_resample_guarded(const dvgo_rays *rays, const int32_t *ray_offsets, const int32_t *counts, float voxel,
                          float *xyz, float *delta, float *s_mid, float *s_len, void *stream);

/* ------------------------------------------------------------------ sample producer
 * Builds the ragged batch on the device from rays: points are placed only where a ray
 * crosses the scene box (DVGO_SAMPLE_BOX: section 3, re-implemented rendering utilities;
 * bounded scenes) or on the planes of a forward-facing volume in normalised device
 * coordinates (DVGO_SAMPLE_NDC: section 5.3), and points in space switched off by the
 * occupancy mask are skipped (section 1).
 *
 * Box mode (every step one float32 operation rounded to nearest even, no fused forms except
 * the two fma below; any IEEE float32 evaluation of these steps gives the same integers):
 *   box interval: per axis t0 = (xyz_min - o)/d, t1 = (xyz_max - o)/d, [min, max] of the two
 *     (an axis with d == 0 is unbounded if xyz_min <= o <= xyz_max, else empty); t_exit = the
 *     smallest upper end, t_near = max(largest lower end, near); the ray misses unless
 *     t_exit > t_near;
 *   candidates: n = ceil((t_exit - t_near)/step - 0.5) (0 if that is not positive), capped at
 *     max_per_ray; candidate k = 0..n-1 is the interval [t_near + k step, t_near + (k+1) step]
 *     at its midpoint t_k = fma(k + 0.5, step, t_near), point x = fma(t_k, d, o) per axis;
 *   mask: candidate kept iff mask[i][j][l] != 0 at the nearest vertex, per axis
 *     u = (x - xyz_min) * ((mask_shape - 1)/(xyz_max - xyz_min)), rounded to nearest even,
 *     clamped to [0, mask_shape - 1] (u < 0 or NaN -> 0);
 *   kept candidate: xyz = x, delta = step/voxel, s_mid = (k + 0.5)/n, s_len = 1/n (s linear in
 *     t over the ray's n candidate intervals); rays in order, each ray's samples by k.
 * Directions should be unit vectors for `step` to be a distance (not checked).
 * NDC mode (same float32 rules; rays in the reference camera's frame, looking down -z):
 *   a ray with d_z >= 0 gets no samples; t0 = -(near + o_z)/d_z, p = fma(t0, d, o) per axis;
 *     NDC origin o' = (-(ndc_fx (p_x/p_z)), -(ndc_fy (p_y/p_z)), 1 + (2 near)/p_z), NDC
 *     direction d' = (-(ndc_fx (d_x/d_z - p_x/p_z)), -(ndc_fy (d_y/d_z - p_y/p_z)),
 *     -((2 near)/p_z)), with ndc_fx = 2 focal/W, ndc_fy = 2 focal/H;
 *   candidates: n = min(floor((ndc_planes - 1)/step) + 1, max_per_ray) for every such ray
 *     (2 ndc_planes - 1 at step 0.5); candidate j at t' = (j step)/(ndc_planes - 1), point
 *     x = fma(t', d', o') per axis; kept iff xyz_min <= x <= xyz_max on the x and y axes (depth
 *     runs between the first and last planes by construction) and the mask keeps it (as above);
 *   kept candidate: xyz = x (NDC), delta = step (planes), s_mid = (j + 0.5)/n, s_len = 1/n;
 *     t_near, t_far outputs: (0, 1) for rays with samples, else (0, 0); `voxel` is unused. */
enum { DVGO_SAMPLE_BOX = 0, DVGO_SAMPLE_NDC = 1 };

typedef struct dvgo_sampler {
    uint32_t struct_size;
    int32_t mode;           /* DVGO_SAMPLE_BOX or DVGO_SAMPLE_NDC */
    float xyz_min[3];       /* scene box; also the box of the mask's vertex grid */
    float xyz_max[3];
    float near;             /* samples start at t >= near (finite) */
    float step;             /* spacing of candidates along t (> 0) */
    float voxel;            /* world size of a voxel (> 0): every sample's delta = step / voxel */
    int32_t max_per_ray;    /* 1 .. 2^20; max_per_ray * n_rays must be < 2^31 */
    int32_t mask_shape[3];  /* vertex grid of the mask, entries >= 1, product < 2^31 */
    const uint8_t *mask;    /* [nx][ny][nz] bytes, non-zero = active; NULL = every point active */
    float ndc_fx, ndc_fy;   /* NDC mode: 2 focal / W, 2 focal / H (> 0) */
    int32_t ndc_planes;     /* NDC mode: number of planes D (>= 2); near must be > 0 */
} dvgo_sampler;

/* Counts kept samples per ray and writes ray_offsets [n_rays+1] (exclusive prefix, int32;
 * ray_offsets[n_rays] = total, which the caller reads to size the emit outputs).  t_near,
 * t_far [n_rays] (each may be NULL) receive the box interval, (0, 0) for a ray that misses.
 * origins, dirs [n_rays,3]. */
int dvgo_sample_count(const dvgo_sampler *sp, int32_t n_rays, const float *origins, const float *dirs,
                      int32_t *ray_offsets, float *t_near, float *t_far, void *stream);

/* Writes the kept samples of the batch laid out by dvgo_sample_count (same sampler, rays and
 * mask contents): xyz [capacity,3], delta, s_mid, s_len [capacity].  Samples whose index
 * falls outside [0, capacity) are dropped, never written. */
int dvgo_sample_emit(const dvgo_sampler *sp, int32_t n_rays, const float *origins, const float *dirs,
                     const int32_t *ray_offsets, int64_t capacity, float *xyz, float *delta, float *s_mid,
                     float *s_len, void *stream);

/* Occupancy mask update (section 1: low-density space is switched off as training goes
 * on).  A vertex is dense when the alpha of its own density logit at the sampling step,
 * 1 - exp(-softplus(raw + act_shift) * delta), is at least alpha_thr; mask[v] (bytes over the
 * density grid's vertices [nx][ny][nz]) becomes 1 iff it was non-zero and some vertex of its
 * 3x3x3 neighbourhood (clipped at the faces) is dense, else 0.  The active set only shrinks;
 * the dilation keeps all eight vertices of every cell that touches a dense vertex active.
 * The alpha test is evaluated as raw >= (the smallest float32 logit that passes it).
 * Needs delta > 0, 0 <= alpha_thr < 1; uses channel 0 of the density grid. */
int dvgo_occupancy_update(const dvgo_grid *density, float act_shift, float delta, float alpha_thr, uint8_t *mask,
                          void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DVGO_H */
