/*
 * sfseg.h -- C ABI of the MI355X (gfx950) SFSeg power-iteration library.
 *
 * Burceanu & Leordeanu, "A 3D Convolutional Approach to Spectral Object
 * Segmentation in Space and Time" (IJCAI 2020, arXiv 1907.02731).
 *
 * The library computes the principal eigenvector of the adjacency matrix M of
 * a video's space-time pixel graph (Sec. 3) by power iteration (Eq. (4)
 * followed by the normalisation of Eq. (8)), with M never formed: every step
 * applies M as three separable 3D Gaussian filterings of the T x H x W volume
 * fused with the element-wise terms of Eq. (7).  Node i = (t, y, x) and
 *
 *     w_i  = S_i^p                         (0^p = 0 for p > 0; p = 0 gives w = 1)
 *     G(d) = exp(-dt^2/(2 sigma_t^2) - (dy^2 + dx^2)/(2 sigma_s^2)),
 *            box |dt| <= r_t, |dy|, |dx| <= r_s, zero outside       (Eq. (1))
 *     M_ij = w_i w_j [1 - alpha (F_i - F_j)^2] G(j - i),
 *            neighbours outside the volume do not exist            (Eq. (2))
 *
 * Conventions shared by every entry point:
 *  - Volumes are contiguous T x H x W arrays, row-major, W fastest; voxel
 *    (t, y, x) is element (t * H + y) * W + x.
 *  - Every array pointer is a DEVICE pointer (for example a torch tensor's
 *    data_ptr()) on the device that was current when the context was created.
 *    Arrays crossing the ABI are float32; the storage precision inside the
 *    library is chosen by sfseg_config.storage.
 *  - Work is ordered on the context's stream.  The host blocks only where an
 *    entry point says so.  A context is not thread-safe.
 *  - Return value: SFSEG_OK (0) or a negative sfseg_status.  Arguments are
 *    validated before any device work; sfseg_last_error() then holds a
 *    message for the calling thread.  No C++ exception crosses the ABI.
 */
#ifndef SFSEG_H
#define SFSEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFSEG_VERSION_MAJOR 0
#define SFSEG_VERSION_MINOR 1

/* Largest radii the compiled kernels support. */
#define SFSEG_MAX_RS 8
#define SFSEG_MAX_RT 4
#define SFSEG_MAX_FEATURES 2 /* pairwise feature channels (Sec. 3.3) */

typedef struct sfseg_ctx sfseg_ctx; /* opaque; owned by the library */

typedef enum {
    SFSEG_OK = 0,
    SFSEG_ERR_INVALID_ARG = -1, /* bad pointer, shape, radius, sigma, alpha, p, dtype */
    SFSEG_ERR_OOM = -2,         /* device or pinned host allocation failed */
    SFSEG_ERR_HIP = -3,         /* a HIP runtime call failed */
    SFSEG_ERR_ZERO_NORM = -4,   /* start vector or an iterate has zero L2 norm */
    SFSEG_ERR_NONFINITE = -5,   /* NaN/Inf in the inputs or the iteration, or S < 0 with p > 0 */
    SFSEG_ERR_STATE = -6,       /* call out of order (e.g. eigvec before iterate) */
    SFSEG_ERR_UNSUPPORTED = -7  /* radius beyond SFSEG_MAX_RS / SFSEG_MAX_RT */
} sfseg_status;

typedef enum {
    SFSEG_F32 = 0,  /* float32 storage of w, F and the iterate */
    SFSEG_BF16 = 1, /* bfloat16 storage, float32 filtering, float64 reductions */
    SFSEG_F16 = 2   /* float16 storage, float32 filtering, float64 reductions */
} sfseg_dtype;

/* Graph and volume parameters (Sec. 3; the paper's experiments use alpha = 1
 * and p = 0.1 or 0.2, Sec. 5).  Constraints: T, H, W >= 1 and
 * T * H * W < 2^31; 0 <= r_t <= SFSEG_MAX_RT; 0 <= r_s <= SFSEG_MAX_RS;
 * sigma_t, sigma_s > 0; alpha >= 0; p >= 0; storage a valid sfseg_dtype. */
typedef struct {
    int32_t T, H, W;
    int32_t r_t, r_s;
    int32_t storage; /* sfseg_dtype */
    double sigma_t, sigma_s;
    double alpha, p;
} sfseg_config;

/* Outcome of sfseg_power_iterate. */
typedef struct {
    int32_t iters;     /* steps taken (Eq. (4) + Eq. (8) each) */
    int32_t converged; /* 1 if delta < tol was reached */
    double delta;      /* ||x_k - x_{k-1}||_2 of the last step (unit iterates) */
    double lambda;     /* x_{k-1}^T M x_{k-1}: Rayleigh quotient (Eq. (3)) of Eq. (2)'s M */
} sfseg_result;

/* GPU-event timings of the last sfseg_power_iterate call on the context's
 * stream.  loop_ms covers only the fused step kernels (one launch per step),
 * so loop_ms / iters is the average step-kernel duration plus launch gaps. */
typedef struct {
    double total_ms; /* whole call: start-vector copy/norm, steps, read-backs */
    double init_ms;  /* start-vector copy and norm */
    double loop_ms;  /* all step launches */
    int32_t iters;
    int32_t launches; /* step kernels launched (>= iters: launches after convergence exit at once) */
} sfseg_timing;

/* Work plan of the step kernel: block shape (0 = 256 threads with 4 outputs
 * each along x, 1 = 512 threads with 2, both filtering on the vector ALUs;
 * 2 = 256 threads with the y and x filter passes on the matrix cores, for
 * float32 storage, one feature channel and r_t <= 2 on single clips; 3 = two
 * power-iteration steps per launch and per pass over HBM (temporal
 * blocking: the intermediate iterate and its halo recomputed in LDS on
 * 32 x 8 tiles), float32 storage, one feature channel, r_s <= 5, r_t <= 2,
 * single clips), number of equal runs of frames each tile's time axis is cut
 * into, and the resulting grid.  Shapes 0 and 1 apply the same per-voxel
 * arithmetic whatever the plan; plans differ only in how the float64 partial
 * sums of the norms are grouped.  Shapes 2 and 3 compute the same products in
 * float32 in another order (shape 2 with the spatial filter sums taken on
 * the matrix cores, each operand split into float16 parts): their results
 * agree with shapes 0/1 to float32 rounding, not bit for bit.  With shape 3
 * a tolerance stop always completes a launch's pair of steps, so a run may
 * take one step more than with the other shapes. */
typedef struct {
    int32_t shape;
    int32_t chunks;
    int32_t blocks;  /* step-kernel grid (filled in by sfseg_get_plan) */
    int32_t threads; /* threads per block (filled in by sfseg_get_plan) */
} sfseg_plan;

/* Fill *cfg with defaults: r_t = 1, r_s = 2, sigma_t = sigma_s = 1, alpha = 1,
 * p = 0.2, storage SFSEG_F32; T, H, W are set to 0 and must be filled in.
 * Host only. */
void sfseg_config_default(sfseg_config *cfg);

/* Check a configuration without touching the GPU.  Host only. */
int sfseg_config_validate(const sfseg_config *cfg);

/* Create a context for one clip (Sec. 3: per-pixel feature maps in, the
 * principal eigenvector out).  Allocates the device buffers, then on `stream` computes w = S^p and
 * copies F (F == NULL means F = S) and S (the default start vector, Alg. 1
 * initialises X with S) into storage precision.  `stream` is a hipStream_t
 * (NULL = the null stream).  The caller may release S and F once the stream
 * has passed this point; the call itself waits for the input check to finish
 * and returns SFSEG_ERR_NONFINITE if S or F holds NaN/Inf or S < 0 with
 * p > 0.  On success *out owns the context; on failure *out is NULL. */
int sfseg_create(const sfseg_config *cfg, const float *S, const float *F, void *stream,
                 sfseg_ctx **out);

/* As sfseg_create with n_features pairwise feature channels (Sec. 3.3,
 * Eq. (9)): one step is the sum of the single-channel steps, i.e. the matrix
 * is M_ij = w_i w_j [C - alpha sum_c (F_c,i - F_c,j)^2] G(j - i).  F holds the
 * n_features channels one after another (n_features x T x H x W, device
 * float32); F == NULL is allowed only for n_features == 1 (F = S).
 * 1 <= n_features <= SFSEG_MAX_FEATURES; more than one channel needs float32
 * storage (SFSEG_ERR_UNSUPPORTED otherwise) and is not available in batches.
 * sfseg_set_features then takes F in the same layout. */
int sfseg_create_mc(const sfseg_config *cfg, const float *S, const float *F, int32_t n_features,
                    void *stream, sfseg_ctx **out);

/* Replace the features of an existing context (same shape and config) without
 * reallocating: the prep of sfseg_create, ordered on the context's stream.
 * Blocks until the input check finishes; invalidates the previous iterate. */
int sfseg_set_features(sfseg_ctx *ctx, const float *S, const float *F);

/* Power iteration (Eqs. (4), (8)): x <- x0 / ||x0|| (x0 == NULL means x0 = S,
 * as in Alg. 1), then up to max_iters steps x <- M x / ||M x||, stopping after
 * the first step whose change delta = ||x_k - x_{k-1}||_2 is below tol
 * (tol <= 0 runs exactly max_iters steps).  x0 is a device float32 volume,
 * read before the call returns.  Blocks the host once per chunk of steps and
 * on return.  max_iters >= 0; max_iters == 0 only normalises x0.  Errors:
 * SFSEG_ERR_ZERO_NORM if x0 or an iterate is zero, SFSEG_ERR_NONFINITE if an
 * iterate overflows.  *res (host) may be NULL. */
int sfseg_power_iterate(sfseg_ctx *ctx, const float *x0, int32_t max_iters, double tol,
                        sfseg_result *res);

/* Write the current unit-norm iterate x_k (float32, T*H*W, device memory
 * owned by the caller) -- the soft segmentation of Eq. (8).  Ordered on the
 * stream; does not block.  SFSEG_ERR_STATE before a successful
 * sfseg_power_iterate. */
int sfseg_eigvec(sfseg_ctx *ctx, float *out);

/* One application of the operator, y = M x (Eq. (2) matrix, applied as the
 * filtering form of Eq. (7)), without normalisation.  x and y are device
 * float32 volumes (they may not alias); x is rounded to storage precision
 * first.  Does not disturb the iteration state.  Blocks until done. */
int sfseg_apply(sfseg_ctx *ctx, const float *x, float *y);

/* Training loss of the learned warm start on the error that survives k
 * power-iteration steps (Algorithm 1 iterates Eq. (4) with the normalisation
 * of Eq. (8) from the start vector; the warm start supplies that vector):
 *     v = M^k xhat,  *loss = 1 - cos(v, target),
 *     grad = dL/dxhat = M^k dL/dv  (M of Eq. (2) is symmetric),
 *     dL/dv = -(target / (|v| |target|) - cos v / |v|^2).
 * xhat, target and grad are device float32 T*H*W volumes of the context's
 * clip (grad may not alias the others); 0 <= k <= 4096 (k = 0 is the plain
 * cosine loss).  The 2k products use the context's step kernel and plan;
 * every product's result is divided by its float64 norm, and the loss's sums
 * are float64.  Allocates a work volume and k norms on the first call (kept
 * until sfseg_destroy); blocks until grad is written.  *loss (host) may be
 * NULL.  Errors: SFSEG_ERR_ZERO_NORM if M^k xhat or target is zero,
 * SFSEG_ERR_NONFINITE on overflow, SFSEG_ERR_STATE for a batch context. */
int sfseg_spectral_grad(sfseg_ctx *ctx, const float *xhat, const float *target, int32_t k,
                        float *grad, double *loss);

/* Frame-wise Rayleigh-Ritz refinement of the current iterate, a start vector
 * for the warm-started form (an addition, not in the paper).  Eq. (3)
 * defines the principal eigenvector as the maximiser of the Rayleigh
 * quotient; this call maximises it over the span of the iterate's frames:
 * with q_t = x_k on frame t (zero elsewhere), B[i][j] = q_i^T M q_j (a band
 * matrix: M couples frames at most r_t apart) and G = diag(|q_t|^2), it
 * writes x_out = sum_t a_t q_t, a the top eigenvector of B a = mu G a, signed
 * for a positive overlap with x_k and scaled to unit norm (frames where x_k
 * is zero get a_t = 0).  x_out is a device float32 T*H*W volume owned by the
 * caller; pass it as x0 to sfseg_power_iterate, which then runs Eq. (4) and
 * Eq. (8) unchanged to its tolerance.  *ritz_value (host, may be NULL)
 * receives mu, the Rayleigh quotient of x_out (<= lambda_1).
 * B takes 2 r_t + 1 products of M through the context's step kernel and
 * plan (frames of one residue modulo 2 r_t + 1 at a time) on the iterate as
 * stored; frame sums are float64, and the band problem is solved on the host
 * in float64.  Allocates two staging volumes and the frame sums on the first
 * call (kept until sfseg_destroy); blocks until x_out is written.  Errors:
 * SFSEG_ERR_STATE before a successful sfseg_power_iterate or for a batch
 * context, SFSEG_ERR_ZERO_NORM if the iterate is zero, SFSEG_ERR_NONFINITE
 * on non-finite values. */
int sfseg_refine_frames(sfseg_ctx *ctx, float *x_out, double *ritz_value);

/* ---- Application without allocation ------------------------------------
 * For callers that cannot allocate device memory or block: code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc.
 * sfseg_apply_noalloc computes what sfseg_apply computes (the same kernels,
 * the same bits) but takes its staging volumes (x and y in padded storage
 * precision), its two state slots and the step kernel's float64 partial sums
 * from one static device array of SFSEG_NOALLOC_SCRATCH_BYTES per GPU,
 * reserved when the library is loaded and held until the process ends.  It
 * calls no allocator and no memset, and does not block: the launches are
 * ordered on the context's stream and y is ready when that stream reaches
 * them.  The array is shared by every call on a GPU and keeps the last call's
 * contents (the call clears what must start at zero), so calls that overlap
 * in time on one GPU (other streams or host threads) race; order them.
 * Errors: SFSEG_ERR_INVALID_ARG for NULL or aliasing pointers and for a
 * context whose staging needs more than the array holds
 * (sfseg_apply_noalloc_bytes tells how much it needs); SFSEG_ERR_STATE for a
 * batch context. */
#define SFSEG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int sfseg_apply_noalloc(sfseg_ctx *ctx, const float *x, float *y);
/* Bytes of the static array sfseg_apply_noalloc needs for this context (0
 * for NULL or batch contexts).  Host only. */
size_t sfseg_apply_noalloc_bytes(const sfseg_ctx *ctx);

/* ---- Binarisation (Sec. 4.1; Alg. 1, step 3) ---------------------------
 * Algorithm 1 projects the normalised solution through a sigmoid after each
 * iteration once a few unconstrained iterations have run, starts the next
 * iteration from the projection, and hard-thresholds the solution after the
 * last one.  The paper leaves the sigmoid's slope, centre, start iteration
 * and scale open; this library reads them as:
 *     z_i  = x_i / max_j x_j                         (scale-free, in [0, 1] for x >= 0)
 *     P_i  = 1 / (1 + exp(-slope (z_i - threshold)))   projection
 *     mask_i = [x_i > threshold * max_j x_j]         hard threshold (strict)
 * The projection is computed in float32 from the stored iterate; the
 * threshold compares the stored values exactly (float64 product of two
 * float32 numbers).  The fixed point is no longer an eigenvector of M. */
typedef struct sfseg_binarize {
    int32_t iters;        /* outer iterations N_i (power steps), >= 1 */
    int32_t project_from; /* project after iterations k with project_from <= k < iters
                             (>= iters: never; must be >= 1) */
    float slope;          /* sigmoid slope, finite and > 0 */
    float threshold;      /* sigmoid centre and hard threshold (relative to the max), finite */
} sfseg_binarize;

/* Defaults: iters = 5 (the paper's experiments), project_from = 3, slope = 10,
 * threshold = 0.5.  Host only. */
void sfseg_binarize_default(sfseg_binarize *b);

/* Replace the current iterate x by the sigmoid projection P(x) above and
 * renormalise (float64 fixed-order norm), so that sfseg_eigvec then returns
 * P / ||P||.  Voxels outside the picture are untouched.  Blocks until done.
 * Errors: SFSEG_ERR_INVALID_ARG for a non-positive or non-finite slope or a
 * non-finite threshold; SFSEG_ERR_STATE before a successful iterate;
 * SFSEG_ERR_ZERO_NORM when no entry of x is positive; SFSEG_ERR_NONFINITE for
 * a non-finite maximum. */
int sfseg_project(sfseg_ctx *ctx, float slope, float threshold);

/* Hard threshold of the current iterate into mask (device uint8, T*H*W, owned
 * by the caller): 1 where x_i > threshold * max_j x_j, else 0.  Ordered on the
 * stream; does not block.  SFSEG_ERR_STATE before a successful iterate. */
int sfseg_threshold(sfseg_ctx *ctx, float threshold, uint8_t *mask);

/* Algorithm 1 with binarisation: x <- x0 / ||x0|| (x0 == NULL: S); for
 * k = 1 .. b->iters one power step (Eqs. (4), (8)), then the projection when
 * b->project_from <= k < b->iters; finally the hard threshold of the last
 * power iterate into mask (device uint8, T*H*W; may be NULL to skip it).  No
 * tolerance: exactly b->iters steps run.  *res (host, may be NULL) receives
 * iters, converged = 0, and delta / lambda of the last step (measured against
 * its unit input, the projected vector when the step before was projected).
 * Leaves the last power iterate as the current iterate.  Blocks until done.
 * Errors as sfseg_power_iterate and sfseg_project. */
int sfseg_segment(sfseg_ctx *ctx, const float *x0, const sfseg_binarize *b, uint8_t *mask,
                  sfseg_result *res);

/* Current work plan of the step kernel.  Host only. */
int sfseg_get_plan(const sfseg_ctx *ctx, sfseg_plan *out);

/* Choose the work plan (see sfseg_plan): shape 0 .. 3, 1 <= chunks <=
 * max(1, T / (4 r_t + 4)), or chunks = 0 for shapes 0 and 1 on single clips:
 * the balanced work list, where each XCD gets a contiguous band of tiles and
 * exactly two work items per resident block slot, some tiles cut into one run
 * of frames more than others, longest items first (SFSEG_ERR_INVALID_ARG if
 * the clip has fewer than 8 tiles or too few frames for it).  Blocks until the
 * new work list is on the device;
 * SFSEG_ERR_INVALID_ARG for values out of range, SFSEG_ERR_UNSUPPORTED for
 * shapes 2 and 3 where they do not exist (16-bit storage, two feature
 * channels, radii beyond their limits, batches).  Does not disturb the
 * iterate. */
int sfseg_set_plan(sfseg_ctx *ctx, int32_t shape, int32_t chunks);

/* Time `steps` steps of every candidate work plan (every block shape the
 * context supports, 1..4 frame runs per tile where the clip allows, and the
 * balanced work list) from the default start vector,
 * keep the fastest, and report it in *best (may be NULL).  Works on single
 * and batch contexts.  Leaves no iterate (call the iterate entry point
 * again).  Blocks for the whole search. */
int sfseg_autotune(sfseg_ctx *ctx, int32_t steps, sfseg_plan *best);

/* ---- Batched form: many clips, one persistent launch per step ----------
 * A batch iterates n clips of uneven size together.  Every step is one launch
 * of a persistent kernel over all (clip, tile, frame run) work items of the
 * clips still iterating; each clip keeps its own norm, Rayleigh quotient,
 * change and convergence flag (Eqs. (4), (8) per clip), and a clip drops out
 * of later launches once it has converged or used its step budget.  All clips
 * must share r_t, r_s, sigma_t, sigma_s, alpha, p and storage (T, H, W may
 * differ).  Batch contexts accept sfseg_get_plan, sfseg_set_plan,
 * sfseg_autotune, sfseg_last_timing and sfseg_destroy; the single-clip calls
 * return SFSEG_ERR_STATE on them. */

/* Create a batch from n >= 1 configurations and device float32 volumes
 * S[i] (T_i x H_i x W_i) and F[i] (F == NULL or F[i] == NULL means F = S).
 * Blocks until the input check has finished (SFSEG_ERR_NONFINITE as for
 * sfseg_create); the caller may then free the inputs. */
int sfseg_batch_create(const sfseg_config *cfgs, int32_t n, const float *const *S,
                       const float *const *F, void *stream, sfseg_ctx **out);

/* Number of clips of a batch context. */
int sfseg_batch_size(const sfseg_ctx *ctx, int32_t *n);

/* Power iteration of every clip (x0 == NULL or x0[i] == NULL: start from
 * S_i), each stopping on its own at delta < tol or after max_iters steps;
 * res (host, n entries, may be NULL) receives each clip's outcome.  Returns
 * the first clip error (its message names the clip); the other clips'
 * results are still filled in. */
int sfseg_batch_iterate(sfseg_ctx *ctx, const float *const *x0, int32_t max_iters, double tol,
                        sfseg_result *res);

/* Write each clip's unit-norm iterate into out[i] (device float32, caller
 * owned).  SFSEG_ERR_STATE before a successful sfseg_batch_iterate. */
int sfseg_batch_eigvec(sfseg_ctx *ctx, float *const *out);

/* Timings of the last sfseg_power_iterate (see sfseg_timing).  Host only. */
int sfseg_last_timing(const sfseg_ctx *ctx, sfseg_timing *out);

/* Release a context and its device buffers.  NULL-safe.  Waits for the
 * context's stream first. */
void sfseg_destroy(sfseg_ctx *ctx);

/* Static description of a status code. */
const char *sfseg_status_string(int status);

/* Message of the last error raised on the calling thread ("" if none). */
const char *sfseg_last_error(void);

/* ---- Learned warm start: a small 3D U-Net --------------------------------
 * Algorithm 1 starts the power iteration from a soft segmentation supplied by
 * another method.  This network maps the input map S (T x H x W, float32) to
 * a non-negative estimate x^ of the principal eigenvector; x^ is then passed
 * as x0 to sfseg_power_iterate, which iterates to the same tolerance as a
 * cold start, so the method itself decides the result.
 *
 * Architecture (fixed): three levels of two 3x3x3 convolutions (zero padding,
 * bias, ReLU) with widths 16 / 32 / 64; 2x2x2 average pooling over zero-padded
 * windows (output size ceil(n / 2)); nearest 2x upsampling cropped to the skip
 * size and concatenated in front of the skip ([up, skip]); a 1x1x1 head and
 * softplus.  Activations bfloat16, weights float32 masters with bfloat16
 * copies for the matrix cores, float32 accumulation; loss 1 - cos(x^, target).
 *
 * Parameter exchange layout (float32, host): for each layer in the order
 * enc1a (1->16), enc1b (16->16), enc2a (16->32), enc2b (32->32), bota
 * (32->64), botb (64->64), dec2a (96->32), dec2b (32->32), dec1a (48->16),
 * dec1b (16->16), head (16->1, 1x1x1): the weights in row-major (Cout, Cin,
 * 3, 3, 3) order ((1, 16) for the head), then the Cout biases.
 *
 * A network object owns its buffers, sized at creation for volumes up to
 * max_T x max_H x max_W; all work is ordered on `stream` (NULL: default).
 * Not thread-safe. */
typedef struct sfseg_unet sfseg_unet;

/* Number of float32 parameters in the exchange layout. */
int64_t sfseg_unet_param_count(void);

/* Create a network (weights zero until sfseg_unet_set_params).  training != 0
 * also allocates gradient buffers and the activations that the backward pass
 * reads; an inference network (training = 0) reads S in its first layer,
 * forms the upsampled halves of the skip concatenations while the
 * convolutions stage their inputs, and runs the head in the last
 * convolution, so it holds neither (same output bit for bit, 124 bytes per
 * voxel less memory).  SFSEG_ERR_INVALID_ARG for sizes < 1 or
 * max_T * max_H * max_W * 48 >= 2^31; SFSEG_ERR_OOM / SFSEG_ERR_HIP. */
int sfseg_unet_create(int32_t max_T, int32_t max_H, int32_t max_W, int32_t training, void *stream,
                      sfseg_unet **out);

/* Copy `count` (= sfseg_unet_param_count()) float32 parameters from / to host
 * memory.  Setting them resets the Adam moments.  Blocks until done. */
int sfseg_unet_set_params(sfseg_unet *net, const float *host_params, int64_t count);
int sfseg_unet_get_params(const sfseg_unet *net, float *host_params, int64_t count);

/* x^ = net(S) for a T x H x W volume (device float32 in and out, caller
 * owned, contiguous).  Stream-ordered: S is read by the call's first kernel
 * (copied first in a training network), `out` written by its last, so they
 * may be the same buffer.  SFSEG_ERR_INVALID_ARG for sizes outside 1..max. */
int sfseg_unet_forward(sfseg_unet *net, const float *S, int32_t T, int32_t H, int32_t W,
                       float *out);

/* Gradients of 1 - cos(x^, target) for the last forward pass (target: device
 * float32 of the same size), written to the network's gradient buffer;
 * *loss (host, may be NULL) receives the loss.  Blocks until done.
 * SFSEG_ERR_STATE without training buffers or forward pass;
 * SFSEG_ERR_ZERO_NORM if x^ or the target has zero norm. */
int sfseg_unet_backward(sfseg_unet *net, const float *target, double *loss);

/* Gradients for an arbitrary loss of the last forward pass, given dL/dx^
 * (device float32, T x H x W of that pass).  Blocks until done.
 * SFSEG_ERR_STATE as for sfseg_unet_backward. */
int sfseg_unet_backward_from(sfseg_unet *net, const float *grad_out);

/* Copy the gradients (exchange layout) to host memory.  Blocks. */
int sfseg_unet_get_grads(const sfseg_unet *net, float *host_grads, int64_t count);

/* One Adam step on the float32 masters with the current gradients (step >= 1
 * is the bias-correction count), then refresh the bfloat16 copies.  Blocks. */
int sfseg_unet_adam_step(sfseg_unet *net, double lr, double beta1, double beta2, double eps,
                         int32_t step);

/* Wait for the network's stream. */
int sfseg_unet_sync(sfseg_unet *net);

/* Release a network.  NULL-safe; waits for its stream first. */
void sfseg_unet_destroy(sfseg_unet *net);

#ifdef __cplusplus
}
#endif

#endif /* SFSEG_H */
