/*
 * gsr.h — C ABI of the MI355X (gfx950) differentiable Gaussian-splat
 * rasterizer with the per-ray entropy constraint on alpha-blending weights.
 *
 * The library computes, on the GPU, the forward and backward of
 *   - the EWA projection of 3D Gaussians to 2D conics, radii and SH colour
 *     (Sec. 3, Eq. 1-2),
 *   - tile-based front-to-back alpha blending (Sec. 3, Eq. 3-5),
 *   - the per-pixel entropy of the blending weights, background included,
 *     and its per-view mean (Sec. 4.3, Eq. 8-11),
 *   - the gradient of L = L_base + gamma L_E with respect to every Gaussian
 *     attribute (Sec. 4.4, Eq. 12-15, Alg. 1, Suppl. B-C).
 * L_base and gamma stay with the caller: the backward takes dL/dC per pixel,
 * dL/dH per pixel and dL/dL_E per view.
 *
 * Conventions (defaults; each is a flag):
 *   - OpenCV camera axes (x right, y down, z forward), world->camera R, t;
 *     pixel (px, py) has its centre at (px + 0.5, py + 0.5);
 *   - 2D covariance dilated by 0.3 on the diagonal (GSR_DILATE);
 *   - x/z and y/z clamped to 1.3x the half field of view inside the EWA
 *     Jacobian only (GSR_JACOBIAN_CLAMP);
 *   - colour = sum_k sh_k Y_k(dir) + 0.5, clamped at 0 (GSR_COLOR_CLAMP),
 *     with Y_k the real SH without the Condon-Shortley phase, k = l*l+l+m;
 *   - Gaussians with camera z <= near_z, det <= 0 or non-finite inputs are
 *     culled; alpha = min(0.99, opacity * g); alpha < 1/255 is skipped;
 *     the first Gaussian that would take T below 1e-4 ends the ray and is
 *     not blended; black background;
 *   - radius = ceil(3 sqrt(lambda_max)); a Gaussian is listed in every tile
 *     that meets [mean - radius, mean + radius] in x and y; each tile list is
 *     ordered by (float32 camera depth, Gaussian index).
 *
 * Memory: every pointer in gsr_gaussians, gsr_fwd_out and gsr_grads is a
 * DEVICE pointer owned by the caller, and must be 4-byte aligned (rgb and
 * params) on the device the context was created on.  Camera arrays and
 * statistics outputs are HOST pointers.  The context owns its scratch (pair
 * keys and lists, tile ranges, projected records, 2D gradient accumulators).
 *
 * Errors: argument errors return before any GPU work is enqueued and leave
 * outputs untouched.  GSR_ERR_HIP wraps a HIP runtime failure (text in
 * gsr_last_error).  No C++ exception crosses this interface.
 *
 * Streams: all work is enqueued on the given stream (NULL = default stream);
 * calls return without synchronising except where stated.  A context is not
 * thread-safe and must be used from one host thread at a time.
 */
#ifndef GSR_H
#define GSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSR_OK = 0,
    GSR_ERR_INVALID_ARG = 1,   /* bad pointer, size, enum value or shape */
    GSR_ERR_UNSUPPORTED = 2,   /* valid but not implemented (tile shape, SH degree) */
    GSR_ERR_CAPACITY = 3,      /* pair count exceeded a fixed capacity (graph mode) */
    GSR_ERR_HIP = 4,           /* HIP runtime error */
    GSR_ERR_STALE_FRAME = 5,   /* backward called with a frame a newer forward replaced */
    GSR_ERR_OOM = 6            /* device allocation failed */
} gsr_status;

/* Pinhole camera.  Projection of camera-space (x, y, z):
 *   u = fx x / z + cx,  v = fy y / z + cy  (pixels). */
typedef struct {
    int32_t width, height;     /* 1 .. 32767 */
    float fx, fy, cx, cy;
    float R[9];                /* world -> camera rotation, row-major */
    float t[3];                /* world -> camera translation: x_cam = R x + t */
    float near_z;              /* cull z <= near_z (0.2 is the usual value) */
} gsr_camera;

/* option flags */
#define GSR_DILATE          1u   /* +0.3 on the 2D covariance diagonal */
#define GSR_JACOBIAN_CLAMP  2u   /* 1.3x field-of-view clamp inside the EWA Jacobian */
#define GSR_COLOR_CLAMP     4u   /* clamp colour at 0 */
#define GSR_GRAPH           8u   /* capture forward / backward into HIP graphs and replay them at a
                                    fixed pair capacity: every capture first runs one plain forward and
                                    sizes the capacity at 1.5x its pairs + 4096; a replay whose count came
                                    within 10 % of the capacity (or past it) makes the next forward capture
                                    again; gsr_backward waits for the replayed forward to finish and refuses
                                    (GSR_ERR_CAPACITY) a frame whose pairs did not fit */
#define GSR_PERSISTENT     16u   /* persistent blend kernels: resident workgroups pull tiles from 8 device
                                    queues (one per XCD) of spatially contiguous tiles, stealing from the
                                    others when their own is empty */
#define GSR_NO_SYNC        32u   /* eager launches with a fixed pair capacity and no host synchronisation:
                                    the first frame of a context sizes the capacity (1.5x its pairs + 4096),
                                    later frames read their pair count back asynchronously and the next
                                    frame grows the capacity when a count came within 10 % of it (a frame
                                    past it is flagged as an overflow, see gsr_stats); stage timing works;
                                    ignored with GSR_GRAPH, which never synchronises either */
#define GSR_DEBUG_INVARIANTS 64u /* after each forward, check Eq. 9 (Sec. 4.3; Suppl. A) per pixel: the weights
                                    of the blended Gaussians plus T_final sum to one, by an independent walk of
                                    every pixel's list (debug speed); gsr_stats reports the largest error and
                                    the pixels past the FP32 bound 4u (n_contrib + 1), u = 2^-24 */
#define GSR_DEFAULT_FLAGS  (GSR_DILATE | GSR_JACOBIAN_CLAMP | GSR_COLOR_CLAMP)

typedef struct {
    int32_t tile_w, tile_h;    /* {8,8}, {16,16} or {32,8} */
    int32_t lds_batch;         /* Gaussians staged per LDS batch of the forward: 32, 64, 128, 256; 0 = 64.
                                  The backward walks windows of min(lds_batch, 128) entries (its LDS
                                  holds per-wavefront partial sums of every window entry), or of
                                  min(lds_batch, 64) when the frame's mean list length is 256 or more */
    int32_t sh_degree;         /* 0 .. 3; K = (sh_degree + 1)^2 coefficients per channel */
    int32_t sh_dtype;          /* 0 = float32, 1 = bfloat16 (SH storage and SH gradients) */
    uint32_t flags;            /* GSR_* flags */
} gsr_opts;

/* Gaussian parameters (device, caller-owned, read-only to the library).
 * means [n][3], scales [n][3] (activated, > 0), quats [n][4] (w, x, y, z;
 * normalised inside), opacities [n] (activated, in (0, 1)),
 * sh [n][K][3] float or bfloat16 per gsr_opts.sh_dtype. */
typedef struct {
    int64_t n;
    const float* means;
    const float* scales;
    const float* quats;
    const float* opacities;
    const void* sh;
} gsr_gaussians;

/* Forward outputs (device, caller-owned).  Views are packed back to back:
 * view v's pixels start at pixel offset gsr_pixel_offsets(...)[v], row-major.
 *   rgb [P][3], entropy [P] (H_j, Eq. 10), t_final [P] (T after the last
 *   blended Gaussian), n_contrib [P] (list positions up to and including the
 *   last blended Gaussian), entropy_mean [n_views] (L_E per view, Eq. 11).
 * t_final and n_contrib are the per-pixel state the backward needs; nothing
 * is saved per Gaussian-pixel pair.  frame_id is written by gsr_forward. */
typedef struct {
    float* rgb;
    float* entropy;
    float* t_final;
    int32_t* n_contrib;
    float* entropy_mean;
    int64_t frame_id;
} gsr_fwd_out;

/* Parameter gradients (device, caller-owned, overwritten), same layouts as
 * gsr_gaussians; sh gradients in the SH dtype. */
typedef struct {
    float* means;
    float* scales;
    float* quats;
    float* opacities;
    void* sh;
} gsr_grads;

typedef struct gsr_ctx gsr_ctx;

const char* gsr_status_string(gsr_status s);

/* Text of the last error on this context (never NULL). */
const char* gsr_last_error(const gsr_ctx* ctx);

/* Create a context on the current HIP device.  max_views bounds n_views of
 * later calls (1..64).  pair_capacity: 0 = grow on demand (plain mode);
 * > 0 = initial capacity (used as is in graph mode). */
gsr_status gsr_create(gsr_ctx** out, int32_t max_views, int64_t pair_capacity);
gsr_status gsr_destroy(gsr_ctx* ctx);

/* Pixel offsets of the packed per-view outputs: offsets[v] = sum of
 * width*height of views < v; offsets[n_views] = total.  Host arrays. */
gsr_status gsr_pixel_offsets(const gsr_camera* cams, int32_t n_views, int64_t* offsets);

/* Render n_views cameras (host array) and their entropy (Sec. 3, Eq. 3-5,
 * 8-11).  In plain mode the call synchronises once on `stream` to size the
 * pair buffers; with GSR_GRAPH or GSR_NO_SYNC it does not (after the first
 * frame of the mode on this context). */
gsr_status gsr_forward(gsr_ctx* ctx, void* stream, const gsr_gaussians* g, const gsr_camera* cams,
                       int32_t n_views, const gsr_opts* opts, gsr_fwd_out* out);

/* Test-time rendering: the colour of n_views cameras (Sec. 3, Eq. 3-5) with
 * the same projection, lists and blending as gsr_forward (bit-identical rgb),
 * without the entropy and without per-pixel saved state.  rgb: device, caller-
 * owned, float [P][3] with views packed as in gsr_fwd_out.  Eager launches
 * only (GSR_GRAPH -> GSR_ERR_UNSUPPORTED; GSR_PERSISTENT and GSR_NO_SYNC are
 * honoured); synchronises once on `stream` unless GSR_NO_SYNC.  It replaces the context's frame: a backward of an earlier
 * forward then fails with GSR_ERR_STALE_FRAME.  gsr_stats describes it. */
gsr_status gsr_render(gsr_ctx* ctx, void* stream, const gsr_gaussians* g, const gsr_camera* cams,
                      int32_t n_views, const gsr_opts* opts, float* rgb);

/* Gradients of a loss of the forward outputs (Sec. 4.4, Eq. 13-15, Alg. 1,
 * Suppl. C): grad_rgb [P][3] = dL/dC, grad_entropy [P] = dL/dH_j (may be
 * NULL), grad_entropy_mean [n_views] = dL/dL_E,v (device, may be NULL).
 * `saved` must be the gsr_fwd_out of the latest gsr_forward on this context
 * with the same gaussians, cameras and options. */
gsr_status gsr_backward(gsr_ctx* ctx, void* stream, const gsr_gaussians* g, const gsr_camera* cams,
                        int32_t n_views, const gsr_opts* opts, const gsr_fwd_out* saved,
                        const float* grad_rgb, const float* grad_entropy, const float* grad_entropy_mean,
                        gsr_grads* grads);

/* gsr_backward with the opacity regulariser of the Sec. 5.4 ablation (the
 * comparator of the entropy constraint) fused into the projection backward:
 * grads->opacities also receives dL_O/dsigma_i of
 *   L_O = opacity_weight / n * sum_i exp(-(sigma_i - 0.5)^2 / 0.05)
 * (bit-identical to gsr_backward followed by gsr_opacity_loss with the same
 * weight), and *opacity_loss (device float, may be NULL) receives L_O, summed
 * in a fixed order.  opacity_weight = 0 and opacity_loss = NULL is gsr_backward. */
gsr_status gsr_backward_opacity_reg(gsr_ctx* ctx, void* stream, const gsr_gaussians* g, const gsr_camera* cams,
                                    int32_t n_views, const gsr_opts* opts, const gsr_fwd_out* saved,
                                    const float* grad_rgb, const float* grad_entropy, const float* grad_entropy_mean,
                                    float opacity_weight, float* opacity_loss, gsr_grads* grads);

/* L1 term of the base loss (Sec. 3, Eq. 6 with lambda = 0) on the packed
 * images of the latest forward's cameras (cams must have the same sizes):
 *   grad_rgb [P][3] = sign(rgb - target) / (3 M_v)   (device, may be NULL),
 *   loss [n_views]  = mean over 3 M_v of |rgb - target| (device, may be NULL).
 * rgb and target are device [P][3]. */
gsr_status gsr_l1_loss(gsr_ctx* ctx, void* stream, const gsr_camera* cams, int32_t n_views, const float* rgb,
                       const float* target, float* grad_rgb, float* loss);

/* gsr_l1_loss for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, the same kernels and bit-identical outputs, with the
 * per-block partial sums in a static 1 MiB device array instead of memory the
 * context allocates.  It calls no hipMalloc / hipFree; the array's device
 * address is looked up once per device by gsr_create.  Limit: 131,071 L1
 * blocks of 1,024 pixels over the views of the latest forward (each view's
 * pixel count rounded up to whole blocks; 134,216,704 pixels in one view), else
 * GSR_ERR_CAPACITY with nothing launched.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (different streams or threads)
 * race, and must be serialised by the caller. */
gsr_status gsr_l1_loss_noalloc(gsr_ctx* ctx, void* stream, const gsr_camera* cams, int32_t n_views, const float* rgb,
                               const float* target, float* grad_rgb, float* loss);

/* Opacity regulariser, the comparator of the entropy constraint in the
 * ablation of Sec. 5.4 (opacity vs entropy constraint): with sigma the
 * activated opacities (device, n floats),
 *   L_O = weight / n * sum_i exp(-(sigma_i - 0.5)^2 / 0.05),
 * grad_opacities[i] += dL_O/dsigma_i (device, accumulated, may be NULL) and
 * *loss = L_O (device float, may be NULL).  Deterministic; asynchronous. */
gsr_status gsr_opacity_loss(gsr_ctx* ctx, void* stream, const float* opacities, int64_t n, float weight,
                            float* grad_opacities, float* loss);

/* D-SSIM term of the base loss (Sec. 3, Eq. 6): per view v,
 *   loss[v] = weight * (1 - SSIM(rgb_v, target_v))
 * with the 3DGS-lineage SSIM (11x11 Gaussian window, sigma 1.5, zero outside
 * the image, C1 = 0.01^2, C2 = 0.03^2, mean over pixels and channels).  rgb,
 * target: device [P][3] packed as in gsr_fwd_out; grad_rgb (device, may be
 * NULL) += dloss/drgb; loss (device, n_views floats, may be NULL).  Views are
 * processed one after another; asynchronous. */
gsr_status gsr_dssim(gsr_ctx* ctx, void* stream, const gsr_camera* cams, int32_t n_views, const float* rgb,
                     const float* target, float weight, float* grad_rgb, float* loss);

/* Base loss of Eq. 6 for the latest forward's cameras: per view
 *   loss_l1[v] = (1 - lambda) L1_v,  loss_dssim[v] = lambda (1 - SSIM_v),
 * and grad_rgb (device [P][3], overwritten) = d(loss_l1 + loss_dssim)/drgb.
 * lambda in [0, 1]; the loss outputs (device, n_views floats) may be NULL.
 * Asynchronous. */
gsr_status gsr_base_loss(gsr_ctx* ctx, void* stream, const gsr_camera* cams, int32_t n_views, const float* rgb,
                         const float* target, float lambda, float* grad_rgb, float* loss_l1, float* loss_dssim);

/* One bias-corrected Adam step (step >= 1) on n raw parameters (device):
 *   g = grad_act * d act/d raw,  m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   raw -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps),
 * act = f(raw) with f = identity (kind 0), exp (1: scales from log-scales) or
 * sigmoid (2: opacities from logits); act may be NULL.  Asynchronous. */
gsr_status gsr_adam(gsr_ctx* ctx, void* stream, float* raw, float* m, float* v, float* act, const float* grad_act,
                    int64_t n, int32_t kind, float lr, float beta1, float beta2, float eps, int64_t step);

/* Scale reset (Sec. 4.2, Eq. 7): scales[i][k] <- zeta * scales[i][k] in place
 * (device, n x 3 floats, zeta > 0); an optimiser's log-scales (device, n x 3,
 * may be NULL) get + log(zeta).  Asynchronous. */
gsr_status gsr_scale_reset(gsr_ctx* ctx, void* stream, float* scales, float* log_scales, int64_t n, float zeta);

/* (tile, Gaussian) pair count of each view (host, n_views int64): the
 * projection and the tile count of the forward, no sort or blend.  Replaces
 * the context's frame; synchronises `stream`. */
gsr_status gsr_pair_counts(gsr_ctx* ctx, void* stream, const gsr_gaussians* g, const gsr_camera* cams,
                           int32_t n_views, const gsr_opts* opts, int64_t* pairs_per_view);

/* The camera at downsampling factor r >= 1 (resolution scheduler, Sec. 5.2
 * Implementation Details): width / r and height / r rounded down (at least 1),
 * fx, fy, cx, cy divided by r; pose and near plane unchanged. */
gsr_camera gsr_scaled_camera(const gsr_camera* cam, int32_t r);

/* r_max of the resolution scheduler (Sec. 5.2 Implementation Details): the
 * largest r in [1, r_cap] whose scaled camera keeps the mean per-tile list
 * length (pairs / tiles) at or below max_mean_len (the paper: about 150, with
 * r capped at 4); 1 if none does.  mean_len (host, r_cap doubles, may be NULL)
 * receives the mean for every r.  Replaces the context's frame; synchronises. */
gsr_status gsr_select_rmax(gsr_ctx* ctx, void* stream, const gsr_gaussians* g, const gsr_camera* cam,
                           const gsr_opts* opts, int32_t r_cap, double max_mean_len, int32_t* r_out,
                           double* mean_len);

/* Statistics of the latest forward: the per-tile Gaussian-list lengths whose
 * shortening is the paper's subject (Sec. 5.4 Ablation Study, "Length of
 * Gaussian Lists" and its list-length distribution figure; Sec. 4.1 Overview),
 * and the work the blend did on them (list positions visited, alpha tests,
 * blended pairs; Sec. 3 Background, Eq. 3-5). */
typedef struct {
    int64_t pairs;             /* (tile, Gaussian) pairs over all views */
    double mean_len;           /* mean per-tile list length over all tiles */
    int32_t p99_len;           /* 99th percentile of the per-tile list length */
    int32_t overflow;          /* 1 if a fixed pair capacity was exceeded: that forward is invalid */
    int64_t evals_fwd;         /* alpha evaluations of the forward blend: per pixel, the list
                                  positions visited until the ray stopped or the list ended */
    int64_t evals_bwd;         /* list positions the backward walks: the sum of n_contrib */
    int64_t blended;           /* (pixel, Gaussian) pairs blended: alpha >= 1/255 before the ray stopped */
    int64_t tested_fwd;        /* alpha tests the forward blend makes: of the positions counted in
                                  evals_fwd, those whose Gaussian survives the exact 8x8-block cull
                                  (the others cannot reach 1/255 at any pixel of the block) */
    int64_t tested_bwd;        /* alpha tests the backward makes: surviving positions up to each
                                  pixel's last contributor (a subset of evals_bwd); counted by the
                                  backward, 0 until a backward of this frame has run */
    double invariant_max_err;  /* GSR_DEBUG_INVARIANTS: max over pixels of |sum w + T_final - 1| (Eq. 9);
                                  -1 if the forward did not check */
    int64_t invariant_violations; /* pixels whose error exceeds 4u (n_contrib + 1); -1 if not checked */
} gsr_frame_stats;

/* Fills `out` (host) and pairs_per_view [n_views] (host, may be NULL) for
 * the latest forward on this context; synchronises `stream`. */
gsr_status gsr_stats(gsr_ctx* ctx, void* stream, int64_t* pairs_per_view, gsr_frame_stats* out);

/* Per-stage GPU timing.  gsr_set_timing's `enable` is a mask of stages (bit s
 * = stage s of gsr_stage; GSR_TIME_ALL = every stage; 0 = off).  While a
 * stage's bit is set, each of its launches by gsr_forward / gsr_backward /
 * gsr_render is bracketed by HIP events on the caller's stream (eager launches:
 * plain mode and GSR_NO_SYNC; never under GSR_GRAPH).  Every pair of events
 * costs a few microseconds of the stream's time, so timing only the stages of
 * interest disturbs a step least.  gsr_stage_times synchronises the device,
 * adds the elapsed milliseconds of each stage since the last reset into
 * total_ms[GSR_N_STAGES] and the number of timed launches into
 * launches[GSR_N_STAGES] (host arrays), and resets if `reset` is non-zero. */
typedef enum {
    GSR_STAGE_PROJECT = 0,     /* EWA projection, SH colour, tile rectangles */
    GSR_STAGE_DEPTH_SORT = 1,  /* LSD radix passes over the depth keys of all (view, Gaussian) */
    GSR_STAGE_SCAN = 2,        /* prefix sum of tiles touched, in depth order */
    GSR_STAGE_DUPLICATE = 3,   /* (tile, Gaussian) pair emission */
    GSR_STAGE_TILE_SORT = 4,   /* stable LSD radix passes over the tile digits of the pairs; the
                                  last pass also records each tile's [start, end) */
    GSR_STAGE_RANGES = 5,      /* tiles without pairs set to [0, 0); the tile order */
    GSR_STAGE_BLEND_FWD = 6,   /* front-to-back blend with entropy */
    GSR_STAGE_ENTROPY_MEAN = 7,/* per-view mean entropy */
    GSR_STAGE_BLEND_BWD = 8,   /* back-to-front blend backward with Alg. 1, per-pair gradient rows */
    GSR_STAGE_PROJECT_BWD = 9, /* projection backward, sum over views */
    GSR_STAGE_GRAD_REDUCE = 10,/* per-Gaussian sum of the per-pair gradient rows */
    GSR_N_STAGES = 11
} gsr_stage;

#define GSR_TIME_ALL 0x7ff

gsr_status gsr_set_timing(gsr_ctx* ctx, int32_t enable);
gsr_status gsr_stage_times(gsr_ctx* ctx, double* total_ms, int64_t* launches, int32_t reset);

/* Tile-size choice (Sec. 5.4 Ablation Study, "Effect of tile sizes" and its
 * tile-size table: smaller tiles shorten the per-tile lists but add tiles).
 * Time forward+backward for every tile shape in {8x8, 16x16, 32x8}, LDS
 * batch in {32, 64, 128, 256} and blend scheduling (hardware dispatch or
 * GSR_PERSISTENT) on the given inputs, and write the fastest into
 * inout->tile_w/tile_h/lds_batch and the GSR_PERSISTENT bit of inout->flags
 * (the other flags are kept; the timing runs use plain mode; a candidate's time is the
 * fastest of five forward+backward iterations after one warm-up).  If cache_path is not NULL the result
 * is read from / appended to that text file, keyed by device and workload.
 * Synchronises `stream`.  Note the image depends on the tile shape. */
gsr_status gsr_autotune(gsr_ctx* ctx, void* stream, const gsr_gaussians* g, const gsr_camera* cams,
                        int32_t n_views, gsr_opts* inout, const char* cache_path);

/* Internal buffers of the latest forward/backward, copied to host memory
 * (synchronises `stream`); for stage-by-stage testing.  *bytes receives the
 * size of the buffer; dst may be NULL to query it. */
typedef enum {
    GSR_BUF_RECORDS = 0,       /* float[V*n][12]: mean x, y, A', B', C', opacity, r, g, b, L, kr, kc with
                                  the conic pre-scaled: A' = -A log2(e)/2, B' = -B log2(e), C' = -C log2(e)/2;
                                  L = log2(255 opacity) + 1e-4, the level the blend uses to skip Gaussians
                                  that cannot reach alpha >= 1/255 anywhere in an 8x8 pixel block, and
                                  kr = -B'/(2C'), kc = -B'/(2A'), the slopes on which the exponent's
                                  maximum along a pixel row / column lies (used by that test) */
    GSR_BUF_RADIUS = 1,        /* int32[V*n], 0 = culled */
    GSR_BUF_DEPTH = 2,         /* float[V*n], camera z */
    GSR_BUF_TILES_TOUCHED = 3, /* int32[V*n] */
    GSR_BUF_PAIR_VALUES = 4,   /* uint32[P]: view*n + Gaussian index, sorted by (tile, depth, index) */
    GSR_BUF_PAIR_TILES = 5,    /* uint32[P]: global tile id of each sorted pair (rebuilt from the
                                  tile ranges: the sort's last pass writes no keys) */
    GSR_BUF_RANGES = 6,        /* uint32[n_tiles_total][2] = [start, end) */
    GSR_BUF_GRAD2D = 7         /* float[V*n][9]: dL/d mean x, y, conic A, B, C, opacity, r, g, b of the
                                  latest backward (zero rows for (view, Gaussian)s none of whose pairs
                                  a pixel blended: the device keeps no row for them) */
} gsr_buffer;

gsr_status gsr_inspect(gsr_ctx* ctx, void* stream, gsr_buffer which, void* dst, int64_t capacity_bytes,
                       int64_t* bytes);

#ifdef __cplusplus
}
#endif
#endif /* GSR_H */
