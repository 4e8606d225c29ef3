// Internal declarations of the gfx950 rasterizer library: device-side camera
// record, kernel argument blocks and the host launchers each .hip file
// provides.  Not part of the public ABI (include/gsr.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsr {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlockPx = 8;        // every wavefront blends one 8x8 pixel block
constexpr int kMaxViews = 64;

// Per-view camera and layout record, resident in device memory.
struct CamDev {
    int32_t W, H;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float near_z;
    float campos[3];               // camera centre in world space, -R^T t
    float limx, limy;              // 1.3 x half field of view (tan), Jacobian clamp
    int32_t gx, gy;                // tile grid of this view
    uint32_t tile_base;            // first global tile id of this view
    uint32_t n_wblocks;            // 8x8 wave blocks of this view (tiles x blocks per tile)
    uint32_t block_base;           // first global wave block of this view (tile-major numbering)
    uint32_t pad0, pad1;
    int64_t pix_base;              // first pixel of this view in the packed outputs
    double limx_d, limy_d;         // the clamp bounds in FP64 (the clamp decision is taken in FP64)
    uint32_t hred_base;            // first entropy-reduction chunk of this view (kRedChunk blocks each)
    uint32_t l1_base;              // first L1 block of this view (kL1Block pixels each)
};

constexpr int kRedChunk = 1024;    // 8x8 blocks summed per entropy-reduction chunk
constexpr int kL1Block = 256;      // threads per L1 block
constexpr int kL1Pix = 4 * kL1Block;   // pixels per L1 block (4 a thread)

// Projected record of one (view, Gaussian): three float4
//   r0 = (mean x, mean y, A', B')
//   r1 = (C', opacity, red, green)
//   r2 = (blue, L, kr, kc)  (L: cull level; kr = -B'/(2C'), kc = -B'/(2A'): where the
//        exponent's maximum along a pixel row / column lies)
// with the conic pre-scaled to log2 units: A' = -A log2(e)/2, B' = -B log2(e),
// C' = -C log2(e)/2, so that the exponent is A' dx^2 + B' dx dy + C' dy^2.
constexpr double kLog2e = 1.4426950408889634;
constexpr int kRecF4 = 3;
// mean per-tile list length from which the forward stages each batch once per
// 16x16 / 32x8 tile instead of once per 8x8 block (measured: 200k Gaussians at
// 1296x840, mean 211, per block 0.105 vs shared 0.116 ms; 1M at 1600x1060, mean
// 1025, 0.232 vs 0.184 ms; its half-scale variant, mean 495, per block 0.244 ms)
constexpr double kSharedBatchMeanLen = 256.0;
// persistent blend kernels: one work queue per XCD, heads 128 bytes apart
constexpr uint32_t kQueues = 8;
constexpr uint32_t kQueueStride = 32;
// 2D gradient accumulator per (view, Gaussian): 9 floats
//   dmean x, dmean y, dA, dB, dC, dopacity, dred, dgreen, dblue
constexpr int kG2 = 9;
// per-pair gradient row: the 9 components and a stamp (uint32 bits) naming the
// frame whose backward wrote it; rows with another stamp count as zero (every
// backward of one frame writes the same rows: the entries some pixel blended)
constexpr int kRowF = 10;

struct ProjectFwdArgs {
    const float* means;
    const float* scales;
    const float* quats;
    const float* opac;
    const void* sh;
    uint32_t n;
    int32_t n_views;
    uint32_t flags;
    int32_t tile_shift_x, tile_shift_y;   // log2 of the tile shape
    const CamDev* cams;
    float4* rec;                          // [V*n][3]
    uint32_t* depth_key;                  // [V*n] float bits of camera z; culled = 0xffffffff
    uint2* trect;                         // [V*n] (x0 | x1 << 16, y0 | y1 << 16), inclusive tile bounds
                                          //   (empty: x1 < x0): one 8-byte gather for the depth-ordered
                                          //   scan, which takes the tile count from the bounds
    uint32_t* tiles_touched;              // [V*n]
    int32_t* radius;                      // [V*n]
    float* depth;                         // [V*n]
};

struct ProjectBwdArgs {
    const float* means;
    const float* scales;
    const float* quats;
    const float* opac;
    const void* sh;
    uint32_t n;
    int32_t n_views;
    uint32_t flags;
    const CamDev* cams;
    const float* grad2d;                  // [V*n][9], valid where rec_stamp == *stamp (else zero)
    const uint32_t* rec_stamp;            // [V*n]
    const uint32_t* stamp;                // the frame's stamp (device)
    float* g_means;
    float* g_scales;
    float* g_quats;
    float* g_opac;
    void* g_sh;
    // opacity regulariser fused into the projection backward (0 / null: none): g_opac also
    // gets dL_O/dsigma of L_O = reg_w / n sum exp(-(sigma - 0.5)^2 / 0.05), and, if reg_partial
    // is set, every wavefront writes the sum of its Gaussians' exp terms (FP64) to
    // reg_partial[4 * block + wavefront]
    float reg_w;
    double* reg_partial;
};

struct BlendFwdArgs {
    const float4* rec;
    const uint32_t* pair_vals;            // sorted pairs: emission index e of each (tile, Gaussian) pair
    const uint32_t* emit_vg;              // [P] record (view*n + Gaussian index) of emission index e
    const uint2* ranges;
    const CamDev* cams;
    int32_t n_views;
    int32_t tile_shift_x, tile_shift_y;
    int32_t spt;                          // 8x8 blocks per tile: 1 or 4
    uint32_t n_blocks;                    // 8x8 wave blocks over all views
    float* out_rgb;
    float* out_H;                         // out_H, out_T, out_nc, block_H: unused by the render-only variant
    float* out_T;
    int32_t* out_nc;
    float* block_H;                       // [n_blocks] sum of H over the block
    uint4* block_cnt;                     // [n_blocks][2]: (list positions visited, sum of n_contrib, blended, 0),
                                          //   (alpha tests made, 0: the backward writes its alpha tests, 0, 0)
    uint32_t* queues;                     // persistent mode: kQueues heads kQueueStride words apart, zeroed; or null
    int32_t render_only;                  // 1: colour only (no entropy, no saved state)
    const uint32_t* tile_order;           // [n_tiles] tiles, longest list first (hardware dispatch); or null
    int32_t shared_batches;               // 16x16 / 32x8 tiles: stage each batch once for the 4 blocks
};

struct BlendBwdArgs {
    const float4* rec;
    const uint32_t* pair_vals;            // sorted pairs: emission index e (the pair's gradient row)
    const uint32_t* emit_vg;              // [P] record of emission index e
    const uint2* ranges;
    const CamDev* cams;
    int32_t n_views;
    int32_t tile_shift_x, tile_shift_y;
    int32_t spt;
    uint32_t n_blocks;
    const float* T_final;
    const int32_t* n_contrib;
    const float* grad_rgb;
    const float* grad_H;                  // may be null
    const float* grad_LE;                 // [V] may be null
    float* pair_grad;                     // [P][10] per-pair gradient rows (9 values), emission order
    uint32_t* pair_stamp;                 // [P] stamp of the frame whose backward wrote each row
    const uint32_t* stamp;                // this frame's row stamp
    uint32_t* queues;                     // persistent mode: kQueues heads kQueueStride words apart, zeroed; or null
    const uint32_t* tile_order;           // [n_tiles] tiles, longest list first (hardware dispatch); or null
    uint4* block_cnt;                     // the forward's block counts: word 1 of [2 wb + 1] gets the
                                          //   backward's alpha tests of block wb
};

// Debug check of Eq. 9 after a forward (GSR_DEBUG_INVARIANTS): per pixel, the sum of
// the blending weights plus the final transmittance equals one.
struct InvArgs {
    const float4* rec;
    const uint32_t* pair_vals;
    const uint32_t* emit_vg;
    const uint2* ranges;
    const CamDev* cams;
    int32_t n_views;
    int32_t tile_shift_x, tile_shift_y;
    int64_t n_pix;
    const float* T_final;
    const int32_t* n_contrib;
    uint32_t* counters;                   // [6] max |sum w + T - 1| (float bits), [7] pixels past the bound
};

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_project_fwd(const ProjectFwdArgs& a, int sh_degree, bool sh_bf16, hipStream_t s);
hipError_t launch_project_bwd(const ProjectBwdArgs& a, int sh_degree, bool sh_bf16, hipStream_t s);

// exclusive scan of vals[order[i]] for i < n  ->  out[i]; total -> *total (uint32),
// *overflow |= 1 if the total does not fit in 32 bits; vals_s[i] = vals[order[i]] and
// rect_s[i] = rect[order[i]].  tmp holds scan_tmp_words(n) words; out and vals_s are
// 16-byte aligned.
size_t scan_tmp_words(uint32_t n);
hipError_t launch_gather_scan(const uint2* trect, const uint32_t* order, uint32_t n, uint32_t* out,
                              uint32_t* vals_s, uint2* rect_s, uint32_t* total, uint32_t* overflow, uint32_t* tmp,
                              hipStream_t s);

// one stable LSD radix pass of 8 bits at `shift` over (key, value) pairs; the
// item count is min(*n_dev, n_max) read on the device (n_dev may be null: n_max);
// vals_in null: the values are the items' indices.  ranges non-null: the last pass
// of the tile sort (the keys have no bits above this digit): keys_out is not written,
// and each key k's [start, end) in the output is folded into ranges[k] by atomic
// min / max (ranges initialised to (0xffffffff, 0), see launch_frame_begin; tiles
// without items keep it until launch_ranges_finish).
size_t radix_tmp_words(uint32_t n_max);
hipError_t launch_radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out,
                             uint32_t* vals_out, const uint32_t* n_dev, uint32_t n_max, int shift,
                             uint32_t* tmp, hipStream_t s, uint2* ranges = nullptr);

// write the tile id of every (tile, Gaussian) pair, Gaussians in depth order, at
// its emission index (keys[e]), and emit_vg[e] = view*n + Gaussian index; the
// pairs' sort values are their emission indices (the tile sort's first pass
// takes them as the items' indices)
hipError_t launch_duplicate(const uint32_t* order, const uint32_t* offsets, const uint32_t* tt_s,
                            const uint2* rect_s, const CamDev* cams, uint32_t n, uint32_t vn,
                            const uint32_t* total, uint32_t cap, uint32_t* keys, uint32_t* emit_vg,
                            uint32_t* overflow, hipStream_t s);
// grad2d[vg] = sum of the per-pair rows pair_grad[10 e .. 10 e + 8] with pair_stamp[e] == *stamp over the Gaussian's
// emission range, written, with rec_stamp[vg] = *stamp, for every (view, Gaussian) with at least one such
// row; every other grad2d row is zero by definition and left untouched, with its old stamp;
// carry holds seg_carry_bytes(cap) bytes
size_t seg_carry_bytes(uint32_t cap);
hipError_t launch_grad_reduce(const float* pair_grad, const uint32_t* pair_stamp, const uint32_t* stamp,
                              const uint32_t* emit_vg, uint32_t vn,
                              const uint32_t* total, uint32_t cap, float* grad2d, uint32_t* rec_stamp, void* carry,
                              hipStream_t s);

// a forward's counters: pair total and overflow flag cleared, row stamp (counters[4]) advanced;
// the n_tiles tile bounds in ranges set to (0xffffffff, 0), the words after them up to
// ranges[n_words) cleared
hipError_t launch_frame_begin(uint32_t* counters, uint32_t* ranges, uint32_t n_tiles, uint32_t n_words,
                              hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t count, hipStream_t s);
// p[i] = i
hipError_t launch_iota_u32(uint32_t* p, uint32_t count, hipStream_t s);
// order[n_tiles]: the tiles by decreasing list length (16 classes per octave);
// hist: 512 words, zeroed (bucket counts, then bucket fill counters)
constexpr uint32_t kTileHistWords = 512;
hipError_t launch_tile_order(const uint2* ranges, uint32_t n_tiles, uint32_t* hist, uint32_t* order, hipStream_t s);
// tiles that the last tile-sort pass gave no bounds (no pairs): [0, 0)
hipError_t launch_ranges_finish(uint2* ranges, uint32_t n_tiles, hipStream_t s);


hipError_t launch_blend_fwd(const BlendFwdArgs& a, int lds_batch, hipStream_t s);
hipError_t launch_blend_bwd(const BlendBwdArgs& a, int lds_batch, hipStream_t s);
hipError_t launch_invariants(const InvArgs& a, hipStream_t s);
// n_l1_blocks = sum over views of ceil(W H / kL1Block); tmp holds n_l1_blocks doubles
// L_O = w / n * sum exp(-(sigma - 0.5)^2 / 0.05); grad[i] += dL_O/dsigma_i (grad may be null);
// *loss (device, may be null); tmp holds opacity_reg_tmp_words(n) doubles
size_t opacity_reg_tmp_words(int64_t n);
hipError_t launch_opacity_reg(const float* opac, int64_t n, float w, float* grad, float* loss, double* tmp,
                              hipStream_t s);
// L_O = w / n * sum of the n_partial FP64 partial sums, in a fixed order -> *loss
hipError_t launch_opacity_reg_reduce(const double* partial, uint32_t n_partial, int64_t n, float w, float* loss,
                                     hipStream_t s);
// D-SSIM of one view: loss (device, may be null) = weight (1 - SSIM(x, y)); grad (may be null)
// += dloss/dx; x, y, grad [W*H][3]; tmp holds ssim_tmp_bytes(W*H) bytes
size_t ssim_tmp_bytes(int64_t M);
hipError_t launch_dssim(const float* x, const float* y, int W, int H, float weight, float* grad, float* loss, void* tmp,
                        hipStream_t s);
// one bias-corrected Adam step on raw parameters (kind 0 identity, 1 exp, 2 sigmoid activation)
hipError_t launch_adam(float* raw, float* m, float* v, float* act, const float* grad_act, int64_t n, int kind,
                       float lr, float b1, float b2, float eps, int64_t step, hipStream_t s);
// s <- zeta * s in place over count floats; log_s (may be null) += log(zeta)
hipError_t launch_scale_reset(float* scales, float* log_scales, int64_t count, float zeta, hipStream_t s);
hipError_t launch_l1(const float* rgb, const float* target, const CamDev* cams, int n_views, uint32_t n_l1_blocks,
                     float weight, float* grad, float* loss, double* tmp, hipStream_t s);
// n_chunks = sum over views of ceil(blocks_v / kRedChunk); tmp holds n_chunks doubles
hipError_t launch_entropy_mean(const float* block_H, const CamDev* cams, int n_views, uint32_t n_chunks,
                               double* tmp, float* out_mean, hipStream_t s);

}  // namespace gsr
