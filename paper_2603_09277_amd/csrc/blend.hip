// Front-to-back alpha blending with the entropy of the blending weights
// (Sec. 3, Eq. 3-5; Sec. 4.3, Eq. 8-11) and the back-to-front backward with
// the O(N) entropy gradient of Alg. 1 (Sec. 4.4, Eq. 13-15; Suppl. C).
//
// Work decomposition.  Every 64-lane wavefront owns one 8x8 pixel block (one
// pixel per lane) and walks the Gaussian list of the tile that contains it.
// Wave blocks are numbered tile-major: a 16x16 or 32x8 tile is one workgroup
// of 4 wavefronts (its 4 blocks), an 8x8 tile is one wavefront.  The tile
// shape sets the sort granularity; the wavefront sets the blend granularity.
//
// Forward, two forms.  Per block: each wavefront stages its list in LDS in
// batches of B records (its own LDS region: no workgroup barrier, and a
// wavefront whose 64 pixels have all stopped leaves at the next batch
// boundary).  Shared (16x16 and 32x8 tiles, long lists): the 4 wavefronts of a
// tile stage each batch once, one entry per thread, and the tile's batch loop
// ends when none of its pixels is open.
//
// Culling: while staging, every wavefront drops the Gaussians that cannot
// reach alpha >= 1/255 at any pixel centre of its 8x8 block: the exact maximum
// of the (concave) exponent over the block's pixel-centre rectangle, plus a
// bound on the FP32 evaluation error, is below the skip threshold.  Those
// entries would be skipped by every lane anyway, so results are unchanged;
// the list walk only visits the survivors, compacted in list order.
//
// Backward: list windows of B entries are walked from the back.  In a 16x16
// or 32x8 tile the 4 wavefronts share each window's records.  An entry that
// no lane of a wavefront blended is skipped by that wavefront.  Per Gaussian,
// every wavefront sums its 9 partial gradients over its 64 lanes (half and
// row lane swaps, then DPP) and writes them to its own LDS slot; the window's
// slots (one per wavefront) are summed in a fixed order and stored once per
// (tile, Gaussian) pair, in the pair's emission slot.  A segmented reduction
// over each Gaussian's contiguous emission range then yields its 2D gradient.
// No float atomics touch global memory, so gradients are bit-reproducible.
//
// The conic is stored pre-scaled by -log2(e)/2 (-log2(e) for B) so the
// exponent is in log2 units: alpha = min(0.99, opacity * 2^p); the entropy is
// accumulated in log2 units and scaled by ln 2 once per pixel.
#include "internal.h"

namespace gsr {
namespace {

constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTStop = 1e-4f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr int kWavesPerGroup = 4;
constexpr int kAccF = 10;            // floats per backward accumulator row: 9 sums and a hit flag
constexpr int kFwdRecF4 = kRecF4 + 1; // a staged forward entry: the record and its list position

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// exponent (log2 units) of the 2D Gaussian at offset (dx, dy) = mean - pixel:
//   p = A' dx^2 + B' dx dy + C' dy^2  with the pre-scaled conic (A', B', C');
// explicit FMAs so forward and backward produce bit-identical alphas.
__device__ __forceinline__ float gauss_p2(float A2, float B2, float C2, float dx, float dy)
{
    return fmaf(dx, fmaf(A2, dx, B2 * dy), (C2 * dy) * dy);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}

// Wavefront sums of the 9 per-pixel gradient terms of one list entry, by
// folding registers in pairs so that one add serves two values: the gfx950
// lane swaps between the two 32-lane halves and between neighbouring 16-lane
// rows, then inside each row a rotation by 8 lanes, a half-row mirror and a
// quad sum.  Fixed order: bit-reproducible.  The total of o[c] ends in lane
// tot_lane(c): lanes 16 r and 16 r + 8 hold o[row_comp(r)] and
// o[4 + row_comp(r)], lane 4 holds o[8] (see wave_sum9).
__device__ __forceinline__ int row_comp(uint32_t r) { return (int)(((r & 1u) << 1) | (r >> 1)); }

// the component whose wavefront total wave_sum9 leaves in this lane, or -1
__device__ __forceinline__ int tot_comp(uint32_t lane)
{
    const uint32_t q = lane & 15u;
    return q == 0u ? row_comp(lane >> 4) : (q == 8u ? 4 + row_comp(lane >> 4) : (lane == 4u ? 8 : -1));
}

// lanes 0-31: x[l] + x[l + 32]; lanes 32-63: y[l - 32] + y[l]
__device__ __forceinline__ float fold_halves(float x, float y)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// rows (0, 1, 2, 3) <- (x.r0 + x.r1, y.r0 + y.r1, x.r2 + x.r3, y.r2 + y.r3), lane by lane
__device__ __forceinline__ float fold_rows(float x, float y)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// LDS_FOLD: o[8], which has no partner, has its halves and rows added through the LDS
// crossbar (ds_bpermute, no register copy), else by lane swaps with a copy of itself
// (two VALU operations more, one LDS round trip less: the per-block backward, which
// runs at three wavefronts a SIMD, is faster so; the shared one, at eight, is not)
template <bool LDS_FOLD>
__device__ __forceinline__ float wave_sum9(const float* o, uint32_t lane)
{
    const float u0 = fold_halves(o[0], o[1]), u1 = fold_halves(o[2], o[3]);
    const float u2 = fold_halves(o[4], o[5]), u3 = fold_halves(o[6], o[7]);
    const float u4 = LDS_FOLD ? o[8] + __shfl_xor(o[8], 32, 64) : fold_halves(o[8], o[8]);
    // row r: x0 holds 16 partial sums of o[row_comp(r)], x1 of o[4 + row_comp(r)], x2 of o[8]
    const float x0 = fold_rows(u0, u1), x1 = fold_rows(u2, u3);
    const float x2 = LDS_FOLD ? u4 + __shfl_xor(u4, 16, 64) : fold_rows(u4, u4);
    // row_ror:8 adds lane l ^ 8: 8 partials in each half row
    const float a0 = x0 + dpp_f<0x128, 0xf>(x0);
    const float a1 = x1 + dpp_f<0x128, 0xf>(x1);
    const float a2 = x2 + dpp_f<0x128, 0xf>(x2);
    const float y0 = (lane & 8u) ? a1 : a0;         // lanes 0-7: o[rc], lanes 8-15: o[4 + rc]
    // row_half_mirror adds lane 7 - l of the same half row: 4 partials
    const float b0 = y0 + dpp_f<0x141, 0xf>(y0);
    const float b2 = a2 + dpp_f<0x141, 0xf>(a2);
    const float z = (lane & 4u) ? b2 : b0;          // quads: o[rc], o[8], o[4 + rc], o[8]
    float t = z + dpp_f<0xb1, 0xf>(z);              // quad_perm [1,0,3,2]
    t += dpp_f<0x4e, 0xf>(t);                       // quad_perm [2,3,0,1]
    return t;
}

__device__ __forceinline__ int wave_max_i32(int x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        int y = __shfl_xor(x, o, 64);
        x = x > y ? x : y;
    }
    return x;
}

__device__ __forceinline__ int wave_sum_all_i(int x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ float wave_sum_all(float x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

struct BlockGeom {
    int view;
    uint32_t tx, ty;                 // tile coordinates in the view
    int px, py;
    bool inside;
    uint32_t tile;
    int64_t pix;
    float cx0, cx1, cy0, cy1;        // pixel-centre rectangle of the block's in-image pixels
};

// max over v in [v0, v1] of the concave f(v) = a u^2 + b u v + c v^2 (c < 0), whose
// stationary point is v = k u with k = -b / (2 c)
__device__ __forceinline__ float edge_max(float a, float b, float c, float u, float v0, float v1, float k)
{
    const float v = fminf(fmaxf(k * u, v0), v1);
    return fmaf(u, fmaf(a, u, b * v), (c * v) * v);
}

// true if the Gaussian cannot reach alpha >= 1/255 at any pixel centre of the
// block: r0 = (mean, A', B'), c2 = C', r2 = (blue, L, -B'/(2C'), -B'/(2A')) with
// L = log2(255 opacity) + 1e-4.  The exponent is concave with its maximum 0 at the
// mean; over a rectangle that does not contain the mean its maximum lies on a side
// that faces the mean (the mean is outside that side's half-plane), and at most one
// side per axis faces it.  So two edge maxima give the exact maximum: the facing
// side of each axis, or, for an axis whose range holds the mean, any side of it
// (a value inside the rectangle, which cannot exceed the maximum).  The blend
// evaluates the exponent in FP32 with an error below 1e-6 (|A'|+|B'|+|C'|) |d|^2;
// the test adds twice that bound (and 1.5 % more) to the maximum.
__device__ __forceinline__ bool culled(const BlockGeom& g, float4 r0, float c2, float4 r2)
{
    const float a = r0.z, b = r0.w, c = c2;
    const float eps = 2.03e-6f * (fabsf(a) + fabsf(b) + fabsf(c));
    const float u0 = g.cx0 - r0.x, u1 = g.cx1 - r0.x;       // pixel - mean
    const float v0 = g.cy0 - r0.y, v1 = g.cy1 - r0.y;
    const float uf = u0 > 0.f ? u0 : u1;                    // the side facing the mean (if any)
    const float vf = v0 > 0.f ? v0 : v1;
    float qmax = fmaxf(edge_max(a, b, c, uf, v0, v1, r2.z), edge_max(c, b, a, vf, u0, u1, r2.w));
    if (u0 <= 0.f && u1 >= 0.f && v0 <= 0.f && v1 >= 0.f) qmax = 0.f;    // the mean lies over the block
    const float um = fmaxf(fabsf(u0), fabsf(u1)), vm = fmaxf(fabsf(v0), fabsf(v1));
    const float dmax2 = fmaf(um, um, vm * vm);
    return qmax + eps * dmax2 < -r2.y;
}

// wave block id -> view, tile, pixel of this lane (tile-major numbering,
// `spt` = 8x8 blocks per tile: 1 or 4)
__device__ __forceinline__ BlockGeom block_geom(const CamDev* cams, int n_views, uint32_t wb, uint32_t lane,
                                                int tsx, int tsy, int spt)
{
    BlockGeom g;
    const uint32_t tile = wb / (uint32_t)spt, sub = wb % (uint32_t)spt;
    int v = 0;
    while (v + 1 < n_views && cams[v + 1].tile_base <= tile) ++v;
    const CamDev& c = cams[v];
    const uint32_t lt = tile - c.tile_base;
    const uint32_t tx = lt % (uint32_t)c.gx, ty = lt / (uint32_t)c.gx;
    uint32_t sx = 0, sy = 0;
    if (spt == 4) {
        if (tsx == 4) { sx = sub & 1u; sy = sub >> 1; }   // 16x16: 2x2 blocks
        else { sx = sub; sy = 0; }                         // 32x8: 4x1 blocks
    }
    g.view = v;
    g.tx = tx;
    g.ty = ty;
    g.tile = tile;
    g.px = (int)((tx << tsx) + sx * kBlockPx + (lane & 7u));
    g.py = (int)((ty << tsy) + sy * kBlockPx + (lane >> 3));
    g.inside = g.px < c.W && g.py < c.H;
    g.pix = c.pix_base + (int64_t)g.py * c.W + g.px;
    const int bx0 = (int)((tx << tsx) + sx * kBlockPx), by0 = (int)((ty << tsy) + sy * kBlockPx);
    g.cx0 = (float)bx0 + 0.5f;
    g.cy0 = (float)by0 + 0.5f;
    g.cx1 = (float)min(bx0 + kBlockPx - 1, c.W - 1) + 0.5f;
    g.cy1 = (float)min(by0 + kBlockPx - 1, c.H - 1) + 0.5f;
    return g;
}

// Persistent scheduling.  The n items (in tile-major, i.e. spatial, order) are
// split into kQueues contiguous ranges, one per XCD: workgroups are dispatched
// to the XCDs round-robin, so workgroup b serves queue b % kQueues first and
// neighbouring tiles, which share most of their Gaussians, meet in one XCD's
// L2.  A drained queue sends its workgroups to the next queues.  Each queue
// head is its own 128-byte line; a claim takes `count` consecutive items.
// Returns [first, end) of the claim, or (n, n) when every queue is drained.
__device__ __forceinline__ uint2 claim_items(uint32_t* queues, uint32_t n, uint32_t count)
{
    const uint32_t home = blockIdx.x % kQueues;
    for (uint32_t t = 0; t < kQueues; ++t) {
        const uint32_t k = (home + t) % kQueues;
        const uint32_t lo = (uint32_t)((uint64_t)n * k / kQueues), hi = (uint32_t)((uint64_t)n * (k + 1) / kQueues);
        if (lo >= hi) continue;
        const uint32_t v = atomicAdd(queues + k * kQueueStride, count);
        if (v < hi - lo) return make_uint2(lo + v, lo + v + count < hi ? lo + v + count : hi);
    }
    return make_uint2(n, n);
}

// items of a persistent wavefront, claimed kClaim at a time
constexpr uint32_t kClaim = 4;

struct WaveQueue {
    uint32_t cur = 0, end = 0;
};

__device__ __forceinline__ uint32_t next_item_wave(WaveQueue& q, uint32_t* queues, uint32_t n, uint32_t lane)
{
    if (q.cur >= q.end) {
        uint2 r = make_uint2(0u, 0u);
        if (lane == 0) r = claim_items(queues, n, kClaim);
        q.cur = __shfl(r.x, 0, 64);
        q.end = __shfl(r.y, 0, 64);
        if (q.cur >= q.end) return n;
    }
    return q.cur++;
}


// Per-lane state of the front-to-back walk of one pixel.
struct FwdPix {
    float T, Cr, Cg, Cb, H2;         // transmittance, colour, entropy in log2 units
    int32_t last;                    // n_contrib
    int32_t stop_pos;                // list position of the stopping entry; -1 while the
                                     // pixel is open (0 from the start outside the image)
};

// Wavefront-uniform state of a block's walk (scalar registers): the mask of its
// open pixels (lane l's bit set while stop_pos of lane l is -1), and the alpha
// tests made (a surviving entry visited by a pixel still open) and the entries
// blended, summed over the wavefront.
struct FwdWave {
    uint64_t open;
    uint32_t tested, blended;
};

__device__ __forceinline__ void fwd_init(FwdPix& q, FwdWave& wc, bool inside)
{
    q.T = 1.f; q.Cr = q.Cg = q.Cb = q.H2 = 0.f;
    q.last = 0; q.stop_pos = inside ? -1 : 0;
    wc.open = __builtin_amdgcn_ballot_w64(inside);
    wc.tested = wc.blended = 0u;
}

__device__ __forceinline__ bool fwd_open(const FwdPix& q) { return q.stop_pos < 0; }

// Alpha of one list entry at this lane's pixel (Eq. 3): g0 = (mean, A', B'),
// g1 = (C', opacity, ...).  A pure function of the record and the pixel, so the
// alphas of consecutive entries can be evaluated together.
__device__ __forceinline__ float fwd_alpha(float4 g0, float4 g1, float fpx, float fpy)
{
    const float p = gauss_p2(g0.z, g0.w, g1.x, g0.x - fpx, g0.y - fpy);
    return fminf(kAlphaMax, g1.y * __builtin_amdgcn_exp2f(p));
}

// One surviving list entry for one pixel, given its alpha: the transmittance stop,
// colour (Eq. 5) and the entropy term -w log2 w (Eq. 10).  pos1: the entry's list
// position + 1.  Whether a lane is open, and the counts, are lane masks and their
// sums (scalar work); the ray stops once per pixel, so its bookkeeping sits in a
// branch the wavefront almost always skips.
template <bool RENDER>
__device__ __forceinline__ void fwd_apply(FwdPix& q, FwdWave& wc, float alpha, float cr, float cg, float cb,
                                          int32_t pos1)
{
    const float Tn = q.T * (1.f - alpha);
    // lane masks: open pixels the entry reaches; of those, the ones it would take below
    // T = 1e-4 (they stop) and the rest (they blend)
    const uint64_t hit = wc.open & __builtin_amdgcn_ballot_w64(alpha >= kAlphaMin);
    const uint64_t low = __builtin_amdgcn_ballot_w64(Tn < kTStop);
    const uint64_t stop = hit & low, blend = hit & ~low;
    wc.tested += (uint32_t)__popcll(wc.open);
    wc.blended += (uint32_t)__popcll(blend);
    wc.open &= ~stop;
    if (__builtin_expect(__builtin_amdgcn_inverse_ballot_w64(stop), 0)) q.stop_pos = pos1 - 1;
    if (__builtin_amdgcn_inverse_ballot_w64(blend)) {
        const float w = alpha * q.T;
        q.Cr = fmaf(w, cr, q.Cr);
        q.Cg = fmaf(w, cg, q.Cg);
        q.Cb = fmaf(w, cb, q.Cb);
        if (!RENDER) q.H2 = fmaf(-w, __builtin_amdgcn_logf(w), q.H2);    // -w log2 w   (Eq. 10)
        q.T = Tn;
        q.last = pos1;
    }
}

template <bool RENDER>
__device__ __forceinline__ void fwd_step(FwdPix& q, FwdWave& wc, float4 g0, float4 g1, float b, float fpx, float fpy,
                                         int32_t pos1)
{
    fwd_apply<RENDER>(q, wc, fwd_alpha(g0, g1, fpx, fpy), g1.z, g1.w, b, pos1);
}

// Outputs of one pixel and the work counts of its 8x8 block.
template <bool RENDER>
__device__ __forceinline__ void fwd_store(const BlendFwdArgs& a, const BlockGeom& g, const FwdPix& q,
                                          const FwdWave& wc, uint2 rg, uint32_t wb, uint32_t lane)
{
    // background weight T_{N+1} (Eq. 9-10), then natural-log units
    const float H = RENDER ? 0.f : kLn2 * fmaf(-q.T, __builtin_amdgcn_logf(q.T), q.H2);
    if (g.inside) {
        a.out_rgb[3 * g.pix + 0] = q.Cr;
        a.out_rgb[3 * g.pix + 1] = q.Cg;
        a.out_rgb[3 * g.pix + 2] = q.Cb;
        if (!RENDER) {
            a.out_H[g.pix] = H;
            a.out_T[g.pix] = q.T;
            a.out_nc[g.pix] = q.last;
        }
    }
    // list positions this pixel visited (the stopping entry included), culled ones counted
    const int32_t n_eval = !g.inside ? 0 : (!fwd_open(q) ? q.stop_pos + 1 : (int32_t)(rg.y - rg.x));
    const uint32_t ne = (uint32_t)wave_sum_all_i(n_eval);
    const uint32_t nc = (uint32_t)wave_sum_all_i(q.last);
    const uint32_t nb = wc.blended;
    // alpha tests at list positions that survived the block cull that this kernel
    // made (until the ray stopped); the backward adds its own count (up to the last
    // contributor) in the next word
    const uint32_t tf = wc.tested;
    const float hs = RENDER ? 0.f : wave_sum_all(g.inside ? H : 0.f);
    if (lane == 0) {
        if (!RENDER) a.block_H[wb] = hs;
        a.block_cnt[2 * wb] = make_uint4(ne, nc, nb, 0u);
        a.block_cnt[2 * wb + 1] = make_uint4(tf, 0u, 0u, 0u);
    }
}

// One wavefront per 8x8 block with its own batches: a wavefront whose pixels
// have all stopped leaves at once, which pays on short lists; on long ones the
// four blocks of a tile restage the same entries (blend_fwd_shared_kernel
// below stages them once).  RENDER: colour only (test-time rendering): no
// entropy, no per-pixel saved state.
template <int B, bool PERSIST, bool RENDER>
__global__ __launch_bounds__(256) void blend_fwd_kernel(BlendFwdArgs a)
{
    __shared__ float4 s_g0[kWavesPerGroup][B];   // mean x, mean y, A', B'
    __shared__ float4 s_g1[kWavesPerGroup][B];   // C', opacity, red, green
    __shared__ float2 s_bp[kWavesPerGroup][B];   // blue, position in the tile list + 1 (int bits)
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    WaveQueue wq;
    uint32_t item;
    if (PERSIST) {
        item = next_item_wave(wq, a.queues, a.n_blocks, lane);
    } else if (a.tile_order) {                   // hardware dispatch, longest tiles first
        if (a.spt == 4) {
            item = a.tile_order[blockIdx.x] * kWavesPerGroup + wid;  // one tile per workgroup
        } else {
            const uint32_t i = blockIdx.x * kWavesPerGroup + wid;    // one tile per wavefront
            item = i < a.n_blocks ? a.tile_order[i] : a.n_blocks;
        }
    } else {
        item = blockIdx.x * kWavesPerGroup + wid;
    }
    for (; item < a.n_blocks; item = PERSIST ? next_item_wave(wq, a.queues, a.n_blocks, lane) : a.n_blocks) {
    const uint32_t wb = item;
    const BlockGeom g = block_geom(a.cams, a.n_views, wb, lane, a.tile_shift_x, a.tile_shift_y, a.spt);
    const uint2 rg = a.ranges[g.tile];
    const float fpx = (float)g.px + 0.5f, fpy = (float)g.py + 0.5f;
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    FwdPix q;
    FwdWave wc;
    fwd_init(q, wc, g.inside);
    // a batch's records are loaded into registers one batch ahead (in flight while the
    // previous batch blends), their record indices (two dependent loads) two batches
    // ahead, 64 entries a register
    constexpr int NH = (B + kWave - 1) / kWave;
    uint32_t pv[NH];
    float4 c0[NH], c1[NH], c2[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        const uint32_t jh = (uint32_t)h * kWave + lane;
        const uint32_t e = rg.x + jh;
        pv[h] = jh < (uint32_t)B && e < rg.y ? a.emit_vg[a.pair_vals[e]] : 0u;
        c0[h] = c1[h] = c2[h] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (jh < (uint32_t)B && e < rg.y) {
            const float4* r = a.rec + (size_t)kRecF4 * pv[h];
            c0[h] = r[0];
            c1[h] = r[1];
            c2[h] = r[2];
        }
        const uint32_t e2 = rg.x + B + jh;
        if (jh < (uint32_t)B && e2 < rg.y) pv[h] = a.emit_vg[a.pair_vals[e2]];
    }
    for (uint32_t bs = rg.x; bs < rg.y; bs += B) {
        if (wc.open == 0ull) break;
        const uint32_t cnt = (rg.y - bs) < (uint32_t)B ? (rg.y - bs) : (uint32_t)B;
        // stage the batch, keeping (in list order) only Gaussians that can reach this block
        uint32_t m = 0;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const uint32_t j0 = (uint32_t)h * kWave;
            if (j0 >= cnt) continue;                           // (uniform; no break, so the registers stay)
            const uint32_t j = j0 + lane;
            const bool keep = j < cnt && !culled(g, c0[h], c1[h].x, c2[h]);
            const uint64_t bal = __ballot(keep);
            if (keep) {
                const uint32_t k = m + (uint32_t)__popcll(bal & lt_mask);
                s_g0[wid][k] = c0[h];
                s_g1[wid][k] = c1[h];
                s_bp[wid][k] = make_float2(c2[h].x, __int_as_float((int32_t)(bs + j - rg.x) + 1));
            }
            m += (uint32_t)__popcll(bal);
        }
        // the next batch's records, the record indices of the one after
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const uint32_t jh = (uint32_t)h * kWave + lane;
            if (jh < (uint32_t)B && bs + B + jh < rg.y) {
                const float4* r = a.rec + (size_t)kRecF4 * pv[h];
                c0[h] = r[0];
                c1[h] = r[1];
                c2[h] = r[2];
            }
            if (jh < (uint32_t)B && bs + 2 * B + jh < rg.y) pv[h] = a.emit_vg[a.pair_vals[bs + 2 * B + jh]];
        }
        wave_lds_sync();
        m = (uint32_t)__builtin_amdgcn_readfirstlane((int)m);   // wavefront-uniform: a scalar loop
        // two entries a step: both alphas evaluated before either is applied
        for (uint32_t k = 0; k < m; k += 2) {
            const uint32_t k1 = k + 1 < m ? k + 1 : k;           // an entry that can be read
            const float4 a1 = s_g1[wid][k], b1 = s_g1[wid][k1];
            const float aa = fwd_alpha(s_g0[wid][k], a1, fpx, fpy);
            const float ab = fwd_alpha(s_g0[wid][k1], b1, fpx, fpy);
            const float2 pa = s_bp[wid][k];
            fwd_apply<RENDER>(q, wc, aa, a1.z, a1.w, pa.x, __float_as_int(pa.y));
            if (k + 1 < m) {
                const float2 pb = s_bp[wid][k1];
                fwd_apply<RENDER>(q, wc, ab, b1.z, b1.w, pb.x, __float_as_int(pb.y));
            }
        }
        wave_lds_sync();
    }
    fwd_store<RENDER>(a, g, q, wc, rg, wb, lane);
    }
}

// The 4 wavefronts of a workgroup are the 4 8x8 blocks of one 16x16 or 32x8
// tile: each batch of the tile's list is staged once for all four (one entry per
// thread), then every wavefront keeps the entries that can reach its block (the
// exact cull, into its own index list) and blends them.  The batch loop ends when
// no pixel of the tile is still open.
template <int B, bool PERSIST, bool RENDER>
__global__ __launch_bounds__(256) void blend_fwd_shared_kernel(BlendFwdArgs a)
{
    static_assert(B <= 256, "one staged entry per thread");
    // a batch entry j: s_rec[0][j] = (mean x, mean y, A', B'), s_rec[1][j] = (C', opacity,
    // red, green), s_rec[2][j] = (blue, L, -B'/(2C'), -B'/(2A')), s_rec[3][j].x = list
    // position + 1 (int bits); one array per part, so that the lanes of the cull, one
    // entry each, read 16-byte strides (no bank conflicts), and the blend loop reads all
    // four parts of entry j at one offset, 16 j
    __shared__ float4 s_rec[kFwdRecF4][B];
    // each wavefront's surviving batch entries (byte offsets), in list order, and after
    // the last of them a valid offset; read two at a time, so a row holds one pair more
    // than a batch needs
    __shared__ int2 s_idx2[kWavesPerGroup][B / 2 + 1];
    __shared__ uint32_t s_item;
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6, tid = threadIdx.x;
    const uint32_t n_items = a.n_blocks / kWavesPerGroup;      // tiles
    auto next = [&]() -> uint32_t {
        if (!PERSIST) return n_items;
        __syncthreads();
        if (tid == 0) s_item = claim_items(a.queues, n_items, 1u).x;
        __syncthreads();
        return s_item;
    };
    uint32_t item;
    if (PERSIST) item = next();
    else item = a.tile_order ? a.tile_order[blockIdx.x] : blockIdx.x;   // longest tiles first
    for (; item < n_items; item = next()) {
    const uint32_t wb = item * kWavesPerGroup + wid;
    const BlockGeom g = block_geom(a.cams, a.n_views, wb, lane, a.tile_shift_x, a.tile_shift_y, a.spt);
    const uint2 rg = a.ranges[g.tile];
    const float fpx = (float)g.px + 0.5f, fpy = (float)g.py + 0.5f;
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    FwdPix q;
    FwdWave wc;
    fwd_init(q, wc, g.inside);
    // each thread stages one entry of a batch: its record is loaded into registers one
    // batch ahead (in flight while the previous batch blends), its record index (two
    // dependent loads) two batches ahead
    uint32_t pv = 0;
    float4 n0 = make_float4(0.f, 0.f, 0.f, 0.f), n1 = n0, n2 = n0;
    if (tid < (uint32_t)B && rg.x + tid < rg.y) {
        pv = a.emit_vg[a.pair_vals[rg.x + tid]];
        const float4* r = a.rec + (size_t)kRecF4 * pv;
        n0 = r[0];
        n1 = r[1];
        n2 = r[2];
    }
    if (tid < (uint32_t)B && rg.x + B + tid < rg.y) pv = a.emit_vg[a.pair_vals[rg.x + B + tid]];
    for (uint32_t bs = rg.x; bs < rg.y; bs += B) {
        // (also orders this batch's staging after every wavefront's reads of the last one)
        if (!__syncthreads_or(wc.open != 0ull ? 1 : 0)) break;  // every pixel of the tile has stopped
        const uint32_t cnt = (rg.y - bs) < (uint32_t)B ? (rg.y - bs) : (uint32_t)B;
        if (tid < cnt) {
            s_rec[0][tid] = n0;
            s_rec[1][tid] = n1;
            s_rec[2][tid] = n2;
            s_rec[3][tid] = make_float4(__int_as_float((int32_t)(bs - rg.x + tid) + 1), 0.f, 0.f, 0.f);
        }
        __syncthreads();
        if (tid < (uint32_t)B && bs + B + tid < rg.y) {
            const float4* r = a.rec + (size_t)kRecF4 * pv;
            n0 = r[0];
            n1 = r[1];
            n2 = r[2];
        }
        if (tid < (uint32_t)B && bs + 2 * B + tid < rg.y) pv = a.emit_vg[a.pair_vals[bs + 2 * B + tid]];
        uint32_t m = 0;
        if (wc.open != 0ull) {                                   // this block still has open pixels
            for (uint32_t j0 = 0; j0 < cnt; j0 += kWave) {
                const uint32_t j = j0 + lane;
                const bool keep = j < cnt && !culled(g, s_rec[0][j], s_rec[1][j].x, s_rec[2][j]);
                const uint64_t bal = __ballot(keep);
                if (keep) {
                    const uint32_t k = m + (uint32_t)__popcll(bal & lt_mask);
                    reinterpret_cast<int32_t*>(&s_idx2[wid][0])[k] = (int32_t)(sizeof(float4) * j);
                }
                m += (uint32_t)__popcll(bal);
            }
        }
        // the slot after the last survivor holds a valid offset (entry 0), so that a step's
        // second entry can always be read
        if (lane == 0) reinterpret_cast<int32_t*>(&s_idx2[wid][0])[m] = 0;
        wave_lds_sync();
        m = (uint32_t)__builtin_amdgcn_readfirstlane((int)m);   // wavefront-uniform: a scalar loop
        // two entries a step: their offsets read together, both alphas evaluated before
        // either is applied (independent chains), then applied in list order
        for (uint32_t k = 0; k < m; k += 2) {
            const int2 off = s_idx2[wid][k / 2];                 // k + 1 <= B: inside the row
            const float4* ra = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(&s_rec[0][0]) + off.x);
            const float4* rb = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(&s_rec[0][0]) + off.y);
            const float4 a1 = ra[B], b1 = rb[B];
            const float aa = fwd_alpha(ra[0], a1, fpx, fpy);
            const float ab = fwd_alpha(rb[0], b1, fpx, fpy);
            fwd_apply<RENDER>(q, wc, aa, a1.z, a1.w, ra[2 * B].x, __float_as_int(ra[3 * B].x));
            if (k + 1 < m) fwd_apply<RENDER>(q, wc, ab, b1.z, b1.w, rb[2 * B].x, __float_as_int(rb[3 * B].x));
        }
    }
    fwd_store<RENDER>(a, g, q, wc, rg, wb, lane);
    }
}

// Per-lane state of the backward walk of one pixel.  The per-pixel sums the
// backward needs, S_{i+1} = sum_{k>i} w_k c_k (colour, Eq. 13-14) and Alg. 1's
// R_{i+1} = sum_{k>i} (ln w_k + 1) w_k + (ln T + 1) T (entropy, Eq. 15), only
// ever enter dL/dalpha_i through Q_{i+1} = gh R_{i+1} - dL/dC . S_{i+1}, so one
// running scalar carries both:
//   dL/dalpha_i = T_i D_i + Q_{i+1} / (1 - alpha_i),
//   D_i = dL/dC . c_i - gh (ln w_i + 1),   Q_i = Q_{i+1} - w_i D_i,
// with gh = dL/dH of the pixel and Q_{N+1} = gh (ln T_final + 1) T_final.
struct BwdPix {
    int32_t n;                       // list positions to walk (n_contrib)
    float T;                         // T_{i+1} while walking back; starts at T_final
    float gCr, gCg, gCb;             // dL/dC of this pixel
    float gh, ghl;                   // dL/dH of this pixel, and gh ln 2 (weights' logs are in log2 units)
    float Q;                         // Q_{i+1}
    float fpx, fpy;
};

// Backward of one list entry for one pixel.  Branch-free per lane: every lane
// evaluates the entry and a lane whose pixel did not blend it (position past its
// last contributor, or alpha < 1/255) contributes zero and keeps its state.
// bwd_alpha evaluates alpha; bwd_grad, run only if some lane of the wavefront
// blended the entry, updates the walk state and returns the 9 per-pixel terms
// whose sums over pixels give the entry's gradient:
//   o[0] = e2 dg          (-> opacity; e2 = 2^p, dg = dL/dalpha in the unclamped branch)
//   o[1] = o[0] dx,  o[2] = o[0] dy                     (-> mean, with the conic)
//   o[3] = o[1] dx,  o[4] = o[1] dy,  o[5] = o[2] dy     (-> conic A, B, C)
//   o[6..8] = w dL/dC                                   (-> colour)
// The per-Gaussian factors (opacity, conic, ln 2) are applied once per
// (tile, Gaussian) after the sum, by finish_row.
struct BwdAlpha {
    float dx, dy, e2, a_raw, alpha;
    bool act;
};

// j: the entry's index in the window, nrel = n - (the window's first list position),
// both scaled by the same positive factor (the record's byte size)
__device__ __forceinline__ BwdAlpha bwd_alpha(const BwdPix& q, int32_t j, int32_t nrel, float4 g0, float4 g1)
{
    BwdAlpha r;
    r.dx = g0.x - q.fpx;
    r.dy = g0.y - q.fpy;
    r.e2 = __builtin_amdgcn_exp2f(gauss_p2(g0.z, g0.w, g1.x, r.dx, r.dy));
    r.a_raw = g1.y * r.e2;
    r.alpha = fminf(kAlphaMax, r.a_raw);
    r.act = (j < nrel) & (r.alpha >= kAlphaMin);
    return r;
}

__device__ __forceinline__ void bwd_grad(BwdPix& q, const BwdAlpha& r, float4 g1, float cb, float* o)
{
    const bool act = r.act;
    const float rom = __builtin_amdgcn_rcpf(1.f - r.alpha);
    const float Ti = q.T * rom;                              // T_i = T_{i+1} / (1 - alpha_i)
    const float w = r.alpha * Ti;
    const float lw2 = __builtin_amdgcn_logf(act ? w : 1.f);  // log2 w_i
    const float D = fmaf(-q.ghl, lw2, fmaf(q.gCr, g1.z, fmaf(q.gCg, g1.w, fmaf(q.gCb, cb, -q.gh))));
    const float dal = rom * fmaf(q.T, D, q.Q);              // (T_{i+1} D_i + Q_{i+1}) / (1 - alpha_i)
    const float wa = act ? w : 0.f;
    const float dg = (act & (r.a_raw <= kAlphaMax)) ? dal : 0.f;   // zero in the clamped branch
    o[0] = r.e2 * dg;
    o[1] = o[0] * r.dx;
    o[2] = o[0] * r.dy;
    o[3] = o[1] * r.dx;
    o[4] = o[1] * r.dy;
    o[5] = o[2] * r.dy;
    o[6] = wa * q.gCr;
    o[7] = wa * q.gCg;
    o[8] = wa * q.gCb;
    q.Q = fmaf(-wa, D, q.Q);                                 // Q_i = Q_{i+1} - w_i D_i
    q.T = act ? Ti : q.T;
}

// Gradient row of one (tile, Gaussian) pair from the summed terms S[0..8] of
// bwd_grad, with g0 = (mean, A', B'), g1 = (C', opacity, ...):  alpha = opacity 2^p and
// p = A' dx^2 + B' dx dy + C' dy^2 (log2 units), so dalpha/dp = alpha ln 2 and
// dalpha/d(natural-log exponent) = alpha.
__device__ __forceinline__ void finish_row(const float* S, float4 g0, float4 g1, float* G)
{
    const float sig = g1.y;
    const float sl = kLn2 * sig;
    G[0] = sl * fmaf(2.f * g0.z, S[1], g0.w * S[2]);         // mean x
    G[1] = sl * fmaf(2.f * g1.x, S[2], g0.w * S[1]);         // mean y
    G[2] = -0.5f * sig * S[3];                               // conic A, B, C (unscaled)
    G[3] = -sig * S[4];
    G[4] = -0.5f * sig * S[5];
    G[5] = S[0];                                             // opacity
    G[6] = S[6];                                             // colour
    G[7] = S[7];
    G[8] = S[8];
}

__device__ __forceinline__ void bwd_init(const BlendBwdArgs& a, const BlockGeom& g, int32_t len, BwdPix& q)
{
    q.n = 0; q.T = 1.f; q.gCr = q.gCg = q.gCb = q.gh = 0.f;
    if (g.inside) {
        int32_t n = a.n_contrib[g.pix];
        q.n = n < 0 ? 0 : (n > len ? len : n);               // never walk past this tile's list
        q.T = a.T_final[g.pix];
        q.gCr = a.grad_rgb[3 * g.pix + 0];
        q.gCg = a.grad_rgb[3 * g.pix + 1];
        q.gCb = a.grad_rgb[3 * g.pix + 2];
        if (a.grad_H) q.gh = a.grad_H[g.pix];
        if (a.grad_LE) {
            const CamDev& c = a.cams[g.view];
            q.gh += a.grad_LE[g.view] / (float)((int64_t)c.W * c.H);
        }
    }
    q.ghl = q.gh * kLn2;
    q.Q = q.gh * ((logf(q.T) + 1.f) * q.T);                 // gh R_{N+1}, Alg. 1's initialisation
    q.fpx = (float)g.px + 0.5f;
    q.fpy = (float)g.py + 0.5f;
}

// SHARED: the 4 wavefronts of the workgroup are the 4 blocks of one tile and
// share each window; otherwise every wavefront has its own tile and window.
//
// Window records in LDS.  SHARED: two buffers (the next window is loaded while this
// one is walked), each as three arrays of one 16-byte part of every entry (part k of
// entry j at s_rec[buffer][k B + j]), filled straight from global memory by direct
// loads to LDS (global_load_lds_dwordx4: lane l's 16 bytes land at the wavefront's
// LDS base + 16 l), so no register holds a record in flight.  Otherwise: per
// wavefront slot, whole 48-byte entries (entry j at s_rec[slot][3 j]) staged through
// registers.
// 16 bytes per lane from global memory straight into LDS: lane l's land at lds + 16 l
// (lds is the wavefront's base; a device function, so that only the device pass sees
// the builtin)
__device__ __forceinline__ void lds_direct_load16(const float4* src, float4* lds)
{
    __builtin_amdgcn_global_load_lds(src, lds, 16, 0, 0);
}

template <int B, bool SHARED>
struct BwdRecLayout {
    static constexpr int kBytes = SHARED ? (int)sizeof(float4) : (int)sizeof(float4) * kRecF4;  // per entry
    static constexpr int kPart = SHARED ? B : 1;               // float4s between an entry's parts
    __device__ static int idx(int j, int k) { return SHARED ? k * B + j : kRecF4 * j + k; }
};

template <int B, bool SHARED, bool PERSIST>
__global__ __launch_bounds__(256, (SHARED && B <= 64 && !PERSIST) ? 8 : 1) void blend_bwd_kernel(BlendBwdArgs a)
{
    using RL = BwdRecLayout<B, SHARED>;
    constexpr int NS = SHARED ? 1 : kWavesPerGroup;          // LDS slots
    // window entries' records (see above) and emission indices (SHARED: s_rec / s_e hold
    // one buffer, s_rec2 / s_e2 the other; two arrays, so that the compiler sees that
    // the direct loads into one never alias the reads of the other and makes those reads
    // wait for nothing), and, per wavefront, each entry's accumulator row (the 9
    // wavefront sums, then 1 where the wavefront blended it)
    __shared__ float4 s_rec[NS][B * kRecF4];
    __shared__ uint32_t s_e[NS][B];
    __shared__ float4 s_rec2[SHARED ? B * kRecF4 : 1];
    __shared__ uint32_t s_e2[SHARED ? B : 1];
    __shared__ float s_acc[kWavesPerGroup][B * kAccF];   // per-wavefront sums of each window entry
    // surviving window entries of each wavefront, as the offsets of their record
    // (float4 index) and of their accumulator row (float index)
    // surviving entries' record offsets and accumulator offsets, entry k at [.][k + 1]
    // (the same row shape, so that one address serves both; the first slot is never used)
    __shared__ int32_t s_idx[kWavesPerGroup][B + 1];
    __shared__ int32_t s_aidx[kWavesPerGroup][B + 1];
    __shared__ int32_t s_max[kWavesPerGroup];
    __shared__ uint32_t s_item;
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    const uint32_t stamp = *a.stamp;
    const int tcomp = tot_comp(lane);
    // work items: tiles (SHARED: one per workgroup; else one per wavefront), claimed from the per-XCD queues
    const uint32_t n_items = SHARED ? a.n_blocks / kWavesPerGroup : a.n_blocks;
    WaveQueue wq;
    auto next = [&]() -> uint32_t {
        if (!PERSIST) return n_items;
        if (SHARED) {
            __syncthreads();
            if (threadIdx.x == 0) s_item = claim_items(a.queues, n_items, 1u).x;
            __syncthreads();
            return s_item;
        }
        return next_item_wave(wq, a.queues, n_items, lane);
    };
    uint32_t item;
    if (PERSIST) item = next();
    else if (a.tile_order) {                     // hardware dispatch, longest tiles first
        const uint32_t i = SHARED ? blockIdx.x : blockIdx.x * kWavesPerGroup + wid;
        item = i < n_items ? a.tile_order[i] : n_items;
    } else item = SHARED ? blockIdx.x : blockIdx.x * kWavesPerGroup + wid;
    for (; item < n_items; item = next()) {
    const uint32_t tile_id = item;
    const uint32_t wb = SHARED ? tile_id * kWavesPerGroup + wid : tile_id;
    const BlockGeom g = block_geom(a.cams, a.n_views, wb, lane, a.tile_shift_x, a.tile_shift_y, a.spt);
    const uint2 rg = a.ranges[g.tile];
    const int32_t len = (int32_t)(rg.y - rg.x);
    BwdPix q;
    bwd_init(a, g, len, q);
    // wavefront-uniform loop bounds live in scalar registers
    const int32_t wave_n = __builtin_amdgcn_readfirstlane(wave_max_i32(q.n));
    int32_t maxn = wave_n;
    if (SHARED) {
        if (lane == 0) s_max[wid] = wave_n;
        __syncthreads();
        maxn = __builtin_amdgcn_readfirstlane(max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3])));
    }
    const int32_t nthr = SHARED ? 256 : 64;
    const int32_t tid = SHARED ? (int32_t)threadIdx.x : (int32_t)lane;
    // only the hit flags start at zero: a slot's sums are read only where its flag is set
    for (int32_t i = (int32_t)lane; i < B; i += kWave) s_acc[wid][kAccF * i + kG2] = 0.f;
    uint32_t tested = 0;                     // alpha tests (list positions before a pixel's n_contrib)

    // window x covers list positions [lo(x), lo(x) + cnt(x)), from the back
    const int32_t nwin = (maxn + B - 1) / B;
    auto win_lo = [&](int32_t x) { const int32_t l = maxn - (x + 1) * B; return l > 0 ? l : 0; };
    auto win_cnt = [&](int32_t x) { const int32_t c = maxn - x * B; return c < B ? c : B; };
    // per-block: each thread stages entries tid, tid + 64, ... of its wavefront's window
    // through registers; their emission and record indices (two dependent loads) are
    // fetched one window ahead
    constexpr int NW = SHARED ? 1 : (B + kWave - 1) / kWave;
    uint32_t pe[NW], pv[NW];
#pragma unroll
    for (int h = 0; h < NW; ++h) pe[h] = pv[h] = 0u;
    auto fetch_indices = [&](int32_t x) {
        const int32_t lo_x = win_lo(x), cnt_x = win_cnt(x);
#pragma unroll
        for (int h = 0; h < NW; ++h) {
            const int32_t j = tid + h * nthr;
            if (j < cnt_x) {
                pe[h] = a.pair_vals[rg.x + (uint32_t)(lo_x + j)];
                pv[h] = a.emit_vg[pe[h]];
            }
        }
    };
    // SHARED: thread tid < cnt(x) holds entry tid of window x.  A window's records are
    // loaded into the other buffer while the one before it is walked, by direct loads
    // (one instruction per 16-byte part for the wavefront's 64 entries); its record
    // indices one window earlier, its emission indices one earlier again, so that every
    // load waits only at the barrier that ends a window (the wait count of vector memory
    // is in order: a dependent load issued after the direct loads would wait for them).
    // e1, v1: emission and record index of the next window; e2: emission index of the
    // one after.
    uint32_t e1 = 0u, v1 = 0u, e2 = 0u;
    auto load_window = [&](float4* rec_b, uint32_t* e_b, int32_t x) {
        if (tid < win_cnt(x)) {
            const float4* r = a.rec + (size_t)kRecF4 * v1;
            const int w0 = tid & ~(kWave - 1);               // the wavefront's first entry
#pragma unroll
            for (int k = 0; k < kRecF4; ++k) lds_direct_load16(r + k, &rec_b[RL::idx(w0, k)]);
            e_b[tid] = e1;
        }
    };
    // one window: its records and emission indices in rec_w / e_w; SHARED: the next
    // window's go to rec_n / e_n
    auto window = [&](float4* rec_w, uint32_t* e_w, float4* rec_n, uint32_t* e_n, int32_t w) {
        const int32_t lo = win_lo(w);
        const int32_t cnt = win_cnt(w);
        if (SHARED) {
            // (the barrier that ended the last window also ended every read of rec_n)
            if (w + 1 < nwin) load_window(rec_n, e_n, w + 1);
            if (w + 2 < nwin && tid < win_cnt(w + 2)) {
                v1 = a.emit_vg[e2];
                e1 = e2;
            }
            if (w + 3 < nwin && tid < win_cnt(w + 3)) e2 = a.pair_vals[rg.x + (uint32_t)(win_lo(w + 3) + tid)];
        } else {
#pragma unroll
            for (int h = 0; h < NW; ++h) {
                const int32_t j = tid + h * nthr;
                if (j < cnt) {
                    const float4* r = a.rec + (size_t)kRecF4 * pv[h];
                    e_w[j] = pe[h];
                    rec_w[kRecF4 * j + 0] = r[0];
                    rec_w[kRecF4 * j + 1] = r[1];
                    rec_w[kRecF4 * j + 2] = r[2];
                }
            }
            wave_lds_sync();
            if (w + 1 < nwin) fetch_indices(w + 1);
        }
        // this wavefront's surviving entries of the window, in list order
        const int32_t jtop = (wave_n - lo) < cnt ? (wave_n - lo) : cnt;
        int32_t m = 0;
        for (int32_t j0 = 0; j0 < jtop; j0 += kWave) {
            const int32_t j = j0 + (int32_t)lane;
            bool keep = false;
            if (j < jtop)
                keep = !culled(g, rec_w[RL::idx(j, 0)], rec_w[RL::idx(j, 1)].x, rec_w[RL::idx(j, 2)]);
            const uint64_t bal = __ballot(keep);
            if (keep) {
                const int32_t k = m + (int32_t)__popcll(bal & ((1ull << lane) - 1ull));
                s_idx[wid][k + 1] = RL::kBytes * j;
                s_aidx[wid][k + 1] = kAccF * j;
            }
            m += (int32_t)__popcll(bal);
        }
        wave_lds_sync();
        // window entries j < nrel lie in this pixel's list (compared as the byte offset
        // of the entry's record in s_rec)
        const int32_t nrel = RL::kBytes * (q.n - lo);
        // walk them back to front, two entries a step (their offsets read together); per
        // Gaussian, the wavefront sums go to this wavefront's slot
        auto entry = [&](int32_t kk, int32_t j3) {
            const float4* r = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(rec_w) + j3);
            const float4 g1 = r[RL::kPart];
            const BwdAlpha al = bwd_alpha(q, j3, nrel, r[0], g1);
            tested += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(j3 < nrel));
            if (__builtin_amdgcn_ballot_w64(al.act) != 0ull) {   // else no lane of this wavefront blended it
                float o[kG2];
                bwd_grad(q, al, g1, r[2 * RL::kPart].x, o);
                const float tot = wave_sum9<SHARED>(o, lane);
                if (tcomp >= 0) {
                    float* acc = &s_acc[wid][s_aidx[wid][kk + 1]];
                    acc[tcomp] = tot;
                    acc[kG2] = 1.f;                          // (every total's lane writes the same flag)
                }
            }
        };
        int32_t kk = m - 1;
        for (; kk >= 1; kk -= 2) {
            const int32_t oa = s_idx[wid][kk + 1], ob = s_idx[wid][kk];   // entries kk, kk - 1
            entry(kk, oa);
            entry(kk - 1, ob);
        }
        if (kk == 0) entry(0, s_idx[wid][1]);
        if (SHARED) __syncthreads(); else wave_lds_sync();
        // store the rows of the window's blended entries (emission slots),
        // summing the flagged wavefront slots in a fixed order and clearing their flags
        // (a slot without its flag holds stale sums and adds nothing); entries no pixel
        // blended keep no row (their stamp is not this frame's)
        for (int32_t j = tid; j < cnt; j += nthr) {
            constexpr int32_t nsl = SHARED ? kWavesPerGroup : 1;
            const int32_t s0 = SHARED ? 0 : (int32_t)wid;
            bool f[nsl];
            bool hit = false;
#pragma unroll
            for (int32_t r = 0; r < nsl; ++r) {
                f[r] = s_acc[s0 + r][kAccF * j + kG2] != 0.f;
                hit |= f[r];
            }
            if (!hit) continue;
            float S[kG2], G[kG2];
#pragma unroll
            for (int k = 0; k < kG2; ++k) S[k] = 0.f;
#pragma unroll
            for (int32_t r = 0; r < nsl; ++r) {
                if (!f[r]) continue;
                const float* src = &s_acc[s0 + r][kAccF * j];
#pragma unroll
                for (int k = 0; k < kG2; ++k) S[k] += src[k];
                s_acc[s0 + r][kAccF * j + kG2] = 0.f;
            }
            finish_row(S, rec_w[RL::idx(j, 0)], rec_w[RL::idx(j, 1)], G);
            float* row = a.pair_grad + (size_t)kRowF * e_w[j];
#pragma unroll
            for (int k = 0; k < kG2; ++k) row[k] = G[k];
            a.pair_stamp[e_w[j]] = stamp;
        }
        if (SHARED) {
            __builtin_amdgcn_s_waitcnt(0);                   // the next window's direct loads have landed
            __syncthreads();
        } else {
            wave_lds_sync();
        }
    };
    if (SHARED) {
        if (nwin > 0) {
            if (tid < win_cnt(0)) {
                e1 = a.pair_vals[rg.x + (uint32_t)(win_lo(0) + tid)];
                v1 = a.emit_vg[e1];
            }
            load_window(s_rec[0], s_e[0], 0);
        }
        if (nwin > 1 && tid < win_cnt(1)) {
            e1 = a.pair_vals[rg.x + (uint32_t)(win_lo(1) + tid)];
            v1 = a.emit_vg[e1];
        }
        if (nwin > 2 && tid < win_cnt(2)) e2 = a.pair_vals[rg.x + (uint32_t)(win_lo(2) + tid)];
        __builtin_amdgcn_s_waitcnt(0);                       // this thread's direct loads have landed
        __syncthreads();
        // two windows an iteration, so that each buffer is one named array in each
        for (int32_t w = 0; w < nwin; w += 2) {
            window(s_rec[0], s_e[0], s_rec2, s_e2, w);
            if (w + 1 < nwin) window(s_rec2, s_e2, s_rec[0], s_e[0], w + 1);
        }
    } else {
        if (nwin > 0) fetch_indices(0);
        for (int32_t w = 0; w < nwin; ++w) window(s_rec[wid], s_e[wid], nullptr, nullptr, w);
    }
    if (lane == 0) reinterpret_cast<uint32_t*>(a.block_cnt + 2 * wb + 1)[1] = tested;
    }
}

// Debug check of Eq. 9 (GSR_DEBUG_INVARIANTS): the weights of the blended Gaussians and
// the background weight T_final sum to one.  An independent per-pixel walk: one thread
// per pixel re-evaluates its tile's list from the front, with the forward's alpha
// arithmetic, sums the weights of the entries it blends up to the forward's n_contrib,
// and compares sum w + T_final (the forward's) with 1.  Each blended step rounds w and T
// within 2u T_i and the running sum within u per add, so |sum w + T - 1| <= 3u n_contrib;
// the check counts pixels beyond 4u (n_contrib + 1).  Debug speed: uncoalesced walks.
__global__ __launch_bounds__(256) void invariant_kernel(InvArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;   // packed pixel index
    float err = 0.f;
    bool bad = false;
    if (p < a.n_pix) {
        int v = 0;
        while (v + 1 < a.n_views && a.cams[v + 1].pix_base <= p) ++v;
        const CamDev& c = a.cams[v];
        const int64_t q = p - c.pix_base;
        const int px = (int)(q % c.W), py = (int)(q / c.W);
        const uint32_t tile = c.tile_base + (uint32_t)((py >> a.tile_shift_y) * c.gx + (px >> a.tile_shift_x));
        const uint2 rg = a.ranges[tile];
        int32_t n = a.n_contrib[p];
        n = n < 0 ? 0 : (n > (int32_t)(rg.y - rg.x) ? (int32_t)(rg.y - rg.x) : n);
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
        float T = 1.f, S = 0.f;
        for (int32_t i = 0; i < n; ++i) {
            const float4* r = a.rec + (size_t)kRecF4 * a.emit_vg[a.pair_vals[rg.x + (uint32_t)i]];
            const float4 g0 = r[0], g1 = r[1];
            const float alpha =
                fminf(kAlphaMax, g1.y * __builtin_amdgcn_exp2f(gauss_p2(g0.z, g0.w, g1.x, g0.x - fpx, g0.y - fpy)));
            if (alpha < kAlphaMin) continue;
            S = fmaf(alpha, T, S);
            T *= 1.f - alpha;
        }
        err = fabsf(S + a.T_final[p] - 1.f);
        bad = !(err <= 4.f * 5.9604645e-8f * (float)(n + 1));     // NaN counts as a violation
        if (!(err == err)) err = __uint_as_float(0x7f800000u);      // reported as +inf
    }
    const uint32_t nbad = (uint32_t)__popcll(__ballot(bad));
    float m = err;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63u) == 0u) {
        if (nbad) atomicAdd(&a.counters[7], nbad);
        atomicMax(&a.counters[6], __float_as_uint(m));           // non-negative floats order as their bits
    }
}

__device__ __forceinline__ double block_sum_f64(double x)
{
    __shared__ double s[256];
    s[threadIdx.x] = x;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    return s[0];
}

// level 1: one workgroup per chunk of kRedChunk wave blocks of one view
__global__ __launch_bounds__(256) void entropy_chunk_kernel(const float* block_H, const CamDev* cams, int n_views,
                                                            double* chunk_sum)
{
    const uint32_t ch = blockIdx.x;
    int v = 0;
    while (v + 1 < n_views && cams[v + 1].hred_base <= ch) ++v;
    const CamDev& c = cams[v];
    const uint32_t nb = c.n_wblocks;
    const uint32_t b0 = (ch - c.hred_base) * kRedChunk;
    // all loads first (clamped index), then the sum in the same order as a plain loop
    constexpr int kPer = kRedChunk / 256;
    static_assert(kRedChunk % 256 == 0, "whole rounds of 256");
    float hv[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const uint32_t b = b0 + threadIdx.x + 256u * (uint32_t)j;
        hv[j] = block_H[c.block_base + (b < nb ? b : nb - 1u)];
    }
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < kPer; ++j)
        if (b0 + threadIdx.x + 256u * (uint32_t)j < nb) acc += (double)hv[j];
    const double tot = block_sum_f64(acc);
    if (threadIdx.x == 0) chunk_sum[ch] = tot;
}

// level 2: one workgroup per view, L_E = sum of its chunks / (W H)   (Eq. 11)
__global__ __launch_bounds__(256) void entropy_mean_kernel(const double* chunk_sum, const CamDev* cams, int n_views,
                                                           uint32_t n_chunks, float* out)
{
    const int v = blockIdx.x;
    if (v >= n_views) return;
    const CamDev& c = cams[v];
    const uint32_t c0 = c.hred_base, c1 = (v + 1 < n_views) ? cams[v + 1].hred_base : n_chunks;
    double acc = 0.0;
    for (uint32_t k = c0 + threadIdx.x; k < c1; k += 256) acc += chunk_sum[k];
    const double tot = block_sum_f64(acc);
    if (threadIdx.x == 0) out[v] = (float)(tot / ((double)c.W * (double)c.H));
}

// persistent grids: as many workgroups as fit on the device at once
template <typename K>
uint32_t resident_groups(K kernel, uint32_t want)
{
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0);
    uint32_t g = (uint32_t)(cus > 0 ? cus : 256) * (uint32_t)(per_cu > 0 ? per_cu : 1);
    return g < want ? g : want;
}

template <int B, bool RENDER>
hipError_t fwd_launch(const BlendFwdArgs& a, hipStream_t s)
{
    const uint32_t groups = (a.n_blocks + kWavesPerGroup - 1) / kWavesPerGroup;
    if (a.spt == 4 && a.shared_batches) {  // one tile per workgroup, batches shared by its 4 blocks
        if (a.queues)
            hipLaunchKernelGGL((blend_fwd_shared_kernel<B, true, RENDER>),
                               dim3(resident_groups(blend_fwd_shared_kernel<B, true, RENDER>, groups)), dim3(256), 0,
                               s, a);
        else
            hipLaunchKernelGGL((blend_fwd_shared_kernel<B, false, RENDER>), dim3(groups), dim3(256), 0, s, a);
    } else {                               // one 8x8 block per wavefront, its own batches
        if (a.queues)
            hipLaunchKernelGGL((blend_fwd_kernel<B, true, RENDER>),
                               dim3(resident_groups(blend_fwd_kernel<B, true, RENDER>, groups)), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((blend_fwd_kernel<B, false, RENDER>), dim3(groups), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

template <int B>
hipError_t fwd_b(const BlendFwdArgs& a, hipStream_t s)
{
    return a.render_only ? fwd_launch<B, true>(a, s) : fwd_launch<B, false>(a, s);
}

template <int B>
hipError_t bwd_b(const BlendBwdArgs& a, hipStream_t s)
{
    static_assert(B <= 128, "the backward window is limited by LDS");
    const uint32_t groups = (a.n_blocks + kWavesPerGroup - 1) / kWavesPerGroup;
    if (a.queues) {
        if (a.spt == 4)
            hipLaunchKernelGGL((blend_bwd_kernel<B, true, true>),
                               dim3(resident_groups(blend_bwd_kernel<B, true, true>, groups)), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((blend_bwd_kernel<B, false, true>),
                               dim3(resident_groups(blend_bwd_kernel<B, false, true>, groups)), dim3(256), 0, s, a);
    } else {
        if (a.spt == 4) hipLaunchKernelGGL((blend_bwd_kernel<B, true, false>), dim3(groups), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((blend_bwd_kernel<B, false, false>), dim3(groups), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_blend_fwd(const BlendFwdArgs& a, int lds_batch, hipStream_t s)
{
    if (a.n_blocks == 0) return hipSuccess;
    switch (lds_batch) {
        case 32: return fwd_b<32>(a, s);
        case 64: return fwd_b<64>(a, s);
        case 128: return fwd_b<128>(a, s);
        case 256: return fwd_b<256>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_blend_bwd(const BlendBwdArgs& a, int lds_batch, hipStream_t s)
{
    if (a.n_blocks == 0) return hipSuccess;
    switch (lds_batch) {
        case 32: return bwd_b<32>(a, s);
        case 64: return bwd_b<64>(a, s);
        case 128: return bwd_b<128>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_invariants(const InvArgs& a, hipStream_t s)
{
    if (a.n_pix <= 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)((a.n_pix + 255) / 256);
    hipLaunchKernelGGL(invariant_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_entropy_mean(const float* block_H, const CamDev* cams, int n_views, uint32_t n_chunks,
                               double* tmp, float* out, hipStream_t s)
{
    if (n_views == 0 || n_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(entropy_chunk_kernel, dim3(n_chunks), dim3(256), 0, s, block_H, cams, n_views, tmp);
    hipLaunchKernelGGL(entropy_mean_kernel, dim3(n_views), dim3(256), 0, s, tmp, cams, n_views, n_chunks, out);
    return hipGetLastError();
}

}  // namespace gsr
