// Tile binning (prefix sum + key duplication), the stable LSD radix sort and
// per-tile range extraction.
//
// Lists are ordered by the 64-bit key (tile | float32 depth bits), ties by
// Gaussian index.  Because every copy of a Gaussian carries the same depth,
// the LSD passes over the depth digits are run once per (view, Gaussian)
// before duplication (4 passes over V*n items), and only the tile digits are
// sorted over the duplicated pairs (2-3 passes over P items).  The result is
// exactly the LSD radix sort of the full key: duplication emits pairs in
// depth-sorted Gaussian order and the tile passes are stable.
#include "internal.h"

namespace gsr {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTileItems = kThreads * kItems;     // 2048 items per block
constexpr int kBins = 256;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// inclusive prefix sum over a 64-wide wavefront
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    return x;
}

// exclusive scan over the 256 threads of a block; returns the block total in *total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* total)
{
    __shared__ uint32_t s_wave[kThreads / 64];
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(x);
    if (lane == 63) s_wave[wid] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        uint32_t v = s_wave[w];
        base += (w < (int)wid) ? v : 0u;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return base + inc - x;
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan (reduce, spine, downsweep) of vals[order[i]].
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const uint32_t* vals, const uint32_t* order, uint32_t n,
                                                               uint32_t* partial)
{
    size_t base = (size_t)blockIdx.x * kTileItems + (size_t)threadIdx.x * kItems;
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        size_t idx = base + k;
        if (idx < n) sum += vals[order ? order[idx] : idx];
    }
    uint32_t tot;
    block_excl_scan(sum, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// single block: exclusive scan of partial[0..nb) in place; total and 32-bit overflow flag
__global__ __launch_bounds__(kThreads) void scan_spine_kernel(uint32_t* partial, uint32_t nb, uint32_t* total,
                                                              uint32_t* overflow)
{
    __shared__ unsigned long long s_carry;
    if (threadIdx.x == 0) s_carry = 0ull;
    __syncthreads();
    for (uint32_t start = 0; start < nb; start += kThreads) {
        uint32_t idx = start + threadIdx.x;
        uint32_t v = idx < nb ? partial[idx] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, &tot);
        unsigned long long carry = s_carry;
        if (idx < nb) partial[idx] = (uint32_t)(carry + ex);
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsigned long long c = s_carry;
        *total = c > 0xffffffffull ? 0xffffffffu : (uint32_t)c;
        if (c > 0xffffffffull) *overflow = 1u;
    }
}

__global__ __launch_bounds__(kThreads) void scan_down_kernel(const uint32_t* vals, const uint32_t* order, uint32_t n,
                                                             const uint32_t* partial, uint32_t* out)
{
    size_t base = (size_t)blockIdx.x * kTileItems + (size_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        size_t idx = base + k;
        v[k] = idx < n ? vals[order ? order[idx] : idx] : 0u;
        sum += v[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(sum, &tot) + partial[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        size_t idx = base + k;
        if (idx < n) out[idx] = run;
        run += v[k];
    }
}

// ---------------------------------------------------------------------------
// Stable LSD radix pass, 8-bit digits:
//   upsweep   per-block digit histograms, digit-major  hist[d * nb + b]
//   spine     one block per digit: exclusive scan of its row; row total
//   downsweep stable block-local ranking (wavefront match via ballots),
//             reorder through LDS, coalesced scatter
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t item_count(const uint32_t* n_dev, uint32_t n_max)
{
    if (!n_dev) return n_max;
    uint32_t n = *n_dev;
    return n < n_max ? n : n_max;
}

__global__ __launch_bounds__(kThreads) void radix_upsweep_kernel(const uint32_t* keys, const uint32_t* n_dev,
                                                                 uint32_t n_max, int shift, uint32_t* hist, uint32_t nb)
{
    __shared__ uint32_t s_h[kBins];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t n = item_count(n_dev, n_max);
    size_t base = (size_t)blockIdx.x * kTileItems;
    if (base < n) {
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            size_t idx = base + (size_t)k * kThreads + threadIdx.x;
            if (idx < n) atomicAdd(&s_h[(keys[idx] >> shift) & 0xffu], 1u);
        }
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nb + blockIdx.x] = s_h[threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void radix_spine_kernel(uint32_t* hist, uint32_t nb, uint32_t* digit_total)
{
    __shared__ unsigned int s_carry;
    uint32_t* row = hist + (size_t)blockIdx.x * nb;
    if (threadIdx.x == 0) s_carry = 0u;
    __syncthreads();
    for (uint32_t start = 0; start < nb; start += kThreads) {
        uint32_t idx = start + threadIdx.x;
        uint32_t v = idx < nb ? row[idx] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, &tot);
        uint32_t carry = s_carry;
        if (idx < nb) row[idx] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) digit_total[blockIdx.x] = s_carry;
}

__global__ __launch_bounds__(kThreads) void radix_downsweep_kernel(const uint32_t* keys_in, const uint32_t* vals_in,
                                                                   uint32_t* keys_out, uint32_t* vals_out,
                                                                   const uint32_t* n_dev, uint32_t n_max, int shift,
                                                                   const uint32_t* hist, uint32_t nb,
                                                                   const uint32_t* digit_total)
{
    __shared__ uint32_t s_keys[kTileItems];
    __shared__ uint32_t s_vals[kTileItems];
    __shared__ uint32_t s_gofs[kBins];        // global start of digit d for this block
    __shared__ uint32_t s_lofs[kBins];        // block-local start of digit d
    __shared__ uint32_t s_run[kBins];         // items of digit d already placed
    __shared__ uint32_t s_wcnt[kThreads / 64][kBins];

    const uint32_t n = item_count(n_dev, n_max);
    const size_t base = (size_t)blockIdx.x * kTileItems;
    if (base >= n) return;                    // whole block leaves together
    const uint32_t tid = threadIdx.x, lane = lane_id(), wid = tid >> 6;
    const uint32_t cnt = (uint32_t)((n - base) < (size_t)kTileItems ? (n - base) : (size_t)kTileItems);

    // global offsets: exclusive prefix of the digit totals + this block's row offset
    uint32_t tot;
    uint32_t dbase = block_excl_scan(digit_total[tid], &tot);
    s_gofs[tid] = dbase + hist[(size_t)tid * nb + blockIdx.x];

    // load this block's keys (round-major: round r, thread t -> item r*256 + t)
    uint32_t k_[kItems], v_[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        uint32_t li = (uint32_t)r * kThreads + tid;
        bool ok = li < cnt;
        k_[r] = ok ? keys_in[base + li] : 0xffffffffu;
        v_[r] = ok ? vals_in[base + li] : 0u;
    }
    // block-local digit histogram -> local starts
    s_run[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        uint32_t li = (uint32_t)r * kThreads + tid;
        if (li < cnt) atomicAdd(&s_run[(k_[r] >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    uint32_t lstart = block_excl_scan(s_run[tid], &tot);
    s_lofs[tid] = lstart;
    s_run[tid] = 0;
    __syncthreads();

    const uint64_t lt_mask = (1ull << lane) - 1ull;
    for (int r = 0; r < kItems; ++r) {
        uint32_t li = (uint32_t)r * kThreads + tid;
        bool ok = li < cnt;
        uint32_t d = (k_[r] >> shift) & 0xffu;
        // peers: lanes of this wavefront holding the same digit
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        uint32_t rank = __popcll(peers & lt_mask);
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) s_wcnt[w][tid] = 0;
        __syncthreads();
        if (ok && rank == 0) s_wcnt[wid][d] = __popcll(peers);
        __syncthreads();
        {   // thread tid owns digit tid: wave offsets in wave order
            uint32_t c = s_run[tid];
#pragma unroll
            for (int w = 0; w < kThreads / 64; ++w) {
                uint32_t t = s_wcnt[w][tid];
                s_wcnt[w][tid] = c;
                c += t;
            }
            s_run[tid] = c;
        }
        __syncthreads();
        if (ok) {
            uint32_t pos = s_lofs[d] + s_wcnt[wid][d] + rank;
            s_keys[pos] = k_[r];
            s_vals[pos] = v_[r];
        }
        __syncthreads();
    }
    // coalesced scatter of the locally sorted block
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        uint32_t li = (uint32_t)r * kThreads + tid;
        if (li < cnt) {
            uint32_t k = s_keys[li];
            uint32_t d = (k >> shift) & 0xffu;
            uint32_t o = s_gofs[d] + (li - s_lofs[d]);
            keys_out[o] = k;
            vals_out[o] = s_vals[li];
        }
    }
}

// ---------------------------------------------------------------------------
// Duplication: every (view, Gaussian) in depth order writes one pair per tile
// of its rectangle, row-major, at its scanned offset.  The pair's value is the
// (view, Gaussian) record index; emit_vg[emission index] holds it too.  All
// pairs of one Gaussian are contiguous in emission order, which the backward
// uses to reduce per-pair gradients without atomics: the pair of local tile
// (tx, ty) has emission index base + ty w + tx (mod 2^32), with
// base = offset - y0 w - x0 and w = x1 - x0 + 1 stored in the record's last
// two words.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void duplicate_kernel(const uint32_t* order, const uint32_t* offsets,
                                                             const uint32_t* tiles_touched, const uint2* rect,
                                                             const CamDev* cams, uint32_t n, uint32_t vn,
                                                             const uint32_t* total, uint32_t cap, uint32_t* keys,
                                                             uint32_t* vals, uint32_t* emit_vg, uint32_t* overflow,
                                                             float4* rec)
{
    uint32_t s = blockIdx.x * kThreads + threadIdx.x;
    if (s == 0 && *total > cap) *overflow = 1u;
    if (s >= vn) return;
    uint32_t vg = order[s];
    uint32_t tt = tiles_touched[vg];
    if (tt == 0) return;
    uint32_t off = offsets[s];
    uint2 rc = rect[vg];
    uint32_t v = vg / n;
    const uint32_t gx = (uint32_t)cams[v].gx, tb = cams[v].tile_base;
    uint32_t x0 = rc.x & 0xffffu, x1 = rc.x >> 16, y0 = rc.y & 0xffffu, y1 = rc.y >> 16;
    const uint32_t w = x1 - x0 + 1u;
    float4* r2 = rec + (size_t)kRecF4 * vg + 2;
    r2->z = __uint_as_float(off - y0 * w - x0);
    r2->w = __uint_as_float(w);
    for (uint32_t ty = y0; ty <= y1; ++ty)
        for (uint32_t tx = x0; tx <= x1; ++tx) {
            if (off < cap) {
                keys[off] = tb + ty * gx + tx;
                vals[off] = vg;
                emit_vg[off] = vg;
            }
            ++off;
        }
}

// Per-Gaussian sum of the per-pair gradient rows.  Rows (9 floats and a stamp)
// are stored in emission order, where all pairs of one (view, Gaussian) are
// contiguous; a row whose stamp is not this backward's was not written by it
// (no pixel blended that pair) and counts as zero.  One wavefront takes 64
// consecutive rows, runs a segmented inclusive scan keyed by the Gaussian,
// and writes every segment that starts and ends inside it; segments that
// cross wavefront boundaries leave their partial sums in `carry` and are
// finished by seg_fixup_kernel in a fixed order.  No atomics: deterministic.
struct SegCarry {
    float head[kG2];         // first segment's sum over this wavefront, if it started earlier and ends here
    float tail[kG2];         // last segment's sum over this wavefront, if it continues past it
    uint32_t first_seg, last_seg;
    uint32_t flags;          // 1: first segment started earlier; 2: last segment continues
    uint32_t pad;
};

__global__ __launch_bounds__(kThreads) void seg_reduce_kernel(const float* pair_grad, const uint32_t* stamp,
                                                              const uint32_t* emit_vg, const uint32_t* total,
                                                              uint32_t cap, float* grad2d, SegCarry* carry)
{
    const uint32_t P = *total < cap ? *total : cap;
    const uint32_t st = *stamp;
    const uint32_t lane = lane_id();
    const uint32_t w = (blockIdx.x * kThreads + threadIdx.x) >> 6;
    const uint32_t e = w * 64u + lane;
    if (w * 64u >= P) return;                                  // whole wavefront
    const bool valid = e < P;
    const uint32_t seg = valid ? emit_vg[e] : 0xffffffffu;
    uint32_t prev = __shfl_up(seg, 1, 64);
    if (lane == 0) prev = e > 0 ? emit_vg[e - 1] : 0xfffffffeu;
    uint32_t next = __shfl_down(seg, 1, 64);
    if (lane == 63) next = (e + 1 < P) ? emit_vg[e + 1] : 0xfffffffeu;
    float v[kG2];
#pragma unroll
    for (int k = 0; k < kG2; ++k) v[k] = 0.f;
    if (valid) {
        const float* row = pair_grad + (size_t)kRowF * e;
        if (__float_as_uint(row[kG2]) == st) {
#pragma unroll
            for (int k = 0; k < kG2; ++k) v[k] = row[k];
        }
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t su = __shfl_up(seg, d, 64);
        const bool same = lane >= (uint32_t)d && su == seg;    // segments are contiguous
#pragma unroll
        for (int k = 0; k < kG2; ++k) {
            const float y = __shfl_up(v[k], d, 64);
            v[k] += same ? y : 0.f;
        }
    }
    const uint32_t first_seg = __shfl(seg, 0, 64);
    const bool crosses_in = __shfl(prev, 0, 64) == first_seg;  // first segment began in an earlier wavefront
    const bool from_before = crosses_in && seg == first_seg;
    const bool ends_here = valid && next != seg;
    const bool last_valid = valid && (lane == 63 || e + 1 >= P);
    if (ends_here && !from_before) {
        float* dst = grad2d + (size_t)kG2 * seg;
#pragma unroll
        for (int k = 0; k < kG2; ++k) dst[k] = v[k];
    }
    SegCarry* c = carry + w;
    if (ends_here && from_before) {
#pragma unroll
        for (int k = 0; k < kG2; ++k) c->head[k] = v[k];
    }
    if (last_valid) {
        const bool crosses_out = !ends_here;
#pragma unroll
        for (int k = 0; k < kG2; ++k) c->tail[k] = crosses_out ? v[k] : 0.f;
        c->first_seg = first_seg;
        c->last_seg = seg;
        c->flags = (crosses_in ? 1u : 0u) | (crosses_out ? 2u : 0u);
    }
}

// one thread per wavefront: a segment that starts in wavefront w and continues
// past it is summed here over the following wavefronts, in order
__global__ __launch_bounds__(kThreads) void seg_fixup_kernel(const SegCarry* carry, const uint32_t* total,
                                                             uint32_t cap, float* grad2d)
{
    const uint32_t P = *total < cap ? *total : cap;
    const uint32_t nw = (P + 63u) / 64u;
    const uint32_t w = blockIdx.x * kThreads + threadIdx.x;
    if (w >= nw) return;
    const SegCarry& c = carry[w];
    if (!(c.flags & 2u)) return;                                 // nothing continues past w
    if ((c.flags & 1u) && c.first_seg == c.last_seg) return;     // w is inside a segment begun earlier
    const uint32_t s = c.last_seg;
    float acc[kG2];
#pragma unroll
    for (int k = 0; k < kG2; ++k) acc[k] = c.tail[k];
    for (uint32_t u = w + 1; u < nw; ++u) {
        const SegCarry& d = carry[u];
        const bool whole = (d.flags & 3u) == 3u && d.first_seg == d.last_seg && d.first_seg == s;
        if (whole) {
#pragma unroll
            for (int k = 0; k < kG2; ++k) acc[k] += d.tail[k];
            continue;
        }
#pragma unroll
        for (int k = 0; k < kG2; ++k) acc[k] += d.head[k];
        break;
    }
    float* dst = grad2d + (size_t)kG2 * s;
#pragma unroll
    for (int k = 0; k < kG2; ++k) dst[k] = acc[k];
}

__global__ void tile_len_keys_kernel(const uint2* ranges, uint32_t n_tiles, uint32_t* keys, uint32_t* vals)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const uint2 r = ranges[t];
    const uint32_t len = r.y > r.x ? r.y - r.x : 0u;
    const uint32_t b = (len + 7u) / 8u;
    keys[t] = 255u - (b < 255u ? b : 255u);
    vals[t] = t;
}

__global__ void iota_u32_kernel(uint32_t* p, uint32_t count)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = i;
}

__global__ void bump_u32_kernel(uint32_t* p)
{
    if (threadIdx.x == 0) *p += 1u;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t value, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

__global__ __launch_bounds__(kThreads) void ranges_kernel(const uint32_t* tiles, const uint32_t* total, uint32_t cap,
                                                          uint2* ranges)
{
    uint32_t P = *total < cap ? *total : cap;
    uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= P) return;
    uint32_t t = tiles[i];
    if (i == 0 || tiles[i - 1] != t) ranges[t].x = i;
    if (i == P - 1 || tiles[i + 1] != t) ranges[t].y = i + 1;
}


}  // namespace

size_t scan_tmp_words(uint32_t n) { return (size_t)(n + kTileItems - 1) / kTileItems + 1; }

hipError_t launch_gather_scan(const uint32_t* vals, const uint32_t* order, uint32_t n, uint32_t* out, uint32_t* total,
                              uint32_t* overflow, uint32_t* tmp, hipStream_t s)
{
    uint32_t nb = (n + kTileItems - 1) / kTileItems;
    if (nb > 0) hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb), dim3(kThreads), 0, s, vals, order, n, tmp);
    hipLaunchKernelGGL(scan_spine_kernel, dim3(1), dim3(kThreads), 0, s, tmp, nb, total, overflow);
    if (nb > 0) hipLaunchKernelGGL(scan_down_kernel, dim3(nb), dim3(kThreads), 0, s, vals, order, n, tmp, out);
    return hipGetLastError();
}

size_t radix_tmp_words(uint32_t n_max)
{
    size_t nb = (n_max + kTileItems - 1) / kTileItems;
    return (size_t)kBins * (nb > 0 ? nb : 1) + kBins;
}

hipError_t launch_radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out,
                             const uint32_t* n_dev, uint32_t n_max, int shift, uint32_t* tmp, hipStream_t s)
{
    uint32_t nb = (n_max + kTileItems - 1) / kTileItems;
    if (nb == 0) return hipSuccess;
    uint32_t* hist = tmp;
    uint32_t* digit_total = tmp + (size_t)kBins * nb;
    hipLaunchKernelGGL(radix_upsweep_kernel, dim3(nb), dim3(kThreads), 0, s, keys_in, n_dev, n_max, shift, hist, nb);
    hipLaunchKernelGGL(radix_spine_kernel, dim3(kBins), dim3(kThreads), 0, s, hist, nb, digit_total);
    hipLaunchKernelGGL(radix_downsweep_kernel, dim3(nb), dim3(kThreads), 0, s, keys_in, vals_in, keys_out, vals_out,
                       n_dev, n_max, shift, hist, nb, digit_total);
    return hipGetLastError();
}

hipError_t launch_duplicate(const uint32_t* order, const uint32_t* offsets, const uint32_t* tiles_touched,
                            const uint2* rect, const CamDev* cams, uint32_t n, uint32_t vn, const uint32_t* total,
                            uint32_t cap, uint32_t* keys, uint32_t* vals, uint32_t* emit_vg, uint32_t* overflow,
                            float4* rec, hipStream_t s)
{
    if (vn == 0) return hipSuccess;
    hipLaunchKernelGGL(duplicate_kernel, dim3((vn + kThreads - 1) / kThreads), dim3(kThreads), 0, s, order, offsets,
                       tiles_touched, rect, cams, n, vn, total, cap, keys, vals, emit_vg, overflow, rec);
    return hipGetLastError();
}

size_t seg_carry_bytes(uint32_t cap) { return ((size_t)cap + 63) / 64 * sizeof(SegCarry) + sizeof(SegCarry); }

hipError_t launch_grad_reduce(const float* pair_grad, const uint32_t* stamp, const uint32_t* emit_vg, uint32_t vn,
                              const uint32_t* total, uint32_t cap, float* grad2d, void* carry, hipStream_t s)
{
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(grad2d), 0u, (size_t)vn * kG2, s);
    if (e != hipSuccess || cap == 0) return e;
    const uint32_t nw = (cap + 63) / 64;
    hipLaunchKernelGGL(seg_reduce_kernel, dim3((nw * 64 + kThreads - 1) / kThreads), dim3(kThreads), 0, s, pair_grad,
                       stamp, emit_vg, total, cap, grad2d, reinterpret_cast<SegCarry*>(carry));
    hipLaunchKernelGGL(seg_fixup_kernel, dim3((nw + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                       reinterpret_cast<const SegCarry*>(carry), total, cap, grad2d);
    return hipGetLastError();
}

hipError_t launch_iota_u32(uint32_t* p, uint32_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(iota_u32_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_tile_len_keys(const uint2* ranges, uint32_t n_tiles, uint32_t* keys, uint32_t* vals, hipStream_t s)
{
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(tile_len_keys_kernel, dim3((n_tiles + 255) / 256), dim3(256), 0, s, ranges, n_tiles, keys, vals);
    return hipGetLastError();
}

hipError_t launch_bump_u32(uint32_t* p, hipStream_t s)
{
    hipLaunchKernelGGL(bump_u32_kernel, dim3(1), dim3(64), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, value, count);
    return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* tiles, const uint32_t* total, uint32_t cap, uint2* ranges, hipStream_t s)
{
    if (cap == 0) return hipSuccess;
    hipLaunchKernelGGL(ranges_kernel, dim3((cap + kThreads - 1) / kThreads), dim3(kThreads), 0, s, tiles, total, cap,
                       ranges);
    return hipGetLastError();
}


}  // namespace gsr
