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
// Device-wide exclusive scan (reduce, spine, downsweep) of the tiles touched
// taken in depth order.  The reduce step gathers each record's tile rectangle
// with one 8-byte load into depth order (rect_s, and its tile count in vals_s),
// so the downsweep and the duplication read them coalesced.  (With the count in
// a 16-byte word the gathered array was 384 MB on the 8-view workload; at 8
// bytes it is half that, within the chip's 256 MB last-level cache.)
// ---------------------------------------------------------------------------

// tiles in the inclusive tile rectangle (x0 | x1 << 16, y0 | y1 << 16); 0 when x1 < x0
__device__ __forceinline__ uint32_t rect_tiles(uint2 r)
{
    const uint32_t w = (r.x >> 16) - (r.x & 0xffffu) + 1u, h = (r.y >> 16) - (r.y & 0xffffu) + 1u;
    return w * h;
}

__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const uint2* trect, const uint32_t* order, uint32_t n,
                                                               uint32_t* partial, uint32_t* vals_s, uint2* rect_s)
{
    size_t base = (size_t)blockIdx.x * kTileItems + threadIdx.x;
    uint32_t sum = 0;
    // the kItems order loads, then the kItems gathers, each batch in flight together
    // (a clamped index instead of a branch; items past the end are not stored or summed)
    uint32_t o[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const size_t idx = base + (size_t)k * kThreads;
        o[k] = order[idx < n ? idx : (size_t)n - 1];
    }
    uint2 t[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) t[k] = trect[o[k]];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const size_t idx = base + (size_t)k * kThreads;
        if (idx < n) {
            const uint32_t tt = rect_tiles(t[k]);
            vals_s[idx] = tt;
            rect_s[idx] = t[k];
            sum += tt;
        }
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

// SELF (at most kThreads blocks): partial holds the raw block sums; each block adds
// up those before it itself, and the last block writes the total (no spine kernel)
template <bool SELF>
__global__ __launch_bounds__(kThreads) void scan_down_kernel(const uint32_t* vals_s, uint32_t n,
                                                             const uint32_t* partial, uint32_t nb, uint32_t* out,
                                                             uint32_t* total, uint32_t* overflow)
{
    uint32_t bpre;
    if (SELF) {
        __shared__ unsigned long long s_w[kThreads / 64];
        unsigned long long x = threadIdx.x < blockIdx.x ? (unsigned long long)partial[threadIdx.x] : 0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if ((threadIdx.x & 63u) == 0u) s_w[threadIdx.x >> 6] = x;
        __syncthreads();
        unsigned long long pre = 0ull;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) pre += s_w[w];
        bpre = (uint32_t)pre;
        if (blockIdx.x == nb - 1u && threadIdx.x == 0) {
            const unsigned long long c = pre + partial[blockIdx.x];
            *total = c > 0xffffffffull ? 0xffffffffu : (uint32_t)c;
            if (c > 0xffffffffull) *overflow = 1u;
        }
    } else {
        bpre = partial[blockIdx.x];
    }
    // kItems consecutive counts a thread, as two 16-byte words where all are in range
    static_assert(kItems == 8, "two 16-byte words a thread");
    const size_t base = (size_t)blockIdx.x * kTileItems + (size_t)threadIdx.x * kItems;
    const bool whole = base + kItems <= n;
    uint32_t v[kItems];
    uint32_t sum = 0;
    if (whole) {
        const uint4 a = reinterpret_cast<const uint4*>(vals_s + base)[0];
        const uint4 b = reinterpret_cast<const uint4*>(vals_s + base)[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k) v[k] = base + k < n ? vals_s[base + k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) sum += v[k];
    uint32_t tot;
    uint32_t run = block_excl_scan(sum, &tot) + bpre;
    uint32_t o[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        o[k] = run;
        run += v[k];
    }
    if (whole) {
        reinterpret_cast<uint4*>(out + base)[0] = make_uint4(o[0], o[1], o[2], o[3]);
        reinterpret_cast<uint4*>(out + base)[1] = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (base + k < n) out[base + k] = o[k];
    }
}

// ---------------------------------------------------------------------------
// Stable LSD radix pass, 8-bit digits, 256 threads x ITEMS items per block
// (32 for large inputs, 8 below 2^21 items so that small sorts still fill the chip;
// 8,192 items a block scatter runs of 32 items a digit on average, 128 bytes of keys:
// on the 8-view workload the two tile passes take about 1.4 ms, 1.7 ms at 16 items):
//   upsweep   per-block digit histograms, block-major  hist[b * 256 + d] (one
//             coalesced 1 KB store a block, and one 1 KB load in the downsweep)
//   spine     one block per 4 digits: exclusive scan of their columns over the
//             blocks that hold items; column totals (a pass of at most
//             kSelfSpineBlocks blocks has no spine: each downsweep block sums the
//             counts of the blocks before it itself)
//   downsweep each wavefront ranks its 64 x ITEMS consecutive items (ITEMS rounds
//             of 64, peers found with 8 ballots, running per-digit counts in
//             LDS); one block scan turns the (digit, wavefront) counts into
//             block-local starts; reorder through LDS; coalesced scatter; blocks
//             take their data blocks in XCD-aware order (xcd_block)
// ---------------------------------------------------------------------------

constexpr int kRadixSmallItems = 8;
constexpr int kRadixLargeItems = 32;
constexpr uint32_t kRadixLargeFrom = 1u << 21;
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kSelfSpineBlocks = 128;

__host__ __device__ constexpr uint32_t radix_items(uint32_t n_max)
{
    return n_max >= kRadixLargeFrom ? kRadixLargeItems : kRadixSmallItems;
}

__device__ __forceinline__ uint32_t item_count(const uint32_t* n_dev, uint32_t n_max)
{
    if (!n_dev) return n_max;
    uint32_t n = *n_dev;
    return n < n_max ? n : n_max;
}

__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int ITEMS>
__global__ __launch_bounds__(kThreads) void radix_upsweep_kernel(const uint32_t* keys, const uint32_t* n_dev,
                                                                 uint32_t n_max, int shift, uint32_t* hist)
{
    constexpr int kRadixTile = kThreads * ITEMS;
    __shared__ uint32_t s_h[kBins];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t n = item_count(n_dev, n_max);
    size_t base = (size_t)blockIdx.x * kRadixTile;
    if (base < n) {
        // a wavefront takes 64 consecutive keys a round; a run of equal digits in
        // neighbouring lanes adds its length with one atomic, from its first lane
        // (sorted tile keys come in long runs, which would otherwise serialise on
        // one LDS address)
        const uint32_t lane = lane_id();
        // all ITEMS loads first, then the counting rounds.  A full block (all but the
        // last) loads without guards (one address, the rest immediate offsets); the last
        // loads with a clamped index instead of a branch, so that its loads are in flight
        // together too
        const bool full = base + kRadixTile <= n;
        const uint32_t cnt = full ? (uint32_t)kRadixTile : (uint32_t)(n - base);
        uint32_t kv[ITEMS];
        if (full) {
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) kv[k] = keys[base + (size_t)k * kThreads + threadIdx.x];
        } else {
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const size_t idx = base + (size_t)k * kThreads + threadIdx.x;
                kv[k] = keys[idx < n ? idx : (size_t)n - 1];
            }
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const bool ok = (uint32_t)k * kThreads + threadIdx.x < cnt;
            const uint32_t d = ok ? (kv[k] >> shift) & 0xffu : kBins;
            // the previous lane's digit by a DPP wave shift (lane 0 takes a value no digit has)
            const uint32_t prv = (uint32_t)__builtin_amdgcn_update_dpp((int)0xffffffffu, (int)d, 0x138, 0xf, 0xf, false);
            const bool lead = ok && prv != d;
            const uint64_t leaders = __builtin_amdgcn_ballot_w64(lead);
            const uint32_t nvalid = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(ok));    // valid lanes are a prefix
            if (lead) {
                const uint64_t later = leaders & ~((2ull << lane) - 1ull);    // leaders above this lane (none for lane 63)
                const uint32_t end = later ? (uint32_t)__builtin_ctzll(later) : nvalid;
                atomicAdd(&s_h[d], end - lane);
            }
        }
    }
    __syncthreads();
    hist[(size_t)blockIdx.x * kBins + threadIdx.x] = s_h[threadIdx.x];
}

// exclusive scan of four counts at once over the 256 threads of a block (the
// per-component form of block_excl_scan); returns the block totals in *total
__device__ __forceinline__ uint4 block_excl_scan4(uint4 x, uint4* total)
{
    __shared__ uint4 s_wave4[kThreads / 64];
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
    uint4 inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t yx = __shfl_up(inc.x, o, 64), yy = __shfl_up(inc.y, o, 64);
        const uint32_t yz = __shfl_up(inc.z, o, 64), yw = __shfl_up(inc.w, o, 64);
        if (lane >= (uint32_t)o) { inc.x += yx; inc.y += yy; inc.z += yz; inc.w += yw; }
    }
    if (lane == 63) s_wave4[wid] = inc;
    __syncthreads();
    uint4 base = make_uint4(0u, 0u, 0u, 0u), tot = base;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        const uint4 v = s_wave4[w];
        if (w < (int)wid) { base.x += v.x; base.y += v.y; base.z += v.z; base.w += v.w; }
        tot.x += v.x; tot.y += v.y; tot.z += v.z; tot.w += v.w;
    }
    __syncthreads();
    *total = tot;
    return make_uint4(base.x + inc.x - x.x, base.y + inc.y - x.y, base.z + inc.z - x.z, base.w + inc.w - x.w);
}

// One workgroup per 4 digits: exclusive scan of their columns of the count rows
// (one 16-byte word a row), column totals.  Only the rows of blocks that hold
// items are scanned (a grid sized for a larger capacity leaves the others zero and
// the downsweep does not read them).  Workgroups are dealt to the 8 XCDs
// round-robin: XCD x takes digits [32 x, 32 x + 32), so the 8 workgroups reading
// one 128-byte line of a count row share that XCD's L2.
template <uint32_t kSpineItems>
__global__ __launch_bounds__(kThreads) void radix_spine_kernel(uint32_t* hist, const uint32_t* n_dev, uint32_t n_max,
                                                               uint32_t tile, uint32_t* digit_total)
{
    __shared__ uint4 s_carry;
    const uint32_t g = (blockIdx.x & 7u) * (uint32_t)(kBins / 32) + (blockIdx.x >> 3);
    uint4* col = reinterpret_cast<uint4*>(hist) + g;         // digits 4 g .. 4 g + 3 of row b: col[b * kBins / 4]
    const uint32_t n = item_count(n_dev, n_max);
    const uint32_t nb = (uint32_t)(((size_t)n + tile - 1) / tile);
    if (threadIdx.x == 0) s_carry = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    // kSpineItems consecutive rows a thread: one block scan per kThreads * kSpineItems
    for (uint32_t start = 0; start < nb; start += kThreads * kSpineItems) {
        const uint32_t i0 = start + threadIdx.x * kSpineItems;
        uint4 v[kSpineItems], sum = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (uint32_t j = 0; j < kSpineItems; ++j) {
            v[j] = i0 + j < nb ? col[(size_t)(i0 + j) * (kBins / 4)] : make_uint4(0u, 0u, 0u, 0u);
            sum.x += v[j].x; sum.y += v[j].y; sum.z += v[j].z; sum.w += v[j].w;
        }
        uint4 tot;
        const uint4 ex = block_excl_scan4(sum, &tot);
        const uint4 carry = s_carry;
        uint4 run = make_uint4(carry.x + ex.x, carry.y + ex.y, carry.z + ex.z, carry.w + ex.w);
#pragma unroll
        for (uint32_t j = 0; j < kSpineItems; ++j) {
            if (i0 + j < nb) col[(size_t)(i0 + j) * (kBins / 4)] = run;
            run.x += v[j].x; run.y += v[j].y; run.z += v[j].z; run.w += v[j].w;
        }
        __syncthreads();
        if (threadIdx.x == 0) s_carry = make_uint4(carry.x + tot.x, carry.y + tot.y, carry.z + tot.z, carry.w + tot.w);
        __syncthreads();
    }
    if (threadIdx.x == 0) reinterpret_cast<uint4*>(digit_total)[g] = s_carry;
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b to XCD b % 8), and each
// XCD has its own L2.  Block b of `nb` takes data block xcd_block(b, nb): XCD x serves
// the x-th eighth of the data blocks in order, so the blocks resident on one XCD are
// neighbours in the input.  Their runs for one digit are neighbours in the output too
// (block k's run ends where block k + 1's begins), and a cache line that two such runs
// share is completed in one L2 instead of being written back in part from two (the
// runs average 128 bytes).  A bijection of [0, nb).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb)
{
    const uint32_t q = nb >> 3, r = nb & 7u, x = b & 7u;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// The last pass of the tile sort writes no keys: it records each tile's [start, end)
// instead.  The item in local slot li goes to output position o; its neighbours in the
// block's local order (slots li - 1, li + 1) are its neighbours in the output only
// inside one digit's group.  There a key change marks a tile's exact start or end; at
// a group's first or last item the neighbour in the output belongs to another block and
// is not known here, so the item offers itself as a candidate.  The start of a tile is
// the smallest of its candidates and its exact start (the item at the exact start is
// one of them), the end the largest: atomicMin / atomicMax on bounds initialised to
// (0xffffffff, 0).  Keys of the last pass have no bits above its digit, so equal keys
// are contiguous inside a group.
__device__ __forceinline__ void tile_bounds(uint32_t k, uint32_t li, uint32_t o, uint32_t cnt, int shift,
                                            const uint32_t* s_keys, uint32_t* ranges)
{
    const uint32_t d = k >> shift;
    const uint32_t kp = li > 0u ? s_keys[li - 1u] : 0u;
    const uint32_t kn = li + 1u < cnt ? s_keys[li + 1u] : 0u;
    const bool in_p = li > 0u && (kp >> shift) == d;          // slot li - 1 is output position o - 1
    const bool in_n = li + 1u < cnt && (kn >> shift) == d;    // slot li + 1 is output position o + 1
    if (!in_p || kp != k) atomicMin(&ranges[2u * k], o);
    if (!in_n || kn != k) atomicMax(&ranges[2u * k + 1u], o + 1u);
}

// SELF: few blocks (nb <= kSelfSpineBlocks); every block sums the raw per-block
// counts itself and no spine kernel runs.  RANGES: the last pass of the tile sort
// (tile_bounds; keys_out is not written).
template <int ITEMS, bool SELF, bool RANGES>
__global__ __launch_bounds__(kThreads) void radix_downsweep_kernel(const uint32_t* keys_in, const uint32_t* vals_in,
                                                                   uint32_t* keys_out, uint32_t* vals_out,
                                                                   const uint32_t* n_dev, uint32_t n_max, int shift,
                                                                   const uint32_t* hist, uint32_t nb,
                                                                   const uint32_t* digit_total, uint32_t* ranges)
{
    constexpr int kRadixItems = ITEMS;
    constexpr int kRadixTile = kThreads * ITEMS;
    constexpr int kPerWave = 64 * ITEMS;
    __shared__ uint32_t s_keys[kRadixTile];
    __shared__ uint32_t s_vals[kRadixTile];
    __shared__ uint32_t s_wh[kWaves][kBins];  // per-wavefront digit counts, then (digit, wavefront) local starts
    __shared__ uint32_t s_gofs[kBins];        // global start of digit d for this block

    const uint32_t n = item_count(n_dev, n_max);
    // the blocks that hold items (the grid may be sized for a larger capacity)
    const uint32_t nb_live = (uint32_t)(((size_t)n + kRadixTile - 1) / kRadixTile);
    if (blockIdx.x >= nb_live) return;        // whole block leaves together
    const uint32_t blk = xcd_block(blockIdx.x, nb_live);
    const size_t base = (size_t)blk * kRadixTile;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wid = tid >> 6;
    const uint32_t cnt = (uint32_t)((n - base) < (size_t)kRadixTile ? (n - base) : (size_t)kRadixTile);

    // global offsets: exclusive prefix of the digit totals + this block's row offset
    uint32_t tot;
    if (SELF) {
        // every digit's count in all blocks and in the blocks before this one: wavefront
        // w sums rows w, w + 4, ... (lane l: digits 4 l .. 4 l + 3, one 16-byte load a row,
        // 8 rows in flight), then the 4 partial sums of digit tid are added
        uint4 all = make_uint4(0u, 0u, 0u, 0u), bef = all;
        for (uint32_t b0 = wid; b0 < nb; b0 += 8u * kWaves) {
            uint4 v[8];
#pragma unroll
            for (uint32_t k = 0; k < 8u; ++k) {
                const uint32_t b = b0 + k * kWaves;
                v[k] = b < nb ? reinterpret_cast<const uint4*>(hist + (size_t)b * kBins)[lane] : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (uint32_t k = 0; k < 8u; ++k) {
                const uint32_t b = b0 + k * kWaves;
                all.x += v[k].x; all.y += v[k].y; all.z += v[k].z; all.w += v[k].w;
                if (b < blk) { bef.x += v[k].x; bef.y += v[k].y; bef.z += v[k].z; bef.w += v[k].w; }
            }
        }
        s_wh[wid][4u * lane + 0u] = all.x; s_wh[wid][4u * lane + 1u] = all.y;
        s_wh[wid][4u * lane + 2u] = all.z; s_wh[wid][4u * lane + 3u] = all.w;
        s_keys[wid * kBins + 4u * lane + 0u] = bef.x; s_keys[wid * kBins + 4u * lane + 1u] = bef.y;
        s_keys[wid * kBins + 4u * lane + 2u] = bef.z; s_keys[wid * kBins + 4u * lane + 3u] = bef.w;
        __syncthreads();
        uint32_t a = 0u, before = 0u;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            a += s_wh[w][tid];
            before += s_keys[w * kBins + tid];
        }
        __syncthreads();                      // s_wh and s_keys are reused below
        s_gofs[tid] = block_excl_scan(a, &tot) + before;
    } else {
        const uint32_t dbase = block_excl_scan(digit_total[tid], &tot);
        s_gofs[tid] = dbase + hist[(size_t)blk * kBins + tid];
    }
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s_wh[w][tid] = 0u;
    __syncthreads();

    // wavefront wid owns items [wid * kPerWave, (wid + 1) * kPerWave): round r, lane l -> + r * 64 + l
    // every load issued before any is used: a clamped index instead of a branch (items
    // past the end are never ranked into place or written)
    uint32_t k_[kRadixItems], v_[kRadixItems], rk[kRadixItems];
#pragma unroll
    for (int r = 0; r < kRadixItems; ++r) {
        const uint32_t li = wid * kPerWave + (uint32_t)r * 64u + lane;
        k_[r] = keys_in[base + (li < cnt ? li : cnt - 1u)];
    }
    if (vals_in) {
#pragma unroll
        for (int r = 0; r < kRadixItems; ++r) {
            const uint32_t li = wid * kPerWave + (uint32_t)r * 64u + lane;
            v_[r] = vals_in[base + (li < cnt ? li : cnt - 1u)];
        }
    } else {                                  // null: the item's index
#pragma unroll
        for (int r = 0; r < kRadixItems; ++r) v_[r] = (uint32_t)(base + wid * kPerWave + (uint32_t)r * 64u + lane);
    }
#pragma unroll
    for (int r = 0; r < kRadixItems; ++r) {
        const uint32_t li = wid * kPerWave + (uint32_t)r * 64u + lane;
        const bool ok = li < cnt;
        const uint32_t d = (k_[r] >> shift) & 0xffu;
        // peers: lanes of this wavefront holding the same digit.  Per digit bit b, m = 0 or
        // ~0 (the bit, sign-extended), and the lanes that agree with this one on it are
        // ~(ballot ^ m): one three-input bit operation per 32-lane half.  `below`: peers in
        // lower lanes, by mbcnt.
        const uint64_t okm = __builtin_amdgcn_ballot_w64(ok);
        uint32_t plo = (uint32_t)okm, phi = (uint32_t)(okm >> 32);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint32_t m = (uint32_t)((int32_t)(d << (31 - b)) >> 31);
            const uint64_t bal = __builtin_amdgcn_ballot_w64(m != 0u);
            plo &= ~((uint32_t)bal ^ m);
            phi &= ~((uint32_t)(bal >> 32) ^ m);
        }
        const uint64_t peers = ((uint64_t)phi << 32) | plo;
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
        const uint32_t before = s_wh[wid][d];                // this digit's items in earlier rounds
        rk[r] = before + below;
        wave_lds_order();
        if (ok && below == 0u) s_wh[wid][d] = before + (uint32_t)__popcll(peers);
        wave_lds_order();
    }
    __syncthreads();
    {   // thread tid owns digit tid: starts of (digit, wavefront) groups, digit-major
        uint32_t cw[kWaves], td = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            cw[w] = s_wh[w][tid];
            td += cw[w];
        }
        uint32_t run = block_excl_scan(td, &tot);
        // digit tid's block-local start is run: from here s_gofs[d] is the global
        // position of the block's local slot 0 for digit d (local slot li -> s_gofs[d] + li)
        s_gofs[tid] -= run;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            s_wh[w][tid] = run;
            run += cw[w];
        }
    }
    __syncthreads();
    // reorder through LDS, then a coalesced scatter of the locally sorted block.  A full
    // block (all but the last) takes the unguarded form, so that the compiler can keep
    // many items' LDS reads in flight instead of waiting on each item in turn.
    if (cnt == (uint32_t)kRadixTile) {
#pragma unroll
        for (int r = 0; r < kRadixItems; ++r) {
            const uint32_t pos = s_wh[wid][(k_[r] >> shift) & 0xffu] + rk[r];
            s_keys[pos] = k_[r];
            s_vals[pos] = v_[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRadixItems; ++r) {
            const uint32_t li = (uint32_t)r * kThreads + tid;
            const uint32_t k = s_keys[li];
            const uint32_t o = s_gofs[(k >> shift) & 0xffu] + li;
            if (!RANGES) keys_out[o] = k;
            vals_out[o] = s_vals[li];
            if (RANGES) tile_bounds(k, li, o, cnt, shift, s_keys, ranges);
        }
    } else {
#pragma unroll
        for (int r = 0; r < kRadixItems; ++r) {
            const uint32_t li = wid * kPerWave + (uint32_t)r * 64u + lane;
            if (li < cnt) {
                const uint32_t pos = s_wh[wid][(k_[r] >> shift) & 0xffu] + rk[r];
                s_keys[pos] = k_[r];
                s_vals[pos] = v_[r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRadixItems; ++r) {
            const uint32_t li = (uint32_t)r * kThreads + tid;
            if (li < cnt) {
                const uint32_t k = s_keys[li];
                const uint32_t o = s_gofs[(k >> shift) & 0xffu] + li;
                if (!RANGES) keys_out[o] = k;
                vals_out[o] = s_vals[li];
                if (RANGES) tile_bounds(k, li, o, cnt, shift, s_keys, ranges);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Duplication: every (view, Gaussian) in depth order writes one pair per tile
// of its rectangle, row-major, at its scanned offset (the pair's emission
// index e): its tile id, and its record index in emit_vg[e].  The pair's sort
// value is e itself, so after the tile sort a list entry names both the pair's
// gradient row (e) and, through emit_vg, its record.  All pairs of one Gaussian
// are contiguous in emission order, which the backward uses to reduce
// per-pair gradients without atomics.  (An earlier form sorted record indices
// and wrote each Gaussian's emission base into its record: 8-byte writes to
// records in depth order, scattered over the record array, which took 2/3 of
// this kernel's time on the 8-view workload.)
//
// One wavefront takes 64 consecutive Gaussians in depth order; their pairs are
// one contiguous output range, which its 64 lanes write together, 64
// consecutive pairs per step (each lane finds its Gaussian by binary search
// over the wavefront's local offsets), so every store is coalesced and a
// Gaussian with many tiles is spread over all lanes.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void duplicate_kernel(const uint32_t* order, const uint32_t* offsets,
                                                             const uint32_t* tt_s, const uint2* rect_s,
                                                             const CamDev* cams, uint32_t n, uint32_t vn,
                                                             const uint32_t* total, uint32_t cap, uint32_t* keys,
                                                             uint32_t* emit_vg, uint32_t* overflow)
{
    __shared__ uint32_t s_loc[kThreads / 64][64];
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
    const uint32_t s = blockIdx.x * kThreads + threadIdx.x;
    if (s == 0 && *total > cap) *overflow = 1u;
    if (s - lane >= vn) return;                               // whole wavefront
    const bool valid = s < vn;
    uint32_t vg = 0, tt = 0, off = 0, tb = 0, gx = 0;
    uint2 rc = make_uint2(0u, 0u);
    if (valid) {
        vg = order[s];
        tt = tt_s[s];
        off = offsets[s];
        rc = rect_s[s];
        const CamDev& c = cams[vg / n];                       // the record's view: its tile numbering
        tb = c.tile_base;
        gx = (uint32_t)c.gx;
    }
    // the wavefront's pairs: [off0, off0 + count)
    const uint32_t off0 = __shfl(off, 0, 64);
    uint32_t end = valid ? off - off0 + tt : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t y = __shfl_xor(end, o, 64);
        end = end > y ? end : y;
    }
    const uint32_t count = end;
    s_loc[wid][lane] = valid ? off - off0 : count;            // non-decreasing
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t q0 = 0; q0 < count; q0 += 64u) {
        const uint32_t q = q0 + lane < count ? q0 + lane : count - 1u;
        // the Gaussian of output q: the last r with s_loc[r] <= q (it has tt > 0)
        uint32_t r = 0;
#pragma unroll
        for (uint32_t st = 32; st > 0; st >>= 1)
            if (s_loc[wid][r + st] <= q) r += st;
        const uint32_t rvg = (uint32_t)__shfl((int)vg, (int)r, 64);
        const uint32_t rx = (uint32_t)__shfl((int)rc.x, (int)r, 64);
        const uint32_t ry = (uint32_t)__shfl((int)rc.y, (int)r, 64);
        const uint32_t rtb = (uint32_t)__shfl((int)tb, (int)r, 64);
        const uint32_t rgx = (uint32_t)__shfl((int)gx, (int)r, 64);
        const uint32_t k = q - s_loc[wid][r];
        const uint32_t rx0 = rx & 0xffffu, rw = (rx >> 16) - rx0 + 1u, ry0 = ry & 0xffffu;
        const uint32_t dy = k / rw, dx = k - dy * rw;
        const uint32_t p = off0 + q;
        if (q0 + lane < count && p < cap) {
            keys[p] = rtb + (ry0 + dy) * rgx + rx0 + dx;
            emit_vg[p] = rvg;
        }
    }
}

// Per-Gaussian sum of the per-pair gradient rows.  Rows (9 floats, 10 apart)
// are stored in emission order, where all pairs of one (view, Gaussian) are
// contiguous; a row whose stamp (a separate array) is not this frame's was not
// written by its backward (no pixel blended that pair) and counts as zero, and
// is not read: on long lists most rows are stale, so the stamps (4 bytes a pair)
// replace most of the row traffic (40 bytes a pair).  One wavefront takes a
// chunk of 256 consecutive rows, 4 per lane: each lane sums its rows segment by segment, one
// segmented scan over the 64 lanes (keyed by the Gaussian) joins segments
// that span lanes, and every segment that starts and ends inside the chunk is
// written; segments that cross chunk boundaries leave their partial sums in
// `carry` and are finished by seg_fixup_kernel in a fixed order.  No atomics:
// deterministic.
struct SegCarry {
    float head[kG2];         // first segment's sum over this chunk, if it started earlier and ends here
    float tail[kG2];         // last segment's sum over this chunk, if it continues past it
    uint32_t first_seg, last_seg;
    uint32_t flags;          // 1: first segment started earlier; 2: last segment continues; 4: tail has a live row
    uint32_t head_live;      // live rows in head
};

constexpr uint32_t kRowsPerLane = 4;
constexpr uint32_t kChunkRows = 64 * kRowsPerLane;           // 256
constexpr uint32_t kNoSeg = 0xffffffffu;
static_assert(kRowF % 2 == 0, "rows read as 8-byte pairs");

__device__ __forceinline__ void add9(float* a, const float* b)
{
#pragma unroll
    for (int k = 0; k < kG2; ++k) a[k] += b[k];
}

__device__ __forceinline__ void store9(float* dst, const float* v)
{
#pragma unroll
    for (int k = 0; k < kG2; ++k) dst[k] = v[k];
}

// one chunk's owners and stamps (4 rows a lane) and the owners of the rows just
// before and just after it
struct ChunkMeta {
    uint32_t sg[kRowsPerLane], sp[kRowsPerLane];
    uint32_t before, after;
};

__device__ __forceinline__ void load_meta(const uint32_t* emit_vg, const uint32_t* pair_stamp, uint32_t P,
                                          uint32_t c, uint32_t lane, ChunkMeta& m)
{
    const uint32_t r0 = c * kChunkRows, e0 = r0 + lane * kRowsPerLane;
    if (e0 + kRowsPerLane <= P) {
        const uint4 o4 = *reinterpret_cast<const uint4*>(emit_vg + e0);
        const uint4 p4 = *reinterpret_cast<const uint4*>(pair_stamp + e0);
        m.sg[0] = o4.x; m.sg[1] = o4.y; m.sg[2] = o4.z; m.sg[3] = o4.w;
        m.sp[0] = p4.x; m.sp[1] = p4.y; m.sp[2] = p4.z; m.sp[3] = p4.w;
    } else {
#pragma unroll
        for (uint32_t r = 0; r < kRowsPerLane; ++r) {
            m.sg[r] = e0 + r < P ? emit_vg[e0 + r] : kNoSeg;
            m.sp[r] = e0 + r < P ? pair_stamp[e0 + r] : 0u;
        }
    }
    m.before = r0 > 0 ? emit_vg[r0 - 1] : kNoSeg;
    m.after = r0 + kChunkRows < P ? emit_vg[r0 + kChunkRows] : kNoSeg;
}

// DPP move: lane i takes `x` of the lane CTRL names; lanes without one (outside the
// row, or in a row ROW_MASK leaves out) take `old`
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, CTRL, ROW_MASK, 0xf, false);
}

// DPP move of a float: lanes without a source lane read 0
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f0(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, true));
}

// one step of the segmented lane scan: add the sums of the lane CTRL names if it
// holds the same segment (Cl: live rows, exact as a float)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_scan_step(float (&C)[kG2], float& Cl, uint32_t sl)
{
    const uint32_t su = dpp_u32<CTRL, ROW_MASK>(kNoSeg, sl);
    // the other lane's sums times 1 (same segment) or 0: a DPP move and a multiply-add
    // a value (the sums are finite, and C + y * 1 rounds as C + y)
    const float sf = (su == sl && sl != kNoSeg) ? 1.f : 0.f;
#pragma unroll
    for (int k = 0; k < kG2; ++k) C[k] = fmaf(dpp_f0<CTRL, ROW_MASK>(C[k]), sf, C[k]);
    Cl = fmaf(dpp_f0<CTRL, ROW_MASK>(Cl), sf, Cl);
}

__global__ __launch_bounds__(kThreads, 3) void seg_reduce_kernel(const float* pair_grad, const uint32_t* pair_stamp,
                                                              const uint32_t* stamp, const uint32_t* emit_vg,
                                                              const uint32_t* total, uint32_t cap, float* grad2d,
                                                              uint32_t* rec_stamp, SegCarry* carry)
{
    const uint32_t P = *total < cap ? *total : cap;
    const uint32_t st = *stamp;
    const uint32_t lane = lane_id();
    const uint32_t nchunk = (P + kChunkRows - 1) / kChunkRows;
    // chunks, grid-stride (the grid does not grow with the pair capacity); each
    // chunk's owners and stamps are loaded while the previous chunk's rows are in
    // flight, so a chunk waits on one round trip to memory, not three
    const uint32_t stride = (gridDim.x * kThreads) >> 6;
    uint32_t c = (blockIdx.x * kThreads + threadIdx.x) >> 6;
    ChunkMeta nx;
    if (c < nchunk) load_meta(emit_vg, pair_stamp, P, c, lane, nx);
    for (; c < nchunk; c += stride) {
        const ChunkMeta m = nx;
        const uint32_t r0 = c * kChunkRows;
        const uint32_t* sg = m.sg;
        const uint32_t* sp = m.sp;
        // each lane reads its own live rows (a row is live if this frame's backward wrote
        // it), 40 bytes each as five 8-byte loads, all in flight before the first is used;
        // stale rows are not read and count as zeros.  (Staging the chunk through LDS with
        // coalesced 16-byte loads needed a per-word liveness lookup that held 40 VGPRs and
        // a third of the kernel's VALU work; on long lists few rows are live, so the
        // scattered loads of this form are few.)
        bool lv[kRowsPerLane];
        float mine[kRowsPerLane * kRowF];
#pragma unroll
        for (uint32_t r = 0; r < kRowsPerLane; ++r) {
            lv[r] = sg[r] != kNoSeg && sp[r] == st;
#pragma unroll
            for (int k = 0; k < kRowF; ++k) mine[r * kRowF + k] = 0.f;
            if (lv[r]) {
                const float2* x = reinterpret_cast<const float2*>(pair_grad + (size_t)kRowF * (r0 + lane * kRowsPerLane + r));
#pragma unroll
                for (int k = 0; k < kRowF / 2; ++k) {
                    const float2 y = x[k];
                    mine[r * kRowF + 2 * k] = y.x;
                    mine[r * kRowF + 2 * k + 1] = y.y;
                }
            }
        }
        if (c + stride < nchunk) load_meta(emit_vg, pair_stamp, P, c + stride, lane, nx);
        auto load_row = [&](uint32_t r, float* row) {
#pragma unroll
            for (int k = 0; k < kG2; ++k) row[k] = mine[r * kRowF + k];
        };
        // lane-local segments: A = first segment's partial, B = last segment's partial,
        // la / lb their numbers of live rows (a segment without one is not written)
        float A[kG2], B[kG2];
        uint32_t s0 = sg[0], sl = sg[0], nseg = 1, la = 0, lb = lv[0] ? 1u : 0u;
        load_row(0, B);
#pragma unroll
        for (uint32_t r = 1; r < kRowsPerLane; ++r) {
            if (sg[r] == kNoSeg) break;
            float row[kG2];
            load_row(r, row);
            const bool live = lv[r];
            if (sg[r] != sl) {                                   // segment sl ends inside this lane
                if (nseg == 1) {
#pragma unroll
                    for (int k = 0; k < kG2; ++k) A[k] = B[k];
                    la = lb;
                } else if (lb) {                                 // started and ended in this lane
                    store9(grad2d + (size_t)kG2 * sl, B);
                    rec_stamp[sl] = st;
                }
                sl = sg[r];
                ++nseg;
#pragma unroll
                for (int k = 0; k < kG2; ++k) B[k] = live ? row[k] : 0.f;
                lb = live ? 1u : 0u;
            } else if (live) {
                add9(B, row);
                ++lb;
            }
        }
        if (nseg == 1) {
#pragma unroll
            for (int k = 0; k < kG2; ++k) A[k] = B[k];
            la = lb;
        }
        // C = segmented inclusive sum of B over lanes, keyed by the last segment (Cl: of lb):
        // shifts by 1, 2, 4 and 8 lanes inside each row of 16, then the last lane of each
        // row into the next row and of the lower half into the upper half, all as DPP
        // moves (segments are contiguous, so an equal key two lanes apart means one
        // segment between them)
        float C[kG2];
        float Cl = (float)lb;
#pragma unroll
        for (int k = 0; k < kG2; ++k) C[k] = B[k];
        seg_scan_step<0x111, 0xf>(C, Cl, sl);                   // row_shr:1
        seg_scan_step<0x112, 0xf>(C, Cl, sl);                   // row_shr:2
        seg_scan_step<0x114, 0xf>(C, Cl, sl);                   // row_shr:4
        seg_scan_step<0x118, 0xf>(C, Cl, sl);                   // row_shr:8
        seg_scan_step<0x142, 0xa>(C, Cl, sl);                   // row_bcast:15 into rows 1 and 3
        seg_scan_step<0x143, 0xc>(C, Cl, sl);                   // row_bcast:31 into rows 2 and 3
        // the chunk's neighbours: the row before it and the row after it; the previous
        // lane's last segment and sums, the next lane's first segment (wave_shr:1, wave_shl:1)
        const uint32_t sfirst = (uint32_t)__builtin_amdgcn_readlane((int)s0, 0);
        const bool crosses_in = r0 > 0 && m.before == sfirst;
        const uint32_t after = m.after;
        const uint32_t nxt = dpp_u32<0x130, 0xf>(after, s0);
        const uint32_t prv_sl = dpp_u32<0x138, 0xf>(kNoSeg, sl);
        float prvC[kG2];
#pragma unroll
        for (int k = 0; k < kG2; ++k) prvC[k] = __uint_as_float(dpp_u32<0x138, 0xf>(0u, __float_as_uint(C[k])));
        const uint32_t prvCl = (uint32_t)__uint_as_float(dpp_u32<0x138, 0xf>(0u, __float_as_uint(Cl)));
        const bool valid = s0 != kNoSeg;
        SegCarry* cr = carry + c;
        if (valid && nseg >= 2) {                                // first segment ends in this lane
            if (lane > 0 && prv_sl == s0) {                      // ... and began in an earlier lane
                add9(A, prvC);
                la += prvCl;
            }
            if (crosses_in && s0 == sfirst) {
                store9(cr->head, A);
                cr->head_live = la;
            } else if (la) {
                store9(grad2d + (size_t)kG2 * s0, A);
                rec_stamp[s0] = st;
            }
        }
        if (valid && nxt != sl) {                                // last segment ends in this lane
            if (crosses_in && sl == sfirst) {
                store9(cr->head, C);
                cr->head_live = (uint32_t)Cl;
            } else if (Cl != 0.f) {
                store9(grad2d + (size_t)kG2 * sl, C);
                rec_stamp[sl] = st;
            }
        }
        // the chunk's last valid lane (the next lane holds no rows, or lane 63) records the chunk
        if (valid && (lane == 63 || nxt == kNoSeg)) {
            const bool crosses_out = lane == 63 && after == sl;
#pragma unroll
            for (int k = 0; k < kG2; ++k) cr->tail[k] = crosses_out ? C[k] : 0.f;
            cr->first_seg = sfirst;
            cr->last_seg = sl;
            cr->flags = (crosses_in ? 1u : 0u) | (crosses_out ? 2u : 0u) | (crosses_out && Cl != 0.f ? 4u : 0u);
        }
    }
}

// one thread per chunk: a segment that starts in chunk w and continues past it
// is summed here over the following chunks, in order
__global__ __launch_bounds__(kThreads) void seg_fixup_kernel(const SegCarry* carry, const uint32_t* total,
                                                             uint32_t cap, const uint32_t* stamp, float* grad2d,
                                                             uint32_t* rec_stamp)
{
    const uint32_t P = *total < cap ? *total : cap;
    const uint32_t nw = (P + kChunkRows - 1) / kChunkRows;
    for (uint32_t w = blockIdx.x * kThreads + threadIdx.x; w < nw; w += gridDim.x * kThreads) {
    const SegCarry& c = carry[w];
    if (!(c.flags & 2u)) continue;                               // nothing continues past w
    if ((c.flags & 1u) && c.first_seg == c.last_seg) continue;   // w is inside a segment begun earlier
    const uint32_t s = c.last_seg;
    float acc[kG2];
    bool live = (c.flags & 4u) != 0u;
#pragma unroll
    for (int k = 0; k < kG2; ++k) acc[k] = c.tail[k];
    for (uint32_t u = w + 1; u < nw; ++u) {
        const SegCarry& d = carry[u];
        const bool whole = (d.flags & 3u) == 3u && d.first_seg == d.last_seg && d.first_seg == s;
        if (whole) {
#pragma unroll
            for (int k = 0; k < kG2; ++k) acc[k] += d.tail[k];
            live = live || (d.flags & 4u) != 0u;
            continue;
        }
#pragma unroll
        for (int k = 0; k < kG2; ++k) acc[k] += d.head[k];
        live = live || d.head_live != 0u;
        break;
    }
    if (!live) continue;                                         // no row of the segment was written
    float* dst = grad2d + (size_t)kG2 * s;
#pragma unroll
    for (int k = 0; k < kG2; ++k) dst[k] = acc[k];
    rec_stamp[s] = *stamp;
    }
}


__global__ void iota_u32_kernel(uint32_t* p, uint32_t count)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = i;
}

// a frame's first kernel: pair count and overflow cleared, the row stamp advanced,
// and the tile ranges (plus the tile-order class counts behind them) cleared
__global__ void frame_begin_kernel(uint32_t* counters, uint32_t* ranges, uint32_t n_tiles, uint32_t n_words)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counters[0] = 0u;
        counters[1] = 0u;
        counters[8] = 0u;                     // set when this frame's invariants are checked
        atomicAdd(&counters[4], 1u);
    }
    // tile bounds (0xffffffff, 0), then the words after them zero
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += gridDim.x * blockDim.x)
        ranges[i] = i < 2u * n_tiles && (i & 1u) == 0u ? 0xffffffffu : 0u;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t value, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

// tiles without pairs: bounds (0xffffffff, 0) from frame_begin -> [0, 0)
__global__ __launch_bounds__(kThreads) void ranges_finish_kernel(uint2* ranges, uint32_t n_tiles)
{
    for (uint32_t t = blockIdx.x * kThreads + threadIdx.x; t < n_tiles; t += gridDim.x * kThreads)
        if (ranges[t].x == 0xffffffffu) ranges[t] = make_uint2(0u, 0u);
}


}  // namespace

// grids of the grid-stride kernels: enough workgroups to fill the chip many
// times over, without growing with a pair capacity that may far exceed the count
static uint32_t grid_cap(uint32_t blocks) { return blocks < 16384u ? (blocks ? blocks : 1u) : 16384u; }

size_t scan_tmp_words(uint32_t n) { return (size_t)(n + kTileItems - 1) / kTileItems + 1; }

hipError_t launch_gather_scan(const uint2* trect, const uint32_t* order, uint32_t n, uint32_t* out,
                              uint32_t* vals_s, uint2* rect_s, uint32_t* total, uint32_t* overflow, uint32_t* tmp,
                              hipStream_t s)
{
    uint32_t nb = (n + kTileItems - 1) / kTileItems;
    if (nb > 0)
        hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb), dim3(kThreads), 0, s, trect, order, n, tmp, vals_s, rect_s);
    if (nb > 0 && nb <= (uint32_t)kThreads) {          // few blocks: no spine
        hipLaunchKernelGGL(scan_down_kernel<true>, dim3(nb), dim3(kThreads), 0, s, vals_s, n, tmp, nb, out, total,
                           overflow);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(scan_spine_kernel, dim3(1), dim3(kThreads), 0, s, tmp, nb, total, overflow);
    if (nb > 0)
        hipLaunchKernelGGL(scan_down_kernel<false>, dim3(nb), dim3(kThreads), 0, s, vals_s, n, tmp, nb, out, total,
                           overflow);
    return hipGetLastError();
}

size_t radix_tmp_words(uint32_t n_max)
{
    // sized for the smaller tile, so that it also covers every pass over fewer items
    const uint32_t tile = kThreads * kRadixSmallItems;
    size_t nb = (n_max + tile - 1) / tile;
    return (size_t)kBins * (nb > 0 ? nb : 1) + kBins;
}

template <int ITEMS, bool SELF>
static void launch_downsweep(uint32_t nb, hipStream_t s, const uint32_t* keys_in, const uint32_t* vals_in,
                             uint32_t* keys_out, uint32_t* vals_out, const uint32_t* n_dev, uint32_t n_max, int shift,
                             const uint32_t* hist, const uint32_t* digit_total, uint2* ranges)
{
    if (ranges)
        hipLaunchKernelGGL((radix_downsweep_kernel<ITEMS, SELF, true>), dim3(nb), dim3(kThreads), 0, s, keys_in,
                           vals_in, keys_out, vals_out, n_dev, n_max, shift, hist, nb, digit_total,
                           reinterpret_cast<uint32_t*>(ranges));
    else
        hipLaunchKernelGGL((radix_downsweep_kernel<ITEMS, SELF, false>), dim3(nb), dim3(kThreads), 0, s, keys_in,
                           vals_in, keys_out, vals_out, n_dev, n_max, shift, hist, nb, digit_total, nullptr);
}

hipError_t launch_radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out,
                             const uint32_t* n_dev, uint32_t n_max, int shift, uint32_t* tmp, hipStream_t s,
                             uint2* ranges)
{
    const uint32_t items = radix_items(n_max), tile = kThreads * items;
    uint32_t nb = (n_max + tile - 1) / tile;
    if (nb == 0) return hipSuccess;
    uint32_t* hist = tmp;
    uint32_t* digit_total = tmp + (size_t)kBins * nb;
    if (items == kRadixLargeItems)
        hipLaunchKernelGGL(radix_upsweep_kernel<kRadixLargeItems>, dim3(nb), dim3(kThreads), 0, s, keys_in, n_dev,
                           n_max, shift, hist);
    else
        hipLaunchKernelGGL(radix_upsweep_kernel<kRadixSmallItems>, dim3(nb), dim3(kThreads), 0, s, keys_in, n_dev,
                           n_max, shift, hist);
    if (nb <= kSelfSpineBlocks) {             // the downsweep blocks find their offsets themselves
        if (items == kRadixLargeItems)
            launch_downsweep<kRadixLargeItems, true>(nb, s, keys_in, vals_in, keys_out, vals_out, n_dev, n_max, shift,
                                                     hist, digit_total, ranges);
        else
            launch_downsweep<kRadixSmallItems, true>(nb, s, keys_in, vals_in, keys_out, vals_out, n_dev, n_max, shift,
                                                     hist, digit_total, ranges);
        return hipGetLastError();
    }
    // counts a thread: enough that a long column takes few block scans, few enough
    // that a short one is spread over the workgroup
    if (nb > 8u * kThreads)
        hipLaunchKernelGGL(radix_spine_kernel<16>, dim3(kBins / 4), dim3(kThreads), 0, s, hist, n_dev, n_max, tile,
                           digit_total);
    else if (nb > kThreads)
        hipLaunchKernelGGL(radix_spine_kernel<8>, dim3(kBins / 4), dim3(kThreads), 0, s, hist, n_dev, n_max, tile,
                           digit_total);
    else
        hipLaunchKernelGGL(radix_spine_kernel<1>, dim3(kBins / 4), dim3(kThreads), 0, s, hist, n_dev, n_max, tile,
                           digit_total);
    if (items == kRadixLargeItems)
        launch_downsweep<kRadixLargeItems, false>(nb, s, keys_in, vals_in, keys_out, vals_out, n_dev, n_max, shift,
                                                  hist, digit_total, ranges);
    else
        launch_downsweep<kRadixSmallItems, false>(nb, s, keys_in, vals_in, keys_out, vals_out, n_dev, n_max, shift,
                                                  hist, digit_total, ranges);
    return hipGetLastError();
}

hipError_t launch_duplicate(const uint32_t* order, const uint32_t* offsets, const uint32_t* tt_s,
                            const uint2* rect_s, const CamDev* cams, uint32_t n, uint32_t vn, const uint32_t* total,
                            uint32_t cap, uint32_t* keys, uint32_t* emit_vg, uint32_t* overflow, hipStream_t s)
{
    if (vn == 0) return hipSuccess;
    hipLaunchKernelGGL(duplicate_kernel, dim3((vn + kThreads - 1) / kThreads), dim3(kThreads), 0, s, order, offsets,
                       tt_s, rect_s, cams, n, vn, total, cap, keys, emit_vg, overflow);
    return hipGetLastError();
}

size_t seg_carry_bytes(uint32_t cap) { return ((size_t)cap + kChunkRows - 1) / kChunkRows * sizeof(SegCarry) + sizeof(SegCarry); }

hipError_t launch_grad_reduce(const float* pair_grad, const uint32_t* pair_stamp, const uint32_t* stamp,
                              const uint32_t* emit_vg, uint32_t vn, const uint32_t* total, uint32_t cap, float* grad2d,
                              uint32_t* rec_stamp, void* carry, hipStream_t s)
{
    (void)vn;
    if (cap == 0) return hipSuccess;
    const uint32_t nw = (cap + kChunkRows - 1) / kChunkRows;
    hipLaunchKernelGGL(seg_reduce_kernel, dim3(grid_cap((nw * 64 + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       pair_grad, pair_stamp, stamp, emit_vg, total, cap, grad2d, rec_stamp,
                       reinterpret_cast<SegCarry*>(carry));
    hipLaunchKernelGGL(seg_fixup_kernel, dim3(grid_cap((nw + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       reinterpret_cast<const SegCarry*>(carry), total, cap, stamp, grad2d, rec_stamp);
    return hipGetLastError();
}

hipError_t launch_iota_u32(uint32_t* p, uint32_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(iota_u32_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
    return hipGetLastError();
}


hipError_t launch_frame_begin(uint32_t* counters, uint32_t* ranges, uint32_t n_tiles, uint32_t n_words, hipStream_t s)
{
    uint32_t blocks = (n_words + 255u) / 256u;
    blocks = blocks < 1u ? 1u : (blocks > 1024u ? 1024u : blocks);
    hipLaunchKernelGGL(frame_begin_kernel, dim3(blocks), dim3(256), 0, s, counters, ranges, n_tiles, n_words);
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

// ---------------------------------------------------------------------------
// Tile order for the blend kernels: longest list first.  Tile list lengths are
// very uneven (the 99th percentile is several times the mean), and with the
// tiles in spatial order a few long tiles dispatched late decide the end of the
// grid.  A counting sort over 256 length classes (16 per octave of the length)
// gives the hardware dispatcher the long tiles first and leaves the short ones
// to fill the end.  Only the scheduling changes: a tile's results do not depend
// on the workgroup that handles it, so the order inside a class (set by
// atomics) is immaterial.
// ---------------------------------------------------------------------------

namespace {

__device__ __forceinline__ uint32_t tile_bucket(uint2 r)
{
    const float c = 16.f * __builtin_amdgcn_logf((float)(r.y - r.x) + 1.f);   // 16 log2(len + 1)
    return 255u - (c < 255.f ? (uint32_t)c : 255u);                            // bucket 0: longest
}

__global__ __launch_bounds__(kThreads) void tile_hist_kernel(const uint2* ranges, uint32_t n_tiles, uint32_t* hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    for (uint32_t t = blockIdx.x * kThreads + threadIdx.x; t < n_tiles; t += gridDim.x * kThreads)
        atomicAdd(&h[tile_bucket(ranges[t])], 1u);
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(kThreads) void tile_order_kernel(const uint2* ranges, uint32_t n_tiles,
                                                              const uint32_t* hist, uint32_t* fill, uint32_t* order)
{
    __shared__ uint32_t s_start[256], s_cnt[256], s_base[256];
    // exclusive prefix of the class counts (the same in every workgroup)
    const uint32_t mine = hist[threadIdx.x];
    s_start[threadIdx.x] = mine;
    __syncthreads();
    for (uint32_t o = 1; o < 256; o <<= 1) {
        const uint32_t v = threadIdx.x >= o ? s_start[threadIdx.x - o] : 0u;
        __syncthreads();
        s_start[threadIdx.x] += v;
        __syncthreads();
    }
    s_start[threadIdx.x] -= mine;
    const uint32_t nchunk = (n_tiles + kThreads - 1) / kThreads;
    for (uint32_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        s_cnt[threadIdx.x] = 0u;
        __syncthreads();
        const uint32_t t = ch * kThreads + threadIdx.x;
        uint32_t b = 0, local = 0;
        if (t < n_tiles) {
            b = tile_bucket(ranges[t]);
            local = atomicAdd(&s_cnt[b], 1u);
        }
        __syncthreads();
        if (s_cnt[threadIdx.x]) s_base[threadIdx.x] = atomicAdd(&fill[threadIdx.x], s_cnt[threadIdx.x]);
        __syncthreads();
        if (t < n_tiles) order[s_start[b] + s_base[b] + local] = t;
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_tile_order(const uint2* ranges, uint32_t n_tiles, uint32_t* hist, uint32_t* order, hipStream_t s)
{
    if (n_tiles == 0) return hipSuccess;
    uint32_t grid = (n_tiles + kThreads - 1) / kThreads;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(tile_hist_kernel, dim3(grid), dim3(kThreads), 0, s, ranges, n_tiles, hist);
    hipLaunchKernelGGL(tile_order_kernel, dim3(grid), dim3(kThreads), 0, s, ranges, n_tiles, hist, hist + 256, order);
    return hipGetLastError();
}

hipError_t launch_ranges_finish(uint2* ranges, uint32_t n_tiles, hipStream_t s)
{
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(ranges_finish_kernel, dim3(grid_cap((n_tiles + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       ranges, n_tiles);
    return hipGetLastError();
}


}  // namespace gsr
