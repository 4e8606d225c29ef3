// Front-to-back alpha blending with the entropy of the blending weights
// (Sec. 3, Eq. 3-5; Sec. 3.3, Eq. 8-11) and the back-to-front backward with
// the O(N) entropy gradient of Alg. 1 (Sec. 3.4, Eq. 13-15; Suppl. C).
//
// Work decomposition: every 64-lane wavefront owns one 8x8 pixel block (one
// pixel per lane) and walks the Gaussian list of the tile that contains the
// block.  Tiles are 8x8, 16x16 or 32x8 pixels, so a tile holds 1 or 4
// blocks; the tile size sets the sort granularity, the wavefront size sets
// the blend granularity.  Each wavefront stages its list in LDS in batches of
// B records (its own LDS region, so no workgroup barrier is ever needed and a
// wavefront whose pixels are all saturated leaves at once), and every lane
// reads the staged record as an LDS broadcast.
#include "internal.h"

namespace gsr {
namespace {

constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTStop = 1e-4f;
constexpr int kWavesPerGroup = 4;

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// exponent of the 2D Gaussian at offset (dx, dy) = mean - pixel centre:
//   -1/2 (A dx^2 + C dy^2) - B dx dy, evaluated with explicit FMAs so the
//   forward and backward kernels produce bit-identical alphas.
__device__ __forceinline__ float gauss_power(float A, float B, float C, float dx, float dy)
{
    float q = fmaf(A * dx, dx, fmaf(C * dy, dy, (2.f * B) * (dx * dy)));
    return -0.5f * q;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

// sum over the 64 lanes; the total is valid in lane 63
__device__ __forceinline__ float wave_sum_to_lane63(float x)
{
    x += dpp_f<0xb1, 0xf>(x);    // quad_perm [1,0,3,2]
    x += dpp_f<0x4e, 0xf>(x);    // quad_perm [2,3,0,1]
    x += dpp_f<0x141, 0xf>(x);   // row_half_mirror
    x += dpp_f<0x140, 0xf>(x);   // row_mirror: every lane holds its row's sum
    x += dpp_f<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
    x += dpp_f<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
    return x;
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
    int px, py;
    bool inside;
    uint32_t tile;
    int64_t pix;
};

__device__ __forceinline__ BlockGeom block_geom(const CamDev* cams, int n_views, uint32_t wblock, uint32_t lane,
                                                int tsx, int tsy)
{
    BlockGeom g;
    int v = 0;
    while (v + 1 < n_views && cams[v + 1].block_base <= wblock) ++v;
    const CamDev& c = cams[v];
    uint32_t b = wblock - c.block_base;
    uint32_t bxi = b % (uint32_t)c.bx, byi = b / (uint32_t)c.bx;
    g.view = v;
    g.px = (int)(bxi * kBlockPx + (lane & 7u));
    g.py = (int)(byi * kBlockPx + (lane >> 3));
    g.inside = g.px < c.W && g.py < c.H;
    g.tile = c.tile_base + ((byi * kBlockPx) >> tsy) * (uint32_t)c.gx + ((bxi * kBlockPx) >> tsx);
    g.pix = c.pix_base + (int64_t)g.py * c.W + g.px;
    return g;
}

template <int B>
__global__ __launch_bounds__(256) void blend_fwd_kernel(BlendFwdArgs a)
{
    __shared__ float4 s_rec[kWavesPerGroup][B][kRecF4];
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    const uint32_t wblock = blockIdx.x * kWavesPerGroup + wid;
    if (wblock >= a.n_blocks) return;
    const BlockGeom g = block_geom(a.cams, a.n_views, wblock, lane, a.tile_shift_x, a.tile_shift_y);
    const uint2 rg = a.ranges[g.tile];
    const float fpx = (float)g.px + 0.5f, fpy = (float)g.py + 0.5f;

    float T = 1.f, Cr = 0.f, Cg = 0.f, Cb = 0.f, H = 0.f;
    int32_t last = 0;
    uint32_t n_eval = 0;
    bool done = !g.inside;
    for (uint32_t bs = rg.x; bs < rg.y; bs += B) {
        if (__ballot(!done) == 0ull) break;
        const uint32_t cnt = (rg.y - bs) < (uint32_t)B ? (rg.y - bs) : (uint32_t)B;
        for (uint32_t j = lane; j < cnt; j += kWave) {
            const float4* r = a.rec + (size_t)kRecF4 * a.pair_vals[bs + j];
            s_rec[wid][j][0] = r[0];
            s_rec[wid][j][1] = r[1];
            s_rec[wid][j][2] = r[2];
        }
        wave_lds_sync();
        for (uint32_t j = 0; j < cnt; ++j) {
            if (__ballot(!done) == 0ull) break;
            if (!done) {
                const float4 r0 = s_rec[wid][j][0];
                const float4 r1 = s_rec[wid][j][1];
                const float dx = r0.x - fpx, dy = r0.y - fpy;
                const float e = __expf(gauss_power(r0.z, r0.w, r1.x, dx, dy));
                const float alpha = fminf(kAlphaMax, r1.y * e);
                ++n_eval;
                if (alpha >= kAlphaMin) {
                    const float Tn = T * (1.f - alpha);
                    if (Tn < kTStop) {
                        done = true;
                    } else {
                        const float w = alpha * T;
                        const float cb = s_rec[wid][j][2].x;
                        Cr = fmaf(w, r1.z, Cr);
                        Cg = fmaf(w, r1.w, Cg);
                        Cb = fmaf(w, cb, Cb);
                        H = fmaf(-w, __logf(w), H);       // -w log w   (Eq. 10)
                        T = Tn;
                        last = (int32_t)(bs + j - rg.x + 1);
                    }
                }
            }
        }
        wave_lds_sync();
    }
    H = fmaf(-T, logf(T), H);                           // background weight T_{N+1}  (Eq. 9-10)
    if (g.inside) {
        a.out_rgb[3 * g.pix + 0] = Cr;
        a.out_rgb[3 * g.pix + 1] = Cg;
        a.out_rgb[3 * g.pix + 2] = Cb;
        a.out_H[g.pix] = H;
        a.out_T[g.pix] = T;
        a.out_nc[g.pix] = last;
    }
    float hs = wave_sum_all(g.inside ? H : 0.f);
    uint32_t ne = (uint32_t)wave_sum_all_i((int)n_eval);
    uint32_t nc = (uint32_t)wave_sum_all_i(last);
    if (lane == 0) {
        a.block_H[wblock] = hs;
        a.block_cnt[wblock] = make_uint2(ne, nc);
    }
}

template <int B>
__global__ __launch_bounds__(256) void blend_bwd_kernel(BlendBwdArgs a)
{
    __shared__ float4 s_rec[kWavesPerGroup][B][kRecF4];
    __shared__ uint32_t s_vg[kWavesPerGroup][B];
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    const uint32_t wblock = blockIdx.x * kWavesPerGroup + wid;
    if (wblock >= a.n_blocks) return;
    const BlockGeom g = block_geom(a.cams, a.n_views, wblock, lane, a.tile_shift_x, a.tile_shift_y);
    const uint2 rg = a.ranges[g.tile];
    const float fpx = (float)g.px + 0.5f, fpy = (float)g.py + 0.5f;

    int32_t n = 0;
    float T = 1.f, gCr = 0.f, gCg = 0.f, gCb = 0.f, gh = 0.f;
    const int32_t len = (int32_t)(rg.y - rg.x);
    if (g.inside) {
        n = a.n_contrib[g.pix];
        n = n < 0 ? 0 : (n > len ? len : n);       // never walk past this tile's list
        T = a.T_final[g.pix];
        gCr = a.grad_rgb[3 * g.pix + 0];
        gCg = a.grad_rgb[3 * g.pix + 1];
        gCb = a.grad_rgb[3 * g.pix + 2];
        if (a.grad_H) gh = a.grad_H[g.pix];
        if (a.grad_LE) {
            const CamDev& c = a.cams[g.view];
            gh += a.grad_LE[g.view] / (float)((int64_t)c.W * c.H);
        }
    }
    // suffix sums, Alg. 1:  R_{N+1} = (log w_{N+1} + 1) w_{N+1} with w_{N+1} = T_final
    float Sr = 0.f, Sg = 0.f, Sb = 0.f;
    float Rs = (logf(T) + 1.f) * T;
    const int32_t maxn = wave_max_i32(n);

    for (int32_t hi = maxn; hi > 0; hi -= B) {
        const int32_t lo = hi - B > 0 ? hi - B : 0;
        const int32_t cnt = hi - lo;
        for (int32_t j = (int32_t)lane; j < cnt; j += kWave) {
            const uint32_t vg = a.pair_vals[rg.x + (uint32_t)(lo + j)];
            const float4* r = a.rec + (size_t)kRecF4 * vg;
            s_vg[wid][j] = vg;
            s_rec[wid][j][0] = r[0];
            s_rec[wid][j][1] = r[1];
            s_rec[wid][j][2] = r[2];
        }
        wave_lds_sync();
        for (int32_t j = cnt - 1; j >= 0; --j) {
            float gmx = 0.f, gmy = 0.f, gA = 0.f, gB = 0.f, gC = 0.f, gop = 0.f, gr = 0.f, gg = 0.f, gb = 0.f;
            bool contrib = false;
            if (lo + j < n) {
                const float4 r0 = s_rec[wid][j][0];
                const float4 r1 = s_rec[wid][j][1];
                const float cb = s_rec[wid][j][2].x;
                const float dx = r0.x - fpx, dy = r0.y - fpy;
                const float e = __expf(gauss_power(r0.z, r0.w, r1.x, dx, dy));
                const float a_raw = r1.y * e;
                const float alpha = fminf(kAlphaMax, a_raw);
                if (alpha >= kAlphaMin) {
                    contrib = true;
                    const float rom = __builtin_amdgcn_rcpf(1.f - alpha);
                    const float Ti = T * rom;                    // T_i = T_{i+1} / (1 - alpha_i)
                    const float w = alpha * Ti;
                    const float lw = __logf(w);
                    // dC/dalpha_i = T_i c_i - S_{i+1} / (1 - alpha_i);  Eq. 15 for dH/dalpha_i
                    float dal = gCr * (Ti * r1.z - Sr * rom) + gCg * (Ti * r1.w - Sg * rom) +
                                gCb * (Ti * cb - Sb * rom);
                    dal += gh * ((-lw - 1.f) * Ti + Rs * rom);
                    gr = w * gCr;
                    gg = w * gCg;
                    gb = w * gCb;
                    if (a_raw <= kAlphaMax) {                    // zero gradient in the clamped branch
                        gop = e * dal;
                        const float dp = alpha * dal;            // d alpha / d power = alpha
                        gA = -0.5f * dx * dx * dp;
                        gB = -dx * dy * dp;
                        gC = -0.5f * dy * dy * dp;
                        gmx = -dp * (r0.z * dx + r0.w * dy);
                        gmy = -dp * (r0.w * dx + r1.x * dy);
                    }
                    Sr = fmaf(w, r1.z, Sr);
                    Sg = fmaf(w, r1.w, Sg);
                    Sb = fmaf(w, cb, Sb);
                    Rs = fmaf(lw + 1.f, w, Rs);                  // R_i = (log w_i + 1) w_i + R_{i+1}
                    T = Ti;
                }
            }
            if (__ballot(contrib) != 0ull) {
                gmx = wave_sum_to_lane63(gmx);
                gmy = wave_sum_to_lane63(gmy);
                gA = wave_sum_to_lane63(gA);
                gB = wave_sum_to_lane63(gB);
                gC = wave_sum_to_lane63(gC);
                gop = wave_sum_to_lane63(gop);
                gr = wave_sum_to_lane63(gr);
                gg = wave_sum_to_lane63(gg);
                gb = wave_sum_to_lane63(gb);
                if (lane == 63u) {
                    float* dst = a.grad2d + (size_t)kG2 * s_vg[wid][j];
                    unsafeAtomicAdd(dst + 0, gmx);
                    unsafeAtomicAdd(dst + 1, gmy);
                    unsafeAtomicAdd(dst + 2, gA);
                    unsafeAtomicAdd(dst + 3, gB);
                    unsafeAtomicAdd(dst + 4, gC);
                    unsafeAtomicAdd(dst + 5, gop);
                    unsafeAtomicAdd(dst + 6, gr);
                    unsafeAtomicAdd(dst + 7, gg);
                    unsafeAtomicAdd(dst + 8, gb);
                }
            }
        }
        wave_lds_sync();
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

// level 1: one workgroup per chunk of kRedChunk 8x8 blocks of one view
__global__ __launch_bounds__(256) void entropy_chunk_kernel(const float* block_H, const CamDev* cams, int n_views,
                                                            double* chunk_sum)
{
    const uint32_t ch = blockIdx.x;
    int v = 0;
    while (v + 1 < n_views && cams[v + 1].hred_base <= ch) ++v;
    const CamDev& c = cams[v];
    const uint32_t nb = (uint32_t)(c.bx * c.by);
    const uint32_t b0 = (ch - c.hred_base) * kRedChunk;
    double acc = 0.0;
    for (uint32_t k = threadIdx.x; k < (uint32_t)kRedChunk; k += 256)
        if (b0 + k < nb) acc += (double)block_H[c.block_base + b0 + k];
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

template <int B>
hipError_t fwd_b(const BlendFwdArgs& a, hipStream_t s)
{
    dim3 grid((a.n_blocks + kWavesPerGroup - 1) / kWavesPerGroup);
    hipLaunchKernelGGL(blend_fwd_kernel<B>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int B>
hipError_t bwd_b(const BlendBwdArgs& a, hipStream_t s)
{
    dim3 grid((a.n_blocks + kWavesPerGroup - 1) / kWavesPerGroup);
    hipLaunchKernelGGL(blend_bwd_kernel<B>, grid, dim3(256), 0, s, a);
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
        case 256: return bwd_b<256>(a, s);
    }
    return hipErrorInvalidValue;
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
