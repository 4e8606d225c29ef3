// L1 photometric term of the base loss (Sec. 3, Eq. 6 with lambda = 0):
//   L1_v = mean over the 3 M_v values of view v of |C - target|,
//   dL1_v/dC = sign(C - target) / (3 M_v), with sign(0) = 0.
// Every block covers kL1Pix pixels of a single view, so the per-view loss is a
// fixed-order FP64 sum of whole blocks: deterministic.
#include <cmath>

#include "internal.h"

namespace gsr {
namespace {

__device__ __forceinline__ int view_of_l1_block(const CamDev* cams, int n_views, uint32_t b)
{
    int v = 0;
    while (v + 1 < n_views && cams[v + 1].l1_base <= b) ++v;
    return v;
}

__device__ __forceinline__ double block_sum_f64(double x)
{
    __shared__ double s[kL1Block];
    s[threadIdx.x] = x;
    __syncthreads();
    for (int o = kL1Block / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    return s[0];
}

// sum over the block in a fixed order: lanes by xor-shuffle, then the 4 wavefronts
__device__ __forceinline__ double block_sum_f64_shfl(double x)
{
    __shared__ double s_w[kL1Block / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63u) == 0u) s_w[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kL1Block / 64; ++w) t += s_w[w];
    return t;
}

__global__ __launch_bounds__(kL1Block) void l1_kernel(const float* rgb, const float* target, const CamDev* cams,
                                                      int n_views, float weight, float* grad, double* block_sum)
{
    constexpr int kPer = kL1Pix / kL1Block;
    const uint32_t b = blockIdx.x;
    const int v = view_of_l1_block(cams, n_views, b);
    const CamDev& c = cams[v];
    const int64_t M = (int64_t)c.W * c.H;
    const int64_t q0 = (int64_t)(b - c.l1_base) * kL1Pix + threadIdx.x;   // pixels q0 + kL1Block k of the view
    const float inv = weight / (3.0f * (float)M);
    // every load before any store (a clamped index for pixels past the view's end)
    float d[kPer][3];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t q = q0 + (int64_t)k * kL1Block;
        const int64_t p = c.pix_base + (q < M ? q : M - 1);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) d[k][ch] = rgb[3 * p + ch] - target[3 * p + ch];
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t q = q0 + (int64_t)k * kL1Block;
        if (q >= M) continue;
        const int64_t p = c.pix_base + q;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float sg = d[k][ch] > 0.f ? 1.f : (d[k][ch] < 0.f ? -1.f : 0.f);
            if (grad) grad[3 * p + ch] = sg * inv;
            acc += (double)fabsf(d[k][ch]);
        }
    }
    const double tot = block_sum_f64_shfl(acc);
    if (threadIdx.x == 0) block_sum[b] = tot;
}

__global__ __launch_bounds__(kL1Block) void l1_reduce_kernel(const double* block_sum, const CamDev* cams, int n_views,
                                                             uint32_t n_blocks, float weight, float* loss)
{
    const int v = blockIdx.x;
    if (v >= n_views) return;
    const CamDev& c = cams[v];
    const uint32_t b0 = c.l1_base, b1 = (v + 1 < n_views) ? cams[v + 1].l1_base : n_blocks;
    double acc = 0.0;
    for (uint32_t b = b0 + threadIdx.x; b < b1; b += kL1Block) acc += block_sum[b];
    const double tot = block_sum_f64(acc);
    if (threadIdx.x == 0) loss[v] = (float)((double)weight * tot / (3.0 * (double)((int64_t)c.W * c.H)));
}

// Opacity regulariser of the comparison in Sec. 5.4 (ablation, opacity vs entropy
// constraint): L_O = w / n * sum_i exp(-(sigma_i - 0.5)^2 / 0.05), pushing
// opacities toward 0 or 1.  dL_O/dsigma_i = w / n * e_i * (-2 (sigma_i - 0.5) / 0.05)
// is added to grad[i].  Block partial sums in FP64, summed in a fixed order.
__global__ __launch_bounds__(kL1Block) void opacity_reg_kernel(const float* opac, int64_t n, float w, float* grad,
                                                               double* block_sum)
{
    const int64_t i = (int64_t)blockIdx.x * kL1Block + threadIdx.x;
    double acc = 0.0;
    if (i < n) {
        const float d = opac[i] - 0.5f;
        const float e = expf(-(d * d) * 20.0f);              // 1 / 0.05 = 20
        if (grad) grad[i] += (w / (float)n) * e * (-40.0f * d);
        acc = (double)e;
    }
    const double tot = block_sum_f64(acc);
    if (threadIdx.x == 0) block_sum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kL1Block) void opacity_reg_reduce_kernel(const double* block_sum, uint32_t n_blocks,
                                                                      int64_t n, float w, float* loss)
{
    double acc = 0.0;
    for (uint32_t b = threadIdx.x; b < n_blocks; b += kL1Block) acc += block_sum[b];
    const double tot = block_sum_f64(acc);
    if (threadIdx.x == 0) *loss = (float)((double)w * tot / (double)n);
}

// Scale reset (Sec. 4.2, Eq. 7): s <- zeta * s for every scale component, and
// log s <- log s + log zeta for an optimiser's log-scales (may be null).
__global__ void scale_reset_kernel(float* s, float* log_s, int64_t count, float zeta, float log_zeta)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        s[i] = zeta * s[i];
        if (log_s) log_s[i] = log_s[i] + log_zeta;
    }
}

}  // namespace

size_t opacity_reg_tmp_words(int64_t n) { return (size_t)((n + kL1Block - 1) / kL1Block) + 1; }

hipError_t launch_opacity_reg(const float* opac, int64_t n, float w, float* grad, float* loss, double* tmp,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const uint32_t nb = (uint32_t)((n + kL1Block - 1) / kL1Block);
    hipLaunchKernelGGL(opacity_reg_kernel, dim3(nb), dim3(kL1Block), 0, s, opac, n, w, grad, tmp);
    if (loss) hipLaunchKernelGGL(opacity_reg_reduce_kernel, dim3(1), dim3(kL1Block), 0, s, tmp, nb, n, w, loss);
    return hipGetLastError();
}

hipError_t launch_opacity_reg_reduce(const double* partial, uint32_t n_partial, int64_t n, float w, float* loss,
                                     hipStream_t s)
{
    if (n <= 0 || !loss) return hipSuccess;
    hipLaunchKernelGGL(opacity_reg_reduce_kernel, dim3(1), dim3(kL1Block), 0, s, partial, n_partial, n, w, loss);
    return hipGetLastError();
}

hipError_t launch_scale_reset(float* scales, float* log_scales, int64_t count, float zeta, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(scale_reset_kernel, dim3((unsigned)blocks), dim3(256), 0, s, scales, log_scales, count, zeta,
                       (float)std::log((double)zeta));
    return hipGetLastError();
}

hipError_t launch_l1(const float* rgb, const float* target, const CamDev* cams, int n_views, uint32_t n_l1_blocks,
                     float weight, float* grad, float* loss, double* tmp, hipStream_t s)
{
    if (n_l1_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(l1_kernel, dim3(n_l1_blocks), dim3(kL1Block), 0, s, rgb, target, cams, n_views, weight, grad,
                       tmp);
    if (loss)
        hipLaunchKernelGGL(l1_reduce_kernel, dim3(n_views), dim3(kL1Block), 0, s, tmp, cams, n_views, n_l1_blocks,
                           weight, loss);
    return hipGetLastError();
}

}  // namespace gsr
