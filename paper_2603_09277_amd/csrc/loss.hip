// L1 photometric term of the base loss (Sec. 3, Eq. 6 with lambda = 0):
//   L1_v = mean over the 3 M_v values of view v of |C - target|,
//   dL1_v/dC = sign(C - target) / (3 M_v), with sign(0) = 0.
// Every block covers pixels of a single view, so the per-view loss is a fixed
// order FP64 sum of whole blocks: deterministic.
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

__global__ __launch_bounds__(kL1Block) void l1_kernel(const float* rgb, const float* target, const CamDev* cams,
                                                      int n_views, float* grad, double* block_sum)
{
    const uint32_t b = blockIdx.x;
    const int v = view_of_l1_block(cams, n_views, b);
    const CamDev& c = cams[v];
    const int64_t M = (int64_t)c.W * c.H;
    const int64_t q = (int64_t)(b - c.l1_base) * kL1Block + threadIdx.x;   // pixel within the view
    double acc = 0.0;
    if (q < M) {
        const int64_t p = c.pix_base + q;
        const float inv = 1.0f / (3.0f * (float)M);
        for (int ch = 0; ch < 3; ++ch) {
            const float d = rgb[3 * p + ch] - target[3 * p + ch];
            const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
            if (grad) grad[3 * p + ch] = sg * inv;
            acc += (double)fabsf(d);
        }
    }
    const double tot = block_sum_f64(acc);
    if (threadIdx.x == 0) block_sum[b] = tot;
}

__global__ __launch_bounds__(kL1Block) void l1_reduce_kernel(const double* block_sum, const CamDev* cams, int n_views,
                                                             uint32_t n_blocks, float* loss)
{
    const int v = blockIdx.x;
    if (v >= n_views) return;
    const CamDev& c = cams[v];
    const uint32_t b0 = c.l1_base, b1 = (v + 1 < n_views) ? cams[v + 1].l1_base : n_blocks;
    double acc = 0.0;
    for (uint32_t b = b0 + threadIdx.x; b < b1; b += kL1Block) acc += block_sum[b];
    const double tot = block_sum_f64(acc);
    if (threadIdx.x == 0) loss[v] = (float)(tot / (3.0 * (double)((int64_t)c.W * c.H)));
}

}  // namespace

hipError_t launch_l1(const float* rgb, const float* target, const CamDev* cams, int n_views, uint32_t n_l1_blocks,
                     float* grad, float* loss, double* tmp, hipStream_t s)
{
    if (n_l1_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(l1_kernel, dim3(n_l1_blocks), dim3(kL1Block), 0, s, rgb, target, cams, n_views, grad, tmp);
    if (loss)
        hipLaunchKernelGGL(l1_reduce_kernel, dim3(n_views), dim3(kL1Block), 0, s, tmp, cams, n_views, n_l1_blocks,
                           loss);
    return hipGetLastError();
}

}  // namespace gsr
