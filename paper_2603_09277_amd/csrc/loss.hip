// L1 photometric term of the base loss (Sec. 3, Eq. 6 with lambda = 0):
//   L1_v = mean over the 3 M_v values of view v of |C - target|,
//   dL1_v/dC = sign(C - target) / (3 M_v), with sign(0) = 0.
// Per-block partial sums are reduced per view in a fixed order (FP64), so
// the loss value is deterministic.
#include "internal.h"

namespace gsr {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void l1_kernel(const float* rgb, const float* target, const CamDev* cams,
                                                      int n_views, int64_t n_pix, float* grad, double* block_sum)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    double acc = 0.0;
    if (p < n_pix) {
        int v = 0;
        while (v + 1 < n_views && cams[v + 1].pix_base <= p) ++v;
        const float inv = 1.0f / (3.0f * (float)((int64_t)cams[v].W * cams[v].H));
        for (int ch = 0; ch < 3; ++ch) {
            float d = rgb[3 * p + ch] - target[3 * p + ch];
            float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
            if (grad) grad[3 * p + ch] = sg * inv;
            acc += (double)fabsf(d);
        }
    }
    __shared__ double s[kThreads];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_sum[blockIdx.x] = s[0];
}

// one block per view: sum the partials of the blocks that lie in this view
__global__ __launch_bounds__(kThreads) void l1_reduce_kernel(const double* block_sum, const CamDev* cams, int n_views,
                                                             float* loss)
{
    const int v = blockIdx.x;
    if (v >= n_views) return;
    const CamDev& c = cams[v];
    const int64_t p0 = c.pix_base, p1 = c.pix_base + (int64_t)c.W * c.H;
    const int64_t b0 = p0 / kThreads, b1 = (p1 - 1) / kThreads;
    // a block that straddles two views is summed again pixel-exactly below; here only whole blocks
    double acc = 0.0;
    for (int64_t b = b0 + threadIdx.x; b <= b1; b += kThreads) {
        int64_t lo = b * kThreads, hi = lo + kThreads;
        if (lo >= p0 && hi <= p1) acc += block_sum[b];
    }
    __shared__ double s[kThreads];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[v] = (float)s[0];
}

// blocks that straddle a view boundary (at most the first and the last block
// of a view): add their pixels of this view one by one
__global__ void l1_edges_kernel(const float* rgb, const float* target, const CamDev* cams, int n_views, float* loss)
{
    const int v = blockIdx.x;
    if (v >= n_views || threadIdx.x != 0) return;
    const CamDev& c = cams[v];
    const int64_t p0 = c.pix_base, p1 = c.pix_base + (int64_t)c.W * c.H;
    const int64_t cand[2] = { p0 / kThreads, (p1 - 1) / kThreads };
    double acc = (double)loss[v];
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && cand[1] == cand[0]) break;
        const int64_t lo = cand[k] * kThreads, hi = lo + kThreads;
        if (lo >= p0 && hi <= p1) continue;                 // whole block: already in loss[v]
        const int64_t a = lo > p0 ? lo : p0, b = hi < p1 ? hi : p1;
        for (int64_t p = a; p < b; ++p)
            for (int ch = 0; ch < 3; ++ch) acc += (double)fabsf(rgb[3 * p + ch] - target[3 * p + ch]);
    }
    loss[v] = (float)(acc / (3.0 * (double)((int64_t)c.W * c.H)));
}

}  // namespace

size_t l1_tmp_doubles(int64_t n_pix) { return (size_t)((n_pix + kThreads - 1) / kThreads) + 1; }

hipError_t launch_l1(const float* rgb, const float* target, const CamDev* cams, int n_views, int64_t n_pix,
                     float* grad, float* loss, double* tmp, hipStream_t s)
{
    if (n_pix == 0) return hipSuccess;
    const int64_t nb = (n_pix + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(l1_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, rgb, target, cams, n_views, n_pix, grad, tmp);
    if (loss) {
        hipLaunchKernelGGL(l1_reduce_kernel, dim3(n_views), dim3(kThreads), 0, s, tmp, cams, n_views, loss);
        hipLaunchKernelGGL(l1_edges_kernel, dim3(n_views), dim3(64), 0, s, rgb, target, cams, n_views, loss);
    }
    return hipGetLastError();
}

}  // namespace gsr
