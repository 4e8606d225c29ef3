// Training-step terms around the rasterizer: the D-SSIM of the base loss
// (Sec. 3, Eq. 6) and a bias-corrected Adam step on raw parameters.
//
// SSIM follows the 3DGS lineage the paper builds on: per channel, local
// statistics over an 11x11 Gaussian window (sigma 1.5, normalised; zero outside
// the image), C1 = 0.01^2, C2 = 0.03^2,
//   S = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2)).
// The window is separable, so the five statistics take a horizontal and a
// vertical 11-tap pass; the gradient runs the same two passes over the three
// per-pixel partials (dS/dmx, dS/dE[x^2], dS/dE[xy]) -- the window is symmetric,
// so the adjoint of each pass is the pass itself -- and combines them as
//   dS/dx_q = W*(dS/dmx) + 2 x_q W*(dS/dExx) + y_q W*(dS/dExy).
#include <cmath>

#include "internal.h"

namespace gsr {
namespace {

constexpr int kTaps = 11;
constexpr int kHalf = 5;
constexpr int kThr = 256;

__constant__ float c_win[kTaps];

__device__ __forceinline__ double block_sum_f64(double x)
{
    __shared__ double s[kThr];
    s[threadIdx.x] = x;
    __syncthreads();
    for (int o = kThr / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    return s[0];
}

// horizontal pass of x, y, x^2, y^2, xy: st[p][15] = per channel (5 values)
__global__ __launch_bounds__(kThr) void ssim_rows_kernel(const float* x, const float* y, int W, int H, float* st)
{
    const int64_t p = (int64_t)blockIdx.x * kThr + threadIdx.x;
    if (p >= (int64_t)W * H) return;
    const int px = (int)(p % W);
    float acc[15];
#pragma unroll
    for (int k = 0; k < 15; ++k) acc[k] = 0.f;
    for (int b = -kHalf; b <= kHalf; ++b) {
        const int qx = px + b;
        if (qx < 0 || qx >= W) continue;
        const float w = c_win[b + kHalf];
        const int64_t q = p + b;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float xv = x[3 * q + ch], yv = y[3 * q + ch];
            acc[5 * ch + 0] = fmaf(w, xv, acc[5 * ch + 0]);
            acc[5 * ch + 1] = fmaf(w, yv, acc[5 * ch + 1]);
            acc[5 * ch + 2] = fmaf(w, xv * xv, acc[5 * ch + 2]);
            acc[5 * ch + 3] = fmaf(w, yv * yv, acc[5 * ch + 3]);
            acc[5 * ch + 4] = fmaf(w, xv * yv, acc[5 * ch + 4]);
        }
    }
#pragma unroll
    for (int k = 0; k < 15; ++k) st[15 * p + k] = acc[k];
}

// vertical pass, S and its partials; block sums of S (FP64)
__global__ __launch_bounds__(kThr) void ssim_map_kernel(const float* st, int W, int H, float* part, double* block_sum)
{
    const int64_t p = (int64_t)blockIdx.x * kThr + threadIdx.x;
    const int64_t M = (int64_t)W * H;
    double sacc = 0.0;
    if (p < M) {
        const int py = (int)(p / W);
        float s5[15];
#pragma unroll
        for (int k = 0; k < 15; ++k) s5[k] = 0.f;
        for (int a = -kHalf; a <= kHalf; ++a) {
            const int qy = py + a;
            if (qy < 0 || qy >= H) continue;
            const float w = c_win[a + kHalf];
            const int64_t q = p + (int64_t)a * W;
#pragma unroll
            for (int k = 0; k < 15; ++k) s5[k] = fmaf(w, st[15 * q + k], s5[k]);
        }
        const float C1 = 1e-4f, C2 = 9e-4f;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float mx = s5[5 * ch], my = s5[5 * ch + 1];
            const float sx = s5[5 * ch + 2] - mx * mx, sy = s5[5 * ch + 3] - my * my, sxy = s5[5 * ch + 4] - mx * my;
            const float ln = 2.f * mx * my + C1, ld = mx * mx + my * my + C1;
            const float cn = 2.f * sxy + C2, cd = sx + sy + C2;
            const float N = ln * cn, D = ld * cd;
            const float iD = 1.f / D;
            sacc += (double)(N * iD);
            const float dN = 2.f * my * (cn - ln), dD = 2.f * mx * (cd - ld);
            part[9 * p + 3 * ch + 0] = (dN - N * iD * dD) * iD;     // dS/dmx
            part[9 * p + 3 * ch + 1] = -N * ld * iD * iD;           // dS/dExx
            part[9 * p + 3 * ch + 2] = 2.f * ln * iD;               // dS/dExy
        }
    }
    const double tot = block_sum_f64(sacc);
    if (threadIdx.x == 0) block_sum[blockIdx.x] = tot;
}

// horizontal pass of the 9 partials
__global__ __launch_bounds__(kThr) void ssim_back_rows_kernel(const float* part, int W, int H, float* tmp)
{
    const int64_t p = (int64_t)blockIdx.x * kThr + threadIdx.x;
    if (p >= (int64_t)W * H) return;
    const int px = (int)(p % W);
    float acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.f;
    for (int b = -kHalf; b <= kHalf; ++b) {
        const int qx = px + b;
        if (qx < 0 || qx >= W) continue;
        const float w = c_win[b + kHalf];
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] = fmaf(w, part[9 * (p + b) + k], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) tmp[9 * p + k] = acc[k];
}

// vertical pass and the combination; grad += scale * dSSIM-sum/dx
__global__ __launch_bounds__(kThr) void ssim_back_cols_kernel(const float* tmp, const float* x, const float* y, int W,
                                                              int H, float scale, float* grad)
{
    const int64_t p = (int64_t)blockIdx.x * kThr + threadIdx.x;
    if (p >= (int64_t)W * H) return;
    const int py = (int)(p / W);
    float acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.f;
    for (int a = -kHalf; a <= kHalf; ++a) {
        const int qy = py + a;
        if (qy < 0 || qy >= H) continue;
        const float w = c_win[a + kHalf];
        const int64_t q = p + (int64_t)a * W;
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] = fmaf(w, tmp[9 * q + k], acc[k]);
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float d = acc[3 * ch] + 2.f * x[3 * p + ch] * acc[3 * ch + 1] + y[3 * p + ch] * acc[3 * ch + 2];
        grad[3 * p + ch] += scale * d;
    }
}

__global__ __launch_bounds__(kThr) void ssim_loss_kernel(const double* block_sum, uint32_t n_blocks, int64_t M,
                                                         float weight, float* loss)
{
    double acc = 0.0;
    for (uint32_t b = threadIdx.x; b < n_blocks; b += kThr) acc += block_sum[b];
    const double tot = block_sum_f64(acc);
    if (threadIdx.x == 0) *loss = (float)((double)weight * (1.0 - tot / (3.0 * (double)M)));
}

// one bias-corrected Adam step on raw parameters; kind 0 identity, 1 exp, 2 sigmoid
struct AdamParams {
    float lr, b1, b2, eps, c1, c2;     // c1, c2: the bias corrections 1 / (1 - b^step)
    int kind;                          // 0 identity, 1 exp, 2 sigmoid
};

// The sigmoid and its derivative from e = exp(-|r|), which never cancels:
// sigmoid(r) = 1 / (1 + e) for r >= 0 and e / (1 + e) below; sigmoid' = e / (1 + e)^2.
__device__ __forceinline__ float act_of(float r, int kind)
{
    if (kind == 1) return expf(r);
    if (kind == 2) {
        const float e = expf(-fabsf(r)), q = 1.f / (1.f + e);
        return r >= 0.f ? q : e * q;
    }
    return r;
}

__device__ __forceinline__ float dact_of(float r, int kind)
{
    if (kind == 1) return expf(r);
    if (kind == 2) {
        const float e = expf(-fabsf(r)), q = 1.f / (1.f + e);
        return e * q * q;
    }
    return 1.f;
}

__device__ __forceinline__ void adam_one(float& r, float& m, float& v, float& a, float ga, const AdamParams& p)
{
    const float g = ga * dact_of(r, p.kind);
    m = p.b1 * m + (1.f - p.b1) * g;
    v = p.b2 * v + (1.f - p.b2) * g * g;
    r = r - p.lr * (m * p.c1) / (sqrtf(v * p.c2) + p.eps);
    a = act_of(r, p.kind);
}

// Element-wise, HBM-bound: 16 B read and 12-16 B written per parameter.  VEC moves
// four parameters per lane with 16-byte accesses (all pointers 16-byte aligned);
// the last n % 4 go one per lane.
template <bool VEC>
__global__ void __launch_bounds__(256) adam_kernel(float* raw, float* m, float* v, float* act, const float* grad_act,
                                                   int64_t n, AdamParams p)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t done = 0;
    if (VEC) {
        const int64_t n4 = n >> 2;
        for (int64_t i = t0; i < n4; i += stride) {
            float4 r = reinterpret_cast<float4*>(raw)[i], mm = reinterpret_cast<float4*>(m)[i];
            float4 vv = reinterpret_cast<float4*>(v)[i];
            const float4 ga = reinterpret_cast<const float4*>(grad_act)[i];
            float4 a;
            adam_one(r.x, mm.x, vv.x, a.x, ga.x, p);
            adam_one(r.y, mm.y, vv.y, a.y, ga.y, p);
            adam_one(r.z, mm.z, vv.z, a.z, ga.z, p);
            adam_one(r.w, mm.w, vv.w, a.w, ga.w, p);
            reinterpret_cast<float4*>(raw)[i] = r;
            reinterpret_cast<float4*>(m)[i] = mm;
            reinterpret_cast<float4*>(v)[i] = vv;
            if (act) reinterpret_cast<float4*>(act)[i] = a;
        }
        done = n4 << 2;
    }
    for (int64_t i = done + t0; i < n; i += stride) {
        float r = raw[i], mm = m[i], vv = v[i], a;
        adam_one(r, mm, vv, a, grad_act[i], p);
        raw[i] = r;
        m[i] = mm;
        v[i] = vv;
        if (act) act[i] = a;
    }
}

bool g_win_ready[64] = {};

hipError_t upload_window()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < 64 && g_win_ready[dev]) return hipSuccess;
    float w[kTaps];
    double s = 0.0, g[kTaps];
    for (int k = 0; k < kTaps; ++k) { g[k] = std::exp(-(double)((k - kHalf) * (k - kHalf)) / (2.0 * 1.5 * 1.5)); s += g[k]; }
    for (int k = 0; k < kTaps; ++k) w[k] = (float)(g[k] / s);
    e = hipMemcpyToSymbol(HIP_SYMBOL(c_win), w, sizeof w, 0, hipMemcpyHostToDevice);
    if (e == hipSuccess && dev >= 0 && dev < 64) g_win_ready[dev] = true;
    return e;
}

}  // namespace

size_t ssim_tmp_bytes(int64_t M) { return (size_t)M * 4 * (15 + 9 + 9) + ((size_t)(M + kThr - 1) / kThr + 1) * 8 + 1024; }

hipError_t launch_dssim(const float* x, const float* y, int W, int H, float weight, float* grad, float* loss, void* tmp,
                        hipStream_t s)
{
    const int64_t M = (int64_t)W * H;
    if (M == 0) return hipSuccess;
    hipError_t e = upload_window();
    if (e != hipSuccess) return e;
    char* t = (char*)tmp;
    float* st = (float*)t;
    float* part = st + 15 * M;
    float* back = part + 9 * M;
    double* bsum = (double*)(((uintptr_t)(back + 9 * M) + 255) & ~(uintptr_t)255);
    const uint32_t nb = (uint32_t)((M + kThr - 1) / kThr);
    hipLaunchKernelGGL(ssim_rows_kernel, dim3(nb), dim3(kThr), 0, s, x, y, W, H, st);
    hipLaunchKernelGGL(ssim_map_kernel, dim3(nb), dim3(kThr), 0, s, st, W, H, part, bsum);
    if (loss) hipLaunchKernelGGL(ssim_loss_kernel, dim3(1), dim3(kThr), 0, s, bsum, nb, M, weight, loss);
    if (grad) {
        hipLaunchKernelGGL(ssim_back_rows_kernel, dim3(nb), dim3(kThr), 0, s, part, W, H, back);
        // L = weight (1 - SSIM), SSIM = sum S / (3 M)
        hipLaunchKernelGGL(ssim_back_cols_kernel, dim3(nb), dim3(kThr), 0, s, back, x, y, W, H,
                           -weight / (3.0f * (float)M), grad);
    }
    return hipGetLastError();
}

hipError_t launch_adam(float* raw, float* m, float* v, float* act, const float* grad_act, int64_t n, int kind,
                       float lr, float b1, float b2, float eps, int64_t step, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)step)));
    const AdamParams p{lr, b1, b2, eps, c1, c2, kind};
    auto a16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
    const bool vec = a16(raw) && a16(m) && a16(v) && a16(grad_act) && (!act || a16(act));
    int64_t blocks = ((vec ? (n + 3) / 4 : n) + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (vec)
        hipLaunchKernelGGL(adam_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, raw, m, v, act, grad_act, n, p);
    else
        hipLaunchKernelGGL(adam_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, raw, m, v, act, grad_act, n, p);
    return hipGetLastError();
}

}  // namespace gsr
