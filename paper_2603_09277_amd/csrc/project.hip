// EWA projection of 3D Gaussians (Sec. 3, Eq. 1-2) and its backward.
//
// One thread per Gaussian; the thread loops over the views of the launch so
// that parameters and SH coefficients are read from HBM once per Gaussian,
// not once per (view, Gaussian).  Everything is FP32 except the 2x2
// determinant / inverse / eigenvalue step, which runs in FP64: near-degenerate
// 2D covariances lose all significant digits of det = ac - b^2 in FP32.
#include "internal.h"

namespace gsr {
namespace {

constexpr uint32_t F_DILATE = 1u, F_JCLAMP = 2u, F_CCLAMP = 4u;

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x40u);   // keep NaN quiet
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// Real spherical harmonics without the Condon-Shortley phase, ordered
// k = l*l + l + m; the coefficients are sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!)
// (times sqrt 2 for m != 0) folded into the polynomial of each (l, m).
constexpr float kC0 = 0.28209479177387814f;
constexpr float kC1 = 0.4886025119029199f;
constexpr float kC2a = 1.0925484305920792f;    // xy, yz, xz
constexpr float kC2b = 0.31539156525252005f;   // 3z^2 - 1
constexpr float kC2c = 0.5462742152960396f;    // x^2 - y^2
constexpr float kC3a = 0.5900435899266435f;    // y(3x^2 - y^2), x(x^2 - 3y^2)
constexpr float kC3b = 2.890611442640554f;     // xyz
constexpr float kC3c = 0.4570457994644658f;    // y(5z^2 - 1), x(5z^2 - 1)
constexpr float kC3d = 0.3731763325901154f;    // z(5z^2 - 3)
constexpr float kC3e = 1.445305721320277f;     // z(x^2 - y^2)

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y)
{
    Y[0] = kC0;
    if constexpr (DEG >= 1) { Y[1] = kC1 * y; Y[2] = kC1 * z; Y[3] = kC1 * x; }
    if constexpr (DEG >= 2) {
        float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = kC2a * x * y;
        Y[5] = kC2a * y * z;
        Y[6] = kC2b * (3.f * zz - 1.f);
        Y[7] = kC2a * x * z;
        Y[8] = kC2c * (xx - yy);
        if constexpr (DEG >= 3) {
            Y[9] = kC3a * y * (3.f * xx - yy);
            Y[10] = kC3b * x * y * z;
            Y[11] = kC3c * y * (5.f * zz - 1.f);
            Y[12] = kC3d * z * (5.f * zz - 3.f);
            Y[13] = kC3c * x * (5.f * zz - 1.f);
            Y[14] = kC3e * z * (xx - yy);
            Y[15] = kC3a * x * (xx - 3.f * yy);
        }
    }
}

// d/d(x, y, z) of sum_k w_k Y_k(x, y, z) (partials of the polynomials above)
template <int DEG>
__device__ __forceinline__ float3 sh_basis_grad(float x, float y, float z, const float* w)
{
    float gx = 0.f, gy = 0.f, gz = 0.f;
    if constexpr (DEG >= 1) { gy += kC1 * w[1]; gz += kC1 * w[2]; gx += kC1 * w[3]; }
    if constexpr (DEG >= 2) {
        gx += kC2a * y * w[4]; gy += kC2a * x * w[4];
        gy += kC2a * z * w[5]; gz += kC2a * y * w[5];
        gz += 6.f * kC2b * z * w[6];
        gx += kC2a * z * w[7]; gz += kC2a * x * w[7];
        gx += 2.f * kC2c * x * w[8]; gy -= 2.f * kC2c * y * w[8];
        if constexpr (DEG >= 3) {
            float xx = x * x, yy = y * y, zz = z * z;
            gx += 6.f * kC3a * x * y * w[9];          gy += 3.f * kC3a * (xx - yy) * w[9];
            gx += kC3b * y * z * w[10];               gy += kC3b * x * z * w[10];     gz += kC3b * x * y * w[10];
            gy += kC3c * (5.f * zz - 1.f) * w[11];    gz += 10.f * kC3c * y * z * w[11];
            gz += kC3d * (15.f * zz - 3.f) * w[12];
            gx += kC3c * (5.f * zz - 1.f) * w[13];    gz += 10.f * kC3c * x * z * w[13];
            gx += 2.f * kC3e * x * z * w[14];         gy -= 2.f * kC3e * y * z * w[14]; gz += kC3e * (xx - yy) * w[14];
            gx += 3.f * kC3a * (xx - yy) * w[15];     gy -= 6.f * kC3a * x * y * w[15];
        }
    }
    return make_float3(gx, gy, gz);
}

// Rotation matrix (row-major) of the unit quaternion (w, x, y, z).
__device__ __forceinline__ void quat_to_rot(float w, float x, float y, float z, float* R)
{
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
}

template <int K, bool BF16>
__device__ __forceinline__ void load_sh(const void* sh, uint32_t i, float* out)
{
    if constexpr (BF16) {
        const uint16_t* p = reinterpret_cast<const uint16_t*>(sh) + (size_t)i * (K * 3);
#pragma unroll
        for (int k = 0; k < K * 3; ++k) out[k] = bf16_to_f32(p[k]);
    } else {
        const float* p = reinterpret_cast<const float*>(sh) + (size_t)i * (K * 3);
#pragma unroll
        for (int k = 0; k < K * 3; ++k) out[k] = p[k];
    }
}

__device__ __forceinline__ bool finite3(float a, float b, float c) { return isfinite(a) && isfinite(b) && isfinite(c); }

// Per-Gaussian, view-independent state: normalised quaternion, rotation,
// 3D covariance (upper triangle 00 01 02 11 12 22).
struct Local {
    bool ok;
    float qn[4], qnorm;
    float R[9];
    float S[6];
};

__device__ __forceinline__ void local_state(const float* mu, const float* s, const float* q, float op,
                                            const float* sh, int nsh, Local& L)
{
    bool ok = finite3(mu[0], mu[1], mu[2]) && finite3(s[0], s[1], s[2]) && finite3(q[0], q[1], q[2]) &&
              isfinite(q[3]) && isfinite(op);
    for (int k = 0; k < nsh; ++k) ok = ok && isfinite(sh[k]);
    float qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    ok = ok && qn2 > 0.f;
    float qn = sqrtf(qn2);
    L.qnorm = qn;
    float iq = ok ? 1.f / qn : 0.f;
    for (int k = 0; k < 4; ++k) L.qn[k] = q[k] * iq;
    quat_to_rot(L.qn[0], L.qn[1], L.qn[2], L.qn[3], L.R);
    float s2[3] = { s[0] * s[0], s[1] * s[1], s[2] * s[2] };
    const float* R = L.R;
    // Sigma = R diag(s^2) R^T  (Eq. 1)
    L.S[0] = R[0] * R[0] * s2[0] + R[1] * R[1] * s2[1] + R[2] * R[2] * s2[2];
    L.S[1] = R[0] * R[3] * s2[0] + R[1] * R[4] * s2[1] + R[2] * R[5] * s2[2];
    L.S[2] = R[0] * R[6] * s2[0] + R[1] * R[7] * s2[1] + R[2] * R[8] * s2[2];
    L.S[3] = R[3] * R[3] * s2[0] + R[4] * R[4] * s2[1] + R[5] * R[5] * s2[2];
    L.S[4] = R[3] * R[6] * s2[0] + R[4] * R[7] * s2[1] + R[5] * R[8] * s2[2];
    L.S[5] = R[6] * R[6] * s2[0] + R[7] * R[7] * s2[1] + R[8] * R[8] * s2[2];
    L.ok = ok;
}

// Per-(view, Gaussian) projection state shared by forward and backward.
struct ViewProj {
    bool ok;
    float tx, ty, tz, u, v, uc, vc;
    bool clx, cly;
    float J00, J02, J11, J12;
    float Tm[6];          // J Rc, 2x3
    float W[6];           // Tm Sigma, 2x3
    double a, b, c, det;  // dilated 2D covariance and its determinant
    double qA, qB, qC;    // conic (inverse)
    float mx, my;
};

__device__ __forceinline__ void view_proj(const CamDev& c, const float* mu, const Local& L, uint32_t flags,
                                          ViewProj& P)
{
    P.ok = false;
    // Camera transform, perspective divide and 2D mean in FP64 (unfused, in a
    // fixed order): the float32 results are then the correctly rounded values
    // of the exact ones, so the depth key and the tile rectangle of a Gaussian
    // do not depend on FP32 cancellation in R mu + t.
    double t3[3];
    for (int r = 0; r < 3; ++r)
        t3[r] = __dadd_rn(__dadd_rn(__dadd_rn(__dmul_rn((double)c.R[3 * r], (double)mu[0]),
                                              __dmul_rn((double)c.R[3 * r + 1], (double)mu[1])),
                                    __dmul_rn((double)c.R[3 * r + 2], (double)mu[2])),
                          (double)c.t[r]);
    P.tx = (float)t3[0]; P.ty = (float)t3[1]; P.tz = (float)t3[2];
    if (!L.ok || !(t3[2] > (double)c.near_z)) return;
    const double du = t3[0] / t3[2], dv = t3[1] / t3[2];
    P.u = (float)du;
    P.v = (float)dv;
    P.uc = P.u; P.vc = P.v; P.clx = false; P.cly = false;
    if (flags & F_JCLAMP) {
        if (du > c.limx_d) { P.uc = c.limx; P.clx = true; }
        if (du < -c.limx_d) { P.uc = -c.limx; P.clx = true; }
        if (dv > c.limy_d) { P.vc = c.limy; P.cly = true; }
        if (dv < -c.limy_d) { P.vc = -c.limy; P.cly = true; }
    }
    P.mx = (float)__dadd_rn(__dmul_rn((double)c.fx, du), (double)c.cx);
    P.my = (float)__dadd_rn(__dmul_rn((double)c.fy, dv), (double)c.cy);
    float iz = 1.f / P.tz;
    P.J00 = c.fx * iz; P.J02 = -c.fx * P.uc * iz;
    P.J11 = c.fy * iz; P.J12 = -c.fy * P.vc * iz;
    for (int j = 0; j < 3; ++j) {
        P.Tm[j] = P.J00 * c.R[j] + P.J02 * c.R[6 + j];
        P.Tm[3 + j] = P.J11 * c.R[3 + j] + P.J12 * c.R[6 + j];
    }
    const float* S = L.S;
    for (int r = 0; r < 2; ++r) {
        const float* T = P.Tm + 3 * r;
        P.W[3 * r + 0] = T[0] * S[0] + T[1] * S[1] + T[2] * S[2];
        P.W[3 * r + 1] = T[0] * S[1] + T[1] * S[3] + T[2] * S[4];
        P.W[3 * r + 2] = T[0] * S[2] + T[1] * S[4] + T[2] * S[5];
    }
    float dil = (flags & F_DILATE) ? 0.3f : 0.f;
    float ca = P.W[0] * P.Tm[0] + P.W[1] * P.Tm[1] + P.W[2] * P.Tm[2] + dil;
    float cb = P.W[0] * P.Tm[3] + P.W[1] * P.Tm[4] + P.W[2] * P.Tm[5];
    float cc = P.W[3] * P.Tm[3] + P.W[4] * P.Tm[4] + P.W[5] * P.Tm[5] + dil;
    // FP64: determinant and inverse of the 2x2 covariance
    P.a = ca; P.b = cb; P.c = cc;
    P.det = P.a * P.c - P.b * P.b;
    if (!(P.det > 0.0)) return;
    double id = 1.0 / P.det;
    P.qA = P.c * id; P.qB = -P.b * id; P.qC = P.a * id;
    P.ok = true;
}

// The forward reads the cameras of a launch from LDS, kCamChunk at a time: read
// from global memory in its view loop, a camera became vector loads, whose wait
// (the shared vector-memory counter) also waited for the previous view's stores.
// The backward stores nothing in its view loop and reads them with scalar loads.
constexpr int kCamChunk = 16;
static_assert(sizeof(CamDev) % 4 == 0, "cameras are copied in 4-byte words");

// cameras [v0, v0 + nv) into s_cam, by the whole workgroup (a barrier before and after)
__device__ __forceinline__ void stage_cams(CamDev* s_cam, const CamDev* cams, int v0, int nv)
{
    __syncthreads();
    const uint32_t* src = reinterpret_cast<const uint32_t*>(cams + v0);
    uint32_t* dst = reinterpret_cast<uint32_t*>(s_cam);
    const uint32_t words = (uint32_t)nv * (uint32_t)(sizeof(CamDev) / 4);
    for (uint32_t w = threadIdx.x; w < words; w += blockDim.x) dst[w] = src[w];
    __syncthreads();
}

// ONE: a launch of one view (a constant view count; fewer registers)
template <int DEG, bool BF16, bool ONE>
__global__ __launch_bounds__(256) void project_fwd_kernel(ProjectFwdArgs a)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    __shared__ CamDev s_cam[kCamChunk];
    const uint32_t i0 = blockIdx.x * 256u + threadIdx.x;
    const bool active = i0 < a.n;
    const uint32_t i = active ? i0 : a.n - 1u;               // past the end: only helps stage the cameras
    float mu[3] = { a.means[3 * (size_t)i], a.means[3 * (size_t)i + 1], a.means[3 * (size_t)i + 2] };
    float s[3] = { a.scales[3 * (size_t)i], a.scales[3 * (size_t)i + 1], a.scales[3 * (size_t)i + 2] };
    float q[4] = { a.quats[4 * (size_t)i], a.quats[4 * (size_t)i + 1], a.quats[4 * (size_t)i + 2], a.quats[4 * (size_t)i + 3] };
    float op = a.opac[i];
    float sh[K * 3];
    load_sh<K, BF16>(a.sh, i, sh);
    Local L;
    local_state(mu, s, q, op, sh, K * 3, L);
    const int tsx = a.tile_shift_x, tsy = a.tile_shift_y;
    const int n_views = ONE ? 1 : a.n_views;
    for (int v0 = 0; v0 < n_views; v0 += kCamChunk) {
    const int nv = n_views - v0 < kCamChunk ? n_views - v0 : kCamChunk;
    stage_cams(s_cam, a.cams, v0, nv);
    if (!active) continue;
    for (int v = v0; v < v0 + nv; ++v) {
        const CamDev& c = s_cam[v - v0];
        size_t o = (size_t)v * a.n + i;
        ViewProj P;
        view_proj(c, mu, L, a.flags, P);
        uint32_t tt = 0;
        int32_t rad = 0;
        uint2 rc = make_uint2(1u, 1u);                      // empty: x1 < x0 and y1 < y0
        float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
        if (P.ok) {
            double mid = 0.5 * (P.a + P.c);
            double disc = mid * mid - P.det;
            double lam = mid + sqrt(disc > 0.0 ? disc : 0.0);
            double rr = ceil(3.0 * sqrt(lam));
            rad = rr > 1073741824.0 ? 1073741824 : (int32_t)rr;
            // tile rectangle of [mean - r, mean + r]; floor(mean) is exact in FP32
            float fx = fminf(fmaxf(floorf(P.mx), -1e9f), 1e9f);
            float fy = fminf(fmaxf(floorf(P.my), -1e9f), 1e9f);
            int64_t ix = (int64_t)fx, iy = (int64_t)fy;
            int64_t x0 = (ix - rad) >> tsx, x1 = (ix + rad) >> tsx;
            int64_t y0 = (iy - rad) >> tsy, y1 = (iy + rad) >> tsy;
            x0 = x0 < 0 ? 0 : x0;
            y0 = y0 < 0 ? 0 : y0;
            x1 = x1 > c.gx - 1 ? c.gx - 1 : x1;
            y1 = y1 > c.gy - 1 ? c.gy - 1 : y1;
            if (rad > 0 && x0 <= x1 && y0 <= y1) {
                tt = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
                rc = make_uint2((uint32_t)x0 | ((uint32_t)x1 << 16), (uint32_t)y0 | ((uint32_t)y1 << 16));
            }
            // colour along the viewing direction
            float dx = mu[0] - c.campos[0], dy = mu[1] - c.campos[1], dz = mu[2] - c.campos[2];
            float idn = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
            float Y[K];
            sh_basis<DEG>(dx * idn, dy * idn, dz * idn, Y);
            float col[3];
            for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < K; ++k) acc += Y[k] * sh[3 * k + ch];
                acc += 0.5f;
                if ((a.flags & F_CCLAMP) && acc < 0.f) acc = 0.f;
                col[ch] = acc;
            }
            const float A2 = (float)(-0.5 * kLog2e * P.qA), B2 = (float)(-kLog2e * P.qB);
            const float C2 = (float)(-0.5 * kLog2e * P.qC);
            r0 = make_float4(P.mx, P.my, A2, B2);
            r1 = make_float4(C2, op, col[0], col[1]);
            // Cull level for the blend: alpha < 1/255 wherever the exponent is
            // below -L, L = log2(255 opacity) + 1e-4; and the slopes of the exponent's
            // ridge lines, where its maximum along a pixel row / column lies (dy = k dx
            // with k = -B'/(2C'), dx = k' dy with k' = -B'/(2A')).
            const double Lc = op > 0.f ? log2(255.0 * (double)op) + 1e-4 : -HUGE_VAL;
            const float kr = (float)(-(double)B2 / (2.0 * (double)C2));
            const float kc = (float)(-(double)B2 / (2.0 * (double)A2));
            r2 = make_float4(col[2], (float)Lc, kr, kc);
        }
        a.rec[3 * o + 0] = r0;
        a.rec[3 * o + 1] = r1;
        a.rec[3 * o + 2] = r2;
        a.depth_key[o] = P.ok ? __float_as_uint(P.tz) : 0xffffffffu;
        a.depth[o] = P.tz;
        a.trect[o] = rc;
        a.tiles_touched[o] = tt;
        a.radius[o] = P.ok ? rad : 0;
    }
    }
}

// ONE: a launch of one view. The view loop then has a constant trip count and the
// kernel fits three wavefronts a SIMD (168 VGPRs; the compiler spills a few bytes)
// instead of two.
template <int DEG, bool BF16, bool ONE>
__device__ __forceinline__ void project_bwd_one(const ProjectBwdArgs& a, uint32_t i)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    float mu[3] = { a.means[3 * (size_t)i], a.means[3 * (size_t)i + 1], a.means[3 * (size_t)i + 2] };
    float s[3] = { a.scales[3 * (size_t)i], a.scales[3 * (size_t)i + 1], a.scales[3 * (size_t)i + 2] };
    float q[4] = { a.quats[4 * (size_t)i], a.quats[4 * (size_t)i + 1], a.quats[4 * (size_t)i + 2], a.quats[4 * (size_t)i + 3] };
    float op = a.opac[i];
    float sh[K * 3];
    load_sh<K, BF16>(a.sh, i, sh);
    Local L;
    local_state(mu, s, q, op, sh, K * 3, L);

    float gmu[3] = { 0.f, 0.f, 0.f };
    float gS[6] = { 0.f, 0.f, 0.f, 0.f, 0.f, 0.f };   // symmetric dL/dSigma, upper triangle
    float gop = 0.f;
    float gsh[K * 3];
#pragma unroll
    for (int k = 0; k < K * 3; ++k) gsh[k] = 0.f;

    // this view's row stamp and 2D gradient row: a row whose stamp is not this frame's
    // is zero (no pixel blended any of its pairs, or the record has no pairs) and is not
    // read.  Stamps are loaded two views ahead, so that the row of the next view is
    // loaded (one view ahead) only where its stamp is this frame's.
    const uint32_t st = *a.stamp;
    const int n_views = ONE ? 1 : a.n_views;
    uint32_t rs_n = n_views > 0 ? a.rec_stamp[i] : 0u;
    uint32_t rs_nn = n_views > 1 ? a.rec_stamp[(size_t)a.n + i] : 0u;
    float g_n[kG2];
#pragma unroll
    for (int k = 0; k < kG2; ++k) g_n[k] = 0.f;
    if (rs_n == st) {
#pragma unroll
        for (int k = 0; k < kG2; ++k) g_n[k] = a.grad2d[(size_t)kG2 * i + k];
    }
    for (int v = 0; v < n_views; ++v) {
        const uint32_t rs_v = rs_n;
        float g[kG2];
#pragma unroll
        for (int k = 0; k < kG2; ++k) g[k] = g_n[k];
        rs_n = rs_nn;
        if (v + 1 < n_views && rs_n == st) {
            const size_t o = (size_t)(v + 1) * a.n + i;
#pragma unroll
            for (int k = 0; k < kG2; ++k) g_n[k] = a.grad2d[(size_t)kG2 * o + k];
        }
        if (v + 2 < n_views) rs_nn = a.rec_stamp[(size_t)(v + 2) * a.n + i];
        if (rs_v != st) continue;                           // zero gradient from this view
        const CamDev& c = a.cams[v];                        // scalar loads here (unlike the forward)
        ViewProj P;
        view_proj(c, mu, L, a.flags, P);
        if (!P.ok) continue;
        float gmx = g[0], gmy = g[1], gA = g[2], gB = g[3], gC = g[4];
        gop += g[5];
        // ---- colour -> SH coefficients and viewing direction
        float dx = mu[0] - c.campos[0], dy = mu[1] - c.campos[1], dz = mu[2] - c.campos[2];
        float dn = sqrtf(dx * dx + dy * dy + dz * dz);
        float idn = 1.f / dn;
        float d0 = dx * idn, d1 = dy * idn, d2 = dz * idn;
        float Y[K];
        sh_basis<DEG>(d0, d1, d2, Y);
        float gcol[3];
        for (int ch = 0; ch < 3; ++ch) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) acc += Y[k] * sh[3 * k + ch];
            acc += 0.5f;
            bool clamped = (a.flags & F_CCLAMP) && acc < 0.f;
            gcol[ch] = clamped ? 0.f : g[6 + ch];
        }
        float wk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            wk[k] = sh[3 * k] * gcol[0] + sh[3 * k + 1] * gcol[1] + sh[3 * k + 2] * gcol[2];
            gsh[3 * k + 0] += Y[k] * gcol[0];
            gsh[3 * k + 1] += Y[k] * gcol[1];
            gsh[3 * k + 2] += Y[k] * gcol[2];
        }
        if constexpr (DEG > 0) {
            float3 gd = sh_basis_grad<DEG>(d0, d1, d2, wk);
            float dd = d0 * gd.x + d1 * gd.y + d2 * gd.z;
            gmu[0] += (gd.x - d0 * dd) * idn;
            gmu[1] += (gd.y - d1 * dd) * idn;
            gmu[2] += (gd.z - d2 * dd) * idn;
        }
        // ---- conic -> 2D covariance (FP64): dL/dSigma' = -Q G Q, G the symmetric gradient of Q
        double hB = 0.5 * (double)gB;
        double QG00 = P.qA * gA + P.qB * hB, QG01 = P.qA * hB + P.qB * gC;
        double QG10 = P.qB * gA + P.qC * hB, QG11 = P.qB * hB + P.qC * gC;
        float g00 = (float)(-(QG00 * P.qA + QG01 * P.qB));
        float g01 = (float)(-(QG00 * P.qB + QG01 * P.qC));
        float g11 = (float)(-(QG10 * P.qB + QG11 * P.qC));
        // ---- Sigma' = Tm Sigma Tm^T: dL/dSigma += Tm^T GS Tm ; dL/dTm = 2 GS Tm Sigma = 2 GS W
        const float* T0 = P.Tm;
        const float* T1 = P.Tm + 3;
        int idx = 0;
        for (int k = 0; k < 3; ++k)
            for (int l = k; l < 3; ++l, ++idx)
                gS[idx] += g00 * T0[k] * T0[l] + g01 * (T0[k] * T1[l] + T1[k] * T0[l]) + g11 * T1[k] * T1[l];
        float gTm[6];
        for (int j = 0; j < 3; ++j) {
            gTm[j] = 2.f * (g00 * P.W[j] + g01 * P.W[3 + j]);
            gTm[3 + j] = 2.f * (g01 * P.W[j] + g11 * P.W[3 + j]);
        }
        // dL/dJ = dL/dTm Rc^T (only the four non-zero entries of J matter)
        float gJ00 = gTm[0] * c.R[0] + gTm[1] * c.R[1] + gTm[2] * c.R[2];
        float gJ02 = gTm[0] * c.R[6] + gTm[1] * c.R[7] + gTm[2] * c.R[8];
        float gJ11 = gTm[3] * c.R[3] + gTm[4] * c.R[4] + gTm[5] * c.R[5];
        float gJ12 = gTm[3] * c.R[6] + gTm[4] * c.R[7] + gTm[5] * c.R[8];
        // ---- J and the 2D mean -> camera-space position
        float iz = 1.f / P.tz, iz2 = iz * iz;
        float gtx = 0.f, gty = 0.f, gtz = 0.f;
        gtz += -(gJ00 * c.fx + gJ11 * c.fy) * iz2;
        if (!P.clx) { gtx += -gJ02 * c.fx * iz2; gtz += 2.f * gJ02 * c.fx * P.tx * iz2 * iz; }
        else        { gtz += gJ02 * c.fx * P.uc * iz2; }
        if (!P.cly) { gty += -gJ12 * c.fy * iz2; gtz += 2.f * gJ12 * c.fy * P.ty * iz2 * iz; }
        else        { gtz += gJ12 * c.fy * P.vc * iz2; }
        gtx += gmx * c.fx * iz;
        gty += gmy * c.fy * iz;
        gtz -= (gmx * c.fx * P.tx + gmy * c.fy * P.ty) * iz2;
        gmu[0] += c.R[0] * gtx + c.R[3] * gty + c.R[6] * gtz;
        gmu[1] += c.R[1] * gtx + c.R[4] * gty + c.R[7] * gtz;
        gmu[2] += c.R[2] * gtx + c.R[5] * gty + c.R[8] * gtz;
    }

    // ---- Sigma = M M^T with M = R diag(s):  dL/dM = 2 G M
    float G[9] = { gS[0], gS[1], gS[2], gS[1], gS[3], gS[4], gS[2], gS[4], gS[5] };
    const float* R = L.R;
    float M[9];
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j) M[3 * r + j] = R[3 * r + j] * s[j];
    float gR[9], gs[3] = { 0.f, 0.f, 0.f };
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j) {
            float gm = 2.f * (G[3 * r] * M[j] + G[3 * r + 1] * M[3 + j] + G[3 * r + 2] * M[6 + j]);
            gs[j] += gm * R[3 * r + j];
            gR[3 * r + j] = gm * s[j];
        }
    // ---- rotation -> normalised quaternion -> raw quaternion
    float w = L.qn[0], x = L.qn[1], y = L.qn[2], z = L.qn[3];
    float gw = 2.f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    float gx = 2.f * (y * gR[1] + z * gR[2] + y * gR[3] - w * gR[5] + z * gR[6] + w * gR[7]) -
               4.f * x * (gR[4] + gR[8]);
    float gy = 2.f * (x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] + z * gR[7]) -
               4.f * y * (gR[0] + gR[8]);
    float gz = 2.f * (-w * gR[1] + x * gR[2] + w * gR[3] + y * gR[5] + x * gR[6] + y * gR[7]) -
               4.f * z * (gR[0] + gR[4]);
    float qd = w * gw + x * gx + y * gy + z * gz;
    float iq = L.ok ? 1.f / L.qnorm : 0.f;

    bool any = L.ok;
    a.g_means[3 * (size_t)i + 0] = any ? gmu[0] : 0.f;
    a.g_means[3 * (size_t)i + 1] = any ? gmu[1] : 0.f;
    a.g_means[3 * (size_t)i + 2] = any ? gmu[2] : 0.f;
    a.g_scales[3 * (size_t)i + 0] = any ? gs[0] : 0.f;
    a.g_scales[3 * (size_t)i + 1] = any ? gs[1] : 0.f;
    a.g_scales[3 * (size_t)i + 2] = any ? gs[2] : 0.f;
    a.g_quats[4 * (size_t)i + 0] = any ? (gw - w * qd) * iq : 0.f;
    a.g_quats[4 * (size_t)i + 1] = any ? (gx - x * qd) * iq : 0.f;
    a.g_quats[4 * (size_t)i + 2] = any ? (gy - y * qd) * iq : 0.f;
    a.g_quats[4 * (size_t)i + 3] = any ? (gz - z * qd) * iq : 0.f;
    {
        float go = any ? gop : 0.f;
        if (a.reg_w != 0.f) {                                // + dL_O/dsigma, as a separate pass would add it
            const float d = op - 0.5f;
            const float e = expf(-(d * d) * 20.0f);
            go += (a.reg_w / (float)a.n) * e * (-40.0f * d);
        }
        a.g_opac[i] = go;
    }
    if constexpr (BF16) {
        uint16_t* p = reinterpret_cast<uint16_t*>(a.g_sh) + (size_t)i * (K * 3);
        if constexpr ((K * 3) % 8 == 0) {                    // eight values a 16-byte store
            uint32_t w[K * 3 / 2];
#pragma unroll
            for (int k = 0; k < K * 3; k += 2)
                w[k / 2] = (uint32_t)f32_to_bf16_rne(any ? gsh[k] : 0.f) |
                           ((uint32_t)f32_to_bf16_rne(any ? gsh[k + 1] : 0.f) << 16);
            if ((reinterpret_cast<uintptr_t>(a.g_sh) & 15u) == 0u) {
                uint4* p4 = reinterpret_cast<uint4*>(p);
#pragma unroll
                for (int k = 0; k < K * 3 / 8; ++k)
                    p4[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
            } else {
#pragma unroll
                for (int k = 0; k < K * 3; ++k) p[k] = (uint16_t)(w[k / 2] >> (16 * (k & 1)));
            }
        } else {
#pragma unroll
            for (int k = 0; k < K * 3; ++k) p[k] = f32_to_bf16_rne(any ? gsh[k] : 0.f);
        }
    } else {
        float* p = reinterpret_cast<float*>(a.g_sh) + (size_t)i * (K * 3);
#pragma unroll
        for (int k = 0; k < K * 3; ++k) p[k] = any ? gsh[k] : 0.f;
    }
}

template <int DEG, bool BF16, bool ONE>
__global__ __launch_bounds__(256, ONE ? 3 : 1) void project_bwd_kernel(ProjectBwdArgs a)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    // the opacity regulariser's loss (Sec. 5.4 ablation): per-wavefront FP64 sums of
    // exp(-(sigma - 0.5)^2 / 0.05), in a fixed order, for a fixed-order final sum; stored
    // after the gradients (with a store ahead of the view loop, some camera fields in it
    // became vector loads that waited on memory: 0.52 -> 0.62 ms on the 8-view workload)
    double e = 0.0;
    if (a.reg_partial && i < a.n) {
        const float d = a.opac[i] - 0.5f;
        e = (double)expf(-(d * d) * 20.0f);                  // 1 / 0.05 = 20
    }
    if (i < a.n) project_bwd_one<DEG, BF16, ONE>(a, i);
    if (a.reg_partial) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
        if ((threadIdx.x & 63u) == 0u) a.reg_partial[4u * blockIdx.x + (threadIdx.x >> 6)] = e;
    }
}

template <int DEG, bool BF16>
hipError_t fwd_dispatch(const ProjectFwdArgs& a, hipStream_t s)
{
    dim3 grid((a.n + 255u) / 256u);
    if (a.n_views == 1) hipLaunchKernelGGL((project_fwd_kernel<DEG, BF16, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((project_fwd_kernel<DEG, BF16, false>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int DEG, bool BF16>
hipError_t bwd_dispatch(const ProjectBwdArgs& a, hipStream_t s)
{
    dim3 grid((a.n + 255u) / 256u);
    if (a.n_views == 1) hipLaunchKernelGGL((project_bwd_kernel<DEG, BF16, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((project_bwd_kernel<DEG, BF16, false>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_project_fwd(const ProjectFwdArgs& a, int deg, bool bf16, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    switch (deg * 2 + (bf16 ? 1 : 0)) {
        case 0: return fwd_dispatch<0, false>(a, s);
        case 1: return fwd_dispatch<0, true>(a, s);
        case 2: return fwd_dispatch<1, false>(a, s);
        case 3: return fwd_dispatch<1, true>(a, s);
        case 4: return fwd_dispatch<2, false>(a, s);
        case 5: return fwd_dispatch<2, true>(a, s);
        case 6: return fwd_dispatch<3, false>(a, s);
        case 7: return fwd_dispatch<3, true>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_project_bwd(const ProjectBwdArgs& a, int deg, bool bf16, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    switch (deg * 2 + (bf16 ? 1 : 0)) {
        case 0: return bwd_dispatch<0, false>(a, s);
        case 1: return bwd_dispatch<0, true>(a, s);
        case 2: return bwd_dispatch<1, false>(a, s);
        case 3: return bwd_dispatch<1, true>(a, s);
        case 4: return bwd_dispatch<2, false>(a, s);
        case 5: return bwd_dispatch<2, true>(a, s);
        case 6: return bwd_dispatch<3, false>(a, s);
        case 7: return bwd_dispatch<3, true>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gsr
