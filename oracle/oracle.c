/*
 * FP64 single-threaded reference ("oracle") for the tile-based differentiable
 * Gaussian-splat rasterizer with the per-ray entropy of blending weights.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; it exists so the HIP kernels can be checked against a plain,
 * slow and obviously correct restatement of the method.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Every floating-point step runs in double precision.  Inputs arrive as
 * float32 and are converted exactly.  Sources followed:
 *   - 3D density and covariance Sigma = R S S^T R^T          (Sec. 3, Eq. 1)
 *   - EWA projection to a 2D mean and covariance              (Sec. 3, Eq. 2)
 *   - alpha = opacity * g, transmittance, blended colour      (Sec. 3, Eq. 3-5)
 *   - blending weights, their sum with the background is one  (Sec. 4.3, Eq. 8-9;
 *                                                              Suppl. A)
 *   - per-pixel entropy and its mean over pixels              (Sec. 4.3, Eq. 10-12)
 *   - dH/dalpha via the suffix variable R                     (Sec. 4.4, Eq. 13-15,
 *                                                              Alg. 1; Suppl. B)
 *   - attribute chain opacity / exponent / conic / 2D mean    (Suppl. C)
 *   - scale reset s <- zeta s                                 (Sec. 4.2, Eq. 7)
 *   - the opacity regulariser compared against the entropy
 *     constraint, exp(-(sigma - 0.5)^2 / 0.05) per Gaussian   (Sec. 5.4, ablation)
 *   - D-SSIM of the base loss and one Adam step               (Sec. 3, Eq. 6)
 * Conventions the paper leaves open (dilation 0.3, Jacobian clamp 1.3,
 * near plane, alpha clamp 0.99, 1/255 skip, 1e-4 transmittance stop, SH
 * basis without the Condon-Shortley phase, colour offset 0.5 and clamp,
 * pixel centres at +0.5, the tile-overlap rule) are listed with the build's
 * design notes; this file implements exactly those readings.
 *
 * Parity pins that constrain each function live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_DILATE      1u   /* add 0.3 to the diagonal of the 2D covariance */
#define ORC_JAC_CLAMP   2u   /* clamp x/z, y/z to 1.3x the half field of view inside J */
#define ORC_COLOR_CLAMP 4u   /* clamp SH colour at 0 per channel */

#define ORC_ALPHA_MAX   0.99
#define ORC_ALPHA_MIN   (1.0 / 255.0)
#define ORC_T_STOP      1e-4

/* relative half-width of the band around a threshold inside which a decision
 * is reported as "near" (FP32 and FP64 may legitimately take it differently) */
#define ORC_BAND        1e-4

/* per-pixel flag bits written by the renderers */
#define ORC_NEAR_SKIP   1u
#define ORC_NEAR_STOP   2u
#define ORC_NEAR_CLAMP  4u

/* projection mask bits */
#define ORC_M_CLAMP_R   1u
#define ORC_M_CLAMP_G   2u
#define ORC_M_CLAMP_B   4u
#define ORC_M_JX        8u
#define ORC_M_JY       16u

typedef struct {
    int W, H;
    double fx, fy, cx, cy;
    double R[9];
    double t[3];
    double near_z;
} cam_t;

static cam_t read_cam(const double* c)
{
    cam_t k;
    k.W = (int)c[0]; k.H = (int)c[1];
    k.fx = c[2]; k.fy = c[3]; k.cx = c[4]; k.cy = c[5];
    for (int i = 0; i < 9; ++i) k.R[i] = c[6 + i];
    for (int i = 0; i < 3; ++i) k.t[i] = c[15 + i];
    k.near_z = c[18];
    return k;
}

/* ------------------------------------------------------------------------- */
/* Real spherical harmonics, no Condon-Shortley phase.                       */
/*   Y_l0  = K_l0 P_l(z)                                                     */
/*   Y_lm  = sqrt2 K_lm Q_l^m(z) Re (x+iy)^m      (m > 0)                    */
/*   Y_l-m = sqrt2 K_lm Q_l^m(z) Im (x+iy)^m      (m > 0)                    */
/* with K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and Q_l^m the polynomial    */
/* part of the associated Legendre function, P_l^m = (1-z^2)^{m/2} Q_l^m.    */
/* Index k = l*l + l + m.  Partial derivatives are those of the polynomial   */
/* extension in (x, y, z); the caller projects out the radial part.          */
/* ------------------------------------------------------------------------- */

static double factorial(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }

void orc_sh_basis(int deg, double x, double y, double z, double* Y, double* dY /* [K][3] or NULL */)
{
    const double PI = 3.14159265358979323846;
    double Q[4][4], dQ[4][4];         /* [l][m] */
    double cr[4], ci[4];              /* Re / Im of (x+iy)^m */
    memset(Q, 0, sizeof Q); memset(dQ, 0, sizeof dQ);
    cr[0] = 1.0; ci[0] = 0.0;
    for (int m = 1; m <= 3; ++m) {
        cr[m] = x * cr[m - 1] - y * ci[m - 1];
        ci[m] = x * ci[m - 1] + y * cr[m - 1];
    }
    for (int m = 0; m <= deg; ++m) {
        double dfact = 1.0;                       /* (2m-1)!! */
        for (int k = 2 * m - 1; k > 1; k -= 2) dfact *= k;
        Q[m][m] = dfact; dQ[m][m] = 0.0;
        if (m + 1 <= deg) {
            Q[m + 1][m] = (2 * m + 1) * z * Q[m][m];
            dQ[m + 1][m] = (2 * m + 1) * Q[m][m];
        }
        for (int l = m + 2; l <= deg; ++l) {
            Q[l][m] = ((2 * l - 1) * z * Q[l - 1][m] - (l + m - 1) * Q[l - 2][m]) / (l - m);
            dQ[l][m] = ((2 * l - 1) * (Q[l - 1][m] + z * dQ[l - 1][m]) - (l + m - 1) * dQ[l - 2][m]) / (l - m);
        }
    }
    for (int l = 0; l <= deg; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double K = sqrt((2 * l + 1) / (4.0 * PI) * factorial(l - am) / factorial(l + am));
            int k = l * l + l + m;
            if (m == 0) {
                Y[k] = K * Q[l][0];
                if (dY) { dY[3 * k + 0] = 0.0; dY[3 * k + 1] = 0.0; dY[3 * k + 2] = K * dQ[l][0]; }
            } else {
                double N = sqrt(2.0) * K;
                double A = m > 0 ? cr[am] : ci[am];
                Y[k] = N * Q[l][am] * A;
                if (dY) {
                    /* d/dx (x+iy)^m = m (x+iy)^{m-1};  d/dy = i m (x+iy)^{m-1} */
                    double dAx = m > 0 ? am * cr[am - 1] : am * ci[am - 1];
                    double dAy = m > 0 ? -am * ci[am - 1] : am * cr[am - 1];
                    dY[3 * k + 0] = N * Q[l][am] * dAx;
                    dY[3 * k + 1] = N * Q[l][am] * dAy;
                    dY[3 * k + 2] = N * dQ[l][am] * A;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Projection (Eq. 1-2 and the colour).                                       */
/* ------------------------------------------------------------------------- */

/* rotation matrix of a unit quaternion (w, x, y, z), row-major */
static void quat_to_rot(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* dR[k][4]: derivative of R entry k with respect to (w, x, y, z) */
static void quat_to_rot_jac(const double q[4], double dR[9][4])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double t[9][4] = {
        { 0,      0,      -4 * y, -4 * z },
        { -2 * z, 2 * y,  2 * x,  -2 * w },
        { 2 * y,  2 * z,  2 * w,  2 * x  },
        { 2 * z,  2 * y,  2 * x,  2 * w  },
        { 0,      -4 * x, 0,      -4 * z },
        { -2 * x, -2 * w, 2 * z,  2 * y  },
        { -2 * y, 2 * z,  -2 * w, 2 * x  },
        { 2 * x,  2 * w,  2 * z,  2 * y  },
        { 0,      -4 * x, -4 * y, 0      },
    };
    memcpy(dR, t, sizeof t);
}

static int finite_all(const float* p, int n)
{
    for (int i = 0; i < n; ++i) if (!isfinite(p[i])) return 0;
    return 1;
}

/* Everything the forward projection produces for one Gaussian in one camera,
 * kept in full so the backward can reuse it. */
typedef struct {
    int valid;
    double qn[4], qnorm;
    double Rq[9], Sigma[9];
    double tcam[3], u, v, uc, vc;
    int clx, cly;
    double J[6], Tm[6];
    double cov[3];            /* a, b, c of the dilated 2D covariance */
    double det, conic[3];
    double mean2d[2];
    double lam, radius;
    double dir[3], dnorm, d[3];
    double Y[16], dY[16 * 3];
    double col[3];
    int cclamp[3];
} proj_t;

static void project_one(const float* mu, const float* s, const float* q, const float* sh, int deg,
                        const cam_t* c, unsigned flags, proj_t* P)
{
    memset(P, 0, sizeof *P);
    int K = (deg + 1) * (deg + 1);
    if (!finite_all(mu, 3) || !finite_all(s, 3) || !finite_all(q, 4) || !finite_all(sh, 3 * K)) return;
    double qq[4] = { q[0], q[1], q[2], q[3] };
    double qn = sqrt(qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2] + qq[3] * qq[3]);
    if (!(qn > 0.0)) return;
    P->qnorm = qn;
    for (int i = 0; i < 4; ++i) P->qn[i] = qq[i] / qn;
    quat_to_rot(P->qn, P->Rq);
    /* Sigma = R diag(s)^2 R^T  (Eq. 1) */
    double sd[3] = { s[0], s[1], s[2] };
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += P->Rq[3 * i + k] * sd[k] * sd[k] * P->Rq[3 * j + k];
            P->Sigma[3 * i + j] = acc;
        }
    /* camera-space position */
    for (int i = 0; i < 3; ++i)
        P->tcam[i] = c->R[3 * i + 0] * mu[0] + c->R[3 * i + 1] * mu[1] + c->R[3 * i + 2] * mu[2] + c->t[i];
    double tz = P->tcam[2];
    if (!(tz > c->near_z)) return;
    P->u = P->tcam[0] / tz;
    P->v = P->tcam[1] / tz;
    P->uc = P->u; P->vc = P->v;
    if (flags & ORC_JAC_CLAMP) {
        double limx = 1.3 * (0.5 * c->W / c->fx), limy = 1.3 * (0.5 * c->H / c->fy);
        if (P->u > limx) { P->uc = limx; P->clx = 1; }
        if (P->u < -limx) { P->uc = -limx; P->clx = 1; }
        if (P->v > limy) { P->vc = limy; P->cly = 1; }
        if (P->v < -limy) { P->vc = -limy; P->cly = 1; }
    }
    /* EWA: local affine approximation J of the perspective map (Eq. 2) */
    P->J[0] = c->fx / tz; P->J[1] = 0.0;         P->J[2] = -c->fx * P->uc / tz;
    P->J[3] = 0.0;        P->J[4] = c->fy / tz;  P->J[5] = -c->fy * P->vc / tz;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            P->Tm[3 * i + j] = P->J[3 * i + 0] * c->R[0 + j] + P->J[3 * i + 1] * c->R[3 + j] + P->J[3 * i + 2] * c->R[6 + j];
    double C2[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += P->Tm[3 * i + k] * P->Sigma[3 * k + l] * P->Tm[3 * j + l];
            C2[2 * i + j] = acc;
        }
    double dil = (flags & ORC_DILATE) ? 0.3 : 0.0;
    P->cov[0] = C2[0] + dil; P->cov[1] = 0.5 * (C2[1] + C2[2]); P->cov[2] = C2[3] + dil;
    P->det = P->cov[0] * P->cov[2] - P->cov[1] * P->cov[1];
    if (!(P->det > 0.0)) return;
    P->conic[0] = P->cov[2] / P->det;
    P->conic[1] = -P->cov[1] / P->det;
    P->conic[2] = P->cov[0] / P->det;
    double mid = 0.5 * (P->cov[0] + P->cov[2]);
    double disc = mid * mid - P->det;
    P->lam = mid + sqrt(disc > 0.0 ? disc : 0.0);
    P->radius = ceil(3.0 * sqrt(P->lam));
    P->mean2d[0] = c->fx * P->u + c->cx;
    P->mean2d[1] = c->fy * P->v + c->cy;
    /* colour from SH along the viewing direction */
    double campos[3];
    for (int i = 0; i < 3; ++i)
        campos[i] = -(c->R[0 + i] * c->t[0] + c->R[3 + i] * c->t[1] + c->R[6 + i] * c->t[2]);
    for (int i = 0; i < 3; ++i) P->dir[i] = mu[i] - campos[i];
    P->dnorm = sqrt(P->dir[0] * P->dir[0] + P->dir[1] * P->dir[1] + P->dir[2] * P->dir[2]);
    for (int i = 0; i < 3; ++i) P->d[i] = P->dir[i] / P->dnorm;
    orc_sh_basis(deg, P->d[0], P->d[1], P->d[2], P->Y, P->dY);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) acc += (double)sh[3 * k + ch] * P->Y[k];
        acc += 0.5;
        if ((flags & ORC_COLOR_CLAMP) && acc < 0.0) { acc = 0.0; P->cclamp[ch] = 1; }
        P->col[ch] = acc;
    }
    P->valid = 1;
}

int orc_project(int64_t n, const float* means, const float* scales, const float* quats, const float* opac,
                const float* sh, int deg, const double* cam, unsigned flags,
                double* mean2d, double* conic, double* cov2d, double* depth, int32_t* radius,
                double* rgb, uint8_t* mask)
{
    cam_t c = read_cam(cam);
    int K = (deg + 1) * (deg + 1);
    for (int64_t i = 0; i < n; ++i) {
        proj_t P;
        project_one(means + 3 * i, scales + 3 * i, quats + 4 * i, sh + 3 * K * i, deg, &c, flags, &P);
        if (!isfinite(opac[i])) P.valid = 0;
        radius[i] = P.valid ? (int32_t)P.radius : 0;
        mean2d[2 * i] = P.mean2d[0]; mean2d[2 * i + 1] = P.mean2d[1];
        for (int k = 0; k < 3; ++k) { conic[3 * i + k] = P.conic[k]; cov2d[3 * i + k] = P.cov[k]; rgb[3 * i + k] = P.col[k]; }
        depth[i] = P.tcam[2];
        mask[i] = (uint8_t)((P.cclamp[0] ? ORC_M_CLAMP_R : 0) | (P.cclamp[1] ? ORC_M_CLAMP_G : 0) |
                            (P.cclamp[2] ? ORC_M_CLAMP_B : 0) | (P.clx ? ORC_M_JX : 0) | (P.cly ? ORC_M_JY : 0));
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Tile binning: a Gaussian is listed in every tile of the rectangle that    */
/* covers [mean - r, mean + r] in x and y.  Lists are ordered by             */
/* (tile, float32 depth bits, Gaussian index).                              */
/* ------------------------------------------------------------------------- */

static int64_t floor_div(int64_t a, int64_t b) { int64_t q = a / b; if ((a % b != 0) && ((a < 0) != (b < 0))) --q; return q; }

/* returns 1 and the inclusive tile rect if non-empty */
static int tile_rect(double mx, double my, int32_t r, int gx, int gy, int tw, int th, int rect[4])
{
    if (r <= 0) return 0;
    double fx = floor(mx), fy = floor(my);
    if (fx > 1e9) fx = 1e9;
    if (fx < -1e9) fx = -1e9;
    if (fy > 1e9) fy = 1e9;
    if (fy < -1e9) fy = -1e9;
    int64_t x0 = floor_div((int64_t)fx - r, tw), x1 = floor_div((int64_t)fx + r, tw);
    int64_t y0 = floor_div((int64_t)fy - r, th), y1 = floor_div((int64_t)fy + r, th);
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > gx - 1) x1 = gx - 1;
    if (y1 > gy - 1) y1 = gy - 1;
    if (x0 > x1 || y0 > y1) return 0;
    rect[0] = (int)x0; rect[1] = (int)y0; rect[2] = (int)x1; rect[3] = (int)y1;
    return 1;
}

typedef struct { int64_t tile; uint32_t dbits; int32_t idx; } pair_t;

static int cmp_pair(const void* a, const void* b)
{
    const pair_t* p = (const pair_t*)a; const pair_t* q = (const pair_t*)b;
    if (p->tile != q->tile) return p->tile < q->tile ? -1 : 1;
    if (p->dbits != q->dbits) return p->dbits < q->dbits ? -1 : 1;
    if (p->idx != q->idx) return p->idx < q->idx ? -1 : 1;
    return 0;
}

/* tiles_touched per Gaussian; returns the total number of (tile, Gaussian) pairs */
int64_t orc_count_pairs(int64_t n, const double* mean2d, const int32_t* radius, int W, int H, int tw, int th,
                        int32_t* tiles_touched, int32_t* rects /* [n][4] or NULL */)
{
    int gx = (W + tw - 1) / tw, gy = (H + th - 1) / th;
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        int rc[4] = { 0, 0, -1, -1 };
        int ok = tile_rect(mean2d[2 * i], mean2d[2 * i + 1], radius[i], gx, gy, tw, th, rc);
        int32_t cnt = ok ? (rc[2] - rc[0] + 1) * (rc[3] - rc[1] + 1) : 0;
        tiles_touched[i] = cnt;
        if (rects) { for (int k = 0; k < 4; ++k) rects[4 * i + k] = ok ? rc[k] : (k < 2 ? 0 : -1); }
        total += cnt;
    }
    return total;
}

/* Sorted per-tile lists: values[P] (Gaussian indices) and ranges[n_tiles][2] = [start, end). */
int orc_bin(int64_t n, const double* mean2d, const int32_t* radius, const float* depth32,
            int W, int H, int tw, int th, int64_t cap, int32_t* values, int32_t* ranges)
{
    int gx = (W + tw - 1) / tw, gy = (H + th - 1) / th;
    int64_t ntiles = (int64_t)gx * gy;
    int64_t P = 0;
    pair_t* pairs = (pair_t*)malloc(sizeof(pair_t) * (size_t)(cap > 0 ? cap : 1));
    if (!pairs) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int rc[4];
        if (!tile_rect(mean2d[2 * i], mean2d[2 * i + 1], radius[i], gx, gy, tw, th, rc)) continue;
        uint32_t db; memcpy(&db, &depth32[i], 4);
        for (int ty = rc[1]; ty <= rc[3]; ++ty)
            for (int tx = rc[0]; tx <= rc[2]; ++tx) {
                if (P >= cap) { free(pairs); return -2; }
                pairs[P].tile = (int64_t)ty * gx + tx; pairs[P].dbits = db; pairs[P].idx = (int32_t)i; ++P;
            }
    }
    qsort(pairs, (size_t)P, sizeof(pair_t), cmp_pair);
    for (int64_t t = 0; t < ntiles; ++t) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
    for (int64_t k = 0; k < P; ++k) {
        values[k] = pairs[k].idx;
        int64_t t = pairs[k].tile;
        if (k == 0 || pairs[k - 1].tile != t) ranges[2 * t] = (int32_t)k;
        if (k == P - 1 || pairs[k + 1].tile != t) ranges[2 * t + 1] = (int32_t)(k + 1);
    }
    free(pairs);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Per-pixel blending with entropy (Eq. 3-5, 8-11).                          */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t g;          /* Gaussian index */
    double alpha, T, w; /* alpha_i, T_i, w_i = T_i alpha_i */
    double e;           /* exp(power) */
    double dx, dy;      /* mean2d - pixel centre */
    int clamped;        /* opacity * e exceeded the 0.99 clamp */
} blended_t;

static uint64_t fnv(uint64_t h, uint64_t v) { for (int i = 0; i < 8; ++i) { h ^= (v >> (8 * i)) & 0xff; h *= 1099511628211ULL; } return h; }

static int near_thr(double x, double thr) { return fabs(x - thr) <= ORC_BAND * thr; }

/* Walk one pixel's ordered candidate list.  `cand` iterates Gaussian indices
 * in list order; `ok` (may be NULL) tells whether a candidate participates.
 * Returns the number of blended entries written to `out` (if non-NULL) and
 * fills the per-pixel results. */
typedef struct {
    double C[3], H, T;
    int32_t ncontrib;   /* list positions up to and including the last blended one */
    int64_t n_eval;     /* alpha evaluations made before the walk stopped */
    uint8_t flags;
    uint64_t sig;
} pixres_t;

static int64_t walk_pixel(double px, double py, const int32_t* cand, int64_t ncand, const uint8_t* ok,
                          const double* mean2d, const double* conic, const double* opac, const double* rgb,
                          blended_t* out, pixres_t* res)
{
    double T = 1.0, H = 0.0, C[3] = { 0, 0, 0 };
    int64_t nb = 0;
    int32_t ncontrib = 0;
    uint8_t fl = 0;
    uint64_t sig = 1469598103934665603ULL;
    int64_t k;
    int64_t n_eval = 0;
    int32_t pos = 0;                 /* position in the pixel's list (participants only) */
    for (k = 0; k < ncand; ++k) {
        if (ok && !ok[k]) continue;
        ++pos;
        int32_t g = cand[k];
        double dx = mean2d[2 * g] - px, dy = mean2d[2 * g + 1] - py;
        double A = conic[3 * g], B = conic[3 * g + 1], Cc = conic[3 * g + 2];
        double power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
        double e = exp(power);
        double a_raw = opac[g] * e;
        double alpha = a_raw < ORC_ALPHA_MAX ? a_raw : ORC_ALPHA_MAX;
        ++n_eval;
        if (near_thr(a_raw, ORC_ALPHA_MIN) && !(a_raw > ORC_ALPHA_MAX)) fl |= ORC_NEAR_SKIP;
        if (near_thr(a_raw, ORC_ALPHA_MAX)) fl |= ORC_NEAR_CLAMP;
        if (alpha < ORC_ALPHA_MIN) { sig = fnv(sig, ((uint64_t)g << 2) | 1u); continue; }
        double Tn = T * (1.0 - alpha);
        if (near_thr(Tn, ORC_T_STOP)) fl |= ORC_NEAR_STOP;
        if (Tn < ORC_T_STOP) { sig = fnv(sig, ((uint64_t)g << 2) | 2u); break; }
        double w = alpha * T;
        for (int ch = 0; ch < 3; ++ch) C[ch] += w * rgb[3 * g + ch];
        H -= w * log(w);
        if (out) {
            out[nb].g = g; out[nb].alpha = alpha; out[nb].T = T; out[nb].w = w; out[nb].e = e;
            out[nb].dx = dx; out[nb].dy = dy; out[nb].clamped = a_raw > ORC_ALPHA_MAX;
        }
        sig = fnv(sig, ((uint64_t)g << 2) | (a_raw > ORC_ALPHA_MAX ? 3u : 0u));
        ++nb;
        T = Tn;
        ncontrib = pos;
    }
    H -= T * log(T);                 /* background weight w_{N+1} = T_{N+1} (Eq. 9-10) */
    for (int ch = 0; ch < 3; ++ch) res->C[ch] = C[ch];
    res->H = H; res->T = T; res->ncontrib = ncontrib; res->n_eval = n_eval; res->flags = fl; res->sig = sig;
    return nb;
}

static int pixel_tile(int px, int py, int tw, int th, int gx) { return (py / th) * gx + (px / tw); }

/* Tiled render of one view.  `pix` (may be NULL) selects pixels; outputs of
 * unselected pixels are left untouched. */
int orc_render(int W, int H, int tw, int th, int64_t n,
               const double* mean2d, const double* conic, const double* opac, const double* rgb,
               const int32_t* ranges, const int32_t* values, const uint8_t* pix,
               double* out_rgb, double* out_H, double* out_T, int32_t* out_nc, uint8_t* out_flags,
               int64_t* n_eval, int64_t* n_blend, uint64_t* sig)
{
    (void)n;
    int gx = (W + tw - 1) / tw;
    int64_t ev = 0, nbl = 0;
    uint64_t s = 1469598103934665603ULL;
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px) {
            int64_t p = (int64_t)py * W + px;
            if (pix && !pix[p]) continue;
            int t = pixel_tile(px, py, tw, th, gx);
            int32_t b = ranges[2 * t], e = ranges[2 * t + 1];
            pixres_t r;
            nbl += walk_pixel(px + 0.5, py + 0.5, values + b, e - b, NULL, mean2d, conic, opac, rgb, NULL, &r);
            for (int ch = 0; ch < 3; ++ch) out_rgb[3 * p + ch] = r.C[ch];
            out_H[p] = r.H; out_T[p] = r.T; out_nc[p] = r.ncontrib; out_flags[p] = r.flags;
            ev += r.n_eval;
            s = fnv(s, r.sig);
        }
    if (n_eval) *n_eval = ev;
    if (n_blend) *n_blend = nbl;
    if (sig) *sig = s;
    return 0;
}

/* Untiled render: every pixel scans all Gaussians in (float32 depth bits,
 * index) order and keeps those whose tile rect contains the pixel's tile.
 * Shares no list construction with orc_bin. */
typedef struct { uint32_t dbits; int32_t idx; } dk_t;
static int cmp_dk(const void* a, const void* b)
{
    const dk_t* p = (const dk_t*)a; const dk_t* q = (const dk_t*)b;
    if (p->dbits != q->dbits) return p->dbits < q->dbits ? -1 : 1;
    return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

int orc_render_bruteforce(int W, int H, int tw, int th, int64_t n,
                          const double* mean2d, const double* conic, const double* opac, const double* rgb,
                          const int32_t* radius, const float* depth32,
                          double* out_rgb, double* out_H, double* out_T, int32_t* out_nc, uint8_t* out_flags)
{
    int gx = (W + tw - 1) / tw, gy = (H + th - 1) / th;
    dk_t* order = (dk_t*)malloc(sizeof(dk_t) * (size_t)(n > 0 ? n : 1));
    int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int* rect = (int*)malloc(sizeof(int) * 4 * (size_t)(n > 0 ? n : 1));
    uint8_t* has = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
    uint8_t* ok = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
    if (!order || !cand || !rect || !has || !ok) { free(order); free(cand); free(rect); free(has); free(ok); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        memcpy(&order[i].dbits, &depth32[i], 4); order[i].idx = (int32_t)i;
        has[i] = (uint8_t)tile_rect(mean2d[2 * i], mean2d[2 * i + 1], radius[i], gx, gy, tw, th, rect + 4 * i);
    }
    qsort(order, (size_t)n, sizeof(dk_t), cmp_dk);
    for (int64_t k = 0; k < n; ++k) cand[k] = order[k].idx;
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px) {
            int tx = px / tw, ty = py / th;
            for (int64_t k = 0; k < n; ++k) {
                int g = cand[k];
                const int* rc = rect + 4 * g;
                ok[k] = (uint8_t)(has[g] && tx >= rc[0] && tx <= rc[2] && ty >= rc[1] && ty <= rc[3]);
            }
            pixres_t r;
            walk_pixel(px + 0.5, py + 0.5, cand, n, ok, mean2d, conic, opac, rgb, NULL, &r);
            int64_t p = (int64_t)py * W + px;
            for (int ch = 0; ch < 3; ++ch) out_rgb[3 * p + ch] = r.C[ch];
            out_H[p] = r.H; out_T[p] = r.T; out_nc[p] = r.ncontrib; out_flags[p] = r.flags;
        }
    free(order); free(cand); free(rect); free(has); free(ok);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* dH/dalpha along one ray, three independent statements (Eq. 15, Alg. 1).   */
/* alphas[0..N-1] are blended in order; T_{N+1} is the background weight.    */
/* ------------------------------------------------------------------------- */

static void weights_of(int n, const double* a, double* T, double* w)
{
    double t = 1.0;
    for (int i = 0; i < n; ++i) { T[i] = t; w[i] = t * a[i]; t *= 1.0 - a[i]; }
    T[n] = t; w[n] = t;
}

/* plain chain rule: dH/dalpha_i = sum_{k>=i} dH/dw_k dw_k/dalpha_i,
 * with dw_i/dalpha_i = T_i and dw_k/dalpha_i = -w_k / (1 - alpha_i) for k > i */
void orc_dH_dalpha_chain(int n, const double* a, double* out)
{
    double* T = (double*)malloc(sizeof(double) * (n + 1));
    double* w = (double*)malloc(sizeof(double) * (n + 1));
    weights_of(n, a, T, w);
    for (int i = 0; i < n; ++i) {
        double acc = (-log(w[i]) - 1.0) * T[i];
        for (int k = i + 1; k <= n; ++k) acc += (-log(w[k]) - 1.0) * (-w[k] / (1.0 - a[i]));
        out[i] = acc;
    }
    free(T); free(w);
}

/* Algorithm 1: back-to-front recurrence on the suffix variable R */
void orc_dH_dalpha_alg1(int n, const double* a, double* out)
{
    double* T = (double*)malloc(sizeof(double) * (n + 1));
    double* w = (double*)malloc(sizeof(double) * (n + 1));
    weights_of(n, a, T, w);
    double R = (log(w[n]) + 1.0) * w[n];
    for (int i = n - 1; i >= 0; --i) {
        out[i] = (-log(w[i]) - 1.0) * T[i] + R / (1.0 - a[i]);
        R += (log(w[i]) + 1.0) * w[i];
    }
    free(T); free(w);
}

/* form with the "+1" terms cancelled, using sum_{k>i} w_k = T_{i+1} (Eq. 9) */
void orc_dH_dalpha_cancelled(int n, const double* a, double* out)
{
    double* T = (double*)malloc(sizeof(double) * (n + 1));
    double* w = (double*)malloc(sizeof(double) * (n + 1));
    weights_of(n, a, T, w);
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = i + 1; k <= n; ++k) s += w[k] * log(w[k]);
        out[i] = -T[i] * log(w[i]) + s / (1.0 - a[i]);
    }
    free(T); free(w);
}

/* entropy of the weights of one ray, background included (Eq. 10) */
double orc_entropy_of_alphas(int n, const double* a)
{
    double t = 1.0, H = 0.0;
    for (int i = 0; i < n; ++i) { double w = t * a[i]; H -= w * log(w); t *= 1.0 - a[i]; }
    return H - t * log(t);
}

/* ------------------------------------------------------------------------- */
/* Backward of the blend: per-Gaussian gradients of the 2D record.           */
/* ------------------------------------------------------------------------- */

/* Accumulates (+=) dL/d{mean2d, conic, opacity, rgb} from per-pixel upstream
 * gradients dL/dC (grad_rgb[H][W][3]) and dL/dH (grad_H[H][W], may be NULL). */
int orc_backward_render(int W, int H, int tw, int th, int64_t n,
                        const double* mean2d, const double* conic, const double* opac, const double* rgb,
                        const int32_t* ranges, const int32_t* values, const uint8_t* pix,
                        const double* grad_rgb, const double* grad_H,
                        double* g_mean2d, double* g_conic, double* g_opac, double* g_rgb)
{
    (void)n;
    int gx = (W + tw - 1) / tw, gy = (H + th - 1) / th;
    int32_t maxlen = 0;
    for (int t = 0; t < gx * gy; ++t) { int32_t L = ranges[2 * t + 1] - ranges[2 * t]; if (L > maxlen) maxlen = L; }
    blended_t* ent = (blended_t*)malloc(sizeof(blended_t) * (size_t)(maxlen > 0 ? maxlen : 1));
    if (!ent) return -1;
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px) {
            int64_t p = (int64_t)py * W + px;
            if (pix && !pix[p]) continue;
            int t = pixel_tile(px, py, tw, th, gx);
            int32_t b = ranges[2 * t], e = ranges[2 * t + 1];
            pixres_t r;
            int64_t m = walk_pixel(px + 0.5, py + 0.5, values + b, e - b, NULL, mean2d, conic, opac, rgb, ent, &r);
            const double* gc = grad_rgb + 3 * p;
            double gh = grad_H ? grad_H[p] : 0.0;
            double S[3] = { 0, 0, 0 };                          /* sum_{k>i} w_k c_k */
            double Rs = (log(r.T) + 1.0) * r.T;                 /* Alg. 1 initialisation */
            for (int64_t i = m - 1; i >= 0; --i) {
                const blended_t* q = &ent[i];
                int g = q->g;
                const double* c = rgb + 3 * g;
                double inv1m = 1.0 / (1.0 - q->alpha);
                double dalpha = 0.0;
                for (int ch = 0; ch < 3; ++ch) dalpha += gc[ch] * (q->T * c[ch] - S[ch] * inv1m);
                dalpha += gh * ((-log(q->w) - 1.0) * q->T + Rs * inv1m);      /* Eq. 15 */
                for (int ch = 0; ch < 3; ++ch) g_rgb[3 * g + ch] += q->w * gc[ch];
                if (!q->clamped) {
                    g_opac[g] += q->e * dalpha;                               /* dalpha/dsigma = g */
                    double dpow = opac[g] * q->e * dalpha;                    /* dalpha/dd = sigma g */
                    double A = conic[3 * g], B = conic[3 * g + 1], Cc = conic[3 * g + 2];
                    g_conic[3 * g + 0] += dpow * (-0.5 * q->dx * q->dx);
                    g_conic[3 * g + 1] += dpow * (-q->dx * q->dy);
                    g_conic[3 * g + 2] += dpow * (-0.5 * q->dy * q->dy);
                    /* d = mean2d - pixel, power = -1/2 d^T Q d */
                    g_mean2d[2 * g + 0] += dpow * -(A * q->dx + B * q->dy);
                    g_mean2d[2 * g + 1] += dpow * -(B * q->dx + Cc * q->dy);
                }
                for (int ch = 0; ch < 3; ++ch) S[ch] += q->w * c[ch];
                Rs += (log(q->w) + 1.0) * q->w;
            }
        }
    free(ent);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Backward of the projection: 2D record gradients -> Gaussian parameters.  */
/* ------------------------------------------------------------------------- */

/* Accumulates (+=) into g_means[n][3], g_scales[n][3], g_quats[n][4],
 * g_sh[n][K][3] from per-Gaussian dL/d{mean2d, conic, rgb}. */
int orc_backward_project(int64_t n, const float* means, const float* scales, const float* quats,
                         const float* sh, int deg, const double* cam, unsigned flags,
                         const double* g_mean2d, const double* g_conic, const double* g_rgb,
                         double* g_means, double* g_scales, double* g_quats, double* g_sh)
{
    cam_t c = read_cam(cam);
    int K = (deg + 1) * (deg + 1);
    for (int64_t i = 0; i < n; ++i) {
        proj_t P;
        project_one(means + 3 * i, scales + 3 * i, quats + 4 * i, sh + 3 * K * i, deg, &c, flags, &P);
        if (!P.valid) continue;
        double gmu[3] = { 0, 0, 0 };
        /* colour -> SH coefficients and viewing direction */
        double gcol[3];
        for (int ch = 0; ch < 3; ++ch) gcol[ch] = P.cclamp[ch] ? 0.0 : g_rgb[3 * i + ch];
        double gd[3] = { 0, 0, 0 };
        for (int k = 0; k < K; ++k)
            for (int ch = 0; ch < 3; ++ch) {
                g_sh[(3 * K) * i + 3 * k + ch] += P.Y[k] * gcol[ch];
                for (int a = 0; a < 3; ++a) gd[a] += (double)sh[3 * K * i + 3 * k + ch] * gcol[ch] * P.dY[3 * k + a];
            }
        double dd = P.d[0] * gd[0] + P.d[1] * gd[1] + P.d[2] * gd[2];
        for (int a = 0; a < 3; ++a) gmu[a] += (gd[a] - P.d[a] * dd) / P.dnorm;
        /* conic -> 2D covariance: dL/dSigma' = -Q G Q with G the symmetric gradient of Q */
        double Q[4] = { P.conic[0], P.conic[1], P.conic[1], P.conic[2] };
        double G[4] = { g_conic[3 * i], 0.5 * g_conic[3 * i + 1], 0.5 * g_conic[3 * i + 1], g_conic[3 * i + 2] };
        double QG[4], GS[4];
        for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) QG[2 * a + b] = Q[2 * a] * G[b] + Q[2 * a + 1] * G[2 + b];
        for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) GS[2 * a + b] = -(QG[2 * a] * Q[b] + QG[2 * a + 1] * Q[2 + b]);
        /* 2D covariance -> Sigma and Tm = J Rc:  Sigma' = Tm Sigma Tm^T (+ dilation) */
        double gSigma[9], gTm[6];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int k = 0; k < 2; ++k) for (int l = 0; l < 2; ++l) acc += P.Tm[3 * k + a] * GS[2 * k + l] * P.Tm[3 * l + b];
                gSigma[3 * a + b] = acc;
            }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int k = 0; k < 2; ++k) for (int l = 0; l < 3; ++l) acc += GS[2 * a + k] * P.Tm[3 * k + l] * P.Sigma[3 * l + b];
                gTm[3 * a + b] = 2.0 * acc;
            }
        double gJ[6];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) gJ[3 * a + b] = gTm[3 * a + 0] * c.R[3 * b + 0] + gTm[3 * a + 1] * c.R[3 * b + 1] + gTm[3 * a + 2] * c.R[3 * b + 2];
        /* J -> camera-space position */
        double tx = P.tcam[0], ty = P.tcam[1], tz = P.tcam[2];
        double gt[3] = { 0, 0, 0 };
        gt[2] += gJ[0] * (-c.fx / (tz * tz)) + gJ[4] * (-c.fy / (tz * tz));
        if (!P.clx) { gt[0] += gJ[2] * (-c.fx / (tz * tz)); gt[2] += gJ[2] * (2.0 * c.fx * tx / (tz * tz * tz)); }
        else        { gt[2] += gJ[2] * (c.fx * P.uc / (tz * tz)); }
        if (!P.cly) { gt[1] += gJ[5] * (-c.fy / (tz * tz)); gt[2] += gJ[5] * (2.0 * c.fy * ty / (tz * tz * tz)); }
        else        { gt[2] += gJ[5] * (c.fy * P.vc / (tz * tz)); }
        /* 2D mean -> camera-space position */
        double gmx = g_mean2d[2 * i], gmy = g_mean2d[2 * i + 1];
        gt[0] += gmx * c.fx / tz;
        gt[1] += gmy * c.fy / tz;
        gt[2] += -gmx * c.fx * tx / (tz * tz) - gmy * c.fy * ty / (tz * tz);
        for (int a = 0; a < 3; ++a) gmu[a] += c.R[0 + a] * gt[0] + c.R[3 + a] * gt[1] + c.R[6 + a] * gt[2];
        /* Sigma = M M^T with M = R diag(s) */
        double M[9], gM[9];
        for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) M[3 * a + b] = P.Rq[3 * a + b] * scales[3 * i + b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += gSigma[3 * a + k] * M[3 * k + b];
                gM[3 * a + b] = 2.0 * acc;
            }
        double gR[9];
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int a = 0; a < 3; ++a) { acc += gM[3 * a + b] * P.Rq[3 * a + b]; gR[3 * a + b] = gM[3 * a + b] * scales[3 * i + b]; }
            g_scales[3 * i + b] += acc;
        }
        double dR[9][4], gqn[4] = { 0, 0, 0, 0 };
        quat_to_rot_jac(P.qn, dR);
        for (int k = 0; k < 9; ++k) for (int a = 0; a < 4; ++a) gqn[a] += gR[k] * dR[k][a];
        double qd = 0.0;
        for (int a = 0; a < 4; ++a) qd += P.qn[a] * gqn[a];
        for (int a = 0; a < 4; ++a) g_quats[4 * i + a] += (gqn[a] - P.qn[a] * qd) / P.qnorm;
        for (int a = 0; a < 3; ++a) g_means[3 * i + a] += gmu[a];
    }
    return 0;
}

/* Opacity regulariser of the ablation in Sec. 5.4: L_O = w / n * sum_i
 * exp(-(sigma_i - 0.5)^2 / 0.05).  Adds dL_O/dsigma_i to grad (may be NULL)
 * and returns L_O. */
double orc_opacity_loss(int64_t n, const float* opac, double w, double* grad)
{
    if (n <= 0) return 0.0;
    double sum = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = (double)opac[i] - 0.5;
        double e = exp(-d * d / 0.05);
        sum += e;
        if (grad) grad[i] += w / (double)n * e * (-2.0 * d / 0.05);
    }
    return w * sum / (double)n;
}

/* Scale reset (Sec. 4.2, Eq. 7): every scale multiplied by zeta, the product
 * rounded once to float32. */
void orc_scale_reset(int64_t n, float* scales, double zeta)
{
    for (int64_t i = 0; i < 3 * n; ++i) scales[i] = (float)((double)scales[i] * zeta);
}

/* ------------------------------------------------------------------------- */
/* Training-step terms around the path                                        */
/* ------------------------------------------------------------------------- */

/* D-SSIM of the base loss (Sec. 3, Eq. 6), with the 3DGS-lineage SSIM the
 * paper inherits: per channel, local statistics over an 11x11 Gaussian window
 * (sigma 1.5, normalised), zero outside the image, C1 = 0.01^2, C2 = 0.03^2,
 *   S = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2)),
 * sx^2 = E[x^2] - mx^2, sxy = E[xy] - mx my; SSIM = mean of S over pixels and
 * channels; L_D-SSIM = 1 - SSIM.  x, y: [H][W][3].  Returns SSIM; grad (may
 * be NULL) receives d SSIM / d x, written out from the definition by the
 * chain rule through the window sums. */
static void ssim_window(double* w)
{
    double g[11], s = 0.0;
    for (int k = 0; k < 11; ++k) { g[k] = exp(-(double)((k - 5) * (k - 5)) / (2.0 * 1.5 * 1.5)); s += g[k]; }
    for (int a = 0; a < 11; ++a)
        for (int b = 0; b < 11; ++b) w[a * 11 + b] = (g[a] / s) * (g[b] / s);
}

double orc_ssim(int W, int H, const double* x, const double* y, double* grad)
{
    const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
    double w[121];
    ssim_window(w);
    const int64_t M = (int64_t)W * H;
    double* dmu = (double*)calloc((size_t)M * 3, sizeof(double));   /* dS/dmx, dS/dExx, dS/dExy per pixel, channel */
    double* dxx = (double*)calloc((size_t)M * 3, sizeof(double));
    double* dxy = (double*)calloc((size_t)M * 3, sizeof(double));
    if (!dmu || !dxx || !dxy) { free(dmu); free(dxx); free(dxy); return NAN; }
    double total = 0.0;
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px)
            for (int ch = 0; ch < 3; ++ch) {
                double mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
                for (int a = -5; a <= 5; ++a)
                    for (int b = -5; b <= 5; ++b) {
                        int qy = py + a, qx = px + b;
                        if (qy < 0 || qy >= H || qx < 0 || qx >= W) continue;
                        double wt = w[(a + 5) * 11 + (b + 5)];
                        double xv = x[((int64_t)qy * W + qx) * 3 + ch], yv = y[((int64_t)qy * W + qx) * 3 + ch];
                        mx += wt * xv; my += wt * yv;
                        exx += wt * xv * xv; eyy += wt * yv * yv; exy += wt * xv * yv;
                    }
                double sx = exx - mx * mx, sy = eyy - my * my, sxy = exy - mx * my;
                double ln = 2 * mx * my + C1, ld = mx * mx + my * my + C1;
                double cn = 2 * sxy + C2, cd = sx + sy + C2;
                double N = ln * cn, D = ld * cd;
                total += N / D;
                int64_t o = ((int64_t)py * W + px) * 3 + ch;
                /* dN/dmx = 2 my cn + ln (-2 my);  dD/dmx = 2 mx cd + ld (-2 mx) */
                double dN = 2 * my * cn - 2 * my * ln, dD = 2 * mx * cd - 2 * mx * ld;
                dmu[o] = (dN * D - N * dD) / (D * D);
                dxx[o] = -N * ld / (D * D);                 /* dD/dExx = ld */
                dxy[o] = 2 * ln / D;                        /* dN/dExy = 2 ln */
            }
    if (grad) {
        /* dS_p/dx_q over the windows that contain q (the window is symmetric) */
        for (int qy = 0; qy < H; ++qy)
            for (int qx = 0; qx < W; ++qx)
                for (int ch = 0; ch < 3; ++ch) {
                    double xv = x[((int64_t)qy * W + qx) * 3 + ch], yv = y[((int64_t)qy * W + qx) * 3 + ch];
                    double acc = 0.0;
                    for (int a = -5; a <= 5; ++a)
                        for (int b = -5; b <= 5; ++b) {
                            int py = qy + a, px = qx + b;
                            if (py < 0 || py >= H || px < 0 || px >= W) continue;
                            double wt = w[(a + 5) * 11 + (b + 5)];
                            int64_t o = ((int64_t)py * W + px) * 3 + ch;
                            acc += wt * (dmu[o] + 2 * xv * dxx[o] + yv * dxy[o]);
                        }
                    grad[((int64_t)qy * W + qx) * 3 + ch] = acc / (3.0 * (double)M);
                }
    }
    free(dmu); free(dxx); free(dxy);
    return total / (3.0 * (double)M);
}

/* One Adam step (bias-corrected, as in the 3DGS lineage's optimiser) on the
 * raw parameters of an attribute whose activated value the renderer uses:
 * kind 0 identity, 1 exp (scales from log-scales), 2 sigmoid (opacity from its
 * logit).  grad_act is dL/d(activated); t >= 1 is the step number.  raw, m, v
 * are updated in place; act receives the new activated values. */
void orc_adam_step(int64_t n, double* raw, double* m, double* v, double* act, const double* grad_act, int kind,
                   double lr, double b1, double b2, double eps, int64_t t)
{
    double c1 = 1.0 / (1.0 - pow(b1, (double)t)), c2 = 1.0 / (1.0 - pow(b2, (double)t));
    for (int64_t i = 0; i < n; ++i) {
        double a = kind == 1 ? exp(raw[i]) : (kind == 2 ? 1.0 / (1.0 + exp(-raw[i])) : raw[i]);
        double g = grad_act[i] * (kind == 1 ? a : (kind == 2 ? a * (1.0 - a) : 1.0));
        m[i] = b1 * m[i] + (1.0 - b1) * g;
        v[i] = b2 * v[i] + (1.0 - b2) * g * g;
        raw[i] -= lr * (m[i] * c1) / (sqrt(v[i] * c2) + eps);
        act[i] = kind == 1 ? exp(raw[i]) : (kind == 2 ? 1.0 / (1.0 + exp(-raw[i])) : raw[i]);
    }
}
