// Per-(Gaussian, view) preprocessing, instance emission and tile ranges, and
// the preprocess backward that chains record gradients to the parameters.
//
// In view space, with L = diag(1/s) Rc^T (Sigma^-1 = L^T L) and m the mean, a
// pixel ray u = (ux, uy, 1) gives the quantities of Sec. 4.2 (eq. betagamma):
//   d^T Sigma^-1 d = |L u|^2 / |u|^2,   beta = |u| / |L u|,
//   minimum Mahalanobis distance D^2 = |Lm x Lu|^2 / |Lu|^2 (Lagrange
//   identity, free of the cancellation in c - b^2/a),
// and the full-line integral x = kappa sqrt(2 pi) beta exp(-D^2/2).  The record
// re-centres this on the ray through the mean, u0 = m / mz: with a = L (u - u0),
// Lm x Lu = mz (v0 x a) for v0 = L u0, which keeps FP32 accuracy when the pixel
// ray passes close to the mean (see the layout in vgr_internal.h).
//
// Tile bound: since beta <= s_max, alpha >= alpha_min requires
// D^2 <= D2max = 2 ln(kappa sqrt(2 pi) s_max / tau), i.e. the pixel's line meets
// the ellipsoid (x-m)^T Sigma^-1 (x-m) <= D2max.  The image of that ellipsoid
// is bounded by the conic whose dual is K (D2max Sigma - m m^T) K^T, and its
// tangent lines x = const give the exact screen bounding box used for binning
// (a conservative replacement of the 3-sigma screen-space heuristic that the
// paper notes should be adjusted for this rendering model, Sec. 8, future work).
// The Epanechnikov kernel (x = (4/3) kappa beta (1 - D^2)^(3/2)) uses the same
// box with D2max = 1 - (3 tau / (4 kappa s_max))^(2/3).
// A second pass replaces s_max by an upper bound of beta over the rays of that
// box (see beta_bound), which shrinks the box of anisotropic Gaussians seen
// along a short axis; the bound pre-test and the tile culling use the same
// D2max.
#include "vgr_internal.h"

namespace vgr {

namespace {

// Real spherical harmonics (Condon-Shortley phase), k = l^2 + l + m, written
// as Cartesian polynomials of the unit direction (x, y, z).
__device__ constexpr float kPi = 3.14159265358979323846f;
#define SHC(num, den) (__builtin_sqrtf((num) / ((den) * kPi)))
__device__ inline void sh_basis(int deg, float x, float y, float z, float *Y)
{
    const float c0 = 0.5f * SHC(1.0f, 1.0f);
    Y[0] = c0;
    if (deg < 1) return;
    const float c1 = SHC(3.0f, 4.0f);
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (deg < 2) return;
    const float a = 0.5f * SHC(15.0f, 1.0f), b = 0.25f * SHC(5.0f, 1.0f),
                c = 0.25f * SHC(15.0f, 1.0f);
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = a * x * y;
    Y[5] = -a * y * z;
    Y[6] = b * (2.0f * zz - xx - yy);
    Y[7] = -a * x * z;
    Y[8] = c * (xx - yy);
    if (deg < 3) return;
    const float d = 0.25f * SHC(35.0f, 2.0f), e = 0.5f * SHC(105.0f, 1.0f),
                f = 0.25f * SHC(21.0f, 2.0f), g = 0.25f * SHC(7.0f, 1.0f),
                h = 0.25f * SHC(105.0f, 1.0f);
    Y[9] = -d * y * (3.0f * xx - yy);
    Y[10] = e * x * y * z;
    Y[11] = -f * y * (4.0f * zz - xx - yy);
    Y[12] = g * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -f * x * (4.0f * zz - xx - yy);
    Y[14] = h * z * (xx - yy);
    Y[15] = -d * x * (xx - 3.0f * yy);
}

// Gradient of the same polynomials: G[k] = (dY/dx, dY/dy, dY/dz).
// sum_k w[k] grad Y_k at (x, y, z): the gradient of sum_k w[k] Y_k, from the
// derivatives of the Cartesian polynomials of sh_basis, without forming the
// 16 gradients.
__device__ inline float3 sh_grad_dot(int deg, float x, float y, float z, const float *w)
{
    float gx = 0.f, gy = 0.f, gz = 0.f;
    if (deg >= 1) {
        const float c1 = SHC(3.0f, 4.0f);
        gy -= c1 * w[1];
        gz += c1 * w[2];
        gx -= c1 * w[3];
    }
    if (deg >= 2) {
        const float a = 0.5f * SHC(15.0f, 1.0f), b = 0.25f * SHC(5.0f, 1.0f),
                    c = 0.25f * SHC(15.0f, 1.0f);
        const float a4 = a * w[4], a5 = a * w[5], b6 = b * w[6], a7 = a * w[7], c8 = c * w[8];
        gx += a4 * y - 2.f * b6 * x - a7 * z + 2.f * c8 * x;
        gy += a4 * x - a5 * z - 2.f * b6 * y - 2.f * c8 * y;
        gz += -a5 * y + 4.f * b6 * z - a7 * x;
    }
    if (deg >= 3) {
        const float d = 0.25f * SHC(35.0f, 2.0f), e = 0.5f * SHC(105.0f, 1.0f),
                    f = 0.25f * SHC(21.0f, 2.0f), g = 0.25f * SHC(7.0f, 1.0f),
                    h = 0.25f * SHC(105.0f, 1.0f);
        const float xx = x * x, yy = y * y, zz = z * z;
        const float d9 = d * w[9], e10 = e * w[10], f11 = f * w[11], g12 = g * w[12],
                    f13 = f * w[13], h14 = h * w[14], d15 = d * w[15];
        gx += -6.f * d9 * x * y + e10 * y * z + 2.f * f11 * x * y - 6.f * g12 * x * z -
              f13 * (4.f * zz - 3.f * xx - yy) + 2.f * h14 * x * z - 3.f * d15 * (xx - yy);
        gy += -3.f * d9 * (xx - yy) + e10 * x * z - f11 * (4.f * zz - xx - 3.f * yy) -
              6.f * g12 * y * z + 2.f * f13 * x * y - 2.f * h14 * y * z + 6.f * d15 * x * y;
        gz += e10 * x * y - 8.f * f11 * y * z + g12 * (6.f * zz - 3.f * xx - 3.f * yy) -
              8.f * f13 * x * z + h14 * (xx - yy);
    }
    return make_float3(gx, gy, gz);
}
#undef SHC

__device__ inline float act_fwd(int act, float y)
{
    if (act == VGR_ACT_SOFTPLUS10) {
        const float s = 10.0f * y;
        return (s > 0.0f ? s + log1pf(expf(-s)) : log1pf(expf(s))) * 0.1f;
    }
    return fmaxf(y, 0.0f);
}

__device__ inline float act_grad(int act, float y)
{
    if (act == VGR_ACT_SOFTPLUS10) return 1.0f / (1.0f + expf(-10.0f * y));
    return y > 0.0f ? 1.0f : 0.0f;
}

// Rotation of the normalised quaternion q = (w, x, y, z), row-major.
__device__ inline void quat_to_rot(float w, float x, float y, float z, float *R)
{
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
}

struct GaussView {
    float qn[4], qlen;
    float Rc[9];     // R_view R(q)
    float inv_s[3];
    float m[3];      // view-space mean (m[2] is the depth key value)
    float L[9];
    float p[3];
};

__device__ inline void gauss_view(const ViewInfo &vi, const float *mu, const float *q,
                                  const float *s, GaussView &g)
{
    const float *R = vi.R;
    g.m[0] = __fmaf_rn(R[0], mu[0], __fmaf_rn(R[1], mu[1], __fmaf_rn(R[2], mu[2], vi.t[0])));
    g.m[1] = __fmaf_rn(R[3], mu[0], __fmaf_rn(R[4], mu[1], __fmaf_rn(R[5], mu[2], vi.t[1])));
    g.m[2] = __fmaf_rn(R[6], mu[0], __fmaf_rn(R[7], mu[1], __fmaf_rn(R[8], mu[2], vi.t[2])));
    float len2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    g.qlen = sqrtf(len2);
    const float il = 1.0f / g.qlen;
    for (int k = 0; k < 4; ++k) g.qn[k] = q[k] * il;
    float Rq[9];
    quat_to_rot(g.qn[0], g.qn[1], g.qn[2], g.qn[3], Rq);
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            g.Rc[a * 3 + c] = R[a * 3] * Rq[c] + R[a * 3 + 1] * Rq[3 + c] + R[a * 3 + 2] * Rq[6 + c];
    for (int k = 0; k < 3; ++k) g.inv_s[k] = 1.0f / s[k];
    // L[k][j] = Rc[j][k] / s_k
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) g.L[k * 3 + j] = g.Rc[j * 3 + k] * g.inv_s[k];
    for (int k = 0; k < 3; ++k)
        g.p[k] = g.L[k * 3] * g.m[0] + g.L[k * 3 + 1] * g.m[1] + g.L[k * 3 + 2] * g.m[2];
}

// Screen extent along one image axis (normalised coordinate u = x/z) of the
// ellipsoid {(x-m)^T S^-1 (x-m) <= 1}: roots of
// (mz^2 - S22) u^2 - 2 (ma mz - Sa2) u + (ma^2 - Saa) = 0.  The discriminant is
// expanded so that the ma^2 mz^2 terms cancel analytically; minor = Saa S22 - Sa2^2.
__device__ inline bool axis_extent(float Saa, float Sa2, float S22, float minor, float ma,
                                   float mz, float &lo, float &hi)
{
    const float A = mz * mz - S22;
    if (!(A > 1e-6f * mz * mz)) return false;
    const float B = ma * mz - Sa2;
    float disc = Saa * mz * mz - 2.0f * Sa2 * ma * mz + S22 * ma * ma - minor;
    disc = fmaxf(disc, 0.0f);
    const float sq = sqrtf(disc);
    // a 1-ulp reciprocal: the pixel span adds a pixel of margin
    const float rA = __builtin_amdgcn_rcpf(A);
    lo = (B - sq) * rA;
    hi = (B + sq) * rA;
    return true;
}

__device__ inline void pixel_span(bool ok, float lo, float hi, float f, float c, int size,
                                  int &p0, int &p1)
{
    if (!ok) {
        p0 = 0;
        p1 = size - 1;
        return;
    }
    float X0 = fmaf(f, lo, c), X1 = fmaf(f, hi, c);
    // pixel centres at p + 0.5; pad one pixel for FP32 rounding
    X0 = fmaxf(X0 - 1.5f, -4.0f);
    X1 = fminf(X1 + 0.5f, (float)size + 4.0f);
    p0 = (int)floorf(X0);
    p1 = (int)ceilf(X1);
    p0 = max(p0, 0);
    p1 = min(p1, size - 1);
}

// The 3 (deg+1)^2 SH coefficients of one Gaussian into registers.  Whole
// float4 loads when the row is a multiple of 16 bytes and the array is
// 16-byte aligned: neighbouring threads read rows 3 (deg+1)^2 floats apart,
// so every load instruction touches one cache line per lane, and four times
// fewer instructions cut the address-unit work by four.
template <int NF>
__device__ __forceinline__ void load_sh_row(const float *__restrict__ sh, int64_t i, bool vec,
                                            float *c)
{
    const float *row = sh + i * NF;
    if constexpr (NF % 4 == 0) {
        if (vec) {
#pragma unroll
            for (int k = 0; k < NF / 4; ++k) {
                const float4 v = reinterpret_cast<const float4 *>(row)[k];
                c[4 * k] = v.x; c[4 * k + 1] = v.y; c[4 * k + 2] = v.z; c[4 * k + 3] = v.w;
            }
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < NF; ++k) c[k] = row[k];
}

// Pixel box of the ellipsoid {(x-m)^T Sigma^-1 (x-m) <= D2} (all rays that
// pass within Mahalanobis distance sqrt(D2) of the mean).
__device__ inline void screen_box(const GaussView &g, const float *s2, float D2,
                                  const ViewInfo &vi, int &x0, int &x1, int &y0, int &y1)
{
    // S = D2 Sigma_view, Sigma_view = Rc diag(s^2) Rc^T
    float S[9];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            S[a * 3 + c] = D2 * (g.Rc[a * 3] * g.Rc[c * 3] * s2[0] +
                                 g.Rc[a * 3 + 1] * g.Rc[c * 3 + 1] * s2[1] +
                                 g.Rc[a * 3 + 2] * g.Rc[c * 3 + 2] * s2[2]);
    // 2x2 minors (rows a and 2) by Cauchy-Binet, free of cancellation
    float minor[2];
    for (int a = 0; a < 2; ++a) {
        float acc = 0.0f;
        for (int k = 0; k < 3; ++k)
            for (int l = k + 1; l < 3; ++l) {
                const float det = g.Rc[a * 3 + k] * g.Rc[6 + l] - g.Rc[a * 3 + l] * g.Rc[6 + k];
                acc += s2[k] * s2[l] * det * det;
            }
        minor[a] = D2 * D2 * acc;
    }
    float lo, hi;
    const bool okx = axis_extent(S[0], S[2], S[8], minor[0], g.m[0], g.m[2], lo, hi);
    pixel_span(okx, lo, hi, vi.fx, vi.cx, vi.width, x0, x1);
    const bool oky = axis_extent(S[4], S[5], S[8], minor[1], g.m[1], g.m[2], lo, hi);
    pixel_span(oky, lo, hi, vi.fy, vi.cy, vi.height, y0, y1);
}

// Upper bound of beta = 1 / |L u| (u unit) over the rays through the pixel box
// [x0, x1 + 1] x [y0, y1 + 1]: with u_c the direction of the mean,
// |L u| >= |L u_c| - |u - u_c| / s_min (the largest singular value of L is
// 1 / s_min), and the chord |u - u_c| over the box is largest at a corner (the
// angle to u_c is quasi-convex on the image plane).  Returns smax when the
// bound is not smaller.
__device__ inline float beta_bound(const GaussView &g, const float *s, float smax,
                                   const ViewInfo &vi, int x0, int x1, int y0, int y1)
{
    // 1-ulp reciprocals and square roots throughout; the returned bound
    // carries a relative slack of 1e-3, far above their rounding
    const float im = __builtin_amdgcn_rsqf(g.m[0] * g.m[0] + g.m[1] * g.m[1] + g.m[2] * g.m[2]);
    const float c0 = g.m[0] * im, c1 = g.m[1] * im, c2 = g.m[2] * im;
    const float ifx = __builtin_amdgcn_rcpf(vi.fx), ify = __builtin_amdgcn_rcpf(vi.fy);
    float chord2 = 0.0f;
    for (int k = 0; k < 4; ++k) {
        const float X = (float)((k & 1) ? x1 + 1 : x0), Y = (float)((k & 2) ? y1 + 1 : y0);
        const float u0 = (X - vi.cx) * ifx, u1 = (Y - vi.cy) * ify;
        const float il = __builtin_amdgcn_rsqf(u0 * u0 + u1 * u1 + 1.0f);
        const float d0 = u0 * il - c0, d1 = u1 * il - c1, d2 = il - c2;
        chord2 = fmaxf(chord2, d0 * d0 + d1 * d1 + d2 * d2);
    }
    const float smin = fminf(s[0], fminf(s[1], s[2]));
    // the relative rounding of den grows like smax / smin (the cancellation
    // in lu - chord / smin); past 1e3 the slack below would not cover it
    if (!(smax < 1.0e3f * smin)) return smax;
    const float lu = __builtin_sqrtf(g.p[0] * g.p[0] + g.p[1] * g.p[1] + g.p[2] * g.p[2]) * im;
    const float den = lu - __builtin_sqrtf(chord2) * __builtin_amdgcn_rcpf(smin);
    if (!(den > 0.0f)) return smax;
    return fminf(smax, 1.001f * __builtin_amdgcn_rcpf(den));
}

// Tile culling.  The bound pre-test rejects a pixel when f(d) > kConicMargin;
// a tile of the Gaussian's rectangle is emitted only if the larger ellipse
// {f <= kCullLevel} meets the pixel-centre span of the tile, so that every
// dropped tile holds only pixels the pre-test would reject (the gap between
// the two levels covers FP32 rounding of both evaluations).  With the ellipse
// written as X = a Y -/+ sqrt(P - R Y^2) (X, Y: pixel column and row minus the
// ellipse centre (cx, cy) in the convention px = d + centre - 0.5), the tiles
// of one tile row form one interval: the extreme X over the row's Y span sits
// at the clamped Y of the ellipse's leftmost (yl) and rightmost (-yl) points.
struct CullRows {
    float cx, cy, a, P, R, ymax, yl, on;
};

__device__ __forceinline__ int floor_div(int a, int b)
{
    return a >= 0 ? a / b : -((b - 1 - a) / b);
}

__device__ __forceinline__ bool cull_row(const CullRows &c, int ty, int tw, int th, int rx0,
                                         int rx1, int &t0, int &t1)
{
    if (!(c.on > 0.0f)) {   // no usable bound form: the whole rectangle row
        t0 = rx0;
        t1 = rx1;
        return true;
    }
    float ya = (float)(ty * th) - c.cy, yb = ya + (float)(th - 1);
    ya = fmaxf(ya, -c.ymax);
    yb = fminf(yb, c.ymax);
    if (!(ya <= yb)) return false;
    const float yl = fminf(fmaxf(c.yl, ya), yb), yr = fminf(fmaxf(-c.yl, ya), yb);
    const float left = c.a * yl - sqrtf(fmaxf(c.P - c.R * yl * yl, 0.0f));
    const float right = c.a * yr + sqrtf(fmaxf(c.P - c.R * yr * yr, 0.0f));
    const float lim = 1.0e6f;
    const float pl = ceilf(fminf(fmaxf(c.cx + left - kCullPad, -lim), lim));
    const float pr = floorf(fminf(fmaxf(c.cx + right + kCullPad, -lim), lim));
    if (!(pl <= pr)) return false;
    t0 = max(rx0, floor_div((int)pl, tw));
    t1 = min(rx1, floor_div((int)pr, tw));
    return t0 <= t1;
}

// Bound pre-test form f(d) = d^T Q d + 2 l^T d - 1 of a record (FP64 in,
// FP32 out) and the tile-culling ellipse {f <= kCullLevel}, kept only when Q
// is positive definite with condition number <= 1e4 (otherwise Q = l = 0:
// no pixel is rejected early and no tile is culled).  (cxp, cyp): projected
// centre in pixels.
__device__ inline void bound_form(double q00, double q01, double q11, double el0, double el1,
                                  double cxp, double cyp, float &Q00, float &Q01, float &Q11,
                                  float &l0, float &l1, CullRows &cr)
{
    Q00 = Q01 = Q11 = l0 = l1 = 0.f;
    cr = CullRows{ 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f };
    const double tr = q00 + q11, det = q00 * q11 - q01 * q01;
    const double disc = sqrt(fmax(0.25 * tr * tr - det, 0.0));
    const double lmax = 0.5 * tr + disc, lmin = 0.5 * tr - disc;
    if (q00 > 0 && det > 0 && lmin > 0 && lmax <= 1e4 * lmin) {
        const double rdet = 1.0 / det;
        Q00 = (float)q00; Q01 = (float)q01; Q11 = (float)q11;
        l0 = (float)el0; l1 = (float)el1;
        // ellipse {f <= kCullLevel}: centre d0 = -Q^-1 l, (d-d0)^T Q (d-d0) <= rho
        const double dx0 = -(q11 * el0 - q01 * el1) * rdet;
        const double dy0 = -(q00 * el1 - q01 * el0) * rdet;
        const double rho = 1.0 + kCullLevel - (el0 * dx0 + el1 * dy0);
        cr.cx = (float)(cxp + dx0 - 0.5);
        cr.cy = (float)(cyp + dy0 - 0.5);
        const double rq00 = 1.0 / q00;
        cr.a = (float)(-q01 * rq00);
        cr.P = (float)(rho * rq00);
        cr.R = (float)(det * rq00 * rq00);
        cr.ymax = (float)sqrt(rho * q00 * rdet);
        cr.yl = (float)(q01 * sqrt(rho * rdet / q11));
        cr.on = 1.0f;
    }
}

// 3DGS splat of one Gaussian (Sec. 3, eq. affine_approx), FP64: the 2D
// covariance Sigma' = J Sigma_v J^T in pixels^2, with Sigma_v = Rc diag(s^2)
// Rc^T the view-space covariance and J the Jacobian of the pinhole map at the
// view-space mean (mx, my, mz).
__device__ inline void splat_cov(const GaussView &g, const float *s, const ViewInfo &vi,
                                 double mx, double my, double mz, double &S00, double &S01,
                                 double &S11)
{
    double V[6];   // V00 V01 V02 V11 V12 V22
    const int ia[6] = { 0, 0, 0, 1, 1, 2 }, ib[6] = { 0, 1, 2, 1, 2, 2 };
    for (int e = 0; e < 6; ++e) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
            acc += (double)g.Rc[ia[e] * 3 + k] * (double)g.Rc[ib[e] * 3 + k] * (double)s[k] *
                   (double)s[k];
        V[e] = acc;
    }
    const double rz = 1.0 / mz;
    const double j00 = vi.fx * rz, j02 = -vi.fx * mx * rz * rz;
    const double j11 = vi.fy * rz, j12 = -vi.fy * my * rz * rz;
    S00 = j00 * j00 * V[0] + 2.0 * j00 * j02 * V[2] + j02 * j02 * V[5];
    S01 = j00 * j11 * V[1] + j00 * j12 * V[2] + j02 * j11 * V[4] + j02 * j12 * V[5];
    S11 = j11 * j11 * V[3] + 2.0 * j11 * j12 * V[4] + j12 * j12 * V[5];
}

// Density kappa from the density input: the input itself, or the paper's
// reparameterisation kappa = -ln(1 - 0.99 theta) (1/s_x + 1/s_y + 1/s_z) / 3
// (Sec. 5, eq. density_reparam) with theta clamped to [0, 1].
__device__ inline float theta_log(float theta)   // -ln(1 - 0.99 theta)
{
    return -log1pf(-0.99f * fminf(fmaxf(theta, 0.0f), 1.0f));
}
__device__ inline float density_of(int density, float in, const float *s)
{
    if (density != VGR_DENSITY_THETA) return in;
    return theta_log(in) * ((1.0f / s[0] + 1.0f / s[1] + 1.0f / s[2]) * (1.0f / 3.0f));
}

// Largest D^2 at which a ray whose integral has peak r tau (r = K beta / tau,
// beta the ray's standard deviation) can still reach the skip threshold tau:
// x = r tau exp(-D^2/2) (Gaussian), x = r tau (1 - D^2)^(3/2) (Epanechnikov).
__device__ inline float d2max_of(bool epan, float r)
{
    return epan ? 1.0f - powf(r, -2.0f / 3.0f) : 2.0f * logf(r);
}

template <int DEG, bool MULTI, bool SPLAT>
__global__ __launch_bounds__(256) void preprocess_kernel(RenderParams rp, Buffers b,
                                                         const float *__restrict__ means,
                                                         const float *__restrict__ quats,
                                                         const float *__restrict__ scales,
                                                         const float *__restrict__ dens,
                                                         const float *__restrict__ sh)
{
    // One thread per Gaussian for all views of the call: its parameters (and
    // its SH row, from the first view that sees it) are read from HBM once.
    // MULTI = false is the one-view form: no loop, and the SH row is not kept
    // across iterations (fewer registers, higher occupancy).  SPLAT: the record
    // of the 3DGS splatting model (the density input is the peak opacity).
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i0 < rp.n;
    const int64_t i = valid ? i0 : rp.n - 1;   // threads past the end mirror the last Gaussian
    const float mu[3] = { means[3 * i], means[3 * i + 1], means[3 * i + 2] };
    const float q[4] = { quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3] };
    const float s[3] = { scales[3 * i], scales[3 * i + 1], scales[3 * i + 2] };
    const float kappa = density_of(rp.density, dens[i], s);
    constexpr int NB = (DEG + 1) * (DEG + 1);
    float c3[NB * 3];
    bool have_sh = false;
    uint32_t total = 0;

    // per view, this block's items with instances (wave ballots, added in LDS)
    __shared__ uint32_t s_vis[kMaxViews];
    const int n_views = MULTI ? rp.n_views : 1;
    for (int v = (int)threadIdx.x; v < n_views; v += (int)blockDim.x) s_vis[v] = 0u;
    __syncthreads();
    for (int v = 0; v < n_views; ++v) {
        const ViewInfo &vi = b.views[v];
        const int64_t item = (int64_t)v * rp.n + i;
        uint32_t key = 0xFFFFFFFFu, count = 0;
        ushort4 rect = make_ushort4(0, 0, 0, 0);
        const float z = __fmaf_rn(vi.R[6], mu[0], __fmaf_rn(vi.R[7], mu[1], __fmaf_rn(vi.R[8], mu[2], vi.t[2])));
        const bool epan = rp.kernel == VGR_KERNEL_EPANECHNIKOV;   // uniform
        // peak line integral per unit beta: kappa sqrt(2 pi) (Gaussian) or
        // (4/3) kappa (Epanechnikov, at D = 0)
        const float K = kappa * (epan ? 4.0f / 3.0f : kSqrt2Pi);
        const float smax = fmaxf(s[0], fmaxf(s[1], s[2]));
        const float op = fminf(fmaxf(kappa, 0.0f), 1.0f);   // splat: peak opacity
        if (SPLAT ? (valid && z > vi.znear && op >= rp.amin)
                  : (valid && z > vi.znear && K * smax > rp.tau)) {
            GaussView g;
            gauss_view(vi, mu, q, s, g);
            int x0, x1, y0, y1;
            float D2max = 0.0f;
            double S00 = 0.0, S01 = 0.0, S11 = 0.0, E2 = 0.0;
            if constexpr (SPLAT) {
                // alpha = o exp(-1/2 d^T Sigma'^-1 d) >= alpha_min inside the ellipse
                // d^T Sigma'^-1 d <= E2 = 2 ln(o / alpha_min); its box is
                // |dx| <= sqrt(E2 S00), |dy| <= sqrt(E2 S11)
                const double mxs = (double)vi.R[0] * mu[0] + (double)vi.R[1] * mu[1] + (double)vi.R[2] * mu[2] + vi.t[0];
                const double mys = (double)vi.R[3] * mu[0] + (double)vi.R[4] * mu[1] + (double)vi.R[5] * mu[2] + vi.t[1];
                const double mzs = (double)vi.R[6] * mu[0] + (double)vi.R[7] * mu[1] + (double)vi.R[8] * mu[2] + vi.t[2];
                splat_cov(g, s, vi, mxs, mys, mzs, S00, S01, S11);
                E2 = 2.0 * log((double)op / (double)rp.amin);
                const double cxs = (double)vi.fx * (mxs / mzs) + vi.cx;
                const double cys = (double)vi.fy * (mys / mzs) + vi.cy;
                const double hwx = sqrt(E2 * S00), hwy = sqrt(E2 * S11);
                if (S00 * S11 - S01 * S01 > 0.0) {
                    pixel_span(true, (float)(cxs - hwx), (float)(cxs + hwx), 1.0f, 0.0f, vi.width, x0, x1);
                    pixel_span(true, (float)(cys - hwy), (float)(cys + hwy), 1.0f, 0.0f, vi.height, y0, y1);
                } else {
                    x0 = y0 = 0; x1 = y1 = -1;   // degenerate splat: no area
                }
            } else {
            // alpha >= alpha_min needs D^2 <= D2max(K beta / tau) with beta the
            // ray's standard deviation; beta <= smax gives a first box ...
            D2max = d2max_of(epan, K * smax / rp.tau);
            const float s2[3] = { s[0] * s[0], s[1] * s[1], s[2] * s[2] };
            screen_box(g, s2, D2max, vi, x0, x1, y0, y1);
            // ... and beta over the rays of that box bounds it tighter (tight for
            // anisotropic Gaussians seen along a short axis)
            if (x0 <= x1 && y0 <= y1) {
                const float beta = beta_bound(g, s, smax, vi, x0, x1, y0, y1);
                if (beta < smax) {
                    if (K * beta > rp.tau) {
                        D2max = d2max_of(epan, K * beta / rp.tau);
                        screen_box(g, s2, D2max, vi, x0, x1, y0, y1);
                    } else {
                        x1 = x0 - 1;   // alpha < alpha_min on every ray of the box
                    }
                }
            }
            }   // volumetric bound
            if (x0 <= x1 && y0 <= y1) {
                const int tx0 = x0 / rp.tile_w, tx1 = x1 / rp.tile_w;
                const int ty0 = y0 / rp.tile_h, ty1 = y1 / rp.tile_h;
                rect = make_ushort4((unsigned short)tx0, (unsigned short)ty0, (unsigned short)tx1,
                                    (unsigned short)ty1);
                key = __float_as_uint(z);
                // view-space mean and projected centre in FP64: their rounding sets
                // how precisely the pixel offsets of small, distant Gaussians are known
                const double mx = (double)vi.R[0] * mu[0] + (double)vi.R[1] * mu[1] + (double)vi.R[2] * mu[2] + vi.t[0];
                const double my = (double)vi.R[3] * mu[0] + (double)vi.R[4] * mu[1] + (double)vi.R[5] * mu[2] + vi.t[1];
                const double mzd = (double)vi.R[6] * mu[0] + (double)vi.R[7] * mu[1] + (double)vi.R[8] * mu[2] + vi.t[2];
                const double rmz = 1.0 / mzd;
                const double u0x = mx * rmz, u0y = my * rmz;
                const double cxp = (double)vi.fx * u0x + vi.cx, cyp = (double)vi.fy * u0y + vi.cy;
                const double hx = rint(cxp), hy = rint(cyp);
                const float v0[3] = {
                    (float)(g.L[0] * u0x + g.L[1] * u0y + g.L[2]),
                    (float)(g.L[3] * u0x + g.L[4] * u0y + g.L[5]),
                    (float)(g.L[6] * u0x + g.L[7] * u0y + g.L[8]) };
                const float mz = (float)mzd;
                const float ifx = 1.0f / vi.fx, ify = 1.0f / vi.fy;
                const float A[6] = { g.L[0] * ifx, g.L[1] * ify, g.L[3] * ifx, g.L[4] * ify,
                                     g.L[6] * ifx, g.L[7] * ify };
                // bound pre-test form (FP64).  Volumetric: with G = A^T A, gv = A^T v0,
                // V = |v0|^2, D' = D2max (1 + 1e-4):
                // Q = (mz^2 (V G - gv gv^T) - D' G) / (D' V), l = -gv / V.
                // Splat: Q = Sigma'^-1 / (E2 (1 + 1e-4)), l = 0.
                float Q00, Q01, Q11, l0, l1;
                CullRows cr;
                double C00 = 0.0, C01 = 0.0, C11 = 0.0;
                if constexpr (SPLAT) {
                    const double rdet = 1.0 / (S00 * S11 - S01 * S01);
                    C00 = S11 * rdet; C01 = -S01 * rdet; C11 = S00 * rdet;
                    const double rE = 1.0 / (E2 * (1.0 + 1e-4));
                    bound_form(C00 * rE, C01 * rE, C11 * rE, 0.0, 0.0, cxp, cyp, Q00, Q01, Q11, l0,
                               l1, cr);
                } else {
                    const double Dp = (double)D2max * (1.0 + 1e-4);
                    double G00 = 0, G01 = 0, G11 = 0, g0 = 0, g1 = 0, V = 0;
                    for (int k = 0; k < 3; ++k) {
                        const double ak0 = A[2 * k], ak1 = A[2 * k + 1], vk = v0[k];
                        G00 += ak0 * ak0; G01 += ak0 * ak1; G11 += ak1 * ak1;
                        g0 += ak0 * vk; g1 += ak1 * vk; V += vk * vk;
                    }
                    const double mz2 = mzd * mzd, rV = 1.0 / V, rden = rV / Dp;
                    const double q00 = (mz2 * (V * G00 - g0 * g0) - Dp * G00) * rden;
                    const double q01 = (mz2 * (V * G01 - g0 * g1) - Dp * G01) * rden;
                    const double q11 = (mz2 * (V * G11 - g1 * g1) - Dp * G11) * rden;
                    bound_form(q00, q01, q11, -g0 * rV, -g1 * rV, cxp, cyp, Q00, Q01, Q11, l0, l1, cr);
                }
                // tiles of the rectangle that the bound ellipse reaches, row by row
                for (int ty = ty0; ty <= ty1; ++ty) {
                    int t0, t1;
                    if (cull_row(cr, ty, rp.tile_w, rp.tile_h, tx0, tx1, t0, t1))
                        count += (uint32_t)(t1 - t0 + 1);
                }
                float4 *gp = b.geom + item * kRecVec;
                gp[0] = make_float4((float)hx, (float)hy, (float)(cxp - hx), (float)(cyp - hy));
                gp[1] = make_float4(Q00, 2.0f * Q01, 2.0f * l0, 2.0f * l1);
                if constexpr (SPLAT) {
                    gp[2] = make_float4(Q11, 0.0f, 0.0f, 0.0f);
                    gp[3] = make_float4((float)(0.5 * kLog2e * C00), (float)(kLog2e * C01),
                                        (float)(0.5 * kLog2e * C11), 0.0f);
                    gp[4] = make_float4(0.0f, 0.0f, op, 0.0f);
                } else {
                    gp[2] = make_float4(Q11, A[0], A[2], A[4]);
                    gp[3] = make_float4(A[1], A[3], A[5], v0[0]);
                    // near-plane segment: every ray that can reach alpha_min passes
                    // within sqrt(D2max) smax of the mean, so its closest point lies
                    // beyond depth mz - sqrt(D2max) smax, and beta <= smax: with
                    // (mz - znear) / smax - sqrt(D2max) > 6, Phi > 1 - 1e-9 there
                    const bool near = rp.near_segment &&
                                      (mz - vi.znear) / smax - sqrtf(D2max) <= 6.0f;
                    gp[4] = make_float4(v0[1], v0[2], near ? -(K * kLog2e) : K * kLog2e,
                                        epan ? mz * mz : (0.5f * kLog2e) * mz * mz);
                }
                gp[6] = make_float4(cr.cx, cr.cy, cr.a, cr.P);
                gp[7] = make_float4(cr.R, cr.ymax, cr.yl, cr.on);
                float rgb[3] = { 0.0f, 0.0f, 0.0f };
                if (rp.mode == VGR_MODE_COLOR) {
                    float dx = mu[0] - vi.o[0], dy = mu[1] - vi.o[1], dz = mu[2] - vi.o[2];
                    const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
                    dx *= il; dy *= il; dz *= il;
                    float Y[16];
                    sh_basis(DEG, dx, dy, dz, Y);
                    if (!have_sh) {
                        load_sh_row<NB * 3>(sh, i, ((uintptr_t)sh & 15) == 0, c3);
                        have_sh = true;
                    }
                    for (int ch = 0; ch < 3; ++ch) {
                        float acc = 0.5f;
#pragma unroll
                        for (int k = 0; k < NB; ++k) acc = fmaf(c3[k * 3 + ch], Y[k], acc);
                        rgb[ch] = act_fwd(rp.act, acc);
                    }
                }
                gp[5] = make_float4(rgb[0], rgb[1], rgb[2], mz);
            }
        }
        if (count == 0) key = 0xFFFFFFFFu;
        if (valid) {
            b.key2[item] = key;   // item order; the compaction moves the items with instances
            b.counts[item] = count;
            b.rect[item] = rect;
            total += count;
        }
        const uint64_t vis = __builtin_amdgcn_ballot_w64(valid && count > 0);
        if ((threadIdx.x & 63) == 0 && vis != 0) atomicAdd(&s_vis[v], (uint32_t)__popcll(vis));
    }
    // total instance count K, for sizing the instance lists before the scan,
    // and the number of items with instances (they come first in depth order,
    // so the scan and the emission need cover no more): one partial sum of
    // each per block (count_total_kernel adds them; one atomic per wave on a
    // single address would serialise thousands of updates)
    __shared__ uint32_t s_wsum[4];
    uint32_t wsum = total;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off, 64);
    if ((threadIdx.x & 63) == 0) s_wsum[threadIdx.x >> 6] = wsum;
    __syncthreads();
    if (threadIdx.x == 0)
        b.blk_counts[blockIdx.x] = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
    // items with instances per (view, block), in item order (view-major)
    for (int v = (int)threadIdx.x; v < n_views; v += (int)blockDim.x)
        b.blk_counts[gridDim.x + (size_t)v * gridDim.x + blockIdx.x] = s_vis[v];
}

// Exclusive scan over the 256 threads of a block; *total gets the sum.
__device__ __forceinline__ uint32_t emit_block_scan(uint32_t v, uint32_t *wsum, uint32_t *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {   // 256 threads
        const uint32_t ws = wsum[i];
        off += i < w ? ws : 0u;
        tot += ws;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// Block 0: instance total into d_total[4].  Block 1: exclusive scan, in
// place, of the nc per-(view, block) counts of items with instances that
// follow the nb instance partials, and their total (the items the depth sort
// takes) into d_total[6].
__global__ __launch_bounds__(256) void count_total_kernel(uint32_t *__restrict__ parts,
                                                           int64_t nb, int64_t nc,
                                                           uint32_t *__restrict__ d_total,
                                                           uint32_t *__restrict__ h_total)
{
    __shared__ uint32_t s_part[4];
    if (blockIdx.x == 0) {
        uint32_t acc = 0;
        for (int64_t k = threadIdx.x; k < nb; k += 256) acc += parts[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t K = s_part[0] + s_part[1] + s_part[2] + s_part[3];
            d_total[4] = K;
            if (h_total) h_total[0] = K;
        }
        return;
    }
    // 4096 counts per round, 16 consecutive ones per thread
    uint32_t *c = parts + nb;
    uint32_t carry = 0;
    for (int64_t base = 0; base < nc; base += 4096) {   // uniform
        const int64_t k0 = base + (int64_t)threadIdx.x * 16;
        uint32_t v[16], sum = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            v[q] = k0 + q < nc ? c[k0 + q] : 0u;
            sum += v[q];
        }
        uint32_t tot;
        uint32_t off = carry + emit_block_scan(sum, s_part, &tot);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (k0 + q < nc) c[k0 + q] = off;
            off += v[q];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        d_total[6] = carry;
        if (h_total) h_total[2] = carry;
    }
}

// The items with instances, in item order, to the front of (depth_key,
// item_ids) for the depth sort: one block per (view, preprocess block) of 256
// items, at the offset the count scan gave it.
__global__ __launch_bounds__(256) void compact_items_kernel(RenderParams rp, Buffers b,
                                                             int64_t nb)
{
    __shared__ uint32_t s_w[4];
    const int64_t c = blockIdx.x;
    const int64_t v = c / nb, blk = c - v * nb;
    const int64_t i = blk * 256 + threadIdx.x;
    const int64_t item = v * rp.n + i;
    const uint32_t key = i < rp.n ? b.key2[item] : 0xFFFFFFFFu;
    const bool vis = key != 0xFFFFFFFFu;
    uint32_t tot;
    const uint32_t r = emit_block_scan(vis ? 1u : 0u, s_w, &tot);
    if (vis) {
        const uint32_t pos = b.blk_counts[nb + c] + r;
        b.depth_key[pos] = key;
        b.item_ids[pos] = (uint32_t)item;
    }
}

// Tile counts in depth order, one item per thread, with each block's sum
// (kScanGrain items) into partial[block] for the scan.  Items past the
// nvis[0] that have instances (they sort last) have none, so their counts are
// not gathered.  The same launch clears the per-tile ranges and the 64
// tile-order counters (read by the range and tile-order kernels later in the
// forward).
constexpr int kGatherThreads = (int)kScanGrain;

__global__ __launch_bounds__(kGatherThreads) void gather_counts_kernel(
    const uint32_t *__restrict__ sorted_items, const uint32_t *__restrict__ counts,
    const uint32_t *__restrict__ nvis, uint32_t *__restrict__ out, int64_t m,
    uint32_t *__restrict__ partial, uint2 *__restrict__ ranges, int32_t n_tiles,
    uint32_t *__restrict__ order_counters)
{
    __shared__ uint32_t s_w[kGatherThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kGatherThreads;
    const int64_t j = base + threadIdx.x;
    uint32_t c = 0;
    if (j < m) {
        c = j < (int64_t)nvis[0] ? counts[sorted_items[j]] : 0u;
        out[j] = c;
    }
    if (j < n_tiles) ranges[j] = make_uint2(0u, 0u);
    if (j < 64) order_counters[j] = 0u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0 && base < m) {
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < kGatherThreads / 64; ++w) t += s_w[w];
        partial[blockIdx.x] = t;
    }
}

// Emission of the (tile, Gaussian) pairs in depth order.  Each 256-thread
// block owns 64 consecutive depth-sorted Gaussians, whose instance ranges are
// contiguous.  Their candidate tile rows (the rows of each rectangle, in
// Gaussian then row order) are processed 1024 at a time, four consecutive
// rows per thread: each thread finds the owning Gaussian by binary search
// over the 64 row prefixes and culls its rows to tile intervals (the same
// intervals the preprocess counted); a block scan of the interval lengths
// gives each row its first instance; then each thread writes instances
// e, e + 256, ..., finding the row of instance e by binary search over the
// row starts.
constexpr int kEmitRows = 1024;
constexpr int kEmitThreads = 256;
constexpr int kEmitRowsPerThread = kEmitRows / kEmitThreads;

__global__ __launch_bounds__(kEmitThreads) void emit_kernel(RenderParams rp, Buffers b, int64_t m,
                                                  int64_t capacity)
{
    __shared__ uint32_t s_item[64];
    __shared__ ushort4 s_rect[64];
    __shared__ CullRows s_cull[64];
    __shared__ int32_t s_toff[64], s_tx[64];
    __shared__ uint32_t s_rowbeg[65];              // first candidate row of each Gaussian
    __shared__ uint32_t s_rstart[kEmitRows + 1];   // first instance of each row of the chunk
    __shared__ uint32_t s_rtile[kEmitRows];        // tile row << 16 | first tile column
    __shared__ uint8_t s_rg[kEmitRows];            // owning Gaussian (0..63)
    __shared__ uint32_t s_wsum[kEmitThreads / 64];
    __shared__ uint32_t s_gemit[64];               // instances found per Gaussian
    const int tid = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    // items past those with instances (they sort last) emit nothing (uniform)
    if (j0 >= (int64_t)b.d_total[6]) return;
    const int64_t jend = min(j0 + 64, m);
    const uint32_t base = b.offsets[j0];
    if (tid < 64) {   // wave 0: the block's Gaussians and their candidate row counts
        const int64_t j = j0 + tid;
        CullRows cr = { 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f };
        ushort4 rect = make_ushort4(0, 0, 0, 0);
        uint32_t item = 0, rows = 0;
        int32_t toff = 0, txs = 0;
        if (j < m && b.offsets[j + 1] > b.offsets[j]) {   // a Gaussian with instances
            item = b.item_ids[j];
            rect = b.rect[item];
            const float4 c6 = b.geom[(size_t)item * kRecVec + 6];
            const float4 c7 = b.geom[(size_t)item * kRecVec + 7];
            cr = CullRows{ c6.x, c6.y, c6.z, c6.w, c7.x, c7.y, c7.z, c7.w };
            const ViewInfo &vi = b.views[(int)(item / (uint64_t)rp.n)];
            toff = vi.tile_off;
            txs = vi.tiles_x;
            rows = (uint32_t)rect.w - (uint32_t)rect.y + 1u;
        }
        s_item[tid] = item;
        s_gemit[tid] = 0u;
        s_rect[tid] = rect;
        s_cull[tid] = cr;
        s_toff[tid] = toff;
        s_tx[tid] = txs;
        uint32_t inc = rows;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = __shfl_up(inc, d, 64);
            if (tid >= d) inc += t;
        }
        s_rowbeg[tid] = inc - rows;
        if (tid == 63) s_rowbeg[64] = inc;
    }
    __syncthreads();
    const uint32_t nrows = s_rowbeg[64];
    uint32_t done = 0;   // instances of the earlier chunks
    for (uint32_t c0 = 0; c0 < nrows; c0 += kEmitRows) {
        const uint32_t cn = min((uint32_t)kEmitRows, nrows - c0);
        uint32_t cnt[kEmitRowsPerThread];
        uint32_t sum = 0;
#pragma unroll
        for (int i = 0; i < kEmitRowsPerThread; ++i) {
            const uint32_t rl = (uint32_t)(tid * kEmitRowsPerThread + i);
            cnt[i] = 0;
            if (rl < cn) {
                const uint32_t r = c0 + rl;
                // largest g with s_rowbeg[g] <= r: Gaussians without rows share
                // their prefix with the next one, which the search prefers
                int lo = 0, hi = 63;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_rowbeg[mid] <= r) lo = mid;
                    else hi = mid - 1;
                }
                const ushort4 rect = s_rect[lo];
                const int row = (int)rect.y + (int)(r - s_rowbeg[lo]);
                int t0 = 0, t1 = -1;
                if (cull_row(s_cull[lo], row, rp.tile_w, rp.tile_h, rect.x, rect.z, t0, t1))
                    cnt[i] = (uint32_t)(t1 - t0 + 1);
                if (cnt[i]) atomicAdd(&s_gemit[lo], cnt[i]);
                s_rtile[rl] = ((uint32_t)row << 16) | (uint32_t)(t0 & 0xFFFF);
                s_rg[rl] = (uint8_t)lo;
            }
            sum += cnt[i];
        }
        uint32_t chunk;
        uint32_t run = done + emit_block_scan(sum, s_wsum, &chunk);
#pragma unroll
        for (int i = 0; i < kEmitRowsPerThread; ++i) {
            const uint32_t rl = (uint32_t)(tid * kEmitRowsPerThread + i);
            if (rl < cn) s_rstart[rl] = run;
            run += cnt[i];
        }
        if (tid == 0) s_rstart[cn] = done + chunk;
        __syncthreads();
        for (uint32_t e = done + (uint32_t)tid; e < done + chunk; e += kEmitThreads) {
            // largest k with s_rstart[k] <= e (rows without instances share the
            // start of the next row, which the search prefers)
            int lo = 0, hi = (int)cn - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_rstart[mid] <= e) lo = mid;
                else hi = mid - 1;
            }
            const int g = s_rg[lo];
            const ushort4 rr = s_rect[g];
            // the preprocess counted exactly these tiles; the clamp only keeps
            // a miscount (none is expected) inside the Gaussian's own rectangle
            const int ty = min(max((int)(s_rtile[lo] >> 16), (int)rr.y), (int)rr.w);
            const int tx = min(max((int)(s_rtile[lo] & 0xFFFFu) + (int)(e - s_rstart[lo]),
                                   (int)rr.x), (int)rr.z);
            const int64_t pos = (int64_t)base + e;
            if (pos < capacity) {
                b.inst_key[pos] = (uint32_t)(s_toff[g] + ty * s_tx[g] + tx);
                b.inst_val[pos] = s_item[g];
            }
        }
        done += chunk;
        __syncthreads();   // the next chunk rewrites the row tables
    }
    // every Gaussian must have produced exactly the tile count the preprocess
    // gave it (which sized the lists): count the items that did not
    if (tid < 64) {
        const int64_t j = j0 + tid;
        const uint32_t want = j < m ? b.offsets[j + 1] - b.offsets[j] : 0u;
        const uint64_t bad = __builtin_amdgcn_ballot_w64(s_gemit[tid] != want);
        if (tid == 0 && bad != 0) atomicAdd(&b.d_total[7], (uint32_t)__builtin_popcountll(bad));
    }
}

// Per-tile [start, end) of the tile-sorted instance list.  Keys at or past
// n_tiles (none are emitted; the check keeps a bad key from writing outside
// the ranges array) are ignored.
__global__ void ranges_kernel(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ d_total,
                              uint2 *__restrict__ ranges, int64_t bound, uint32_t n_tiles)
{
    const int64_t K = d_total[0];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < K && j < bound;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = keys[j];
        if (k >= n_tiles) continue;
        if (j == 0 || keys[j - 1] != k) ranges[k].x = (uint32_t)j;
        if (j == K - 1 || keys[j + 1] != k) ranges[k].y = (uint32_t)(j + 1);
    }
}

// Heaviest-first launch order of the tiles, by a counting sort on 32 buckets
// of the list length (2 buckets per octave, longest first).  The order within
// a bucket is arbitrary: it only steers scheduling, never results.
// Per-tile re-sorting key of instance j: the view depth s* = mz (v0 . w) / |w|^2
// of the closest point to the mean on the ray through the centre of its tile
// (w = L u for that ray, from the record), as order-preserving bits.
__global__ void resort_key_kernel(RenderParams rp, Buffers b, uint32_t *__restrict__ key,
                                  uint32_t *__restrict__ idx, int64_t bound)
{
    const int64_t K = b.d_total[0];
    const int64_t m = rp.n * (int64_t)rp.n_views;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < K && j < bound;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t gt = b.inst_key[j], item = b.inst_val[j];
        uint32_t k = 0xFFFFFFFFu;
        if (gt < (uint32_t)rp.total_tiles && (int64_t)item < m) {
            int v = 0;
            for (int q = 1; q < rp.n_views; ++q)
                if (b.views[q].tile_off <= (int)gt) v = q;
            const ViewInfo &vi = b.views[v];
            const int lt = (int)gt - vi.tile_off;
            const int tx = lt % vi.tiles_x, ty = lt / vi.tiles_x;
            const float4 *gp = b.geom + (size_t)item * kRecVec;
            const float4 g0 = gp[0], g2 = gp[2], g3 = gp[3], g4 = gp[4], g5 = gp[5];
            const float dx = ((float)(tx * rp.tile_w) + 0.5f * rp.tile_w - g0.x) - g0.z;
            const float dy = ((float)(ty * rp.tile_h) + 0.5f * rp.tile_h - g0.y) - g0.w;
            // A = [[g2.y, g3.x], [g2.z, g3.y], [g2.w, g3.z]], v0 = (g3.w, g4.x, g4.y)
            const float w0 = __fmaf_rn(g3.x, dy, __fmaf_rn(g2.y, dx, g3.w));
            const float w1 = __fmaf_rn(g3.y, dy, __fmaf_rn(g2.z, dx, g4.x));
            const float w2 = __fmaf_rn(g3.z, dy, __fmaf_rn(g2.w, dx, g4.y));
            const float vw = __fmaf_rn(g3.w, w0, __fmaf_rn(g4.x, w1, g4.y * w2));
            const float ww = __fmaf_rn(w0, w0, __fmaf_rn(w1, w1, w2 * w2));
            const float depth = g5.w * vw / ww;
            const uint32_t u = __float_as_uint(depth);
            k = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
            if (k == 0xFFFFFFFFu) k = 0xFFFFFFFEu;   // keep the invalid slot last
        }
        key[j] = k;
        idx[j] = (uint32_t)j;
    }
}

__global__ void resort_gather_kernel(const uint32_t *__restrict__ d_total,
                                     const uint32_t *__restrict__ src_key,
                                     const uint32_t *__restrict__ src_val,
                                     const uint32_t *__restrict__ idx, uint32_t *__restrict__ dst_key,
                                     uint32_t *__restrict__ dst_val, int64_t bound)
{
    const int64_t K = d_total[0];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < K && j < bound;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t i = idx ? idx[j] : (uint32_t)j;
        const bool ok = (int64_t)i < K && (int64_t)i < bound;
        dst_key[j] = ok ? src_key[i] : 0xFFFFFFFFu;
        dst_val[j] = ok ? src_val[i] : 0u;
    }
}

__device__ inline int tile_bucket(uint32_t len)
{
    if (len == 0) return 31;
    const int lg = 31 - __clz(len);                        // floor(log2 len)
    const int half = (len >> (lg > 0 ? lg - 1 : 0)) & 1;   // upper half of the octave
    return max(0, 30 - min(30, 2 * lg + half));
}

__global__ void tile_hist_kernel(const uint2 *__restrict__ ranges, uint32_t *__restrict__ hist,
                                 int32_t n)
{
    __shared__ uint32_t h[32];
    if (threadIdx.x < 32) h[threadIdx.x] = 0;
    __syncthreads();
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const uint2 r = ranges[t];
        atomicAdd(&h[tile_bucket(r.y - r.x)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 32 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void tile_place_kernel(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ hist,
                                  uint32_t *__restrict__ cursor, uint32_t *__restrict__ order,
                                  int32_t n)
{
    __shared__ uint32_t base[32], local[32], start[32];
    if (threadIdx.x < 32) local[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int k = 0; k < 32; ++k) {
            base[k] = acc;
            acc += hist[k];
        }
    }
    __syncthreads();
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    int k = 0;
    uint32_t rank = 0;
    if (t < n) {
        const uint2 r = ranges[t];
        k = tile_bucket(r.y - r.x);
        rank = atomicAdd(&local[k], 1u);   // LDS: rank within this block's bucket
    }
    __syncthreads();
    // one global cursor update per (block, bucket)
    if (threadIdx.x < 32 && local[threadIdx.x])
        start[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], local[threadIdx.x]);
    __syncthreads();
    if (t < n) order[base[k] + start[k] + rank] = (uint32_t)t;
}

__global__ void fill_u32_kernel(uint32_t *__restrict__ p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_f32_kernel(float *__restrict__ p, float v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------ backward ---

// Gradient of one view's splatting record (Sec. 3, eq. 3dgs_alpha, eq.
// affine_approx), FP64.  gr: sum tau dx^2, sum tau dx dy, sum tau dy^2,
// sum tau dx, sum tau dy (tau = dL/dalpha alpha, d = pixel - mu').  With
// C = Sigma'^-1, Sigma' = J V J^T, V = Rc D Rc^T, D = diag(s^2):
//   dL/dC = -1/2 [[A, B], [B, Cq]],  dL/dSigma' = -C (dL/dC) C,
//   dL/dmu' = C (Px, Py),  dL/dV = J^T (dL/dSigma') J,  dL/dJ = 2 (dL/dSigma') J V,
//   H = Rc^T (dL/dV) Rc:  dL/ds_k = 2 s_k H_kk,  body-frame rotation
//   dL/dtheta = 2 (H12 (D1 - D2), H20 (D2 - D0), H01 (D0 - D1)),
// and the view-space mean through J and mu'.  Adds the world-space mean
// gradient to gmw, the scales' to gs and the rotation's to gth.
__device__ inline void splat_view_grad(const GaussView &g, const float *s, const float *mu,
                                       const ViewInfo &vi, const float *gr, float *gmw,
                                       float *gs, float *gth)
{
    const double mx = (double)vi.R[0] * mu[0] + (double)vi.R[1] * mu[1] + (double)vi.R[2] * mu[2] + vi.t[0];
    const double my = (double)vi.R[3] * mu[0] + (double)vi.R[4] * mu[1] + (double)vi.R[5] * mu[2] + vi.t[1];
    const double mz = (double)vi.R[6] * mu[0] + (double)vi.R[7] * mu[1] + (double)vi.R[8] * mu[2] + vi.t[2];
    double Rc[9], D[3], V[9];
    for (int k = 0; k < 9; ++k) Rc[k] = g.Rc[k];
    for (int k = 0; k < 3; ++k) D[k] = (double)s[k] * (double)s[k];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            V[a * 3 + c] = Rc[a * 3] * Rc[c * 3] * D[0] + Rc[a * 3 + 1] * Rc[c * 3 + 1] * D[1] +
                           Rc[a * 3 + 2] * Rc[c * 3 + 2] * D[2];
    const double rz = 1.0 / mz;
    // J = [[j00, 0, j02], [0, j11, j12]]
    const double j00 = vi.fx * rz, j02 = -vi.fx * mx * rz * rz;
    const double j11 = vi.fy * rz, j12 = -vi.fy * my * rz * rz;
    const double J[6] = { j00, 0.0, j02, 0.0, j11, j12 };
    double JV[6];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c)
            JV[a * 3 + c] = J[a * 3] * V[c] + J[a * 3 + 1] * V[3 + c] + J[a * 3 + 2] * V[6 + c];
    const double S00 = JV[0] * J[0] + JV[1] * J[1] + JV[2] * J[2];
    const double S01 = JV[0] * J[3] + JV[1] * J[4] + JV[2] * J[5];
    const double S11 = JV[3] * J[3] + JV[4] * J[4] + JV[5] * J[5];
    const double rdet = 1.0 / (S00 * S11 - S01 * S01);
    const double C00 = S11 * rdet, C01 = -S01 * rdet, C11 = S00 * rdet;
    // dL/dSigma' = C N C / 2 with N = [[A, B], [B, Cq]]
    const double A = gr[0], B = gr[1], Cq = gr[2];
    const double T00 = C00 * A + C01 * B, T01 = C00 * B + C01 * Cq;
    const double T10 = C01 * A + C11 * B, T11 = C01 * B + C11 * Cq;
    const double G00 = 0.5 * (T00 * C00 + T01 * C01);
    const double G01 = 0.5 * (T00 * C01 + T01 * C11);
    const double G11 = 0.5 * (T10 * C01 + T11 * C11);
    const double GS[4] = { G00, G01, G01, G11 };
    // dL/dmu' = C (Px, Py)
    const double gpx = C00 * gr[3] + C01 * gr[4], gpy = C01 * gr[3] + C11 * gr[4];
    // dL/dV = J^T GS J;  dL/dJ = 2 GS J V
    double GV[9];
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            double acc = 0.0;
            for (int a = 0; a < 2; ++a)
                for (int c = 0; c < 2; ++c) acc += J[a * 3 + k] * GS[a * 2 + c] * J[c * 3 + l];
            GV[k * 3 + l] = acc;
        }
    double GJ[6];
    for (int a = 0; a < 2; ++a)
        for (int l = 0; l < 3; ++l)
            GJ[a * 3 + l] = 2.0 * (GS[a * 2] * JV[l] + GS[a * 2 + 1] * JV[3 + l]);
    // view-space mean: J(m) and mu' = (fx mx / mz + cx, fy my / mz + cy)
    const double rz2 = rz * rz, rz3 = rz2 * rz;
    double gm[3];
    gm[0] = -vi.fx * rz2 * GJ[2] + vi.fx * rz * gpx;
    gm[1] = -vi.fy * rz2 * GJ[5] + vi.fy * rz * gpy;
    gm[2] = -vi.fx * rz2 * GJ[0] + 2.0 * vi.fx * mx * rz3 * GJ[2] - vi.fy * rz2 * GJ[4] +
            2.0 * vi.fy * my * rz3 * GJ[5] - vi.fx * mx * rz2 * gpx - vi.fy * my * rz2 * gpy;
    for (int j = 0; j < 3; ++j)
        gmw[j] += (float)(vi.R[j] * gm[0] + vi.R[3 + j] * gm[1] + vi.R[6 + j] * gm[2]);
    // H = Rc^T GV Rc
    double GR[9], H[9];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            GR[a * 3 + c] = GV[a * 3] * Rc[c] + GV[a * 3 + 1] * Rc[3 + c] + GV[a * 3 + 2] * Rc[6 + c];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            H[a * 3 + c] = Rc[a] * GR[c] + Rc[3 + a] * GR[3 + c] + Rc[6 + a] * GR[6 + c];
    for (int k = 0; k < 3; ++k) gs[k] += (float)(2.0 * s[k] * H[k * 4]);
    gth[0] += (float)(2.0 * H[5] * (D[1] - D[2]));
    gth[1] += (float)(2.0 * H[2] * (D[2] - D[0]));
    gth[2] += (float)(2.0 * H[1] * (D[0] - D[1]));
}

template <int DEG, bool SPLAT>
__global__ __launch_bounds__(128) void preprocess_bwd_kernel(
    RenderParams rp, Buffers b, const float *__restrict__ means, const float *__restrict__ quats,
    const float *__restrict__ scales, const float *__restrict__ dens, const float *__restrict__ sh,
    float *__restrict__ d_means, float *__restrict__ d_quats, float *__restrict__ d_scales,
    float *__restrict__ d_dens, float *__restrict__ d_sh, int acc, float *__restrict__ gnorm,
    int32_t *__restrict__ vcount)
{
    constexpr int NB = (DEG + 1) * (DEG + 1);
    constexpr int NF = 3 * NB, LS = NF + 1;   // floats per Gaussian, LDS row stride
    // The block's SH gradients leave through LDS, so that HBM sees whole
    // lines written (a thread's own coefficients are NF floats apart from its
    // neighbours'; scattered partial-line stores without a prior read of the
    // lines are slow).
    __shared__ float s_sh[128 * LS];
    const int64_t blk0 = (int64_t)blockIdx.x * 128;
    const int64_t i = blk0 + threadIdx.x;
    const bool valid = i < rp.n;
    const bool color = rp.mode == VGR_MODE_COLOR && sh != nullptr;   // uniform
    // floats of the block's SH span that belong to real Gaussians
    const int64_t nvalid = (rp.n - blk0 < 128 ? rp.n - blk0 : 128) * NF;
    float gsh[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) gsh[k] = 0.f;
    bool any = false;
    if (valid) {
    const float mu[3] = { means[3 * i], means[3 * i + 1], means[3 * i + 2] };
    const float q[4] = { quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3] };
    const float s[3] = { scales[3 * i], scales[3 * i + 1], scales[3 * i + 2] };
    float gmu[3] = { 0.f, 0.f, 0.f }, gth[3] = { 0.f, 0.f, 0.f }, gs[3] = { 0.f, 0.f, 0.f };
    float gk = 0.f;
    float qn[4] = { 0.f, 0.f, 0.f, 0.f }, qlen = 1.f;
    // densification statistics: sum over views of |dL_v/dmu| and the views
    // in which the Gaussian had tiles
    const bool stats = gnorm != nullptr || vcount != nullptr;   // uniform
    float nsum = 0.f;
    int32_t nvis = 0;
    for (int v = 0; v < rp.n_views; ++v) {
        const int64_t item = (int64_t)v * rp.n + i;
        if (stats) nvis += b.counts[item] > 0u ? 1 : 0;
        const float4 *rg = b.rgrad + item * 4;
        const float4 r0 = rg[0], r1 = rg[1], r2 = rg[2], r3 = rg[3];
        const float gr[16] = { r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w,
                               r2.x, r2.y, r2.z, r2.w, r3.x, r3.y, r3.z, r3.w };
        bool nz = false;
#pragma unroll
        for (int k = 0; k < 16; ++k) nz |= gr[k] != 0.0f;
        if (!nz) continue;
        any = true;
        const ViewInfo &vi = b.views[v];
        GaussView g;
        gauss_view(vi, mu, q, s, g);
        for (int k = 0; k < 4; ++k) qn[k] = g.qn[k];
        qlen = g.qlen;
        gk += gr[9];   // sum t = K' dL/dK' = kappa dL/dkappa (splat: sum tau = o dL/do)
        float gmv[3] = { 0.f, 0.f, 0.f };   // this view's dL/dmu
        if constexpr (SPLAT) {
            splat_view_grad(g, s, mu, vi, gr, gmv, gs, gth);
        } else {
        // Sigma^-1 = Rc diag(s^-2) Rc^T with dL/dSigma^-1 = -1/2 L^-1 M L^-T, L^-1 = Rc diag(s),
        // so dL/dRc = -Rc diag(s) M diag(1/s):
        //   scales: dL/ds_k = M_kk / s_k;
        //   rotation: for the body-frame perturbation Rc -> Rc (I + [dtheta]x),
        //   dL/dtheta = vee(W - W^T) with W = Rc^T dL/dRc = -diag(s) M diag(1/s),
        //   i.e. dL/dtheta_x = M12 (s1/s2 - s2/s1) and cyclically.
        // near-plane segment: M -= p U^T + U p^T (p = L m) and Z -= U (U = 0 elsewhere)
        float Mm[6] = { gr[0], gr[1], gr[2], gr[3], gr[4], gr[5] };
        float Zm[3] = { gr[6], gr[7], gr[8] };
        if (rp.near_segment) {
            const float *U = gr + 13;
            Mm[0] -= 2.0f * g.p[0] * U[0];
            Mm[1] -= g.p[0] * U[1] + U[0] * g.p[1];
            Mm[2] -= g.p[0] * U[2] + U[0] * g.p[2];
            Mm[3] -= 2.0f * g.p[1] * U[1];
            Mm[4] -= g.p[1] * U[2] + U[1] * g.p[2];
            Mm[5] -= 2.0f * g.p[2] * U[2];
            for (int j = 0; j < 3; ++j) Zm[j] -= U[j];
        }
        for (int k = 0; k < 3; ++k) gs[k] += Mm[k == 0 ? 0 : (k == 1 ? 3 : 5)] * g.inv_s[k];
        gth[0] += Mm[4] * ((s[1] * s[1] - s[2] * s[2]) * g.inv_s[1] * g.inv_s[2]);
        gth[1] += Mm[2] * ((s[2] * s[2] - s[0] * s[0]) * g.inv_s[2] * g.inv_s[0]);
        gth[2] += Mm[1] * ((s[0] * s[0] - s[1] * s[1]) * g.inv_s[0] * g.inv_s[1]);
        // dL/dm = -L^T Z
        float dm[3];
        for (int j = 0; j < 3; ++j)
            dm[j] = -(g.L[j] * Zm[0] + g.L[3 + j] * Zm[1] + g.L[6 + j] * Zm[2]);
        // m = R_view mu + t
        for (int j = 0; j < 3; ++j)
            gmv[j] = vi.R[j] * dm[0] + vi.R[3 + j] * dm[1] + vi.R[6 + j] * dm[2];
        }   // volumetric record
        if (rp.mode == VGR_MODE_COLOR) {
            float vx = mu[0] - vi.o[0], vy = mu[1] - vi.o[1], vz = mu[2] - vi.o[2];
            const float len = sqrtf(vx * vx + vy * vy + vz * vz);
            const float il = 1.0f / len;
            vx *= il; vy *= il; vz *= il;
            float Y[16];
            sh_basis(DEG, vx, vy, vz, Y);
            float c3[NF];
            load_sh_row<NF>(sh, i, ((uintptr_t)sh & 15) == 0, c3);
            float graw[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float raw = 0.5f;
#pragma unroll
                for (int k = 0; k < NB; ++k) raw = fmaf(c3[k * 3 + ch], Y[k], raw);
                graw[ch] = gr[10 + ch] * act_grad(rp.act, raw);
            }
            // the direction gradient is sum_k w_k grad Y_k with w_k = sum_ch graw c_k
            float wk[16];
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                wk[k] = graw[0] * c3[k * 3] + graw[1] * c3[k * 3 + 1] + graw[2] * c3[k * 3 + 2];
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) gsh[k * 3 + ch] += graw[ch] * Y[k];
            }
            const float3 gv = sh_grad_dot(DEG, vx, vy, vz, wk);
            const float vg = vx * gv.x + vy * gv.y + vz * gv.z;
            gmv[0] += (gv.x - vx * vg) * il;
            gmv[1] += (gv.y - vy * vg) * il;
            gmv[2] += (gv.z - vz * vg) * il;
        }
        for (int j = 0; j < 3; ++j) gmu[j] += gmv[j];
        if (stats) nsum += sqrtf(gmv[0] * gmv[0] + gmv[1] * gmv[1] + gmv[2] * gmv[2]);
    }
    if (gnorm) gnorm[i] += nsum;
    if (vcount) vcount[i] += nvis;
    // acc: add to the caller's arrays; otherwise overwrite them (no read)
    auto put = [acc](float *p, float v) {
        if (acc) *p += v;
        else *p = v;
    };
    if (!any) {
        if (!acc) {   // nothing reached this Gaussian: its gradients are zero
            for (int j = 0; j < 3; ++j) d_means[3 * i + j] = 0.f;
            for (int j = 0; j < 4; ++j) d_quats[4 * i + j] = 0.f;
            for (int j = 0; j < 3; ++j) d_scales[3 * i + j] = 0.f;
            d_dens[i] = 0.f;
        }
    } else {
    for (int j = 0; j < 3; ++j) put(d_means + 3 * i + j, gmu[j]);
    // body-frame rotation gradient -> quaternion: q -> q (x) (1, dtheta/2), so
    // dL/dq = 2 q (x) (0, dL/dtheta) / |q| (already orthogonal to q)
    {
        const float w = qn[0], x = qn[1], y = qn[2], z = qn[3];
        const float c = 2.0f / qlen;
        put(d_quats + 4 * i + 0, c * -(x * gth[0] + y * gth[1] + z * gth[2]));
        put(d_quats + 4 * i + 1, c * (w * gth[0] + y * gth[2] - z * gth[1]));
        put(d_quats + 4 * i + 2, c * (w * gth[1] + z * gth[0] - x * gth[2]));
        put(d_quats + 4 * i + 3, c * (w * gth[2] + x * gth[1] - y * gth[0]));
    }
    // gk = kappa dL/dkappa.  Density input kappa: dL/dkappa = gk / kappa.
    // Input theta, kappa = phi(theta) h(s) with phi = -ln(1 - 0.99 theta) and
    // h = mean of 1/s_k: dL/dtheta = gk phi'/phi and dL/ds_k gains
    // gk d ln h / ds_k = -gk / (s_k^2 sum_j 1/s_j).
    if constexpr (SPLAT) {
        // opacity o = clamp(input, 0, 1): dL/do = sum tau / o
        const float o = dens[i];
        put(d_dens + i, (o < 0.0f || o > 1.0f) ? 0.0f : gk / o);
    } else if (rp.density == VGR_DENSITY_THETA) {
        const float th = dens[i];
        const float dth = (th < 0.0f || th > 1.0f)
                              ? 0.0f
                              : gk * (0.99f / (fmaf(-0.99f, th, 1.0f) * theta_log(th)));
        put(d_dens + i, dth);
        const float is[3] = { 1.0f / s[0], 1.0f / s[1], 1.0f / s[2] };
        const float r = gk / (is[0] + is[1] + is[2]);
        for (int k = 0; k < 3; ++k) gs[k] -= r * (is[k] * is[k]);
    } else {
        put(d_dens + i, gk / dens[i]);
    }
    for (int k = 0; k < 3; ++k) put(d_scales + 3 * i + k, gs[k]);
    }
    }   // valid
    if (color && d_sh) {
#pragma unroll
        for (int k = 0; k < NF; ++k) s_sh[threadIdx.x * LS + k] = gsh[k];
        __syncthreads();
        float4 o4[NF / 4 > 0 ? NF / 4 : 1];
#pragma unroll
        for (int r = 0; r < NF / 4; ++r) {
            const int e = 4 * (r * 128 + threadIdx.x);
            float f[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int g = (e + c) / NF;
                f[c] = s_sh[g * LS + (e + c - g * NF)];
            }
            o4[r] = make_float4(f[0], f[1], f[2], f[3]);
        }
        if (acc) {   // uniform: add the caller's values, all loads in flight first
            float4 a4[NF / 4 > 0 ? NF / 4 : 1];
#pragma unroll
            for (int r = 0; r < NF / 4; ++r) {
                const int64_t e = 4 * ((int64_t)r * 128 + threadIdx.x);
                a4[r] = e + 3 < nvalid ? *reinterpret_cast<const float4 *>(d_sh + blk0 * NF + e)
                                       : make_float4(0.f, 0.f, 0.f, 0.f);
                if (e + 3 >= nvalid) {
                    if (e < nvalid) a4[r].x = d_sh[blk0 * NF + e];
                    if (e + 1 < nvalid) a4[r].y = d_sh[blk0 * NF + e + 1];
                    if (e + 2 < nvalid) a4[r].z = d_sh[blk0 * NF + e + 2];
                }
            }
#pragma unroll
            for (int r = 0; r < NF / 4; ++r) {
                o4[r].x += a4[r].x; o4[r].y += a4[r].y; o4[r].z += a4[r].z; o4[r].w += a4[r].w;
            }
        }
#pragma unroll
        for (int r = 0; r < NF / 4; ++r) {
            const int64_t e = 4 * ((int64_t)r * 128 + threadIdx.x);
            float *dst = d_sh + blk0 * NF + e;
            if (e + 3 < nvalid) {
                *reinterpret_cast<float4 *>(dst) = o4[r];
            } else {
                if (e < nvalid) dst[0] = o4[r].x;
                if (e + 1 < nvalid) dst[1] = o4[r].y;
                if (e + 2 < nvalid) dst[2] = o4[r].z;
            }
        }
        for (int e = 4 * (NF / 4) * 128 + threadIdx.x; e < 128 * NF; e += 128) {
            if (e < nvalid) {
                const int g = e / NF;
                float *p = d_sh + blk0 * NF + e;
                const float v = s_sh[g * LS + (e - g * NF)];
                if (acc) *p += v;
                else *p = v;
            }
        }
    }
}

inline unsigned grid_for(int64_t n, int threads)
{
    int64_t g = (n + threads - 1) / threads;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    unsigned g = grid_for(n, 256);
    if (g > 4096) g = 4096;
    fill_u32_kernel<<<g, 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    unsigned g = grid_for(n, 256);
    if (g > 4096) g = 4096;
    fill_f32_kernel<<<g, 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_preprocess(const RenderParams &rp, const Buffers &b, const float *means,
                             const float *quats, const float *scales, const float *dens,
                             const float *sh, hipStream_t s)
{
    const unsigned grid = grid_for(rp.n, 256);
    const int deg = rp.mode == VGR_MODE_COLOR ? rp.sh_degree : 0;
    const bool multi = rp.n_views > 1, splat = rp.alpha_model == VGR_ALPHA_SPLAT;
#define VGR_PRE(D, M, S) preprocess_kernel<D, M, S><<<grid, 256, 0, s>>>(rp, b, means, quats, scales, dens, sh)
#define VGR_PRE_DEG(M, S)            \
    switch (deg) {                   \
    case 0: VGR_PRE(0, M, S); break; \
    case 1: VGR_PRE(1, M, S); break; \
    case 2: VGR_PRE(2, M, S); break; \
    default: VGR_PRE(3, M, S); break; \
    }
    if (splat) {
        if (multi) { VGR_PRE_DEG(true, true) } else { VGR_PRE_DEG(false, true) }
    } else {
        if (multi) { VGR_PRE_DEG(true, false) } else { VGR_PRE_DEG(false, false) }
    }
#undef VGR_PRE_DEG
#undef VGR_PRE
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    count_total_kernel<<<2, 256, 0, s>>>(b.blk_counts, (int64_t)grid,
                                         (int64_t)grid * rp.n_views, b.d_total, b.h_total);
    return hipGetLastError();
}

hipError_t launch_compact_items(const RenderParams &rp, const Buffers &b, hipStream_t s)
{
    const int64_t nb = grid_for(rp.n, 256);
    const int64_t blocks = nb * rp.n_views;
    if (blocks <= 0) return hipSuccess;
    compact_items_kernel<<<dim3((unsigned)blocks), 256, 0, s>>>(rp, b, nb);
    return hipGetLastError();
}

int64_t preprocess_blocks(int64_t n, int32_t n_views)
{
    // instance partial sums, then the per-(view, block) counts of items with
    // instances (one thread per Gaussian covers all views)
    return (1 + (int64_t)n_views) * (int64_t)grid_for(n, 256);
}

hipError_t launch_gather_counts(const Buffers &b, int64_t m, int32_t total_tiles,
                                uint32_t *partial, hipStream_t s)
{
    int64_t n = m > total_tiles ? m : total_tiles;
    if (n < 64) n = 64;
    gather_counts_kernel<<<grid_for(n, kGatherThreads), kGatherThreads, 0, s>>>(
        b.item_ids, b.counts, b.d_total + 6, b.cnt_sorted, m, partial, b.ranges, total_tiles,
        b.tile_key);
    return hipGetLastError();
}

hipError_t launch_emit(const RenderParams &rp, const Buffers &b, int64_t m, int64_t capacity,
                       hipStream_t s)
{
    emit_kernel<<<grid_for(m, 64), kEmitThreads, 0, s>>>(rp, b, m, capacity);   // 64 Gaussians per block
    return hipGetLastError();
}

hipError_t launch_ranges(const Buffers &b, int64_t bound, int32_t total_tiles, bool clear,
                         hipStream_t s)
{
    if (clear) {
        hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(b.ranges), 0u,
                                       2 * (int64_t)total_tiles, s);
        if (e != hipSuccess) return e;
    }
    if (bound <= 0) return hipSuccess;
    unsigned g = grid_for(bound, 256);
    if (g > 16384) g = 16384;
    ranges_kernel<<<g, 256, 0, s>>>(b.inst_key, b.d_total, b.ranges, bound, (uint32_t)total_tiles);
    return hipGetLastError();
}

hipError_t launch_resort_keys(const RenderParams &rp, const Buffers &b, uint32_t *key,
                              uint32_t *idx, int64_t bound, hipStream_t s)
{
    if (bound <= 0) return hipSuccess;
    unsigned g = grid_for(bound, 256);
    if (g > 16384) g = 16384;
    resort_key_kernel<<<g, 256, 0, s>>>(rp, b, key, idx, bound);
    return hipGetLastError();
}

hipError_t launch_resort_permute(const Buffers &b, const uint32_t *idx, uint32_t *tmp_key,
                                 uint32_t *tmp_val, int64_t bound, hipStream_t s)
{
    if (bound <= 0) return hipSuccess;
    unsigned g = grid_for(bound, 256);
    if (g > 16384) g = 16384;
    resort_gather_kernel<<<g, 256, 0, s>>>(b.d_total, b.inst_key, b.inst_val, idx, tmp_key,
                                           tmp_val, bound);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // and back (a plain copy of the first K entries)
    resort_gather_kernel<<<g, 256, 0, s>>>(b.d_total, tmp_key, tmp_val, nullptr, b.inst_key,
                                           b.inst_val, bound);
    return hipGetLastError();
}

hipError_t launch_tile_order(const Buffers &b, int32_t total_tiles, bool clear, hipStream_t s)
{
    if (total_tiles <= 0) return hipSuccess;
    uint32_t *hist = b.tile_key, *cursor = b.tile_key + 32;   // 64 words of scratch
    if (clear) {
        hipError_t e = launch_fill_u32(hist, 0u, 64, s);
        if (e != hipSuccess) return e;
    }
    tile_hist_kernel<<<grid_for(total_tiles, 256), 256, 0, s>>>(b.ranges, hist, total_tiles);
    tile_place_kernel<<<grid_for(total_tiles, 256), 256, 0, s>>>(b.ranges, hist, cursor,
                                                                  b.tile_order, total_tiles);
    return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const RenderParams &rp, const Buffers &b, const float *means,
                                 const float *quats, const float *scales, const float *dens,
                                 const float *sh, float *d_means, float *d_quats,
                                 float *d_scales, float *d_dens, float *d_sh, bool accumulate,
                                 float *gnorm, int32_t *vcount, hipStream_t s)
{
    const unsigned g = grid_for(rp.n, 128);
    const int acc = accumulate ? 1 : 0;
    const int deg = rp.mode == VGR_MODE_COLOR ? rp.sh_degree : 0;
#define VGR_PBW(D, S) preprocess_bwd_kernel<D, S><<<g, 128, 0, s>>>(rp, b, means, quats, scales, dens, sh, d_means, d_quats, d_scales, d_dens, d_sh, acc, gnorm, vcount)
#define VGR_PBW_DEG(S)            \
    switch (deg) {                \
    case 0: VGR_PBW(0, S); break; \
    case 1: VGR_PBW(1, S); break; \
    case 2: VGR_PBW(2, S); break; \
    default: VGR_PBW(3, S); break; \
    }
    if (rp.alpha_model == VGR_ALPHA_SPLAT) {
        VGR_PBW_DEG(true)
    } else {
        VGR_PBW_DEG(false)
    }
#undef VGR_PBW_DEG
#undef VGR_PBW
    return hipGetLastError();
}

}  // namespace vgr
