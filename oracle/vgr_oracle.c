/*
 * FP64 reference renderer for volumetrically consistent 3D Gaussian
 * rasterisation (arXiv 2412.03378).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the HIP library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the library never does.  It shares no
 * code, header, table or constant with the HIP path.
 *
 * Everything is evaluated per pixel, over every Gaussian, in double precision,
 * straight from the paper's definitions, in world space:
 *
 *   density field        sigma(x) = sum_i kappa_i G_i(x)                (Sec. 3.2, eq. gauss_mixture)
 *   unnormalised Gaussian G_i(x) = exp(-1/2 (x-mu)^T Sigma^-1 (x-mu))   (Sec. 3.2, eq. 3dgs_pdf)
 *   ray                   r(t) = o + t d, |d| = 1, through the pixel centre
 *   1D Gaussian on a ray  gamma = (mu-o)^T Sigma^-1 d / d^T Sigma^-1 d,
 *                         beta  = (d^T Sigma^-1 d)^(-1/2)                (Sec. 4.2, eq. betagamma)
 *   full-line integral    x = kappa sqrt(2 pi) beta G(o + gamma d),
 *                         alpha = 1 - exp(-x)                            (Sec. 4.2, eq. our_trans_final)
 *   compositing           C = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j) (Sec. 4.1, eq. our_alpha_blend)
 *   X-ray mode            I = sum_i x_i  (order independent)             (Sec. 6.2)
 *
 * Readings where the paper is silent (each is a settings field):
 *   - Gaussians whose view-space mean depth is <= znear are dropped; the
 *     remaining ones are composited in ascending (depth key, index) order,
 *     where the depth key is the FP32 value fmaf(R20,mx, fmaf(R21,my,
 *     fmaf(R22,mz, t2))) so that both implementations order ties identically.
 *   - a Gaussian is skipped when alpha < alpha_min (x < -ln(1-alpha_min));
 *     alpha is clamped to alpha_max (zero gradient when clamped);
 *   - compositing stops before Gaussian i when T (1 - alpha_i) < T_min
 *     (Gaussian i is not blended); afterwards C += T bg.
 *   - colour c = act(sum_k sh_k Y_k(v) + 0.5), v = normalize(mu - o), with
 *     real orthonormal spherical harmonics (Condon-Shortley phase), act =
 *     max(.,0) or softplus with sharpness 10 (Supp. D).
 *   - comparison model (alpha_model = 1): the 3DGS splatting opacity the
 *     paper replaces (Sec. 3, eq. 3dgs_alpha, eq. affine_approx), with the
 *     density input read as the peak opacity o in [0, 1] (clamped) and the
 *     same compositing rules; its backward is the analytic chain of
 *     chain_splat.
 *   - near_segment = 1: the integral along each ray starts where the ray
 *     crosses the near plane z = znear instead of covering the whole line,
 *     x = kappa sqrt(2 pi) beta G(o + gamma d) Phi((gamma - t_n) / beta), Phi the
 *     standard normal distribution function (Sec. 4.2, the finite-limit erf
 *     form with the argument (t - gamma) / (sqrt 2 beta)).
 *   - tile_resort = 1 (colour mode): instead of the mean depth, each pixel
 *     composites in ascending order of gamma on the ray through the centre of
 *     its tile_w x tile_h screen tile (the position of each Gaussian's maximum
 *     along that ray; ties by the depth key, then the index): the per-tile
 *     level of the re-sorting that the paper points to against popping
 *     (Sec. 7, Limitations).  Each pixel reports the smallest relative gap
 *     between the keys of two Gaussians that reach it as its order margin.
 *   - pixel_window = W > 0 (with tile_resort): the per-pixel level of that
 *     re-sorting.  The Gaussians that reach alpha_min at a pixel, in the
 *     per-tile order, pass through a window of W entries kept in ascending
 *     gamma on the pixel's own ray (ties by list position); when it is full
 *     the smallest entry is composited, and at the end of the list the rest
 *     in order; termination ends the pixel.  The order margin adds, over the
 *     pops, the relative gap between the entry taken and the next smallest.
 *   - the density input is kappa itself, or theta with the reparameterisation
 *     kappa = -ln(1 - 0.99 theta) (1/s_x + 1/s_y + 1/s_z) / 3 (Sec. 5, eq.
 *     density_reparam); theta outside the paper's range [0, 1] is clamped to
 *     it, with zero gradient outside.
 *
 * Decision margins: for every threshold test that decides the output (skip,
 * clamp, X-ray cut; terminate) the oracle reports the smallest relative
 * distance to the threshold in units of that value's FP32 error amplification
 * (see dec_margin), and under tile_resort the smallest relative gap between
 * the order keys of two Gaussians that reach the pixel, so callers can set
 * aside pixels where two results are both correct up to rounding.
 *
 * The backward pass is the analytic chain rule of the same formulas, with the
 * transmittance in front of each Gaussian taken from forward prefix products.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

typedef struct {
    float R[9];     /* world -> view rotation, row-major */
    float t[3];     /* world -> view translation */
    float fx, fy, cx, cy;
    int32_t width, height;
    float znear;
    int32_t pad;
} orc_camera;

typedef struct {
    int32_t mode;       /* 0 colour, 1 X-ray */
    int32_t sh_degree;  /* 0..3 */
    int32_t act;        /* 0 max(.,0), 1 softplus(10 y)/10 */
    int32_t density;    /* 0: dens holds kappa; 1: dens holds theta (kappa_of) */
    int32_t alpha_model;/* 0: the paper's ray integral; 1: 3DGS splatting (splat_setup) */
    int32_t near_segment;/* 1: integrate each ray from the near plane on (finite segment) */
    int32_t tile_resort; /* 1: per-tile order by the depth of each Gaussian's maximum */
    int32_t tile_w, tile_h;
    int32_t kernel;     /* 0: Gaussian; 1: Epanechnikov (compact, see ray_integral) */
    int32_t pixel_window; /* > 0 (with tile_resort): per-pixel re-sorting window (shade_pixel) */
    int32_t pad3;
    double alpha_min, alpha_max, T_min, x_min_xray;
    double bg[3];
    double near_threshold; /* > 0, X-ray backward only: chain just the pairs whose
                              x-decision margin is below this value (see orc_render_backward) */
} orc_settings;

/* ------------------------------------------------------------------------ */
/* small linear algebra                                                      */

static void quat_rotation(const float qf[4], double R[9], double qn[4], double *qlen)
{
    double w = qf[0], x = qf[1], y = qf[2], z = qf[3];
    double len = sqrt(w * w + x * x + y * y + z * z);
    w /= len; x /= len; y /= len; z /= len;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
    if (qn) { qn[0] = w; qn[1] = x; qn[2] = y; qn[3] = z; }
    if (qlen) *qlen = len;
}

/* Sigma^-1 = R diag(s^-2) R^T  (row-major 3x3) */
static void precision_matrix(const double R[9], const float s[3], double P[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k)
                acc += R[i * 3 + k] * R[j * 3 + k] / ((double)s[k] * (double)s[k]);
            P[i * 3 + j] = acc;
        }
}

static double quad_form(const double P[9], const double a[3], const double b[3])
{
    double acc = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) acc += a[i] * P[i * 3 + j] * b[j];
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Ray integral of one Gaussian (Sec. 4.2).                                  */

typedef struct {
    double gamma, beta, Gmax, x;
    double v[3];     /* mu - (o + gamma d) */
    double a;        /* d^T P d */
    double D2;       /* v^T P v, the minimum Mahalanobis distance squared of the ray */
} ray_terms;

/* Line integral of kappa K(r^2), r^2 = (x-mu)^T P (x-mu), along o + t d.  On
   the ray r^2 = (t - gamma)^2 / beta^2 + D^2 (Sec. 4.2, eq. betagamma), so
     Gaussian      K = exp(-r^2/2):       x = kappa sqrt(2 pi) beta exp(-D^2/2)
     Epanechnikov  K = max(0, 1 - r^2):   x = kappa beta int_{|s| < h} (h^2 - s^2) ds
                                            = (4/3) kappa beta h^3, h^2 = 1 - D^2 > 0
   (0 where the ray misses the support, D^2 >= 1; the compact kernel of Sec. 8,
   future work).  kernel selects the profile; gamma, beta, D^2 are shared. */
static void ray_integral(const double mu[3], const double P[9], double kappa,
                         const double o[3], const double d[3], ray_terms *rt, int kernel)
{
    double dm[3] = { mu[0] - o[0], mu[1] - o[1], mu[2] - o[2] };
    double a = quad_form(P, d, d);
    double b = quad_form(P, dm, d);
    double gamma = b / a;
    double beta = 1.0 / sqrt(a);
    double xp[3], diff[3];
    for (int k = 0; k < 3; ++k) {
        xp[k] = o[k] + gamma * d[k];
        diff[k] = xp[k] - mu[k];
    }
    const double D2 = quad_form(P, diff, diff);
    double Gmax = exp(-0.5 * D2);
    rt->D2 = D2;
    rt->gamma = gamma;
    rt->beta = beta;
    rt->Gmax = Gmax;
    rt->a = a;
    for (int k = 0; k < 3; ++k) rt->v[k] = -diff[k];
    if (kernel == 1) {
        const double h2 = 1.0 - D2;
        rt->x = h2 > 0.0 ? kappa * (4.0 / 3.0) * beta * h2 * sqrt(h2) : 0.0;
    } else {
        rt->x = kappa * sqrt(2.0 * ORC_PI) * beta * Gmax;
    }
}

/* d ln x / d D^2 of the kernel's line integral: -1/2 (Gaussian), -(3/2)/(1 - D^2)
   (Epanechnikov, inside the support). */
static double dlnx_dD2(int kernel, double D2)
{
    return kernel == 1 ? -1.5 / (1.0 - D2) : -0.5;
}

/* Standard normal distribution function and density. */
static double norm_cdf(double e) { return 0.5 * erfc(-e / sqrt(2.0)); }
static double norm_pdf(double e) { return exp(-0.5 * e * e) / sqrt(2.0 * ORC_PI); }

/* Ray parameter t_n at which the unit ray o + t d crosses the near plane
   z_view = znear (o is the camera centre, so z_view(t) = t zrow . d). */
static double near_t(const double zrow[3], double znear, const double d[3])
{
    return znear / (zrow[0] * d[0] + zrow[1] * d[1] + zrow[2] * d[2]);
}

/* Exported for closed-form pins: out = {gamma, beta, Gmax, x}. */
int orc_ray_integral(const float mean[3], const float quat[4], const float scale[3],
                     float dens, const double o[3], const double d[3], int kernel, double out[4])
{
    double R[9], P[9], mu[3] = { mean[0], mean[1], mean[2] };
    quat_rotation(quat, R, NULL, NULL);
    precision_matrix(R, scale, P);
    ray_terms rt;
    ray_integral(mu, P, (double)dens, o, d, &rt, kernel);
    out[0] = rt.gamma; out[1] = rt.beta; out[2] = rt.Gmax; out[3] = rt.x;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics from the associated Legendre functions.          */
/*   Y_l^0  = K_l^0 P_l(z)                                                   */
/*   Y_l^m  = sqrt2 K_l^m (-1)^m (d^m P_l/dz^m)(z) Re((x+iy)^m)   m > 0       */
/*   Y_l^-m = sqrt2 K_l^m (-1)^m (d^m P_l/dz^m)(z) Im((x+iy)^m)   m > 0       */
/* with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), valid on the unit sphere  */
/* (sin^m(theta) e^{i m phi} = (x+iy)^m).  Index k = l^2 + l + m.            */
/* The gradient is that of this polynomial extension; callers project it     */
/* onto the tangent plane.                                                   */

#define ORC_MAX_DEG 4

static double polyval(const double *c, int n, double z)
{
    double acc = 0;
    for (int k = n - 1; k >= 0; --k) acc = acc * z + c[k];
    return acc;
}

static double factorial(int n)
{
    double f = 1;
    for (int k = 2; k <= n; ++k) f *= k;
    return f;
}

int orc_sh_basis(int deg, const double v[3], double *Y, double *dY)
{
    if (deg < 0 || deg > ORC_MAX_DEG) return -1;
    /* Legendre polynomial coefficients by Bonnet's recurrence */
    double Pl[ORC_MAX_DEG + 2][ORC_MAX_DEG + 2];
    memset(Pl, 0, sizeof Pl);
    Pl[0][0] = 1;
    Pl[1][1] = 1;
    for (int l = 1; l < ORC_MAX_DEG; ++l)
        for (int k = 0; k <= l + 1; ++k) {
            double zp = k > 0 ? Pl[l][k - 1] : 0;
            Pl[l + 1][k] = ((2 * l + 1) * zp - l * Pl[l - 1][k]) / (l + 1);
        }
    double x = v[0], y = v[1], z = v[2];
    /* powers (x+iy)^m */
    double re[ORC_MAX_DEG + 1], im[ORC_MAX_DEG + 1];
    re[0] = 1; im[0] = 0;
    for (int m = 1; m <= ORC_MAX_DEG; ++m) {
        re[m] = re[m - 1] * x - im[m - 1] * y;
        im[m] = re[m - 1] * y + im[m - 1] * x;
    }
    for (int l = 0; l <= deg; ++l) {
        /* derivatives d^m P_l / dz^m for m = 0..l+1 */
        double D[ORC_MAX_DEG + 3][ORC_MAX_DEG + 2];
        memset(D, 0, sizeof D);
        for (int k = 0; k <= l; ++k) D[0][k] = Pl[l][k];
        for (int m = 1; m <= l + 1; ++m)
            for (int k = 0; k <= l; ++k) D[m][k] = (k + 1 <= l) ? (k + 1) * D[m - 1][k + 1] : 0;
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double K = sqrt((2 * l + 1) / (4 * ORC_PI) * factorial(l - am) / factorial(l + am));
            double dm = polyval(D[am], l + 1, z);
            double dm1 = polyval(D[am + 1], l + 1, z);
            int k = l * l + l + m;
            double yv, gx, gy, gz;
            if (m == 0) {
                yv = K * dm; gx = 0; gy = 0; gz = K * dm1;
            } else {
                double c = sqrt(2.0) * K * ((am & 1) ? -1.0 : 1.0);
                if (m > 0) {
                    yv = c * dm * re[am];
                    gx = c * dm * am * re[am - 1];
                    gy = -c * dm * am * im[am - 1];
                    gz = c * dm1 * re[am];
                } else {
                    yv = c * dm * im[am];
                    gx = c * dm * am * im[am - 1];
                    gy = c * dm * am * re[am - 1];
                    gz = c * dm1 * im[am];
                }
            }
            Y[k] = yv;
            if (dY) { dY[3 * k] = gx; dY[3 * k + 1] = gy; dY[3 * k + 2] = gz; }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Per-view set-up                                                           */

typedef struct {
    int64_t n;
    int64_t nvis;
    int64_t *order;      /* visible Gaussians, ascending (key, index) */
    float *key;
    double *P;           /* n x 9 world-space Sigma^-1 */
    double *rgb;         /* n x 3 colour for this view */
    double *raw;         /* n x 3 colour before activation */
    double *kappa;       /* n densities kappa */
    double *splat;       /* alpha_model 1: n x 6 (mu'_x, mu'_y, C00, C01, C11, o) */
    double *aniso;       /* n: s_max / s_min (error amplification, see dec_margin) */
    double o[3];
    double zrow[3];      /* view-space depth axis in world coordinates (third row of R) */
    double znear;
} view_state;

static const float *g_sort_key;

static int cmp_key(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    float ka = g_sort_key[a], kb = g_sort_key[b];
    if (ka < kb) return -1;
    if (ka > kb) return 1;
    return (a > b) - (a < b);
}

static double act_apply(int act, double y)
{
    if (act == 1) {
        double s = 10.0 * y;
        return (s > 0 ? s + log1p(exp(-s)) : log1p(exp(s))) / 10.0;
    }
    return y > 0 ? y : 0;
}

static double act_grad(int act, double y)
{
    if (act == 1) return 1.0 / (1.0 + exp(-10.0 * y));
    return y > 0 ? 1.0 : 0.0;
}

/* Inverse of the world->view rotation as stored (FP32 storage makes R only
   approximately orthonormal, so the exact inverse of the affine map is used). */
static void inverse3(const float *Rf, double Ri[9])
{
    double R[9];
    for (int k = 0; k < 9; ++k) R[k] = Rf[k];
    double c0 = R[4] * R[8] - R[5] * R[7];
    double c1 = R[5] * R[6] - R[3] * R[8];
    double c2 = R[3] * R[7] - R[4] * R[6];
    double det = R[0] * c0 + R[1] * c1 + R[2] * c2;
    Ri[0] = c0 / det; Ri[1] = (R[2] * R[7] - R[1] * R[8]) / det; Ri[2] = (R[1] * R[5] - R[2] * R[4]) / det;
    Ri[3] = c1 / det; Ri[4] = (R[0] * R[8] - R[2] * R[6]) / det; Ri[5] = (R[2] * R[3] - R[0] * R[5]) / det;
    Ri[6] = c2 / det; Ri[7] = (R[1] * R[6] - R[0] * R[7]) / det; Ri[8] = (R[0] * R[4] - R[1] * R[3]) / det;
}

/* world-space camera centre o = -R^-1 t */
static void camera_origin(const orc_camera *cam, double o[3])
{
    double Ri[9];
    inverse3(cam->R, Ri);
    for (int i = 0; i < 3; ++i)
        o[i] = -(Ri[i * 3] * cam->t[0] + Ri[i * 3 + 1] * cam->t[1] + Ri[i * 3 + 2] * cam->t[2]);
}

/* world-space unit direction of the ray through the centre of pixel (px, py):
   the view-space ray s*u with u = ((px+0.5-cx)/fx, (py+0.5-cy)/fy, 1) */
static void pixel_ray(const orc_camera *cam, int px, int py, double d[3])
{
    double u[3] = { ((double)px + 0.5 - cam->cx) / cam->fx,
                    ((double)py + 0.5 - cam->cy) / cam->fy, 1.0 };
    double Ri[9];
    inverse3(cam->R, Ri);
    double len = 0;
    for (int i = 0; i < 3; ++i) {
        d[i] = Ri[i * 3] * u[0] + Ri[i * 3 + 1] * u[1] + Ri[i * 3 + 2] * u[2];
        len += d[i] * d[i];
    }
    len = sqrt(len);
    for (int i = 0; i < 3; ++i) d[i] /= len;
}

/* world-space unit direction of the ray through image point (X, Y) (pixel
   units, pixel p spans [p, p + 1]) */
static void point_ray(const orc_camera *cam, double X, double Y, double d[3])
{
    double u[3] = { (X - cam->cx) / cam->fx, (Y - cam->cy) / cam->fy, 1.0 };
    double Ri[9];
    inverse3(cam->R, Ri);
    double len = 0;
    for (int i = 0; i < 3; ++i) {
        d[i] = Ri[i * 3] * u[0] + Ri[i * 3 + 1] * u[1] + Ri[i * 3 + 2] * u[2];
        len += d[i] * d[i];
    }
    len = sqrt(len);
    for (int i = 0; i < 3; ++i) d[i] /= len;
}

static float depth_key(const orc_camera *cam, const float *mu)
{
    const float *R = cam->R;
    return fmaf(R[6], mu[0], fmaf(R[7], mu[1], fmaf(R[8], mu[2], cam->t[2])));
}

/* Density kappa of a Gaussian from its density input and scales: the input
   itself, or, for the reparameterisation of Sec. 5 (eq. density_reparam),
   kappa = -ln(1 - 0.99 theta) (1/s_x + 1/s_y + 1/s_z) / 3 with theta in [0, 1]. */
static double theta_clamped(float th)
{
    return th < 0.0f ? 0.0 : (th > 1.0f ? 1.0 : (double)th);
}

static double kappa_of(const orc_settings *st, float dens, const float s[3])
{
    if (st->density == 0) return (double)dens;
    double h = (1.0 / s[0] + 1.0 / s[1] + 1.0 / s[2]) / 3.0;
    return -log1p(-0.99 * theta_clamped(dens)) * h;
}

/* d kappa / d(input) and d kappa / d s_k of kappa_of. */
static void kappa_grad(const orc_settings *st, float dens, const float s[3], double *dk_din,
                       double dk_ds[3])
{
    if (st->density == 0) {
        *dk_din = 1.0;
        dk_ds[0] = dk_ds[1] = dk_ds[2] = 0.0;
        return;
    }
    double th = theta_clamped(dens);
    double h = (1.0 / s[0] + 1.0 / s[1] + 1.0 / s[2]) / 3.0;
    double phi = -log1p(-0.99 * th);
    *dk_din = (dens < 0.0f || dens > 1.0f) ? 0.0 : 0.99 / (1.0 - 0.99 * th) * h;
    for (int k = 0; k < 3; ++k) dk_ds[k] = -phi / (3.0 * (double)s[k] * (double)s[k]);
}

/* 3DGS splatting of Gaussian (mu, R, s) in camera cam (Sec. 3, eq. 3dgs_alpha
   and eq. affine_approx): the 2D mean mu' is the projection of the view-space
   mean m = W mu + t, and the 2D covariance Sigma' = J W Sigma W^T J^T with W the
   world-to-view rotation, Sigma = R diag(s^2) R^T and J the Jacobian of the
   pinhole map (x, y, z) -> (fx x/z + cx, fy y/z + cy) at m.  out = (mu'_x,
   mu'_y, C00, C01, C11, o) with C = Sigma'^-1 and o the peak opacity in [0, 1]. */
static void splat_setup(const orc_camera *cam, const float *mu, const double R[9],
                        const float s[3], float dens, double out[6])
{
    const float *Wf = cam->R;
    double m[3];
    for (int a = 0; a < 3; ++a)
        m[a] = (double)Wf[3 * a] * mu[0] + (double)Wf[3 * a + 1] * mu[1] +
               (double)Wf[3 * a + 2] * mu[2] + (double)cam->t[a];
    double S[9], WS[9], V[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k)
                acc += R[i * 3 + k] * R[j * 3 + k] * (double)s[k] * (double)s[k];
            S[i * 3 + j] = acc;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += (double)Wf[i * 3 + k] * S[k * 3 + j];
            WS[i * 3 + j] = acc;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += WS[i * 3 + k] * (double)Wf[j * 3 + k];
            V[i * 3 + j] = acc;
        }
    const double fx = cam->fx, fy = cam->fy, z = m[2];
    const double J[6] = { fx / z, 0.0, -fx * m[0] / (z * z), 0.0, fy / z, -fy * m[1] / (z * z) };
    double Sp[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double acc = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) acc += J[a * 3 + i] * V[i * 3 + j] * J[b * 3 + j];
            Sp[a * 2 + b] = acc;
        }
    const double det = Sp[0] * Sp[3] - Sp[1] * Sp[2];
    out[0] = fx * m[0] / z + cam->cx;
    out[1] = fy * m[1] / z + cam->cy;
    out[2] = Sp[3] / det;
    out[3] = -0.5 * (Sp[1] + Sp[2]) / det;
    out[4] = Sp[0] / det;
    out[5] = dens < 0.0f ? 0.0 : (dens > 1.0f ? 1.0 : (double)dens);
}

static int view_setup(view_state *vs, int64_t n, const float *means, const float *quats,
                      const float *scales, const float *dens, const float *sh,
                      const orc_camera *cam, const orc_settings *st)
{
    memset(vs, 0, sizeof *vs);
    vs->n = n;
    vs->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    vs->key = (float *)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    vs->P = (double *)malloc(sizeof(double) * 9 * (size_t)(n > 0 ? n : 1));
    vs->rgb = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    vs->raw = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    vs->kappa = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    vs->aniso = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!vs->order || !vs->key || !vs->P || !vs->rgb || !vs->raw || !vs->kappa || !vs->aniso)
        return -3;
    if (st->alpha_model == 1) {
        vs->splat = (double *)malloc(sizeof(double) * 6 * (size_t)(n > 0 ? n : 1));
        if (!vs->splat) return -3;
    }
    camera_origin(cam, vs->o);
    for (int k = 0; k < 3; ++k) vs->zrow[k] = cam->R[6 + k];
    vs->znear = cam->znear;
    int nb = (st->sh_degree + 1) * (st->sh_degree + 1);
    int64_t nvis = 0;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double R[9];
        quat_rotation(quats + 4 * i, R, NULL, NULL);
        precision_matrix(R, scales + 3 * i, vs->P + 9 * i);
        vs->kappa[i] = kappa_of(st, dens[i], scales + 3 * i);
        {
            const float *sc = scales + 3 * i;
            const double smax = fmax(sc[0], fmax(sc[1], sc[2]));
            const double smin = fmin(sc[0], fmin(sc[1], sc[2]));
            vs->aniso[i] = smax / smin;
        }
        if (vs->splat) splat_setup(cam, means + 3 * i, R, scales + 3 * i, dens[i], vs->splat + 6 * i);
        vs->key[i] = depth_key(cam, means + 3 * i);
        if (st->mode == 0) {
            double v[3], len = 0, Y[(ORC_MAX_DEG + 1) * (ORC_MAX_DEG + 1)];
            for (int k = 0; k < 3; ++k) { v[k] = means[3 * i + k] - vs->o[k]; len += v[k] * v[k]; }
            len = sqrt(len);
            for (int k = 0; k < 3; ++k) v[k] /= len;
            orc_sh_basis(st->sh_degree, v, Y, NULL);
            for (int ch = 0; ch < 3; ++ch) {
                double acc = 0.5;
                for (int k = 0; k < nb; ++k) acc += sh[((size_t)i * nb + k) * 3 + ch] * Y[k];
                vs->raw[3 * i + ch] = acc;
                vs->rgb[3 * i + ch] = act_apply(st->act, acc);
            }
        }
    }
    for (int64_t i = 0; i < n; ++i)
        if (vs->key[i] > cam->znear) vs->order[nvis++] = i;
    g_sort_key = vs->key;
    qsort(vs->order, (size_t)nvis, sizeof(int64_t), cmp_key);
    vs->nvis = nvis;
    return 0;
}

static void view_free(view_state *vs)
{
    free(vs->order); free(vs->key); free(vs->P); free(vs->rgb); free(vs->raw); free(vs->kappa);
    free(vs->splat); free(vs->aniso);
}

/* Decision margins.  A test of a computed value v against a threshold can go
   the other way in an FP32 implementation only if the relative rounding error
   of v reaches |v - thr| / |v|.  That error is a few units of roundoff times
   an amplification factor `amp' that depends on the decision: for a line
   integral x = kappa sqrt(2 pi) beta exp(-D^2/2), a relative error e in D^2
   becomes D^2 e/2 in x, and a rotation error of angle e (the rounding of a
   rotation matrix) changes D^2 by up to about D^2 e s_max/s_min for a Gaussian
   with scales s, so amp = 1 + (D^2/2) s_max/s_min (plus, with the near-plane
   factor Phi(eta), h(eta) (|gamma| + t_n)/beta, h = phi/Phi, for an error in
   eta proportional to the lengths it is formed from); for the splatting
   opacity alpha = o exp(-q/2), with q from the inverse of a 2x2 covariance
   whose rounding is amplified by its condition number c, amp = 1 + c q/2;
   for the transmittance T (1 - alpha_i) after a run of blends, the
   amplifications of its factors 1 - alpha_j (x_j times the amplification of
   x_j, or alpha_j/(1 - alpha_j) times that of a splat's alpha_j, 0 for a
   clamped alpha), each plus one rounding for the product, combined as a
   root sum of squares: the roundings of different factors are independent,
   so their sum grows like a random walk (the probabilistic rounding-error
   analysis of Higham and Mary, SIAM J. Sci. Comput. 2019) rather than like
   the worst-case sum.  The margin
   reported is |v - thr| / (|v| amp): the relative distance in units of the
   amplified error, so one bound in units of roundoff decides which pixels
   have two correct results. */
static double dec_margin(double v, double thr, double amp)
{
    if (v == 0.0) return v == thr ? 0.0 : INFINITY;
    return fabs(v - thr) / (fabs(v) * amp);
}

/* amplification of the line integral's relative error (see dec_margin) */
static double x_amp(const ray_terms *rt, int kernel, double aniso, int near, double eta,
                    double tn)
{
    /* |d ln x / d ln D^2|: D^2/2 (Gaussian), (3/2) D^2/(1 - D^2) (Epanechnikov) */
    double amp = 1.0 + fabs(dlnx_dD2(kernel, rt->D2)) * rt->D2 * aniso;
    if (near) {
        const double Phi = norm_cdf(eta);
        const double h = Phi > 0 ? norm_pdf(eta) / Phi : fabs(eta);
        amp += h * (fabs(rt->gamma) + tn) / rt->beta;
    }
    return amp;
}

/* ------------------------------------------------------------------------ */
/* Per-tile order (tile_resort).                                             */

typedef struct {
    double g;      /* gamma on the tile-centre ray */
    float key;     /* depth key of the mean */
    int64_t idx;
} resort_item;

static int cmp_resort(const void *pa, const void *pb)
{
    const resort_item *a = (const resort_item *)pa, *b = (const resort_item *)pb;
    if (a->g < b->g) return -1;
    if (a->g > b->g) return 1;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

/* Order of the visible Gaussians for pixel (px, py) under tile_resort, into
   order[nvis]; returns the smallest relative gap between consecutive gammas
   of Gaussians whose integral at the pixel (ray d) reaches the skip
   threshold tau (INFINITY if fewer than two). */
static double resort_order(const view_state *vs, const float *means, const orc_camera *cam,
                           const orc_settings *st, int px, int py, const double d[3], double tau,
                           int64_t *order)
{
    const int tx = px / st->tile_w, ty = py / st->tile_h;
    double dc[3];
    point_ray(cam, tx * st->tile_w + 0.5 * st->tile_w, ty * st->tile_h + 0.5 * st->tile_h, dc);
    resort_item *it = (resort_item *)malloc(sizeof(resort_item) * (size_t)(vs->nvis > 0 ? vs->nvis : 1));
    for (int64_t r = 0; r < vs->nvis; ++r) {
        const int64_t i = vs->order[r];
        const double mu[3] = { means[3 * i], means[3 * i + 1], means[3 * i + 2] };
        ray_terms rt;
        ray_integral(mu, vs->P + 9 * i, 1.0, vs->o, dc, &rt, 0);
        it[r].g = rt.gamma;
        it[r].key = vs->key[i];
        it[r].idx = i;
    }
    qsort(it, (size_t)vs->nvis, sizeof(resort_item), cmp_resort);
    double gap = INFINITY, prev = NAN;
    for (int64_t r = 0; r < vs->nvis; ++r) {
        const int64_t i = it[r].idx;
        order[r] = i;
        const double mu[3] = { means[3 * i], means[3 * i + 1], means[3 * i + 2] };
        ray_terms rt;
        ray_integral(mu, vs->P + 9 * i, vs->kappa[i], vs->o, d, &rt, st->kernel);
        if (rt.x < tau) continue;
        if (!isnan(prev)) {
            const double m = fabs(it[r].g - prev) / fmax(fabs(it[r].g), 1e-300);
            if (m < gap) gap = m;
        }
        prev = it[r].g;
    }
    free(it);
    return gap;
}

/* ------------------------------------------------------------------------ */
/* Forward.                                                                  */

typedef struct {
    int64_t idx;
    double x, alpha, T;   /* T: transmittance in front of this Gaussian */
    int clamped;
} blend_rec;

typedef struct {
    blend_rec *rec;
    int64_t cnt, cap;
} blend_list;

static void list_push(blend_list *bl, blend_rec r)
{
    if (bl->cnt == bl->cap) {
        bl->cap = bl->cap ? 2 * bl->cap : 64;
        bl->rec = (blend_rec *)realloc(bl->rec, sizeof(blend_rec) * (size_t)bl->cap);
    }
    bl->rec[bl->cnt++] = r;
}

/* A Gaussian that reaches alpha_min at the pixel: index, list position,
   line integral, (clamped) alpha, amplification of its 1 - alpha, gamma on
   the pixel's ray. */
typedef struct {
    int64_t idx, pos;
    double x, alpha, amp_om, gamma;
    int clamped;
} cand_rec;

#define ORC_MAX_WINDOW 64

/* Front-to-back compositing of one candidate (Sec. 4.1, eq. our_alpha_blend):
   stops (returns 1, not blended) when T (1 - alpha) < T_min. */
static int composite(const cand_rec *c, const view_state *vs, const orc_settings *st, double *T,
                     double C[3], double *ampT2, double *mT, int64_t *last, int32_t *cnt,
                     blend_list *bl)
{
    const double Tn = *T * (1.0 - c->alpha);
    if (st->T_min > 0) {
        const double m = dec_margin(Tn, st->T_min,
                                    1.0 + sqrt(*ampT2 + (c->amp_om + 1.0) * (c->amp_om + 1.0)));
        if (m < *mT) *mT = m;
    }
    if (Tn < st->T_min) return 1;                      /* stop before blending */
    for (int ch = 0; ch < 3; ++ch) C[ch] += vs->rgb[3 * c->idx + ch] * c->alpha * *T;
    if (bl) {
        blend_rec br = { c->idx, c->x, c->alpha, *T, c->clamped };
        list_push(bl, br);
    }
    *T = Tn;
    *ampT2 += (c->amp_om + 1.0) * (c->amp_om + 1.0);
    *last = c->idx;
    ++*cnt;
    return 0;
}

/* Composite one pixel; fills out[3] (colour) or out[0] (X-ray).  margin_out
   (if given) receives the decision margins (see dec_margin): [0] the smallest
   over the tests on x or alpha (skip, clamp, X-ray cut), [1] the smallest over
   the termination tests T (1 - alpha) < T_min, [2] with the per-pixel window
   the smallest relative gap, over the window's pops, between the key of the
   entry taken and the next smallest key in the window (else inf). */
static void shade_pixel(const view_state *vs, const float *means, const orc_settings *st,
                        const double d[3], const double pc[2], double *out,
                        double *T_out, int64_t *last_out, int32_t *nblend_out,
                        double *margin_out, double *untrunc_out, blend_list *bl)
{
    double mx = INFINITY, mT = INFINITY;
    const double tn = st->near_segment ? near_t(vs->zrow, vs->znear, d) : 0.0;
    if (st->mode == 1) {
        /* X-ray: sum of line integrals, every visible Gaussian, any order */
        double I = 0, full = 0;
        int32_t cnt = 0;
        for (int64_t r = 0; r < vs->nvis; ++r) {
            int64_t i = vs->order[r];
            double mu[3] = { means[3 * i], means[3 * i + 1], means[3 * i + 2] };
            ray_terms rt;
            ray_integral(mu, vs->P + 9 * i, vs->kappa[i], vs->o, d, &rt, st->kernel);
            const double eta = (rt.gamma - tn) / rt.beta;
            if (st->near_segment) rt.x *= norm_cdf(eta);
            full += rt.x;
            double m = dec_margin(rt.x, st->x_min_xray,
                                  x_amp(&rt, st->kernel, vs->aniso[i], st->near_segment, eta, tn));
            if (m < mx) mx = m;
            if (rt.x >= st->x_min_xray) {
                I += rt.x;
                ++cnt;
                if (bl) {
                    blend_rec br = { i, rt.x, 0, 0, 0 };
                    list_push(bl, br);
                }
            }
        }
        out[0] = I;
        if (T_out) *T_out = exp(-I);
        if (last_out) *last_out = -1;
        if (nblend_out) *nblend_out = cnt;
        if (margin_out) { margin_out[0] = mx; margin_out[1] = mT; margin_out[2] = INFINITY; }
        if (untrunc_out) *untrunc_out = full;
        return;
    }
    double tau = -log1p(-st->alpha_min);
    double xmax = -log1p(-st->alpha_max);
    double T = 1.0, C[3] = { 0, 0, 0 };
    double ampT2 = 0.0;  /* sum of squared amplifications of T's factors so far */
    int64_t last = -1;
    int32_t cnt = 0;
    /* Per-pixel re-sorting (pixel_window = W > 0): the Gaussians that reach
       alpha_min at this pixel, taken in the list order, pass through a window
       of W entries ordered by gamma on this pixel's own ray (ties by list
       position); when the window is full its smallest entry is composited,
       and at the end of the list the rest in order.  W = 1 is the list order;
       a W of at least the number of such Gaussians is the exact per-pixel
       order by gamma. */
    const int W = st->pixel_window;
    cand_rec win[ORC_MAX_WINDOW];
    int nw = 0, stopped = 0;
    /* smallest relative gap between the entry each pop takes and the next
       smallest one in the window: the only comparison that decides the pop */
    double pgap = INFINITY;
    for (int64_t r = 0; r < vs->nvis && !stopped; ++r) {
        int64_t i = vs->order[r];
        double alpha, m, amp_om;
        ray_terms rt;
        if (vs->splat) {
            /* alpha = o exp(-1/2 dp^T C dp), dp = pixel centre - mu' */
            const double *sp = vs->splat + 6 * i;
            const double dx = pc[0] - sp[0], dy = pc[1] - sp[1];
            const double q = sp[2] * dx * dx + 2.0 * sp[3] * dx * dy + sp[4] * dy * dy;
            alpha = sp[5] * exp(-0.5 * q);
            rt.x = -log1p(-alpha);
            rt.gamma = 0.0;
            /* condition number of the 2x2 conic */
            const double tr = 0.5 * (sp[2] + sp[4]);
            const double dd = sqrt(0.25 * (sp[2] - sp[4]) * (sp[2] - sp[4]) + sp[3] * sp[3]);
            const double cond = (tr + dd) / fmax(tr - dd, 1e-300 * (tr + dd));
            const double amp = 1.0 + 0.5 * q * cond;
            m = dec_margin(alpha, st->alpha_min, amp);
            if (m < mx) mx = m;
            if (alpha < st->alpha_min) continue;
            m = dec_margin(alpha, st->alpha_max, amp);
            if (m < mx) mx = m;
            amp_om = alpha < st->alpha_max ? alpha / (1.0 - alpha) * amp : 0.0;
        } else {
            double mu[3] = { means[3 * i], means[3 * i + 1], means[3 * i + 2] };
            ray_integral(mu, vs->P + 9 * i, vs->kappa[i], vs->o, d, &rt, st->kernel);
            const double eta = (rt.gamma - tn) / rt.beta;
            if (st->near_segment) rt.x *= norm_cdf(eta);
            const double amp = x_amp(&rt, st->kernel, vs->aniso[i], st->near_segment, eta, tn);
            m = dec_margin(rt.x, tau, amp);
            if (m < mx) mx = m;
            if (rt.x < tau) continue;                  /* alpha < alpha_min */
            alpha = -expm1(-rt.x);
            m = dec_margin(rt.x, xmax, amp);
            if (m < mx) mx = m;
            amp_om = rt.x < xmax ? rt.x * amp : 0.0;
        }
        int clamped = 0;
        if (alpha > st->alpha_max) { alpha = st->alpha_max; clamped = 1; }
        const cand_rec cr = { i, r, rt.x, alpha, amp_om, rt.gamma, clamped };
        if (W <= 0) {
            stopped = composite(&cr, vs, st, &T, C, &ampT2, &mT, &last, &cnt, bl);
            continue;
        }
        /* insert into the window, ordered by (gamma, list position) */
        int k = nw++;
        while (k > 0 && win[k - 1].gamma > cr.gamma) { win[k] = win[k - 1]; --k; }
        win[k] = cr;
        if (nw == W) {
            if (nw > 1) {
                const double g = fabs(win[1].gamma - win[0].gamma) / fmax(fabs(win[1].gamma), 1e-300);
                if (g < pgap) pgap = g;
            }
            const cand_rec first = win[0];
            for (int j = 1; j < nw; ++j) win[j - 1] = win[j];
            --nw;
            stopped = composite(&first, vs, st, &T, C, &ampT2, &mT, &last, &cnt, bl);
        }
    }
    for (int j = 0; j < nw && !stopped; ++j) {
        if (j + 1 < nw) {
            const double g = fabs(win[j + 1].gamma - win[j].gamma) / fmax(fabs(win[j + 1].gamma), 1e-300);
            if (g < pgap) pgap = g;
        }
        stopped = composite(&win[j], vs, st, &T, C, &ampT2, &mT, &last, &cnt, bl);
    }
    for (int ch = 0; ch < 3; ++ch) out[ch] = C[ch] + T * st->bg[ch];
    if (T_out) *T_out = T;
    if (last_out) *last_out = last;
    if (nblend_out) *nblend_out = cnt;
    if (margin_out) { margin_out[0] = mx; margin_out[1] = mT; margin_out[2] = pgap; }
    if (untrunc_out) *untrunc_out = 0;
}

int orc_render(int64_t n, const float *means, const float *quats, const float *scales,
               const float *dens, const float *sh, const orc_camera *cam,
               const orc_settings *st, int64_t npix, const int32_t *pix, double *out,
               double *T_out, int64_t *last_out, int32_t *nblend_out, double *margin_out,
               double *untrunc_out)
{
    if (n < 0 || npix < 0 || !cam || !st) return -1;
    if (st->mode == 0 && n > 0 && !sh) return -1;
    if (st->alpha_model != 0 && (st->mode != 0 || st->density != 0 || st->near_segment)) return -1;
    if (st->tile_resort && (st->mode != 0 || st->alpha_model != 0 || st->tile_w < 1 || st->tile_h < 1))
        return -1;
    if (st->kernel != 0 && (st->kernel != 1 || st->alpha_model != 0 || st->near_segment)) return -1;
    if (st->pixel_window < 0 || st->pixel_window > ORC_MAX_WINDOW ||
        (st->pixel_window > 0 && !st->tile_resort))
        return -1;
    view_state vs;
    int rc = view_setup(&vs, n, means, quats, scales, dens, sh, cam, st);
    if (rc) { view_free(&vs); return rc; }
    int C = st->mode == 1 ? 1 : 3;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < npix; ++p) {
        double d[3];
        const double pc[2] = { pix[2 * p] + 0.5, pix[2 * p + 1] + 0.5 };
        pixel_ray(cam, pix[2 * p], pix[2 * p + 1], d);
        view_state vp = vs;
        double ogap = INFINITY;
        if (st->tile_resort) {
            vp.order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(vs.nvis > 0 ? vs.nvis : 1));
            ogap = resort_order(&vs, means, cam, st, pix[2 * p], pix[2 * p + 1], d,
                                -log1p(-st->alpha_min), vp.order);
        }
        shade_pixel(&vp, means, st, d, pc, out + C * p, T_out ? T_out + p : NULL,
                    last_out ? last_out + p : NULL, nblend_out ? nblend_out + p : NULL,
                    margin_out ? margin_out + 3 * p : NULL,
                    untrunc_out ? untrunc_out + p : NULL, NULL);
        if (margin_out && ogap < margin_out[3 * p + 2]) margin_out[3 * p + 2] = ogap;
        if (st->tile_resort) free(vp.order);
    }
    view_free(&vs);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Backward.                                                                 */

/* dR/dq for R(q) with q = (w, x, y, z) unit; J[c][9] */
static void rot_jacobian(const double q[4], double J[4][9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double Jw[9] = { 0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0 };
    double Jx[9] = { 0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x };
    double Jy[9] = { -4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y };
    double Jz[9] = { -4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0 };
    memcpy(J[0], Jw, sizeof Jw);
    memcpy(J[1], Jx, sizeof Jx);
    memcpy(J[2], Jy, sizeof Jy);
    memcpy(J[3], Jz, sizeof Jz);
}

static void atomic_add(double *dst, double v)
{
    #pragma omp atomic
    *dst += v;
}

/* g_*: gradients; a_*: sums of |per-pixel contribution|; e_*: FP32 error
   scales, sums of w |contribution| where the contribution is formed from an
   upstream factor without cancellation and w counts how strongly a relative
   rounding error in its inputs is amplified (see orc_render_backward). */
typedef struct {
    double *g_means, *g_quats, *g_scales, *g_dens, *g_sh;
    double *a_means, *a_quats, *a_scales, *a_dens, *a_sh;
    double *e_means, *e_quats, *e_scales, *e_dens, *e_sh;
} grad_out;

/* unit: the contribution per unit upstream factor; g: the upstream factor;
   ge: its cancellation-free magnitude times the amplification weight. */
static void add3(double *g, double *a, double *e, int64_t off, double unit, double gx, double ge)
{
    atomic_add(g + off, gx * unit);
    if (a) atomic_add(a + off, fabs(gx * unit));
    if (e) atomic_add(e + off, fabs(ge * unit));
}

/* Chain dL/dx = gx (line integral of Gaussian i on ray (o, d)) to mu, q, s
   and the density input (kappa, or theta with its path into s).  For the error scale (see grad_out), gabs is |gx| formed without
   cancellation and the weight is 1 + D^2/2 + w_extra: a relative error e in
   D^2 becomes D^2 e / 2 in x = ... exp(-D^2/2). */
static void chain_integral(int64_t i, double gx, double gabs, double w_extra, const float *means,
                           const float *quats, const float *scales, const float *dens,
                           const orc_settings *st, const view_state *vs, const double d[3],
                           grad_out *go)
{
    const double *o = vs->o;
    double R[9], qn[4], qlen, P[9];
    quat_rotation(quats + 4 * i, R, qn, &qlen);
    precision_matrix(R, scales + 3 * i, P);
    double mu[3] = { means[3 * i], means[3 * i + 1], means[3 * i + 2] };
    double kappa = kappa_of(st, dens[i], scales + 3 * i);
    ray_terms rt;
    ray_integral(mu, P, kappa, o, d, &rt, st->kernel);
    /* x = kappa sqrt(2pi) a^-1/2 exp(-D^2/2),  D^2 = v^T P v, v = mu - o - gamma d
       dx/dkappa = sqrt(2pi) beta Gmax
       dx/dP     = x (-1/2 d d^T / a - 1/2 v v^T)
       dx/dmu    = -x P v
       With the finite segment, x_seg = x Phi(e), e = (gamma - t_n)/beta
       = (mu-o)^T P d a^-1/2 - t_n a^1/2:  dx_seg = Phi dx + x phi(e) de, with
       de/dmu = P d a^-1/2 and de/dP = ((mu-o) d^T + d (mu-o)^T) a^-1/2 / 2
       - ((mu-o)^T P d) a^-3/2 d d^T / 2 - t_n a^-1/2 d d^T / 2.            */
    double x = rt.x;
    double Phi = 1.0, xphi = 0.0, tn = 0.0;
    if (st->near_segment) {
        tn = near_t(vs->zrow, vs->znear, d);
        const double e = (rt.gamma - tn) / rt.beta;
        Phi = norm_cdf(e);
        xphi = x * norm_pdf(e);
    }
    double Pv[3], D2 = 0;
    for (int r = 0; r < 3; ++r) {
        Pv[r] = P[r * 3] * rt.v[0] + P[r * 3 + 1] * rt.v[1] + P[r * 3 + 2] * rt.v[2];
        D2 += rt.v[r] * Pv[r];
    }
    /* c = d ln x / d D^2 (-1/2 for the Gaussian): dx/dP gets c x v v^T and
       dx/dmu = 2 c x P v (envelope: gamma is the minimiser, D^2 = v^T P v) */
    const double cD = dlnx_dD2(st->kernel, D2);
    const double ge = gabs * (1.0 + fabs(cD) * D2 * vs->aniso[i] + w_extra);
    const double dx_dk = (st->kernel == 1 ? (4.0 / 3.0) * rt.beta * pow(1.0 - D2, 1.5)
                                          : sqrt(2 * ORC_PI) * rt.beta * rt.Gmax) * Phi;
    double dk_din, dk_ds[3];
    kappa_grad(st, dens[i], scales + 3 * i, &dk_din, dk_ds);
    add3(go->g_dens, go->a_dens, go->e_dens, i, dx_dk * dk_din, gx, ge);
    if (st->density != 0)
        for (int k = 0; k < 3; ++k)
            add3(go->g_scales, go->a_scales, go->e_scales, 3 * i + k, dx_dk * dk_ds[k], gx, ge);
    double G[9];   /* dx/dP per unit gx */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            G[r * 3 + c] = Phi * x * (-0.5 * d[r] * d[c] / rt.a + cD * rt.v[r] * rt.v[c]);
    double Pd[3] = { 0, 0, 0 };
    if (st->near_segment) {
        const double dm[3] = { mu[0] - o[0], mu[1] - o[1], mu[2] - o[2] };
        double b = 0;
        for (int r = 0; r < 3; ++r) {
            Pd[r] = P[r * 3] * d[0] + P[r * 3 + 1] * d[1] + P[r * 3 + 2] * d[2];
            b += dm[r] * Pd[r];
        }
        const double ra = 1.0 / sqrt(rt.a);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                G[r * 3 + c] += xphi * (0.5 * (dm[r] * d[c] + d[r] * dm[c]) * ra -
                                        0.5 * b * ra * ra * ra * d[r] * d[c] -
                                        0.5 * tn * ra * d[r] * d[c]);
        for (int r = 0; r < 3; ++r) Pd[r] *= ra;
    }
    for (int r = 0; r < 3; ++r)
        add3(go->g_means, go->a_means, go->e_means, 3 * i + r,
             2.0 * cD * Phi * x * Pv[r] + xphi * Pd[r], gx, ge);
    /* P = sum_k s_k^-2 r_k r_k^T, r_k = column k of R */
    double dR[9];
    for (int k = 0; k < 3; ++k) {
        double s = scales[3 * i + k];
        double rk[3] = { R[k], R[3 + k], R[6 + k] };
        double Gr[3];
        for (int r = 0; r < 3; ++r) Gr[r] = G[r * 3] * rk[0] + G[r * 3 + 1] * rk[1] + G[r * 3 + 2] * rk[2];
        double rGr = rk[0] * Gr[0] + rk[1] * Gr[1] + rk[2] * Gr[2];
        add3(go->g_scales, go->a_scales, go->e_scales, 3 * i + k, -2.0 * rGr / (s * s * s), gx, ge);
        for (int r = 0; r < 3; ++r) dR[r * 3 + k] = 2.0 * Gr[r] / (s * s);
    }
    double J[4][9], dqn[4];
    rot_jacobian(qn, J);
    for (int c = 0; c < 4; ++c) {
        double acc = 0;
        for (int e = 0; e < 9; ++e) acc += dR[e] * J[c][e];
        dqn[c] = acc;
    }
    double dot = qn[0] * dqn[0] + qn[1] * dqn[1] + qn[2] * dqn[2] + qn[3] * dqn[3];
    for (int c = 0; c < 4; ++c)
        add3(go->g_quats, go->a_quats, go->e_quats, 4 * i + c, (dqn[c] - qn[c] * dot) / qlen, gx, ge);
}

/* Chain dL/d(colour after activation) to the SH coefficients and mu. */
static void chain_colour(int64_t i, const double gc[3], double w, const view_state *vs,
                         const float *means, const float *sh, const orc_settings *st,
                         grad_out *go)
{
    int nb = (st->sh_degree + 1) * (st->sh_degree + 1);
    double v[3], len = 0;
    for (int k = 0; k < 3; ++k) { v[k] = means[3 * i + k] - vs->o[k]; len += v[k] * v[k]; }
    len = sqrt(len);
    for (int k = 0; k < 3; ++k) v[k] /= len;
    double Y[(ORC_MAX_DEG + 1) * (ORC_MAX_DEG + 1)], dY[3 * (ORC_MAX_DEG + 1) * (ORC_MAX_DEG + 1)];
    orc_sh_basis(st->sh_degree, v, Y, dY);
    double gv[3] = { 0, 0, 0 }, gva[3] = { 0, 0, 0 };
    for (int ch = 0; ch < 3; ++ch) {
        double graw = gc[ch] * act_grad(st->act, vs->raw[3 * i + ch]);
        for (int k = 0; k < nb; ++k) {
            size_t e = ((size_t)i * nb + k) * 3 + ch;
            /* FP32 evaluation of Y_k at a direction known to a few units of
               roundoff errs by about u (|Y_k| + |grad Y_k|), not u |Y_k|: near
               a nodal line of Y_k its relative error is unbounded */
            const double yk_mag = fabs(Y[k]) + sqrt(dY[3 * k] * dY[3 * k] + dY[3 * k + 1] * dY[3 * k + 1] +
                                                    dY[3 * k + 2] * dY[3 * k + 2]);
            atomic_add(go->g_sh + e, graw * Y[k]);
            if (go->a_sh) atomic_add(go->a_sh + e, fabs(graw * Y[k]));
            if (go->e_sh) atomic_add(go->e_sh + e, fabs(w * graw) * yk_mag);
            for (int j = 0; j < 3; ++j) {
                gv[j] += graw * sh[e] * dY[3 * k + j];
                gva[j] += fabs(graw * sh[e] * dY[3 * k + j]);
            }
        }
    }
    double vg = v[0] * gv[0] + v[1] * gv[1] + v[2] * gv[2];
    double vga = fabs(v[0]) * gva[0] + fabs(v[1]) * gva[1] + fabs(v[2]) * gva[2];
    for (int j = 0; j < 3; ++j) {
        double c = (gv[j] - v[j] * vg) / len;
        double ca = (gva[j] + fabs(v[j]) * vga) / len;
        add3(go->g_means, go->a_means, NULL, 3 * i + j, c, 1.0, 0.0);
        if (go->e_means) atomic_add(go->e_means + 3 * i + j, w * ca);
    }
}

/* Chain dL/dalpha = ga (the splatting alpha of Gaussian i at the pixel centre
   pc, unclamped) to mu, q, s and the opacity input.  With d = pc - mu',
   alpha = o exp(-1/2 d^T C d), C = Sigma'^-1, Sigma' = J V J^T, V = W R D R^T W^T,
   D = diag(s^2):
     dalpha/do = G,  dalpha/dC = -1/2 alpha d d^T,  dalpha/dmu' = alpha C d,
     dL/dSigma' = -C (dL/dC) C,  dL/dV = J^T (dL/dSigma') J,
     dL/dJ = 2 (dL/dSigma') J V,  dL/dR = 2 W^T (dL/dV) W R D,
     dL/ds_k = 2 s_k (R^T W^T (dL/dV) W R)_kk,
   and J, mu' depend on the view-space mean m = W mu + t.  The error-scale
   weight is 1 + q/2 + w_extra, q = d^T C d (a relative error e in q becomes
   q e / 2 in alpha).  Returns q. */
static double chain_splat(int64_t i, double ga, double gabs, double w_extra, const float *means,
                          const float *quats, const float *scales, const float *dens,
                          const orc_camera *cam, const double pc[2], grad_out *go)
{
    double R[9], qn[4], qlen;
    quat_rotation(quats + 4 * i, R, qn, &qlen);
    const float *s = scales + 3 * i;
    const float *Wf = cam->R;
    double W[9], m[3], WR[9], V[9];
    for (int k = 0; k < 9; ++k) W[k] = Wf[k];
    for (int a = 0; a < 3; ++a)
        m[a] = W[3 * a] * means[3 * i] + W[3 * a + 1] * means[3 * i + 1] +
               W[3 * a + 2] * means[3 * i + 2] + (double)cam->t[a];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += W[a * 3 + k] * R[k * 3 + b];
            WR[a * 3 + b] = acc;
        }
    double D[3];
    for (int k = 0; k < 3; ++k) D[k] = (double)s[k] * (double)s[k];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += WR[a * 3 + k] * D[k] * WR[b * 3 + k];
            V[a * 3 + b] = acc;
        }
    const double fx = cam->fx, fy = cam->fy, x = m[0], y = m[1], z = m[2];
    double J[6] = { fx / z, 0.0, -fx * x / (z * z), 0.0, fy / z, -fy * y / (z * z) };
    double Sp[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += J[a * 3 + k] * V[k * 3 + l] * J[b * 3 + l];
            Sp[a * 2 + b] = acc;
        }
    const double det = Sp[0] * Sp[3] - Sp[1] * Sp[2];
    const double Cm[4] = { Sp[3] / det, -Sp[1] / det, -Sp[2] / det, Sp[0] / det };
    const double dx = pc[0] - (fx * x / z + cam->cx), dy = pc[1] - (fy * y / z + cam->cy);
    const double Cd[2] = { Cm[0] * dx + Cm[1] * dy, Cm[2] * dx + Cm[3] * dy };
    const double q = dx * Cd[0] + dy * Cd[1];
    const double G = exp(-0.5 * q);
    const float di = dens[i];
    const double o = di < 0.0f ? 0.0 : (di > 1.0f ? 1.0 : (double)di);
    const double alpha = o * G;
    const double ge = gabs * (1.0 + 0.5 * q + w_extra);
    /* opacity (zero gradient where the input was clamped) */
    add3(go->g_dens, go->a_dens, go->e_dens, i, (di < 0.0f || di > 1.0f) ? 0.0 : G, ga, ge);
    /* per unit ga: dL/dC (full symmetric) and dL/dSigma' = -C GC C */
    const double GC[4] = { -0.5 * alpha * dx * dx, -0.5 * alpha * dx * dy,
                           -0.5 * alpha * dx * dy, -0.5 * alpha * dy * dy };
    double T1[4], GS[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            T1[a * 2 + b] = Cm[a * 2] * GC[b] + Cm[a * 2 + 1] * GC[2 + b];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            GS[a * 2 + b] = -(T1[a * 2] * Cm[b] + T1[a * 2 + 1] * Cm[2 + b]);
    /* dL/dV = J^T GS J, dL/dJ = 2 GS J V */
    double GV[9], GJ[6], JV[6];
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            double acc = 0;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) acc += J[a * 3 + k] * GS[a * 2 + b] * J[b * 3 + l];
            GV[k * 3 + l] = acc;
        }
    for (int a = 0; a < 2; ++a)
        for (int l = 0; l < 3; ++l) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += J[a * 3 + k] * V[k * 3 + l];
            JV[a * 3 + l] = acc;
        }
    for (int a = 0; a < 2; ++a)
        for (int l = 0; l < 3; ++l)
            GJ[a * 3 + l] = 2.0 * (GS[a * 2] * JV[l] + GS[a * 2 + 1] * JV[3 + l]);
    /* view-space mean: through J and through mu' (dL/dmu' = alpha C d) */
    const double gmu_p[2] = { alpha * Cd[0], alpha * Cd[1] };
    double gm[3];
    gm[0] = GJ[2] * (-fx / (z * z)) + gmu_p[0] * fx / z;
    gm[1] = GJ[5] * (-fy / (z * z)) + gmu_p[1] * fy / z;
    gm[2] = GJ[0] * (-fx / (z * z)) + GJ[2] * (2.0 * fx * x / (z * z * z)) +
            GJ[4] * (-fy / (z * z)) + GJ[5] * (2.0 * fy * y / (z * z * z)) -
            gmu_p[0] * fx * x / (z * z) - gmu_p[1] * fy * y / (z * z);
    for (int r = 0; r < 3; ++r)
        add3(go->g_means, go->a_means, go->e_means, 3 * i + r,
             W[r] * gm[0] + W[3 + r] * gm[1] + W[6 + r] * gm[2], ga, ge);
    /* H = (W R)^T GV (W R): scales dL/ds_k = 2 s_k H_kk; rotation via
       dL/dR = 2 W^T GV W R D */
    double GVW[9], H[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += GV[a * 3 + k] * WR[k * 3 + b];
            GVW[a * 3 + b] = acc;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += WR[k * 3 + a] * GVW[k * 3 + b];
            H[a * 3 + b] = acc;
        }
    for (int k = 0; k < 3; ++k)
        add3(go->g_scales, go->a_scales, go->e_scales, 3 * i + k, 2.0 * (double)s[k] * H[k * 4],
             ga, ge);
    double dR[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += W[k * 3 + a] * GVW[k * 3 + b];
            dR[a * 3 + b] = 2.0 * acc * D[b];
        }
    double Jq[4][9], dqn[4];
    rot_jacobian(qn, Jq);
    for (int c = 0; c < 4; ++c) {
        double acc = 0;
        for (int e = 0; e < 9; ++e) acc += dR[e] * Jq[c][e];
        dqn[c] = acc;
    }
    double dot = qn[0] * dqn[0] + qn[1] * dqn[1] + qn[2] * dqn[2] + qn[3] * dqn[3];
    for (int c = 0; c < 4; ++c)
        add3(go->g_quats, go->a_quats, go->e_quats, 4 * i + c, (dqn[c] - qn[c] * dot) / qlen, ga, ge);
    return q;
}

/* q = dp^T C dp of Gaussian i's splat at the pixel centre pc. */
static double splat_q(const view_state *vs, int64_t i, const double pc[2])
{
    const double *sp = vs->splat + 6 * i;
    const double dx = pc[0] - sp[0], dy = pc[1] - sp[1];
    return sp[2] * dx * dx + 2.0 * sp[3] * dx * dy + sp[4] * dy * dy;
}

/* Squared Mahalanobis distance of Gaussian i from the ray (o, d). */
static double pair_D2(int64_t i, const float *means, const float *quats, const float *scales,
                      const double o[3], const double d[3])
{
    double R[9], qn[4], qlen, P[9];
    quat_rotation(quats + 4 * i, R, qn, &qlen);
    precision_matrix(R, scales + 3 * i, P);
    double mu[3] = { means[3 * i], means[3 * i + 1], means[3 * i + 2] };
    ray_terms rt;
    ray_integral(mu, P, 1.0, o, d, &rt, 0);   /* D^2 does not depend on kappa */
    double D2 = 0;
    for (int r = 0; r < 3; ++r)
        D2 += rt.v[r] * (P[r * 3] * rt.v[0] + P[r * 3 + 1] * rt.v[1] + P[r * 3 + 2] * rt.v[2]);
    return D2;
}

/* Error scales (e_*): the contribution of each blended pair is weighted by
   1 + (D^2/2) s_max/s_min (the exponential's amplification of a relative
   error in D^2, which a rounded rotation makes up to s_max/s_min times the
   rotation's error; see dec_margin) plus,
   in colour mode, the number of compositing steps between the pair and the end
   of the pixel's list (a reverse replay of T and the colour behind carries one
   rounding per step); the upstream factor dL/dalpha is taken as
   sum |dL/dC| T (|c| + |S|), without the cancellation of c - S. */
int orc_render_backward(int64_t n, const float *means, const float *quats, const float *scales,
                        const float *dens, const float *sh, const orc_camera *cam,
                        const orc_settings *st, int64_t npix, const int32_t *pix,
                        const double *dL, double *g_means, double *g_quats, double *g_scales,
                        double *g_dens, double *g_sh, double *a_means, double *a_quats,
                        double *a_scales, double *a_dens, double *a_sh, double *e_means,
                        double *e_quats, double *e_scales, double *e_dens, double *e_sh)
{
    if (n < 0 || npix < 0 || !cam || !st) return -1;
    if (st->mode == 0 && n > 0 && !sh) return -1;
    if (st->alpha_model != 0 && (st->mode != 0 || st->density != 0 || st->near_segment)) return -1;
    if (st->tile_resort && (st->mode != 0 || st->alpha_model != 0 || st->tile_w < 1 || st->tile_h < 1))
        return -1;
    if (st->near_threshold > 0 && st->mode != 1) return -1;
    if (st->kernel != 0 && (st->kernel != 1 || st->alpha_model != 0 || st->near_segment)) return -1;
    if (st->pixel_window < 0 || st->pixel_window > ORC_MAX_WINDOW ||
        (st->pixel_window > 0 && !st->tile_resort))
        return -1;
    view_state vs;
    int rc = view_setup(&vs, n, means, quats, scales, dens, sh, cam, st);
    if (rc) { view_free(&vs); return rc; }
    grad_out go = { g_means, g_quats, g_scales, g_dens, g_sh,
                    a_means, a_quats, a_scales, a_dens, a_sh,
                    e_means, e_quats, e_scales, e_dens, e_sh };
    int C = st->mode == 1 ? 1 : 3;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < npix; ++p) {
        const double *g = dL + C * p;
        if (C == 1 ? g[0] == 0 : (g[0] == 0 && g[1] == 0 && g[2] == 0)) continue;
        double d[3], out[3];
        pixel_ray(cam, pix[2 * p], pix[2 * p + 1], d);
        blend_list bl = { NULL, 0, 0 };
        const double pc[2] = { pix[2 * p] + 0.5, pix[2 * p + 1] + 0.5 };
        view_state vp = vs;
        if (st->tile_resort) {
            vp.order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(vs.nvis > 0 ? vs.nvis : 1));
            resort_order(&vs, means, cam, st, pix[2 * p], pix[2 * p + 1], d,
                         -log1p(-st->alpha_min), vp.order);
        }
        if (st->mode == 1 && st->near_threshold > 0) {
            /* only the pairs whose X-ray cut decision lies within the given
               margin, on either side of the cut: their summed |contributions|
               (the abs_* output) bound what flipping those decisions can
               change in each gradient element */
            const double tn = st->near_segment ? near_t(vs.zrow, vs.znear, d) : 0.0;
            for (int64_t r = 0; r < vs.nvis; ++r) {
                const int64_t i = vs.order[r];
                const double mu[3] = { means[3 * i], means[3 * i + 1], means[3 * i + 2] };
                ray_terms rt;
                ray_integral(mu, vs.P + 9 * i, vs.kappa[i], vs.o, d, &rt, st->kernel);
                const double eta = (rt.gamma - tn) / rt.beta;
                if (st->near_segment) rt.x *= norm_cdf(eta);
                const double m = dec_margin(rt.x, st->x_min_xray,
                                            x_amp(&rt, st->kernel, vs.aniso[i], st->near_segment, eta, tn));
                if (m < st->near_threshold)
                    chain_integral(i, g[0], fabs(g[0]), 0.0, means, quats, scales, dens, st, &vs,
                                   d, &go);
            }
            if (st->tile_resort) free(vp.order);
            continue;
        }
        shade_pixel(&vp, means, st, d, pc, out, NULL, NULL, NULL, NULL, NULL, &bl);
        if (st->mode == 1) {
            for (int64_t r = 0; r < bl.cnt; ++r)
                chain_integral(bl.rec[r].idx, g[0], fabs(g[0]), 0.0, means, quats, scales, dens,
                               st, &vs, d, &go);
        } else {
            /* S: colour composited behind the current Gaussian, ending in bg */
            double S[3] = { st->bg[0], st->bg[1], st->bg[2] };
            for (int64_t r = bl.cnt - 1; r >= 0; --r) {
                const blend_rec *br = &bl.rec[r];
                int64_t i = br->idx;
                double galpha = 0, gabs = 0, gc[3];
                for (int ch = 0; ch < 3; ++ch) {
                    double c = vs.rgb[3 * i + ch];
                    galpha += g[ch] * br->T * (c - S[ch]);
                    gabs += fabs(g[ch]) * br->T * (fabs(c) + fabs(S[ch]));
                    gc[ch] = g[ch] * br->alpha * br->T;
                }
                const double steps = (double)(bl.cnt - 1 - r);
                double w = 1.0 + steps;
                if (vs.splat) {
                    /* splatting model: the chain starts at dL/dalpha; the
                       colour's error weight uses q = d^T C d in place of D^2 */
                    const double q = br->clamped ? splat_q(&vs, i, pc)
                                                 : chain_splat(i, galpha, gabs, steps, means,
                                                               quats, scales, dens, cam, pc, &go);
                    w += 0.5 * q;
                } else {
                    const double ex = exp(-br->x);
                    if (!br->clamped)
                        chain_integral(i, galpha * ex, gabs * ex, steps, means, quats, scales,
                                       dens, st, &vs, d, &go);
                    if (go.e_means || go.e_sh) {
                        const double D2 = pair_D2(i, means, quats, scales, vs.o, d);
                        w += fabs(dlnx_dD2(st->kernel, D2)) * D2 * vs.aniso[i];
                    }
                }
                chain_colour(i, gc, w, &vs, means, sh, st, &go);
                for (int ch = 0; ch < 3; ++ch)
                    S[ch] = vs.rgb[3 * i + ch] * br->alpha + (1.0 - br->alpha) * S[ch];
            }
        }
        free(bl.rec);
        if (st->tile_resort) free(vp.order);
    }
    view_free(&vs);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
