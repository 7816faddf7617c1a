/*
 * kde_oracle.c -- plain, slow, FP64 CPU reference for the KDE heat map of
 * Huang, Li, Zhang and Liu, "GPU-Accelerated Compression and Visualization of
 * Large-Scale Vessel Trajectories in Maritime IoT Industries" (arXiv 2004.13653).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only tests/, the smoke check and the CPU-baseline leg of the bench
 * do.  It shares no code, header, table or constant with the HIP library.
 *
 * What it computes (Sec. III-C, Eq. (7)-(8), Table I), in the reading that the
 * kernel argument is s = (grid node - point) / h with support |s| <= 1:
 *
 *   S[j][i] = sum_p k((gx_i - x_p)/hx) * k((gy_j - y_p)/hy)      (Table I: every
 *             kernel is a product f(s,t) = k(s) k(t))
 *   f[j][i] = S[j][i] / (n * hx * hy)                             (density)
 *
 * Grid nodes: gx_i = xmin + i*dx, dx = (xmax - xmin)/(nx - 1), i = 0..nx-1, the
 * node spacing of Eq. (5)-(6) with both box edges on nodes.  Output is row-major
 * out[j*nx + i], x fastest, the index order of Algorithm 3's density matrix.
 *
 * Every per-output sum runs over points (or pairs) in index order, one term at a
 * time, in double precision; threads split outputs, never a sum, so the result
 * does not depend on the thread count.
 *
 * "Grid-unit" entry points take the FP32 pixel coordinates X_p = fl32((x_p -
 * xmin)/dx) and FP32 bandwidths Hx = fl32(hx/dx) that a GPU is fed, and evaluate
 * everything else in FP64 with node i at X = i: this is the parity mode.  The
 * support test there is |i - X_p| <= Hx on the exact difference.
 *
 * Differentiation (not in the paper): the vector-Jacobian product of the map and
 * the least-squares cross-validation (LSCV) bandwidth objective of Rudemo (1982)
 * and Bowman (1984), both written from their definitions below.
 *
 * The trajectory side (Sec. III-B, V-B): the binned count matrix, recursive
 * Douglas-Peucker, and the compression-quality measures (track lengths for the
 * rate of length loss, squared-Euclidean DTW), each a plain loop over its
 * definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KO_UNIFORM 0
#define KO_TRIANGULAR 1
#define KO_EPANECHNIKOV 2
#define KO_QUARTIC 3
#define KO_TRIWEIGHT 4
#define KO_TRICUBE 5
#define KO_GAUSSIAN 6
#define KO_COSINE 7
/* Not in Table I: the Gaussian truncated at |u| <= KO_TRUNC_SIGMAS (inclusive),
 * same constant 1/sqrt(2 pi); every pair it drops is below e^-32 of the peak
 * pair value. */
#define KO_GAUSS_TRUNC 8
#define KO_TRUNC_SIGMAS 8.0

static const double PI = 3.14159265358979323846;

/* Number of threads the parallel loops below use. */
int ko_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of threads of the parallel loops (n >= 1); the per-output
 * sums do not depend on it. */
void ko_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* One-dimensional factor k(u) of the Table I product kernels, in Table I order.
 * The indicator I(u) is 1 for |u| <= 1 (inclusive) and the Gaussian has none. */
double ko_k(int kernel, double u)
{
    double a = fabs(u);
    if (kernel == KO_GAUSSIAN) return exp(-0.5 * u * u) / sqrt(2.0 * PI);
    if (kernel == KO_GAUSS_TRUNC) return a <= KO_TRUNC_SIGMAS ? exp(-0.5 * u * u) / sqrt(2.0 * PI) : 0.0;
    if (a > 1.0) return 0.0;
    switch (kernel) {
    case KO_UNIFORM: return 0.5;
    case KO_TRIANGULAR: return 1.0 - a;
    case KO_EPANECHNIKOV: return 0.75 * (1.0 - u * u);
    case KO_QUARTIC: { double w = 1.0 - u * u; return (15.0 / 16.0) * w * w; }
    case KO_TRIWEIGHT: { double w = 1.0 - u * u; return (35.0 / 32.0) * w * w * w; }
    case KO_TRICUBE: { double w = 1.0 - a * a * a; return (70.0 / 81.0) * w * w * w; }
    case KO_COSINE: return (PI / 4.0) * cos(0.5 * PI * u);
    default: return NAN;
    }
}

/* dk/du, taken from the formula inside the support (|u| <= 1), 0 outside; at the
 * kink u = 0 of the triangular kernel the two one-sided slopes average to 0. */
double ko_dk(int kernel, double u)
{
    double a = fabs(u);
    if (kernel == KO_GAUSSIAN) return -u * exp(-0.5 * u * u) / sqrt(2.0 * PI);
    if (a > 1.0) return 0.0;
    switch (kernel) {
    case KO_UNIFORM: return 0.0;
    case KO_TRIANGULAR: return u > 0.0 ? -1.0 : (u < 0.0 ? 1.0 : 0.0);
    case KO_EPANECHNIKOV: return -1.5 * u;
    case KO_QUARTIC: return (15.0 / 16.0) * 2.0 * (1.0 - u * u) * (-2.0 * u);
    case KO_TRIWEIGHT: { double w = 1.0 - u * u; return (35.0 / 32.0) * 3.0 * w * w * (-2.0 * u); }
    case KO_TRICUBE: { double w = 1.0 - a * a * a; return (70.0 / 81.0) * 3.0 * w * w * (-3.0 * u * a); }
    case KO_COSINE: return -(PI / 4.0) * (0.5 * PI) * sin(0.5 * PI * u);
    default: return NAN;
    }
}

/* 16-point Gauss-Legendre rule on [-1, 1], computed once at load time by Newton
 * iteration on the Legendre polynomial P_16 (three-term recurrence).  It
 * integrates polynomials up to degree 31 exactly. */
#define KO_GL 16
static double gl_x[KO_GL], gl_w[KO_GL];

__attribute__((constructor)) static void gl_init(void)
{
    for (int i = 0; i < KO_GL; ++i) {
        double x = cos(PI * (i + 0.75) / (KO_GL + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= KO_GL; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = KO_GL * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        gl_x[i] = x;
        gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

/* Integral over u in [lo, hi] of k(u) k(a - u) (deriv = 0) or k(u) k'(a - u). */
static double conv_piece(int kernel, double a, double lo, double hi, int deriv)
{
    double c = 0.5 * (hi + lo), h = 0.5 * (hi - lo), s = 0.0;
    for (int i = 0; i < KO_GL; ++i) {
        double u = c + h * gl_x[i];
        s += gl_w[i] * ko_k(kernel, u) * (deriv ? ko_dk(kernel, a - u) : ko_k(kernel, a - u));
    }
    return s * h;
}

/* For a compact kernel and 0 <= a < 2: the integral of k(u) k(a - u) over the
 * overlap [a - 1, 1] of the two supports, split where |u| or |a - u| has a
 * kink (u = 0, u = a), each piece by Gauss-Legendre.  The factors are
 * polynomials of degree <= 9 on every piece (cosine: smooth), so the rule is
 * exact up to rounding (cosine: to far below it). */
static double conv_compact(int kernel, double a, int deriv)
{
    if (a >= 1.0) return conv_piece(kernel, a, a - 1.0, 1.0, deriv);
    return conv_piece(kernel, a, a - 1.0, 0.0, deriv) + conv_piece(kernel, a, 0.0, a, deriv) +
           conv_piece(kernel, a, a, 1.0, deriv);
}

/* Autoconvolution kbar = k * k (the integral of k(v) k(u - v) dv) and its
 * derivative.  Gaussian: kbar is the N(0, 2) density.  Epanechnikov: its
 * piecewise polynomial on |u| <= 2.  The other Table I kernels: the defining
 * integral itself, by the quadrature above (kbar is even, zero for |u| >= 2).
 * The derivative of the integral over [u - 1, 1] is, by Leibniz's rule,
 * -k(u - 1) k(1) (the moving lower end; non-zero only for the uniform kernel,
 * whose factor jumps at the support's edge) plus the integral of k(v) k'(u - v). */
double ko_kbar(int kernel, double u)
{
    double a = fabs(u);
    if (kernel == KO_GAUSSIAN) return exp(-0.25 * u * u) / (2.0 * sqrt(PI));
    if (kernel == KO_EPANECHNIKOV) {
        if (a > 2.0) return 0.0;
        double b = 2.0 - a;
        return (3.0 / 160.0) * b * b * b * (a * a + 6.0 * a + 4.0);
    }
    if (kernel < KO_UNIFORM || kernel > KO_COSINE) return NAN;
    if (a >= 2.0) return 0.0;
    return conv_compact(kernel, a, 0);
}

double ko_dkbar(int kernel, double u)
{
    double a = fabs(u);
    if (kernel == KO_GAUSSIAN) return -0.5 * u * exp(-0.25 * u * u) / (2.0 * sqrt(PI));
    if (kernel == KO_EPANECHNIKOV) {
        if (a > 2.0) return 0.0;
        double b = 2.0 - a;
        return -(3.0 / 32.0) * u * (a + 4.0) * b * b;
    }
    if (kernel < KO_UNIFORM || kernel > KO_COSINE) return NAN;
    if (a >= 2.0) return 0.0;
    double d = -ko_k(kernel, a - 1.0) * ko_k(kernel, 1.0) + conv_compact(kernel, a, 1);
    return u < 0.0 ? -d : d;
}

void ko_k_array(int kernel, const double *u, int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) out[q] = ko_k(kernel, u[q]);
}

void ko_dk_array(int kernel, const double *u, int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) out[q] = ko_dk(kernel, u[q]);
}

void ko_kbar_array(int kernel, const double *u, int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) out[q] = ko_kbar(kernel, u[q]);
}

void ko_dkbar_array(int kernel, const double *u, int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) out[q] = ko_dkbar(kernel, u[q]);
}

/* World mode: points xy[n][2] (x, y) in world units, grid box and size as above.
 * Writes the window rows j0..j1-1, columns i0..i1-1 into out[(j-j0)*(i1-i0) +
 * (i-i0)].  raw != 0 gives S; otherwise the density S/(n hx hy). */
void ko_map_world(const double *xy, int64_t n, int kernel, double hx, double hy,
                  double xmin, double xmax, double ymin, double ymax, int nx, int ny,
                  int i0, int i1, int j0, int j1, int raw, double *out)
{
    double dx = (xmax - xmin) / (double)(nx - 1);
    double dy = (ymax - ymin) / (double)(ny - 1);
    int w = i1 - i0, h = j1 - j0;
    double scale = raw ? 1.0 : 1.0 / ((double)n * hx * hy);
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < h * w; ++r) {
        int j = j0 + r / w, i = i0 + r % w;
        double gx = xmin + i * dx, gy = ymin + j * dy;
        double s = 0.0;
        for (int64_t p = 0; p < n; ++p)
            s += ko_k(kernel, (gx - xy[2 * p]) / hx) * ko_k(kernel, (gy - xy[2 * p + 1]) / hy);
        out[r] = s * scale;
    }
}

/* One factor in grid units: node index i against FP32 coordinate X with FP32
 * bandwidth H.  For compact kernels the support test is |i - X| <= H on the
 * exact difference, then k((i - X)/H). */
static double unit_factor(int kernel, int i, float X, float H)
{
    double d = (double)i - (double)X;
    if (kernel == KO_GAUSS_TRUNC) /* support |d| <= 8 H on the exact difference */
        return fabs(d) <= KO_TRUNC_SIGMAS * (double)H ? ko_k(KO_GAUSSIAN, d / (double)H) : 0.0;
    if (kernel != KO_GAUSSIAN && fabs(d) > (double)H) return 0.0;
    return ko_k(kernel, d / (double)H); /* |d| <= H implies |d/H| <= 1 */
}

static double unit_dfactor(int kernel, int i, float X, float H)
{
    double d = (double)i - (double)X;
    if (kernel != KO_GAUSSIAN && fabs(d) > (double)H) return 0.0;
    return ko_dk(kernel, d / (double)H);
}

/* Parity mode: XY[n][2] FP32 pixel coordinates, Hx, Hy FP32 pixel bandwidths.
 * Raw sum S over the window (density scaling is a separate FP64 factor). */
void ko_map_units(const float *XY, int64_t n, int kernel, float Hx, float Hy,
                  int i0, int i1, int j0, int j1, double *out)
{
    int w = i1 - i0, h = j1 - j0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < h * w; ++r) {
        int j = j0 + r / w, i = i0 + r % w;
        double s = 0.0;
        for (int64_t p = 0; p < n; ++p)
            s += unit_factor(kernel, i, XY[2 * p], Hx) * unit_factor(kernel, j, XY[2 * p + 1], Hy);
        out[r] = s;
    }
}

/* Parity mode at a list of pixels ij[m][2] = (i, j): raw sums. */
void ko_map_units_at(const float *XY, int64_t n, int kernel, float Hx, float Hy,
                     const int32_t *ij, int64_t m, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < m; ++r) {
        int i = ij[2 * r], j = ij[2 * r + 1];
        double s = 0.0;
        for (int64_t p = 0; p < n; ++p)
            s += unit_factor(kernel, i, XY[2 * p], Hx) * unit_factor(kernel, j, XY[2 * p + 1], Hy);
        out[r] = s;
    }
}

/* Vector-Jacobian product of the raw map in grid units.  Given gbar[ny][nx]
 * (dL/dS), for each selected point p = sel[r] (r = 0..m-1):
 *   g[r][0]  = dL/dX_p = sum_{j,i} gbar[j][i] * k'((i-X_p)/Hx) * (-1/Hx) * k((j-Y_p)/Hy)
 *   g[r][1]  = dL/dY_p   (the same with the roles of x and y swapped)
 *   gh[r][0] = sum_{j,i} gbar[j][i] * k'(s) * (-s/Hx) * k(t),  s = (i-X_p)/Hx, t = (j-Y_p)/Hy
 *   gh[r][1] = sum_{j,i} gbar[j][i] * k(s) * k'(t) * (-t/Hy)
 * gh is point p's share of dL/dHx and dL/dHy; summed over all points it is the
 * bandwidth gradient.  Each sum runs over pixels j-major, i fastest. */
void ko_vjp_units(const float *XY, int64_t n, int kernel, float Hx, float Hy,
                  int nx, int ny, const double *gbar, const int64_t *sel, int64_t m,
                  double *g, double *gh)
{
    (void)n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < m; ++r) {
        int64_t p = sel[r];
        double X = (double)XY[2 * p], Y = (double)XY[2 * p + 1];
        double gx = 0.0, gy = 0.0, hx = 0.0, hy = 0.0;
        for (int j = 0; j < ny; ++j) {
            double ky = unit_factor(kernel, j, XY[2 * p + 1], Hy);
            double dky = unit_dfactor(kernel, j, XY[2 * p + 1], Hy);
            double t = ((double)j - Y) / (double)Hy;
            for (int i = 0; i < nx; ++i) {
                double gb = gbar[(int64_t)j * nx + i];
                double kx = unit_factor(kernel, i, XY[2 * p], Hx);
                double dkx = unit_dfactor(kernel, i, XY[2 * p], Hx);
                double s = ((double)i - X) / (double)Hx;
                gx += gb * dkx * (-1.0 / (double)Hx) * ky;
                gy += gb * kx * dky * (-1.0 / (double)Hy);
                hx += gb * dkx * (-s / (double)Hx) * ky;
                hy += gb * kx * dky * (-t / (double)Hy);
            }
        }
        g[2 * r] = gx;
        g[2 * r + 1] = gy;
        gh[2 * r] = hx;
        gh[2 * r + 1] = hy;
    }
}

/* LSCV objective in world units for points xy[n][2] (n >= 2):
 *   LSCV(hx, hy) = A - B
 *   A = 1/(n^2 hx hy)        * sum_{p,q}     kbar(dx_pq/hx) kbar(dy_pq/hy)   (= integral of f^2)
 *   B = 2/(n (n-1) hx hy)    * sum_{p != q}  k(dx_pq/hx)    k(dy_pq/hy)      (leave-one-out term)
 * with dx_pq = x_p - x_q.  grad[2] = (dLSCV/dhx, dLSCV/dhy) uses
 *   d/dh [g(a/h)/h] = -(g(u) + u g'(u)) / h^2,  u = a/h.
 * The pair sums run q fastest inside p, p in order.  Every Table I kernel
 * (kbar as above). */
void ko_lscv_world(const double *xy, int64_t n, int kernel, double hx, double hy,
                   double *value, double *grad)
{
    double *pa = (double *)malloc(sizeof(double) * 6 * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < n; ++p) {
        double sa = 0.0, sb = 0.0, sax = 0.0, say = 0.0, sbx = 0.0, sby = 0.0;
        for (int64_t q = 0; q < n; ++q) {
            double u = (xy[2 * p] - xy[2 * q]) / hx;
            double v = (xy[2 * p + 1] - xy[2 * q + 1]) / hy;
            double ku = ko_kbar(kernel, u), kv = ko_kbar(kernel, v);
            sa += ku * kv;
            sax += (ku + u * ko_dkbar(kernel, u)) * kv;
            say += ku * (kv + v * ko_dkbar(kernel, v));
            if (q != p) {
                double lu = ko_k(kernel, u), lv = ko_k(kernel, v);
                sb += lu * lv;
                sbx += (lu + u * ko_dk(kernel, u)) * lv;
                sby += lu * (lv + v * ko_dk(kernel, v));
            }
        }
        pa[6 * p + 0] = sa;
        pa[6 * p + 1] = sb;
        pa[6 * p + 2] = sax;
        pa[6 * p + 3] = say;
        pa[6 * p + 4] = sbx;
        pa[6 * p + 5] = sby;
    }
    double SA = 0, SB = 0, SAX = 0, SAY = 0, SBX = 0, SBY = 0;
    for (int64_t p = 0; p < n; ++p) {
        SA += pa[6 * p + 0];
        SB += pa[6 * p + 1];
        SAX += pa[6 * p + 2];
        SAY += pa[6 * p + 3];
        SBX += pa[6 * p + 4];
        SBY += pa[6 * p + 5];
    }
    free(pa);
    double nn = (double)n;
    double ca = 1.0 / (nn * nn), cb = 2.0 / (nn * (nn - 1.0));
    *value = ca * SA / (hx * hy) - cb * SB / (hx * hy);
    /* A = ca * SA/(hx hy): dA/dhx = ca * sum -(kbar(u) + u kbar'(u)) kbar(v) / (hx^2 hy) */
    grad[0] = -ca * SAX / (hx * hx * hy) + cb * SBX / (hx * hx * hy);
    grad[1] = -ca * SAY / (hx * hy * hy) + cb * SBY / (hx * hy * hy);
}

/* LSCV in grid units (parity mode): FP32 pixel coordinates and bandwidths, FP64
 * arithmetic.  Same sums as ko_lscv_world with dx_pq = X_p - X_q and h = H; the
 * value and gradient are returned in grid units (multiply by 1/(dx dy) and
 * 1/(dx^2 dy), 1/(dx dy^2) for world units). */
void ko_lscv_units(const float *XY, int64_t n, int kernel, float Hx, float Hy,
                   double *value, double *grad)
{
    double *xy = (double *)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
    for (int64_t q = 0; q < 2 * n; ++q) xy[q] = (double)XY[q];
    ko_lscv_world(xy, n, kernel, (double)Hx, (double)Hy, value, grad);
    free(xy);
}

/* ---------------------------------------------------------------------------
 * The paper's own binned visualisation (Sec. III-C and IV-B): a count matrix
 * from the ceil projection of Eq. (5)-(6), gap filling between consecutive
 * points of one trajectory by the linear interpolation of Eq. (12)-(13), then
 * the convolution of Eq. (7) with a table of Table I kernel values.
 *
 * Readings (the paper leaves these open):
 *  - Grid units X = (x - xmin)/dx.  Eq. (5) with 1-based indices is
 *    ceil(X) + 1, so the 0-based cell is i = ceil(X) (likewise j = ceil(Y)).
 *    The box is given (it is not the data's extremes), so a point counts only
 *    when 0 <= i < nx and 0 <= j < ny.
 *  - Interpolation joins consecutive points p, p+1 with equal labels when both
 *    cells lie in the grid.  With di = i' - i, dj = j' - j and
 *    cmax = max(|di|, |dj|) > 1, cells c = 1 .. cmax-1 are added at the rounded
 *    positions of Eq. (12)-(13).  The rounded quantity is the positive 1-based
 *    coordinate, so rounding half away from zero is rounding half up; it is done
 *    exactly, in integers: i_c = floor((2 i cmax + 2 c di + cmax) / (2 cmax)).
 *  - Convolution taps are f(s, t) = k(s/Hx) k(t/Hy) at integer offsets
 *    |s| <= a, |t| <= b (support test |s| <= Hx on the offset for compact
 *    kernels); cells outside the grid count zero.
 * -------------------------------------------------------------------------*/

/* 0-based cell of one FP32 coordinate, or -1 when it falls outside [0, n). */
static int64_t bin_cell(float X, int n)
{
    double c = ceil((double)X);
    if (!(c >= 0.0 && c <= (double)(n - 1))) return -1; /* also rejects NaN */
    return (int64_t)c;
}

/* Count matrix counts[ny][nx] (zeroed here) of the points XY[n][2] (FP32 grid
 * units) plus, when labels is not NULL, the interpolated cells of Eq. (12)-(13)
 * between consecutive points with equal labels.  *total receives the number of
 * counted cells (points plus interpolated cells).  Sequential, point order. */
void ko_bin_counts(const float *XY, int64_t n, const int32_t *labels, int nx, int ny, uint32_t *counts,
                   int64_t *total)
{
    int64_t tot = 0;
    for (int64_t k = 0; k < (int64_t)nx * ny; ++k) counts[k] = 0;
    for (int64_t p = 0; p < n; ++p) {
        int64_t i = bin_cell(XY[2 * p], nx), j = bin_cell(XY[2 * p + 1], ny);
        if (i < 0 || j < 0) continue;
        counts[j * nx + i] += 1;
        tot += 1;
        if (labels == NULL || p + 1 >= n || labels[p] != labels[p + 1]) continue;
        int64_t i2 = bin_cell(XY[2 * p + 2], nx), j2 = bin_cell(XY[2 * p + 3], ny);
        if (i2 < 0 || j2 < 0) continue;
        int64_t di = i2 - i, dj = j2 - j;
        int64_t cmax = llabs(di) > llabs(dj) ? llabs(di) : llabs(dj);
        for (int64_t c = 1; c < cmax; ++c) {
            int64_t ic = (2 * i * cmax + 2 * c * di + cmax) / (2 * cmax);
            int64_t jc = (2 * j * cmax + 2 * c * dj + cmax) / (2 * cmax);
            counts[jc * nx + ic] += 1;
            tot += 1;
        }
    }
    *total = tot;
}

/* One convolution tap: k(s/H) at integer offset s (0 outside a compact support). */
static double tap(int kernel, int s, float H)
{
    double d = (double)s;
    if (kernel != KO_GAUSSIAN && fabs(d) > (double)H) return 0.0;
    return ko_k(kernel, d / (double)H);
}

/* Eq. (7) over the window [i0, i1) x [j0, j1):
 *   out[r] = sum_{t=-b..b} sum_{s=-a..a} f(s, t) counts[j - t][i - s]
 * with f(s, t) = tap(s; Hx) tap(t; Hy), raw (no normalisation). */
void ko_conv_counts(const uint32_t *counts, int nx, int ny, int kernel, float Hx, float Hy, int a, int b,
                    int i0, int i1, int j0, int j1, double *out)
{
    int w = i1 - i0, h = j1 - j0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < h * w; ++r) {
        int j = j0 + r / w, i = i0 + r % w;
        double sum = 0.0;
        for (int t = -b; t <= b; ++t) {
            int jj = j - t;
            if (jj < 0 || jj >= ny) continue;
            for (int s = -a; s <= a; ++s) {
                int ii = i - s;
                if (ii < 0 || ii >= nx) continue;
                sum += tap(kernel, s, Hx) * tap(kernel, t, Hy) * (double)counts[(int64_t)jj * nx + ii];
            }
        }
        out[r] = sum;
    }
}

/* ---------------------------------------------------------------------------
 * Douglas-Peucker compression of every trajectory (Sec. III-B, its GPU form in
 * Sec. IV-A): keep both end points of a track; for the chord between two kept
 * points, the interior point farthest from the chord's line (Eq. (9), the
 * vertical Euclidean distance) is kept when that distance is larger than eps,
 * which splits the chord in two; repeat until no chord has such a point.
 *
 * Readings: the lowest index wins a tie for the largest distance; a chord with
 * coinciding end points uses the distance to that point; the test
 * D > eps is taken as cross^2 > eps^2 |chord|^2 (cross = the 2-D cross product
 * of Eq. (9)'s numerator), or |P - Ps|^2 > eps^2 for a zero chord, so that no
 * square root or division enters the decision.  FP64, no fused multiply-add.
 * -------------------------------------------------------------------------*/

/* Score of point i against chord (s, e): |cross| (or the squared distance to
 * P_s when the chord has zero length).  *zero tells which. */
static double dp_score(const double *xy, int64_t s, int64_t e, int64_t i, int *zero)
{
    double cx = xy[2 * e] - xy[2 * s], cy = xy[2 * e + 1] - xy[2 * s + 1];
    double px = xy[2 * i] - xy[2 * s], py = xy[2 * i + 1] - xy[2 * s + 1];
    double c2 = cx * cx + cy * cy;
    *zero = c2 == 0.0;
    if (*zero) return px * px + py * py;
    double a = px * cy, b = py * cx;
    return fabs(a - b);
}

/* keep[n] (0/1) for points xy[n][2] (metres, FP64) in tracks
 * [start[t], start[t+1]), t < n_tracks.  Returns the number kept. */
int64_t ko_dp_keep(const double *xy, int64_t n, const int64_t *start, int64_t n_tracks, double eps, uint8_t *keep)
{
    (void)n;
    int64_t kept = 0;
    double eps2 = eps * eps;
    for (int64_t t = 0; t < n_tracks; ++t) {
        int64_t a = start[t], z = start[t + 1];
        for (int64_t i = a; i < z; ++i) keep[i] = 0;
        if (z <= a) continue;
        keep[a] = 1;
        keep[z - 1] = 1;
        /* explicit stack of chords (s, e) */
        int64_t cap = 64, top = 0;
        int64_t *st = (int64_t *)malloc((size_t)cap * 2 * sizeof(int64_t));
        st[0] = a;
        st[1] = z - 1;
        top = 1;
        while (top > 0) {
            --top;
            int64_t s = st[2 * top], e = st[2 * top + 1];
            if (e - s < 2) continue;
            int64_t best = -1;
            double bs = -1.0;
            int zero = 0;
            for (int64_t i = s + 1; i < e; ++i) {
                double sc = dp_score(xy, s, e, i, &zero);
                if (sc > bs) { bs = sc; best = i; } /* strict: the lowest index wins ties */
            }
            double cx = xy[2 * e] - xy[2 * s], cy = xy[2 * e + 1] - xy[2 * s + 1];
            double c2 = cx * cx + cy * cy;
            int split = zero ? (bs > eps2) : (bs * bs > eps2 * c2);
            if (!split) continue;
            keep[best] = 1;
            if (top + 2 > cap) {
                cap *= 2;
                st = (int64_t *)realloc(st, (size_t)cap * 2 * sizeof(int64_t));
            }
            st[2 * top] = best; st[2 * top + 1] = e; ++top;
            st[2 * top] = s; st[2 * top + 1] = best; ++top;
        }
        free(st);
    }
    for (int64_t t = 0; t < n_tracks; ++t)
        for (int64_t i = start[t]; i < start[t + 1]; ++i) kept += keep[i];
    return kept;
}

/* ------------------------------------------------------------------------
 * Compression quality (Sec. V-B).  Points are planar FP64 pairs (x, y).
 * ------------------------------------------------------------------------ */

/* Track length: sum over consecutive points of the Euclidean distance
 * |P_n P_{n+1}| (the |T| inside the RLL definition, Eq. (15)).  Index order. */
double ko_track_length(const double *xy, int64_t n)
{
    double len = 0.0;
    for (int64_t i = 0; i + 1 < n; ++i) {
        double dx = xy[2 * (i + 1)] - xy[2 * i];
        double dy = xy[2 * (i + 1) + 1] - xy[2 * i + 1];
        len += sqrt(dx * dx + dy * dy);
    }
    return len;
}

/* DTW distance of Eq. (16)-(18): the accumulated cost matrix
 *   D[i][j] = d(P_i, P'_j) + min(D[i-1][j-1], D[i-1][j], D[i][j-1]),
 * d the squared Euclidean distance, with D[-1][-1] = 0 and every other border
 * entry +inf, filled row by row (two rows kept); returns sqrt(D[na-1][nb-1]).
 * No warping path joins an empty series to a non-empty one (+inf); two empty
 * series are at distance 0. */
double ko_dtw(const double *a, int64_t na, const double *b, int64_t nb)
{
    if (na == 0 || nb == 0) return (na == 0 && nb == 0) ? 0.0 : INFINITY;
    double *prev = (double *)malloc((size_t)(nb + 1) * sizeof(double));
    double *cur = (double *)malloc((size_t)(nb + 1) * sizeof(double));
    /* column 0 of these rows is the border j = -1 */
    prev[0] = 0.0;
    for (int64_t j = 1; j <= nb; ++j) prev[j] = INFINITY;
    for (int64_t i = 0; i < na; ++i) {
        cur[0] = INFINITY;
        for (int64_t j = 0; j < nb; ++j) {
            double dx = a[2 * i] - b[2 * j], dy = a[2 * i + 1] - b[2 * j + 1];
            double d = dx * dx + dy * dy;
            double m = prev[j];                    /* D[i-1][j-1] */
            if (prev[j + 1] < m) m = prev[j + 1];  /* D[i-1][j] */
            if (cur[j] < m) m = cur[j];            /* D[i][j-1] */
            cur[j + 1] = d + m;
        }
        double *t = prev;
        prev = cur;
        cur = t;
    }
    double r = sqrt(prev[nb]);
    free(prev);
    free(cur);
    return r;
}

/* Per-track lengths and DTW distances of a track set and its compressed
 * version, tracks [start_o[m], start_o[m+1]) and [start_c[m], start_c[m+1]).
 * Tracks are independent: one OpenMP task each. */
void ko_track_metrics(const double *xy_o, const int64_t *start_o, const double *xy_c, const int64_t *start_c,
                      int64_t n_tracks, double *len_o, double *len_c, double *dtw)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < n_tracks; ++m) {
        const double *o = xy_o + 2 * start_o[m], *c = xy_c + 2 * start_c[m];
        int64_t no = start_o[m + 1] - start_o[m], nc = start_c[m + 1] - start_c[m];
        len_o[m] = ko_track_length(o, no);
        len_c[m] = ko_track_length(c, nc);
        dtw[m] = ko_dtw(o, no, c, nc);
    }
}
