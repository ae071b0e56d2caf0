/*
 * CPU FP64 oracle for the x-ray transform of a tensor-product B-spline image.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the HIP library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the GPU path, and the GPU path never calls it.
 *
 * What it computes is the plain definition of the discretised operator
 * (Section I-B, eqs. (2)-(4); Section IV-A, the entries of H_phi):
 *
 *     s_m       = sum_k c_k * h * phi_{theta_m}( (y_m - <x_k, theta_m^perp>) / h )
 *     (H^T s)_k = sum_m s_m * h * phi_{theta_m}( (y_m - <x_k, theta_m^perp>) / h )
 *
 * with theta = (cos t, sin t), theta^perp = (sin t, -cos t) (eq. (1)), the
 * generator phi(x1,x2) = beta^n(x1) beta^n(x2) (Section III-C) and its
 * projection phi_theta = beta^n_{|cos t|} * beta^n_{|sin t|}, where
 * beta_a(x) = beta(x/a)/a (Proposition 1 / eq. (6), Section III-A,B).  The
 * grid spacing is h (the paper takes h = 1 without loss of generality) and the
 * grid centres are x_ij = (cx + (i - (nx-1)/2) h, cy + (j - (ny-1)/2) h).
 *
 * No ray tracing happens here: for every line and every grid row (or column)
 * the set of centres with |u| <= w, w = (n+1)(|cos|+|sin|)/2, is found by
 * interval arithmetic and every centre in it is evaluated.  Sums are
 * Neumaier-compensated.
 *
 * The footprint phi_theta(u) has two independent FP64 evaluations:
 *   - orc_footprint_tp: the truncated-power closed form that follows from
 *     eq. (6) for B-splines (the general-degree version of the degree-1
 *     formula printed in Section III-C);  it divides by (|cos| |sin|)^(n+1)
 *     and is used only when min(|cos|,|sin|) >= 0.25, where its FP64
 *     error stays below about 1e-11;
 *   - orc_footprint_gl: the convolution integral of eq. (6) written as
 *     int beta(v) beta((u - B v)/A)/A dv  (A = max, B = min of |cos|,|sin|),
 *     split at every knot of both factors and integrated with (n+1)-point
 *     Gauss-Legendre, which is exact for the degree-2n polynomial pieces.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1

/* ---------------------------------------------------------------- B-splines
 * Centred B-spline of degree n (Unser, "B-spline signal processing", 1993),
 * written as its explicit piecewise polynomials.  Degree 0 takes the value
 * 1/2 at |x| = 1/2 (the symmetric convention). */
double orc_bspline(int n, double x)
{
    double ax = fabs(x);
    switch (n) {
    case 0:
        if (ax < 0.5) return 1.0;
        if (ax == 0.5) return 0.5;
        return 0.0;
    case 1:
        return ax < 1.0 ? 1.0 - ax : 0.0;
    case 2:
        if (ax < 0.5) return 0.75 - ax * ax;
        if (ax < 1.5) { double t = 1.5 - ax; return 0.5 * t * t; }
        return 0.0;
    case 3:
        if (ax < 1.0) return (4.0 - 6.0 * ax * ax + 3.0 * ax * ax * ax) / 6.0;
        if (ax < 2.0) { double t = 2.0 - ax; return t * t * t / 6.0; }
        return 0.0;
    default:
        return NAN;
    }
}

static double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

static double factorial(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= (double)i;
    return r;
}

/* Basis code of the 3-directional box spline (directions e1, e2, e1+e2),
 * Section III-C; degrees 0..3 are the tensor-product B-splines. */
#define ORC_BOX3 16

/* Support half-width of phi_theta (c = cos, s = sin, signed):
 * B-splines (n+1)(|c|+|s|)/2; the box spline (|s| + |c| + |s - c|)/2, half
 * the summed widths |<theta_perp, u_d>| of its three directions. */
static double support_halfwidth(int n, double c, double s)
{
    if (n == ORC_BOX3) return 0.5 * (fabs(s) + fabs(c) + fabs(s - c));
    return 0.5 * (double)(n + 1) * (fabs(c) + fabs(s));
}

/* --------------------------------------------- box spline, in space
 * M(x) = int_0^1 1_[0,1]^2(x - t(1,1)) dt = max(0, min(1, x1, x2) - max(0, x1-1, x2-1)),
 * the box spline of the directions e1, e2, e1+e2 (a hat on a hexagon, value
 * 1 at the centre (1,1)); centred: Mc(x) = M(x + (1,1)). */
double orc_box_spline(double x1, double x2)
{
    double lo = fmax(0.0, fmax(x1 - 1.0, x2 - 1.0));
    double hi = fmin(1.0, fmin(x1, x2));
    return fmax(0.0, hi - lo);
}

/* Footprint of the centred box spline: the line integral
 *   phi_theta(u) = int Mc(t theta + u theta_perp) dt,  theta = (c, s), theta_perp = (s, -c),
 * computed exactly: along the line Mc is piecewise linear in t with kinks only
 * where x1 = 0, x2 = 0 or x1 = x2, and zero for |t| > sqrt(2); between
 * consecutive kinks the positive part of a linear function is integrated in
 * closed form. */
double orc_footprint_box(double c, double s, double u)
{
    double pts[5];
    int np = 0;
    const double T = 2.0;
    pts[np++] = -T;
    if (c != 0.0) pts[np++] = -u * s / c;          /* x1 = t c + u s = 0 */
    if (s != 0.0) pts[np++] = u * c / s;           /* x2 = t s - u c = 0 */
    if (c != s) pts[np++] = -u * (s + c) / (c - s); /* x1 = x2 */
    pts[np++] = T;
    /* sort and clip to [-T, T] */
    for (int i = 1; i < np; ++i)
        for (int k = i; k > 0 && pts[k] < pts[k - 1]; --k) {
            double t = pts[k]; pts[k] = pts[k - 1]; pts[k - 1] = t;
        }
    double acc = 0.0;
    for (int i = 0; i + 1 < np; ++i) {
        double p = fmax(pts[i], -T), q = fmin(pts[i + 1], T);
        if (!(q > p)) continue;
        /* Mc = max(0, g), g = min(1, x1+1, x2+1) - max(0, x1, x2) linear on [p, q] */
        double xp1 = p * c + u * s, xp2 = p * s - u * c, xq1 = q * c + u * s, xq2 = q * s - u * c;
        double rp = fmin(1.0, fmin(xp1 + 1.0, xp2 + 1.0)) - fmax(0.0, fmax(xp1, xp2));
        double rq = fmin(1.0, fmin(xq1 + 1.0, xq2 + 1.0)) - fmax(0.0, fmax(xq1, xq2));
        if (rp >= 0.0 && rq >= 0.0) acc += 0.5 * (rp + rq) * (q - p);
        else if (rp > 0.0) acc += 0.5 * rp * (q - p) * rp / (rp - rq);
        else if (rq > 0.0) acc += 0.5 * rq * (q - p) * rq / (rq - rp);
    }
    return acc;
}

/* ------------------------------------------------ footprint, closed form
 * Each of beta^n_a and beta^n_b is an (n+1)-th central difference of a
 * one-sided power; their convolution (eq. (6)) is therefore
 *   phi(u) = sum_{i,j=0}^{n+1} (-1)^(i+j) C(n+1,i) C(n+1,j)
 *            (u + (n+1)(a+b)/2 - i a - j b)_+^(2n+1) / ((2n+1)! a^(n+1) b^(n+1)).
 * Requires a > 0 and b > 0. */
double orc_footprint_tp(int n, double c, double s, double u)
{
    double a = fabs(c), b = fabs(s);
    if (n < 0 || n > 3 || !(a > 0.0) || !(b > 0.0)) return NAN;
    double w = support_halfwidth(n, c, s);
    if (fabs(u) >= w) return 0.0;
    int p = 2 * n + 1;
    double acc = 0.0, comp = 0.0;
    for (int i = 0; i <= n + 1; ++i) {
        for (int j = 0; j <= n + 1; ++j) {
            double arg = u + w - (double)i * a - (double)j * b;
            if (arg <= 0.0) continue;
            double term = binom(n + 1, i) * binom(n + 1, j) * pow(arg, p);
            if ((i + j) & 1) term = -term;
            double t = acc + term;
            if (fabs(acc) >= fabs(term)) comp += (acc - t) + term;
            else comp += (term - t) + acc;
            acc = t;
        }
    }
    return (acc + comp) / (factorial(p) * pow(a, n + 1) * pow(b, n + 1));
}

/* ------------------------------------------------ footprint, quadrature
 * Gauss-Legendre nodes and weights on [-1, 1] for 1..4 points. */
static const double GL_X[4][4] = {
    {0.0, 0, 0, 0},
    {-0.57735026918962576451, 0.57735026918962576451, 0, 0},
    {-0.77459666924148337704, 0.0, 0.77459666924148337704, 0},
    {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
     0.86113631159405257522}};
static const double GL_W[4][4] = {
    {2.0, 0, 0, 0},
    {1.0, 1.0, 0, 0},
    {0.55555555555555555556, 0.88888888888888888889, 0.55555555555555555556, 0},
    {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
     0.34785484513745385737}};

static int cmp_double(const void* x, const void* y)
{
    double a = *(const double*)x, b = *(const double*)y;
    return (a > b) - (a < b);
}

double orc_footprint_gl(int n, double c, double s, double u)
{
    double a = fabs(c), b = fabs(s);
    if (n < 0 || n > 3 || !(a >= 0.0) || !(b >= 0.0) || !(a + b > 0.0)) return NAN;
    double A = a > b ? a : b;
    double B = a > b ? b : a;
    double hw = 0.5 * (double)(n + 1);
    if (B == 0.0) {
        /* the factor with zero scale is a Dirac (Proposition 1) */
        return orc_bspline(n, u / A) / A;
    }
    if (fabs(u) >= support_halfwidth(n, c, s)) return 0.0;
    double pts[2 * 5 + 2];
    int np = 0;
    for (int k = 0; k <= n + 1; ++k) pts[np++] = (double)k - hw;          /* knots of beta(v) */
    for (int k = 0; k <= n + 1; ++k) {                                     /* knots of beta((u-Bv)/A) */
        double v = (u - A * ((double)k - hw)) / B;
        if (v > -hw && v < hw) pts[np++] = v;
    }
    qsort(pts, (size_t)np, sizeof(double), cmp_double);
    int q = n + 1; /* nodes: exact for polynomials of degree 2n+1 >= 2n */
    double acc = 0.0;
    for (int k = 0; k + 1 < np; ++k) {
        double lo = pts[k], hi = pts[k + 1];
        if (!(hi > lo)) continue;
        double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
        double part = 0.0;
        for (int g = 0; g < q; ++g) {
            double v = mid + half * GL_X[q - 1][g];
            part += GL_W[q - 1][g] * orc_bspline(n, v) * orc_bspline(n, (u - B * v) / A);
        }
        acc += part * half;
    }
    return acc / A;
}

/* Footprint used by the operator: closed form where it is well conditioned
 * (min(|cos|,|sin|) >= 0.25), the quadrature otherwise. */
double orc_footprint(int n, double c, double s, double u)
{
    if (n == ORC_BOX3) return orc_footprint_box(c, s, u);
    double B = fmin(fabs(c), fabs(s));
    if (B >= 0.25) return orc_footprint_tp(n, c, s, u);
    return orc_footprint_gl(n, c, s, u);
}

/* ------------------------------------------------------------------ lines
 * Line (theta, y) of eq. (1) from the float32 inputs, widened to FP64. */
int orc_lines_theta_y(int64_t m, const float* theta, const float* y, double* cs, double* sn,
                      double* yy)
{
    for (int64_t i = 0; i < m; ++i) {
        double t = (double)theta[i];
        cs[i] = cos(t);
        sn[i] = sin(t);
        yy[i] = (double)y[i];
    }
    return ORC_OK;
}

/* Line through two points p, q (endpoints [m][4] = px, py, qx, qy): its
 * direction is theta = (q - p)/|q - p| and its offset y = <p, theta^perp>.
 * Coincident endpoints are an error. */
int orc_lines_endpoints(int64_t m, const float* ep, double* cs, double* sn, double* yy)
{
    for (int64_t i = 0; i < m; ++i) {
        double px = ep[4 * i + 0], py = ep[4 * i + 1];
        double qx = ep[4 * i + 2], qy = ep[4 * i + 3];
        double dx = qx - px, dy = qy - py;
        double L = hypot(dx, dy);
        if (!(L > 0.0)) return ORC_EINVAL;
        cs[i] = dx / L;
        sn[i] = dy / L;
        yy[i] = px * sn[i] - py * cs[i];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ grid */
typedef struct {
    int32_t nx, ny;
    double spacing, cx, cy;
} orc_grid;

static double gx(const orc_grid* g, int i) { return g->cx + ((double)i - 0.5 * (g->nx - 1)) * g->spacing; }
static double gy(const orc_grid* g, int j) { return g->cy + ((double)j - 0.5 * (g->ny - 1)) * g->spacing; }

/* Offset of centre (i, j) from the line, in grid units:
 * u = (y - <x_ij, theta^perp>) / h,  <x, theta^perp> = x1 sin - x2 cos. */
static double offset_u(const orc_grid* g, double c, double s, double y, int i, int j)
{
    return (y - (gx(g, i) * s - gy(g, j) * c)) / g->spacing;
}

/* Neumaier accumulator */
typedef struct { double s, c; } nsum;
static void nadd(nsum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

/* Indices k with |t0 + k*dt| <= lim, k in [0, kmax): the closed interval is
 * widened by a relative 1e-12 so that no centre on the support boundary is
 * dropped (the footprint returns the exact value there). */
static void band(double t0, double dt, double lim, int kmax, int* lo, int* hi)
{
    /* solve -lim <= t0 + k dt <= lim for k (dt != 0) */
    double a = (-lim - t0) / dt, b = (lim - t0) / dt;
    if (a > b) { double t = a; a = b; b = t; }
    double pad = 1e-12 * (fabs(a) + fabs(b) + 1.0);
    double fa = ceil(a - pad), fb = floor(b + pad);
    if (fa < 0) fa = 0;
    if (fb > kmax - 1) fb = kmax - 1;
    *lo = (int)fa;
    *hi = (int)fb;
}

/* Visits every centre of the band of one line, in the order: major index
 * (rows when |sin| >= |cos|, columns otherwise) then minor index. */
#define FOR_BAND(g, n, c, s, y, BODY)                                                    \
    do {                                                                                 \
        double w_ = support_halfwidth((n), (c), (s));                                    \
        if (fabs(s) >= fabs(c)) {                                                        \
            /* u = (y + x2 c - x1 s)/h ; x1 = cx + (i - ox) h  => u linear in i */      \
            for (int j = 0; j < (g)->ny; ++j) {                                          \
                double u0 = offset_u((g), (c), (s), (y), 0, j);                          \
                double du = -(s);                                                        \
                int lo_, hi_;                                                            \
                band(u0, du, w_, (g)->nx, &lo_, &hi_);                                   \
                for (int i = lo_; i <= hi_; ++i) {                                       \
                    double u = offset_u((g), (c), (s), (y), i, j);                       \
                    BODY                                                                 \
                }                                                                        \
            }                                                                            \
        } else {                                                                         \
            for (int i = 0; i < (g)->nx; ++i) {                                          \
                double u0 = offset_u((g), (c), (s), (y), i, 0);                          \
                double du = (c);                                                         \
                int lo_, hi_;                                                            \
                band(u0, du, w_, (g)->ny, &lo_, &hi_);                                   \
                for (int j = lo_; j <= hi_; ++j) {                                       \
                    double u = offset_u((g), (c), (s), (y), i, j);                       \
                    BODY                                                                 \
                }                                                                        \
            }                                                                            \
        }                                                                                \
    } while (0)

static int check_args(int n, const orc_grid* g)
{
    if ((n < 0 || n > 3) && n != ORC_BOX3) return ORC_EINVAL;
    if (!g || g->nx <= 0 || g->ny <= 0 || !(g->spacing > 0.0)) return ORC_EINVAL;
    return ORC_OK;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* --------------------------------------------------------------- forward
 * s_m = sum_k c_k h phi(u_mk) over the band (eq. (4)); coeffs is [ny][nx]. */
int orc_forward(int n, const orc_grid* g, const double* coeffs, int64_t m, const double* cs,
                const double* sn, const double* yy, double* out, int nthreads)
{
    if (check_args(n, g) != ORC_OK || m < 0) return ORC_EINVAL;
    set_threads(nthreads);
    const int nx = g->nx;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < m; ++r) {
        double c = cs[r], s = sn[r], y = yy[r];
        nsum acc = {0.0, 0.0};
        FOR_BAND(g, n, c, s, y, {
            double f = orc_footprint(n, c, s, u);
            if (f != 0.0) nadd(&acc, coeffs[(int64_t)j * nx + i] * f);
        });
        out[r] = (acc.s + acc.c) * g->spacing;
    }
    return ORC_OK;
}

/* Same sum over every grid centre, with the same major/minor visiting order
 * (used to check the band enumeration). */
int orc_forward_dense(int n, const orc_grid* g, const double* coeffs, int64_t m,
                      const double* cs, const double* sn, const double* yy, double* out)
{
    if (check_args(n, g) != ORC_OK || m < 0) return ORC_EINVAL;
    const int nx = g->nx, ny = g->ny;
    for (int64_t r = 0; r < m; ++r) {
        double c = cs[r], s = sn[r], y = yy[r];
        nsum acc = {0.0, 0.0};
        int vertical = fabs(s) >= fabs(c);
        int nmaj = vertical ? ny : nx, nmin = vertical ? nx : ny;
        for (int a = 0; a < nmaj; ++a)
            for (int b = 0; b < nmin; ++b) {
                int i = vertical ? b : a, j = vertical ? a : b;
                double u = offset_u(g, c, s, y, i, j);
                double f = orc_footprint(n, c, s, u);
                if (f != 0.0) nadd(&acc, coeffs[(int64_t)j * nx + i] * f);
            }
        out[r] = (acc.s + acc.c) * g->spacing;
    }
    return ORC_OK;
}

/* --------------------------------------------------------------- adjoint
 * (H^T s)_k = sum_m s_m h phi(u_mk): ray-major scatter into one FP64 image
 * per thread, summed at the end.  out is [ny][nx], overwritten. */
int orc_adjoint(int n, const orc_grid* g, int64_t m, const double* cs, const double* sn,
                const double* yy, const double* sino, double* out, int nthreads)
{
    if (check_args(n, g) != ORC_OK || m < 0) return ORC_EINVAL;
    set_threads(nthreads);
    const int nx = g->nx;
    const int64_t npx = (int64_t)g->nx * g->ny;
    int nt = orc_max_threads();
    double* part = (double*)calloc((size_t)nt * (size_t)npx, sizeof(double));
    if (!part) return ORC_EINVAL;
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* img = part + (int64_t)tid * npx;
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < m; ++r) {
            double c = cs[r], s = sn[r], y = yy[r], sv = sino[r];
            if (sv == 0.0) continue;
            FOR_BAND(g, n, c, s, y, {
                double f = orc_footprint(n, c, s, u);
                if (f != 0.0) img[(int64_t)j * nx + i] += sv * f;
            });
        }
    }
    for (int64_t k = 0; k < npx; ++k) {
        nsum acc = {0.0, 0.0};
        for (int t = 0; t < nt; ++t) nadd(&acc, part[(int64_t)t * npx + k]);
        out[k] = (acc.s + acc.c) * g->spacing;
    }
    free(part);
    return ORC_OK;
}

/* Adjoint at a list of pixels only (flat index j*nx + i): for each listed
 * pixel every line is tested, and the lines within the support contribute.
 * Used for sampled checks on grids too large for the full adjoint. */
int orc_adjoint_pixels(int n, const orc_grid* g, int64_t m, const double* cs, const double* sn,
                       const double* yy, const double* sino, int64_t npix, const int64_t* pix,
                       double* out, int nthreads)
{
    if (check_args(n, g) != ORC_OK || m < 0 || npix < 0) return ORC_EINVAL;
    set_threads(nthreads);
    const int nx = g->nx;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < npix; ++p) {
        int i = (int)(pix[p] % nx), j = (int)(pix[p] / nx);
        nsum acc = {0.0, 0.0};
        for (int64_t r = 0; r < m; ++r) {
            double c = cs[r], s = sn[r];
            double u = offset_u(g, c, s, yy[r], i, j);
            double w = support_halfwidth(n, c, s);
            if (fabs(u) > w * (1.0 + 1e-12)) continue;
            double f = orc_footprint(n, c, s, u);
            if (f != 0.0) nadd(&acc, sino[r] * f);
        }
        out[p] = (acc.s + acc.c) * g->spacing;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------ work count
 * Number of (line, centre) pairs with |u| < w strictly: the structural
 * nonzeros of H.  Counted by interval arithmetic only. */
int64_t orc_nnz(int n, const orc_grid* g, int64_t m, const double* cs, const double* sn,
                const double* yy, int nthreads)
{
    if (check_args(n, g) != ORC_OK || m < 0) return -1;
    set_threads(nthreads);
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int64_t r = 0; r < m; ++r) {
        double c = cs[r], s = sn[r], y = yy[r];
        int64_t cnt = 0;
        FOR_BAND(g, n, c, s, y, {
            if (fabs(u) < w_) ++cnt;
        });
        total += cnt;
    }
    return total;
}
