/*
 * xrt.h -- x-ray transform of tensor-product B-spline images (degree 0..3)
 * over an arbitrary list of lines, and its exact adjoint, on AMD Instinct
 * MI355X (gfx950).  C ABI of libxrt.so.
 *
 * Mathematical definition (Haouchat et al., "Generalized Ray Tracing with Basis
 * Functions for Tomographic Projections"):
 *
 *   image       f = sum_k c_k phi((x - x_k)/h),  phi = beta^n (x) beta^n
 *               (eq. (3) with the tensor B-spline generator of Section III-C);
 *   line        {t theta + y theta_perp}, theta = (cos t, sin t),
 *               theta_perp = (sin t, -cos t)                      (eq. (1));
 *   forward     s_m = P_{theta_m}{f}(y_m)
 *                   = sum_k c_k h phi_{theta_m}((y_m - <x_k, theta_m_perp>)/h)
 *               (eqs. (2) and (4); the matrix H_phi of Section IV-A);
 *   footprint   phi_theta = beta^n_{|cos t|} * beta^n_{|sin t|},
 *               beta_a(x) = beta(x/a)/a  (Proposition 1 / eq. (6));
 *   adjoint     (H^T s)_k = sum_m s_m h phi_{theta_m}((y_m - <x_k, theta_m_perp>)/h)
 *               (the matched back-projection of Section II-B).
 *
 * Grid: coefficients are a row-major float32 array [ny][nx]; element (j, i)
 * sits at x_ij = (cx + (i - (nx-1)/2) h, cy + (j - (ny-1)/2) h): column i along
 * x1, row j along x2.  The image extends (n+1)h/2 beyond the outer centres;
 * lines that only graze that margin are included.
 *
 * Conventions for every entry point:
 *   - All array pointers are DEVICE pointers owned by the caller; the library
 *     never frees them.  Outputs are overwritten, not accumulated.  Inputs and
 *     outputs must not alias.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     Entry points that create a plan (xrt_plan_create, and xrt_forward /
 *     xrt_adjoint, which build a temporary plan) synchronise with `stream` once,
 *     during plan creation, to read the plan header back (that is where
 *     degenerate or non-finite lines are found); they do not wait for the
 *     transform itself.  xrt_plan_forward / xrt_plan_adjoint and
 *     xrt_adjoint_noalloc do not synchronise.
 *   - Argument errors are returned synchronously before any work is enqueued.
 *     A failing HIP call returns XRT_EHIP; xrt_last_error() then gives the HIP
 *     message for the calling thread.
 *   - Arithmetic is float32 with float64 line geometry; results match the
 *     plain FP64 definition above to about 1e-6 relative (L2 over a sinogram).
 */
#ifndef XRT_H
#define XRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    XRT_OK = 0,
    XRT_EINVAL = -1,  /* null pointer, negative count, bad grid, non-finite or degenerate line */
    XRT_EDEGREE = -2, /* degree neither 0..3 nor XRT_BOX3 */
    XRT_ESIZE = -3,   /* grid or line count beyond the supported range */
    XRT_ENOMEM = -4,  /* device allocation failed; nothing is left allocated */
    XRT_EHIP = -5,    /* a HIP call or kernel launch failed */
    XRT_EPLAN = -6    /* plan and call disagree (null or foreign plan) */
} xrt_status;

/* Basis: `degree` 0..3 selects the tensor-product B-spline beta^n (x) beta^n
 * (Section III-C, eq. (6)); XRT_BOX3 selects the 3-directional box spline of
 * directions e1, e2, e1+e2 (Section III-C): centred, a piecewise-linear hat
 * on a hexagon, phi(x) = max(0, min(1, x1+1, x2+1) - max(0, x1, x2)).  By
 * Proposition 1 its footprint is the convolution of three centred unit-mass
 * boxes of widths |<theta_perp, u_d>| = |sin t|, |cos t|, |sin t - cos t|
 * (eq. (projbox) written for the line direction theta = (cos t, sin t)). */
#define XRT_BOX3 16

/* Coefficient grid.  nx, ny >= 1 and <= 32768; spacing h > 0 (the paper
 * takes h = 1); (cx, cy) is the centre of the grid of centres. */
typedef struct {
    int32_t nx, ny;
    double spacing;
    double cx, cy;
} xrt_grid;

typedef enum {
    XRT_LINES_THETA_Y = 0,  /* theta[n], y[n]: the (theta, y) of eq. (1), float32 */
    XRT_LINES_ENDPOINTS = 1 /* endpoints[n][4] = (px, py, qx, qy), float32: the infinite
                               line through p and q; p == q is an error */
} xrt_line_kind;

/* A list of n lines (0 <= n < 2^31).  Pointers are device pointers; only the
 * ones of the chosen kind are read. */
typedef struct {
    int32_t kind;
    int64_t n;
    const float* theta;
    const float* y;
    const float* endpoints;
} xrt_lines;

/* Opaque plan: the line list canonicalised in FP64 and sorted into
 * (orientation, slope bin, crossing bucket) order, the bucket offsets the
 * adjoint uses to find the lines crossing each image tile, and a workspace for
 * the per-call coefficient layouts.  The geometry part is immutable; the
 * workspace is reused by every call, so calls with one plan must not overlap
 * (use one plan per concurrent stream). */
typedef struct xrt_plan xrt_plan;

/* Forward projection (eq. (4)) of coeffs [g.ny][g.nx] along every line into
 * sino [lines->n].  Builds a temporary plan (synchronising once, in its
 * creation) and frees it stream-ordered after the launches. */
xrt_status xrt_forward(const float* coeffs, xrt_grid g, int degree, const xrt_lines* lines,
                       float* sino, void* stream);

/* Adjoint (back-projection, the transpose of H of Section IV-A, as in
 * Section II-B) of sino [lines->n] into coeffs_out [g.ny][g.nx].  Builds a
 * temporary plan (synchronising once, in its creation) and frees it
 * stream-ordered after the launches. */
xrt_status xrt_adjoint(const float* sino, const xrt_lines* lines, int degree, xrt_grid g,
                       float* coeffs_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * adjoint of xrt_adjoint, same arguments, same result bit for bit, with no
 * device allocation or free and no synchronisation.  Its temporary plan
 * lives in one static device array of 64 MiB that each GPU the library runs
 * on holds until the process ends (about 56 B per line, 8 B per
 * (orientation, slope bin, crossing bucket) key and up to 16 partial images,
 * 8 per pass, both passes sharing one launch on small grids: e.g. 700,000
 * lines on a 512^2 grid); larger problems return XRT_ESIZE.
 * The first call on a device sets the array up (looks up its address,
 * synchronously).  Every call on one GPU
 * shares that array: calls that overlap on one GPU race and must be
 * serialised by the caller.  Degenerate or non-finite lines are not
 * reported (that needs a synchronisation); they contribute nothing.
 * Use xrt_plan_create to validate a line list. */
xrt_status xrt_adjoint_noalloc(const float* sino, const xrt_lines* lines, int degree, xrt_grid g,
                               float* coeffs_out, void* stream);

/* Builds a plan for (grid, degree, lines).  The line arrays are read during
 * the call only.  On error *out is NULL and nothing stays allocated.
 * Device memory held by the plan: about 24 B per line (sorted line records,
 * scaled sinogram), 4 B per line and strip of 128 grid rows (the forward's
 * strip sums; per half or quarter strip on small problems; 8 B per line
 * instead when that would pass 4 GiB), four padded copies of the
 * coefficient grid, up to 16 partial images (8 per adjoint pass), and 4 B
 * per (orientation, slope bin, crossing bucket) key. */
xrt_status xrt_plan_create(xrt_grid g, int degree, const xrt_lines* lines, void* stream,
                           xrt_plan** out);

/* Forward / adjoint with a plan: the hot path.  xrt_plan_forward computes
 * eq. (4), s_m = sum_k c_k h phi_theta_m((y_m - <x_k, theta_m_perp>)/h), for
 * every line of the plan into sino [n] (the caller's line order);
 * xrt_plan_adjoint computes its exact transpose (Section II-B: the
 * back-projection with the same footprint) of sino [n] into
 * coeffs_out [ny][nx], overwriting it.  coeffs/sino/coeffs_out are
 * caller-owned device arrays; work is enqueued on `stream`.  No
 * synchronisation, no allocation.  Repeated calls with one plan give
 * bitwise-identical results, and so do two plans built from the same lines
 * (the plan's sort is stable: lines of one bucket keep their input order).
 * Errors: XRT_EPLAN (not a plan), XRT_EINVAL (null array), XRT_EHIP. */
xrt_status xrt_plan_forward(const xrt_plan* p, const float* coeffs, float* sino, void* stream);
xrt_status xrt_plan_adjoint(const xrt_plan* p, const float* sino, float* coeffs_out,
                            void* stream);

/* Number of lines of the plan, and of those that cross the padded grid. */
xrt_status xrt_plan_info(const xrt_plan* p, int64_t* n_lines, int64_t* n_crossing);

/* Exact number of (line, centre) pairs inside the footprint support
 * (|u| < (n+1)(|cos|+|sin|)/2): the structural nonzeros of H_phi, i.e. the
 * basis evaluations one forward or adjoint pass performs.  Counted on the
 * device; synchronises with `stream`. */
xrt_status xrt_plan_nnz(const xrt_plan* p, int64_t* nnz, void* stream);

/* Frees the plan (waits for the device to finish using it).  NULL is a no-op. */
void xrt_plan_destroy(xrt_plan* p);

/* Static description of a status code. */
const char* xrt_status_string(xrt_status st);

/* Message of the last XRT_EHIP / XRT_ENOMEM failure on the calling thread
 * ("" if none). */
const char* xrt_last_error(void);

/* Library version "major.minor.patch". */
const char* xrt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* XRT_H */
