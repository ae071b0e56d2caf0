// Line geometry and the adjoint's accumulator index arithmetic, shared by
// the HIP kernels and by host-side replays that check every LDS address the
// adjoint forms (the functions compile for the host and for the device).
//
// A line of eq. (1), <x, theta_perp> = y, is written in the index space of
// the grid as minor = X0 + kappa * major, with "vertical" lines
// (|sin| >= |cos|, the case split of Section II-B) taking rows as the major
// direction and horizontal ones columns; |kappa| <= 1.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define XRT_HD __host__ __device__
#else
#define XRT_HD
#endif

namespace xrt {

// Adjoint tile (pixels): kTileI columns (x1) by kTileJ rows (x2) for the
// vertical lines, and the transposed tile for the horizontal ones (kTileI
// across the lines either way).  64 x 32 measured fastest among 16..128-pixel
// tile sides on the 2048^2 cubic workload.
#ifndef XRT_TILE_I
#define XRT_TILE_I 64
#endif
#ifndef XRT_TILE_J
#define XRT_TILE_J 32
#endif
constexpr int kTileI = XRT_TILE_I;
constexpr int kTileJ = XRT_TILE_J;
// Halo (cells) of the LDS accumulators of the adjoint on each minor side:
// with crossings kept within n+1 cells of the tile, taps and knot slots stay
// within 7 cells (degree 3) of it.
constexpr int kHalo = 8;
// Accumulator pitch: the tile's kTileI columns across the lines plus halos,
// odd so that the rows the lanes of a wave update fall into different LDS
// banks.
constexpr int kAccPitch = kTileI + 2 * kHalo + 1;

struct GridGeom {
    int nx, ny;
    double h, cx, cy;
};

struct Canon {
    double xc;   // crossing at the centre major index
    double kap;  // slope
    int cls;     // 0 vertical, 1 horizontal, 2 misses the padded grid
    int bad;     // degenerate / non-finite input
};

// (cos t, sin t, y) in world coordinates -> crossing form in index space.
// A line is kept (cls 0 or 1) when the band of half-width
// (n+1)(1 + |kappa|)/2 around its crossings reaches the grid's centres.
XRT_HD inline Canon canon_core(double c, double s, double yw, const GridGeom& g, int degree, int bad)
{
    Canon o;
    o.bad = bad;
    // i*s - j*c = Y in index space
    const double ox = 0.5 * (g.nx - 1), oy = 0.5 * (g.ny - 1);
    const double Y = (yw - (g.cx * s - g.cy * c)) / g.h + ox * s - oy * c;
    const bool vert = fabs(s) >= fabs(c);
    const int nmaj = vert ? g.ny : g.nx, nmin = vert ? g.nx : g.ny;
    double X0, kap;
    if (vert) {
        X0 = Y / s;
        kap = c / s;
    } else {
        X0 = -Y / c;
        kap = s / c;
    }
    const double jc = 0.5 * (nmaj - 1);
    o.xc = X0 + kap * jc;
    o.kap = kap;
    // rows whose band reaches the grid: -W < X(j) < nmin - 1 + W
    const double W = 0.5 * (degree + 1) * (1.0 + fabs(kap));
    bool hit;
    if (kap == 0.0) {
        hit = X0 > -W && X0 < nmin - 1 + W;
    } else {
        double a = (-W - X0) / kap, b = (nmin - 1 + W - X0) / kap;
        double lo = fmin(a, b), hi = fmax(a, b);
        hit = hi > 0.0 && lo < (double)(nmaj - 1);
    }
    o.cls = o.bad ? 2 : (hit ? (vert ? 0 : 1) : 2);
    return o;
}

// Rows [jlo, jhi] (closed) of a line whose band may reach the grid.
// inv = 1/kap (unused when kap = 0); a product with it instead of a
// quotient moves the bounds by ~1e-16 relative, far inside the 1e-9 slack
XRT_HD inline void row_range(double x0, double kap, double inv, double W, int nmaj, int nmin, int* jlo, int* jhi)
{
    if (kap == 0.0) {
        *jlo = 0;
        *jhi = nmaj - 1;
        return;
    }
    double a = (-W - x0) * inv, b = (nmin - 1 + W - x0) * inv;
    double lo = fmin(a, b), hi = fmax(a, b);
    double flo = ceil(lo - 1e-9), fhi = floor(hi + 1e-9);
    // clamped to [-1, nmaj] before the conversion (a nearly axis-parallel
    // line can put the bounds far outside the int range)
    *jlo = (int)fmin(fmax(0.0, flo), (double)nmaj);
    *jhi = (int)fmax(fmin((double)(nmaj - 1), fhi), -1.0);
}

// Rows [ra, rb] of a line that an adjoint tile walks: the rows of the tile
// (major [maj0, maj0 + TM)) whose crossing X(j) = x0 + kappa j lies within
// ml of the tile's minor range [min0, min0 + TN - 1], and inside the rows
// whose band reaches the grid.  ra > rb: nothing to walk.  x0 is the
// crossing at major index 0.
struct AdjRows {
    int ra, rb;
    double x0;
};

XRT_HD inline AdjRows adj_rows(double xc, double kap, double jc, double ml, int nmaj, int nmin, int maj0, int min0,
                               int TM, int TN)
{
    AdjRows r;
    r.x0 = xc - kap * jc;
    const double inv = 1.0 / kap;
    int jlo, jhi;
    row_range(r.x0, kap, inv, ml, nmaj, nmin, &jlo, &jhi);
    r.ra = jlo > maj0 ? jlo : maj0;
    r.rb = jhi < maj0 + TM - 1 ? jhi : maj0 + TM - 1;
    if (kap != 0.0) {
        double a = (min0 - ml - r.x0) * inv, b = (min0 + TN - 1 + ml - r.x0) * inv;
        double lo2 = fmin(a, b), hi2 = fmax(a, b);
        const int c0 = (int)fmin(fmax(ceil(lo2 - 1e-9), -1.0e9), 1.0e9);
        const int c1 = (int)fmin(fmax(floor(hi2 + 1e-9), -1.0e9), 1.0e9);
        r.ra = r.ra > c0 ? r.ra : c0;
        r.rb = r.rb < c1 ? r.rb : c1;
    } else if (!(r.x0 >= min0 - ml && r.x0 <= min0 + TN - 1 + ml)) {
        r.rb = r.ra - 1;
    }
    return r;
}

// Column coordinate of a line's crossing of tile row ra within the
// accumulator row (halo included), shifted by H = (n+1)/2 for the B-splines
// (so that floor(q) is the last tap J) and by 0 for the box spline.
XRT_HD inline double adj_q0(double x0, double kap, int ra, int min0, double H)
{
    return x0 + kap * (double)ra + H - (double)min0 + (double)kHalo;
}

// Fraction of q > 0 (exact in FP64).
XRT_HD inline double frac_pos(double q)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_fract(q);
#else
    return q - floor(q);
#endif
}

XRT_HD inline uint32_t mul24(uint32_t a, uint32_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul24(a, b);
#else
    return (a & 0xffffffu) * (b & 0xffffffu);
#endif
}

// Offset o of the first of the S knot slots of a row from J = floor(q),
// q = X + (n+1)/2: the S knots nearest to q, centred on round(q) for odd S
// (up: the fraction of q is at least 1/2) and on q for even S.
template <int S>
XRT_HD constexpr int knot_o(bool up)
{
    if constexpr (S % 2 == 0) {
        return 1 - S / 2;
    } else {
        return (up ? 1 : 0) - (S - 1) / 2;
    }
}

// First knot slot of a row relative to its first tap J - n.
template <int N, int S>
XRT_HD inline int adj_knot_offset(bool up)
{
    return knot_o<S>(up) + N;
}

// Start row (0 .. cnt-1) of the lane's walk over its cnt rows: lanes of a
// wave start at rows spread by a multiply and shift of the scrambled lane
// index (M l mod 64), so that neighbouring lanes, which hold neighbouring
// lines, rarely update the same LDS word in one instruction.  M = 19 for the
// B-splines: a simulation of the 2048^2 benchmark tiles' LDS address streams
// (the plan's candidate order, every atomic's address, the cost per
// half-wave measured with xrt_calib_lds) gave 5.66 cycles per atomic with
// 19 against 6.00 with 37 (and 5.6-6.7 over 100 multiplier and pitch pairs);
// the cubic adjoint went from 22.2 to 21.6 ms.  Neighbouring rows for
// neighbouring lanes (l cnt / 64) took a third longer.
template <unsigned M>
XRT_HD inline int adj_start_row(unsigned lane, int cnt)
{
    return (int)((((lane * M) & 63u) * (unsigned)cnt) >> 6);
}

// the multiplier (also for the box spline's rows: 10.75 -> 10.62 ms with 19)
constexpr unsigned kAdjSpread = 19u;

// The adjoint walks a line's rows in 32.32 fixed point: Q(jj) = Q0 + jj Kq
// with Q0 = round((q - n) 2^32) at the line's first row in the tile and
// Kq = round(kappa 2^32), so that floor(q - n) (the first tap's column) is
// the high word and the fraction the low word.  Consecutive rows differ by
// one 32-bit add with carry into the accumulator address; the rounding of
// Q0 and Kq moves a row's position by at most (1 + jj) 2^-33 cells.
struct AdjFix {
    int64_t Q0;    // fixed-point q - n at tile row row0 (jj = 0)
    int64_t Kq;    // fixed-point slope
    uint32_t Kf;   // low word of Kq (fraction step)
    uint32_t Wk;   // W + high word of Kq: address step before the carry
    int row0, W;
};

XRT_HD inline AdjFix adj_fix(double qn, double kap, int row0, int W)
{
    AdjFix f;
    f.Q0 = (int64_t)rint(qn * 4294967296.0);
    f.Kq = (int64_t)rint(kap * 4294967296.0);
    f.Kf = (uint32_t)f.Kq;
    f.Wk = (uint32_t)W + (uint32_t)(int32_t)(f.Kq >> 32);
    f.row0 = row0;
    f.W = W;
    return f;
}

// Row jj of the walk: its fraction (low word) and the accumulator word of its
// first tap, row (row0 + jj) times the pitch W plus floor(q - n).
struct AdjStep {
    uint32_t tf;
    uint32_t base;
};

XRT_HD inline AdjStep adj_fix_at(const AdjFix& f, int jj)
{
    const int64_t Q = f.Q0 + (int64_t)jj * f.Kq;
    AdjStep st;
    st.tf = (uint32_t)Q;
    st.base = mul24((uint32_t)(f.row0 + jj), (uint32_t)f.W) + (uint32_t)(int32_t)(Q >> 32);
    return st;
}

// Row jj -> jj + 1 (exact: equals adj_fix_at(f, jj + 1)).
XRT_HD inline void adj_fix_next(const AdjFix& f, AdjStep& st)
{
    const uint32_t tn = st.tf + f.Kf;
    st.base += f.Wk + (tn < st.tf ? 1u : 0u);
    st.tf = tn;
}

// Accumulator word of a row's first tap: row (within the tile) times the
// pitch W, plus the tap's column (floor(q) - n for the B-splines, where
// q - n > 0 on every row a line walks, so that truncation is the floor).
XRT_HD inline uint32_t adj_tap_base(int row, int W, int col)
{
    return mul24((uint32_t)row, (uint32_t)W) + (uint32_t)col;
}

}  // namespace xrt
