// Host replay of the adjoint's LDS index arithmetic (test infrastructure).
//
// For random lines on several grids, every (pixel tile, line) pair of both
// adjoint passes goes through the same functions the kernels use
// (canon_core, adj_rows, adj_q0, the fixed-point walk adj_fix / adj_fix_at /
// adj_fix_next, adj_start_row, adj_tap_base, adj_knot_offset, from
// xrt_geom.h), and every
// accumulator word a row would update is checked to lie inside its own
// accumulator row: taps and knot slots in [0, W) of row (row0 + jj), rows in
// [0, TM).  The walk must visit every row once, wrap and end on the
// addresses it tests for, and each step must equal the direct evaluation.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer (float-to-int overflow included) by
// tests/test_sanitizers.py.  Exit status 0: every address in bounds.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "xrt_geom.h"

using namespace xrt;

static long long g_rows = 0, g_pairs = 0, g_fail = 0;

static void fail(const char* what, int n, double xc, double kap, int maj0, int min0, int row, int col)
{
    if (g_fail++ < 20)
        fprintf(stderr, "OUT OF BOUNDS %s: degree %d xc %.17g kap %.17g tile (%d, %d) row %d col %d\n", what, n, xc,
                kap, maj0, min0, row, col);
}

// One line on one tile, for every slot count S a wave may use (the wave's S
// is the largest of its lines' counts, so any S from 1 to n+1).
template <int N, int S>
static void walk_bspline(double xc, double kap, const AdjRows& rr, int maj0, int min0, int TM, int W)
{
    const double H = 0.5 * (N + 1);
    const double q0 = adj_q0(rr.x0, kap, rr.ra, min0, H);
    const int cnt = rr.rb - rr.ra + 1, row0 = rr.ra - maj0;
    // the kernel's fixed-point walk: rows jj0 .. cnt-1, then back to row 0
    // and on to jj0-1, for start rows jj0 of several lanes
    const AdjFix F = adj_fix(q0 - (double)N, kap, row0, W);
    const uint32_t end = adj_fix_at(F, cnt).base;
    for (int lane = 0; lane < 64; lane += 7) {
        const int jj0 = adj_start_row<kAdjSpread>((unsigned)lane, cnt);
        AdjStep st = adj_fix_at(F, jj0);
        const uint32_t mid = st.base;
        int jj = jj0, steps = 0;
        auto visit = [&](const AdjStep& a, int j) {
            const int row = row0 + j;
            if (row < 0 || row >= TM) fail("row", N, xc, kap, maj0, min0, row, 0);
            const uint32_t lo = (uint32_t)row * (uint32_t)W, hi = lo + (uint32_t)W;
            // the step must equal the direct evaluation at this row
            const AdjStep d = adj_fix_at(F, j);
            if (d.base != a.base || d.tf != a.tf) fail("step", N, xc, kap, maj0, min0, row, 0);
            const bool up = (float)a.tf * 0x1p-32f >= 0.5f;
            for (int t = 0; t <= N; ++t)
                if (a.base + t < lo || a.base + t >= hi) fail("tap", N, xc, kap, maj0, min0, row, (int)(a.base + t - lo));
            const uint32_t kb = a.base + (uint32_t)adj_knot_offset<N, S>(up);
            for (int sl = 0; sl < S; ++sl)
                if (kb + sl < lo || kb + sl >= hi) fail("knot", N, xc, kap, maj0, min0, row, (int)(kb + sl - lo));
            ++g_rows;
        };
        const AdjStep st0 = adj_fix_at(F, 0);
        do {
            visit(st, jj);
            adj_fix_next(F, st);
            ++jj;
            if (st.base == end) {
                if (jj != cnt) fail("wrap row", N, xc, kap, maj0, min0, jj, cnt);
                st = st0;
                jj = 0;
            }
            if (++steps > TM + 1) { fail("no end", N, xc, kap, maj0, min0, jj, 0); break; }
        } while (st.base != mid);
        if (steps != cnt) fail("row count", N, xc, kap, maj0, min0, steps, cnt);
        if (jj != jj0) fail("end row", N, xc, kap, maj0, min0, jj, jj0);
    }
}

template <int N>
static void line_tile(double xc, double kap, int nmaj, int nmin, int maj0, int min0, int TM, int TN)
{
    const int W = TN + 2 * kHalo + 1;
    const double jc = 0.5 * (nmaj - 1);
    const double H = 0.5 * (N + 1);
    const AdjRows rr = adj_rows(xc, kap, jc, H * (1.0 + fabs(kap)), nmaj, nmin, maj0, min0, TM, TN);
    ++g_pairs;
    if (rr.ra > rr.rb) return;
    walk_bspline<N, 1>(xc, kap, rr, maj0, min0, TM, W);
    if constexpr (N >= 1) walk_bspline<N, 2>(xc, kap, rr, maj0, min0, TM, W);
    if constexpr (N >= 2) walk_bspline<N, 3>(xc, kap, rr, maj0, min0, TM, W);
    if constexpr (N >= 3) walk_bspline<N, 4>(xc, kap, rr, maj0, min0, TM, W);
}

// box spline: columns floor(q) - 1 .. floor(q) + 2 of each row
static void line_tile_box(double xc, double kap, int nmaj, int nmin, int maj0, int min0, int TM, int TN)
{
    const int W = TN + 2 * kHalo + 1;
    const double jc = 0.5 * (nmaj - 1);
    const double ml = kap >= 0.0 ? 1.0 : 1.0 - kap;
    const AdjRows rr = adj_rows(xc, kap, jc, ml, nmaj, nmin, maj0, min0, TM, TN);
    ++g_pairs;
    if (rr.ra > rr.rb) return;
    const double q0 = adj_q0(rr.x0, kap, rr.ra, min0, 0.0);
    const int cnt = rr.rb - rr.ra + 1, row0 = rr.ra - maj0;
    // the kernel's walk on q - 1: base = row W + floor(q) - 1
    const AdjFix F = adj_fix(q0 - 1.0, kap, row0, W);
    const uint32_t end = adj_fix_at(F, cnt).base;
    for (int lane = 0; lane < 64; lane += 7) {
        const int jj0 = adj_start_row<kAdjSpread>((unsigned)lane, cnt);
        AdjStep st = adj_fix_at(F, jj0);
        const AdjStep st0 = adj_fix_at(F, 0);
        const uint32_t mid = st.base;
        int jj = jj0, steps = 0;
        do {
            const int row = row0 + jj;
            if (row < 0 || row >= TM) fail("row", 16, xc, kap, maj0, min0, row, 0);
            const uint32_t lo = (uint32_t)row * (uint32_t)W, hi = lo + (uint32_t)W;
            for (int d = 0; d < 4; ++d)
                if (st.base + d < lo || st.base + d >= hi)
                    fail("box column", 16, xc, kap, maj0, min0, row, (int)(st.base + d - lo));
            ++g_rows;
            adj_fix_next(F, st);
            ++jj;
            if (st.base == end) {
                st = st0;
                jj = 0;
            }
            if (++steps > TM + 1) { fail("no end", 16, xc, kap, maj0, min0, jj, 0); break; }
        } while (st.base != mid);
        if (steps != cnt) fail("row count", 16, xc, kap, maj0, min0, steps, cnt);
    }
}

static void line_all_tiles(int n, double xc, double kap, bool vert, int nx, int ny, std::mt19937_64& rng)
{
    // the tiles of this line's pass: kTileI across the lines, kTileJ along
    const int TM = kTileJ, TN = kTileI;
    const int nmaj = vert ? ny : nx, nmin = vert ? nx : ny;
    const int tmaj = (nmaj + TM - 1) / TM, tmin = (nmin + TN - 1) / TN;
    const double jc = 0.5 * (nmaj - 1);
    for (int a = 0; a < tmaj; ++a) {
        const int maj0 = a * TM;
        int b0 = 0, b1 = tmin - 1;
        if ((long long)tmaj * tmin > 64) {
            // large grids: the tiles within two of those the line crosses
            const double x0 = xc - kap * jc;
            const double X1 = x0 + kap * maj0, X2 = x0 + kap * (maj0 + TM - 1);
            const double lo = fmin(X1, X2) - 6.0, hi = fmax(X1, X2) + 6.0;
            b0 = (int)fmax(floor(lo / TN) - 2.0, 0.0);
            b1 = (int)fmin(floor(hi / TN) + 2.0, (double)(tmin - 1));
            if (rng() % 8 == 0) b0 = b1 = (int)(rng() % (uint64_t)tmin);  // and a random one
        }
        for (int b = b0; b <= b1; ++b) {
            const int min0 = b * TN;
            switch (n) {
            case 0: line_tile<0>(xc, kap, nmaj, nmin, maj0, min0, TM, TN); break;
            case 1: line_tile<1>(xc, kap, nmaj, nmin, maj0, min0, TM, TN); break;
            case 2: line_tile<2>(xc, kap, nmaj, nmin, maj0, min0, TM, TN); break;
            case 3: line_tile<3>(xc, kap, nmaj, nmin, maj0, min0, TM, TN); break;
            default: line_tile_box(xc, kap, nmaj, nmin, maj0, min0, TM, TN); break;
            }
        }
    }
}

int main()
{
    std::mt19937_64 rng(20250);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    struct G { int nx, ny, lines; };
    const G grids[] = {{1, 1, 400}, {1, 37, 400}, {53, 1, 400}, {65, 64, 2000}, {150, 97, 2000},
                       {200, 230, 1500}, {2048, 2048, 300}, {4097, 3, 200}, {3, 4097, 200}};
    const int bases[] = {0, 1, 2, 3, 16};
    for (const G& gr : grids) {
        GridGeom g{gr.nx, gr.ny, 1.0, 0.0, 0.0};
        const double R = 0.75 * (gr.nx > gr.ny ? gr.nx : gr.ny) + 4.0;
        for (int bi = 0; bi < 5; ++bi) {
            const int n = bases[bi];
            const int gd = n == 16 ? 1 : n;  // the box spline's plans use the degree-1 margins
            for (int l = 0; l < gr.lines; ++l) {
                double t = U(rng) * 3.0 * M_PI - M_PI, y = (2.0 * U(rng) - 1.0) * R;
                // special directions and offsets: axes, diagonals, grazing the margin
                switch (l % 16) {
                case 0: t = 0.0; break;
                case 1: t = M_PI / 2; break;
                case 2: t = M_PI / 4; break;
                case 3: t = -M_PI / 4; break;
                case 4: t = (double)(float)(M_PI / 2); break;
                case 5: t = 1e-7; break;
                case 6: y = 0.5 * (gr.ny - 1) + 0.5 * (gd + 1) - 1e-9; t = 0.0; break;
                case 7: y = -(0.5 * (gr.nx - 1) + 0.5 * (gd + 1)) + 1e-9; t = M_PI / 2; break;
                default: break;
                }
                const float tf = (float)t, yf = (float)y;
                double s, c;
                s = sin((double)tf);
                c = cos((double)tf);
                const Canon o = canon_core(c, s, (double)yf, g, gd, 0);
                if (o.cls == 2) continue;
                line_all_tiles(n, o.xc, o.kap, o.cls == 0, gr.nx, gr.ny, rng);
            }
        }
    }
    // slopes at and next to their limits, crossings at the margins of tiles
    for (int l = 0; l < 20000; ++l) {
        const int nx = 150, ny = 97;
        const bool vert = l % 2 == 0;
        const int nmin = vert ? nx : ny;
        double kap;
        switch (l % 6) {
        case 0: kap = 1.0; break;
        case 1: kap = -1.0; break;
        case 2: kap = 0.0; break;
        case 3: kap = (U(rng) - 0.5) * 1e-12; break;
        default: kap = 2.0 * U(rng) - 1.0; break;
        }
        const double xc = (U(rng) * 1.2 - 0.1) * nmin + (U(rng) - 0.5) * 1e-9;
        for (int n : bases) line_all_tiles(n, xc, kap, vert, nx, ny, rng);
    }
    // crossings placed at the very edge of what a tile accepts: for a tile,
    // a row of it and a slope, X(row) = min0 - ml + d or min0 + TN - 1 + ml - d
    // with ml the basis' half-width (n+1)(1 + |kappa|)/2 (box: 1 or 1 + |kappa|)
    // and d from 0 to 1e-6
    {
        const int nx = 330, ny = 290;
        const double ds[] = {0.0, 1e-15, 1e-12, 1e-9, 1e-6};
        for (int l = 0; l < 40000; ++l) {
            const bool vert = l % 2 == 0;
            const int nmaj = vert ? ny : nx, nmin = vert ? nx : ny;
            const int TM = kTileJ, TN = kTileI;
            const int n = bases[(l / 2) % 5];
            double kap;
            switch ((l / 10) % 5) {
            case 0: kap = 1.0; break;
            case 1: kap = -1.0; break;
            case 2: kap = 1.0 - 1e-12; break;
            case 3: kap = 0.0; break;
            default: kap = 2.0 * U(rng) - 1.0; break;
            }
            const int tmaj = (nmaj + TM - 1) / TM, tmin = (nmin + TN - 1) / TN;
            const int maj0 = (int)(rng() % (uint64_t)tmaj) * TM, min0 = (int)(rng() % (uint64_t)tmin) * TN;
            const int jr = maj0 + (int)(rng() % (uint64_t)TM);
            const double ml = n == 16 ? (kap >= 0.0 ? 1.0 : 1.0 - kap) : 0.5 * (n + 1) * (1.0 + fabs(kap));
            const double d = ds[rng() % 5];
            const double X = (l / 50) % 2 == 0 ? min0 - ml + d : min0 + TN - 1 + ml - d;
            const double jc = 0.5 * (nmaj - 1);
            const double xc = X + kap * (jc - jr);
            switch (n) {
            case 0: line_tile<0>(xc, kap, nmaj, nmin, maj0, min0, TM, TN); break;
            case 1: line_tile<1>(xc, kap, nmaj, nmin, maj0, min0, TM, TN); break;
            case 2: line_tile<2>(xc, kap, nmaj, nmin, maj0, min0, TM, TN); break;
            case 3: line_tile<3>(xc, kap, nmaj, nmin, maj0, min0, TM, TN); break;
            default: line_tile_box(xc, kap, nmaj, nmin, maj0, min0, TM, TN); break;
            }
        }
    }
    printf("pairs %lld rows %lld failures %lld\n", g_pairs, g_rows, g_fail);
    return g_fail == 0 ? 0 : 1;
}
