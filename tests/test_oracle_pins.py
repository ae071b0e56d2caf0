"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own formula: each compares the oracle with
an independent computation (geometry, a library B-spline or quadrature, the
paper's printed formula, a closed form or an invariant).  A plausible mistake
in the oracle (dropped term, wrong sign, transposed operand, wrong grid origin
or orientation) fails at least one of them.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.interpolate import BSpline

import xrt_workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def scipy_beta(n):
    """Centred cardinal B-spline of degree n from scipy (a library routine)."""
    knots = np.arange(n + 2) - (n + 1) / 2.0
    b = BSpline.basis_element(knots, extrapolate=False)
    return lambda x: np.nan_to_num(b(np.asarray(x, dtype=np.float64)))


# ------------------------------------------------------------------ B-splines
def test_bspline_textbook_values(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "bspline_textbook.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) >= 12
    for n, x, v in rows:
        n, x, v = int(n), float(x), float(Fraction(v))
        for xx in (x, -x):
            assert orc.bspline(n, xx)[0] == pytest.approx(v, abs=1e-15)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_bspline_matches_scipy(orc, n):
    x = np.linspace(-2.7, 2.7, 541)
    x = x[np.abs(np.abs(x) - 0.5) > 1e-9] if n == 0 else x
    np.testing.assert_allclose(orc.bspline(n, x), scipy_beta(n)(x), atol=1e-14)


# ------------------------------------------------------------- footprints
def square_chord(theta, u):
    """Length of the line {t theta + u theta_perp} inside [-1/2,1/2]^2
    (Liang-Barsky clipping)."""
    c, s = math.cos(theta), math.sin(theta)
    p0 = np.array([u * s, -u * c])
    d = np.array([c, s])
    t0, t1 = -1e9, 1e9
    for k in range(2):
        if abs(d[k]) < 1e-300:
            if abs(p0[k]) > 0.5:
                return 0.0
            continue
        a = (-0.5 - p0[k]) / d[k]
        b = (0.5 - p0[k]) / d[k]
        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
    return max(0.0, t1 - t0)


def test_degree0_is_pixel_chord(orc):
    """P1: the degree-0 footprint is the intersection length of the line with
    one pixel (Siddon's quantity, Section II-A/II-B)."""
    rng = np.random.default_rng(11)
    for _ in range(400):
        th = rng.uniform(0, 2 * math.pi)
        u = rng.uniform(-0.8, 0.8)
        assert orc.footprint(0, th, u)[0] == pytest.approx(square_chord(th, u), abs=1e-12)


def test_degree1_printed_formula(orc):
    """P2: the formula printed in Section III-C equals the oracle's degree-1
    footprint once y is measured from the left end of the support."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "degree1_printed.txt"))
            if l.strip() and not l.startswith("#")]
    terms = [(float(c), int(p), int(q)) for c, p, q in rows]
    assert len(terms) == 9
    rng = np.random.default_rng(12)
    for _ in range(60):
        th = rng.uniform(0.15, math.pi / 2 - 0.15)
        a1, a2 = abs(math.cos(th)), abs(math.sin(th))
        for u in rng.uniform(-(a1 + a2) * 1.1, (a1 + a2) * 1.1, size=7):
            y = u + a1 + a2
            val = sum(c * max(y - (p * a1 + q * a2), 0.0) ** 3 for c, p, q in terms)
            val /= 6.0 * a1 * a1 * a2 * a2
            assert orc.footprint(1, th, u)[0] == pytest.approx(val, abs=1e-12)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_axis_aligned_limit_is_bspline(orc, n):
    """P3: at theta = 0 (and near it) phi_theta = beta^n (the Dirac case of
    Proposition 1).  Near 0 the quadrature path must agree with scipy's
    B-spline away from the knots (distance >> sin theta)."""
    B = scipy_beta(n)
    u = np.linspace(-2.3, 2.3, 233)
    knots = np.arange(n + 2) - (n + 1) / 2.0
    for th in (0.0, 1e-7, -3e-6, math.pi / 2 + 2e-7):
        b = abs(math.sin(th)) if abs(math.sin(th)) < 0.5 else abs(math.cos(th))
        far = np.min(np.abs(u[:, None] - knots[None, :]), axis=1) > max(10 * b, 1e-12)
        f = orc.footprint(n, th, u[far])
        ref = B(u[far] / max(abs(math.cos(th)), abs(math.sin(th))))
        np.testing.assert_allclose(f, ref, atol=1e-9)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_diagonal_is_dilated_bspline(orc, n):
    """P4: at theta = pi/4 both factors are beta^n(sqrt2 .)sqrt2, whose
    convolution is sqrt2 beta^{2n+1}(sqrt2 u)."""
    B = scipy_beta(2 * n + 1)
    u = np.linspace(-3.0, 3.0, 301)
    th = math.pi / 4
    np.testing.assert_allclose(orc.footprint(n, th, u),
                               math.sqrt(2) * B(math.sqrt(2) * u), atol=1e-12)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_footprint_mass_parity_symmetry(orc, n):
    """P5: int phi_theta = 1, phi_theta even, invariant under
    theta -> -theta, theta + pi/2, pi - theta."""
    for th in (0.05, 0.31, 0.7853, 1.1, 2.9):
        c, s = abs(math.cos(th)), abs(math.sin(th))
        w = (n + 1) * (c + s) / 2
        pts = sorted({i * c + j * s - w for i in range(n + 2) for j in range(n + 2)})
        pts = [p for p in pts if -w < p < w]
        mass = quad(lambda v: orc.footprint(n, th, v)[0], -w, w, points=pts, limit=200,
                    epsabs=1e-13)[0]
        assert mass == pytest.approx(1.0, abs=1e-10)
        u = np.linspace(-w * 1.05, w * 1.05, 41)
        f = orc.footprint(n, th, u)
        np.testing.assert_allclose(f, orc.footprint(n, th, -u), atol=1e-10)
        for th2 in (-th, th + math.pi / 2, math.pi - th):
            np.testing.assert_allclose(f, orc.footprint(n, th2, u), atol=1e-10)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_closed_form_matches_quadrature(orc, n):
    """P6: the truncated-power closed form and the knot-split Gauss-Legendre
    path are independent evaluations of eq. (6); they agree where the closed
    form is well conditioned."""
    rng = np.random.default_rng(13 + n)
    for _ in range(200):
        th = rng.uniform(0, 2 * math.pi)
        c, s = math.cos(th), math.sin(th)
        if min(abs(c), abs(s)) < 0.1:
            continue
        u = rng.uniform(-(n + 1), n + 1)
        tp = orc.footprint(n, th, u, "tp")[0]
        gl = orc.footprint(n, th, u, "gl")[0]
        assert tp == pytest.approx(gl, abs=1e-9)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_quadrature_path_vs_adaptive_quadrature(orc, n):
    """The Gauss-Legendre path at small min(|cos|,|sin|), against scipy's
    adaptive quadrature of the same convolution integral of eq. (6)."""
    B = scipy_beta(n)
    hw = (n + 1) / 2
    for b in (0.07, 1e-3, 1e-5):
        a = math.sqrt(1 - b * b)
        th = math.atan2(b, a)
        for u in (-1.7, -0.5001, 0.0, 0.3, 1.234, hw * (a + b) - 1e-3):
            def integrand(v):
                return float(B(v)) * float(B((u - b * v) / a)) / a
            brk = sorted({k - hw for k in range(n + 2)} |
                         {(u - a * (k - hw)) / b for k in range(n + 2)
                          if -hw < (u - a * (k - hw)) / b < hw})
            ref = quad(integrand, -hw, hw, points=brk, limit=400, epsabs=1e-14,
                       epsrel=1e-12)[0]
            assert orc.footprint(n, th, u, "gl")[0] == pytest.approx(ref, abs=1e-11)


# --------------------------------------------------------------- operator
def line_integral_bruteforce(n, coeffs, th, y, spacing=1.0, cx=0.0, cy=0.0):
    """P_theta{f}(y) = int f(t theta + y theta_perp) dt (eq. (2)) with f from
    eq. (3) evaluated directly (scipy B-splines) and scipy's adaptive
    quadrature between consecutive knot-line crossings."""
    ny, nx = coeffs.shape
    B = scipy_beta(n)
    hw = (n + 1) / 2
    c, s = math.cos(th), math.sin(th)
    xs = cx + (np.arange(nx) - (nx - 1) / 2) * spacing
    ys = cy + (np.arange(ny) - (ny - 1) / 2) * spacing

    def f(t):
        x1 = t * c + y * s
        x2 = t * s - y * c
        bx = B((x1 - xs) / spacing)
        by = B((x2 - ys) / spacing)
        return float(by @ coeffs @ bx)

    # crossings with every knot line x1 = xs + k*h, x2 = ys + k*h
    R = (max(nx, ny) / 2 + hw + 2) * spacing * 1.5 + abs(cx) + abs(cy)
    tb = [-R - abs(y), R + abs(y)]
    kn = np.arange(-(n + 1), n + 2) * 0.5 * spacing
    for k1 in np.unique((xs[:, None] + kn[None, :]).ravel()):
        if abs(c) > 1e-14:
            tb.append((k1 - y * s) / c)
    for k2 in np.unique((ys[:, None] + kn[None, :]).ravel()):
        if abs(s) > 1e-14:
            tb.append((k2 + y * c) / s)
    tb = np.unique(np.clip(tb, tb[0], tb[1]))
    tot = 0.0
    for a, b in zip(tb[:-1], tb[1:]):
        if b - a > 1e-13:
            tot += quad(f, a, b, epsabs=1e-13, epsrel=1e-12, limit=100)[0]
    return tot


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_forward_vs_bruteforce_line_integral(orc, n):
    """P7: the banded FP64 forward equals the line integral of the continuous
    image of eq. (3) on tiny grids, including lines that only graze the
    margin beyond the outer cells."""
    rng = np.random.default_rng(20 + n)
    coeffs = rng.normal(size=(5, 6))
    th = rng.uniform(0, 2 * math.pi, size=10)
    y = rng.uniform(-5.5, 5.5, size=10)
    th = np.append(th, [0.0, math.pi / 2, math.pi / 4]).astype(np.float32)
    y = np.append(y, [0.4, -1.3, 2.2]).astype(np.float32)
    lines = orc.lines_from_theta_y(th, y)
    got = orc.forward(n, coeffs, lines)
    for k in range(th.size):
        if n == 0 and (abs(math.sin(th[k])) < 1e-6 or abs(math.cos(th[k])) < 1e-6):
            continue  # quadrature cannot resolve the degree-0 jump on a cell edge
        ref = line_integral_bruteforce(n, coeffs, float(th[k]), float(y[k]))
        assert got[k] == pytest.approx(ref, abs=2e-9 * (1 + abs(ref)))


def test_forward_vs_bruteforce_spacing_and_centre(orc):
    """P7 with a non-unit spacing and an offset grid centre."""
    rng = np.random.default_rng(31)
    coeffs = rng.normal(size=(4, 5))
    th = rng.uniform(0, 2 * math.pi, size=8).astype(np.float32)
    y = rng.uniform(-4, 4, size=8).astype(np.float32)
    lines = orc.lines_from_theta_y(th, y)
    for n in (1, 3):
        got = orc.forward(n, coeffs, lines, spacing=0.7, cx=0.3, cy=-0.45)
        for k in range(8):
            ref = line_integral_bruteforce(n, coeffs, float(th[k]), float(y[k]), 0.7, 0.3, -0.45)
            assert got[k] == pytest.approx(ref, abs=2e-9 * (1 + abs(ref)))


def square_chord_len(th, y, half):
    """Chord of the line (th, y) through the square [-half, half]^2."""
    return square_chord(th, y / (2 * half)) * 2 * half


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_partition_of_unity_chord(orc, n):
    """P8: c = 1 on an N x N grid projects to the chord of the square of side
    N wherever y is at least n(a+b)/2 away from the projections of its four
    corners (the image is the square's indicator smoothed by a symmetric
    unit-mass kernel)."""
    N = 12
    coeffs = np.ones((N, N))
    rng = np.random.default_rng(40 + n)
    th = rng.uniform(0, math.pi, size=300)
    y = rng.uniform(-9, 9, size=300)
    th32, y32 = th.astype(np.float32), y.astype(np.float32)
    lines = orc.lines_from_theta_y(th32, y32)
    got = orc.forward(n, coeffs, lines)
    checked = 0
    for k in range(300):
        t, yy = float(th32[k]), float(y32[k])
        c, s = math.cos(t), math.sin(t)
        corners = [sx * N / 2 * s - sy * N / 2 * c for sx in (-1, 1) for sy in (-1, 1)]
        margin = min(abs(yy - p) for p in corners) - n * (abs(c) + abs(s)) / 2
        if margin <= 1e-6:
            continue
        checked += 1
        assert got[k] == pytest.approx(square_chord_len(t, yy, N / 2), abs=1e-10)
    assert checked > 100


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_single_coefficient(orc, n):
    """P9: c = delta_k gives s_m = phi(y_m - <x_k, theta_perp>) (eq. (4)), with
    x_k at (i - (nx-1)/2, j - (ny-1)/2), column i along x1, row j along x2."""
    nx, ny = 7, 5
    i, j = 5, 1
    coeffs = np.zeros((ny, nx))
    coeffs[j, i] = 1.0
    rng = np.random.default_rng(50 + n)
    th = rng.uniform(0, 2 * math.pi, size=50).astype(np.float32)
    y = rng.uniform(-4, 4, size=50).astype(np.float32)
    got = orc.forward(n, coeffs, orc.lines_from_theta_y(th, y))
    x1, x2 = i - (nx - 1) / 2, j - (ny - 1) / 2
    for k in range(50):
        t = float(th[k])
        u = float(y[k]) - (x1 * math.sin(t) - x2 * math.cos(t))
        assert got[k] == pytest.approx(orc.footprint(n, t, u)[0], abs=1e-14)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_adjoint_identity(orc, n):
    """P10: <H c, s> = <c, H^T s> (the matched back-projection, Section II-B)."""
    rng = np.random.default_rng(60 + n)
    nx, ny = 23, 17
    c = rng.normal(size=(ny, nx))
    th = rng.uniform(0, 2 * math.pi, size=400).astype(np.float32)
    y = rng.uniform(-16, 16, size=400).astype(np.float32)
    L = orc.lines_from_theta_y(th, y)
    s = rng.normal(size=400)
    Hc = orc.forward(n, c, L, spacing=1.3, cx=0.2)
    Hts = orc.adjoint(n, s, L, nx, ny, spacing=1.3, cx=0.2)
    lhs, rhs = float(Hc @ s), float(np.sum(c * Hts))
    assert lhs == pytest.approx(rhs, rel=1e-13, abs=1e-12)


def test_adjoint_pixels_matches_adjoint(orc):
    rng = np.random.default_rng(61)
    nx, ny = 19, 14
    th = rng.uniform(0, 2 * math.pi, size=300).astype(np.float32)
    y = rng.uniform(-12, 12, size=300).astype(np.float32)
    L = orc.lines_from_theta_y(th, y)
    s = rng.normal(size=300)
    for n in (0, 3):
        full = orc.adjoint(n, s, L, nx, ny)
        pix = rng.choice(nx * ny, size=40, replace=False)
        got = orc.adjoint_pixels(n, s, L, nx, ny, pix)
        np.testing.assert_allclose(got, full.ravel()[pix], atol=1e-12)


def test_line_invariances(orc):
    """P11: (theta + pi, -y) and swapped endpoints are the same line; moving
    the image by one cell along x1 moves the projection by <e1, theta_perp>."""
    rng = np.random.default_rng(70)
    N = 14
    c = np.zeros((N, N))
    c[3:11, 3:11] = rng.normal(size=(8, 8))
    th = rng.uniform(0, math.pi, size=60)
    y = rng.uniform(-6, 6, size=60)
    n = 2
    base = orc.forward(n, c, orc.lines_from_theta_y(th.astype(np.float32), y.astype(np.float32)))
    flip = orc.forward(n, c, orc.lines_from_theta_y((th + math.pi).astype(np.float32),
                                                     (-y).astype(np.float32)))
    np.testing.assert_allclose(base, flip, atol=2e-6)  # float32 rounding of theta + pi
    # endpoints vs reversed endpoints
    p = np.stack([y * np.sin(th) - 9 * np.cos(th), -y * np.cos(th) - 9 * np.sin(th)], 1)
    q = np.stack([y * np.sin(th) + 9 * np.cos(th), -y * np.cos(th) + 9 * np.sin(th)], 1)
    ep = np.concatenate([p, q], 1).astype(np.float32)
    er = np.concatenate([q, p], 1).astype(np.float32)
    np.testing.assert_allclose(orc.forward(n, c, orc.lines_from_endpoints(ep)),
                               orc.forward(n, c, orc.lines_from_endpoints(er)), atol=1e-12)
    # shift by one column
    cs = np.roll(c, 1, axis=1)
    th32, y32 = th.astype(np.float32), y.astype(np.float32)
    shifted = orc.forward(n, cs, orc.lines_from_theta_y(th32, y32))
    L2 = orc.lines_from_theta_y(th32, y32)
    moved = (L2[0], L2[1], L2[2] - L2[1])  # y - <e1, theta_perp> = y - sin
    np.testing.assert_allclose(shifted, orc.forward(n, c, moved), atol=1e-12)


def _endpoint_reference(ep):
    """Direction and offset of the line through p and q, by formulas other
    than the oracle's: theta = atan2(dy, dx), and y = <p, theta_perp> written
    as the 2-D cross product p x q / |q - p| (eq. (1): theta_perp =
    (sin, -cos), so <p, theta_perp> = (px dy - py dx)/|q - p| = p x q / |q - p|)."""
    e = np.asarray(ep, dtype=np.float64).reshape(-1, 4)
    px, py, qx, qy = e[:, 0], e[:, 1], e[:, 2], e[:, 3]
    th = np.arctan2(qy - py, qx - px)
    y = (px * qy - py * qx) / np.hypot(qx - px, qy - py)
    return th, y


@pytest.mark.parametrize("geometry", ["random", "fan"])
def test_endpoint_lines_match_theta_y(orc, geometry):
    """P11 / eq. (1): the line through two points equals the (theta, y) line
    with theta along q - p and y = <p, theta_perp>; reversing the points gives
    the same line as (theta + pi, -y).  Checked against atan2 and the cross
    product, and through the forward of both line forms."""
    import xrt_workloads as W
    rng = np.random.default_rng(71)
    N, n = 24, 3
    if geometry == "random":
        m = 400
        th = rng.uniform(-math.pi, 2 * math.pi, size=m)
        y = rng.uniform(-14, 14, size=m)
        a = rng.uniform(-40, 40, size=m)
        b = a + rng.choice([-1, 1], size=m) * rng.uniform(0.5, 60, size=m)
        tv = np.stack([np.cos(th), np.sin(th)], 1)
        nv = np.stack([np.sin(th), -np.cos(th)], 1)
        p = y[:, None] * nv + a[:, None] * tv
        q = y[:, None] * nv + b[:, None] * tv
        ep = np.concatenate([p, q], 1).astype(np.float32)
    else:
        ep = W.fan_beam(30, 40, 60.0, N, n)["endpoints"]
    c = rng.normal(size=(N, N))
    ref_th, ref_y = _endpoint_reference(ep)
    cs, sn, yy = orc.lines_from_endpoints(ep)
    np.testing.assert_allclose(cs, np.cos(ref_th), atol=1e-12)
    np.testing.assert_allclose(sn, np.sin(ref_th), atol=1e-12)
    np.testing.assert_allclose(yy, ref_y, atol=1e-9)
    # the reversed pair is the same line as (theta + pi, -y)
    cr, sr, yr = orc.lines_from_endpoints(ep[:, [2, 3, 0, 1]])
    np.testing.assert_allclose(cr, -cs, atol=1e-12)
    np.testing.assert_allclose(sr, -sn, atol=1e-12)
    np.testing.assert_allclose(yr, -yy, atol=1e-9)
    # forward of the endpoint form against the theta_y form of the same lines
    # (theta and y rounded to float32 on their way in: ~1e-7 relative)
    f_ep = orc.forward(n, c, (cs, sn, yy))
    f_ty = orc.forward(n, c, orc.lines_from_theta_y(ref_th.astype(np.float32), ref_y.astype(np.float32)))
    scale = np.abs(f_ty).max()
    assert scale > 1.0
    np.testing.assert_allclose(f_ep, f_ty, atol=2e-4 * scale)
    # most lines cross the grid: the comparison is not between zeros
    assert np.count_nonzero(np.abs(f_ty) > 1e-3 * scale) > 0.5 * len(f_ty)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_band_equals_dense(orc, n):
    """P12: the band enumeration drops no nonzero term: bit-for-bit equal to
    the sum over every centre in the same order."""
    rng = np.random.default_rng(80 + n)
    c = rng.normal(size=(13, 16))
    th = rng.uniform(0, 2 * math.pi, size=120)
    th[:4] = [0.0, math.pi / 2, math.pi / 4, math.pi]
    y = rng.uniform(-11, 11, size=120)
    y[:4] = [0.5, -1.5, 0.0, 2.0]
    L = orc.lines_from_theta_y(th.astype(np.float32), y.astype(np.float32))
    np.testing.assert_array_equal(orc.forward(n, c, L), orc.forward(n, c, L, dense=True))


def test_nnz_counts_support(orc):
    """The work counter equals the number of centres strictly inside the
    footprint support, counted by brute force."""
    rng = np.random.default_rng(90)
    nx, ny = 11, 9
    th = rng.uniform(0, 2 * math.pi, size=50).astype(np.float32)
    y = rng.uniform(-8, 8, size=50).astype(np.float32)
    L = orc.lines_from_theta_y(th, y)
    for n in range(4):
        cnt = 0
        for k in range(50):
            c, s, yy = L[0][k], L[1][k], L[2][k]
            w = (n + 1) * (abs(c) + abs(s)) / 2
            for j in range(ny):
                for i in range(nx):
                    u = yy - ((i - (nx - 1) / 2) * s - (j - (ny - 1) / 2) * c)
                    cnt += abs(u) < w
        assert orc.nnz(n, L, nx, ny) == cnt


def test_workloads_shapes():
    coeffs, lines = W.small_parallel()
    assert coeffs.shape == (64, 64) and coeffs.dtype == np.float32
    assert lines["theta"].size == 90 * 96
    assert lines["theta"][96] == np.float32(math.pi / 90)
    assert lines["y"][0] == np.float32(-47.5) and lines["y"][95] == np.float32(47.5)
    fan = W.fan_beam(8, 16, 1000.0, 512, 3)
    assert fan["endpoints"].shape == (128, 4)
