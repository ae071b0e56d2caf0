"""Pins of the 3-directional box-spline oracle (directions e1, e2, e1+e2;
Section III-C): the spatial box spline against its definition, the footprint
against dense line integrals, Proposition 1 (eq. (conv)) with the widths
|<theta_perp, u_d>|, the paper's printed sum formula (eq. (projbox)) and the
forward operator against brute-force line integrals of the continuous image."""
import math

import numpy as np
import pytest

import oracle

BOX = oracle.BOX3


def box_conv(widths, u):
    """Prop. 1 for three centred unit-mass boxes: the 8-term truncated-power
    form (1/(2 w1 w2 w3)) sum_S (-1)^|S| (u + W/2 - sum S)_+^2 (all widths > 0)."""
    w = list(widths)
    W = sum(w)
    acc = 0.0
    for m in range(8):
        S = sum(w[i] for i in range(3) if m >> i & 1)
        sgn = -1.0 if bin(m).count("1") % 2 else 1.0
        acc += sgn * max(u + W / 2 - S, 0.0) ** 2
    return acc / (2 * w[0] * w[1] * w[2])


def dense_line_integral(f2, c, s, u, n=400001, T=2.0):
    t = np.linspace(-T, T, n)
    v = f2(t * c + u * s, t * s - u * c)
    return float(np.trapezoid(v, t))


def mc(x1, x2):
    """centred box spline, vectorised, written from the definition
    M(x) = |{t in [0,1] : x - t(1,1) in [0,1]^2}| with x -> x + (1,1)"""
    x1 = np.asarray(x1) + 1.0
    x2 = np.asarray(x2) + 1.0
    lo = np.maximum(0.0, np.maximum(x1 - 1.0, x2 - 1.0))
    hi = np.minimum(1.0, np.minimum(x1, x2))
    return np.maximum(0.0, hi - lo)


def test_box_spline_is_the_measure_of_its_defining_set():
    rng = np.random.default_rng(1)
    t = np.linspace(0.0, 1.0, 200001)
    for _ in range(30):
        x1, x2 = rng.uniform(-0.5, 2.5, 2)
        inside = (x1 - t >= 0) & (x1 - t <= 1) & (x2 - t >= 0) & (x2 - t <= 1)
        ref = float(np.count_nonzero(inside)) / (len(t) - 1)
        assert abs(oracle.box_spline(x1, x2) - ref) < 2e-5
    assert oracle.box_spline(1.0, 1.0) == 1.0
    # unit mass: exact integral of a hat of height 1 over a hexagon of area 3
    g = np.linspace(0, 2, 1601)
    X1, X2 = np.meshgrid(g, g)
    vals = np.vectorize(oracle.box_spline)(X1, X2)
    assert abs(np.trapezoid(np.trapezoid(vals, g, axis=1), g) - 1.0) < 1e-5


@pytest.mark.parametrize("theta", [0.0, 0.3, math.pi / 4, 1.2, math.pi / 2, 2.0, 3 * math.pi / 4, 2.9, -0.7, 4.0])
def test_footprint_equals_dense_line_integral(theta):
    c, s = math.cos(theta), math.sin(theta)
    for u in np.linspace(-1.6, 1.6, 17):
        ref = dense_line_integral(mc, c, s, u)
        got = oracle.footprint(BOX, theta, [u])[0]
        assert abs(got - ref) < 2e-6, (theta, u, got, ref)


def test_footprint_is_even_with_unit_mass_and_exact_support():
    for theta in [0.1, 0.7, 1.9, 2.6]:
        c, s = math.cos(theta), math.sin(theta)
        W = 0.5 * (abs(s) + abs(c) + abs(s - c))
        u = np.linspace(-W, W, 4001)
        f = oracle.footprint(BOX, theta, u)
        assert np.allclose(f, f[::-1], atol=1e-14)
        assert abs(np.trapezoid(f, u) - 1.0) < 1e-6
        assert oracle.footprint(BOX, theta, [W * (1 + 1e-9)])[0] == 0.0
        assert oracle.footprint(BOX, theta, [W * (1 - 1e-3)])[0] > 0.0


def test_proposition_1_with_theta_perp_widths():
    # eq. (conv): phi_theta is the convolution of boxes of widths |<theta_perp, u_d>|
    # (theta_perp = (sin, -cos), u = e1, e2, e1+e2); with |<theta, u_d>| it is not
    # (reading of which direction the proposition's inner products use).
    rng = np.random.default_rng(2)
    n_other_differs = 0
    for _ in range(40):
        theta = rng.uniform(0, 2 * math.pi)
        c, s = math.cos(theta), math.sin(theta)
        perp = (abs(s), abs(c), abs(s - c))
        along = (abs(c), abs(s), abs(c + s))
        if min(perp) < 0.15 or min(along) < 0.15:
            continue
        for u in rng.uniform(-1.5, 1.5, 8):
            assert abs(oracle.footprint(BOX, theta, [u])[0] - box_conv(perp, u)) < 1e-10
        if max(abs(oracle.footprint(BOX, theta, [u])[0] - box_conv(along, u)) for u in np.linspace(-1, 1, 9)) > 1e-3:
            n_other_differs += 1
    assert n_other_differs > 5


def test_paper_sum_formula_matches_at_theta_plus_pi_over_2():
    # eq. (projbox): phi(y) = -1/(a1 a3 a5) sum_{n=1}^{6} (-1)^n (y - alpha_n)_+^2 with
    # alpha = (0, s, 2s+c, c, s+2c, 2(s+c)) (s, c of the paper's theta), the sum
    # 1-indexed, the product 0-indexed (a1 = s, a3 = c, a5 = 2(s+c)), and y
    # measured from the left end of the support.  The paper's theta is the normal
    # of the line: it equals our footprint at t = theta + pi/2, centred.
    for theta in [0.2, 0.5, 0.785, 1.0, 1.4]:
        s, c = math.sin(theta), math.cos(theta)
        alpha = [0.0, s, 2 * s + c, c, s + 2 * c, 2 * (s + c)]
        pref = -1.0 / (alpha[1] * alpha[3] * alpha[5])
        for y in np.linspace(0.0, alpha[5], 23):
            paper = pref * sum((-1) ** n * max(y - alpha[n - 1], 0.0) ** 2 for n in range(1, 7))
            ours = oracle.footprint(BOX, theta + math.pi / 2, [y - alpha[5] / 2])[0]
            assert abs(paper - ours) < 1e-12, (theta, y, paper, ours)


def test_forward_matches_brute_force_line_integrals():
    # s = sum_k c_k phi_theta(y - <x_k, theta_perp>) is the line integral of the
    # continuous image sum_k c_k Mc(x - x_k) (eq. (2)-(4) with the box basis)
    rng = np.random.default_rng(3)
    nx, ny = 5, 4
    coeffs = rng.normal(size=(ny, nx))
    th = np.concatenate([rng.uniform(0, 2 * math.pi, 25), [0.0, math.pi / 4, math.pi / 2, 3 * math.pi / 4]])
    yv = rng.uniform(-3, 3, th.size)
    lc = oracle.lines_from_theta_y(th.astype(np.float32), yv.astype(np.float32))
    got = oracle.forward(BOX, coeffs, lc)
    xs = np.arange(nx) - 0.5 * (nx - 1)
    ys = np.arange(ny) - 0.5 * (ny - 1)
    c_all, s_all, y_all = lc

    def image(x1, x2):
        out = np.zeros_like(x1)
        for j in range(ny):
            for i in range(nx):
                out += coeffs[j, i] * mc(x1 - xs[i], x2 - ys[j])
        return out

    for m in range(th.size):
        c, s, y = c_all[m], s_all[m], y_all[m]
        ref = dense_line_integral(image, c, s, y, n=200001, T=6.0)
        assert abs(got[m] - ref) < 1e-5 * max(1.0, abs(ref)), (m, got[m], ref)


def test_paper_piecewise_expansion_with_corrected_bounds():
    # eq. (projectionbox) for theta in (0, pi/4), alpha 0-indexed.  Its
    # polynomials are right; two interval bounds are garbled in the text: the
    # third piece ends at alpha_3 (printed alpha_5) and the fourth starts at
    # alpha_3 (printed alpha_5).  With those bounds it equals eq. (projbox).
    for theta in [0.1, 0.4, 0.7]:
        s, c = math.sin(theta), math.cos(theta)
        a = [0.0, s, 2 * s + c, c, s + 2 * c, 2 * (s + c)]
        p3 = a[1] * a[3] * a[5]

        def piecewise(y):
            if y < a[0]:
                return 0.0
            if y < a[1]:
                return y * y / p3
            if y < a[3]:
                return (2 * y - a[1]) / (a[3] * a[5])
            if y < a[2]:
                return (-y * y + a[5] * y - 1.0) / p3
            if y < a[4]:
                return (-2 * y + 4 * a[3] + 3 * a[1]) / (a[3] * a[5])
            if y < a[5]:
                return (y - 2 * a[1] - 2 * a[3]) ** 2 / p3
            return 0.0

        for y in np.linspace(-0.1, a[5] + 0.1, 41):
            ours = oracle.footprint(BOX, theta + math.pi / 2, [y - a[5] / 2])[0]
            assert abs(piecewise(y) - ours) < 1e-12, (theta, y)


def hat(u, w):
    """convolution of two centred unit-mass boxes of width w: (1/w)(1 - |u|/w)_+"""
    u = np.abs(np.asarray(u, np.float64))
    return np.maximum(1.0 - u / w, 0.0) / w


def test_fig2_family_of_projected_box_splines():
    """The curves of Fig. 2, theta in [-pi/4, pi/4).  Where a direction of the
    box spline is parallel to the lines, its box projects to width 0 and the
    footprint is the convolution of the other two boxes, the linear B-spline
    (hat): theta = 0 leaves widths (1, 1), so (1 - |u|)_+; theta = pi/4 leaves
    (1/sqrt 2, 1/sqrt 2).  Between them the support half-width
    (|sin| + |cos| + |sin - cos|)/2 shrinks from sqrt 2 while the peak rises
    from 1/sqrt 2, every curve has unit mass, and where all three widths are
    nonzero the curve is C^1: its second differences over h^2 stay bounded as
    h shrinks, where at the hats' kinks they grow like 1/h."""
    u = np.linspace(-1.6, 1.6, 3201)
    assert np.max(np.abs(oracle.footprint(BOX, 0.0, u) - hat(u, 1.0))) < 1e-13
    assert np.max(np.abs(oracle.footprint(BOX, math.pi / 4, u) - hat(u, 1 / math.sqrt(2)))) < 1e-12
    ths = np.linspace(-math.pi / 4, math.pi / 4, 33)[:-1]
    W = np.array([0.5 * (abs(math.sin(t)) + abs(math.cos(t)) + abs(math.sin(t) - math.cos(t))) for t in ths])
    peak = np.array([oracle.footprint(BOX, t, [0.0])[0] for t in ths])
    assert abs(W[0] - math.sqrt(2)) < 1e-12 and np.all(np.diff(W) < 0)
    assert abs(peak[0] - 1 / math.sqrt(2)) < 1e-12 and np.all(np.diff(peak) > 0)
    for t, w in zip(ths[::4], W[::4]):
        v = np.linspace(-w, w, 8001)
        assert abs(np.trapezoid(oracle.footprint(BOX, t, v), v) - 1.0) < 1e-6

    def curvature(t, h):
        f = oracle.footprint(BOX, t, np.arange(-2.0, 2.0, h))
        return np.max(np.abs(np.diff(f, 2))) / h ** 2

    for t in (-0.5, -0.2, 0.3, 0.6):
        assert curvature(t, 1e-4) < 1.01 * curvature(t, 1e-3) + 1e-6
    for t in (0.0, math.pi / 4):
        assert curvature(t, 1e-4) > 5 * curvature(t, 1e-3)
