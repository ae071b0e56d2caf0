"""GPU parity: the HIP library against the FP64 oracle on the same seeded inputs.

Tolerance: the relative L2 error of a sinogram (or back-projected image) must
be <= 1e-5, and the adjoint identity <Hc, s> = <c, H^T s> must hold to 1e-5
(relative to |<Hc, s>|), as required for FP32 kernels against the FP64
definition.  Small cases are compared in full, element by element; the 512^2 and 2048^2
benchmark workloads are in test_gpu_coverage.py.
"""
import math
import sys

import numpy as np
import pytest

import xrt_workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return t


@pytest.fixture(scope="module")
def ops(torch):
    from paper_2503_20907_amd import ops as o
    return o


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(torch, x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def orc_lines(orc, spec):
    return orc.lines(spec)


# ---------------------------------------------------------------- small cases
def test_small_parallel_forward_adjoint(orc, torch, ops):
    """64x64 degree 1, parallel beam 90 x 96: full forward and adjoint."""
    say("case: small parallel 64x64 deg1")
    coeffs, spec = W.small_parallel()
    Lo = orc_lines(orc, spec)
    ref_f = orc.forward(1, coeffs.astype(np.float64), Lo)
    lines = ops.Lines.from_spec(spec)
    c = to_dev(torch, coeffs)
    plan = ops.Plan(64, 64, 1, lines)
    s = plan.forward(c).cpu().numpy()
    assert rel_l2(s, ref_f) <= TOL
    np.testing.assert_allclose(s, ref_f, atol=TOL * np.abs(ref_f).max())
    rng = np.random.default_rng(3)
    sv = rng.normal(size=lines.n).astype(np.float32)
    ref_a = orc.adjoint(1, sv.astype(np.float64), Lo, 64, 64)
    a = plan.adjoint(to_dev(torch, sv)).cpu().numpy()
    assert rel_l2(a, ref_a) <= TOL
    # plan-less entry points give the same numbers
    s2 = ops.forward(c, lines, 1).cpu().numpy()
    np.testing.assert_array_equal(s, s2)
    a2 = ops.adjoint(to_dev(torch, sv), lines, 1, 64, 64).cpu().numpy()
    assert rel_l2(a2, ref_a) <= TOL


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_random_lines_all_degrees(orc, torch, ops, n):
    """Non-square grid spanning several tiles with a ragged tail, random lines
    incl. axis-aligned, diagonal and margin-grazing ones, non-unit spacing and
    offset centre."""
    say(f"case: random lines 150x97 deg{n}")
    rng = np.random.default_rng(100 + n)
    nx, ny, h, cx, cy = 150, 97, 0.8, 3.0, -2.5
    coeffs = rng.normal(size=(ny, nx)).astype(np.float32)
    m = 3000
    th = rng.uniform(-math.pi, 2 * math.pi, m)
    y = rng.uniform(-110, 110, m)
    th[:6] = [0.0, math.pi / 2, math.pi / 4, -math.pi / 4, math.pi, 3 * math.pi / 4]
    y[:6] = [cy + 0.5 * h * (ny - 1) + 0.4 * h * (n + 1), 1.0, 0.0, 2.0, -3.3, 10.0]
    spec = {"kind": "theta_y", "theta": th.astype(np.float32), "y": y.astype(np.float32)}
    Lo = orc_lines(orc, spec)
    lines = ops.Lines.from_spec(spec)
    plan = ops.Plan(nx, ny, n, lines, spacing=h, cx=cx, cy=cy)
    ref = orc.forward(n, coeffs.astype(np.float64), Lo, spacing=h, cx=cx, cy=cy)
    got = plan.forward(to_dev(torch, coeffs)).cpu().numpy()
    assert rel_l2(got, ref) <= TOL
    np.testing.assert_allclose(got, ref, atol=20 * TOL * np.abs(ref).max())
    sv = rng.normal(size=m)
    ref_a = orc.adjoint(n, sv, Lo, nx, ny, spacing=h, cx=cx, cy=cy)
    got_a = plan.adjoint(to_dev(torch, sv)).cpu().numpy()
    assert rel_l2(got_a, ref_a) <= TOL
    np.testing.assert_allclose(got_a, ref_a, atol=20 * TOL * np.abs(ref_a).max())


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_adjoint_identity_gpu(torch, ops, n):
    say(f"case: adjoint identity deg{n}")
    rng = np.random.default_rng(200 + n)
    nx, ny = 131, 140
    th = rng.uniform(0, 2 * math.pi, 5000).astype(np.float32)
    y = rng.uniform(-100, 100, 5000).astype(np.float32)
    lines = ops.Lines(theta=th, y=y)
    plan = ops.Plan(nx, ny, n, lines)
    c = to_dev(torch, rng.normal(size=(ny, nx)))
    s = to_dev(torch, rng.normal(size=5000))
    Hc = plan.forward(c).double()
    Hts = plan.adjoint(s).double()
    lhs = float((Hc * s.double()).sum())
    rhs = float((c.double() * Hts).sum())
    assert abs(lhs - rhs) <= TOL * abs(lhs)


def test_endpoint_lines_and_invariances(orc, torch, ops):
    """Endpoint input (both orders) against the oracle; a line equals its
    reverse."""
    say("case: endpoints")
    rng = np.random.default_rng(300)
    nx, ny = 90, 90
    coeffs = rng.normal(size=(ny, nx)).astype(np.float32)
    fan = W.fan_beam(24, 64, 120.0, 90, 2)
    ep = fan["endpoints"]
    rev = np.concatenate([ep[:, 2:], ep[:, :2]], axis=1)
    Lo = orc.lines_from_endpoints(ep)
    ref = orc.forward(2, coeffs.astype(np.float64), Lo)
    p1 = ops.Plan(nx, ny, 2, ops.Lines(endpoints=ep))
    p2 = ops.Plan(nx, ny, 2, ops.Lines(endpoints=rev))
    c = to_dev(torch, coeffs)
    g1 = p1.forward(c).cpu().numpy()
    g2 = p2.forward(c).cpu().numpy()
    assert rel_l2(g1, ref) <= TOL
    assert rel_l2(g2, ref) <= TOL


def test_edge_cases(torch, ops):
    say("case: edge cases")
    from paper_2503_20907_amd import _lib as L
    c = to_dev(torch, np.ones((8, 8)))
    # empty line list
    empty = ops.Lines(theta=np.zeros(0, np.float32), y=np.zeros(0, np.float32))
    p = ops.Plan(8, 8, 3, empty)
    assert p.forward(c).numel() == 0
    assert float(p.adjoint(torch.zeros(0, device="cuda")).abs().sum()) == 0.0
    # lines that miss the padded grid give exactly 0; the adjoint ignores them
    miss = ops.Lines(theta=[0.3, 1.0, 2.0], y=[50.0, -40.0, 9.0])
    pm = ops.Plan(8, 8, 3, miss)
    assert pm.info() == (3, 0)
    assert float(pm.forward(c).abs().sum()) == 0.0
    assert float(pm.adjoint(to_dev(torch, [1.0, 2.0, 3.0])).abs().sum()) == 0.0
    # degenerate and non-finite lines are rejected
    with pytest.raises(L.XrtError) as ei:
        ops.Plan(8, 8, 1, ops.Lines(endpoints=[[1.0, 2.0, 1.0, 2.0]]))
    assert ei.value.status == L.XRT_EINVAL
    with pytest.raises(L.XrtError):
        ops.Plan(8, 8, 1, ops.Lines(theta=[float("nan")], y=[0.0]))
    with pytest.raises(L.XrtError):
        ops.Plan(8, 8, 1, ops.Lines(theta=[0.0], y=[float("inf")]))
    with pytest.raises(L.XrtError) as ei:
        ops.Plan(8, 8, 4, ops.Lines(theta=[0.0], y=[0.0]))
    assert ei.value.status == L.XRT_EDEGREE
    # NaN coefficients propagate to the lines that see them
    cn = np.zeros((8, 8), np.float32)
    cn[2, 2] = np.nan
    out = ops.Plan(8, 8, 0, ops.Lines(theta=[math.pi / 2, math.pi / 2], y=[-1.5, 3.5])) \
        .forward(to_dev(torch, cn)).cpu().numpy()
    assert np.isnan(out[0]) and out[1] == 0.0


@pytest.mark.parametrize("shape", [(1, 1), (1, 37), (53, 1), (65, 64), (64, 129)])
def test_degenerate_grids(orc, torch, ops, shape):
    say(f"case: grid {shape}")
    ny, nx = shape
    rng = np.random.default_rng(400 + nx + ny)
    coeffs = rng.normal(size=(ny, nx)).astype(np.float32)
    th = rng.uniform(0, math.pi, 400).astype(np.float32)
    y = rng.uniform(-0.7 * max(nx, ny), 0.7 * max(nx, ny), 400).astype(np.float32)
    Lo = orc.lines_from_theta_y(th, y)
    lines = ops.Lines(theta=th, y=y)
    for n in (1, 3):
        plan = ops.Plan(nx, ny, n, lines)
        ref = orc.forward(n, coeffs.astype(np.float64), Lo)
        got = plan.forward(to_dev(torch, coeffs)).cpu().numpy()
        assert rel_l2(got, ref) <= TOL
        sv = rng.normal(size=400)
        ref_a = orc.adjoint(n, sv, Lo, nx, ny)
        got_a = plan.adjoint(to_dev(torch, sv)).cpu().numpy()
        assert rel_l2(got_a, ref_a) <= TOL


def test_nnz_matches_oracle(orc, torch, ops):
    say("case: nnz")
    rng = np.random.default_rng(500)
    th = rng.uniform(0, 2 * math.pi, 2000).astype(np.float32)
    y = rng.uniform(-80, 80, 2000).astype(np.float32)
    Lo = orc.lines_from_theta_y(th, y)
    lines = ops.Lines(theta=th, y=y)
    for n in range(4):
        plan = ops.Plan(120, 90, n, lines)
        assert plan.nnz() == orc.nnz(n, Lo, 120, 90)


def test_forward_deterministic_and_stream(torch, ops):
    say("case: determinism / stream")
    rng = np.random.default_rng(600)
    th = rng.uniform(0, math.pi, 20000).astype(np.float32)
    y = rng.uniform(-100, 100, 20000).astype(np.float32)
    lines = ops.Lines(theta=th, y=y)
    plan = ops.Plan(200, 200, 3, lines)
    c = to_dev(torch, rng.normal(size=(200, 200)))
    a = plan.forward(c)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b = plan.forward(c)
    st.synchronize()
    assert torch.equal(a, b)


# The 512^2 and 2048^2 cubic workloads: tests/test_gpu_coverage.py (whole
# 512^2 operator; 1% of the 2048^2 lines, 1000 pixels and the 1% subset's
# adjoint over every pixel).


def test_large_sampled_box_spline(orc, torch, ops):
    """The same 2048^2 lines with the 3-directional box spline (as the
    benchmark times it): forward at 20,000 sampled lines, adjoint at 300
    sampled pixels, and the adjoint identity over the whole operator."""
    say("case: 2048 box spline fan+random")
    box = orc.BOX3
    spec, nfan = W.large_lines()
    coeffs = W.large_phantom()
    lines = ops.Lines.from_spec(spec)
    plan = ops.Plan(2048, 2048, box, lines)
    got = plan.forward(to_dev(torch, coeffs)).cpu().numpy()
    Lo = orc_lines(orc, spec)
    rng = np.random.default_rng(801)
    pick = rng.choice(lines.n, size=20000, replace=False)
    ref = orc.forward(box, coeffs.astype(np.float64), tuple(v[pick] for v in Lo))
    assert rel_l2(got[pick], ref) <= TOL
    sv = rng.normal(size=lines.n).astype(np.float32)
    got_a = plan.adjoint(to_dev(torch, sv)).cpu().numpy().ravel()
    pix = rng.choice(2048 * 2048, size=300, replace=False)
    ref_a = orc.adjoint_pixels(box, sv.astype(np.float64), Lo, 2048, 2048, pix)
    assert rel_l2(got_a[pix], ref_a) <= TOL
    lhs = float(np.dot(got.astype(np.float64), sv.astype(np.float64)))
    rhs = float(np.dot(coeffs.astype(np.float64).ravel(), got_a.astype(np.float64)))
    assert abs(lhs - rhs) <= TOL * abs(lhs)
    plan.close()


# ------------------------------------------- schedules kept for large problems
@pytest.mark.parametrize("n", [0, 1, 2, 3, 16])
def test_plain_schedules_match_defaults(torch, ops, n):
    """The forward's one launch per strip (used when the per-strip sums of
    the persistent launch would exceed its memory cap) gives the same
    sinogram bit for bit: both add the strip sums in strip order.  Unsplit
    adjoint tiles (used on grids with very many tiles) agree with split ones
    to FP32 rounding: only the order of the partial images' sums differs."""
    import os
    say(f"case: plain vs default schedules, basis {n}")
    rng = np.random.default_rng(900 + n)
    m = 30000
    th = rng.uniform(0, math.pi, m).astype(np.float32)
    y = rng.uniform(-190, 190, m).astype(np.float32)
    lines = ops.Lines(theta=th, y=y)
    c = to_dev(torch, rng.normal(size=(290, 330)))
    s = to_dev(torch, rng.normal(size=m))
    fwd, adj = [], []
    for sched in ("default", "plain"):
        if sched == "plain":
            os.environ["XRT_SCHEDULE"] = "plain"
        try:
            plan = ops.Plan(330, 290, n, lines)
        finally:
            os.environ.pop("XRT_SCHEDULE", None)
        fwd.append(plan.forward(c).cpu().numpy())
        adj.append(plan.adjoint(s).cpu().numpy())
        plan.close()
    assert np.array_equal(fwd[0], fwd[1])
    assert rel_l2(adj[0], adj[1]) < 1e-6
