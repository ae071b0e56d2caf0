"""Differentiation: Project / BackProject autograd functions against central
finite differences (h = 1e-3) of a quadratic data-fit loss computed in FP64 by
the oracle, at 8 random coefficients per problem, over problems of several
grid sizes, degrees 1 and 3, parallel and fan geometries."""
import math

import numpy as np
import pytest

import xrt_workloads as W

pytestmark = pytest.mark.gpu

PROBLEMS = [  # (N, degree, geometry, n_angles)
    (64, 1, "parallel", 60),
    (96, 3, "fan", 75),
    (128, 3, "parallel", 120),
    (80, 1, "fan", 90),
]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return t


@pytest.mark.parametrize("N,n,geom,na", PROBLEMS)
def test_autograd_vs_finite_differences(orc, torch, N, n, geom, na):
    from paper_2503_20907_amd import ops
    print(f"case: autograd N={N} n={n} {geom} angles={na}", flush=True)
    rng = np.random.default_rng(1000 + N + n)
    nb = int(math.ceil(1.5 * N))
    if geom == "parallel":
        spec = W.parallel_beam(na, nb, 1.0)
    else:
        spec = W.fan_beam(na, nb, 2.0 * N, N, n)
    coeffs = W.ellipse_phantom(N, 8, seed=int(rng.integers(1 << 30)), texture_sigma=0.1)
    lines = ops.Lines.from_spec(spec)
    plan = ops.Plan(N, N, n, lines)
    p = rng.normal(size=lines.n)
    c = torch.tensor(coeffs, device="cuda", requires_grad=True)
    pt = torch.tensor(p, dtype=torch.float32, device="cuda")
    loss = 0.5 * ((ops.project(c, plan) - pt) ** 2).sum()
    loss.backward()
    grad = c.grad.detach().cpu().numpy().astype(np.float64)
    # FP64 central differences of the same loss through the oracle
    Lo = orc.lines(spec)
    c64 = coeffs.astype(np.float64)
    h = 1e-3
    picks = rng.choice(N * N, size=8, replace=False)

    def loss64(img):
        r = orc.forward(n, img, Lo) - p
        return 0.5 * float(r @ r)

    for k in picks:
        e = np.zeros_like(c64)
        e.flat[k] = h
        fd = (loss64(c64 + e) - loss64(c64 - e)) / (2 * h)
        assert grad.flat[k] == pytest.approx(fd, rel=1e-5, abs=1e-5 * np.abs(grad).max())
    # the adjoint's own backward is the forward: <BackProject(s), c> gradient wrt s
    s = torch.tensor(p, dtype=torch.float32, device="cuda", requires_grad=True)
    (ops.backproject(s, plan) * c.detach()).sum().backward()
    ref = plan.forward(c.detach()).cpu().numpy()
    np.testing.assert_allclose(s.grad.cpu().numpy(), ref, rtol=0, atol=1e-6 * np.abs(ref).max())
