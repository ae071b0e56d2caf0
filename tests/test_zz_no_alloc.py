"""The adjoint entry point that allocates nothing (xrt_adjoint_noalloc),
called through the C ABI: the same result as xrt_adjoint, bit for bit, on
two calls in a row (the second with a smaller problem, so that the shared
scratch array holds the first call's data when the second starts), against
the FP64 oracle, an empty line list, and a problem too large for the array."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return t


def _lines(L, torch, th, y):
    thd = torch.as_tensor(th, dtype=torch.float32, device="cuda")
    yd = torch.as_tensor(y, dtype=torch.float32, device="cuda")
    c = L.XrtLines(L.XRT_LINES_THETA_Y, th.size, thd.data_ptr(), yd.data_ptr(), None)
    return c, (thd, yd)


def _both(L, torch, s, lc, degree, grid, ny, nx):
    stream = torch.cuda.current_stream().cuda_stream
    a = torch.full((ny, nx), 7.0, device="cuda")
    b = torch.full((ny, nx), -3.0, device="cuda")
    L.check(L.xrt_adjoint_noalloc(s.data_ptr(), lc, degree, grid, a.data_ptr(), stream), "xrt_adjoint_noalloc")
    L.check(L.xrt_adjoint(s.data_ptr(), lc, degree, grid, b.data_ptr(), stream), "xrt_adjoint")
    torch.cuda.synchronize()
    return a, b


def test_noalloc_matches_adjoint_twice(orc, torch):
    from paper_2503_20907_amd import _lib as L
    rng = np.random.default_rng(1300)
    # first call: 300 x 260, cubic, 120,000 lines; second: 90 x 70, degree 2
    # (then the box spline), 5,000 lines
    for (nx, ny, m, degree) in [(300, 260, 120000, 3), (90, 70, 5000, 2), (90, 70, 5000, L.XRT_BOX3)]:
        print(f"case: no-alloc adjoint {nx}x{ny}, {m} lines, basis {degree}", flush=True)
        th = rng.uniform(-math.pi, 2 * math.pi, m).astype(np.float32)
        y = rng.uniform(-0.7 * max(nx, ny), 0.7 * max(nx, ny), m).astype(np.float32)
        lc, keep = _lines(L, torch, th, y)
        s_host = rng.normal(size=m).astype(np.float32)
        s = torch.as_tensor(s_host, device="cuda")
        grid = L.XrtGrid(nx, ny, 1.0, 0.0, 0.0)
        a, b = _both(L, torch, s, lc, degree, grid, ny, nx)
        assert torch.equal(a, b)
        ref = orc.adjoint(degree, s_host.astype(np.float64), orc.lines_from_theta_y(th, y), nx, ny)
        got = a.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


def test_noalloc_empty_and_too_large(torch):
    from paper_2503_20907_amd import _lib as L
    stream = torch.cuda.current_stream().cuda_stream
    th = np.zeros(0, np.float32)
    lc, keep = _lines(L, torch, th, th)
    out = torch.full((20, 30), 5.0, device="cuda")
    L.check(L.xrt_adjoint_noalloc(None, lc, 1, L.XrtGrid(30, 20, 1.0, 0.0, 0.0), out.data_ptr(), stream),
            "xrt_adjoint_noalloc")
    torch.cuda.synchronize()
    assert float(out.abs().sum()) == 0.0
    # 2,000,000 lines need more than the 64 MiB array: rejected before any launch
    m = 2_000_000
    th = np.zeros(m, np.float32)
    lc, keep = _lines(L, torch, th, th)
    s = torch.zeros(m, device="cuda")
    out = torch.zeros((64, 64), device="cuda")
    st = L.xrt_adjoint_noalloc(s.data_ptr(), lc, 3, L.XrtGrid(64, 64, 1.0, 0.0, 0.0), out.data_ptr(), stream)
    assert st == L.XRT_ESIZE
    assert "maximum" in L.last_error()


def test_noalloc_holds_the_documented_example(torch):
    """The header's example fits the array: 700,000 lines on a 512^2 grid
    (a small grid, so the two adjoint passes share one launch and 16 partial
    images), and the result equals xrt_adjoint's bit for bit."""
    from paper_2503_20907_amd import _lib as L
    print("case: no-alloc adjoint 512x512, 700000 lines, cubic", flush=True)
    rng = np.random.default_rng(1301)
    m, n = 700_000, 512
    th = rng.uniform(-math.pi, 2 * math.pi, m).astype(np.float32)
    y = rng.uniform(-0.7 * n, 0.7 * n, m).astype(np.float32)
    lc, keep = _lines(L, torch, th, y)
    s = torch.as_tensor(rng.normal(size=m).astype(np.float32), device="cuda")
    a, b = _both(L, torch, s, lc, 3, L.XrtGrid(n, n, 1.0, 0.0, 0.0), n, n)
    assert torch.equal(a, b)
    assert float(b.abs().max()) > 0
