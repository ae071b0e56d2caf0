"""Host-side tests of the C ABI: the library loads without a GPU, exports every
symbol include/*.h declares, and rejects bad arguments synchronously,
before any HIP call."""
import ctypes
import os
import re

import pytest

from paper_2503_20907_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(xrt_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = header_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTS) == names


def test_version_and_status_strings():
    assert re.match(r"\d+\.\d+\.\d+", L.xrt_version())
    for st in (L.XRT_OK, L.XRT_EINVAL, L.XRT_EDEGREE, L.XRT_ESIZE, L.XRT_ENOMEM, L.XRT_EHIP,
               L.XRT_EPLAN):
        assert L.xrt_status_string(st)
    assert L.xrt_status_string(12345) == "unknown status"


def grid(nx=16, ny=16, h=1.0):
    return L.XrtGrid(nx, ny, h, 0.0, 0.0)


def lines(n=4, kind=L.XRT_LINES_THETA_Y, ptr=0x1000):
    return L.XrtLines(kind, n, ptr, ptr, ptr)


FAKE = 0x1000  # never dereferenced: every call below fails validation first


@pytest.mark.parametrize("args,expected", [
    (dict(coeffs=None), L.XRT_EINVAL),
    (dict(degree=4), L.XRT_EDEGREE),
    (dict(degree=-1), L.XRT_EDEGREE),
    (dict(g=grid(0, 5)), L.XRT_EINVAL),
    (dict(g=grid(5, -1)), L.XRT_EINVAL),
    (dict(g=grid(5, 5, 0.0)), L.XRT_EINVAL),
    (dict(g=grid(5, 5, float("nan"))), L.XRT_EINVAL),
    (dict(g=grid(40000, 5)), L.XRT_ESIZE),
    (dict(lines=lines(-1)), L.XRT_EINVAL),
    (dict(lines=lines(2 ** 31)), L.XRT_ESIZE),
    (dict(lines=lines(4, kind=7)), L.XRT_EINVAL),
    (dict(lines=L.XrtLines(L.XRT_LINES_THETA_Y, 4, None, FAKE, None)), L.XRT_EINVAL),
    (dict(lines=L.XrtLines(L.XRT_LINES_ENDPOINTS, 4, FAKE, FAKE, None)), L.XRT_EINVAL),
    (dict(sino=None), L.XRT_EINVAL),
])
def test_forward_argument_errors(args, expected):
    a = dict(coeffs=FAKE, g=grid(), degree=1, lines=lines(), sino=FAKE)
    a.update(args)
    st = L.xrt_forward(a["coeffs"], a["g"], a["degree"], a["lines"], a["sino"], None)
    assert st == expected


@pytest.mark.parametrize("args,expected", [
    (dict(out=None), L.XRT_EINVAL),
    (dict(sino=None), L.XRT_EINVAL),
    (dict(degree=9), L.XRT_EDEGREE),
    (dict(g=grid(3, 0)), L.XRT_EINVAL),
    (dict(lines=lines(-5)), L.XRT_EINVAL),
])
def test_adjoint_argument_errors(args, expected):
    a = dict(sino=FAKE, lines=lines(), degree=2, g=grid(), out=FAKE)
    a.update(args)
    assert L.xrt_adjoint(a["sino"], a["lines"], a["degree"], a["g"], a["out"], None) == expected


def test_plan_argument_errors():
    lib = L.load()
    out = ctypes.c_void_p(123)
    assert lib.xrt_plan_create(grid(), 5, ctypes.byref(lines()), None, ctypes.byref(out)) == \
        L.XRT_EDEGREE
    assert out.value is None
    assert lib.xrt_plan_create(grid(0, 1), 1, ctypes.byref(lines()), None, ctypes.byref(out)) == \
        L.XRT_EINVAL
    assert lib.xrt_plan_create(grid(), 1, ctypes.byref(lines()), None, None) == L.XRT_EINVAL
    # null / foreign plans
    assert L.xrt_plan_forward(None, FAKE, FAKE, None) == L.XRT_EPLAN
    assert L.xrt_plan_adjoint(None, FAKE, FAKE, None) == L.XRT_EPLAN
    assert L.xrt_plan_info(None)[0] == L.XRT_EPLAN
    assert L.xrt_plan_nnz(None, None)[0] == L.XRT_EPLAN
    junk = (ctypes.c_uint64 * 64)()
    assert L.xrt_plan_forward(ctypes.addressof(junk), FAKE, FAKE, None) == L.XRT_EPLAN
    L.xrt_plan_destroy(None)
    L.xrt_plan_destroy(ctypes.addressof(junk))  # not a plan: ignored


def test_product_path_has_no_cpu_fallback():
    torch = pytest.importorskip("torch")
    from paper_2503_20907_amd import ops
    with pytest.raises(ValueError):
        ops.forward(torch.zeros(4, 4), ops.Lines(theta=[0.0], y=[0.0], device="cpu"), 1)


# ------------------------------------------------------------ include/xrt_learn.h
def test_learn_entry_points_reject_bad_arguments():
    lib = L.load()
    out = ctypes.c_void_p()
    # levels, base, channel cap, image size: rejected before any allocation
    assert lib.xrt_unet_create(1, 32, 0, 64, 64, 1, 0, ctypes.byref(out)) == L.XRT_EINVAL
    assert lib.xrt_unet_create(4, 48, 0, 64, 64, 1, 0, ctypes.byref(out)) == L.XRT_EINVAL
    assert lib.xrt_unet_create(4, 32, 16, 64, 64, 1, 0, ctypes.byref(out)) == L.XRT_EINVAL
    assert lib.xrt_unet_create(4, 32, 0, 60, 64, 1, 0, ctypes.byref(out)) == L.XRT_ESIZE
    assert lib.xrt_unet_create(4, 32, 0, 64, 64, 0, 0, ctypes.byref(out)) == L.XRT_ESIZE
    assert lib.xrt_unet_create(4, 32, 0, 64, 64, 1, 0, None) == L.XRT_EINVAL
    assert out.value is None
    # operations on a null network / plan
    assert lib.xrt_unet_apply(None, 1, 1, 1, None) == L.XRT_EINVAL
    assert lib.xrt_unet_set_gain(None, ctypes.c_float(1.0)) == L.XRT_EINVAL
    assert lib.xrt_unet_set_relu(None, 1) == L.XRT_EINVAL
    assert lib.xrt_unet_set_fusion(None, 1) == L.XRT_EINVAL
    n = ctypes.c_int64()
    assert lib.xrt_unet_num_params(None, ctypes.byref(n)) == L.XRT_EINVAL
    assert lib.xrt_reg_apply(None, 8, 8, ctypes.c_float(1.0), 1, None) == L.XRT_EINVAL
    assert lib.xrt_reg_apply(1, 0, 8, ctypes.c_float(1.0), 1, None) == L.XRT_EINVAL
    assert lib.xrt_normal_apply(None, ctypes.c_float(1.0), 1, 1, None, None) == L.XRT_EPLAN
    info = L.XrtSolveInfo()
    assert lib.xrt_solve(None, ctypes.c_float(1.0), 1, 1, ctypes.c_float(1e-3), 10, None, 1, 1,
                         ctypes.byref(info), None, 0, None) == L.XRT_EPLAN
    assert lib.xrt_solve(1, ctypes.c_float(1.0), 1, 1, ctypes.c_float(0.0), 10, None, 1, 1,
                         ctypes.byref(info), None, 0, None) == L.XRT_EINVAL
    # xrt_solve_ex: the options are checked before the plan or the network is
    # read (a dummy non-null network pointer is never dereferenced here)
    assert lib.xrt_solve_ex(None, ctypes.c_float(1.0), 1, 1, ctypes.c_float(1e-3), 10, None, None,
                            ctypes.byref(info), None, 0, None) == L.XRT_EPLAN
    assert lib.xrt_solve_ex(1, ctypes.c_float(1.0), 1, 1, ctypes.c_float(1e-3), 10, 1, None,
                            ctypes.byref(info), None, 0, None) == L.XRT_EINVAL
    for bad in [(0, 1, 0, 0), (17, 1, 0, 0), (1, 0, 0, 0), (1, 1, -1, 0), (1, 1, 0, 1), (1, 1, 2, 2)]:
        o = L.XrtSolveOpts(*bad)
        assert lib.xrt_solve_ex(1, ctypes.c_float(1.0), 1, 1, ctypes.c_float(1e-3), 10, 1, ctypes.byref(o),
                                ctypes.byref(info), None, 0, None) == L.XRT_EINVAL, bad
    # convolutions need channel counts that are multiples of 32
    assert lib.xrt_conv3x3_forward(1, 1, 1, 8, 8, 16, 32, 0, 1, None) == L.XRT_EINVAL
    assert lib.xrt_conv3x3_grad_weight(1, 1, 1, 8, 8, 32, 48, 1, None) == L.XRT_EINVAL
    assert lib.xrt_conv3x3_grad_input(None, 1, 1, 8, 8, 32, 32, 1, None) == L.XRT_EINVAL


# ------------------------------------------------------------ include/xrt_batch.h
def test_batch_entry_points_reject_bad_arguments():
    lib = L.load()
    out = ctypes.c_void_p()
    assert lib.xrt_batch_create(None, 1, None, ctypes.byref(out)) == L.XRT_EINVAL
    probs = (L.XrtProblem * 1)()
    assert lib.xrt_batch_create(probs, 0, None, ctypes.byref(out)) == L.XRT_EINVAL
    assert lib.xrt_batch_create(probs, 1, None, None) == L.XRT_EINVAL
    # a problem with an invalid degree fails in its plan, before any device work
    probs[0].grid = grid()
    probs[0].degree = 7
    probs[0].lines = L.XrtLines(0, 0, None, None, None)
    assert lib.xrt_batch_create(probs, 1, None, ctypes.byref(out)) == L.XRT_EDEGREE
    assert out.value is None
    cfg = L.XrtBatchConfig(4, 256, 2, 0)
    assert lib.xrt_batch_forward(None, None) == L.XRT_EINVAL
    assert lib.xrt_batch_adjoint(None, None) == L.XRT_EINVAL
    assert lib.xrt_batch_run(None, 1, None) == L.XRT_EINVAL
    assert lib.xrt_batch_set_config(None, ctypes.byref(cfg)) == L.XRT_EINVAL
    assert lib.xrt_batch_get_config(None, ctypes.byref(cfg)) == L.XRT_EINVAL
    assert lib.xrt_batch_autotune(None, 1, None, None) == L.XRT_EINVAL
    assert lib.xrt_batch_info(None, None, None, None) == L.XRT_EINVAL
    assert lib.xrt_batch_buffers(None, 0, None, None, None) == L.XRT_EINVAL


def test_sino_filter_and_pcg_reject_bad_arguments():
    lib = L.load()
    F = 0x1000  # never dereferenced: validation fails first
    assert lib.xrt_sino_filter(None, 2, 8, F, 3, F, None) == L.XRT_EINVAL
    assert lib.xrt_sino_filter(F, 2, 8, None, 3, F, None) == L.XRT_EINVAL
    assert lib.xrt_sino_filter(F, 2, 8, F, 3, None, None) == L.XRT_EINVAL
    assert lib.xrt_sino_filter(F, -1, 8, F, 3, F, None) == L.XRT_EINVAL
    assert lib.xrt_sino_filter(F, 2, 0, F, 3, F, None) == L.XRT_EINVAL
    for taps in (0, 2, 65, -3):
        assert lib.xrt_sino_filter(F, 2, 8, F, taps, F, None) == L.XRT_EINVAL, taps
    info = L.XrtSolveInfo()
    pc = L.XrtSinoPrecond(2, 8, 3, F, 0.0, 0)
    assert lib.xrt_solve_sino_pcg(None, ctypes.c_float(1.0), F, F, ctypes.c_float(1e-3), 10, ctypes.byref(pc),
                                  ctypes.byref(info), None, 0, None) == L.XRT_EPLAN
