"""ctypes binding of libxrt.so: argument marshalling only.

Every entry point has the name of its C counterpart in include/xrt.h.  Array
arguments are raw device addresses (ints) and the stream is a hipStream_t
handle (int, 0 for the null stream).  The library is loaded from this package
directory; if it is missing the import fails loudly, since there is no other
implementation of the operator on the product path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxrt.so")

XRT_OK = 0
XRT_EINVAL = -1
XRT_EDEGREE = -2
XRT_ESIZE = -3
XRT_ENOMEM = -4
XRT_EHIP = -5
XRT_EPLAN = -6

XRT_BOX3 = 16   # basis code of the 3-directional box spline

XRT_LINES_THETA_Y = 0
XRT_LINES_ENDPOINTS = 1

# every symbol declared in include/*.h
EXPORTS = (
    # xrt.h
    "xrt_forward", "xrt_adjoint", "xrt_plan_create", "xrt_plan_forward", "xrt_plan_adjoint",
    "xrt_plan_info", "xrt_plan_nnz", "xrt_plan_destroy", "xrt_status_string", "xrt_last_error",
    "xrt_version", "xrt_adjoint_noalloc",
    # xrt_learn.h
    "xrt_reg_apply", "xrt_normal_apply", "xrt_unet_create", "xrt_unet_destroy", "xrt_unet_num_params",
    "xrt_unet_set_params", "xrt_unet_get_params", "xrt_unet_set_gain", "xrt_unet_get_gain",
    "xrt_unet_set_relu", "xrt_unet_set_fusion", "xrt_unet_apply", "xrt_unet_loss_grad", "xrt_unet_train_step",
    "xrt_unet_loss_grad_normal", "xrt_unet_train_step_normal", "xrt_unet_loss_grad_energy",
    "xrt_unet_train_step_energy", "xrt_conv3x3_forward",
    "xrt_conv3x3_grad_input", "xrt_conv3x3_grad_weight", "xrt_solve", "xrt_solve_ex", "xrt_sino_filter",
    "xrt_solve_sino_pcg",
    # xrt_batch.h
    "xrt_batch_create", "xrt_batch_destroy", "xrt_batch_buffers", "xrt_batch_info", "xrt_batch_forward",
    "xrt_batch_adjoint", "xrt_batch_run", "xrt_batch_get_config", "xrt_batch_set_config",
    "xrt_batch_autotune",
    # xrt_bench.h
    "xrt_calib_valu",
    "xrt_calib_lds",
)


class XrtGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("spacing", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double)]


class XrtLines(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int64),
                ("theta", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("endpoints", ctypes.c_void_p)]


class XrtSolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("operator_applies", ctypes.c_int32),
                ("learned_accepted", ctypes.c_int32), ("learned_rejected", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("rel_residual", ctypes.c_double)]


class XrtSolveOpts(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int32), ("period", ctypes.c_int32), ("net_steps", ctypes.c_int32),
                ("restart", ctypes.c_int32)]


class XrtSinoPrecond(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int64), ("n_bins", ctypes.c_int32), ("taps", ctypes.c_int32),
                ("filter", ctypes.c_void_p), ("mu", ctypes.c_float), ("pad", ctypes.c_int32)]


class XrtProblem(ctypes.Structure):
    _fields_ = [("grid", XrtGrid), ("degree", ctypes.c_int32), ("lines", XrtLines)]


class XrtBatchConfig(ctypes.Structure):
    _fields_ = [("fwd_blocks_per_cu", ctypes.c_int32), ("lines_per_item", ctypes.c_int32),
                ("adj_blocks_per_cu", ctypes.c_int32), ("pad", ctypes.c_int32)]


class XrtError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {status_string(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2503_20907_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    lib.xrt_forward.argtypes = [vp, XrtGrid, i32, ctypes.POINTER(XrtLines), vp, vp]
    lib.xrt_adjoint.argtypes = [vp, ctypes.POINTER(XrtLines), i32, XrtGrid, vp, vp]
    lib.xrt_adjoint_noalloc.argtypes = [vp, ctypes.POINTER(XrtLines), i32, XrtGrid, vp, vp]
    lib.xrt_calib_valu.argtypes = [i32, i32, i32, vp, vp]
    lib.xrt_calib_valu.restype = i32
    lib.xrt_calib_lds.argtypes = [i32, i32, i32, vp, vp]
    lib.xrt_calib_lds.restype = i32
    lib.xrt_plan_create.argtypes = [XrtGrid, i32, ctypes.POINTER(XrtLines), vp,
                                    ctypes.POINTER(vp)]
    lib.xrt_plan_forward.argtypes = [vp, vp, vp, vp]
    lib.xrt_plan_adjoint.argtypes = [vp, vp, vp, vp]
    lib.xrt_plan_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.xrt_plan_nnz.argtypes = [vp, ctypes.POINTER(i64), vp]
    lib.xrt_plan_destroy.argtypes = [vp]
    lib.xrt_plan_destroy.restype = None
    lib.xrt_status_string.argtypes = [i32]
    lib.xrt_status_string.restype = ctypes.c_char_p
    lib.xrt_last_error.argtypes = []
    lib.xrt_last_error.restype = ctypes.c_char_p
    lib.xrt_version.restype = ctypes.c_char_p
    f32, u64 = ctypes.c_float, ctypes.c_uint64
    lib.xrt_reg_apply.argtypes = [vp, i32, i32, f32, vp, vp]
    lib.xrt_normal_apply.argtypes = [vp, f32, vp, vp, vp, vp]
    lib.xrt_unet_create.argtypes = [i32, i32, i32, i32, i32, i32, u64, ctypes.POINTER(vp)]
    lib.xrt_unet_destroy.argtypes = [vp]
    lib.xrt_unet_destroy.restype = None
    lib.xrt_unet_num_params.argtypes = [vp, ctypes.POINTER(i64)]
    lib.xrt_unet_set_params.argtypes = [vp, vp, vp]
    lib.xrt_unet_get_params.argtypes = [vp, vp, vp]
    lib.xrt_unet_set_gain.argtypes = [vp, f32]
    lib.xrt_unet_get_gain.argtypes = [vp, ctypes.POINTER(f32)]
    lib.xrt_unet_set_relu.argtypes = [vp, i32]
    lib.xrt_unet_set_fusion.argtypes = [vp, i32]
    lib.xrt_unet_apply.argtypes = [vp, vp, vp, i32, vp]
    lib.xrt_unet_loss_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    lib.xrt_unet_train_step.argtypes = [vp, vp, vp, i32, f32, vp, vp]
    lib.xrt_unet_loss_grad_normal.argtypes = [vp, vp, f32, vp, i32, vp, vp, vp]
    lib.xrt_unet_train_step_normal.argtypes = [vp, vp, f32, vp, i32, f32, vp, vp]
    lib.xrt_unet_loss_grad_energy.argtypes = [vp, vp, f32, vp, vp, i32, vp, vp, vp]
    lib.xrt_unet_train_step_energy.argtypes = [vp, vp, f32, vp, vp, i32, f32, vp, vp]
    lib.xrt_conv3x3_forward.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, vp, vp]
    lib.xrt_conv3x3_grad_input.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp]
    lib.xrt_conv3x3_grad_weight.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp]
    lib.xrt_solve.argtypes = [vp, f32, vp, vp, f32, i32, vp, i32, i32, ctypes.POINTER(XrtSolveInfo),
                              ctypes.POINTER(ctypes.c_double), i32, vp]
    lib.xrt_solve_ex.argtypes = [vp, f32, vp, vp, f32, i32, vp, ctypes.POINTER(XrtSolveOpts),
                                 ctypes.POINTER(XrtSolveInfo), ctypes.POINTER(ctypes.c_double), i32, vp]
    lib.xrt_sino_filter.argtypes = [vp, i64, i32, vp, i32, vp, vp]
    lib.xrt_solve_sino_pcg.argtypes = [vp, f32, vp, vp, f32, i32, ctypes.POINTER(XrtSinoPrecond),
                                       ctypes.POINTER(XrtSolveInfo), ctypes.POINTER(ctypes.c_double), i32, vp]
    fpp = ctypes.POINTER(ctypes.c_void_p)
    lib.xrt_batch_create.argtypes = [ctypes.POINTER(XrtProblem), i32, vp, ctypes.POINTER(vp)]
    lib.xrt_batch_destroy.argtypes = [vp]
    lib.xrt_batch_destroy.restype = None
    lib.xrt_batch_buffers.argtypes = [vp, i32, fpp, fpp, fpp]
    lib.xrt_batch_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.xrt_batch_forward.argtypes = [vp, vp]
    lib.xrt_batch_adjoint.argtypes = [vp, vp]
    lib.xrt_batch_run.argtypes = [vp, i32, vp]
    lib.xrt_batch_get_config.argtypes = [vp, ctypes.POINTER(XrtBatchConfig)]
    lib.xrt_batch_set_config.argtypes = [vp, ctypes.POINTER(XrtBatchConfig)]
    lib.xrt_batch_autotune.argtypes = [vp, i32, ctypes.POINTER(XrtBatchConfig), vp]
    for name in ("xrt_batch_create", "xrt_batch_buffers", "xrt_batch_info", "xrt_batch_forward",
                 "xrt_batch_adjoint", "xrt_batch_run", "xrt_batch_get_config", "xrt_batch_set_config",
                 "xrt_batch_autotune"):
        getattr(lib, name).restype = i32
    for name in ("xrt_forward", "xrt_adjoint", "xrt_adjoint_noalloc", "xrt_plan_create", "xrt_plan_forward",
                 "xrt_plan_adjoint", "xrt_plan_info", "xrt_plan_nnz", "xrt_reg_apply",
                 "xrt_normal_apply", "xrt_unet_create", "xrt_unet_num_params",
                 "xrt_unet_set_params", "xrt_unet_get_params", "xrt_unet_apply",
                 "xrt_unet_set_gain", "xrt_unet_get_gain", "xrt_unet_set_relu", "xrt_unet_set_fusion", "xrt_unet_loss_grad", "xrt_unet_train_step", "xrt_unet_loss_grad_normal",
                 "xrt_unet_train_step_normal", "xrt_unet_loss_grad_energy", "xrt_unet_train_step_energy",
                 "xrt_conv3x3_forward", "xrt_conv3x3_grad_input", "xrt_conv3x3_grad_weight", "xrt_solve",
                 "xrt_solve_ex", "xrt_sino_filter", "xrt_solve_sino_pcg"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def status_string(st: int) -> str:
    return load().xrt_status_string(int(st)).decode()


def last_error() -> str:
    return load().xrt_last_error().decode()


def check(st: int, where: str):
    if st != XRT_OK:
        raise XrtError(st, where, last_error() if st in (XRT_EHIP, XRT_ENOMEM, XRT_ESIZE) else "")


def xrt_forward(coeffs, grid: XrtGrid, degree: int, lines: XrtLines, sino, stream) -> int:
    return load().xrt_forward(coeffs, grid, int(degree), ctypes.byref(lines), sino, stream)


def xrt_adjoint(sino, lines: XrtLines, degree: int, grid: XrtGrid, coeffs_out, stream) -> int:
    return load().xrt_adjoint(sino, ctypes.byref(lines), int(degree), grid, coeffs_out, stream)


def xrt_adjoint_noalloc(sino, lines: XrtLines, degree: int, grid: XrtGrid, coeffs_out, stream) -> int:
    return load().xrt_adjoint_noalloc(sino, ctypes.byref(lines), int(degree), grid, coeffs_out, stream)


def xrt_calib_valu(mode: int, iters: int, blocks: int, out, stream) -> int:
    return load().xrt_calib_valu(int(mode), int(iters), int(blocks), out, stream)


def xrt_calib_lds(pattern: int, iters: int, blocks: int, out, stream) -> int:
    return load().xrt_calib_lds(int(pattern), int(iters), int(blocks), out, stream)


def xrt_plan_create(grid: XrtGrid, degree: int, lines: XrtLines, stream):
    out = ctypes.c_void_p()
    st = load().xrt_plan_create(grid, int(degree), ctypes.byref(lines), stream,
                                ctypes.byref(out))
    return st, out.value


def xrt_plan_forward(plan, coeffs, sino, stream) -> int:
    return load().xrt_plan_forward(plan, coeffs, sino, stream)


def xrt_plan_adjoint(plan, sino, coeffs_out, stream) -> int:
    return load().xrt_plan_adjoint(plan, sino, coeffs_out, stream)


def xrt_plan_info(plan):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    st = load().xrt_plan_info(plan, ctypes.byref(a), ctypes.byref(b))
    return st, a.value, b.value


def xrt_plan_nnz(plan, stream):
    a = ctypes.c_int64()
    st = load().xrt_plan_nnz(plan, ctypes.byref(a), stream)
    return st, a.value


def xrt_plan_destroy(plan) -> None:
    load().xrt_plan_destroy(plan)


def xrt_status_string(st: int) -> str:
    return status_string(st)


def xrt_last_error() -> str:
    return last_error()


def xrt_version() -> str:
    return load().xrt_version().decode()


# ---------------------------------------------------------- include/xrt_learn.h
def xrt_reg_apply(c, nx, ny, lam, out, stream) -> int:
    return load().xrt_reg_apply(c, int(nx), int(ny), float(lam), out, stream)


def xrt_normal_apply(plan, lam, c, out, sino_ws, stream) -> int:
    return load().xrt_normal_apply(plan, float(lam), c, out, sino_ws, stream)


def xrt_unet_create(levels, base, max_channels, height, width, max_batch, seed):
    out = ctypes.c_void_p()
    st = load().xrt_unet_create(int(levels), int(base), int(max_channels), int(height), int(width),
                                int(max_batch), int(seed), ctypes.byref(out))
    return st, out.value


def xrt_unet_destroy(net) -> None:
    load().xrt_unet_destroy(net)


def xrt_unet_num_params(net):
    a = ctypes.c_int64()
    st = load().xrt_unet_num_params(net, ctypes.byref(a))
    return st, a.value


def xrt_unet_set_params(net, params, stream) -> int:
    return load().xrt_unet_set_params(net, params, stream)


def xrt_unet_get_params(net, params, stream) -> int:
    return load().xrt_unet_get_params(net, params, stream)


def xrt_unet_set_gain(net, gain) -> int:
    return load().xrt_unet_set_gain(net, float(gain))


def xrt_unet_set_relu(net, on) -> int:
    return load().xrt_unet_set_relu(net, int(on))


def xrt_unet_set_fusion(net, on) -> int:
    return load().xrt_unet_set_fusion(net, int(on))


def xrt_unet_get_gain(net):
    g = ctypes.c_float()
    st = load().xrt_unet_get_gain(net, ctypes.byref(g))
    return st, g.value


def xrt_unet_apply(net, r, z, batch, stream) -> int:
    return load().xrt_unet_apply(net, r, z, int(batch), stream)


def xrt_unet_loss_grad(net, r, e, batch, loss, grad, stream) -> int:
    return load().xrt_unet_loss_grad(net, r, e, int(batch), loss, grad, stream)


def xrt_unet_train_step(net, r, e, batch, lr, loss, stream) -> int:
    return load().xrt_unet_train_step(net, r, e, int(batch), float(lr), loss, stream)


def xrt_unet_loss_grad_normal(net, plan, lam, r, batch, loss, grad, stream) -> int:
    return load().xrt_unet_loss_grad_normal(net, plan, float(lam), r, int(batch), loss, grad, stream)


def xrt_unet_train_step_normal(net, plan, lam, r, batch, lr, loss, stream) -> int:
    return load().xrt_unet_train_step_normal(net, plan, float(lam), r, int(batch), float(lr), loss, stream)


def xrt_unet_loss_grad_energy(net, plan, lam, r, e, batch, loss, grad, stream) -> int:
    return load().xrt_unet_loss_grad_energy(net, plan, float(lam), r, e, int(batch), loss, grad, stream)


def xrt_unet_train_step_energy(net, plan, lam, r, e, batch, lr, loss, stream) -> int:
    return load().xrt_unet_train_step_energy(net, plan, float(lam), r, e, int(batch), float(lr), loss, stream)


def xrt_conv3x3_forward(x, w, B, H, W, cin, cout, relu, y, stream) -> int:
    return load().xrt_conv3x3_forward(x, w, int(B), int(H), int(W), int(cin), int(cout), int(relu), y,
                                      stream)


def xrt_conv3x3_grad_input(gy, w, B, H, W, cin, cout, gx, stream) -> int:
    return load().xrt_conv3x3_grad_input(gy, w, int(B), int(H), int(W), int(cin), int(cout), gx, stream)


def xrt_conv3x3_grad_weight(x, gy, B, H, W, cin, cout, gw, stream) -> int:
    return load().xrt_conv3x3_grad_weight(x, gy, int(B), int(H), int(W), int(cin), int(cout), gw, stream)


def xrt_solve_ex(plan, lam, b, x, tol, maxit, net, window, period, net_steps, restart, history_cap, stream):
    info = XrtSolveInfo()
    opts = XrtSolveOpts(int(window), int(period), int(net_steps), int(restart))
    hist = (ctypes.c_double * max(1, int(history_cap)))()
    st = load().xrt_solve_ex(plan, float(lam), b, x, float(tol), int(maxit), net, ctypes.byref(opts),
                             ctypes.byref(info), hist if history_cap > 0 else None, int(history_cap), stream)
    return st, info, [hist[i] for i in range(min(int(history_cap), info.iterations))]


def xrt_sino_filter(sino, n_views, n_bins, filt, taps, out, stream) -> int:
    return load().xrt_sino_filter(sino, int(n_views), int(n_bins), filt, int(taps), out, stream)


def xrt_solve_sino_pcg(plan, lam, b, x, tol, maxit, n_views, n_bins, filt, taps, mu, history_cap, stream):
    info = XrtSolveInfo()
    pc = XrtSinoPrecond(int(n_views), int(n_bins), int(taps), filt, float(mu), 0)
    hist = (ctypes.c_double * max(1, int(history_cap)))()
    st = load().xrt_solve_sino_pcg(plan, float(lam), b, x, float(tol), int(maxit), ctypes.byref(pc),
                                   ctypes.byref(info), hist if history_cap > 0 else None, int(history_cap),
                                   stream)
    return st, info, [hist[i] for i in range(min(int(history_cap), info.iterations))]


def xrt_solve(plan, lam, b, x, tol, maxit, net, window, period, history_cap, stream):
    info = XrtSolveInfo()
    hist = (ctypes.c_double * max(1, int(history_cap)))()
    st = load().xrt_solve(plan, float(lam), b, x, float(tol), int(maxit), net, int(window), int(period),
                          ctypes.byref(info),
                          hist if history_cap > 0 else None, int(history_cap), stream)
    return st, info, [hist[i] for i in range(min(int(history_cap), info.iterations))]


# ---------------------------------------------------------- include/xrt_batch.h
def xrt_batch_create(problems, stream):
    arr = (XrtProblem * len(problems))(*problems)
    out = ctypes.c_void_p()
    st = load().xrt_batch_create(arr, len(problems), stream, ctypes.byref(out))
    return st, out.value


def xrt_batch_destroy(b) -> None:
    load().xrt_batch_destroy(b)


def xrt_batch_buffers(b, p):
    c, s, k = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    st = load().xrt_batch_buffers(b, int(p), ctypes.byref(c), ctypes.byref(s), ctypes.byref(k))
    return st, c.value, s.value, k.value


def xrt_batch_info(b):
    n, f, a = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    st = load().xrt_batch_info(b, ctypes.byref(n), ctypes.byref(f), ctypes.byref(a))
    return st, n.value, f.value, a.value


def xrt_batch_forward(b, stream) -> int:
    return load().xrt_batch_forward(b, stream)


def xrt_batch_adjoint(b, stream) -> int:
    return load().xrt_batch_adjoint(b, stream)


def xrt_batch_run(b, use_graph, stream) -> int:
    return load().xrt_batch_run(b, int(use_graph), stream)


def xrt_batch_get_config(b):
    c = XrtBatchConfig()
    st = load().xrt_batch_get_config(b, ctypes.byref(c))
    return st, c


def xrt_batch_set_config(b, cfg: XrtBatchConfig) -> int:
    return load().xrt_batch_set_config(b, ctypes.byref(cfg))


def xrt_batch_autotune(b, reps, stream):
    c = XrtBatchConfig()
    st = load().xrt_batch_autotune(b, int(reps), ctypes.byref(c), stream)
    return st, c
