"""CPU FP64 oracle for the B-spline x-ray transform and its adjoint.

TEST INFRASTRUCTURE ONLY.  This package is the reference that the HIP library
is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
GPU path (``paper_2503_20907_amd``), and that path never imports it.

The arithmetic lives in ``xrt_oracle.c`` (FP64, OpenMP over lines); this module
only builds it with gcc and marshals NumPy arrays through ctypes.  Each entry
point states the passage of the paper it follows:

* ``footprint``: phi_theta(u) = (beta^n_{|cos|} * beta^n_{|sin|})(u),
  Proposition 1 / eq. (6) (Sections III-A, III-B).
* ``forward``:  s_m = sum_k c_k h phi_theta_m((y_m - <x_k, theta_m^perp>)/h),
  eq. (4) and the entries of H_phi (Section IV-A).
* ``adjoint``:  (H^T s)_k, the back-projection of Section II-B (matched to the
  forward), ray-major in FP64.
* ``adjoint_pixels``: the same quantity at selected pixels only.
* ``nnz``: the number of (line, centre) pairs inside the footprint support.
* ``n = BOX3`` anywhere a degree is taken: the 3-directional box spline of
  Section III-C (directions e1, e2, e1 + e2); its footprint is the exact line
  integral of the spatial box spline (a hat on a hexagon).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xrt_oracle.c")
# XRT_ORACLE_LIB names another build of the same source (the sanitizer
# build of tests/test_sanitizers.py); by default the library built here
_LIB = os.environ.get("XRT_ORACLE_LIB") or os.path.join(_HERE, "liborc.so")
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined,float-cast-overflow",
                  "-fno-sanitize-recover=all"]

_lib = None


def build(force: bool = True, out: str | None = None, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (IEEE FP64, OpenMP); with sanitize, with
    AddressSanitizer and UndefinedBehaviorSanitizer (into `out`)."""
    lib = out or _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        opt = SANITIZE_FLAGS if sanitize else ["-O2"]
        cmd = ["gcc"] + opt + ["-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, lib)
    return lib


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("spacing", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    gp = ctypes.POINTER(_Grid)
    i64 = ctypes.c_int64
    for name in ("orc_footprint", "orc_footprint_tp", "orc_footprint_gl"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        f.restype = ctypes.c_double
    lib.orc_bspline.argtypes = [ctypes.c_int, ctypes.c_double]
    lib.orc_bspline.restype = ctypes.c_double
    lib.orc_box_spline.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.orc_box_spline.restype = ctypes.c_double
    lib.orc_footprint_box.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.orc_footprint_box.restype = ctypes.c_double
    lib.orc_lines_theta_y.argtypes = [i64, fp, fp, dp, dp, dp]
    lib.orc_lines_endpoints.argtypes = [i64, fp, dp, dp, dp]
    lib.orc_forward.argtypes = [ctypes.c_int, gp, dp, i64, dp, dp, dp, dp, ctypes.c_int]
    lib.orc_forward_dense.argtypes = [ctypes.c_int, gp, dp, i64, dp, dp, dp, dp]
    lib.orc_adjoint.argtypes = [ctypes.c_int, gp, i64, dp, dp, dp, dp, dp, ctypes.c_int]
    lib.orc_adjoint_pixels.argtypes = [ctypes.c_int, gp, i64, dp, dp, dp, dp, i64,
                                       ctypes.POINTER(ctypes.c_int64), dp, ctypes.c_int]
    lib.orc_nnz.argtypes = [ctypes.c_int, gp, i64, dp, dp, dp, ctypes.c_int]
    lib.orc_nnz.restype = ctypes.c_int64
    lib.orc_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _grid(nx, ny, spacing=1.0, cx=0.0, cy=0.0):
    return _Grid(int(nx), int(ny), float(spacing), float(cx), float(cy))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def bspline(n: int, x) -> np.ndarray:
    lib = _load()
    xs = np.atleast_1d(np.asarray(x, dtype=np.float64))
    return np.array([lib.orc_bspline(int(n), float(v)) for v in xs])


BOX3 = 16   # basis code of the 3-directional box spline (directions e1, e2, e1+e2)


def box_spline(x1, x2) -> float:
    """The (uncentred) 3-directional box spline M(x) at one point."""
    return float(_load().orc_box_spline(float(x1), float(x2)))


def footprint(n: int, theta: float, u, method: str = "auto") -> np.ndarray:
    """phi_theta(u) for the tensor B-spline of degree n (or the box spline,
    n = BOX3), FP64."""
    lib = _load()
    f = {"auto": lib.orc_footprint, "tp": lib.orc_footprint_tp,
         "gl": lib.orc_footprint_gl}[method]
    c, s = np.cos(float(theta)), np.sin(float(theta))
    us = np.atleast_1d(np.asarray(u, dtype=np.float64))
    return np.array([f(int(n), c, s, float(v)) for v in us])


def footprint_cs(n: int, c: float, s: float, u, method: str = "auto") -> np.ndarray:
    """phi_theta(u) given cos(theta), sin(theta) directly."""
    lib = _load()
    f = {"auto": lib.orc_footprint, "tp": lib.orc_footprint_tp,
         "gl": lib.orc_footprint_gl}[method]
    us = np.atleast_1d(np.asarray(u, dtype=np.float64))
    return np.array([f(int(n), float(c), float(s), float(v)) for v in us])


def lines_from_theta_y(theta, y):
    """FP64 (cos, sin, y) of lines given as float32 (theta, y) (eq. (1))."""
    lib = _load()
    th = np.ascontiguousarray(theta, dtype=np.float32)
    yy = np.ascontiguousarray(y, dtype=np.float32)
    m = th.size
    c, s, yd = np.empty(m), np.empty(m), np.empty(m)
    lib.orc_lines_theta_y(m, _ptr(th, ctypes.c_float), _ptr(yy, ctypes.c_float),
                          _ptr(c, ctypes.c_double), _ptr(s, ctypes.c_double),
                          _ptr(yd, ctypes.c_double))
    return c, s, yd


def lines_from_endpoints(ep):
    """FP64 (cos, sin, y) of the lines through float32 endpoint pairs [m, 4]."""
    lib = _load()
    e = np.ascontiguousarray(ep, dtype=np.float32).reshape(-1, 4)
    m = e.shape[0]
    c, s, yd = np.empty(m), np.empty(m), np.empty(m)
    rc = lib.orc_lines_endpoints(m, _ptr(e, ctypes.c_float), _ptr(c, ctypes.c_double),
                                 _ptr(s, ctypes.c_double), _ptr(yd, ctypes.c_double))
    if rc != 0:
        raise ValueError("coincident endpoints")
    return c, s, yd


def lines(spec):
    """Accept ('theta_y', theta, y) / ('endpoints', ep) tuples or dicts."""
    if isinstance(spec, dict):
        if spec.get("kind") == "endpoints":
            return lines_from_endpoints(spec["endpoints"])
        return lines_from_theta_y(spec["theta"], spec["y"])
    kind = spec[0]
    if kind == "endpoints":
        return lines_from_endpoints(spec[1])
    return lines_from_theta_y(spec[1], spec[2])


def forward(n, coeffs, line_cs, spacing=1.0, cx=0.0, cy=0.0, nthreads=0, dense=False):
    """Sinogram s_m = P_theta_m{f}(y_m) in FP64; coeffs is [ny, nx]."""
    lib = _load()
    C = np.ascontiguousarray(coeffs, dtype=np.float64)
    ny, nx = C.shape
    c, s, y = (np.ascontiguousarray(v, dtype=np.float64) for v in line_cs)
    m = c.size
    out = np.empty(m)
    g = _grid(nx, ny, spacing, cx, cy)
    if dense:
        rc = lib.orc_forward_dense(int(n), ctypes.byref(g), _ptr(C, ctypes.c_double), m,
                                   _ptr(c, ctypes.c_double), _ptr(s, ctypes.c_double),
                                   _ptr(y, ctypes.c_double), _ptr(out, ctypes.c_double))
    else:
        rc = lib.orc_forward(int(n), ctypes.byref(g), _ptr(C, ctypes.c_double), m,
                             _ptr(c, ctypes.c_double), _ptr(s, ctypes.c_double),
                             _ptr(y, ctypes.c_double), _ptr(out, ctypes.c_double), int(nthreads))
    if rc != 0:
        raise ValueError("oracle forward: invalid arguments")
    return out


def adjoint(n, sino, line_cs, nx, ny, spacing=1.0, cx=0.0, cy=0.0, nthreads=0):
    """Back-projection (H^T s) in FP64 as a [ny, nx] array."""
    lib = _load()
    sv = np.ascontiguousarray(sino, dtype=np.float64)
    c, s, y = (np.ascontiguousarray(v, dtype=np.float64) for v in line_cs)
    out = np.empty((ny, nx))
    g = _grid(nx, ny, spacing, cx, cy)
    rc = lib.orc_adjoint(int(n), ctypes.byref(g), c.size, _ptr(c, ctypes.c_double),
                         _ptr(s, ctypes.c_double), _ptr(y, ctypes.c_double),
                         _ptr(sv, ctypes.c_double), _ptr(out, ctypes.c_double), int(nthreads))
    if rc != 0:
        raise ValueError("oracle adjoint: invalid arguments")
    return out


def adjoint_pixels(n, sino, line_cs, nx, ny, pix, spacing=1.0, cx=0.0, cy=0.0, nthreads=0):
    """(H^T s) at flat pixel indices ``pix`` (j*nx + i), FP64."""
    lib = _load()
    sv = np.ascontiguousarray(sino, dtype=np.float64)
    c, s, y = (np.ascontiguousarray(v, dtype=np.float64) for v in line_cs)
    p = np.ascontiguousarray(pix, dtype=np.int64)
    out = np.empty(p.size)
    g = _grid(nx, ny, spacing, cx, cy)
    rc = lib.orc_adjoint_pixels(int(n), ctypes.byref(g), c.size, _ptr(c, ctypes.c_double),
                                _ptr(s, ctypes.c_double), _ptr(y, ctypes.c_double),
                                _ptr(sv, ctypes.c_double), p.size, _ptr(p, ctypes.c_int64),
                                _ptr(out, ctypes.c_double), int(nthreads))
    if rc != 0:
        raise ValueError("oracle adjoint_pixels: invalid arguments")
    return out


def nnz(n, line_cs, nx, ny, spacing=1.0, cx=0.0, cy=0.0, nthreads=0) -> int:
    """Structural nonzeros of H (pairs with |u| < w)."""
    lib = _load()
    c, s, y = (np.ascontiguousarray(v, dtype=np.float64) for v in line_cs)
    g = _grid(nx, ny, spacing, cx, cy)
    return int(lib.orc_nnz(int(n), ctypes.byref(g), c.size, _ptr(c, ctypes.c_double),
                           _ptr(s, ctypes.c_double), _ptr(y, ctypes.c_double), int(nthreads)))
