"""Torch-facing wrappers: tensors in, tensors out, on the current HIP stream.

These only check shapes/dtypes/devices and pass device pointers and the
current stream to libxrt.so; every step of the computation runs in the
library's kernels.
"""
from __future__ import annotations

import torch

from . import _lib as L

# basis code of the 3-directional box spline (degrees 0..3 are the tensor B-splines)
BOX3 = L.XRT_BOX3


def _stream() -> int:
    return int(torch.cuda.current_stream().cuda_stream)


def _check(t: torch.Tensor, name: str, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def make_grid(nx: int, ny: int, spacing: float = 1.0, cx: float = 0.0, cy: float = 0.0):
    return L.XrtGrid(int(nx), int(ny), float(spacing), float(cx), float(cy))


class Lines:
    """A device-resident line list: (theta, y) pairs or endpoint pairs."""

    def __init__(self, theta=None, y=None, endpoints=None, device="cuda"):
        if endpoints is not None:
            ep = torch.as_tensor(endpoints, dtype=torch.float32, device=device).contiguous()
            if ep.dim() != 2 or ep.shape[1] != 4:
                raise ValueError("endpoints must be [n, 4]")
            self.kind = L.XRT_LINES_ENDPOINTS
            self.endpoints = ep
            self.n = ep.shape[0]
            self._refs = (ep,)
            self.c = L.XrtLines(self.kind, self.n, None, None, ep.data_ptr() if self.n else None)
        else:
            th = torch.as_tensor(theta, dtype=torch.float32, device=device).contiguous().view(-1)
            yy = torch.as_tensor(y, dtype=torch.float32, device=device).contiguous().view(-1)
            if th.shape != yy.shape:
                raise ValueError("theta and y must have the same length")
            self.kind = L.XRT_LINES_THETA_Y
            self.theta, self.y = th, yy
            self.n = th.shape[0]
            self._refs = (th, yy)
            self.c = L.XrtLines(self.kind, self.n, th.data_ptr() if self.n else None,
                                yy.data_ptr() if self.n else None, None)

    @staticmethod
    def from_spec(spec: dict, device="cuda") -> "Lines":
        if spec["kind"] == "endpoints":
            return Lines(endpoints=spec["endpoints"], device=device)
        return Lines(theta=spec["theta"], y=spec["y"], device=device)


def forward(coeffs: torch.Tensor, lines: Lines, degree: int, spacing=1.0, cx=0.0, cy=0.0):
    _check(coeffs, "coeffs")
    ny, nx = coeffs.shape
    out = torch.empty(lines.n, dtype=torch.float32, device=coeffs.device)
    st = L.xrt_forward(coeffs.data_ptr(), make_grid(nx, ny, spacing, cx, cy), degree, lines.c,
                       out.data_ptr() if lines.n else None, _stream())
    L.check(st, "xrt_forward")
    return out


def adjoint(sino: torch.Tensor, lines: Lines, degree: int, nx: int, ny: int, spacing=1.0,
            cx=0.0, cy=0.0):
    _check(sino, "sino", (lines.n,))
    out = torch.empty((ny, nx), dtype=torch.float32, device=sino.device)
    st = L.xrt_adjoint(sino.data_ptr() if lines.n else None, lines.c, degree,
                       make_grid(nx, ny, spacing, cx, cy), out.data_ptr(), _stream())
    L.check(st, "xrt_adjoint")
    return out


class Plan:
    """Plan for a fixed (grid, degree, line list): forward / adjoint without
    host synchronisation or allocation of library memory."""

    def __init__(self, nx: int, ny: int, degree: int, lines: Lines, spacing=1.0, cx=0.0, cy=0.0):
        self.nx, self.ny, self.degree = int(nx), int(ny), int(degree)
        self.lines = lines
        self.grid = make_grid(nx, ny, spacing, cx, cy)
        st, h = L.xrt_plan_create(self.grid, degree, lines.c, _stream())
        L.check(st, "xrt_plan_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def forward(self, coeffs: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _check(coeffs, "coeffs", (self.ny, self.nx))
        if out is None:
            out = torch.empty(self.lines.n, dtype=torch.float32, device=coeffs.device)
        _check(out, "out", (self.lines.n,))
        L.check(L.xrt_plan_forward(self._h, coeffs.data_ptr(),
                                   out.data_ptr() if self.lines.n else None, _stream()),
                "xrt_plan_forward")
        return out

    def adjoint(self, sino: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _check(sino, "sino", (self.lines.n,))
        if out is None:
            out = torch.empty((self.ny, self.nx), dtype=torch.float32, device=sino.device)
        _check(out, "out", (self.ny, self.nx))
        L.check(L.xrt_plan_adjoint(self._h, sino.data_ptr() if self.lines.n else None,
                                   out.data_ptr(), _stream()), "xrt_plan_adjoint")
        return out

    def info(self):
        st, n, nc = L.xrt_plan_info(self._h)
        L.check(st, "xrt_plan_info")
        return n, nc

    def nnz(self) -> int:
        st, v = L.xrt_plan_nnz(self._h, _stream())
        L.check(st, "xrt_plan_nnz")
        return v

    def close(self):
        if getattr(self, "_h", None):
            L.xrt_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Project(torch.autograd.Function):
    """s = H c as a differentiable operation: the backward pass is the exact
    adjoint, grad_c = H^T grad_s (the matched back-projection).  The plan
    (geometry, degree) is not differentiable."""

    @staticmethod
    def forward(ctx, coeffs: torch.Tensor, plan: "Plan") -> torch.Tensor:
        ctx.plan = plan
        return plan.forward(coeffs.contiguous())

    @staticmethod
    def backward(ctx, grad_sino: torch.Tensor):
        return ctx.plan.adjoint(grad_sino.contiguous()), None


class BackProject(torch.autograd.Function):
    """c = H^T s as a differentiable operation (its backward is H)."""

    @staticmethod
    def forward(ctx, sino: torch.Tensor, plan: "Plan") -> torch.Tensor:
        ctx.plan = plan
        return plan.adjoint(sino.contiguous())

    @staticmethod
    def backward(ctx, grad_coeffs: torch.Tensor):
        return ctx.plan.forward(grad_coeffs.contiguous()), None


def project(coeffs: torch.Tensor, plan: "Plan") -> torch.Tensor:
    return Project.apply(coeffs, plan)


def backproject(sino: torch.Tensor, plan: "Plan") -> torch.Tensor:
    return BackProject.apply(sino, plan)
