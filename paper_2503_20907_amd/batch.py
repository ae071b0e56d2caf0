"""Batches of x-ray transform problems on torch tensors (include/xrt_batch.h).

Argument marshalling only: plans, buffers, the persistent launches, the
graph capture and the autotuner are in libxrt.so.  Each problem's buffers are
device memory owned by the batch; ``coeffs(p)``, ``sino(p)`` and ``back(p)``
return torch views of them (valid while the batch is open).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .ops import Lines, _stream, make_grid


class _Ext:
    """A device range owned by the library, exposed through
    __cuda_array_interface__ so that torch can view it without copying."""

    def __init__(self, ptr: int, shape):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": "<f4", "data": (ptr, False),
                                         "version": 2, "strides": None}


class Batch:
    def __init__(self, problems):
        """problems: list of (nx, ny, degree, Lines[, spacing, cx, cy])."""
        self._keep = []
        arr = []
        self.shapes = []
        for pr in problems:
            nx, ny, degree, lines = pr[:4]
            spacing = pr[4] if len(pr) > 4 else 1.0
            cx = pr[5] if len(pr) > 5 else 0.0
            cy = pr[6] if len(pr) > 6 else 0.0
            self._keep.append(lines)
            arr.append(L.XrtProblem(make_grid(nx, ny, spacing, cx, cy), int(degree), lines.c))
            self.shapes.append((int(ny), int(nx), int(lines.n)))
        st, h = L.xrt_batch_create(arr, _stream())
        L.check(st, "xrt_batch_create")
        self._h = h
        self._bufs = []
        for p, (ny, nx, m) in enumerate(self.shapes):
            st, c, s, k = L.xrt_batch_buffers(h, p)
            L.check(st, "xrt_batch_buffers")
            self._bufs.append((torch.as_tensor(_Ext(c, (ny, nx)), device="cuda"),
                               torch.as_tensor(_Ext(s, (m,)), device="cuda") if m else
                               torch.empty(0, device="cuda"),
                               torch.as_tensor(_Ext(k, (ny, nx)), device="cuda")))

    def __len__(self):
        return len(self.shapes)

    def coeffs(self, p: int) -> torch.Tensor:
        return self._bufs[p][0]

    def sino(self, p: int) -> torch.Tensor:
        return self._bufs[p][1]

    def back(self, p: int) -> torch.Tensor:
        return self._bufs[p][2]

    def info(self):
        st, n, f, a = L.xrt_batch_info(self._h)
        L.check(st, "xrt_batch_info")
        return {"lines": n, "forward_items": f, "adjoint_items": a}

    def forward(self):
        L.check(L.xrt_batch_forward(self._h, _stream()), "xrt_batch_forward")

    def adjoint(self):
        L.check(L.xrt_batch_adjoint(self._h, _stream()), "xrt_batch_adjoint")

    def run(self, graph: bool = False):
        L.check(L.xrt_batch_run(self._h, int(graph), _stream()), "xrt_batch_run")

    @property
    def config(self) -> dict:
        st, c = L.xrt_batch_get_config(self._h)
        L.check(st, "xrt_batch_get_config")
        return {"fwd_blocks_per_cu": c.fwd_blocks_per_cu, "lines_per_item": c.lines_per_item,
                "adj_blocks_per_cu": c.adj_blocks_per_cu}

    def set_config(self, fwd_blocks_per_cu: int, lines_per_item: int, adj_blocks_per_cu: int):
        c = L.XrtBatchConfig(int(fwd_blocks_per_cu), int(lines_per_item), int(adj_blocks_per_cu), 0)
        L.check(L.xrt_batch_set_config(self._h, c), "xrt_batch_set_config")

    def autotune(self, reps: int = 3) -> dict:
        st, c = L.xrt_batch_autotune(self._h, reps, _stream())
        L.check(st, "xrt_batch_autotune")
        return {"fwd_blocks_per_cu": c.fwd_blocks_per_cu, "lines_per_item": c.lines_per_item,
                "adj_blocks_per_cu": c.adj_blocks_per_cu}

    def close(self):
        if getattr(self, "_h", None):
            self._bufs = []
            L.xrt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
