"""MI355X-native neural-preconditioned Poisson solver (arXiv 2310.00177).

The solve runs entirely in the HIP library libnps.so (C ABI in include/nps.h);
this package only marshals torch device tensors into its calls.  PyTorch
provides device memory and the current HIP stream, nothing else.

    import paper_2310_00177_amd as nps
    net = nps.Net(params, levels=6)                 # float64 blob, host
    x, info = nps.solve(net, labels, b, tol=1e-6, precision=nps.FP32)
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import _lib
from ._lib import (NPS_FP64 as FP64, NPS_FP32 as FP32, NPS_MIXED_BF16 as MIXED_BF16,  # noqa: F401
                   NPS_MIXED_FP16 as MIXED_FP16, STATUS_NAMES)

__all__ = ["Net", "solve", "apply_laplacian", "apply_precond", "NpsError", "SolveInfo",
           "FP64", "FP32", "MIXED_BF16", "MIXED_FP16", "workspace", "vector_dtype"]


class NpsError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {_lib.nps_last_error()}")


@dataclasses.dataclass
class SolveInfo:
    iterations: int
    status: int
    rel_residual: float
    rel_residual_rec: float
    refinements: int
    n_fluid: int

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dims(shape) -> _lib.nps_dims:
    nz, ny, nx = (int(s) for s in shape)
    return _lib.nps_dims(nz, ny, nx)


def _check_device(*ts):
    for t in ts:
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("tensors must be contiguous device tensors")


def vector_dtype(precision: int) -> torch.dtype:
    return torch.float64 if precision == FP64 else torch.float32


def workspace(shape, levels: int, precision: int, n_ortho: int = 2, device="cuda") -> torch.Tensor:
    """Device workspace for nps_solve / nps_apply_precond (256 bytes of slack for alignment).

    nps_workspace_bytes returns 0 for arguments the library rejects; the
    returned minimal buffer then lets the solve call report the precise error.
    """
    nbytes = _lib.nps_workspace_bytes(_dims(shape), levels, precision, n_ortho)
    return torch.empty(nbytes + 256, dtype=torch.uint8, device=device)


def _aligned(buf: torch.Tensor) -> int:
    p = buf.data_ptr()
    return (p + 255) & ~255


class Net:
    """A network (Alg. 2 weights) resident on the current device."""

    def __init__(self, params, levels: int = 6, device="cuda"):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
        nbytes = _lib.nps_net_bytes(levels)
        if nbytes == 0:
            raise NpsError(_lib.NPS_EINVAL, "nps_net_bytes")
        self.levels = levels
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        rc, handle = _lib.nps_net_create(p.ctypes.data, p.size, levels, _aligned(self._buf), nbytes, _stream())
        if rc != _lib.NPS_OK:
            raise NpsError(rc, "nps_net_create")
        self.handle = handle

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            _lib.nps_net_destroy(h)
            self.handle = None


def solve(net: Net, labels: torch.Tensor, b: torch.Tensor, tol: float = 1e-6, max_iter: int = 1000,
          n_ortho: int = 2, precision: int = FP32, refine_every: int = 20, fixed_iters: bool = False,
          x: torch.Tensor | None = None, ws: torch.Tensor | None = None, check: bool = True):
    """x, info = solve(...): labels uint8 (nz,ny,nx), b float64, both on device.

    Soft statuses (NPS_NOT_CONVERGED) are returned in info; hard errors raise
    NpsError when check is true.
    """
    _check_device(labels, b)
    if labels.dtype != torch.uint8 or b.dtype != torch.float64:
        raise ValueError("labels must be uint8 and b float64")
    if x is None:
        x = torch.empty_like(b)
    if ws is None:
        ws = workspace(labels.shape, net.levels, precision, n_ortho, device=labels.device)
    opts = _lib.nps_opts(tol, max_iter, n_ortho, precision, refine_every, 1 if fixed_iters else 0)
    info = _lib.nps_info()
    ws_bytes = ws.numel() - (_aligned(ws) - ws.data_ptr())
    rc = _lib.nps_solve(net.handle, labels.data_ptr(), _dims(labels.shape), b.data_ptr(), x.data_ptr(),
                        opts, info, _aligned(ws), ws_bytes, _stream())
    if rc < 0 and check and rc != _lib.NPS_EBREAKDOWN:
        raise NpsError(rc, "nps_solve")
    return x, SolveInfo(info.iterations, rc, info.rel_residual, info.rel_residual_rec,
                        info.refinements, info.n_fluid)


def apply_laplacian(labels: torch.Tensor, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    """y = A x with the library's stencil kernel (float64 or float32)."""
    _check_device(labels, x)
    prec = FP64 if x.dtype == torch.float64 else FP32
    if x.dtype not in (torch.float64, torch.float32):
        raise ValueError("x must be float64 or float32")
    y = torch.empty_like(x) if y is None else y
    rc = _lib.nps_apply_laplacian(labels.data_ptr(), _dims(labels.shape), x.data_ptr(), y.data_ptr(), prec,
                                  _stream())
    if rc != _lib.NPS_OK:
        raise NpsError(rc, "nps_apply_laplacian")
    return y


def apply_precond(net: Net, labels: torch.Tensor, r: torch.Tensor, precision: int | None = None,
                  ws: torch.Tensor | None = None) -> torch.Tensor:
    """d = P(I, r): one network evaluation with the solve's kernels."""
    _check_device(labels, r)
    if precision is None:
        precision = FP64 if r.dtype == torch.float64 else FP32
    if r.dtype != vector_dtype(precision):
        raise ValueError(f"r must be {vector_dtype(precision)} for precision {precision}")
    if ws is None:
        ws = workspace(labels.shape, net.levels, precision, 0, device=labels.device)
    d = torch.empty_like(r)
    ws_bytes = ws.numel() - (_aligned(ws) - ws.data_ptr())
    rc = _lib.nps_apply_precond(net.handle, labels.data_ptr(), _dims(labels.shape), r.data_ptr(), d.data_ptr(),
                                precision, _aligned(ws), ws_bytes, _stream())
    if rc != _lib.NPS_OK:
        raise NpsError(rc, "nps_apply_precond")
    return d
