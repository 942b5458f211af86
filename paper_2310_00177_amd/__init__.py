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
                   NPS_MIXED_FP16 as MIXED_FP16, NPS_NPSDO as NPSDO, NPS_PCG as PCG, NPS_FPCG as FPCG,
                   STATUS_NAMES)

__all__ = ["Net", "solve", "apply_laplacian", "apply_precond", "apply_precond_noalloc", "apply_precond_transpose", "asymmetry", "lanczos", "ritz_rhs", "NpsError", "SolveInfo", "Server",
           "train_workspace", "net_forward", "net_backward", "train_loss", "train_step", "Precond", "TrainLoss",
           "FP64", "FP32", "MIXED_BF16", "MIXED_FP16", "NPSDO", "PCG", "FPCG", "workspace", "vector_dtype"]


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
    t_setup_ms: float = 0.0
    t_iter_ms: float = 0.0

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
          n_ortho: int | None = None, precision: int = FP32, fixed_iters: bool = False,
          x: torch.Tensor | None = None, ws: torch.Tensor | None = None, check: bool = True, method: int = 0,
          symmetric: bool = False):
    """x, info = solve(...): labels uint8 (nz,ny,nx), b float64, both on device.

    method: NPSDO (default; n_ortho defaults to 2), PCG or FPCG (n_ortho 1).
    symmetric: precondition with P^T o P instead of P.
    Soft statuses (NPS_NOT_CONVERGED) are returned in info; hard errors raise
    NpsError when check is true.
    """
    if n_ortho is None:
        n_ortho = 2 if method == NPSDO else 1
    _check_device(labels, b)
    if labels.dtype != torch.uint8 or b.dtype != torch.float64:
        raise ValueError("labels must be uint8 and b float64")
    if x is None:
        x = torch.empty_like(b)
    opts = _lib.nps_opts(tol, max_iter, n_ortho, precision, 1 if fixed_iters else 0, method,
                         1 if symmetric else 0)
    if ws is None:
        nbytes = _lib.nps_solve_workspace_bytes(_dims(labels.shape), net.levels, opts)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=labels.device)
    info = _lib.nps_info()
    ws_bytes = ws.numel() - (_aligned(ws) - ws.data_ptr())
    rc = _lib.nps_solve(net.handle, labels.data_ptr(), _dims(labels.shape), b.data_ptr(), x.data_ptr(),
                        opts, info, _aligned(ws), ws_bytes, _stream())
    if rc < 0 and check and rc != _lib.NPS_EBREAKDOWN:
        raise NpsError(rc, "nps_solve")
    return x, SolveInfo(info.iterations, rc, info.rel_residual, info.rel_residual_rec,
                        info.refinements, info.n_fluid, info.t_setup_ms, info.t_iter_ms)


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


def apply_precond_noalloc(net: Net, labels: torch.Tensor, r: torch.Tensor, precision: int | None = None,
                          d: torch.Tensor | None = None) -> torch.Tensor:
    """d = P(I, r) with the library's static scratch (nps_apply_precond_noalloc:
    the library allocates nothing; pass d to allocate nothing here either)."""
    _check_device(labels, r)
    if precision is None:
        precision = FP64 if r.dtype == torch.float64 else FP32
    if r.dtype != vector_dtype(precision):
        raise ValueError(f"r must be {vector_dtype(precision)} for precision {precision}")
    d = torch.empty_like(r) if d is None else d
    rc = _lib.nps_apply_precond_noalloc(net.handle, labels.data_ptr(), _dims(labels.shape), r.data_ptr(),
                                        d.data_ptr(), precision, _stream())
    if rc != _lib.NPS_OK:
        raise NpsError(rc, "nps_apply_precond_noalloc")
    return d


def apply_precond_transpose(net: Net, labels: torch.Tensor, g: torch.Tensor,
                            ws: torch.Tensor | None = None) -> torch.Tensor:
    """y = P(I, .)^T g (float64 or float32 vectors)."""
    _check_device(labels, g)
    prec = FP64 if g.dtype == torch.float64 else FP32
    if g.dtype not in (torch.float64, torch.float32):
        raise ValueError("g must be float64 or float32")
    if ws is None:
        ws = train_workspace(labels.shape, net.levels, prec, device=labels.device)
    y = torch.empty_like(g)
    wp, wb = _ws_args(ws)
    rc = _lib.nps_apply_precond_transpose(net.handle, labels.data_ptr(), _dims(labels.shape), g.data_ptr(),
                                          y.data_ptr(), prec, wp, wb, _stream())
    if rc != _lib.NPS_OK:
        raise NpsError(rc, "nps_apply_precond_transpose")
    return y


def asymmetry(net: Net, labels: torch.Tensor, x: torch.Tensor, y: torch.Tensor, precision: int | None = None,
              ws: torch.Tensor | None = None) -> float:
    """S(x, y) = |x.P(y) - y.P(x)| / sqrt(|x.P(x)| |y.P(y)|) on the GPU."""
    _check_device(labels, x)
    if precision is None:
        precision = FP64 if x.dtype == torch.float64 else FP32
    if x.dtype != vector_dtype(precision) or y.dtype != x.dtype:
        raise ValueError(f"x and y must be {vector_dtype(precision)} for precision {precision}")
    if ws is None:
        ws = workspace(labels.shape, net.levels, precision, 0, device=labels.device)
    px, py = torch.empty_like(x), torch.empty_like(y)
    wp, wb = _ws_args(ws)
    rc, val = _lib.nps_asymmetry(net.handle, labels.data_ptr(), _dims(labels.shape), x.data_ptr(), y.data_ptr(),
                                 px.data_ptr(), py.data_ptr(), precision, wp, wb, _stream())
    if rc != _lib.NPS_OK:
        raise NpsError(rc, "nps_asymmetry")
    return val


def lanczos(labels: torch.Tensor, v0: torch.Tensor, m: int, reorth: bool = True):
    """V, alpha, beta, steps = lanczos(labels, v0, m): m Lanczos steps on A~,
    with full reorthogonalisation unless reorth is false (float64).  V has
    shape (m, nz, ny, nx)."""
    _check_device(labels, v0)
    if v0.dtype != torch.float64:
        raise ValueError("v0 must be float64")
    dims = _dims(labels.shape)
    V = torch.empty((m,) + tuple(labels.shape), dtype=torch.float64, device=labels.device)
    alpha = torch.empty(m, dtype=torch.float64, device=labels.device)
    beta = torch.empty(m, dtype=torch.float64, device=labels.device)
    ws = torch.empty(_lib.nps_lanczos_workspace_bytes(dims, m) + 256, dtype=torch.uint8, device=labels.device)
    wp, wb = _ws_args(ws)
    rc, steps = _lib.nps_lanczos(labels.data_ptr(), dims, m, 1 if reorth else 0, v0.data_ptr(), V.data_ptr(),
                                 alpha.data_ptr(), beta.data_ptr(), wp, wb, _stream())
    if rc != _lib.NPS_OK:
        raise NpsError(rc, "nps_lanczos")
    return V, alpha, beta, steps


def ritz_rhs(V: torch.Tensor, alpha: torch.Tensor, beta: torch.Tensor, coef: torch.Tensor):
    """rhs, theta = ritz_rhs(V, alpha, beta, coef): coef has shape (m, k);
    rhs has shape (k, nz, ny, nx), unit-norm normalised Ritz combinations."""
    m = V.shape[0]
    if coef.shape[0] != m or coef.dtype != torch.float64:
        raise ValueError("coef must be float64 of shape (m, k)")
    k = coef.shape[1]
    shape = tuple(V.shape[1:])
    cm = coef.t().contiguous()                      # column-major (m x k)
    rhs = torch.empty((k,) + shape, dtype=torch.float64, device=V.device)
    theta = torch.empty(m, dtype=torch.float64, device=V.device)
    ws = torch.empty(_lib.nps_ritz_workspace_bytes(m, k) + 256, dtype=torch.uint8, device=V.device)
    wp, wb = _ws_args(ws)
    rc = _lib.nps_ritz_rhs(V.data_ptr(), _dims(shape), m, alpha.data_ptr(), beta.data_ptr(), cm.data_ptr(), k,
                           rhs.data_ptr(), theta.data_ptr(), wp, wb, _stream())
    if rc != _lib.NPS_OK:
        raise NpsError(rc, "nps_ritz_rhs")
    return rhs, theta


class Server:
    """Continuous-batching request server (nps_server_* in the C ABI).

    submit() queues a request (the server keeps a reference to its host
    arrays, which must not be modified until the request is polled); step()
    admits requests by HBM footprint and advances every admitted one by at most
    one iteration on its own stream; poll() returns (x, info, latency_ms) once
    a request has finished, else None.
    """

    def __init__(self, net: Net, hbm_budget: int, max_slots: int = 8):
        self.net = net   # keeps the network alive
        rc, h = _lib.nps_server_create(net.handle, int(hbm_budget), int(max_slots))
        if rc != _lib.NPS_OK:
            raise NpsError(rc, "nps_server_create")
        self.handle = h
        self._held = {}   # request id -> the host arrays the library reads at admission

    def request_bytes(self, shape, tol=1e-6, max_iter=1000, n_ortho=2, precision=MIXED_BF16, method=0) -> int:
        opts = _lib.nps_opts(tol, max_iter, n_ortho, precision, 0, method, 0)
        return _lib.nps_server_request_bytes(self.handle, _dims(shape), opts)

    def submit(self, labels: np.ndarray, b: np.ndarray, tol: float = 1e-6, max_iter: int = 1000,
               n_ortho: int = 2, precision: int = MIXED_BF16, fixed_iters: bool = False, method: int = 0) -> int:
        lab = np.ascontiguousarray(labels, dtype=np.uint8)
        bb = np.ascontiguousarray(b, dtype=np.float64)
        if lab.shape != bb.shape or lab.ndim != 3:
            raise ValueError("labels and b must be (nz, ny, nx) arrays of one shape")
        opts = _lib.nps_opts(tol, max_iter, n_ortho, precision, 1 if fixed_iters else 0, method, 0)
        rc, rid = _lib.nps_server_submit(self.handle, lab.ctypes.data, _dims(lab.shape), bb.ctypes.data, opts)
        if rc != _lib.NPS_OK:
            raise NpsError(rc, "nps_server_submit")
        self._held[rid] = (lab, bb)
        return rid

    def step(self) -> tuple:
        rc, active, queued = _lib.nps_server_step(self.handle)
        if rc != _lib.NPS_OK:
            raise NpsError(rc, "nps_server_step")
        return active, queued

    def poll(self, rid: int):
        x = np.empty(self._held[rid][0].shape, dtype=np.float64)
        info = _lib.nps_info()
        rc, lat = _lib.nps_server_poll(self.handle, rid, x.ctypes.data, info)
        if rc == _lib.NPS_PENDING:
            return None
        del self._held[rid]
        if rc < 0 and rc != _lib.NPS_EBREAKDOWN:
            x = None   # rejected before its solve ran: no solution
        return x, SolveInfo(info.iterations, rc, info.rel_residual, info.rel_residual_rec, info.refinements,
                            info.n_fluid), lat

    def close(self):
        h = getattr(self, "handle", None)
        if h:
            _lib.nps_server_destroy(h)
            self.handle = None
        self._held = {}

    def __del__(self):
        self.close()


# ---------------------------------------------------------------------------
# training (loss of Sec. "Training")
# ---------------------------------------------------------------------------
def train_workspace(shape, levels: int, precision: int, device="cuda") -> torch.Tensor:
    nbytes = _lib.nps_train_workspace_bytes(_dims(shape), levels, precision)
    return torch.empty(nbytes + 256, dtype=torch.uint8, device=device)


def _ws_args(ws: torch.Tensor):
    return _aligned(ws), ws.numel() - (_aligned(ws) - ws.data_ptr())


def _train_precision(t: torch.Tensor, precision: int | None) -> int:
    prec = (FP64 if t.dtype == torch.float64 else FP32) if precision is None else precision
    if t.dtype != vector_dtype(prec):
        raise ValueError(f"vectors must be {vector_dtype(prec)} for training precision {prec}")
    return prec


def net_forward(net: Net, labels: torch.Tensor, r: torch.Tensor, ws: torch.Tensor,
                precision: int | None = None) -> torch.Tensor:
    """y = P(I, r); the activations stay in ws for net_backward.  precision:
    FP64, FP32 or MIXED_BF16 (default from r's dtype)."""
    _check_device(labels, r)
    prec = _train_precision(r, precision)
    y = torch.empty_like(r)
    wp, wb = _ws_args(ws)
    rc = _lib.nps_net_forward(net.handle, labels.data_ptr(), _dims(labels.shape), r.data_ptr(), y.data_ptr(), prec,
                              wp, wb, _stream())
    if rc != _lib.NPS_OK:
        raise NpsError(rc, "nps_net_forward")
    return y


def train_loss(labels: torch.Tensor, b: torch.Tensor, y: torch.Tensor, levels: int, ws: torch.Tensor,
               precision: int | None = None):
    """(loss, dL/dy) of || b - A y ||_2."""
    _check_device(labels, b, y)
    prec = _train_precision(y, precision)
    gy = torch.empty_like(y)
    wp, wb = _ws_args(ws)
    rc, loss = _lib.nps_train_loss(labels.data_ptr(), _dims(labels.shape), levels, b.data_ptr(), y.data_ptr(),
                                   gy.data_ptr(), prec, wp, wb, _stream())
    if rc != _lib.NPS_OK:
        raise NpsError(rc, "nps_train_loss")
    return loss, gy


def net_backward(net: Net, labels: torch.Tensor, r: torch.Tensor, gy: torch.Tensor, grad: torch.Tensor,
                 ws: torch.Tensor, precision: int | None = None) -> torch.Tensor:
    """grad += dL/dparams (float64 device tensor of nps_param_count entries)."""
    _check_device(labels, r, gy, grad)
    prec = _train_precision(r, precision)
    wp, wb = _ws_args(ws)
    rc = _lib.nps_net_backward(net.handle, labels.data_ptr(), _dims(labels.shape), r.data_ptr(), gy.data_ptr(),
                               grad.data_ptr(), prec, wp, wb, _stream())
    if rc != _lib.NPS_OK:
        raise NpsError(rc, "nps_net_backward")
    return grad


_net_cache: list = [None]   # (weak reference to the params tensor, its version, levels, device, Net)


def _cached_net(params: torch.Tensor, levels: int, device) -> Net:
    """The device network of a parameter tensor, rebuilt only when another
    tensor is passed, the tensor was modified in place (its version counter
    moved) or the level count or device changed."""
    import weakref
    c = _net_cache[0]
    if c is not None and c[0]() is params and c[1:4] == (params._version, levels, str(device)):
        return c[4]
    net = Net(params.detach().cpu().numpy(), levels, device=device)
    _net_cache[0] = (weakref.ref(params), params._version, levels, str(device), net)
    return net


def train_step(net: Net, labels: torch.Tensor, b: torch.Tensor, grad: torch.Tensor, ws: torch.Tensor,
               precision: int | None = None) -> float:
    """One step over a batch (nps_train_step): labels uint8 (B, nz, ny, nx),
    b (B, nz, ny, nx) float64 / float32; grad += d(mean loss)/dparams; returns
    the mean loss.  ws: train_workspace of one system."""
    _check_device(labels, b, grad)
    if labels.dim() != 4 or labels.shape != b.shape or labels.dtype != torch.uint8:
        raise ValueError("labels (uint8) and b must both have shape (batch, nz, ny, nx)")
    prec = _train_precision(b, precision)
    wp, wb = _ws_args(ws)
    rc, loss = _lib.nps_train_step(net.handle, labels.data_ptr(), _dims(labels.shape[1:]), labels.shape[0],
                                   b.data_ptr(), grad.data_ptr(), prec, wp, wb, _stream())
    if rc != _lib.NPS_OK:
        raise NpsError(rc, "nps_train_step")
    return loss


class Precond(torch.autograd.Function):
    """y = P(I, r) with the library's forward and hand-written backward.

    params: float64 tensor (nps_param_count(levels)); gradients flow to it
    (nps_net_backward) and to r (P is linear in r: dL/dr = P^T dL/dy, the
    library's adjoint).  Each call keeps its own activation workspace until
    backward."""

    @staticmethod
    def forward(ctx, params, labels, r, levels):
        net = _cached_net(params, levels, r.device)
        ws = train_workspace(labels.shape, levels, FP64 if r.dtype == torch.float64 else FP32, device=r.device)
        y = net_forward(net, labels, r.contiguous(), ws)
        ctx.net, ctx.ws, ctx.labels, ctx.levels = net, ws, labels, levels
        ctx.save_for_backward(r)
        return y

    @staticmethod
    def backward(ctx, gy):
        (r,) = ctx.saved_tensors
        gy = gy.contiguous().to(r.dtype)
        grad = None
        if ctx.needs_input_grad[0]:
            grad = torch.zeros(_lib.nps_param_count(ctx.levels), dtype=torch.float64, device=r.device)
            net_backward(ctx.net, ctx.labels, r.contiguous(), gy, grad, ctx.ws)
        gr = apply_precond_transpose(ctx.net, ctx.labels, gy, ws=ctx.ws) if ctx.needs_input_grad[2] else None
        ctx.ws = None
        return grad, None, gr, None


class TrainLoss(torch.autograd.Function):
    """loss = || b - A y ||_2 (A the mixed-BC matrix of the labels).
    Differentiable in y only: b is data."""

    @staticmethod
    def forward(ctx, y, labels, b, levels):
        if b.requires_grad:
            raise NotImplementedError("TrainLoss has no gradient with respect to b")
        ws = train_workspace(labels.shape, levels, FP64 if y.dtype == torch.float64 else FP32, device=y.device)
        loss, gy = train_loss(labels, b.contiguous(), y.contiguous(), levels, ws)
        ctx.save_for_backward(gy)
        return torch.tensor(loss, dtype=torch.float64, device=y.device)

    @staticmethod
    def backward(ctx, gl):
        (gy,) = ctx.saved_tensors
        return gy * gl.to(gy.dtype), None, None, None
