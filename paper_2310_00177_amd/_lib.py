"""ctypes binding of libnps.so: one Python function per C-ABI entry point,
same names, argument marshalling only (the declarations live in include/nps.h).

Importing this module loads the library; if libnps.so is missing it raises,
so nothing silently falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnps.so")

# enum nps_status
NPS_OK, NPS_NOT_CONVERGED = 0, 1
NPS_EINVAL, NPS_ESHAPE, NPS_ELABEL, NPS_ENOFLUID = -1, -2, -3, -4
NPS_ENONFINITE, NPS_EBREAKDOWN, NPS_ENOMEM, NPS_EDEVICE = -5, -6, -7, -8
# enum nps_precision
NPS_FP64, NPS_FP32, NPS_MIXED_BF16, NPS_MIXED_FP16 = 0, 1, 2, 3
NPS_NPSDO, NPS_PCG, NPS_FPCG = 0, 1, 2
# enum nps_label
NPS_FLUID, NPS_AIR, NPS_SOLID = 0, 1, 2

STATUS_NAMES = {
    0: "NPS_OK", 1: "NPS_NOT_CONVERGED", -1: "NPS_EINVAL", -2: "NPS_ESHAPE", -3: "NPS_ELABEL",
    -4: "NPS_ENOFLUID", -5: "NPS_ENONFINITE", -6: "NPS_EBREAKDOWN", -7: "NPS_ENOMEM", -8: "NPS_EDEVICE",
}


class nps_dims(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int), ("ny", ctypes.c_int), ("nx", ctypes.c_int)]


class nps_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("n_ortho", ctypes.c_int),
                ("precision", ctypes.c_int), ("fixed_iters", ctypes.c_int),
                ("method", ctypes.c_int), ("symmetric", ctypes.c_int)]


class nps_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("status", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("rel_residual_rec", ctypes.c_double), ("refinements", ctypes.c_int), ("n_fluid", ctypes.c_int),
                ("t_setup_ms", ctypes.c_double), ("t_iter_ms", ctypes.c_double)]


class nps_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int), ("total_ms", ctypes.c_double),
                ("cells", ctypes.c_double)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_2310_00177_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)
_vp, _sz, _int = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int

_lib.nps_param_count.argtypes, _lib.nps_param_count.restype = [_int], _sz
_lib.nps_net_bytes.argtypes, _lib.nps_net_bytes.restype = [_int], _sz
_lib.nps_net_create.argtypes = [_vp, _sz, _int, _vp, _sz, _vp, ctypes.POINTER(_vp)]
_lib.nps_net_create.restype = _int
_lib.nps_net_destroy.argtypes, _lib.nps_net_destroy.restype = [_vp], None
_lib.nps_net_levels.argtypes, _lib.nps_net_levels.restype = [_vp], _int
_lib.nps_workspace_bytes.argtypes, _lib.nps_workspace_bytes.restype = [nps_dims, _int, _int, _int], _sz
_lib.nps_solve_workspace_bytes.argtypes = [nps_dims, _int, ctypes.POINTER(nps_opts)]
_lib.nps_solve_workspace_bytes.restype = _sz
_lib.nps_apply_precond_transpose.argtypes = [_vp, _vp, nps_dims, _vp, _vp, _int, _vp, _sz, _vp]
_lib.nps_apply_precond_transpose.restype = _int
_lib.nps_asymmetry.argtypes = [_vp, _vp, nps_dims, _vp, _vp, _vp, _vp, _int, _vp, _sz, ctypes.POINTER(ctypes.c_double),
                               _vp]
_lib.nps_asymmetry.restype = _int
_lib.nps_lanczos_workspace_bytes.argtypes, _lib.nps_lanczos_workspace_bytes.restype = [nps_dims, _int], _sz
_lib.nps_lanczos.argtypes = [_vp, nps_dims, _int, _int, _vp, _vp, _vp, _vp, ctypes.POINTER(_int), _vp, _sz, _vp]
_lib.nps_lanczos.restype = _int
_lib.nps_ritz_workspace_bytes.argtypes, _lib.nps_ritz_workspace_bytes.restype = [_int, _int], _sz
_lib.nps_ritz_rhs.argtypes = [_vp, nps_dims, _int, _vp, _vp, _vp, _int, _vp, _vp, _vp, _sz, _vp]
_lib.nps_ritz_rhs.restype = _int
_lib.nps_solve.argtypes = [_vp, _vp, nps_dims, _vp, _vp, ctypes.POINTER(nps_opts), ctypes.POINTER(nps_info),
                           _vp, _sz, _vp]
_lib.nps_solve.restype = _int
_lib.nps_apply_laplacian.argtypes = [_vp, nps_dims, _vp, _vp, _int, _vp]
_lib.nps_apply_laplacian.restype = _int
_lib.nps_apply_precond.argtypes = [_vp, _vp, nps_dims, _vp, _vp, _int, _vp, _sz, _vp]
_lib.nps_apply_precond.restype = _int
_lib.nps_apply_precond_noalloc.argtypes = [_vp, _vp, nps_dims, _vp, _vp, _int, _vp]
_lib.nps_apply_precond_noalloc.restype = _int
_u64 = ctypes.c_uint64
_lib.nps_server_create.argtypes = [_vp, _sz, _int, ctypes.POINTER(_vp)]
_lib.nps_server_create.restype = _int
_lib.nps_server_destroy.argtypes, _lib.nps_server_destroy.restype = [_vp], None
_lib.nps_server_request_bytes.argtypes = [_vp, nps_dims, ctypes.POINTER(nps_opts)]
_lib.nps_server_request_bytes.restype = _sz
_lib.nps_server_submit.argtypes = [_vp, _vp, nps_dims, _vp, ctypes.POINTER(nps_opts), ctypes.POINTER(_u64)]
_lib.nps_server_submit.restype = _int
_lib.nps_server_step.argtypes = [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int)]
_lib.nps_server_step.restype = _int
_lib.nps_server_poll.argtypes = [_vp, _u64, _vp, ctypes.POINTER(nps_info), ctypes.POINTER(ctypes.c_double)]
_lib.nps_server_poll.restype = _int
_lib.nps_train_workspace_bytes.argtypes = [nps_dims, _int, _int]
_lib.nps_train_workspace_bytes.restype = _sz
_lib.nps_net_forward.argtypes = [_vp, _vp, nps_dims, _vp, _vp, _int, _vp, _sz, _vp]
_lib.nps_net_forward.restype = _int
_lib.nps_train_loss.argtypes = [_vp, nps_dims, _int, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double), _int, _vp, _sz, _vp]
_lib.nps_train_loss.restype = _int
_lib.nps_net_backward.argtypes = [_vp, _vp, nps_dims, _vp, _vp, _vp, _int, _vp, _sz, _vp]
_lib.nps_net_backward.restype = _int
_lib.nps_train_step.argtypes = [_vp, _vp, nps_dims, _int, _vp, _vp, ctypes.POINTER(ctypes.c_double), _int, _vp, _sz, _vp]
_lib.nps_train_step.restype = _int
_lib.nps_profile_enable.argtypes, _lib.nps_profile_enable.restype = [_int], _int
_lib.nps_profile_read.argtypes = [ctypes.POINTER(nps_kernel_stat), _int, ctypes.POINTER(_int)]
_lib.nps_profile_read.restype = _int
_lib.nps_last_error.argtypes, _lib.nps_last_error.restype = [], ctypes.c_char_p

EXPORTED = ["nps_param_count", "nps_net_bytes", "nps_net_create", "nps_net_destroy", "nps_net_levels",
            "nps_workspace_bytes", "nps_solve_workspace_bytes", "nps_solve", "nps_apply_laplacian",
            "nps_apply_precond", "nps_apply_precond_noalloc",
            "nps_apply_precond_transpose", "nps_asymmetry", "nps_lanczos_workspace_bytes",
            "nps_lanczos", "nps_ritz_workspace_bytes", "nps_ritz_rhs", "nps_server_create",
            "nps_server_destroy", "nps_server_request_bytes", "nps_server_submit", "nps_server_step",
            "nps_server_poll", "nps_train_workspace_bytes", "nps_net_forward", "nps_train_loss", "nps_net_backward",
            "nps_train_step",
            "nps_profile_enable", "nps_profile_read", "nps_last_error"]
NPS_PENDING = 2


def nps_param_count(levels: int) -> int:
    return _lib.nps_param_count(levels)


def nps_net_bytes(levels: int) -> int:
    return _lib.nps_net_bytes(levels)


def nps_net_create(params_h: int, n_params: int, levels: int, dev_buf_d: int, dev_bytes: int,
                   stream: int) -> tuple:
    """Returns (status, net handle)."""
    out = _vp()
    rc = _lib.nps_net_create(params_h, n_params, levels, dev_buf_d, dev_bytes, stream, ctypes.byref(out))
    return rc, out.value


def nps_net_destroy(net: int) -> None:
    _lib.nps_net_destroy(net)


def nps_net_levels(net: int) -> int:
    return _lib.nps_net_levels(net)


def nps_workspace_bytes(dims: nps_dims, levels: int, precision: int, n_ortho: int) -> int:
    return _lib.nps_workspace_bytes(dims, levels, precision, n_ortho)


def nps_solve_workspace_bytes(dims: nps_dims, levels: int, opts: nps_opts) -> int:
    return _lib.nps_solve_workspace_bytes(dims, levels, ctypes.byref(opts))


def nps_apply_precond_transpose(net: int, labels_d: int, dims: nps_dims, g_d: int, y_d: int, precision: int,
                                ws_d: int, ws_bytes: int, stream: int) -> int:
    return _lib.nps_apply_precond_transpose(net, labels_d, dims, g_d, y_d, precision, ws_d, ws_bytes, stream)


def nps_asymmetry(net: int, labels_d: int, dims: nps_dims, x_d: int, y_d: int, px_d: int, py_d: int,
                  precision: int, ws_d: int, ws_bytes: int, stream: int) -> tuple:
    """Returns (status, S)."""
    out = ctypes.c_double()
    rc = _lib.nps_asymmetry(net, labels_d, dims, x_d, y_d, px_d, py_d, precision, ws_d, ws_bytes,
                            ctypes.byref(out), stream)
    return rc, out.value


def nps_lanczos_workspace_bytes(dims: nps_dims, m: int) -> int:
    return _lib.nps_lanczos_workspace_bytes(dims, m)


def nps_ritz_workspace_bytes(m: int, k: int) -> int:
    return _lib.nps_ritz_workspace_bytes(m, k)


def nps_lanczos(labels_d: int, dims: nps_dims, m: int, reorth: int, v0_d: int, V_d: int, alpha_d: int, beta_d: int,
                ws_d: int, ws_bytes: int, stream: int) -> tuple:
    """Returns (status, steps)."""
    steps = _int()
    rc = _lib.nps_lanczos(labels_d, dims, m, reorth, v0_d, V_d, alpha_d, beta_d, ctypes.byref(steps), ws_d, ws_bytes,
                          stream)
    return rc, steps.value


def nps_ritz_rhs(V_d: int, dims: nps_dims, m: int, alpha_d: int, beta_d: int, coef_d: int, k: int, rhs_d: int,
                 theta_d: int, ws_d: int, ws_bytes: int, stream: int) -> int:
    return _lib.nps_ritz_rhs(V_d, dims, m, alpha_d, beta_d, coef_d, k, rhs_d, theta_d, ws_d, ws_bytes, stream)


def nps_solve(net: int, labels_d: int, dims: nps_dims, b_d: int, x_d: int, opts: nps_opts,
              info: nps_info, ws_d: int, ws_bytes: int, stream: int) -> int:
    return _lib.nps_solve(net, labels_d, dims, b_d, x_d, ctypes.byref(opts), ctypes.byref(info),
                          ws_d, ws_bytes, stream)


def nps_apply_laplacian(labels_d: int, dims: nps_dims, x_d: int, y_d: int, precision: int, stream: int) -> int:
    return _lib.nps_apply_laplacian(labels_d, dims, x_d, y_d, precision, stream)


def nps_apply_precond_noalloc(net: int, labels_d: int, dims: nps_dims, r_d: int, d_d: int, precision: int,
                              stream: int) -> int:
    return _lib.nps_apply_precond_noalloc(net, labels_d, dims, r_d, d_d, precision, stream)


def nps_apply_precond(net: int, labels_d: int, dims: nps_dims, r_d: int, d_d: int, precision: int,
                      ws_d: int, ws_bytes: int, stream: int) -> int:
    return _lib.nps_apply_precond(net, labels_d, dims, r_d, d_d, precision, ws_d, ws_bytes, stream)


def nps_server_create(net: int, hbm_budget: int, max_slots: int) -> tuple:
    """Returns (status, server handle)."""
    out = _vp()
    rc = _lib.nps_server_create(net, hbm_budget, max_slots, ctypes.byref(out))
    return rc, out.value


def nps_server_destroy(srv: int) -> None:
    _lib.nps_server_destroy(srv)


def nps_server_request_bytes(srv: int, dims: nps_dims, opts: nps_opts) -> int:
    return _lib.nps_server_request_bytes(srv, dims, ctypes.byref(opts))


def nps_server_submit(srv: int, labels_h: int, dims: nps_dims, b_h: int, opts: nps_opts) -> tuple:
    """Returns (status, request id)."""
    rid = _u64(0)
    rc = _lib.nps_server_submit(srv, labels_h, dims, b_h, ctypes.byref(opts), ctypes.byref(rid))
    return rc, rid.value


def nps_server_step(srv: int) -> tuple:
    """Returns (status, n_active, n_queued)."""
    a, q = _int(0), _int(0)
    rc = _lib.nps_server_step(srv, ctypes.byref(a), ctypes.byref(q))
    return rc, a.value, q.value


def nps_server_poll(srv: int, req_id: int, x_h: int, info: nps_info) -> tuple:
    """Returns (status, latency_ms); status NPS_PENDING while the request runs."""
    lat = ctypes.c_double(0.0)
    rc = _lib.nps_server_poll(srv, req_id, x_h, ctypes.byref(info), ctypes.byref(lat))
    return rc, lat.value


def nps_train_workspace_bytes(dims: nps_dims, levels: int, precision: int) -> int:
    return _lib.nps_train_workspace_bytes(dims, levels, precision)


def nps_net_forward(net: int, labels_d: int, dims: nps_dims, r_d: int, y_d: int, precision: int, ws_d: int,
                    ws_bytes: int, stream: int) -> int:
    return _lib.nps_net_forward(net, labels_d, dims, r_d, y_d, precision, ws_d, ws_bytes, stream)


def nps_train_loss(labels_d: int, dims: nps_dims, levels: int, b_d: int, y_d: int, gy_d: int, precision: int,
                   ws_d: int, ws_bytes: int, stream: int) -> tuple:
    """Returns (status, loss)."""
    loss = ctypes.c_double(0.0)
    rc = _lib.nps_train_loss(labels_d, dims, levels, b_d, y_d, gy_d, ctypes.byref(loss), precision, ws_d, ws_bytes,
                             stream)
    return rc, loss.value


def nps_net_backward(net: int, labels_d: int, dims: nps_dims, r_d: int, gy_d: int, grad_d: int, precision: int,
                     ws_d: int, ws_bytes: int, stream: int) -> int:
    return _lib.nps_net_backward(net, labels_d, dims, r_d, gy_d, grad_d, precision, ws_d, ws_bytes, stream)


def nps_train_step(net: int, labels_d: int, dims: nps_dims, batch: int, b_d: int, grad_d: int, precision: int,
                   ws_d: int, ws_bytes: int, stream: int) -> tuple[int, float]:
    loss = ctypes.c_double(0.0)
    rc = _lib.nps_train_step(net, labels_d, dims, batch, b_d, grad_d, ctypes.byref(loss), precision, ws_d, ws_bytes,
                             stream)
    return rc, loss.value


def nps_profile_enable(on: int) -> int:
    return _lib.nps_profile_enable(on)


def nps_profile_read(max_records: int = 64) -> tuple:
    """Returns (status, [nps_kernel_stat, ...])."""
    buf = (nps_kernel_stat * max_records)()
    n = _int(0)
    rc = _lib.nps_profile_read(buf, max_records, ctypes.byref(n))
    return rc, [buf[i] for i in range(min(n.value, max_records))]


def nps_last_error() -> str:
    return _lib.nps_last_error().decode()
