"""The C-ABI library loads on the CPU host and exports every entry point
include/nps.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

import nps_inputs as gi


def declared_functions(repo_root):
    src = open(os.path.join(repo_root, "include", "nps.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nps_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_solver_entry_points(repo_root):
    names = declared_functions(repo_root)
    for must in ("nps_solve", "nps_apply_laplacian", "nps_apply_precond", "nps_net_create",
                 "nps_workspace_bytes", "nps_param_count", "nps_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(repo_root):
    path = os.path.join(repo_root, "paper_2310_00177_amd", "libnps.so")
    if not os.path.exists(path):
        pytest.skip("libnps.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name in declared_functions(repo_root):
        assert hasattr(lib, name), name
    from paper_2310_00177_amd import _lib
    assert sorted(_lib.EXPORTED) == declared_functions(repo_root)


def test_host_only_queries(repo_root):
    path = os.path.join(repo_root, "paper_2310_00177_amd", "libnps.so")
    if not os.path.exists(path):
        pytest.skip("libnps.so not built")
    from paper_2310_00177_amd import _lib
    assert _lib.nps_param_count(6) == gi.param_count(6) == 25174
    assert _lib.nps_param_count(5) == gi.param_count(5)
    assert _lib.nps_net_bytes(6) > 0 and _lib.nps_net_bytes(7) == 0
    d = _lib.nps_dims(128, 128, 128)
    ws32 = _lib.nps_workspace_bytes(d, 6, _lib.NPS_FP32, 2)
    ws64 = _lib.nps_workspace_bytes(d, 6, _lib.NPS_FP64, 2)
    wsm = _lib.nps_workspace_bytes(d, 6, _lib.NPS_MIXED_BF16, 2)
    n = 128 ** 3
    assert 40 * n < ws32 < 70 * n and ws64 > ws32 and wsm > ws32
    assert _lib.nps_workspace_bytes(_lib.nps_dims(128, 128, 120), 6, _lib.NPS_FP32, 2) == 0   # 120 % 32
    assert _lib.nps_workspace_bytes(d, 6, _lib.NPS_FP32, 5) == 0                              # n_ortho > 4


def test_every_exported_symbol_has_a_python_wrapper():
    from paper_2310_00177_amd import _lib
    assert [n for n in _lib.EXPORTED if not callable(getattr(_lib, n, None))] == []
