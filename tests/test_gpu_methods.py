"""GPU parity of the PCG and flexible PCG solvers (the variants of the appendix
comparing PCG variants) against the FP64 oracle, through the C ABI.

FP64 fixed-iteration iterates match the oracle's PCG / flexible PCG; the
FP32 and mixed paths reach the tolerance on the oracle's true residual;
with identity weights both are CG; option errors are reported.
"""
import numpy as np
import pytest
import torch

import nps_inputs as gi
from oracle import laplacian as lap
from oracle import network as onet
from oracle import npsdo as onpsdo
from oracle import pcg as opcg

pytestmark = pytest.mark.gpu

nps = pytest.importorskip("paper_2310_00177_amd")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

METHODS = {"pcg": (1, False), "fpcg": (2, True)}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def problem(seed, shape=None):
    spec = gi.scene_c1() if shape is None else gi.SceneSpec(shape, 8, (3.0, 10.0), 2, ("flat", 24, 40))
    lab = gi.gen_labels(spec, seed=seed)
    return lab, gi.gen_rhs(lab, seed=seed + 1)


@pytest.mark.parametrize("name", ["pcg", "fpcg"])
@pytest.mark.parametrize("wkind", ["multilevel", "xavier"])
def test_fixed_iterations_fp64_match_oracle(name, wkind):
    method, flexible = METHODS[name]
    lab, b = problem(2)
    params = gi.multilevel_params(6) if wkind == "multilevel" else gi.xavier_params(6, 0)
    net = nps.Net(params, 6)
    P = onet.Network(params, 6, lab)
    for k in (1, 2, 3, 7):
        print(f"{name} fixed-iter fp64 {wkind} k={k}", flush=True)
        ref = opcg.solve(lab, b, P.apply, max_iter=k, flexible=flexible, fixed_iters=True)
        x, info = nps.solve(net, dev(lab), dev(b), max_iter=k, fixed_iters=True, precision=nps.FP64, method=method)
        assert info.iterations == k and info.status == 0
        assert rel_err(x.cpu().numpy(), ref.x) <= 1e-9, (k, rel_err(x.cpu().numpy(), ref.x))
        assert info.rel_residual == pytest.approx(ref.rel_residual, rel=1e-6)


@pytest.mark.parametrize("name", ["pcg", "fpcg"])
def test_multi_tile_fixed_iterations_fp64(name):
    method, flexible = METHODS[name]
    lab, b = problem(4, shape=(64, 64, 96))
    params = gi.multilevel_params(6)
    P = onet.Network(params, 6, lab)
    print(f"{name} multi-tile fp64", flush=True)
    ref = opcg.solve(lab, b, P.apply, max_iter=4, flexible=flexible, fixed_iters=True)
    x, info = nps.solve(nps.Net(params, 6), dev(lab), dev(b), max_iter=4, fixed_iters=True, precision=nps.FP64,
                        method=method)
    assert rel_err(x.cpu().numpy(), ref.x) <= 1e-9


@pytest.mark.parametrize("name", ["pcg", "fpcg"])
@pytest.mark.parametrize("precision", ["fp32", "mixed_bf16"])
def test_solve_reaches_tolerance(name, precision):
    method, flexible = METHODS[name]
    lab, b = problem(1)
    params = gi.multilevel_params(6)
    p = {"fp32": nps.FP32, "mixed_bf16": nps.MIXED_BF16}[precision]
    print(f"{name} solve {precision}", flush=True)
    x, info = nps.solve(nps.Net(params, 6), dev(lab), dev(b), tol=1e-6, max_iter=500, precision=p, method=method)
    assert info.status == 0, info
    xs = x.cpu().numpy()
    true_rel = lap.rel_residual(lab, b, xs)
    assert true_rel < 1e-6, true_rel
    ref = opcg.solve(lab, b, onet.Network(params, 6, lab).apply, tol=1e-6, max_iter=500, flexible=flexible)
    assert abs(info.iterations - ref.iterations) <= max(2, ref.iterations // 10), (info.iterations, ref.iterations)
    assert np.all(xs[lab != gi.FLUID] == 0)


@pytest.mark.parametrize("name", ["pcg", "fpcg"])
def test_identity_weights_is_cg(name):
    method, _ = METHODS[name]
    lab, b = problem(3)
    params = gi.identity_params(6)
    ref = onpsdo.solve_with_network(lab, b, params, 6, max_iter=20, fixed_iters=True)   # NPSDO with P = I is CG
    x, info = nps.solve(nps.Net(params, 6), dev(lab), dev(b), max_iter=20, fixed_iters=True, precision=nps.FP64,
                        method=method)
    assert rel_err(x.cpu().numpy(), ref.x) <= 1e-8


def test_method_option_errors():
    lab, b = problem(5)
    net = nps.Net(gi.multilevel_params(6), 6)
    with pytest.raises(nps.NpsError) as e:
        nps.solve(net, dev(lab), dev(b), method=nps.PCG, n_ortho=2)
    assert e.value.code == -1
    with pytest.raises(nps.NpsError) as e:
        nps.solve(net, dev(lab), dev(b), method=7, n_ortho=1)
    assert e.value.code == -1


def test_server_runs_pcg_like_standalone():
    lab, b = problem(6)
    net = nps.Net(gi.multilevel_params(6), 6)
    srv = nps.Server(net, hbm_budget=1 << 30, max_slots=2)
    rid = srv.submit(lab, b, n_ortho=1, method=nps.FPCG)
    res = None
    while res is None:
        srv.step()
        res = srv.poll(rid)
    x, info, _ = res
    xs, infos = nps.solve(net, dev(lab), dev(b), precision=nps.MIXED_BF16, method=nps.FPCG)
    assert info.status == 0 and info.iterations == infos.iterations
    np.testing.assert_array_equal(x, xs.cpu().numpy())
    srv.close()
