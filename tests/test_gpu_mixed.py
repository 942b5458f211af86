"""Accuracy of the mixed-precision solve against the FP64 oracle.

The paper runs its network in single precision and everything else in
double, and reports that this does not limit the solver's accuracy (Sec.
"Results and Analysis"; appendix on the capacity for residual reduction).
Here the network runs in bf16 / fp16 on matrix cores with float Krylov
vectors; the solution is accumulated in double and the residual b - A x is
formed in double every iteration.  The oracle solves the same system to a
1e-12 relative residual (x_ref); each GPU result states its error
||x - x_ref|| / ||x_ref|| and its FP64 true residual (oracle matvec).
"""
import numpy as np
import pytest
import torch

import nps_inputs as gi
from oracle import laplacian as lap
from oracle import npsdo as onpsdo

pytestmark = pytest.mark.gpu

nps = pytest.importorskip("paper_2310_00177_amd")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

PREC = {"fp64": nps.FP64, "fp32": nps.FP32, "mixed_bf16": nps.MIXED_BF16, "mixed_fp16": nps.MIXED_FP16}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def system64():
    """64^3 scene of the serving recipe (the 128^3 recipe scaled by 1/2), the
    oracle's x_ref to 1e-12 and the FP64 GPU path's error at each tolerance."""
    lab = gi.gen_labels(gi.scene_serving(64), seed=5)
    b = gi.gen_rhs(lab, seed=6)
    params = gi.multilevel_params(6)
    print("oracle x_ref 64^3 to 1e-12", flush=True)
    ref = onpsdo.solve_with_network(lab, b, params, 6, tol=1e-12, max_iter=3000)
    assert ref.status == 0
    return lab, b, params, ref.x


# FP32 mode keeps the iterate in float, which bounds its attainable relative
# residual near 4e-7 on this system (measured: 2000 iterations end at 3.75e-7
# for a 1e-8 target), so it is held to 1e-6 only; the mixed modes keep the
# iterate in double and are held to both tolerances.
CASES = [("fp64", 1e-6), ("fp64", 1e-8), ("fp32", 1e-6), ("mixed_bf16", 1e-6), ("mixed_bf16", 1e-8),
         ("mixed_fp16", 1e-6), ("mixed_fp16", 1e-8)]


@pytest.mark.parametrize("precision,tol", CASES)
def test_solution_error_vs_oracle(system64, precision, tol):
    lab, b, params, xref = system64
    net = nps.Net(params, 6)
    x, info = nps.solve(net, dev(lab), dev(b), tol=tol, max_iter=2000, precision=PREC[precision])
    xs = x.cpu().numpy()
    true_rel = lap.rel_residual(lab, b, xs)
    err = float(np.linalg.norm(xs - xref) / np.linalg.norm(xref))
    # the same tolerance in FP64: the error the tolerance itself allows
    x64, _ = nps.solve(net, dev(lab), dev(b), tol=tol, max_iter=2000, precision=nps.FP64)
    err64 = float(np.linalg.norm(x64.cpu().numpy() - xref) / np.linalg.norm(xref))
    print(f"64^3 {precision} tol {tol:.0e}: {info.iterations} its, true rel residual {true_rel:.3e}, "
          f"error vs x_ref {err:.3e} (FP64 path at this tol: {err64:.3e})", flush=True)
    assert info.status == 0 and true_rel < tol
    assert info.rel_residual == pytest.approx(true_rel, rel=1e-3)
    # reduced precision inside the iteration does not limit the attainable
    # accuracy: the error stays at the level the tolerance allows
    assert err <= 4.0 * err64 + 1e-12, (err, err64)


@pytest.fixture(scope="module")
def system256():
    """The 256^3 scene (60 spheres, 3 slabs, sinusoidal free surface), N(0,1)
    right-hand side on fluid."""
    print("generating the 256^3 scene", flush=True)
    lab = gi.gen_labels(gi.scene_c3(), seed=1)
    return lab, gi.gen_rhs(lab, seed=2)


@pytest.mark.parametrize("precision", ["mixed_bf16", "mixed_fp16"])
def test_256cubed_mixed_solve_reaches_1e8(system256, precision):
    """The largest configuration: the mixed modes reach a 1e-8 relative
    residual at 256^3, judged by the oracle's FP64 matvec (the oracle's own
    x_ref at this size takes hours; the error against it is in the committed
    256^3 report)."""
    lab, b = system256
    net = nps.Net(gi.multilevel_params(6), 6)
    print(f"256^3 {precision} solve to 1e-8", flush=True)
    x, info = nps.solve(net, dev(lab), dev(b), tol=1e-8, max_iter=3000, precision=PREC[precision])
    true_rel = lap.rel_residual(lab, b, x.cpu().numpy())
    print(f"256^3 {precision}: {info.iterations} its, status {info.status}, true rel residual {true_rel:.3e}",
          flush=True)
    assert info.status == 0 and true_rel < 1e-8
    assert info.rel_residual == pytest.approx(true_rel, rel=1e-3)
