"""GPU tests of the training path: forward, loss and the hand-written backward.

Checked against the FP64 oracle's forward, loss and adjoint gradient, and
against central finite differences (eps = 1e-3) of the GPU loss, on the 16^3
gradient-check scene with a 5-level network and on a 64^3 multi-tile scene.
"""
import numpy as np
import pytest
import torch

import nps_inputs as gi
from oracle import gradient as og
from oracle import network as onet

pytestmark = pytest.mark.gpu

nps = pytest.importorskip("paper_2310_00177_amd")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def params_with_biases(L, seed):
    p = gi.xavier_params(L, seed)
    rng = np.random.default_rng(seed + 1)
    for name, _l, off, size in gi.blob_layout(L):
        if name.endswith("B"):
            p[off:off + size] = rng.uniform(-0.5, 0.5, size)
    return p


CASES = {
    "grad16": (gi.scene_gradcheck(), 5),
    "multi64": (gi.SceneSpec((64, 64, 96), 8, (3.0, 10.0), 2, ("flat", 32, 56)), 6),
}


def problem(name, seed=3):
    spec, L = CASES[name]
    lab = gi.gen_labels(spec, seed=seed)
    b = gi.gen_rhs(lab, seed=seed + 1, normalize=True)
    return lab, b, L


def gpu_grad(params, L, lab, b, dtype):
    labels = torch.from_numpy(lab).cuda()
    bt = torch.from_numpy(b).to(dtype).cuda()
    net = nps.Net(params, L)
    prec = nps.FP64 if dtype == torch.float64 else nps.FP32
    ws = nps.train_workspace(lab.shape, L, prec)
    y = nps.net_forward(net, labels, bt, ws)
    loss, gy = nps.train_loss(labels, bt, y, L, ws)
    grad = torch.zeros(gi.param_count(L), dtype=torch.float64, device="cuda")
    nps.net_backward(net, labels, bt, gy, grad, ws)
    return y.cpu().double().numpy(), loss, grad.cpu().numpy()


@pytest.mark.parametrize("name", ["grad16", "multi64"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_forward_loss_gradient_match_oracle(name, dtype):
    lab, b, L = problem(name)
    params = params_with_biases(L, 7)
    print(f"train parity {name} {dtype}", flush=True)
    y, loss, grad = gpu_grad(params, L, lab, b, dtype)
    y_ref = onet.Network(params, L, lab).apply(b)
    loss_ref, grad_ref = og.loss_and_grad(params, L, lab, b)
    # FP32: the weight-gradient contraction runs on fp32 matrix cores (exact
    # products, fp32 sums); measured gradient error 3e-8 .. 7e-8
    tol_y, tol_g = (1e-12, 1e-9) if dtype == torch.float64 else (1e-5, 1e-6)
    assert rel(y, y_ref) <= tol_y
    assert loss == pytest.approx(loss_ref, rel=10 * tol_y)
    assert rel(grad, grad_ref) <= tol_g, rel(grad, grad_ref)


def test_gradient_matches_central_differences_on_gpu():
    lab, b, L = problem("grad16", seed=5)
    params = params_with_biases(L, 9)
    _, _, grad = gpu_grad(params, L, lab, b, torch.float64)
    rng = np.random.default_rng(11)
    eps = 1e-3
    for _ in range(3):
        v = rng.standard_normal(params.size)
        v /= np.linalg.norm(v)
        lp = gpu_grad(params + eps * v, L, lab, b, torch.float64)[1]
        lm = gpu_grad(params - eps * v, L, lab, b, torch.float64)[1]
        assert float(grad @ v) == pytest.approx((lp - lm) / (2 * eps), rel=1e-5, abs=1e-9)


def test_autograd_functions_match_oracle_batch_mean():
    spec, L = CASES["grad16"]
    labs = [gi.gen_labels(spec, seed=s) for s in (21, 22)]
    bs = [gi.gen_rhs(lab, seed=s + 100, normalize=True) for lab, s in zip(labs, (21, 22))]
    params = params_with_biases(L, 13)
    p = torch.tensor(params, dtype=torch.float64, device="cuda", requires_grad=True)
    total = 0.0
    for lab, b in zip(labs, bs):
        labels = torch.from_numpy(lab).cuda()
        bt = torch.from_numpy(b).cuda()
        y = nps.Precond.apply(p, labels, bt, L)
        total = total + nps.TrainLoss.apply(y, labels, bt, L)
    loss = total / len(labs)
    loss.backward()
    loss_ref, grad_ref = og.batch_loss_and_grad(params, L, labs, bs)
    assert loss.item() == pytest.approx(loss_ref, rel=1e-11)
    assert rel(p.grad.cpu().numpy(), grad_ref) <= 1e-9


def test_autograd_input_gradient_is_the_adjoint():
    """P is linear in r, so dL/dr = P^T dL/dy: Precond's gradient for r equals
    the oracle's transpose apply of the loss gradient (FP64)."""
    spec, L = CASES["grad16"]
    lab = gi.gen_labels(spec, seed=31)
    b = gi.gen_rhs(lab, seed=32, normalize=True)
    params = params_with_biases(L, 17)
    p = torch.tensor(params, dtype=torch.float64, device="cuda", requires_grad=True)
    labels = torch.from_numpy(lab).cuda()
    r = torch.from_numpy(np.random.default_rng(33).standard_normal(lab.shape)).cuda().requires_grad_(True)
    gy = np.random.default_rng(34).standard_normal(lab.shape)
    y = nps.Precond.apply(p, labels, r, L)
    (y * torch.from_numpy(gy).cuda()).sum().backward()
    ref = og.transpose_apply(onet.Network(params, L, lab), gy)
    assert rel(r.grad.cpu().numpy(), ref) <= 1e-12
    assert p.grad is not None
    # a second call with the same parameter tensor reuses its device network
    net = nps._cached_net(p, L, r.device)
    assert nps._cached_net(p, L, r.device) is net
    with torch.no_grad():
        p.mul_(1.0)          # an in-place update moves the version: rebuilt
    assert nps._cached_net(p, L, r.device) is not net


def gpu_grad_prec(params, L, lab, b, prec):
    labels = torch.from_numpy(lab).cuda()
    bt = torch.from_numpy(b).to(nps.vector_dtype(prec)).cuda()
    net = nps.Net(params, L)
    ws = nps.train_workspace(lab.shape, L, prec)
    y = nps.net_forward(net, labels, bt, ws, precision=prec)
    loss, gy = nps.train_loss(labels, bt, y, L, ws, precision=prec)
    grad = torch.zeros(gi.param_count(L), dtype=torch.float64, device="cuda")
    nps.net_backward(net, labels, bt, gy, grad, ws, precision=prec)
    return y.cpu().double().numpy(), loss, grad.cpu().numpy()


# The bf16 training leg rounds the count-form weights to bf16 (relative
# 2^-9) and contracts the weight gradient on bf16 matrix cores; its error
# against the FP64 oracle is measured here and bounded.
# Measured: forward 3.4e-3 / 3.6e-3, gradient 3.0e-3 / 2.2e-3 (16^3 at L = 5,
# 64 x 64 x 96 at L = 6); the bounds are about twice that.
BF16_BOUNDS = {"y": 8e-3, "grad": 6e-3}


@pytest.mark.parametrize("name", ["grad16", "multi64"])
def test_bf16_training_leg_error_vs_oracle(name):
    lab, b, L = problem(name)
    params = params_with_biases(L, 7)
    y, loss, grad = gpu_grad_prec(params, L, lab, b, nps.MIXED_BF16)
    y_ref = onet.Network(params, L, lab).apply(b)
    loss_ref, grad_ref = og.loss_and_grad(params, L, lab, b)
    ey, eg = rel(y, y_ref), rel(grad, grad_ref)
    print(f"bf16 training {name}: forward {ey:.3e}, loss {abs(loss - loss_ref) / loss_ref:.3e}, gradient {eg:.3e}",
          flush=True)
    assert ey <= BF16_BOUNDS["y"] and eg <= BF16_BOUNDS["grad"]
    # the FP32 leg on the same system, for comparison
    _, _, g32 = gpu_grad_prec(params, L, lab, b, nps.FP32)
    print(f"  fp32 gradient {rel(g32, grad_ref):.3e}", flush=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_step_matches_oracle_batch_mean(prec):
    """nps_train_step over a batch of three systems: the mean loss and its
    gradient against the oracle's batch mean (Sec. "Training")."""
    spec, L = CASES["grad16"]
    seeds = (41, 42, 43)
    labs = [gi.gen_labels(spec, seed=s) for s in seeds]
    bs = [gi.gen_rhs(lab, seed=s + 100, normalize=True) for lab, s in zip(labs, seeds)]
    params = params_with_biases(L, 19)
    p = nps.FP64 if prec == "fp64" else nps.FP32
    dt = nps.vector_dtype(p)
    net = nps.Net(params, L)
    labels = torch.from_numpy(np.stack(labs)).cuda()
    b = torch.from_numpy(np.stack(bs)).to(dt).cuda()
    ws = nps.train_workspace(labs[0].shape, L, p)
    grad = torch.zeros(gi.param_count(L), dtype=torch.float64, device="cuda")
    loss = nps.train_step(net, labels, b, grad, ws, precision=p)
    loss_ref, grad_ref = og.batch_loss_and_grad(params, L, labs, bs)
    tol = 1e-9 if prec == "fp64" else 1e-6
    print(f"batch step {prec}: loss {abs(loss - loss_ref) / loss_ref:.2e}, gradient {rel(grad.cpu().numpy(), grad_ref):.2e}",
          flush=True)
    assert loss == pytest.approx(loss_ref, rel=max(tol, 1e-11))
    assert rel(grad.cpu().numpy(), grad_ref) <= tol
