"""Pins for the oracle's training loss and adjoint (Sec. "Training").

Adjoint identities <T x, y> = <x, T^T y> for every transposed operator, and
central finite differences (eps = 1e-3) of the loss along random directions
and along single parameters, on a 16^3 scene with a 5-level network.
"""
import numpy as np
import pytest

import nps_inputs as gi
from oracle import gradient as og
from oracle import network as onet


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_pool_and_interpolation_adjoints():
    x, y = _rand((4, 6, 8), 1), _rand((2, 3, 4), 2)
    assert np.dot(onet.pool(x).ravel(), y.ravel()) == pytest.approx(np.dot(x.ravel(), og.pool_transpose(y).ravel()), rel=1e-13)
    c, f = _rand((3, 5, 4), 3), _rand((6, 10, 8), 4)
    lhs = np.dot(onet.interpolate(c).ravel(), f.ravel())
    assert lhs == pytest.approx(np.dot(c.ravel(), og.interpolate_transpose(f).ravel()), rel=1e-12)


def test_cconv_apply_adjoint():
    r, g = _rand((5, 6, 7), 5), _rand((5, 6, 7), 6)
    K = _rand((27, 5, 6, 7), 7)
    lhs = np.dot(onet.cconv_apply(K, r).ravel(), g.ravel())
    assert lhs == pytest.approx(np.dot(r.ravel(), og.cconv_apply_transpose(K, g).ravel()), rel=1e-12)


def test_cconv_param_grads_match_finite_differences():
    rng = np.random.default_rng(8)
    lab = rng.choice(3, size=(4, 5, 6)).astype(np.uint8)
    I = onet.image(lab)
    r, g = rng.standard_normal((2,) + lab.shape)
    W, B = rng.standard_normal((27, 3, 3, 3, 3)), rng.standard_normal(27)
    gW, gB = og.cconv_param_grads(I, r, g)
    f = lambda W_, B_: float(np.sum(g * onet.cconv(I, W_, B_, r)))  # noqa: E731  linear in W and B
    dW, dB = rng.standard_normal(W.shape), rng.standard_normal(27)
    assert f(dW, np.zeros(27)) == pytest.approx(float(np.sum(gW * dW)), rel=1e-12)
    assert f(np.zeros_like(W), dB) == pytest.approx(float(np.sum(gB * dB)), rel=1e-12)


@pytest.fixture(scope="module")
def problem():
    lab = gi.gen_labels(gi.scene_gradcheck(), seed=5)
    b = gi.gen_rhs(lab, seed=6, normalize=True)
    params = gi.xavier_params(5, seed=4)
    rng = np.random.default_rng(9)
    for name, _l, off, size in gi.blob_layout(5):   # non-zero biases exercise every term
        if name.endswith("B"):
            params[off:off + size] = rng.uniform(-0.5, 0.5, size)
    return lab, b, params


def test_directional_derivatives_match_central_differences(problem):
    lab, b, params = problem
    loss, grad = og.loss_and_grad(params, 5, lab, b)
    assert loss == pytest.approx(og.loss_only(params, 5, lab, b), rel=1e-14)
    rng = np.random.default_rng(10)
    eps = 1e-3
    for _ in range(3):
        v = rng.standard_normal(params.size)
        v /= np.linalg.norm(v)
        fd = (og.loss_only(params + eps * v, 5, lab, b) - og.loss_only(params - eps * v, 5, lab, b)) / (2 * eps)
        assert float(grad @ v) == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_single_parameter_derivatives(problem):
    lab, b, params = problem
    _, grad = og.loss_and_grad(params, 5, lab, b)
    eps = 1e-3
    lay = {(n, l): off for n, l, off, _s in gi.blob_layout(5)}
    picks = [lay[("c1W", 1)] + 13, lay[("c1B", 3)] + 4, lay[("c2W", 2)] + 100, lay[("c2B", 1)] + 13,
             lay[("a1W", 1)] + 40, lay[("a1B", 2)], lay[("a2W", 4)] + 7, lay[("a2B", 1)], lay[("c1W", 5)] + 2000]
    for i in picks:
        e = np.zeros(params.size)
        e[i] = eps
        fd = (og.loss_only(params + e, 5, lab, b) - og.loss_only(params - e, 5, lab, b)) / (2 * eps)
        assert grad[i] == pytest.approx(fd, rel=1e-4, abs=1e-8), i


def test_transpose_apply_is_the_adjoint_of_the_network():
    """<y, P x> = <P^T y, x> for random x, y (P from the pinned forward oracle)."""
    lab = gi.gen_labels(gi.scene_gradcheck(), seed=8)
    for L, params in ((5, gi.xavier_params(5, seed=2)), (4, gi.multilevel_params(4))):
        P = onet.Network(params, L, lab)
        rng = np.random.default_rng(L)
        for _ in range(3):
            x, y = rng.standard_normal(lab.shape), rng.standard_normal(lab.shape)
            lhs = float(np.sum(y * P.apply(x)))
            rhs = float(np.sum(og.transpose_apply(P, y) * x))
            assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-12)


def test_transpose_apply_matches_the_dense_transpose_on_a_tiny_grid():
    """Brute force: P as a dense matrix from unit vectors, then transposed."""
    lab = np.random.default_rng(3).choice(np.array([gi.FLUID, gi.AIR, gi.SOLID], np.uint8), size=(4, 4, 8),
                                          p=[0.6, 0.2, 0.2])
    params = gi.xavier_params(3, seed=5)
    P = onet.Network(params, 3, lab)
    n = lab.size
    M = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M[:, j] = P.apply(e.reshape(lab.shape)).ravel()
    g = np.random.default_rng(1).standard_normal(n)
    np.testing.assert_allclose(og.transpose_apply(P, g.reshape(lab.shape)).ravel(), M.T @ g, rtol=1e-11, atol=1e-12)


def test_symmetric_variant_is_symmetric_positive():
    """P_sym = P^T o P (appendix on symmetry): S(x, y) = 0 and x.P_sym x = |P x|^2."""
    lab = gi.gen_labels(gi.scene_gradcheck(), seed=9)
    P = onet.Network(gi.xavier_params(5, seed=6), 5, lab)

    class Sym:
        def apply(self, v):
            return og.transpose_apply(P, P.apply(v))
    rng = np.random.default_rng(4)
    x, y = rng.standard_normal(lab.shape), rng.standard_normal(lab.shape)
    assert onet.asymmetry(P, x, y) > 1e-3
    assert onet.asymmetry(Sym(), x, y) < 1e-12
    assert float(np.sum(x * Sym().apply(x))) == pytest.approx(float(np.sum(P.apply(x) ** 2)), rel=1e-12)
