"""Pins for the oracle's Ritz-vector right-hand-side generator (Sec. "Training").

A full Lanczos run on a tiny grid reproduces the dense matrix's eigenvalues
(numpy eigvalsh); the basis is orthonormal and satisfies the three-term
relation A V^T = V^T T + beta_m v_(m+1) e_m^T; every Ritz pair satisfies
the classical residual identity ||A u - theta u|| = beta_m |y_m|; the
generated right-hand sides have unit norm and their components along the
Ritz vectors (from numpy's dense eigh of T) are the coefficients, up to sign.
"""
import numpy as np
import pytest

import nps_inputs as gi
from oracle import laplacian as lap
from oracle import lanczos as olz


def tiny_labels(seed=0):
    lab = np.full((4, 4, 8), gi.SOLID, np.uint8)
    lab[1:3, 1:3, 1:7] = gi.FLUID
    lab[3, 1:3, 2:6] = gi.AIR
    lab[1, 1, 3] = gi.SOLID
    return lab


def test_full_run_reproduces_the_spectrum():
    lab = tiny_labels()
    A, cells = lap.dense_reduced(lab)
    v0 = np.random.default_rng(1).standard_normal(lab.shape)
    V, alpha, beta, steps = olz.lanczos(lab, v0, m=len(cells) + 10)
    assert steps == len(cells)
    theta, _ = olz.ritz(alpha, beta)
    np.testing.assert_allclose(theta, np.linalg.eigvalsh(A), rtol=1e-9, atol=1e-10)


def test_basis_is_orthonormal_and_satisfies_the_three_term_relation():
    lab = gi.gen_labels(gi.scene_gradcheck(), seed=2)
    v0 = np.random.default_rng(2).standard_normal(lab.shape)
    m = 30
    V, alpha, beta, steps = olz.lanczos(lab, v0, m)
    assert steps == m
    B = V.reshape(m, -1)
    np.testing.assert_allclose(B @ B.T, np.eye(m), atol=1e-12)
    fluid = lab == gi.FLUID
    assert np.all(V[:, ~fluid] == 0)
    for j in range(m - 1):
        av = lap.matvec(lab, V[j])
        rhs = alpha[j] * V[j] + beta[j] * V[j + 1] + (beta[j - 1] * V[j - 1] if j > 0 else 0.0)
        assert np.linalg.norm(av - rhs) <= 1e-10 * np.linalg.norm(av), j


def test_ritz_residual_identity():
    lab = gi.gen_labels(gi.scene_gradcheck(), seed=3)
    v0 = np.random.default_rng(3).standard_normal(lab.shape)
    m = 25
    V, alpha, beta, _ = olz.lanczos(lab, v0, m)
    theta, Y = olz.ritz(alpha, beta)
    B = V.reshape(m, -1)
    for i in (0, 1, m // 2, m - 1):
        u = (B.T @ Y[:, i]).reshape(lab.shape)
        res = np.linalg.norm(lap.matvec(lab, u) - theta[i] * u)
        assert res == pytest.approx(beta[m - 1] * abs(Y[m - 1, i]), rel=1e-7, abs=1e-11)


def test_rhs_are_normalised_ritz_combinations():
    lab = gi.gen_labels(gi.scene_gradcheck(), seed=4)
    rng = np.random.default_rng(4)
    m, k = 20, 6
    V, alpha, beta, _ = olz.lanczos(lab, rng.standard_normal(lab.shape), m)
    coef = rng.standard_normal((m, k))
    R = olz.ritz_rhs(V, alpha, beta, coef)
    assert R.shape == (k,) + lab.shape
    T = np.diag(alpha) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
    _, Yd = np.linalg.eigh(T)
    U = Yd.T @ V.reshape(m, -1)                   # Ritz vectors as rows, numpy's signs
    for i in range(k):
        r = R[i].ravel()
        assert np.linalg.norm(r) == pytest.approx(1.0, rel=1e-12)
        comp = U @ r
        np.testing.assert_allclose(np.abs(comp), np.abs(coef[:, i]) / np.linalg.norm(coef[:, i]), rtol=1e-8,
                                   atol=1e-12)


def test_plain_recurrence_agrees_while_orthogonality_holds():
    """Without reorthogonalisation the first steps (before any Ritz value
    converges) give the same T; the three-term relation holds at every step."""
    lab = gi.gen_labels(gi.scene_gradcheck(), seed=5)
    v0 = np.random.default_rng(5).standard_normal(lab.shape)
    Vf, af, bf, _ = olz.lanczos(lab, v0, 8)
    Vp, ap, bp, _ = olz.lanczos(lab, v0, 60, reorth=False)
    np.testing.assert_allclose(ap[:8], af, rtol=1e-9)
    np.testing.assert_allclose(bp[:8], bf, rtol=1e-9)
    for j in range(1, 59):
        av = lap.matvec(lab, Vp[j])
        rhs = ap[j] * Vp[j] + bp[j] * Vp[j + 1] + bp[j - 1] * Vp[j - 1]
        assert np.linalg.norm(av - rhs) <= 1e-10 * np.linalg.norm(av), j
