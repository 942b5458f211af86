"""Pins for the oracle's NPSDO iteration (Alg. 1).

Special cases the paper states (Sec. "Algorithm"): with the identity
preconditioner and n_ortho >= 1 the iteration is unpreconditioned CG; with
n_ortho = 0 it is steepest descent.  Also: a dense direct solve on tiny grids,
one-step convergence on an eigenvector, monotone energy and the orthogonality
relations that exact line search and A-orthogonalisation impose.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import nps_inputs as gi
from oracle import laplacian as lap
from oracle import network as net
from oracle import npsdo


def small_scene(seed=1):
    return gi.gen_labels(gi.scene_gradcheck(), seed=seed)


def masked_identity(lab):
    fluid = lab == gi.FLUID
    return lambda r: np.where(fluid, r, 0.0)


@pytest.mark.parametrize("n_ortho", [1, 2, 3])
def test_identity_preconditioner_reproduces_cg_iterates(n_ortho):
    lab = small_scene()
    b = gi.gen_rhs(lab, seed=5)
    A, cells = lap.dense_reduced(lab)
    bf = np.array([b[p] for p in cells])
    cg_iters = []
    spla.cg(A, bf, x0=np.zeros_like(bf), rtol=1e-30, maxiter=25,
            callback=lambda xk: cg_iters.append(xk.copy()))
    fluid = lab == gi.FLUID
    for k in range(1, 26):
        res = npsdo.solve(lab, b, masked_identity(lab), tol=0.0, max_iter=k, n_ortho=n_ortho)
        assert res.iterations == k
        xk = res.x[fluid]
        ref = cg_iters[k - 1]
        assert np.linalg.norm(xk - ref) <= 1e-9 * np.linalg.norm(ref), k


def test_no_orthogonalisation_is_steepest_descent():
    lab = small_scene(2)
    b = gi.gen_rhs(lab, seed=6)
    A, cells = lap.dense_reduced(lab)
    bf = np.array([b[p] for p in cells])
    x = np.zeros_like(bf)
    res = npsdo.solve(lab, b, masked_identity(lab), tol=0.0, max_iter=15, n_ortho=0)
    for _ in range(15):
        r = bf - A @ x
        x = x + (r @ r) / (r @ (A @ r)) * r
    np.testing.assert_allclose(res.x[lab == gi.FLUID], x, rtol=1e-10, atol=1e-12)


def test_eigenvector_converges_in_one_step():
    N, h = 16, 11
    lab = np.full((N, N, N), gi.SOLID, dtype=np.uint8)
    lab[1:h, 1:N - 1, 1:N - 1] = gi.FLUID
    lab[h:N - 1, 1:N - 1, 1:N - 1] = gi.AIR
    n, m = N - 2, h - 1
    th = np.pi * 3 / (2 * m + 1)
    vx = np.cos(np.pi * 2 * (np.arange(n) + 0.5) / n)
    wz = np.cos(th * (np.arange(m) + 0.5))
    lam = (2 - 2 * np.cos(2 * np.pi / n)) + (2 - 2 * np.cos(th))
    b = np.zeros(lab.shape)
    b[1:h, 1:N - 1, 1:N - 1] = wz[:, None, None] * vx[None, None, :]
    res = npsdo.solve(lab, b, masked_identity(lab), tol=1e-12, max_iter=5)
    assert res.iterations == 1
    np.testing.assert_allclose(res.x, b / lam, atol=1e-13)


@pytest.mark.parametrize("L,blob", [(5, "multilevel"), (5, "identity")])
def test_converges_to_dense_solution(L, blob):
    lab = small_scene(3)
    b = gi.gen_rhs(lab, seed=7)
    params = gi.multilevel_params(L) if blob == "multilevel" else gi.identity_params(L)
    res = npsdo.solve_with_network(lab, b, params, L, tol=1e-12, max_iter=500)
    assert res.status == npsdo.OK
    A, cells = lap.dense_reduced(lab)
    xs = np.linalg.solve(A, np.array([b[p] for p in cells]))
    kappa = np.linalg.cond(A)
    err = np.linalg.norm(res.x[lab == gi.FLUID] - xs) / np.linalg.norm(xs)
    assert err <= kappa * 1e-12
    assert lap.rel_residual(lab, b, res.x) < 1e-12


@pytest.mark.parametrize("blob", ["xavier", "multilevel"])
def test_energy_monotone_and_orthogonality(blob):
    lab = small_scene(4)
    b = gi.gen_rhs(lab, seed=8)
    L = 5
    params = gi.xavier_params(L, seed=1) if blob == "xavier" else gi.multilevel_params(L)
    res = npsdo.solve_with_network(lab, b, params, L, tol=0.0, max_iter=12, keep_dirs=True,
                                   fixed_iters=True)
    e = np.array(res.history["energy"])
    assert np.all(np.diff(e) <= 1e-12 * np.abs(e).max())
    A = lambda v: lap.matvec(lab, v)  # noqa: E731
    D, R = res.history["d"], res.history["r"]
    for k in range(len(D)):
        dk = D[k]
        scale = np.linalg.norm(dk) * np.linalg.norm(R[k]) + 1e-300
        assert abs(R[k].ravel() @ dk.ravel()) <= 1e-10 * max(scale, np.linalg.norm(b) * np.linalg.norm(dk))
        Adk = A(dk)
        for j in (k - 1, k - 2):
            if j >= 0:
                c = abs(D[j].ravel() @ Adk.ravel())
                assert c <= 1e-9 * np.sqrt((D[j].ravel() @ A(D[j]).ravel()) * (dk.ravel() @ Adk.ravel()))
    # energy drop per step = (r.d)^2 / (2 d.Ad)
    drop = -np.diff(e)
    assert np.all(drop >= -1e-12)


def test_zero_rhs_returns_zero():
    lab = small_scene(5)
    res = npsdo.solve_with_network(lab, np.zeros(lab.shape), gi.multilevel_params(5), 5)
    assert res.iterations == 0 and np.all(res.x == 0.0) and res.status == npsdo.OK


def test_breakdown_on_zero_network():
    lab = small_scene(6)
    b = gi.gen_rhs(lab, seed=9)
    res = npsdo.solve_with_network(lab, b, np.zeros(gi.param_count(5)), 5, max_iter=5)
    assert res.status == npsdo.BREAKDOWN and res.iterations == 0


def test_fixed_iteration_mode_runs_exactly():
    lab = small_scene(7)
    b = gi.gen_rhs(lab, seed=10)
    res = npsdo.solve_with_network(lab, b, gi.multilevel_params(5), 5, tol=1e-3, max_iter=80,
                                   fixed_iters=True)
    assert res.iterations == 80 and res.status == npsdo.OK
    assert res.rel_residual < 1e-10


def test_relative_residual_is_reported_in_fp64():
    lab = small_scene(8)
    b = gi.gen_rhs(lab, seed=11)
    res = npsdo.solve_with_network(lab, b, gi.multilevel_params(5), 5, tol=1e-6, max_iter=200)
    assert res.status == npsdo.OK
    assert res.rel_residual == pytest.approx(lap.rel_residual(lab, b, res.x), rel=1e-12)
    assert res.rel_residual < 1e-6


def test_asymmetry_measure_zero_for_symmetric_operator():
    """S(x, y) vanishes for a symmetric operator (identity weights = fluid mask)."""
    lab = small_scene(9)
    P = net.Network(gi.identity_params(5), 5, lab)
    rng = np.random.default_rng(12)
    x, y = rng.standard_normal((2,) + lab.shape)
    assert net.asymmetry(P, x, y) < 1e-14
