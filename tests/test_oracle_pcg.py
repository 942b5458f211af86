"""Pins for the oracle's PCG and flexible PCG (the solver variants of the
appendix comparing PCG variants).

With the identity preconditioner both are unpreconditioned CG, and with a
symmetric positive definite preconditioner M both are PCG with M (the extra
term of the flexible form vanishes because PCG keeps M r_k orthogonal to the
earlier residuals): compared with SciPy's CG iterates.  A direct dense solve
pins convergence on tiny grids; the first step coincides with NPSDO's; and
with the nonsymmetric network the flexible term is non-zero, so the two forms
really differ.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import nps_inputs as gi
from oracle import laplacian as lap
from oracle import network as net
from oracle import npsdo, pcg


def small_scene(seed=1):
    return gi.gen_labels(gi.scene_gradcheck(), seed=seed)


def reduced(lab, b):
    A, cells = lap.dense_reduced(lab)
    return A, cells, np.array([b[p] for p in cells])


def as_grid_map(lab, cells, M):
    """The grid callable v -> M v on fluid cells (0 elsewhere) for a dense M."""
    idx = tuple(np.array(cells).T)

    def apply(v):
        out = np.zeros(lab.shape)
        out[idx] = M @ v[idx]
        return out
    return apply


def scipy_cg_iterates(A, bf, n, M=None):
    its = []
    spla.cg(A, bf, x0=np.zeros_like(bf), rtol=1e-30, maxiter=n, M=M, callback=lambda xk: its.append(xk.copy()))
    return its


@pytest.mark.parametrize("flexible", [False, True])
def test_identity_preconditioner_is_cg(flexible):
    lab = small_scene()
    b = gi.gen_rhs(lab, seed=5)
    A, cells, bf = reduced(lab, b)
    ref = scipy_cg_iterates(A, bf, 25)
    ident = as_grid_map(lab, cells, np.eye(len(cells)))
    fluid = lab == gi.FLUID
    for k in (1, 2, 5, 12, 25):
        res = pcg.solve(lab, b, ident, tol=0.0, max_iter=k, flexible=flexible, fixed_iters=True)
        assert res.iterations == k
        assert np.linalg.norm(res.x[fluid] - ref[k - 1]) <= 1e-9 * np.linalg.norm(ref[k - 1]), k


@pytest.mark.parametrize("flexible", [False, True])
def test_jacobi_preconditioner_matches_scipy_pcg(flexible):
    lab = small_scene(3)
    b = gi.gen_rhs(lab, seed=7)
    A, cells, bf = reduced(lab, b)
    Minv = np.diag(1.0 / np.diag(A))
    ref = scipy_cg_iterates(A, bf, 20, M=Minv)
    jac = as_grid_map(lab, cells, Minv)
    fluid = lab == gi.FLUID
    for k in (1, 3, 8, 20):
        res = pcg.solve(lab, b, jac, tol=0.0, max_iter=k, flexible=flexible, fixed_iters=True)
        assert np.linalg.norm(res.x[fluid] - ref[k - 1]) <= 1e-9 * np.linalg.norm(ref[k - 1]), k


def test_flexible_equals_plain_for_dense_spd_preconditioner():
    lab = small_scene(4)
    b = gi.gen_rhs(lab, seed=8)
    A, cells, _ = reduced(lab, b)
    rng = np.random.default_rng(3)
    Q = rng.standard_normal((len(cells), len(cells)))
    M = Q @ Q.T / len(cells) + np.eye(len(cells))
    P = as_grid_map(lab, cells, M)
    a = pcg.solve(lab, b, P, tol=0.0, max_iter=15, flexible=False, fixed_iters=True)
    f = pcg.solve(lab, b, P, tol=0.0, max_iter=15, flexible=True, fixed_iters=True)
    assert np.linalg.norm(a.x - f.x) <= 1e-7 * np.linalg.norm(a.x)
    np.testing.assert_allclose(f.history["beta"][1:], a.history["beta"][1:], rtol=1e-6)


def test_tiny_grid_reaches_direct_solution():
    lab = np.full((4, 4, 4), gi.SOLID, np.uint8)
    lab[1:3, 1:3, 1:3] = gi.FLUID
    lab[3, 1:3, 1:3] = gi.AIR
    lab[1, 1, 1] = gi.SOLID
    b = gi.gen_rhs(lab, seed=2)
    A, cells, bf = reduced(lab, b)
    x_ref = np.linalg.solve(A, bf)
    jac = as_grid_map(lab, cells, np.diag(1.0 / np.diag(A)))
    for flexible in (False, True):
        res = pcg.solve(lab, b, jac, tol=1e-12, max_iter=len(cells) + 5, flexible=flexible)
        assert res.status == npsdo.OK and res.iterations <= len(cells) + 2
        xs = np.array([res.x[p] for p in cells])
        np.testing.assert_allclose(xs, x_ref, rtol=1e-9, atol=1e-12)


def test_first_step_equals_npsdo_with_the_network():
    lab = small_scene(5)
    b = gi.gen_rhs(lab, seed=9, normalize=True)
    params = gi.multilevel_params(5)
    P = net.Network(params, 5, lab).apply
    a = pcg.solve(lab, b, P, tol=0.0, max_iter=1, fixed_iters=True)
    n = npsdo.solve(lab, b, P, tol=0.0, max_iter=1, n_ortho=2, fixed_iters=True)
    np.testing.assert_allclose(a.x, n.x, rtol=1e-12, atol=1e-14)


def test_flexible_term_is_active_for_the_nonsymmetric_network():
    lab = small_scene(6)
    b = gi.gen_rhs(lab, seed=10, normalize=True)
    params = gi.xavier_params(5, seed=4)
    Pn = net.Network(params, 5, lab)
    x, y = gi.gen_rhs(lab, seed=11), gi.gen_rhs(lab, seed=12)
    assert net.asymmetry(Pn, x, y) > 1e-3          # the network is not symmetric
    a = pcg.solve(lab, b, Pn.apply, tol=0.0, max_iter=3, fixed_iters=True)
    f = pcg.solve(lab, b, Pn.apply, tol=0.0, max_iter=3, flexible=True, fixed_iters=True)
    assert abs(a.history["beta"][1] - f.history["beta"][1]) > 1e-6 * abs(a.history["beta"][1])
