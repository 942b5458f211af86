"""Pins for the oracle's mixed-BC Laplacian (Sec. "Spatial Discretization").

Each test checks the oracle against something other than itself: an entry-by-
entry assembly loop, symmetry / definiteness / row-sum invariants, the
separable closed-form eigenpairs of a tank, and a DST-I exact solve of the
Dirichlet box.
"""
import numpy as np
import pytest
import scipy.fft

import nps_inputs as gi
from oracle import laplacian as lap

FLUID, AIR, SOLID = gi.FLUID, gi.AIR, gi.SOLID


def random_labels(shape, seed, p=(0.6, 0.2, 0.2)):
    rng = np.random.default_rng(seed)
    return rng.choice(3, size=shape, p=p).astype(np.uint8)


@pytest.mark.parametrize("seed", range(4))
def test_matvec_matches_entrywise_assembly(seed):
    lab = random_labels((5, 6, 7), seed)
    A, cells = lap.dense_reduced(lab)
    x = np.random.default_rng(100 + seed).standard_normal(lab.shape)
    y = lap.matvec(lab, x)
    xf = np.array([x[p] for p in cells])
    np.testing.assert_allclose([y[p] for p in cells], A @ xf, rtol=0, atol=1e-13)
    assert np.all(y[lab != FLUID] == 0.0)


@pytest.mark.parametrize("seed", range(3))
def test_reduced_matrix_symmetric_and_row_sums(seed):
    lab = random_labels((6, 5, 6), seed)
    A, cells = lap.dense_reduced(lab)
    assert np.array_equal(A, A.T)
    nz, ny, nx = lab.shape
    for i, p in enumerate(cells):
        n_air = 0
        for d in lap.NEIGHBOURS:
            q = tuple(np.add(p, d))
            if all(0 <= q[a] < lab.shape[a] for a in range(3)) and lab[q] == AIR:
                n_air += 1
        assert A[i].sum() == n_air


def test_reduced_matrix_spd_for_generated_scene():
    lab = gi.gen_labels(gi.scene_gradcheck(), seed=3)
    A, _ = lap.dense_reduced(lab)
    np.linalg.cholesky(A)  # raises if not positive definite
    assert np.array_equal(A, A.T)


def tank(N, h):
    lab = np.full((N, N, N), SOLID, dtype=np.uint8)
    lab[1:h, 1:N - 1, 1:N - 1] = FLUID
    lab[h:N - 1, 1:N - 1, 1:N - 1] = AIR
    return lab


@pytest.mark.parametrize("a,b,c", [(0, 0, 0), (1, 2, 0), (3, 1, 2), (5, 5, 4)])
def test_tank_closed_form_eigenpairs(a, b, c):
    """Neumann walls and floor, Dirichlet free surface: separable DCT eigenpairs."""
    N, h = 12, 8
    lab = tank(N, h)
    n, m = N - 2, h - 1
    i = np.arange(n) + 0.5
    iz = np.arange(m) + 0.5
    vx = np.cos(np.pi * a * i / n)
    vy = np.cos(np.pi * b * i / n)
    th = np.pi * (2 * c + 1) / (2 * m + 1)
    wz = np.cos(th * iz)
    lam = (2 - 2 * np.cos(np.pi * a / n)) + (2 - 2 * np.cos(np.pi * b / n)) + (2 - 2 * np.cos(th))
    u = np.zeros(lab.shape)
    u[1:h, 1:N - 1, 1:N - 1] = wz[:, None, None] * vy[None, :, None] * vx[None, None, :]
    np.testing.assert_allclose(lap.matvec(lab, u), lam * u, atol=1e-12)


def test_air_surrounded_box_matches_dst_solve():
    """A fluid block with air on every face is the textbook Dirichlet Laplacian."""
    n = 9
    lab = np.full((n + 4,) * 3, SOLID, dtype=np.uint8)
    lab[1:n + 3, 1:n + 3, 1:n + 3] = AIR
    lab[2:n + 2, 2:n + 2, 2:n + 2] = FLUID
    rng = np.random.default_rng(7)
    bb = rng.standard_normal((n, n, n))
    k = np.arange(1, n + 1)
    mu = 2 - 2 * np.cos(np.pi * k / (n + 1))
    lam = mu[:, None, None] + mu[None, :, None] + mu[None, None, :]
    xb = scipy.fft.dstn(scipy.fft.dstn(bb, type=1, norm="ortho") / lam, type=1, norm="ortho")
    x = np.zeros(lab.shape)
    x[2:n + 2, 2:n + 2, 2:n + 2] = xb
    y = lap.matvec(lab, x)
    np.testing.assert_allclose(y[2:n + 2, 2:n + 2, 2:n + 2], bb, atol=1e-12)


def test_values_outside_fluid_are_ignored():
    lab = random_labels((4, 4, 4), 11)
    x = np.random.default_rng(1).standard_normal(lab.shape)
    x2 = x.copy()
    x2[lab != FLUID] = 1e6
    np.testing.assert_array_equal(lap.matvec(lab, x), lap.matvec(lab, x2))


def test_grid_boundary_counts_as_solid():
    """An all-fluid grid: diagonal = number of in-grid neighbours."""
    lab = np.zeros((3, 3, 3), dtype=np.uint8)
    assert lap.diag_count(lab)[1, 1, 1] == 6
    assert lap.diag_count(lab)[0, 0, 0] == 3
    assert lap.diag_count(lab)[0, 1, 1] == 5
