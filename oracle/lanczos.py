"""Right-hand sides from Ritz vectors (the training-data generator of Sec.
"Training"), oracle, FP64.

The paper runs Lanczos iterations on the system matrix, takes Ritz vectors,
and forms normalised random linear combinations of them.  Readings (the
paper gives no more detail): Lanczos starts from a caller-given vector
restricted to fluid cells and keeps the basis orthonormal by full
reorthogonalisation (classical Gram-Schmidt, applied twice), or, where that
is too costly (it re-reads the whole basis every step), runs the plain
three-term recurrence; the Ritz pairs
come from the m x m tridiagonal T_m; a right-hand side is V_m Y_m c for a
caller-given coefficient vector c (the random numbers are inputs), scaled to
unit 2-norm.

TEST INFRASTRUCTURE ONLY: never called by the product path.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import laplacian


def lanczos(labels: np.ndarray, v0: np.ndarray, m: int, reorth: bool = True):
    """m Lanczos steps on A (matrix-free) from v0 restricted to fluid.

    reorth=False runs the plain three-term recurrence (the basis loses
    orthogonality as Ritz values converge, but spans the same Krylov space).

    Returns (V, alpha, beta, steps): V has shape (steps, *grid) with
    orthonormal rows v_1..v_steps; alpha[j], beta[j] are T's diagonal and
    sub-diagonal (beta[j] couples v_(j+1) and v_(j+2); the last beta is the
    norm of the final residual).  steps < m when an invariant subspace is
    reached (beta below 1e-12 of the first matvec's scale).
    """
    fluid = labels == laplacian.FLUID
    v = np.where(fluid, v0, 0.0).astype(np.float64)
    v = v / np.linalg.norm(v)
    V, alpha, beta = [], [], []
    v_prev, b_prev = np.zeros_like(v), 0.0
    scale = None
    for _ in range(m):
        V.append(v)
        w = laplacian.matvec(labels, v)
        a = float(np.sum(w * v))
        w = w - a * v - b_prev * v_prev
        if reorth:
            B = np.stack(V).reshape(len(V), -1)
            for _ in range(2):                              # full reorthogonalisation
                w = w - (B.T @ (B @ w.ravel())).reshape(w.shape)
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        scale = scale or max(abs(a), 1.0)
        if b < 1e-12 * scale:
            break
        v_prev, v, b_prev = v, w / b, b
    return np.stack(V), np.array(alpha), np.array(beta), len(V)


def ritz(alpha: np.ndarray, beta: np.ndarray):
    """Ritz values (ascending) and eigenvectors Y of the tridiagonal T_m."""
    return scipy.linalg.eigh_tridiagonal(alpha, beta[:len(alpha) - 1])


def ritz_rhs(V: np.ndarray, alpha: np.ndarray, beta: np.ndarray, coef: np.ndarray) -> np.ndarray:
    """Right-hand sides b_i = V Y c_i / ||V Y c_i|| for the columns c_i of coef (m x k).

    Returns shape (k, *grid).
    """
    _, Y = ritz(alpha, beta)
    m = V.shape[0]
    flat = V.reshape(m, -1)
    out = []
    for i in range(coef.shape[1]):
        b = flat.T @ (Y @ coef[:, i])
        out.append((b / np.linalg.norm(b)).reshape(V.shape[1:]))
    return np.stack(out)
