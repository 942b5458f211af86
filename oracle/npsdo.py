"""NPSDO: steepest descent on the network-preconditioned residual with exact
line search and A-orthogonalisation against the last n_ortho directions
(Alg. 1, Sec. "Algorithm").  Oracle, FP64.

Readings (see design notes): the loop test is relative, ||r_k|| >= tol ||b||
with x_0 = 0 (the paper's "reduction of the residual norm by 10^6");
directions with index i < 1 are skipped; the orthogonalisation is applied in
place, oldest direction first, as written; the residual is the literal
r_k = b - A x_k.

TEST INFRASTRUCTURE ONLY: never called by the product path.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import laplacian
from .network import Network

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, -6


@dataclasses.dataclass
class SolveResult:
    x: np.ndarray
    iterations: int
    status: int
    rel_residual: float
    history: dict


def _dot(a, b) -> float:
    return float(np.dot(a.ravel(), b.ravel()))


def solve(labels: np.ndarray, b: np.ndarray, precond, tol: float = 1e-6,
          max_iter: int = 1000, n_ortho: int = 2, x0: np.ndarray | None = None,
          fixed_iters: bool = False, keep_dirs: bool = False) -> SolveResult:
    """Run Alg. 1.

    precond: a callable r -> d (the network P(I, .), or any other map).
    fixed_iters: run exactly max_iter iterations with no convergence test
    (the attainable-accuracy protocol of the appendix on residual capacity).
    keep_dirs: also return every d_k and r_k in the history (for invariants).
    """
    fluid = labels == FLUID_LABEL
    b = np.where(fluid, b, 0.0).astype(np.float64)
    A = lambda v: laplacian.matvec(labels, v)  # noqa: E731
    x = np.zeros(labels.shape) if x0 is None else np.where(fluid, x0, 0.0).astype(np.float64)
    r = b - A(x)
    bnorm = np.linalg.norm(b)
    hist = {"rnorm": [float(np.linalg.norm(r))], "alpha": [], "beta": [], "energy": [
        0.5 * _dot(x, A(x)) - _dot(b, x)]}
    if bnorm == 0.0:
        return SolveResult(np.zeros(labels.shape), 0, OK, 0.0, hist)
    D, AD = {}, {}          # D[i] = d_i, AD[i] = A d_i for the last n_ortho directions
    k = 0
    status = OK
    while True:
        rnorm = np.linalg.norm(r)
        if not fixed_iters and rnorm < tol * bnorm:
            break
        if k >= max_iter:
            status = NOT_CONVERGED if not fixed_iters else OK
            break
        k += 1
        d = precond(r / rnorm)
        betas = []
        for i in range(max(1, k - n_ortho), k):       # k - n_ortho <= i < k, i >= 1
            di, adi = D[i], AD[i]
            beta = _dot(d, adi) / _dot(di, adi)
            d = d - beta * di
            betas.append(beta)
        Ad = A(d)
        dAd = _dot(d, Ad)
        if not np.isfinite(dAd) or dAd <= 0.0:
            status = BREAKDOWN
            k -= 1
            break
        alpha = _dot(r, d) / dAd
        x = x + alpha * d
        r = b - A(x)
        D[k], AD[k] = d, Ad
        D.pop(k - n_ortho, None)                       # no longer in any window
        AD.pop(k - n_ortho, None)
        hist["rnorm"].append(float(np.linalg.norm(r)))
        hist["alpha"].append(alpha)
        hist["beta"].append(betas)
        hist["energy"].append(0.5 * _dot(x, A(x)) - _dot(b, x))
        if keep_dirs:
            hist.setdefault("d", []).append(d)
            hist.setdefault("r", []).append(r)
    rel = float(np.linalg.norm(r) / bnorm)
    return SolveResult(x, k, status, rel, hist)


FLUID_LABEL = laplacian.FLUID


def solve_with_network(labels, b, params, levels=6, **kw) -> SolveResult:
    """NPSDO with the network P(I, .) built from `params` (Alg. 1 with Alg. 2)."""
    net = Network(params, levels, labels)
    return solve(labels, b, net.apply, **kw)
