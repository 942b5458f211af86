"""PCG and flexible PCG with the network as preconditioner (oracle, FP64).

The solver variants the paper compares NPSDO against (Sec. "Algorithm" and
the appendix comparing PCG variants).  The paper cites them without writing
them out; this oracle takes the textbook forms:
  * PCG (Shewchuk's preconditioned conjugate gradients):
        s_k = P(r_k),  delta_k = r_k . s_k,
        d_1 = s_1,  d_k = s_k + beta_k d_(k-1),  beta_k = delta_k / delta_(k-1),
        alpha_k = delta_k / (d_k . A d_k),  x_k = x_(k-1) + alpha_k d_k;
  * flexible PCG (the Polak-Ribiere form of Bouwmeester, Dougherty and
    Knyazev for nonsymmetric preconditioners, one more dot product):
        beta_k = s_k . (r_k - r_(k-1)) / delta_(k-1), otherwise as PCG.
Shared readings with the NPSDO oracle: x_0 = 0, relative stopping test
||r_k|| < tol ||b||, literal residual r_k = b - A x_k every iteration.  The
preconditioner is applied to r_k / ||r_k|| as in Alg. 1 and the result
scaled back by ||r_k||: the network is linear in its input vector, so this is
P(r_k) up to rounding.

TEST INFRASTRUCTURE ONLY: never called by the product path.
"""
from __future__ import annotations

import numpy as np

from . import laplacian
from .npsdo import BREAKDOWN, NOT_CONVERGED, OK, SolveResult


def _dot(a, b) -> float:
    return float(np.dot(a.ravel(), b.ravel()))


def solve(labels: np.ndarray, b: np.ndarray, precond, tol: float = 1e-6, max_iter: int = 1000,
          flexible: bool = False, fixed_iters: bool = False, keep_dirs: bool = False) -> SolveResult:
    """PCG (flexible=False) or flexible PCG (flexible=True) on A x = b.

    precond: a callable v -> P(v), linear in v.  History: rnorm, alpha, beta
    per iteration (and d, r with keep_dirs).
    """
    fluid = labels == laplacian.FLUID
    b = np.where(fluid, b, 0.0).astype(np.float64)
    A = lambda v: laplacian.matvec(labels, v)  # noqa: E731
    x = np.zeros(labels.shape)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    hist = {"rnorm": [float(bnorm)], "alpha": [], "beta": []}
    if bnorm == 0.0:
        return SolveResult(np.zeros(labels.shape), 0, OK, 0.0, hist)
    d = None
    r_prev = None
    delta_prev = None
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
        s = rnorm * precond(r / rnorm)
        delta = _dot(r, s)
        if d is None:
            beta = 0.0
            d = s
        else:
            num = _dot(s, r - r_prev) if flexible else delta
            beta = num / delta_prev
            d = s + beta * d
        Ad = A(d)
        dAd = _dot(d, Ad)
        if not np.isfinite(dAd) or dAd <= 0.0 or not np.isfinite(delta):
            status = BREAKDOWN
            k -= 1
            break
        alpha = delta / dAd
        x = x + alpha * d
        r_prev, delta_prev = r, delta
        r = b - A(x)
        hist["rnorm"].append(float(np.linalg.norm(r)))
        hist["alpha"].append(alpha)
        hist["beta"].append(beta)
        if keep_dirs:
            hist.setdefault("d", []).append(d)
            hist.setdefault("r", []).append(r)
    rel = float(np.linalg.norm(r) / bnorm)
    return SolveResult(x, k, status, rel, hist)
