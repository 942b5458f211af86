"""The discrete Poisson matrix with mixed boundary conditions (oracle, FP64).

Sec. "Spatial Discretization": pressure lives at cell centres; the standard
7-point stencil is used, stencil points outside the fluid are dropped, and the
diagonal entry is the number of neighbouring cells that are fluid or air.
Rows and columns of non-fluid cells are empty.  Cells outside the grid count
as solid (Sec. "Boundary Conditions").  Unit spacing; the positive-definite
sign convention (diagonal positive, off-diagonals -1).

TEST INFRASTRUCTURE ONLY: never called by the product path.
"""
from __future__ import annotations

import numpy as np

FLUID, AIR, SOLID = 0, 1, 2

# The six face neighbours (dz, dy, dx).
NEIGHBOURS = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))


def shifted(a: np.ndarray, off, fill) -> np.ndarray:
    """b[p] = a[p + off] where p + off lies in the grid, else `fill` (last 3 axes)."""
    pad = [(0, 0)] * (a.ndim - 3) + [(1, 1)] * 3
    ap = np.pad(a, pad, mode="constant", constant_values=fill)
    nz, ny, nx = a.shape[-3:]
    oz, oy, ox = off
    return ap[..., 1 + oz:1 + oz + nz, 1 + oy:1 + oy + ny, 1 + ox:1 + ox + nx]


def diag_count(labels: np.ndarray) -> np.ndarray:
    """Number of face neighbours in fluid or air (out-of-grid counts as solid)."""
    open_ = (labels == FLUID) | (labels == AIR)
    cnt = np.zeros(labels.shape, dtype=np.int64)
    for off in NEIGHBOURS:
        cnt += shifted(open_, off, False)
    return cnt


def matvec(labels: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = A x on the full grid; entries of x outside fluid are ignored, y is 0 there."""
    fluid = labels == FLUID
    xf = np.where(fluid, x, 0.0).astype(np.float64)
    y = diag_count(labels) * xf
    for off in NEIGHBOURS:
        y -= shifted(xf, off, 0.0)
    y[~fluid] = 0.0
    return y


def dense_reduced(labels: np.ndarray):
    """(A_tilde, fluid_index): the n_f x n_f reduced matrix built entry by entry.

    A plain loop over fluid cells, for tiny grids only: used to check `matvec`
    and to solve with a dense factorisation.
    """
    nz, ny, nx = labels.shape
    cells = [p for p in np.ndindex(nz, ny, nx) if labels[p] == FLUID]
    index = {p: i for i, p in enumerate(cells)}
    A = np.zeros((len(cells), len(cells)))
    for p in cells:
        i = index[p]
        for dz, dy, dx in NEIGHBOURS:
            q = (p[0] + dz, p[1] + dy, p[2] + dx)
            inside = 0 <= q[0] < nz and 0 <= q[1] < ny and 0 <= q[2] < nx
            if not inside:
                continue  # outside the grid is solid: dropped, not counted
            if labels[q] == FLUID:
                A[i, i] += 1.0
                A[i, index[q]] -= 1.0
            elif labels[q] == AIR:
                A[i, i] += 1.0
    return A, cells


def residual(labels: np.ndarray, b: np.ndarray, x: np.ndarray) -> np.ndarray:
    """r = b - A x restricted to fluid cells (b outside fluid is ignored)."""
    fluid = labels == FLUID
    return np.where(fluid, b, 0.0) - matvec(labels, x)


def rel_residual(labels: np.ndarray, b: np.ndarray, x: np.ndarray) -> float:
    """||b - A x||_2 / ||b||_2 over fluid cells, in FP64."""
    fluid = labels == FLUID
    bn = np.linalg.norm(np.where(fluid, b, 0.0))
    return float(np.linalg.norm(residual(labels, b, x)) / bn) if bn > 0 else 0.0
