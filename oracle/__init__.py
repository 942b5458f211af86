"""CPU FP64 oracle for the neural-preconditioned Poisson solve (arXiv 2310.00177).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never calls it and shares no code with it.

Plain, slow, obviously correct NumPy in float64:
  laplacian  -- the mixed Dirichlet/Neumann 7-point matrix (Sec. "Spatial
                Discretization"), as a matvec and as a dense matrix.
  network    -- the spatially-varying-kernel network (Alg. 2, CConv and Aff
                formulas of Sec. "Architecture", 3D extension).
  npsdo      -- the NPSDO iteration (Alg. 1).
  pcg        -- PCG and flexible PCG with the network (the solver variants
                of the appendix comparing PCG variants).
  gradient   -- the training loss of Sec. "Training" and its adjoint; the
                network's transpose (the symmetric variant's second half).
  lanczos    -- Ritz-vector right-hand sides (the training-data generator).

Every function states the passage it follows.  Readings of passages that are
silent or ambiguous are collected in the design notes of the repository.

Parity status: every function is pinned by the CPU test suite against
closed forms, library routines or brute force, except the asymmetry measure
S (a diagnostic: parity unpinned).
"""
from . import gradient, lanczos, laplacian, network, npsdo, pcg  # noqa: F401
