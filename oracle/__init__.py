"""FP64 CPU oracle for the chiral rank-k multigrid setup and solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The GPU library never uses it, and it shares no code with the GPU
path (kernels, headers, helpers, tables or constants).  Inputs come from the
standalone ``synth`` module, which holds none of the method's arithmetic.

Everything is plain NumPy complex128; LAPACK is reached only through
``numpy.linalg``.  Each function cites the passage of the paper (Whyte,
Stathopoulos, Romero, "Chiral rank-k truncations for the multigrid
preconditioner of Wilson fermions in lattice QCD", LATTICE2024) it follows.

Modules:
  lattice   -- site/neighbour/block maps (Sec. 2, domain decomposition Lambda_j)
  gamma     -- chiral-basis Dirac matrices (Sec. 2, Eq. (2) split)
  wilson    -- Wilson-Dirac operator D (Sec. 1-2), optionally with the clover term
  clover    -- clover site term of the Wilson-clover operator (Sec. 4 ensembles)
  stencil   -- generic nearest-neighbour block-stencil operator (coarse levels)
  mr        -- minimal-residual smoother (Sec. 2, Eq. (1))
  chiral    -- chiral split, truncated SVD, prolongator (Sec. 3, Eqs. (2), (5), (6))
  galerkin  -- coarse operator R D P (Sec. 2, Eq. (4))
  mg        -- setup recursion, K-cycle, flexible GCR (Sec. 2, last paragraph)

Parity pins: every function here is checked by ``tests/test_oracle_*.py``
against closed forms, invariants or brute force; none is "parity unpinned".
"""
