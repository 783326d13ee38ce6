"""Plain FP64 CPU oracle of the localized model-order-reduction method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The HIP library never
calls it, links it or falls back to it.

The oracle is slow and obviously correct on purpose: numpy/scipy in float64,
scipy's SuperLU for the sparse solves and LAPACK for the dense factorizations
and the SVD, each function citing the part of the paper it follows.  It shares
no code with the HIP path; only the seeded inputs of ``workloads`` serve both.

Modules
  fem      P1 element matrices and assembly (Sections 2 and 4)
  decomp   index sets I, B, V_i, P_i, omega_0 (Sections 3, 4 and 6)
  reduce   local reduction: lifting, weights, weighted SVD, stitching (Sections 3, 4, 6)
  project  memory-efficient Galerkin projection and reduced solve (Section 6, step 3)
  solve    the full FE solution and error measures (Sections 2 and 7.1)

Parity unpinned against the paper: the basis update of Section 6, step 2 (its
details are only in the authors' code).  `reduce.basis_update` implements one
reading of it (whitening of the stitched diagonal block with a drop tolerance);
it is pinned by identities, not by the paper.
"""
from . import fem, decomp, reduce, project, solve  # noqa: F401
