"""Plain FP64 CPU oracle for the implicit difference schemes of Gu, Sun, Zhang & Zhao
(fast implicit difference schemes for time-space fractional diffusion with the
integral fractional Laplacian).

TEST INFRASTRUCTURE ONLY.  It exists to check the GPU library, not to be used
by it: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import or call anything in this package.  It shares
no code with the HIP library (no kernels, headers, tables or helpers) and it
imports nothing from the library package.

What it computes is the direct scheme (DIDS, eq. (3.16) / matrix form (4.1)):
the full graded-L1 history sum at every step, the dense IFL matrix A of
(3.16x), and a dense LU solve (LAPACK ``gesv``) per time level.  The fast
scheme (FIDS) that the GPU implements differs from it only by the
sum-of-exponentials tolerance (Theorem 3.4) and the Krylov tolerance.

Every function is pinned by tests under ``tests/test_oracle_*.py`` against
values printed in the paper's tables, closed forms, invariants of Prop. 3.1 /
Lemma 4.1 and brute force; see the docstrings for the passage each follows.
"""
from .fids_oracle import (  # noqa: F401
    c1_alpha, graded_mesh, step_sizes, l1_weights, ifl_column, ifl_matrix,
    strang_column, dids_solve, dids_adjoint, errors,
    soe_relative_error, fids_history_weights,
)
from .ifl2d import (  # noqa: F401
    c2_alpha, corner_integral, cell_integrals, node_weights, exterior_integral, lattice_error, mu_star,
    ifl2d_coefficients, ifl2d_matrix, ifl2d_apply_at, grid as grid2d, dids2d_solve,
)
