"""Plain FP64 CPU oracle for the split exponential Euler method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import this package; the HIP library
never calls it and shares no code, table or constant with it.

Everything here is written for readability against the paper
(Caliari & Cassini, "A tensor-based exponential integrator for
diffusion-reaction equations in common curvilinear coordinates"):

* ``operators``  -- grids and 1D finite-difference matrices (Section 3,
  Table 1, eqs. (A_theta), (disk_discr), (ball_discr), (syscn), (A_phi),
  (A_z)) and the phi-grid parameter sigma (Appendix A).
* ``assemble``   -- Kronecker-sum operators M = M_1 + ... + M_d
  (Section 2, eqs. (disk), (sphere), (ball), (cylinder)).
* ``phi``        -- scalar and matrix phi_1 (Section 4): symmetrised
  eigen-decomposition (Proposition 1) and, for tiny matrices, the
  exponential of the augmented block matrix.
* ``splitee``    -- the split exponential Euler step in matrix / tensor form
  (eqs. (ee_disk), (ee_sphere), (ee_ball), (ee_cylinder)) for N-coupled
  systems (eq. (BVAM_SExpE)), plus dense tiny-grid references.
* ``reactions``  -- reaction terms (eqs. (BVAMnl), (schnaknl)) and the
  builder's 3-species model; manufactured sources of Section 5.1.
* ``adjoint``    -- discrete adjoint of the split step (gradient oracle).

Parity status of each function is stated in its docstring; every
function is pinned by a ``-m "not gpu"`` test unless it says
"parity unpinned".
"""
from . import operators, assemble, phi, reactions, splitee, adjoint  # noqa: F401
