"""FP64 CPU oracle for the TR-BDF2 / discontinuous Galerkin projection scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark do.  The oracle is a plain, slow transcription of the
paper's definitions (Orlando, Della Rocca, Barbante, Bonaventura, Parolini,
"An efficient and accurate implicit DG solver for the incompressible
Navier-Stokes equations", arXiv 2107.07776):

* ``basis``    - Gauss-Legendre rule and Lagrange bases on [0,1] (Sec. 3, the
                 spaces Q_k and Q_{k-1}).
* ``mesh``     - structured hexahedral / quadrilateral box meshes, optionally
                 Q1-mapped, periodic or with boundary faces (Sec. 3, T_h and E).
* ``forms``    - dense per-cell and per-face tabulation of the bilinear,
                 trilinear and linear forms of Sec. 3 (eq. bilin_diff,
                 eq. trilinear, eq. rhs1, the pressure SIP form a_p, the
                 functionals F_p and the projection matrix P) assembled into
                 scipy CSR matrices.
* ``stepper``  - the two TR-BDF2 stages in algebraic form (Sec. 2 eqs.
                 first_stage, helmholtz2a, second_stage, helmholtz3a and the
                 algebraic systems at the end of Sec. 3), solved directly.
* ``projection`` - the Bell-Colella-Glaz (Crank-Nicolson) and Guermond-
                 Quartapelle (BDF2) projection steps of Sec. 2 on the same
                 forms (eq. momentum_BCG, helmholtz_BCG, momentum_HI,
                 helmholtz_HI).
* ``adaptive`` - 2D quadtree meshes with hanging nodes, a_p and M^p on
                 them, the refinement indicator, marking and field transfer
                 of the adaptive runs of Sec. 4.

Closed-form reference fields (Taylor-Green, Kovasznay) live in the separate
``synthetic`` package, which holds no arithmetic of the method.

Every operator is an assembled sparse matrix: no sum factorisation, no
fusion.  Readings of passages that are silent or garbled are listed in the
module docstrings where they are applied.
"""

from .basis import gauss_legendre_01, lagrange_values, lagrange_derivatives
from .mesh import BoxMesh
from .forms import Discretization
from .stepper import TRBDF2, trbdf2_constants, trbdf2_scalar_step
from .projection import BCG, BDF2GQ

__all__ = [
    "gauss_legendre_01", "lagrange_values", "lagrange_derivatives",
    "BoxMesh", "Discretization", "TRBDF2", "trbdf2_constants", "trbdf2_scalar_step",
    "BCG", "BDF2GQ",
]
