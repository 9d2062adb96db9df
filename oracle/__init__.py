"""Plain FP64 CPU oracle for the adaptive multigrid of Brannick, Brower, Clark, Osborn
and Rebbi, "Adaptive Multigrid Algorithm for the QCD Dirac-Wilson Operator"
(Lattice 2007, arXiv:0710.3612).

THIS PACKAGE IS TEST INFRASTRUCTURE.  It exists to check the GPU library; it is
never part of the product path.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.

It is deliberately slow and literal: operators are scipy sparse matrices built
entry by entry from the paper's formulas, the coarse operator is the matrix
product P^H A P of Eq. (2), and the V-cycle follows the five steps of the
Multigrid section in the paper's order.  It shares no code with the HIP library.

Modules
-------
wilson     the Wilson-Dirac matrix D (Introduction), D^H and A = D^H D.
multigrid  smoother calibration, aggregates, block Gram-Schmidt, Galerkin
           operator, V-cycle, coarsest solve, adaptive setup, CG and MG-CG.
"""

from .wilson import dirac_matrix, normal_matrix, GAMMA, SIGMA3
from . import multigrid

__all__ = ["dirac_matrix", "normal_matrix", "GAMMA", "SIGMA3", "multigrid"]
