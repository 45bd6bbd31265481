"""Plain FP64 CPU oracle for the low-memory upwind S_N-DG method (Sun & Hauck,
"Low-memory, discrete ordinates, discontinuous Galerkin methods for radiative
transport").

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it.
The GPU library shares no code with it: the oracle assembles every matrix by
Gauss quadrature from the variational forms and solves the discrete systems
directly (or by its own straightforward reduced route), while the GPU path uses
closed-form local blocks and wavefront sweeps.

Modules
-------
quadrature  level-symmetric S_N sets satisfying conditions (i)-(iii) of Sec. 2.1
dg          Q^1 Legendre basis, mesh, and Gauss assembly of L, M, P, Q (App. A)
schemes     standard, low-memory (LMDG) and reconstructed (RLMDG) systems, direct
            solves, the reduced Krylov route of Secs. 2.1.1, 3.2, 3.3.2, scalar flux
diffusion   the eps -> 0 limit schemes of Sec. 3.1 (Q^1 CG and the Pi_0 form)
adjoint     adjoint solves and gradients of a detector functional
precond     two-level preconditioner of the reduced systems (cell blocks + the Pi_0
            diffusion limit of Sec. 3.1)

Every function states the passage of the paper it follows.  Readings of passages
that are silent, ambiguous or misprinted are listed in the module docstrings.
"""
