"""CPU oracle for the normal-mode eigenproblem -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 implementation of what the GPU library computes, written
from the paper (Shi, Li, Xi, Saad, de Hoop: "A non-perturbative approach to
computing seismic normal modes in rotating planets", arXiv 1906.11082):

* ``refelem``  -- nodal Lagrange bases and exact reference integrals
                  (Appendix A, construction of the reference element).
* ``mesh``     -- node numbering and sparsity patterns (Sec. 4.1 and the
                  global-assembly paragraph of Appendix A).
* ``assemble`` -- the matrices of the table of implicit matrix definitions
                  (Sec. 4.2) through the element formulas of Appendix A.
* ``solve``    -- the Cowling pencil (eq. "cowling"), its sparse products,
                  the Chebyshev-Jacobi mass solve, the Jackson-Chebyshev
                  polynomial filter, filtered Lanczos and Rayleigh-Ritz
                  (Sec. 6.1 and the polynomial-filtering remark of Sec. 2.5).
* ``rotation`` -- the projected Hermitian problem for the Coriolis QEP
                  (Sec. 7, eqs. "simplequad", "linearpb", "sublinear0").
* ``dos``      -- density of states by the kernel polynomial method and
                  equal-count spectrum slices (Sec. 6.1, spectrum slicing).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  It shares no code with the GPU
library and the library never calls it.

Parity status: every function is pinned by tests in ``tests/test_oracle_*``
against closed forms, invariants or brute force, except the ones whose
docstring says "parity unpinned".
"""
