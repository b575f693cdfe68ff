"""CPU FP64 oracle for the implicit 3D wave-propagation analysis.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links anything here; only the tests, the smoke check and the benchmark's
CPU-baseline leg may.  It shares no code with the HIP library: the only
common module is ``casegen``, which produces seeded inputs and holds none of
the method's arithmetic.

What it computes (the plain definition the GPU path must reproduce):
  * the Galerkin semi-discretisation, on 10-node (quadratic) tetrahedra, of
    the linear elastodynamic equation of Section 2 (Eq. GE:ORG), with a
    traction-free top, viscous (Lysmer) absorbing sides and base, and the
    input velocity wave applied at the base as a force (Sections 2 and 3);
  * Rayleigh damping C = alpha M + beta K plus the dashpot matrix;
  * the Newmark-beta time march (beta = 1/4, gamma = 1/2) named in
    Section 3, with every step's linear system solved directly (sparse LU)
    or by conjugate gradients to a stated tolerance;
  * velocities at surface observation points and the misfit ERR of
    Eq. (eqerr).

Modules:
  fem      element and boundary-face matrices by numerical quadrature
  assemble global sparse matrices
  march    Newmark time march
  bsr      the same system assembled as symmetric 3x3 block-sparse FP64
           matrices and marched with block-Jacobi CG (C++/OpenMP,
           native/bsr_march.cpp), for meshes too large for SciPy
  misfit   ERR of Eq. (eqerr)
  mlp      FP64 forward/backward of the initial-guess network

Every function is pinned by a CPU test against closed forms, invariants or
exact solutions: the tests in tests/test_oracle_*.py.
"""
