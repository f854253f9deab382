"""FP64 CPU oracle for the greedy low-rank connectome regression solver.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that
the GPU library is checked against.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import it; the product path never
does, and it shares no code with the HIP library (the two meet only at the
seeded input arrays).

What it computes (Kuerschner, Dolgov, Harris & Benner, "Greedy low-rank
algorithm for spatial connectome regression"):

* ``operator``  the regularised least-squares objective (eq. obj_fun), the
  normal-equation operator A = lambda*B + C and right-hand side D
  (eq. multitermSylv), its Kronecker matrix (eq. system_matrix), the
  factored application A(U Z V^T) and the factored residual;
* ``dense``     the exact solution W* by a dense Cholesky solve of the
  Kronecker system (tiny sizes), and the closed form for Omega = 1 on
  boxes by the DCT-II diagonalisation of the graph Laplacians;
* ``als``       the ALS half-step systems (eqs. ALS_linsys, ALS_linsys_v),
  solved directly (dense / sparse LU / Sherman-Morrison-Woodbury) or by CG;
* ``galerkin``  the projected equation (eq. Proj_Sylv): Grams, the projected
  operator, a dense r^2 x r^2 solve and the matrix-valued CG;
* ``greedy``    Algorithm 1 (greedy rank-1 ALS + Galerkin);
* ``metrics``   factored Frobenius norms: residual, delta W, errors E, E_rel;
* ``rng``       SplitMix64, the counter-based generator the solver draws its
  initial ALS vectors from.

Every floating-point quantity is float64.
"""
