"""Plain, slow FP64 CPU oracle for the full multigrid method of Jia, Xie, Xie and Xu,
"A Full Multigrid Method for Nonlinear Eigenvalue Problems" (arXiv:1502.04657).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the HIP library:
meshes, element matrices, transfer operators and solvers are all built here from the
paper's definitions with generic finite-element loops (numpy / scipy.sparse).

Modules
  mesh   -- nested uniform simplicial meshes and P1 spaces (Section 2, (2.3); (3.1)-(3.2))
  fem    -- exact P1 integration of the forms a-hat, b, the potential and the nonlinear
            term (weak form (2.2), (2.4), Example 4.1)
  mg     -- red-black symmetric Gauss-Seidel V-cycle for the auxiliary problem (3.4)-(3.5)
  scf    -- self-consistent-field solves of the small nonlinear eigenproblems
            (Algorithm 3.2 step 1 and (3.6))
  fmg    -- one correction step (Algorithm 3.1) and the full multigrid scheme
            (Algorithm 3.2), fixed schedule (O1) and converged (O2)

Parity status: every function is pinned by a `-m "not gpu"` test against closed forms,
brute-force dense eigensolves or invariants, except the exact iterate sequence of the
fixed FMG schedule, which the paper does not print; that schedule is pinned only through
Theorem 3.1/3.2 behaviour and agreement with the converged discrete solution.
"""
