"""CPU FP64 oracle for the multi-case element-by-element (EBE) solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
reference of what the GPU path computes, written from the paper (Yamaguchi
et al., "Implicit Low-Order Unstructured Finite-Element Multiple Simulation
Enhanced by Dense Computation using OpenACC", WACCPD 2017) and from textbook
finite-element theory.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does and
shares no code, tables or helpers with it.

Modules
-------
fem      element stiffness by isoparametric B-matrix quadrature (Eq. (1), Eq. (2)),
         global assembly K = sum_i Q_i K_i Q_i^T (Eq. (3)), EBE product by definition.
solve    Dirichlet elimination, dense Cholesky, sparse direct, block-Jacobi PCG,
         the paper's adaptive (flexible) CG of Algorithm 1.
alg1     Algorithm 1 (outer flexible CG, inner CG levels 0, 1 and optionally 2).
amg      level 2: aggregation of the corner graph, P2, A2 = P2^T K1 P2 (Section 2,
         "inner loop level 2"; the coarsening itself is a reading, see the module).
adjoint  misfit, adjoint solve and dL/dE_e (extension beyond the paper).
greens   split-node forces of unit fault slips, Green's functions at surface
         stations, the regularised inversion of Eq. (5) with the L-curve (Section 5).
material Lame parameters; (Vp, Vs, rho) -> (E, nu) for Table 3.

Parity status: every function here is pinned by tests under ``tests/`` against
closed forms, invariants, brute force or library routines, except the
iteration counts and intermediate values of Algorithm 1's preconditioner
("parity unpinned": any valid preconditioner gives the same converged u).
"""
