"""FP64 CPU oracle for the QTT finite element method for 2-D elasticity.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark use it.
It shares no code with the HIP path: the only common module is ``workloads``,
which holds seeded input parameters and no arithmetic of the method.

Modules
-------
fem        plain sparse Q1 finite elements: element loop with 2x2 Gauss
           quadrature (Sec. 3.2-3.4), consistent loads (the load-vector
           equation of Sec. 3.5), Dirichlet masks (Sec. 3.8), subdomain coupling
           (Sec. 3.6.1 and the solution-concatenation subsection) and a
           sparse direct solve.
qtt        plain tensor-train algebra on NumPy arrays: TT-SVD and TT
           rounding (the cited Oseledets algorithms 1 and 2), matrix-vector
           product by the strong Kronecker product of cores (Sec. 4),
           sums, inner products, Hadamard and matrix-matrix products.
assembly   the QTT stiffness matrix and load vector built directly in
           Z-ordered QTT form from 1-D factors (Alg. 1 with z-kron).
solve      TT conjugate gradients with FP64 iterative refinement.
"""
