"""Plain FP64 CPU oracle for the vertex-star FDM/sparse relaxation solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library.

The oracle writes out, step by step and in the paper's order, what the
method computes (Brubeck & Farrell, "A scalable and robust vertex-star
relaxation for high-order FEM", Sec. 2):

* ``gll``       -- GLL nodes/weights and the Lagrange basis (Sec. 2.1)
* ``fdm1d``     -- reference-interval stiffness/mass matrices, the interior
                   generalized eigenproblem and the FDM dual basis (Sec. 2.2-2.4)
* ``mesh``      -- trilinear cell maps, the weighted inverse metric and the
                   separable surrogate coefficients (Sec. 2.7)
* ``operator``  -- the Galerkin stiffness operator, assembled (definition)
                   and sum-factorized, and the load vector (Sec. 2.1)
* ``transfer``  -- GLL<->FDM basis change and the Q1 coarse space (Sec. 2.4, 2.5)
* ``patches``   -- vertex-star patches and their solves (Sec. 2.5, 2.6)
* ``gmg``       -- geometric multigrid for the Q1 coarse problem (Sec. 2.8)
* ``solver``    -- Lanczos damping, hybrid V(1,1) preconditioner, PCG (Sec. 2.5, 2.8)

Everything is float64 numpy/scipy.  Library primitives (matmul, symmetric
eigensolver, dense Cholesky) serve as individual steps; there is no blocking
or fusion beyond what the paper states.
"""
