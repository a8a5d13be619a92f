"""CPU FP64 oracle for the projection methods of Palitta & Simoncini,
"Computationally enhanced projection methods for symmetric Sylvester and
Lyapunov matrix equations".

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or runs anything here.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

It is written plainly from the paper, in float64, with NumPy/SciPy (LAPACK)
primitives as single steps, and shares no code with the GPU path: the only
common dependency is the seeded input generator package ``workloads``, which
holds no arithmetic of the method.

Modules
-------
``dense``   Krylov-free reference solutions X of A X + X A + C C^T = 0
            (Kronecker solve, diagonalisation of A, diagonal closed form,
            sine-transform diagonalisation of the 5-point Laplacian and an
            exponential-sum low-rank factor for large grids) and of the
            Sylvester equation.
``krylov``  Algorithm 1 with the block Lanczos step of Algorithm 2, the
            reduced-problem residual (Jaimoukha-Kasenally identity), the
            residual of Proposition 1 / Algorithm 3, rank truncation, the
            factor Z from the stored basis or from a second Lanczos pass, the
            explicit low-rank residual and the factor-error comparator.
``extended`` the extended Krylov variant (Section 4).
``sylvester`` two-sided projection for A X + X B + C1 C2^T = 0 (Section 5.1)
            with the corrected Algorithm 4.
``smallb``  large A and small B (Section 5.2): one Krylov space, the
            one-sided Galerkin reduction, Algorithm 5, truncated Y~ and the
            factors Z1 = V_m Q Y1, Z2 = P Y2.
``generalized`` A X E + E X A + C C^T = 0 with E symmetric positive definite,
            by the Cholesky transformation to a standard equation (Section 6,
            Example 3), and a dense Kronecker reference.
``pcg``     IC(0)/Jacobi preconditioned CG for the inner solves.
``cnn``     forward/backward of the small convolutional preconditioner.
"""
