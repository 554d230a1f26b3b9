"""FP64 CPU oracle for the SMPM Poisson/Helmholtz Schur-complement solver.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the GPU library never does, and it
shares no code, tables or helpers with the GPU library (the seeded input
generators live in their own module, ``paper_1512_01756_amd.workloads``, which
holds none of the method's arithmetic).

Paper: Joshi, Thomsen & Diamessis, "Deflation-accelerated preconditioning of
the Poisson-Neumann Schur problem on long domains with a high-order
discontinuous element-based collocation method" (arXiv:1512.01756).

Modules
-------
gll      Gauss-Lobatto-Legendre nodes, weights, differentiation matrix (Sec. 2.2)
smpm     grid, SMPM operator L (Eq. smpm_poisson), strip split L = A + E B
         (Sec. 2.3), right-hand side f + tau g
schur    strip blocks of S = I + B A^-1 E (Eq. operator_decomp), block-Jacobi
         blocks (Sec. 3.2), deflation Z, C, P, Q (Sec. 3.3), null vectors
         (Sec. 2.4, Claim 1)
gmres    GMRES with Householder Arnoldi (Sec. 3.1)
solve    Algorithm 2 (DBJ-Schur), per-mode Helmholtz (Sec. 5), the dense direct
         solve used to pin it, and FP32-inner iterative refinement emulation
fourier  the 3-D problem through a Fourier series in y (Sec. 5): transforms
         and the mode-by-mode solve

Parity status: every function is pinned by a test in ``tests/test_oracle_*``
(printed GLL nodes, closed forms, manufactured solutions, dense direct solves,
algebraic identities).  None is "parity unpinned".
"""
