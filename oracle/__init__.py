"""CPU FP64 oracle for the HSS-structured multifrontal solver of
Ghysels, Li, Rouet, Williams, Napov (arXiv 1502.07405).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference the HIP
library is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does, and the
oracle never imports the library.  The two share nothing but the seeded input
generators in ``paper_1502_07405_amd.problems``.

Modules
-------
rng        counter-based keyed Gaussian generator for the sampling matrix R
symbolic   fronts, update index sets and per-front HSS trees from an ordering
dense      dense fronts: extend-add and partial LU (Sec. 3)
hss        ID, randomized HSS compression (Alg. 1), HSS matvec / extraction,
           ULV-like factorization and solves (Sec. 2)
complexeq  complex systems through their real-equivalent form (Helmholtz)
mf         multifrontal factorization with dense and HSS fronts (Sec. 3, 4)
krylov     iterative refinement and GMRES(30) (Sec. 4.6, Sec. 6.1)
adjoint    transpose solve based gradients

Parity pins live in ``tests/test_oracle_*.py``.  Functions without a pin say
"parity unpinned" in their docstring.
"""
