"""FP64 CPU oracle for the subspace-accelerated sequence solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product path (the HIP library and
its Python binding) never imports, calls or links anything in here, and this package
imports nothing from the product path; the two share only the seeded input
generators in ``gen``.

What each module follows (sections / equations / algorithms of arXiv 2309.02156):

* ``philox``   - the counter-based generator the method's random draws come from
                 (Philox4x64-10 of Salmon et al., SC'11) and Box-Muller normals.
* ``sketch``   - the left sketch S (Gaussian or subsampled randomized Hadamard).
* ``basis``    - Alg. 1 (basis) with the randomized range finder of Section 2.2
                 (Alg. 3 (initialisation and reduced QR of Omega)), the sketched-QR orthonormalisation, the
                 reduced problem of Alg. 1 (reduced problem) (Section 2 minimum residual, plus
                 the Galerkin variant), POD (Alg. 2) and the literal progressive
                 update of Alg. 3 (rank-one updates of Omega) with periodic refresh.
* ``krylov``   - CG (Hestenes-Stiefel) and restarted GMRES (Saad-Schultz) with
                 modified Gram-Schmidt and Givens rotations (Section 1, Alg. 1 (Krylov solve)).
* ``sequence`` - the per-step driver of Alg. 1 over a stream of systems (eq. (seq)).
* ``theory``   - the bounds of Theorems 1 and 2 and eq. (errorrandsvd), used as pins.

Parity status of each function is stated in its docstring; the functions whose
results no independent pin fixes say "parity unpinned".
"""
