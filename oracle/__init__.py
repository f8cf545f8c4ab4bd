"""FP64 CPU oracle for partial-circulant LASSO recovery (test infrastructure).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  The HIP library never
calls it, links it or falls back to it, and it shares no code with the HIP
path: the two meet only through the seeded float32 inputs of `workloads`.

What it computes (paper: Fiandrotti, Fosson, Ravazzi, Magli, arXiv 1707.02244):

* dense.py   -- the plain definitions with an explicit dense A = P C:
                the sensing model y = A x (Eq. 1), the LASSO objective (Eq. 3),
                the soft threshold (Eq. 4), ISTA (Alg. 1) and ADMM (Alg. 2)
                with a brute-force Cholesky factor of A^T A + rho I.
* fftref.py  -- the same operators and solvers evaluated through numpy's FFT
                (circulant matrices are diagonalised by the DFT, Section 4.2),
                for sizes where a dense A cannot be stored; ADMM's inverse is
                applied with the Woodbury identity through the m x m
                circulant A A^T.
* problem.py -- turns a `workloads` draw into the float32 problem instance
                (y = A x*, step size, lambda) that both sides solve.
* unrolled.py / twod.py -- the unrolled-ISTA adjoint and the 2-D operator.

Readings of the paper that the oracle fixes (the paper is silent, ambiguous
or garbled on these points):

* Objective: 1/2 ||y - A x||^2 + lam ||x||_1 with lam = alpha of Eq. 3 (same
  minimiser as Eq. 3; makes Alg. 2's threshold alpha/rho the scaled-form ADMM).
* ISTA threshold is tau*lam (proximal gradient).  Alg. 1 prints eta_alpha;
  with tau folded in, lam_max = ||A^T y||_inf holds exactly.
* C is stored by its first COLUMN: C[i,j] = c[(i-j) mod n].
* P keeps rows 0, d, 2d, ..., (m-1)d (Section 4.3 chooses Omega at random;
  an every-d-th selection keeps A A^T circulant).
* y has length m (the algorithm headers print y in R^n).
* Strict '>' in the threshold: |v| == gamma maps to 0 (Eq. 4).
"""
