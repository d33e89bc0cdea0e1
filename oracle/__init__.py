"""Oracle for the ANOVA fast-summation path: plain, slow, obviously correct.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check and
the CPU-baseline leg of the benchmark may import, call, link or execute
anything in this directory.  The product library never does, and the two
share no code: no kernels, headers, helpers, tables or constant generators.
The only thing both sides use is the seeded input generator module
``workloads``, which holds none of the method's arithmetic.

Contents (each function cites the passage of the paper it writes out):

* ``direct.anova_matvec``  (K + beta I) alpha by direct O(N^2) summation in
  float64 (C + OpenMP, ``direct.c``): Sec. 2 eq. mult_with_K, Sec. 3 eq.
  extended_Gaussian_ANOVA_kernel, Sec. 5 combined kernel.
* ``direct.kernel_block`` / ``kernel_matrix``  dense kernel entries.
* ``cg.cg_solve``  plain conjugate gradients for (K + beta I) alpha = y (Sec. 2).
* ``fastsum``  NDFT / adjoint NDFT (Sec. 4.1, eqs. nfft and adjnfft), the
  sampled Fourier coefficients of the periodised kernel (Sec. 4.2), the
  analytic Gaussian coefficients, the fast summation formula with exact sums
  (Sec. 4.2, eq. fastsum) and the Kaiser-Bessel window pair.

Every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` against things other than itself: brute force on
tiny inputs, closed forms, invariants (symmetry, diagonal, positive
definiteness), special cases that reduce to library routines (numpy.fft,
numpy.linalg.solve, scipy quadrature) and the values printed in the paper's
fast-summation figure (``tests/golden/``).
"""
from . import cg, direct, fastsum  # noqa: F401
