"""FP64 CPU oracle for the truncated-SVD update (test infrastructure).

This package is the checker, not the product.  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import it; the library under
``paper_2401_09703_amd`` never does, and nothing here imports that library.

Contents
  brute       O0: the definition itself, a dense SVD of the updated matrix
              (small inputs only).
  zha_simon   O1: the Zha-Simon projection scheme (Section 2.1), an exact
              factorisation of the updated matrix through the (k+s) matrix K,
              with a Householder QR of the dense augmented matrix.  This is the
              oracle the GPU path is compared with.
  svlcov      O2: the paper's own method as written, on the CPU: SV-LCOV
              modified Gram-Schmidt (Algorithm 2) and the extended
              decomposition (Section 3.2) driven by Algorithms 3, 4 and 11.
  approx      O3: the -GKL and -RPI variants (the appendix on approximating
              the augmented space): an l-dimensional basis of a Krylov or
              power-iteration subspace of the augmented matrix in place of its
              QR, then the Zha-Simon rotation with K of k + l columns.
  query       O4: Query(i) of Theorem 1 and the pair score U[i]^T Sigma V[j]
              of the link-prediction / collaborative-filtering workloads.
  rsvd        O5: the initial truncated SVD of a sparse matrix, by the
              randomised range finder with power iterations that the
              introduction cites (Halko, Martinsson and Tropp), with the
              Gaussian test matrix passed in.
  metrics     comparison metrics (singular values, principal angles,
              orthonormality, spectral-gap prefix).

Every floating-point computation is FP64.  What each function follows is cited
in its docstring by section, equation, algorithm or table of arXiv 2401.09703.
"""
from . import brute, zha_simon, svlcov, metrics  # noqa: F401
