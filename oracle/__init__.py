"""FP64 CPU oracle for entropy-regularized optimal transport by Sinkhorn scaling.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call,
link or execute anything under this directory; only the test suite, the smoke
check of the entry module and the CPU-baseline leg of the benchmark do.  It
shares no code, tables or constants with the HIP path: every function here is
written directly from the definitions of the paper (Lakshmanan, Pichler, Potts,
"Nonequispaced Fast Fourier Transform Boost for the Sinkhorn Algorithm",
arXiv 2201.07524), slowly and in double precision:

* ``sinkhorn_dense``  - the dense Gibbs kernel, Algorithm 1, the dual
  (Proposition 2.3, eq. (14)), the result formula of Algorithm 3, the primal
  cost (eq. (15)), the residual (eq. (Error)) and the envelope gradient.
* ``ndft``            - the trigonometric sums of the fast summation
  (Section 3.1, eq. (fastsum)) evaluated directly, and the Fourier
  coefficients of the periodized Gaussian kernel (eq. (ansatz_NFFT)).
* ``direct``          - a matrix-free FP64 kernel sum in plain C with OpenMP
  (``direct_sum.c``) for point clouds too large for a dense matrix.

Every function is pinned in ``tests/test_oracle_pins.py`` against closed
forms, invariants of the paper's lemmas and brute force on tiny inputs.
"""
