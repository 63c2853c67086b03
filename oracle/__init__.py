"""CPU oracle for the randomized range finder and randomized SVD.

TEST INFRASTRUCTURE ONLY.  Plain, slow float64 numpy written from the paper
(P.-G. Martinsson, "Randomized methods for matrix computations").  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import
it; the product path never does, and the oracle imports nothing from the
product package.  It shares no code, headers, tables or helpers with the HIP
library.

Modules
  philox   counter-based Philox4x32-10 generator and Box-Muller Gaussians
           (Salmon, Moraes, Dror, Shaw, SC'11), used to reproduce a test
           matrix from a seed.
  rsvd     orth, the small SVD, Figures 1/4/5 (basic, power and
           re-orthonormalised power RSVD), the Gaussian-probe bound
           (Lemma of Section 13), the certificate of Section 14, the
           adaptive range finders of Sections 12-13.
  quant    round-to-nearest-even bfloat16 and block-scaled FP8 (E4M3)
           rounding used by the quantisation-aware mode.
  mlp      float64 forward/backward of the (p, q) selector network.
  batched  per-block tolerance driver for the batched workload.
  srft     the structured test matrix of Section 6 (random signs, Walsh-
           Hadamard transform, subsampled columns) and Figure 5 with it.
  nystrom  the Nystrom eigenvalue decomposition of Section 9 for symmetric
           positive semidefinite matrices, with a dropping Cholesky.
  idcur    partial column-pivoted QR, the column / row ID, the randomized
           row ID and the randomized CUR of Sections 10-11.
  singlepass  the single-pass factorisations of Section 5 (symmetric EVD
           and general SVD, each entry of A read once), least squares on
           the vectorised systems.

Parity status of each function is listed in its docstring; every function
here is pinned by a ``-m "not gpu"`` test unless it says "parity unpinned".
"""
