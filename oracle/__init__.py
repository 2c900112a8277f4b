"""CPU oracle for the MRCQR factorization (TEST INFRASTRUCTURE ONLY).

This package is the slow, plain reference the GPU library is checked
against. Only the tests, the smoke check and the bench's CPU-baseline leg
may import it; the library itself never does, and it shares no code with
the HIP kernels (the two implement the same written definitions
independently). All floating point is float64 unless the paper fixes a
lower precision for a step (the sketch, and the sketch QR in single
precision when the sketch is half/bfloat16/single).

Modules
  rng        counter-based draw of the Rademacher signs D and the sample set S
  precision  rounding to FP32 / FP16 / BF16 and the block power-of-two prescale
  sketch     the subsampled DCT-II sketch  Y = S F D A  by its definition
  householder  textbook Householder thin QR (the stable reference)
  cholqr     forward substitution, Gram, Cholesky, R product (Algorithm 1 pieces)
  condest    incremental condition estimation (Bischof 1990) on triangular R
  mrcqr      the three stages of Algorithm 2 in order, plus the adaptive policy
  metrics    orthogonality and backward error with accurate accumulation
"""
from . import rng, precision, sketch, householder, cholqr, condest, mrcqr, metrics  # noqa: F401
