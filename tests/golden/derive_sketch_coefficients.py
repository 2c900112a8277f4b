"""Derives tests/golden/sketch_coefficients.txt from the mathematics alone
(no import of the oracle): 60-digit cosines, then round-to-nearest-even
onto each format's grid by exact rational arithmetic.

Case: m = 8 rows, sampled DCT-II rows S = [1, 2] with s = 2, so both
normalizations gamma_k = sqrt(2/s) equal 1 and every expected value is a
plain grid point. Signs d = (+1, +1, +1, -1, +1, +1, -1, +1).
Columns 0..7 of A are the unit vectors e_0..e_7, so
    Y[i, j] = fl_p(cos(pi (2j+1) k_i / 16)) * d_j
which is exact in float32: these entries pin the rounding of the cosine
coefficients to the sketch precision p. Column 8 holds 1 in row 0 and
2^-20 in row 1 (both exact in every format, no block prescale effect), so
    Y[i, 8] = fl_32(fl_p(c(k_i, 0)) + 2^-20 fl_p(c(k_i, 1)))
whose exact sum needs more than 24 significant bits: this entry pins the
final rounding of Y to float32 (the sketch accumulates in float32).

Formats: binary16 keeps 11 significant bits, bfloat16 8, binary32 24.
Run: python tests/golden/derive_sketch_coefficients.py > tests/golden/sketch_coefficients.txt
"""
from fractions import Fraction

import mpmath

mpmath.mp.dps = 60
M = 8
S = [1, 2]
D = [1, 1, 1, -1, 1, 1, -1, 1]
BITS = {"fp16": 11, "bf16": 8, "fp32": 24}


def grid_round(x: Fraction, bits: int) -> Fraction:
    """Nearest-even point of the `bits`-significant-bit grid (normal range)."""
    if x == 0:
        return x
    sgn = 1 if x > 0 else -1
    x = abs(x)
    e = 0
    while x >= Fraction(2) ** (e + 1):
        e += 1
    while x < Fraction(2) ** e:
        e -= 1
    q = Fraction(2) ** (e - bits + 1)
    k = x / q
    f = k.numerator // k.denominator
    r = k - f
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and f % 2 == 1):
        f += 1
    return sgn * f * q


def coef(k: int, t: int) -> Fraction:
    phi = ((2 * t + 1) * k) % (4 * M)
    return Fraction(mpmath.nstr(mpmath.cos(mpmath.pi * phi / (2 * M)), 55))


def main():
    print("# Subsampled DCT-II sketch of unit-vector columns: hand-checkable values")
    print("# (derivation and case in derive_sketch_coefficients.py beside this file).")
    print("# m = 8, S = [1, 2], s = 2 (gamma = 1), d = +1 +1 +1 -1 +1 +1 -1 +1;")
    print("# columns 0..7 = e_0..e_7, column 8 = e_0 + 2^-20 e_1.")
    print("# format  i  j  Y[i,j] (float64 hex)")
    for fmt, bits in BITS.items():
        for i, k in enumerate(S):
            for j in range(M):
                y = grid_round(coef(k, j), bits) * D[j]
                print(f"{fmt} {i} {j} {float(y).hex()}")
            exact = grid_round(coef(k, 0), bits) * D[0] + Fraction(1, 2 ** 20) * grid_round(coef(k, 1), bits) * D[1]
            y = grid_round(exact, 24)
            assert y != exact
            print(f"{fmt} {i} 8 {float(y).hex()}")


if __name__ == "__main__":
    main()
