"""Seeded synthetic inputs shared by the tests, the bench and the oracle.

This module only draws random numbers and builds matrices with prescribed
structure. It holds none of the factorization's arithmetic (no sketch, no
triangular solve, no Cholesky): both the CPU oracle and the GPU path receive
the same arrays from here and must agree on what they compute from them.

The test-matrix family is A = U diag(sigma) V^T with U, V having orthonormal
columns and geometric singular values, so that kappa_2(A) is known by
construction (the paper's experimental setup, Section "Numerical Stability",
builds its matrices the same way; here U and V come from Gaussians and sigma
runs from 1 down to 1/kappa).
"""
from .matrices import (
    test_matrix,
    test_matrix_factors,
    singular_values,
    gaussian,
    upper_triangular,
    spd_matrix,
    instance_mix,
    rising_kappas,
    device_test_matrix,
    paper_sweep_matrix,
)

__all__ = [
    "test_matrix",
    "test_matrix_factors",
    "singular_values",
    "gaussian",
    "upper_triangular",
    "spd_matrix",
    "instance_mix",
    "rising_kappas",
    "device_test_matrix",
    "paper_sweep_matrix",
]
