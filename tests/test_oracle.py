"""Pins of the CPU oracle against facts fixed by mathematics, not by the oracle itself.

The oracle computes, per entry, beta*c + alpha*sum_p a_ip b_pj (the ordinary
matrix product of Sec. 2.1) with a compensated dot product.  Each test below
checks it against an independent truth: exact rational arithmetic, integer
arithmetic, identity/permutation/rank-1 closed forms, or a symmetry of the
definition.  A dropped error term, a sign error, a wrong index or a transposed
operand in the oracle fails at least one of them (tests/test_oracle_mutants.py
plants such mistakes in a copy of the oracle and checks that they are caught).
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

U = 2.0 ** -53


def exact_entry(A, B, C, alpha, beta, i, j):
    s = sum((Fraction(float(A[i, p])) * Fraction(float(B[p, j])) for p in range(A.shape[1])), Fraction(0))
    r = Fraction(float(alpha)) * s
    if beta != 0.0:
        r += Fraction(float(beta)) * Fraction(float(C[i, j]))
    return r


def check_against_fraction(A, B, C, alpha, beta, out, slack=4.0):
    """|out - exact| <= u|exact| + slack*(k+2)^2 u^2 (|alpha||A||B| + |beta||C|)."""
    m, k = A.shape
    n = B.shape[1]
    absab = np.abs(A) @ np.abs(B)
    for i in range(m):
        for j in range(n):
            ex = exact_entry(A, B, C, alpha, beta, i, j)
            scale = abs(alpha) * absab[i, j] + (abs(beta) * abs(C[i, j]) if beta != 0.0 else 0.0)
            bound = U * abs(float(ex)) + slack * (k + 2) ** 2 * U * U * scale
            err = abs(Fraction(float(out[i, j])) - ex)
            assert float(err) <= bound, (i, j, float(out[i, j]), float(ex), float(err), bound)


def test_integer_inputs_bit_exact():
    # Integer-valued inputs: every partial sum is an exact integer, so the
    # result must equal exact integer matrix arithmetic.
    m, n, k = 37, 29, 53
    A, B, C = workloads.gemm_operands(m, n, k, kind="int")
    Ai, Bi, Ci = A.astype(np.int64), B.astype(np.int64), C.astype(np.int64)
    np.testing.assert_array_equal(oracle.gemm(A, B), (Ai @ Bi).astype(np.float64))
    np.testing.assert_array_equal(oracle.gemm(A, B, C, alpha=2.0, beta=-3.0),
                                  (2 * (Ai @ Bi) - 3 * Ci).astype(np.float64))
    np.testing.assert_array_equal(oracle.gemm(A, B, C, alpha=1.0, beta=1.0),
                                  (Ai @ Bi + Ci).astype(np.float64))


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 7), (8, 8, 8), (6, 2, 8)])
@pytest.mark.parametrize("ab", [(1.0, 0.0), (2.5, -0.75), (-1.0, 1.0)])
def test_fraction_brute_force_uniform(shape, ab):
    m, n, k = shape
    alpha, beta = ab
    A = workloads.uniform((m, k), 11)
    B = workloads.uniform((k, n), 12)
    C = workloads.uniform((m, n), 13)
    check_against_fraction(A, B, C, alpha, beta, oracle.gemm(A, B, C, alpha, beta))


@pytest.mark.parametrize("seed", range(6))
def test_fraction_brute_force_wide_range(seed):
    # Magnitudes over 16 decades with both signs: plain summation loses
    # digits to cancellation; the compensated sum must still meet the bound.
    m, n, k = 4, 5, 8
    A = workloads.signed_log_uniform((m, k), 100 + seed)
    B = workloads.signed_log_uniform((k, n), 200 + seed)
    C = workloads.uniform((m, n), 300 + seed)
    check_against_fraction(A, B, C, 1.0, 0.0, oracle.gemm(A, B))
    check_against_fraction(A, B, C, -0.5, 2.0, oracle.gemm(A, B, C, -0.5, 2.0))


def test_ill_conditioned_dot_products_exact():
    # Sums whose exact value is tiny next to the terms: naive left-to-right
    # summation returns 0 (or 2), the compensated sum the exact value.
    A = np.array([[1e16, 1.0, -1e16, 1.0]])
    B = np.array([[1.0], [1.0], [1.0], [1.0]])
    assert oracle.gemm(A, B)[0, 0] == 2.0
    # products whose rounding errors carry the answer
    a = 1.0 + 2.0 ** -30
    A = np.array([[a, -1.0]])
    B = np.array([[a], [1.0 + 2.0 ** -29]])
    # exact: a^2 - (1 + 2^-29) = 2^-60
    assert oracle.gemm(A, B)[0, 0] == 2.0 ** -60


def test_identity_returns_b_bitwise():
    k, n = 40, 33
    B = workloads.uniform((k, n), 5)
    np.testing.assert_array_equal(oracle.gemm(np.eye(k), B), B)
    np.testing.assert_array_equal(oracle.gemm(B.T.copy(), np.eye(k)), B.T)


def test_rank1_is_correctly_rounded_product():
    # k = 1: each entry is the single product a_i b_j rounded once.
    A = workloads.uniform((17, 1), 6)
    B = workloads.uniform((1, 19), 7)
    np.testing.assert_array_equal(oracle.gemm(A, B), A * B)


def test_permutation_matrices_permute_exactly():
    rng = np.random.Generator(np.random.PCG64(9))
    p = rng.permutation(23)
    P = np.eye(23)[p]
    X = workloads.uniform((23, 23), 8)
    np.testing.assert_array_equal(oracle.gemm(P, X), X[p])
    np.testing.assert_array_equal(oracle.gemm(X, P.T.copy()), X[:, p])


def test_transpose_symmetry_bitwise():
    # (A B)^T = B^T A^T entry by entry with the same summation order.
    A = workloads.uniform((21, 34), 1)
    B = workloads.uniform((34, 15), 2)
    np.testing.assert_array_equal(oracle.gemm(B.T.copy(), A.T.copy()), oracle.gemm(A, B).T)


def test_k_zero_and_beta_conventions():
    C = workloads.uniform((4, 6), 3)
    A = np.zeros((4, 0))
    B = np.zeros((0, 6))
    np.testing.assert_array_equal(oracle.gemm(A, B, C, alpha=2.0, beta=0.5), 0.5 * C)
    # beta == 0: C is not read, NaNs do not propagate
    Cn = np.full((3, 3), np.nan)
    A = workloads.uniform((3, 4), 4)
    B = workloads.uniform((4, 3), 5)
    np.testing.assert_array_equal(oracle.gemm(A, B, Cn, beta=0.0), oracle.gemm(A, B))


def test_entries_match_full_product():
    A, B, C = workloads.gemm_operands(64, 48, 80)
    full = oracle.gemm(A, B, C, alpha=1.5, beta=-2.0)
    rows = np.array([0, 63, 17, 5, 40])
    cols = np.array([0, 47, 3, 46, 20])
    got = oracle.gemm_entries(A, B, rows, cols, C, alpha=1.5, beta=-2.0)
    np.testing.assert_array_equal(got, full[rows, cols])


def test_within_error_bound_of_numpy():
    # numpy's BLAS result and the oracle both lie within the forward error
    # bound of the exact product, so they differ by at most twice that.
    A, B, C = workloads.gemm_operands(96, 80, 112)
    ref = oracle.gemm(A, B, C, 1.0, 1.0)
    tol = oracle.error_bound(A, B, C, 1.0, 1.0)
    assert np.all(np.abs(ref - (A @ B + C)) <= 2 * tol)
