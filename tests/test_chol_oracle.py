"""Pins of the Cholesky definition (oracle/chol.py) against facts that do not
come from it."""
import numpy as np
import pytest

import oracle
from oracle import chol

U53 = 2.0 ** -53


def test_exact_integer_factor():
    # U upper triangular with ones on the diagonal and small integers above:
    # A = U^T U is an integer matrix and every step is exact
    rng = np.random.Generator(np.random.PCG64(1))
    n = 40
    U = np.triu(rng.integers(-2, 3, (n, n)).astype(np.float64), 1) + np.eye(n)
    A = (U.T.astype(np.int64) @ U.astype(np.int64)).astype(np.float64)
    got, info = chol.potrf_upper(A)
    assert info == 0
    np.testing.assert_array_equal(got, U)


def test_closed_forms():
    d = np.array([4.0, 9.0, 2.25, 1e-6])
    got, info = chol.potrf_upper(np.diag(d))
    assert info == 0
    np.testing.assert_array_equal(got, np.diag(np.sqrt(d)))
    got, info = chol.potrf_upper(np.array([[6.25]]))
    assert info == 0 and got[0, 0] == 2.5


@pytest.mark.parametrize("n", [5, 64, 150])
def test_residual_bound_and_library_factor(n):
    rng = np.random.Generator(np.random.PCG64(n))
    M = rng.uniform(-1, 1, (n, n))
    A = M @ M.T + n * np.eye(n)
    A_upper_only = np.triu(A) + np.tril(np.full((n, n), np.nan), -1)   # the lower triangle is not read
    U, info = chol.potrf_upper(A_upper_only)
    assert info == 0 and np.all(np.tril(U, -1) == 0)
    R = oracle.gemm(U.T.copy(), U, A, 1.0, -1.0)
    assert np.all(np.abs(R) <= 2 * (n + 2) * U53 * (np.abs(U.T) @ np.abs(U) + np.abs(A)))
    ref = np.linalg.cholesky(A).T
    assert np.max(np.abs(U - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_indefinite_reports_the_pivot():
    A = np.array([[4.0, 2.0, 0.0], [2.0, 1.0, 3.0], [0.0, 3.0, 5.0]])   # second pivot 1 - 1 = 0
    _, info = chol.potrf_upper(A)
    assert info == 2
    _, info = chol.potrf_upper(-np.eye(3))
    assert info == 1
