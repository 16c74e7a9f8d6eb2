"""Pins of the triangular definitions (oracle/tri.py) against facts that do
not come from them: hand-masked matrices, exact integer systems, identity and
diagonal closed forms, the backward error bound of substitution, and an
independent library solver."""
import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import tri

U = 2.0 ** -53


def test_op_tri_masks_by_hand():
    A = np.arange(1.0, 10.0).reshape(3, 3)
    np.testing.assert_array_equal(tri.op_tri(A, "L"), [[1, 0, 0], [4, 5, 0], [7, 8, 9]])
    np.testing.assert_array_equal(tri.op_tri(A, "U", diag="U"), [[1, 2, 3], [0, 1, 6], [0, 0, 1]])
    np.testing.assert_array_equal(tri.op_tri(A, "L", trans=True), [[1, 4, 7], [0, 5, 8], [0, 0, 9]])


def unit_integer_system(m, n, uplo, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.integers(-2, 3, (m, m)).astype(np.float64)
    X = rng.integers(-3, 4, (m, n)).astype(np.float64)
    return A, X


@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("trans", [False, True])
def test_integer_unit_systems_solve_exactly(uplo, trans):
    # op(T) unit triangular with small integers, X integers: B = op(T) X is
    # exact, every step of substitution stays an integer below 2^53
    m, n = 24, 7
    A, X = unit_integer_system(m, n, uplo, 3)
    T = tri.op_tri(A, uplo, trans, "U")
    B = (T.astype(np.int64) @ X.astype(np.int64)).astype(np.float64)
    np.testing.assert_array_equal(tri.trsm(A, B, uplo, trans, "U"), X)
    np.testing.assert_array_equal(tri.trmm(A, X, uplo, trans, "U"), B)


def test_identity_and_diagonal_closed_forms():
    rng = np.random.Generator(np.random.PCG64(4))
    B = rng.uniform(-1, 1, (10, 6))
    I = np.eye(10)
    np.testing.assert_array_equal(tri.trsm(I, B, "L", False, "N", 2.5), 2.5 * B)
    d = rng.uniform(1, 2, 10)
    D = np.diag(d) + np.tril(rng.uniform(-1, 1, (10, 10)), -1) * 0.0
    np.testing.assert_array_equal(tri.trsm(D, B, "L"), B / d[:, None])
    np.testing.assert_array_equal(tri.trsm(D, B, "U", True), B / d[:, None])


@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("diag", ["N", "U"])
def test_substitution_backward_error_and_library_solver(uplo, trans, diag):
    # well-conditioned op(T): off-diagonal U[-1,1] / m, diagonal in [1, 2]
    m, n = 60, 9
    rng = np.random.Generator(np.random.PCG64(5))
    A = rng.uniform(-1, 1, (m, m)) / m
    A[np.diag_indices(m)] = rng.uniform(1, 2, m)
    B = rng.uniform(-1, 1, (m, n))
    X = tri.trsm(A, B, uplo, trans, diag, alpha=0.75)
    T = tri.op_tri(A, uplo, trans, diag)
    R = oracle.gemm(T, X, B, 1.0, -0.75)                  # op(T) X - alpha B, rounded once
    bound = 2 * (m + 2) * U * (np.abs(T) @ np.abs(X) + 0.75 * np.abs(B))
    assert np.all(np.abs(R) <= bound)
    lower = (uplo == "L") != trans
    ref = scipy.linalg.solve_triangular(T, 0.75 * B, lower=lower, unit_diagonal=(diag == "U"))
    assert np.max(np.abs(X - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_a_planted_wrong_order_is_caught():
    # solving in the wrong direction must violate the residual bound
    m, n = 30, 4
    rng = np.random.Generator(np.random.PCG64(6))
    A = rng.uniform(-1, 1, (m, m)) / m
    A[np.diag_indices(m)] = rng.uniform(1, 2, m)
    B = rng.uniform(-1, 1, (m, n))
    X_wrong = tri.trsm(A, B, "U")                          # solves the upper system
    T = tri.op_tri(A, "L")
    R = oracle.gemm(T, X_wrong, B, 1.0, -1.0)
    assert np.max(np.abs(R)) > 1e-3
