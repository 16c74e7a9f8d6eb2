"""CPU definition of the Cholesky factorization (test infrastructure only).

The paper names recursive blocked factorizations on the family as future work
(Sec. 6).  This is the plain definition: for a symmetric positive definite A
(only its upper triangle is read), the upper triangular U with U^T U = A, one
row at a time:
    u_jj = sqrt(a_jj - sum_{k<j} u_kj^2),
    u_ji = (a_ji - sum_{k<j} u_kj u_ki) / u_jj   for i > j,
with the sums taken by a library dot product.  info is 0, or j + 1 for the
first j whose pivot a_jj - sum_k u_kj^2 is not positive (the factorization
stops there, as LAPACK's does).

Pins (tests/test_chol_oracle.py): exact integer factors, diagonal and 1 x 1
closed forms, the residual bound |U^T U - A| <= c n u |U^T| |U|, agreement with
an independent library factorization, and the failing pivot of an indefinite
matrix.
"""
import numpy as np


def potrf_upper(A):
    """(U, info): U upper triangular (zeros below), U^T U = A."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    U = np.zeros_like(A)
    for j in range(n):
        d = A[j, j] - U[:j, j] @ U[:j, j]
        if not d > 0.0:
            return U, j + 1
        U[j, j] = np.sqrt(d)
        if j + 1 < n:
            U[j, j + 1:] = (A[j, j + 1:] - U[:j, j] @ U[:j, j + 1:]) / U[j, j]
    return U, 0
