"""CPU definitions of the triangular level-3 operations (test infrastructure only).

The paper names the other level-3 BLAS as the family's next target (Sec. 6);
these are their plain definitions, independent of the GPU library:

  op_tri(A, uplo, trans, diag)   the m x m matrix op(T): T is the triangle of
                                  A named by uplo ('L' keeps i >= j, 'U' keeps
                                  i <= j), with ones on the diagonal when
                                  diag == 'U' (the diagonal of A is then not
                                  read); op(T) = T or T^T.
  trmm(A, B, ...)                 C = alpha op(T) B, through the compensated
                                  FP64 product of the C oracle.
  trsm(A, B, ...)                 X with op(T) X = alpha B, by plain
                                  substitution one row at a time: forward when
                                  op(T) is lower triangular, backward when it
                                  is upper; x_i = (alpha b_i - sum_j t_ij x_j) / t_ii
                                  with the sum over the already solved rows
                                  taken by a library dot product (no division
                                  for a unit diagonal).

Pins (tests/test_tri_oracle.py): integer systems solved exactly, identity and
diagonal closed forms, op(T) X reproducing alpha B within the backward error
bound of substitution, agreement with an independent library solver, and the
masking of op_tri on hand-written matrices.
"""
import numpy as np

from . import gemm as _gemm


def op_tri(A, uplo="L", trans=False, diag="N"):
    A = np.asarray(A, dtype=np.float64)
    T = np.tril(A) if uplo == "L" else np.triu(A)
    if diag == "U":
        np.fill_diagonal(T, 1.0)
    return np.ascontiguousarray(T.T if trans else T)


def trmm(A, B, uplo="L", trans=False, diag="N", alpha=1.0):
    """alpha op(T) B with one rounding per entry."""
    return _gemm(op_tri(A, uplo, trans, diag), np.asarray(B, dtype=np.float64), alpha=alpha)


def trsm(A, B, uplo="L", trans=False, diag="N", alpha=1.0):
    """X with op(T) X = alpha B by substitution."""
    T = op_tri(A, uplo, trans, diag)
    Bs = alpha * np.asarray(B, dtype=np.float64)
    m = T.shape[0]
    X = np.zeros_like(Bs)
    lower = (uplo == "L") != bool(trans)
    order = range(m) if lower else range(m - 1, -1, -1)
    for i in order:
        js = slice(0, i) if lower else slice(i + 1, m)
        acc = Bs[i] - T[i, js] @ X[js]
        X[i] = acc if diag == "U" else acc / T[i, i]
    return X
