"""CPU emulation of the split-precision FP64 product (test infrastructure only).

The paper does not contain this method; it is the Ozaki-style error-free
splitting of Ozaki, Ogita, Oishi & Rump (Numer. Algorithms 59, 2012), in the
reading used by the GPU library:

  s1  exponent scan: e_i with max_p |A_ip| < 2**e_i (frexp exponent of the row
      maximum; 0 for a zero row), f_j likewise for the columns of B.
  s2  error-free slicing: with a' = A_ip * 2**-e_i, d_0 = R(a' * 2**w_0),
      r_1 = a' - d_0 * 2**-w_0, d_s = R(r_s * 2**w_s),
      r_{s+1} = r_s - d_s * 2**-w_s, where w_s = b0 + s*b.  Every d_s is an
      integer exact in the slice type:
        BF16 (R = round to nearest, b0 = 8, b = 9): |d_0| <= 256 and
          |d_s| <= 2**(b-1) = 256 (integers up to 256 are exact);
        FP8 E4M3 (R = round to nearest, b0 = 4, b = 5): |d| <= 16;
        INT8 (R = truncation toward zero, b0 = b = 7): |d| <= 127, because
          each residual is below one unit of the previous slice.
  s3  slice products on the pairs s + t <= S - 1, grouped by diagonal
      d = s + t: Q_d = sum_s D^A_s D^B_{d-s}.  All terms are integers and every
      partial sum stays below 2**53, so Q_d is exact in any summation order
      (on the GPU: BF16 products in exact FP32 sums of at most 256 terms
      added exactly in FP64; INT8 products in INT32, exact while
      (d+1) k 127**2 < 2**31).
  s4  recombination, smallest diagonal first:
      V = sum_{d = S-1 .. 0} Q_d * 2**-(2 b0 + d b)  (FP64, in that order),
      T_ij = V_ij * 2**(e_i + f_j),  C = fl(fl(alpha T) + fl(beta C)).

Because s1-s3 are exact and s4 fixes its order, the GPU result must equal
this emulation bit for bit.  Parity with the mathematical product is pinned in
tests/test_split_oracle.py (integer inputs, the slicing residual bound, and an
error bound against the compensated FP64 oracle).
"""
import numpy as np

SLICE_BITS = {"bf16": (8, 9), "fp8": (4, 5), "int8": (7, 7)}
ROUNDING = {"bf16": np.rint, "fp8": np.rint, "int8": np.trunc}


def exponents(X, axis):
    """e with max |X| along `axis` < 2**e (frexp exponent); 0 where the max is 0."""
    mx = np.max(np.abs(X), axis=axis) if X.shape[axis] > 0 else np.zeros(X.shape[1 - axis])
    _, e = np.frexp(mx)
    return e.astype(np.int64)


def slices(X, e, S, kind, axis):
    """Integer slices D_0..D_{S-1} (as float64) of X scaled by 2**-e along `axis`.

    axis=1: e has one entry per row of X (the A side); axis=0: one per column
    (the B side).
    """
    b0, b = SLICE_BITS[kind]
    rnd = ROUNDING[kind]
    ee = e[:, None] if axis == 1 else e[None, :]
    r = np.ldexp(X, -ee)
    out = []
    for s in range(S):
        w = b0 + s * b
        d = rnd(np.ldexp(r, w))
        out.append(d)
        r = r - np.ldexp(d, -w)
    return out


def diagonal_products(DA, DB):
    """Q_d = sum_{s+t=d} D^A_s @ D^B_t for d = 0..S-1 (exact integer matrices)."""
    S = len(DA)
    Q = []
    for d in range(S):
        acc = None
        for s in range(d + 1):
            p = DA[s] @ DB[d - s]
            acc = p if acc is None else acc + p
        Q.append(acc)
    return Q


def recombine(Q, e, f, kind, C=None, alpha=1.0, beta=0.0):
    b0, b = SLICE_BITS[kind]
    S = len(Q)
    V = None
    for d in range(S - 1, -1, -1):
        term = np.ldexp(Q[d], -(2 * b0 + d * b))
        V = term if V is None else V + term
    T = np.ldexp(V, e[:, None] + f[None, :])
    out = alpha * T
    if C is not None and beta != 0.0:
        out = out + beta * C
    return out


def split_gemm(A, B, S, kind="bf16", C=None, alpha=1.0, beta=0.0):
    """alpha * A @ B + beta * C by S-slice splitting, exactly as the GPU orders it."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    e = exponents(A, 1)
    f = exponents(B, 0)
    DA = slices(A, e, S, kind, 1)
    DB = slices(B, f, S, kind, 0)
    return recombine(diagonal_products(DA, DB), e, f, kind, C, alpha, beta)


def split_gemm_entries(A, B, rows, cols, S, kind="bf16", C=None, alpha=1.0, beta=0.0):
    """Selected entries of split_gemm, each computed from its own row and column."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    b0, b = SLICE_BITS[kind]
    e = exponents(A, 1)
    f = exponents(B, 0)
    DA = slices(A[rows], e[rows], S, kind, 1)          # len(rows) x k each
    DB = slices(B[:, cols], f[cols], S, kind, 0)       # k x len(cols) each
    V = None
    for d in range(S - 1, -1, -1):
        q = None
        for s in range(d + 1):
            p = np.einsum("tk,kt->t", DA[s], DB[d - s])
            q = p if q is None else q + p
        term = np.ldexp(q, -(2 * b0 + d * b))
        V = term if V is None else V + term
    T = np.ldexp(V, e[rows] + f[cols])
    out = alpha * T
    if C is not None and beta != 0.0:
        out = out + beta * np.asarray(C)[rows, cols]
    return out
