"""CPU definition of the modular (CRT) split product (test infrastructure only).

The paper does not contain this method.  It is the integer modular scheme of
Ozaki, Uchino & Imamura ("Ozaki scheme II", 2025), in the reading used by the
GPU library.  What the method computes has a plain definition, and this module
is that definition written out:

  1  moduli: the N largest integers in [2, 256] that are pairwise coprime,
     taken greedily from 256 downward; M = their product.
  2  bits: t = the largest integer <= 60 with 2 k 4^t < M (at least 1, else
     the product is infeasible).  Then every |X_ij| below is < M / 2.
  3  exponents e_i of the rows of A and f_j of the columns of B as in the
     slice emulation (|A_ip| < 2^e_i; 0 for a zero row).
  4  integer operands: A'_ip = rint(A_ip 2^(t - e_i)), B'_pj = rint(B_pj 2^(t - f_j))
     (round half to even), so |A'|, |B'| <= 2^t.
  5  X = A' B' exactly (Python integers), T_ij = RN(X_ij) 2^(e_i + f_j - 2t),
     C = fl(fl(alpha T) + fl(beta C)); beta = 0 does not read C.

The GPU computes X by residues: X mod p_l = (A' mod p_l)(B' mod p_l) mod p_l
on INT8 MFMA (residues in [-128, 127], exact INT32 sums while k <= 2^17) and
the Chinese remainder theorem in 128-bit integers, then rounds X once.  Since
X is determined exactly, the GPU must equal this module bit for bit.  The
residues and the reconstruction are not part of this definition.

Pins (tests/test_crt_oracle.py): the hand-derived moduli lists, the choice of
t against its defining inequality, integer inputs that need at most t bits
(exact integer product), and the rounding error bound against the
compensated FP64 oracle.
"""
import math

import numpy as np

from .split_emul import exponents

MAX_MODULI = 16
MAX_BITS = 60


def moduli(N):
    """The N largest pairwise coprime integers in [2, 256], greedily from 256 down."""
    out = []
    for p in range(256, 1, -1):
        if len(out) == N:
            break
        if all(math.gcd(p, q) == 1 for q in out):
            out.append(p)
    return out


def bits(k, N):
    """t: the largest integer <= 60 with 2 k 4^t < M; None if not even t = 1 fits."""
    M = math.prod(moduli(N))
    kk = max(int(k), 1)
    t = None
    for cand in range(1, MAX_BITS + 1):
        if 2 * kk * 4 ** cand < M:
            t = cand
    return t


def integer_operands(A, B, t):
    """A', B' and the exponents (step 4)."""
    e = exponents(A, 1)
    f = exponents(B, 0)
    Ai = np.rint(np.ldexp(A, (t - e)[:, None]))
    Bi = np.rint(np.ldexp(B, (t - f)[None, :]))
    return Ai, Bi, e, f


def _as_int_objects(X):
    return np.array([[int(v) for v in row] for row in X], dtype=object).reshape(X.shape)


def crt_gemm(A, B, N, C=None, alpha=1.0, beta=0.0):
    """alpha * T + beta * C with T the rounded exact product of the t-bit integer operands."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    t = bits(k, N)
    if t is None:
        raise ValueError("infeasible: too few moduli for this k")
    Ai, Bi, e, f = integer_operands(A, B, t)
    X = _as_int_objects(Ai).dot(_as_int_objects(Bi)) if k > 0 else np.zeros((m, n), dtype=object)
    T = np.empty((m, n))
    for i in range(m):
        for j in range(n):
            T[i, j] = math.ldexp(float(int(X[i, j])), int(e[i] + f[j] - 2 * t))
    out = alpha * T
    if C is not None and beta != 0.0:
        out = out + beta * np.asarray(C)
    return out


def crt_gemm_entries(A, B, rows, cols, N, C=None, alpha=1.0, beta=0.0):
    """Selected entries of crt_gemm, each from its own row of A and column of B
    (the exponents still come from the whole row / column)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    k = A.shape[1]
    t = bits(k, N)
    if t is None:
        raise ValueError("infeasible: too few moduli for this k")
    e = exponents(A, 1)
    f = exponents(B, 0)
    out = np.empty(len(rows))
    for q, (i, j) in enumerate(zip(rows, cols)):
        a = np.rint(np.ldexp(A[i], int(t - e[i])))
        b = np.rint(np.ldexp(B[:, j], int(t - f[j])))
        x = sum(int(u) * int(v) for u, v in zip(a, b))
        T = math.ldexp(float(x), int(e[i] + f[j] - 2 * t))
        o = alpha * T
        if C is not None and beta != 0.0:
            o = o + beta * float(np.asarray(C)[i, j])
        out[q] = o
    return out
