"""Plant plausible mistakes in a copy of the C oracle and check the pins catch them.

Each mutant is compiled from a textual edit of oracle/gemm_dot2.c into a
temporary library (CPU only).  The battery below reuses the independent truths
of test_oracle.py (exact rationals, integer arithmetic, closed forms); every
mutant must fail at least one check.  All shapes are square so that a
transposed-index mutant still reads in bounds.
"""
import ctypes
import os
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "gemm_dot2.c")
U = 2.0 ** -53

MUTANTS = {
    "drop_product_error": ("s = s + (e + r);", "s = s + e;"),
    "drop_sum_error": ("s = s + (e + r);", "s = s + r;"),
    "wrong_sign": ("s = s + (e + r);", "s = s - (e + r);"),
    "first_error_lost": ("s = r;", "s = 0.0;"),
    "transposed_a": ("A[i * lda + q]", "A[q * lda + i]"),
    "transposed_b": ("B[q * ldb + j]", "B[j * ldb + q]"),
    "alpha_tail_dropped": ("+ tail_a)", ")"),
    "beta_sign": ("two_product(beta, c, &h2, &r2);", "two_product(beta, -c, &h2, &r2);"),
    "skip_last_term": ("for (int64_t q = 0; q < k; ++q)", "for (int64_t q = 0; q + 1 < k; ++q)"),
}


def _build(src_text, tmp):
    c = os.path.join(tmp, "m.c")
    so = os.path.join(tmp, "m.so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           "-o", so, c, "-lm"])
    lib = ctypes.CDLL(so)
    i64, dbl, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.oracle_dgemm.argtypes = [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64]
    return lib


def _gemm(lib, A, B, C, alpha, beta):
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B)
    out = np.array(C, copy=True)
    m, k = A.shape
    n = B.shape[1]
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    lib.oracle_dgemm(m, n, k, alpha, p(A), k, p(B), n, beta, p(out), n)
    return out


def _battery(lib):
    """Return the list of failed check names."""
    failed = []
    n = 6
    # exact rationals on wide-range data, alpha/beta general
    for seed in range(4):
        A = workloads.signed_log_uniform((n, n), 400 + seed)
        B = workloads.signed_log_uniform((n, n), 500 + seed)
        C = workloads.uniform((n, n), 600 + seed)
        for alpha, beta in ((1.0, 0.0), (1.5, -2.0)):
            out = _gemm(lib, A, B, C, alpha, beta)
            absab = np.abs(A) @ np.abs(B)
            for i in range(n):
                for j in range(n):
                    ex = Fraction(alpha) * sum((Fraction(A[i, p]) * Fraction(B[p, j]) for p in range(n)),
                                               Fraction(0))
                    if beta != 0.0:
                        ex += Fraction(beta) * Fraction(C[i, j])
                    bound = U * abs(float(ex)) + 4 * (n + 2) ** 2 * U * U * (
                        abs(alpha) * absab[i, j] + abs(beta) * abs(C[i, j]))
                    if float(abs(Fraction(out[i, j]) - ex)) > bound:
                        failed.append("fraction")
                        break
                else:
                    continue
                break
    # integer arithmetic
    A, B, C = workloads.gemm_operands(n, n, n, kind="int")
    want = A.astype(np.int64) @ B.astype(np.int64)
    if not np.array_equal(_gemm(lib, A, B, C, 1.0, 0.0), want.astype(np.float64)):
        failed.append("integer")
    if not np.array_equal(_gemm(lib, A, B, C, 1.0, 1.0), (want + C.astype(np.int64)).astype(np.float64)):
        failed.append("integer_beta")
    return failed


def test_unmutated_oracle_passes_battery():
    with open(SRC) as f:
        text = f.read()
    with tempfile.TemporaryDirectory() as tmp:
        assert _battery(_build(text, tmp)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    with open(SRC) as f:
        text = f.read()
    assert old in text, "mutation site not found; update the mutant table"
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build(text.replace(old, new, 1), tmp)
        assert _battery(lib), f"mutant {name} passed every pin"
