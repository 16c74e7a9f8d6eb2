"""Pins of the modular split product's definition (oracle/crt_emul.py) against
facts that do not come from it: moduli lists derived by hand, the defining
inequality of the bit count, exact integer products, and the error bound of
rounding the operands to t bits against the compensated FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import crt_emul as ce


def test_moduli_lists_derived_by_hand():
    # 254, 252, ... are even; 249 = 3*83 and 245 = 5*7^2 share a factor with
    # 255 = 3*5*17; 221 = 13*17; 209 = 11*19; 203 = 7*29 (after 217 = 7*31).
    assert ce.moduli(1) == [256]
    assert ce.moduli(4) == [256, 255, 253, 251]
    assert ce.moduli(6) == [256, 255, 253, 251, 247, 241]
    assert ce.moduli(16) == [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197, 193]
    for N in range(1, 17):
        p = ce.moduli(N)
        assert all(math.gcd(a, b) == 1 for i, a in enumerate(p) for b in p[i + 1:])


@pytest.mark.parametrize("N", [2, 5, 8, 12, 14, 15, 16])
@pytest.mark.parametrize("k", [1, 3, 200, 8192, 131072])
def test_bits_is_the_largest_t_with_2k4t_below_M(N, k):
    M = math.prod(ce.moduli(N))
    t = ce.bits(k, N)
    if t is None:   # infeasible: not even t = 1 fits
        assert 2 * k * 4 >= M
        return
    assert 1 <= t <= 60
    assert 2 * k * 4 ** t < M
    assert t == 60 or 2 * k * 4 ** (t + 1) >= M


def test_bits_hand_values():
    # M = 256 * 255 = 65280: 2 * 4^7 = 32768 < M <= 2 * 4^8
    assert ce.bits(1, 2) == 7
    # one modulus: 2 k 4^t < 256 needs 4^t < 128 / k
    assert ce.bits(1, 1) == 3
    assert ce.bits(31, 1) == 1
    assert ce.bits(32, 1) is None
    # 2 * 8192 * 4 = 65536 > 65280
    assert ce.bits(8192, 2) is None


def test_integer_inputs_are_exact():
    # entries in [-8, 8] need 4 bits below 2^e = 16; N = 6 gives t = 19 at k = 300
    m, n, k = 37, 29, 300
    A, B, C = workloads.gemm_operands(m, n, k, kind="int")
    assert ce.bits(k, 6) == 19
    want = (A.astype(np.int64) @ B.astype(np.int64) + C.astype(np.int64)).astype(np.float64)
    np.testing.assert_array_equal(ce.crt_gemm(A, B, 6, C, 1.0, 1.0), want)
    rows, cols = np.array([0, 5, 36]), np.array([28, 0, 13])
    np.testing.assert_array_equal(ce.crt_gemm_entries(A, B, rows, cols, 6, C, 1.0, 1.0), want[rows, cols])


def test_round_half_to_even_on_operands():
    # row maximum 1 (e = 1), t = 3: 0.3125 * 2^2 = 1.25 -> 1, 0.375 * 4 = 1.5 -> 2, 0.625 * 4 = 2.5 -> 2
    A = np.array([[1.0, 0.3125, 0.375, 0.625]])
    B = np.ones((4, 1))
    Ai, _, e, _ = ce.integer_operands(A, B, 3)
    assert e[0] == 1
    np.testing.assert_array_equal(Ai[0], [4.0, 1.0, 2.0, 2.0])


@pytest.mark.parametrize("N", [4, 8, 12, 16])
def test_error_bound_against_compensated_oracle(N):
    # A = 2^(e-t) A' + dA with |dA_ip| <= 2^(e_i - t - 1) (likewise B), so
    # |T - AB| <= 2^(e_i-t-1) sum|b| + 2^(f_j-t-1) sum|a| + k 2^(e_i+f_j-2t-2) + u |T|.
    m, n, k = 48, 40, 200
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    t = ce.bits(k, N)
    got = ce.crt_gemm(A, B, N)
    want = oracle.gemm(A, B)
    e = oracle.split_emul.exponents(A, 1)
    f = oracle.split_emul.exponents(B, 0)
    sa = np.abs(A).sum(axis=1)
    sb = np.abs(B).sum(axis=0)
    bound = (np.ldexp(sb[None, :], e[:, None] - t - 1) + np.ldexp(sa[:, None], f[None, :] - t - 1)
             + k * np.ldexp(1.0, e[:, None] + f[None, :] - 2 * t - 2)) * 1.001 + 2.0 ** -52 * np.abs(want)
    assert np.all(np.abs(got - want) <= bound)
    if N == 16:   # t = 58 at k = 200
        assert np.max(np.abs(got - want) / (np.abs(A) @ np.abs(B))) < 1e-13


def test_zero_rows_columns_and_beta_zero():
    m, n, k = 12, 9, 30
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    A[3] = 0.0
    B[:, 4] = 0.0
    got = ce.crt_gemm(A, B, 10, np.full((m, n), np.nan), 2.0, 0.0)
    assert (got[3] == 0).all() and (got[:, 4] == 0).all()
    assert np.isfinite(got).all()


# Plausible mistakes planted in a copy of the definition (CPU only): each must
# fail one of the pins above.
CRT_MUTANTS = {
    "truncate_operands": ("Ai = np.rint(np.ldexp(A", "Ai = np.trunc(np.ldexp(A"),
    "operand_shift_sign": ("np.ldexp(A, (t - e)[:, None])", "np.ldexp(A, (e - t)[:, None])"),
    "b_exponents_reversed": ("np.ldexp(B, (t - f)[None, :])", "np.ldexp(B, (t - f[::-1])[None, :])"),
    "result_shift_off_by_one": ("int(e[i] + f[j] - 2 * t))\n    out = alpha", "int(e[i] + f[j] - 2 * t + 1))\n    out = alpha"),
    "bits_one_too_many": ("            t = cand\n", "            t = cand + 1\n"),
    "moduli_upward": ("range(256, 1, -1)", "range(2, 257)"),
    "beta_dropped": ("out = out + beta * np.asarray(C)", "out = out + 0.0 * np.asarray(C)"),
}


def _mutant_module(name):
    import types

    src_path = ce.__file__
    with open(src_path) as fh:
        text = fh.read()
    old, new = CRT_MUTANTS[name]
    assert text.count(old) >= 1, name
    text = text.replace(old, new, 1).replace("from .split_emul import exponents",
                                            "from oracle.split_emul import exponents")
    mod = types.ModuleType("crt_mutant_" + name)
    exec(compile(text, "crt_mutant_" + name, "exec"), mod.__dict__)
    return mod


def _battery(mod):
    """True when every pin holds for the module."""
    checks = []
    checks.append(mod.moduli(6) == [256, 255, 253, 251, 247, 241])
    checks.append(mod.bits(1, 2) == 7 and mod.bits(31, 1) == 1)
    m, n, k = 37, 29, 300
    A, B, C = workloads.gemm_operands(m, n, k, kind="int")
    want = (A.astype(np.int64) @ B.astype(np.int64) + C.astype(np.int64)).astype(np.float64)
    checks.append(np.array_equal(mod.crt_gemm(A, B, 6, C, 1.0, 1.0), want))
    Ai, _, _, _ = mod.integer_operands(np.array([[1.0, 0.3125, 0.375, 0.625]]), np.ones((4, 1)), 3)
    checks.append(np.array_equal(Ai[0], [4.0, 1.0, 2.0, 2.0]))
    m, n, k = 48, 40, 200
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    t = mod.bits(k, 8)
    got = mod.crt_gemm(A, B, 8)
    ref = oracle.gemm(A, B)
    e = oracle.split_emul.exponents(A, 1)
    f = oracle.split_emul.exponents(B, 0)
    bound = (np.ldexp(np.abs(B).sum(axis=0)[None, :], e[:, None] - t - 1)
             + np.ldexp(np.abs(A).sum(axis=1)[:, None], f[None, :] - t - 1)
             + k * np.ldexp(1.0, e[:, None] + f[None, :] - 2 * t - 2)) * 1.001 + 2.0 ** -52 * np.abs(ref)
    checks.append(bool(np.all(np.abs(got - ref) <= bound)))
    return all(checks)


def test_unmutated_definition_passes_battery():
    assert _battery(ce)


@pytest.mark.parametrize("name", sorted(CRT_MUTANTS))
def test_crt_mutant_is_caught(name):
    assert not _battery(_mutant_module(name))
