"""Pins of the split-precision emulation (oracle/split_emul.py) against facts
that do not come from the emulation: exact integer arithmetic, the residual
bound of round-to-nearest slicing, representability of every slice in the
target type, and an error bound against the compensated FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import split_emul as se


@pytest.mark.parametrize("kind", ["bf16", "fp8", "int8"])
def test_slices_are_small_integers_exact_in_the_slice_type(kind):
    b0, b = se.SLICE_BITS[kind]
    X = workloads.signed_log_uniform((40, 70), 31)
    e = se.exponents(X, 1)
    D = se.slices(X, e, 6, kind, 1)
    ttype = {"bf16": torch.bfloat16, "fp8": torch.float8_e4m3fn, "int8": torch.int8}[kind]
    for s, d in enumerate(D):
        assert np.array_equal(d, np.rint(d))
        if kind == "int8":
            lim = 127
        else:
            lim = 2 ** b0 if s == 0 else 2 ** (b - 1)
        assert np.abs(d).max() <= lim
        back = torch.from_numpy(d).to(ttype).to(torch.float64).numpy()
        np.testing.assert_array_equal(back, d)


@pytest.mark.parametrize("kind", ["bf16", "fp8", "int8"])
@pytest.mark.parametrize("S", [1, 2, 4, 7])
def test_slicing_residual_bound(kind, S):
    # After S round-to-nearest slices the residual is at most half a unit of
    # the last slice's grid, |x - sum_s d_s 2^(e - w_s)| <= 2^(e - w_{S-1} - 1);
    # after S truncated slices it is below one unit, < 2^(e - w_{S-1}).
    b0, b = se.SLICE_BITS[kind]
    X = workloads.signed_log_uniform((30, 50), 32)
    e = se.exponents(X, 1)
    D = se.slices(X, e, S, kind, 1)
    recon = sum(np.ldexp(D[s], e[:, None] - (b0 + s * b)) for s in range(S))
    if kind == "int8":
        bound = np.ldexp(np.ones_like(X), e[:, None] - (b0 + (S - 1) * b))
        assert np.all(np.abs(X - recon) < bound)
    else:
        bound = np.ldexp(np.ones_like(X), e[:, None] - (b0 + (S - 1) * b) - 1)
        assert np.all(np.abs(X - recon) <= bound)


def test_exponent_scan():
    X = np.array([[0.75, -0.1], [1.0, 0.0], [0.0, 0.0], [-3.0, 2.5]])
    np.testing.assert_array_equal(se.exponents(X, 1), [0, 1, 0, 2])  # 0.75 < 2^0, 1 < 2^1, 3 < 2^2
    np.testing.assert_array_equal(se.exponents(X, 0), [2, 2])


def test_full_slicing_reconstructs_doubles_exactly():
    # Entries within one binade of their row maximum need at most 53 bits
    # below 2^e, which 7 BF16 slices (8 + 6*9 = 62 bits) cover.
    rng = np.random.Generator(np.random.PCG64(7))
    X = rng.uniform(0.5, 1.0, (20, 30)) * np.where(rng.integers(0, 2, (20, 30)) == 0, -1, 1)
    e = se.exponents(X, 1)
    D = se.slices(X, e, 7, "bf16", 1)
    recon = np.zeros_like(X)
    for s in range(6, -1, -1):
        recon = recon + np.ldexp(D[s], e[:, None] - (8 + 9 * s))
    np.testing.assert_array_equal(recon, X)


@pytest.mark.parametrize("kind", ["bf16", "fp8", "int8"])
def test_small_integers_are_reproduced_exactly(kind):
    # Integers with |x| <= 8 fit in the first slice of either type, so the
    # split product is the exact integer product for every S >= 1.
    m, n, k = 33, 29, 47
    A, B, C = workloads.gemm_operands(m, n, k, kind="int")
    want = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    for S in (1, 3):
        np.testing.assert_array_equal(se.split_gemm(A, B, S, kind), want)
    np.testing.assert_array_equal(se.split_gemm(A, B, 2, kind, C, 1.0, 1.0), want + C)


def test_zero_rows_and_columns():
    A, B, C = workloads.gemm_operands(12, 10, 9)
    A[3] = 0.0
    B[:, 4] = 0.0
    out = se.split_gemm(A, B, 6, "bf16", C, 2.0, 0.5)
    np.testing.assert_array_equal(out[3], 0.5 * C[3])
    np.testing.assert_array_equal(out[:, 4], 0.5 * C[:, 4])


def relative_to_absab(got, want, A, B):
    return np.max(np.abs(got - want) / (np.abs(A) @ np.abs(B)))


def split_error_bound(A, B, S, kind, k):
    """Per-entry bound on |split - exact| (derivation in the oracle module doc).

    With tau the slicing residual (2^-(w_{S-1} + 1) rounding to nearest,
    2^-w_{S-1} truncating), every product term 2^(e_i + f_j) a'_ip b'_pj is
    reproduced up to the two residual terms (<= tau each, |a'|, |b'| < 1),
    their product, and the dropped pairs s + t >= S (both s, t >= 1: at most
    (S-1) tau (1 + 2^-b + ...)); the FP64 recombination adds at most
    (S + 2) u |result|.
    """
    b0, b = se.SLICE_BITS[kind]
    tau = 2.0 ** -(b0 + (S - 1) * b + (0 if kind == "int8" else 1))
    e = se.exponents(A, 1)
    f = se.exponents(B, 0)
    scale = np.ldexp(np.ones((A.shape[0], B.shape[1])), e[:, None] + f[None, :])
    u = 2.0 ** -53
    return (S + 2) * 1.01 * tau * k * scale + (S + 2) * u * (np.abs(A) @ np.abs(B))


@pytest.mark.parametrize("kind", ["bf16", "fp8", "int8"])
@pytest.mark.parametrize("S", [2, 4, 6, 7])
def test_split_error_within_per_entry_bound(kind, S):
    m, n, k = 48, 40, 200
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    got = se.split_gemm(A, B, S, kind)
    want = oracle.gemm(A, B)
    bound = split_error_bound(A, B, S, kind, k)
    assert np.all(np.abs(got - want) <= bound)


def test_bf16_seven_slices_meet_1e13_relative():
    # The target reading: max_ij |dC_ij| / (|A||B|)_ij <= 1e-13.
    m, n, k = 64, 48, 256
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    assert relative_to_absab(se.split_gemm(A, B, 7, "bf16"), oracle.gemm(A, B), A, B) <= 1e-13


def test_error_decreases_with_slices():
    m, n, k = 32, 32, 128
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = oracle.gemm(A, B)
    errs = [relative_to_absab(se.split_gemm(A, B, S, "bf16"), want, A, B) for S in (2, 3, 4, 5)]
    assert all(errs[i + 1] < errs[i] / 16 for i in range(3)), errs


def test_entries_match_full_emulation():
    A, B, C = workloads.gemm_operands(40, 36, 90, kind="loguniform")
    full = se.split_gemm(A, B, 5, "bf16", C, 1.5, -0.5)
    rows = np.array([0, 39, 7, 20])
    cols = np.array([0, 35, 11, 3])
    got = se.split_gemm_entries(A, B, rows, cols, 5, "bf16", C, 1.5, -0.5)
    np.testing.assert_array_equal(got, full[rows, cols])
