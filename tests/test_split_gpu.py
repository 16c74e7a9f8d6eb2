"""Parity of the split-precision GPU path with its CPU emulation (bit for bit:
every step but the fixed-order recombination is exact) and with the FP64
oracle (per-entry error bound; 1e-13 of |A||B| at seven slices)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import split_emul as se

pytestmark = pytest.mark.gpu
mm = pytest.importorskip("paper_1904_05717_amd")
DEV = "cuda:0"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def run(A, B, C, alpha, beta, S, member="AUTO", ta=False, tb=False, kind="bf16"):
    Cd = dev(C.copy()) if C is not None else None
    out = mm.gemm_split(dev(A), dev(B), Cd, alpha=alpha, beta=beta, slices=S, member=member, transA=ta, transB=tb,
                        slice_type=kind)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("S", [1, 2, 3, 5, 7, 8])
@pytest.mark.parametrize("kind", ["uniform", "loguniform"])
def test_bit_exact_against_emulation(S, kind):
    m = n = k = 256
    A, B, C = workloads.gemm_operands(m, n, k, kind=kind)
    want = se.split_gemm(A, B, S, "bf16", C, 1.0, 1.0)
    np.testing.assert_array_equal(run(A, B, C, 1.0, 1.0, S), want)


@pytest.mark.parametrize("shape", [(300, 280, 260), (1, 1, 1), (129, 7, 65), (17, 200, 3), (520, 390, 700)])
@pytest.mark.parametrize("member", ["AUTO", "C0"])
def test_ragged_shapes_bit_exact(shape, member):
    m, n, k = shape
    A, B, C = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = se.split_gemm(A, B, 6, "bf16", C, -1.5, 0.25)
    np.testing.assert_array_equal(run(A, B, C, -1.5, 0.25, 6, member), want)


@pytest.mark.parametrize("ta,tb", [(False, True), (True, False), (True, True)])
def test_transposed_operands_bit_exact(ta, tb):
    m, n, k = 200, 150, 170
    A, B, C = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = se.split_gemm(A, B, 5, "bf16", C, 1.0, 1.0)
    got = run(A.T.copy() if ta else A, B.T.copy() if tb else B, C, 1.0, 1.0, 5, ta=ta, tb=tb)
    np.testing.assert_array_equal(got, want)


def test_integers_exact():
    m, n, k = 160, 144, 300
    A, B, C = workloads.gemm_operands(m, n, k, kind="int")
    want = (A.astype(np.int64) @ B.astype(np.int64) + C.astype(np.int64)).astype(np.float64)
    np.testing.assert_array_equal(run(A, B, C, 1.0, 1.0, 1), want)


def test_zero_rows_columns_and_beta_zero_nan():
    m, n, k = 130, 120, 90
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    A[5] = 0.0
    B[:, 7] = 0.0
    Cn = np.full((m, n), np.nan)
    got = run(A, B, Cn, 1.0, 0.0, 4)
    np.testing.assert_array_equal(got, se.split_gemm(A, B, 4, "bf16"))
    assert (got[5] == 0).all() and (got[:, 7] == 0).all()


def test_error_against_fp64_oracle():
    m, n, k = 192, 160, 512
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = oracle.gemm(A, B)
    absab = np.abs(A) @ np.abs(B)
    got7 = run(A, B, None, 1.0, 0.0, 7)
    assert np.max(np.abs(got7 - want) / absab) <= 1e-13
    e = se.exponents(A, 1)
    f = se.exponents(B, 0)
    for S in (3, 6):
        got = run(A, B, None, 1.0, 0.0, S)
        tau = 2.0 ** -(8 + (S - 1) * 9 + 1)
        bound = (S + 2) * 1.01 * tau * k * np.ldexp(1.0, e[:, None] + f[None, :]) + (S + 2) * 2.0 ** -53 * absab
        assert np.all(np.abs(got - want) <= bound), S


def test_argument_errors():
    f = mm._lib.momms_gemm_split
    big = 1 << 20
    assert f(0, 0, 4, 4, 4, 1.0, big, 4, big, 4, 0.0, big, 4, 0, 0, 0, big, 1 << 30, None) == -14
    assert f(0, 0, 4, 4, 4, 1.0, big, 4, big, 4, 0.0, big, 4, 9, 0, 0, big, 1 << 30, None) == -14
    assert f(0, 0, 4, 4, 4, 1.0, big, 4, big, 4, 0.0, big, 4, 3, 7, 0, big, 1 << 30, None) == -15
    assert f(0, 0, 4, 4, 4, 1.0, big, 4, big, 4, 0.0, big, 4, 3, 0, 5, big, 1 << 30, None) == -16
    assert f(0, 0, 4, 4, 4, 1.0, big, 4, big, 4, 0.0, big, 4, 3, 0, 0, big + 8, 1 << 30, None) == -17
    assert f(0, 0, 4, 4, 4, 1.0, big, 4, big, 4, 0.0, big, 4, 3, 0, 0, big, 16, None) == -18


def test_config3_sampled_8192():
    # m = n = k = 8192, signed log-uniform over [1e-8, 1e8], seven BF16 slices.
    m = n = k = 8192
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform", with_c=False)
    got = run(A, B, None, 1.0, 0.0, 7)
    rng = np.random.Generator(np.random.PCG64(3))
    rows = np.concatenate([rng.integers(0, m, 300), [0, m - 1, 127, 128, 255, 256]])
    cols = np.concatenate([rng.integers(0, n, 300), [n - 1, 0, 128, 127, 63, 64]])
    emu = se.split_gemm_entries(A, B, rows, cols, 7, "bf16")
    np.testing.assert_array_equal(got[rows, cols], emu)
    exact = oracle.gemm_entries(A, B, rows, cols)
    absab = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
    assert np.max(np.abs(got[rows, cols] - exact) / absab) <= 1e-13


# INT8 slices: 7-bit truncated slices on INT8 MFMA with INT32 accumulation.

@pytest.mark.parametrize("S", [1, 2, 4, 7, 9, 10])
@pytest.mark.parametrize("kind", ["uniform", "loguniform"])
def test_int8_bit_exact_against_emulation(S, kind):
    # 300 x 280 x 260: two 256 x 256 tiles along m and along n, both with
    # ragged tails, k over three 128-deep steps (ragged), so the staggered k
    # start wraps.
    m, n, k = 300, 280, 260
    A, B, C = workloads.gemm_operands(m, n, k, kind=kind)
    want = se.split_gemm(A, B, S, "int8", C, 1.0, 1.0)
    np.testing.assert_array_equal(run(A, B, C, 1.0, 1.0, S, kind="int8"), want)


@pytest.mark.parametrize("shape", [(1, 1, 1), (129, 7, 65), (17, 200, 3), (520, 130, 1000), (256, 128, 128)])
@pytest.mark.parametrize("member", ["AUTO", "C0"])
def test_int8_ragged_shapes_bit_exact(shape, member):
    m, n, k = shape
    A, B, C = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = se.split_gemm(A, B, 7, "int8", C, -1.5, 0.25)
    np.testing.assert_array_equal(run(A, B, C, -1.5, 0.25, 7, member, kind="int8"), want)


@pytest.mark.parametrize("ta,tb", [(False, True), (True, False), (True, True)])
def test_int8_transposed_operands_bit_exact(ta, tb):
    m, n, k = 200, 150, 170
    A, B, C = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = se.split_gemm(A, B, 5, "int8", C, 1.0, 1.0)
    got = run(A.T.copy() if ta else A, B.T.copy() if tb else B, C, 1.0, 1.0, 5, ta=ta, tb=tb, kind="int8")
    np.testing.assert_array_equal(got, want)


def test_int8_integers_exact_and_zero_lines():
    m, n, k = 160, 144, 300
    A, B, C = workloads.gemm_operands(m, n, k, kind="int")
    want = (A.astype(np.int64) @ B.astype(np.int64) + C.astype(np.int64)).astype(np.float64)
    np.testing.assert_array_equal(run(A, B, C, 1.0, 1.0, 1, kind="int8"), want)
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    A[5] = 0.0
    B[:, 7] = 0.0
    got = run(A, B, np.full((m, n), np.nan), 1.0, 0.0, 4, kind="int8")
    np.testing.assert_array_equal(got, se.split_gemm(A, B, 4, "int8"))
    assert (got[5] == 0).all() and (got[:, 7] == 0).all()


def test_int8_error_against_fp64_oracle():
    m, n, k = 192, 160, 512
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = oracle.gemm(A, B)
    absab = np.abs(A) @ np.abs(B)
    # 9 INT8 slices carry 63 bits, as many as 7 BF16 slices
    assert np.max(np.abs(run(A, B, None, 1.0, 0.0, 9, kind="int8") - want) / absab) <= 1e-13
    e = se.exponents(A, 1)
    f = se.exponents(B, 0)
    for S in (3, 6, 8, 10):
        got = run(A, B, None, 1.0, 0.0, S, kind="int8")
        tau = 2.0 ** -(7 * S)
        bound = (S + 2) * 1.01 * tau * k * np.ldexp(1.0, e[:, None] + f[None, :]) + (S + 2) * 2.0 ** -53 * absab
        assert np.all(np.abs(got - want) <= bound), S


def test_int8_config3_sampled_8192():
    # m = n = k = 8192, signed log-uniform over [1e-8, 1e8], nine INT8 slices.
    m = n = k = 8192
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform", with_c=False)
    got = run(A, B, None, 1.0, 0.0, 9, kind="int8")
    rng = np.random.Generator(np.random.PCG64(4))
    rows = np.concatenate([rng.integers(0, m, 300), [0, m - 1, 255, 256]])
    cols = np.concatenate([rng.integers(0, n, 300), [n - 1, 0, 128, 127]])
    emu = se.split_gemm_entries(A, B, rows, cols, 9, "int8")
    np.testing.assert_array_equal(got[rows, cols], emu)
    exact = oracle.gemm_entries(A, B, rows, cols)
    absab = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
    assert np.max(np.abs(got[rows, cols] - exact) / absab) <= 1e-13


# FP8 slices: 4 + 5 s bit slices (round to nearest, exact in OCP E4M3) on FP8
# MFMA with FP32 accumulation.

@pytest.mark.parametrize("S", [1, 2, 3, 6, 9, 12])
@pytest.mark.parametrize("kind", ["uniform", "loguniform"])
def test_fp8_bit_exact_against_emulation(S, kind):
    m, n, k = 300, 280, 260
    A, B, C = workloads.gemm_operands(m, n, k, kind=kind)
    want = se.split_gemm(A, B, S, "fp8", C, 1.0, 1.0)
    np.testing.assert_array_equal(run(A, B, C, 1.0, 1.0, S, kind="fp8"), want)


@pytest.mark.parametrize("shape", [(1, 1, 1), (129, 7, 65), (17, 200, 3), (520, 130, 1000), (256, 128, 128)])
@pytest.mark.parametrize("member", ["AUTO", "C0"])
def test_fp8_ragged_shapes_bit_exact(shape, member):
    m, n, k = shape
    A, B, C = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = se.split_gemm(A, B, 7, "fp8", C, -1.5, 0.25)
    np.testing.assert_array_equal(run(A, B, C, -1.5, 0.25, 7, member, kind="fp8"), want)


@pytest.mark.parametrize("ta,tb", [(False, True), (True, False), (True, True)])
def test_fp8_transposed_operands_bit_exact(ta, tb):
    m, n, k = 200, 330, 190
    A, B, C = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = se.split_gemm(A, B, 5, "fp8", C, 1.0, 1.0)
    got = run(A.T.copy() if ta else A, B.T.copy() if tb else B, C, 1.0, 1.0, 5, ta=ta, tb=tb, kind="fp8")
    np.testing.assert_array_equal(got, want)


def test_fp8_small_integers_exact_and_zero_lines():
    # entries in [-15, 15] with a 16 in every row of A and every column of B:
    # 2^e = 32, so the first slice holds half of each value rounded to even
    # and the second slice the rest exactly; with three slices the diagonal
    # s + t = 2 adds the product of the second slices, giving the integer
    # product (two slices would drop it).
    m, n, k = 160, 144, 300
    rng = np.random.Generator(np.random.PCG64(11))
    A = rng.integers(-15, 16, (m, k)).astype(np.float64)
    B = rng.integers(-15, 16, (k, n)).astype(np.float64)
    A[:, 0] = 16.0
    B[0, :] = 16.0
    C = rng.integers(-100, 101, (m, n)).astype(np.float64)
    want = (A.astype(np.int64) @ B.astype(np.int64) + C.astype(np.int64)).astype(np.float64)
    np.testing.assert_array_equal(run(A, B, C, 1.0, 1.0, 3, kind="fp8"), want)
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    A[5] = 0.0
    B[:, 7] = 0.0
    got = run(A, B, np.full((m, n), np.nan), 1.0, 0.0, 4, kind="fp8")
    np.testing.assert_array_equal(got, se.split_gemm(A, B, 4, "fp8"))
    assert (got[5] == 0).all() and (got[:, 7] == 0).all()


def test_fp8_error_against_fp64_oracle():
    m, n, k = 192, 160, 512
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = oracle.gemm(A, B)
    absab = np.abs(A) @ np.abs(B)
    # 12 FP8 slices carry 59 bits
    assert np.max(np.abs(run(A, B, None, 1.0, 0.0, 12, kind="fp8") - want) / absab) <= 1e-13
    e = se.exponents(A, 1)
    f = se.exponents(B, 0)
    for S in (3, 6, 9, 12):
        got = run(A, B, None, 1.0, 0.0, S, kind="fp8")
        tau = 2.0 ** -(5 * S)
        bound = (S + 2) * 1.01 * tau * k * np.ldexp(1.0, e[:, None] + f[None, :]) + (S + 2) * 2.0 ** -53 * absab
        assert np.all(np.abs(got - want) <= bound), S


def test_fp8_sampled_8192_at_the_exactness_limit():
    # m = n = k = 8192, signed log-uniform over [1e-8, 1e8], eight FP8 slices:
    # 8 * 8192 = 2^16 products per diagonal, the largest exact FP32 sum.
    m = n = k = 8192
    S = 8
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform", with_c=False)
    got = run(A, B, None, 1.0, 0.0, S, kind="fp8")
    rng = np.random.Generator(np.random.PCG64(5))
    rows = np.concatenate([rng.integers(0, m, 300), [0, m - 1, 255, 256]])
    cols = np.concatenate([rng.integers(0, n, 300), [n - 1, 0, 128, 127]])
    emu = se.split_gemm_entries(A, B, rows, cols, S, "fp8")
    np.testing.assert_array_equal(got[rows, cols], emu)
    exact = oracle.gemm_entries(A, B, rows, cols)
    e = se.exponents(A, 1)[rows]
    f = se.exponents(B, 0)[cols]
    absab = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
    bound = (S + 2) * 1.01 * 2.0 ** -(5 * S) * k * np.ldexp(1.0, e + f) + (S + 2) * 2.0 ** -53 * absab
    assert np.all(np.abs(got[rows, cols] - exact) <= bound)


# Modular form: INT8 products of residues modulo N moduli, Chinese remainder
# reconstruction; equal bit for bit to the exact-integer definition.
from oracle import crt_emul as ce  # noqa: E402


@pytest.mark.parametrize("N", [2, 5, 9, 14, 16])
@pytest.mark.parametrize("kind", ["uniform", "loguniform"])
def test_crt_bit_exact_against_definition(N, kind):
    m, n, k = 300, 280, 260
    A, B, C = workloads.gemm_operands(m, n, k, kind=kind)
    want = ce.crt_gemm(A, B, N, C, 1.0, 1.0)
    np.testing.assert_array_equal(run(A, B, C, 1.0, 1.0, N, kind="crt"), want)


@pytest.mark.parametrize("shape", [(1, 1, 1), (129, 7, 65), (17, 200, 3), (520, 130, 1000)])
@pytest.mark.parametrize("member", ["AUTO", "C0"])
def test_crt_ragged_shapes_bit_exact(shape, member):
    m, n, k = shape
    A, B, C = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = ce.crt_gemm(A, B, 15, C, -1.5, 0.25)
    np.testing.assert_array_equal(run(A, B, C, -1.5, 0.25, 15, member, kind="crt"), want)


@pytest.mark.parametrize("ta,tb", [(False, True), (True, False), (True, True)])
def test_crt_transposed_operands_bit_exact(ta, tb):
    m, n, k = 200, 330, 190
    A, B, C = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = ce.crt_gemm(A, B, 12, C, 1.0, 1.0)
    got = run(A.T.copy() if ta else A, B.T.copy() if tb else B, C, 1.0, 1.0, 12, ta=ta, tb=tb, kind="crt")
    np.testing.assert_array_equal(got, want)


def test_crt_integers_exact_and_zero_lines():
    m, n, k = 160, 144, 300
    A, B, C = workloads.gemm_operands(m, n, k, kind="int")
    want = (A.astype(np.int64) @ B.astype(np.int64) + C.astype(np.int64)).astype(np.float64)
    np.testing.assert_array_equal(run(A, B, C, 1.0, 1.0, 6, kind="crt"), want)
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    A[5] = 0.0
    B[:, 7] = 0.0
    got = run(A, B, np.full((m, n), np.nan), 1.0, 0.0, 14, kind="crt")
    np.testing.assert_array_equal(got, ce.crt_gemm(A, B, 14))
    assert (got[5] == 0).all() and (got[:, 7] == 0).all()


def test_crt_error_against_fp64_oracle():
    m, n, k = 192, 160, 512
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform")
    want = oracle.gemm(A, B)
    absab = np.abs(A) @ np.abs(B)
    e = se.exponents(A, 1)
    f = se.exponents(B, 0)
    sa = np.abs(A).sum(axis=1)
    sb = np.abs(B).sum(axis=0)
    for N in (8, 12, 16):
        t = ce.bits(k, N)
        got = run(A, B, None, 1.0, 0.0, N, kind="crt")
        bound = (np.ldexp(sb[None, :], e[:, None] - t - 1) + np.ldexp(sa[:, None], f[None, :] - t - 1)
                 + k * np.ldexp(1.0, e[:, None] + f[None, :] - 2 * t - 2)) * 1.001 + 2.0 ** -52 * np.abs(want)
        assert np.all(np.abs(got - want) <= bound), N
    assert np.max(np.abs(got - want) / absab) <= 1e-13


@pytest.mark.parametrize("N", [14, 15])
def test_crt_sampled_8192(N):
    # m = n = k = 8192, signed log-uniform over [1e-8, 1e8]; 14 moduli (t = 48,
    # the fastest configuration within 1e-13) and 15 (t = 51).  Sampled
    # entries plus every row and column on either side of a 256-wide tile
    # edge: bit for bit against the exact-integer definition, and within
    # 1e-13 of (|A||B|)_ij against the compensated oracle.
    m = n = k = 8192
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform", with_c=False)
    got = run(A, B, None, 1.0, 0.0, N, kind="crt")
    rng = np.random.Generator(np.random.PCG64(6))
    edges = np.concatenate([np.arange(0, m, 256), np.arange(255, m, 256)])
    rows = np.concatenate([rng.integers(0, m, 200), [0, m - 1, 255, 256], edges, rng.integers(0, m, edges.size)])
    cols = np.concatenate([rng.integers(0, n, 200), [n - 1, 0, 128, 127], rng.integers(0, n, edges.size), edges])
    np.testing.assert_array_equal(got[rows, cols], ce.crt_gemm_entries(A, B, rows, cols, N))
    exact = oracle.gemm_entries(A, B, rows, cols)
    absab = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
    assert np.max(np.abs(got[rows, cols] - exact) / absab) <= 1e-13


@pytest.mark.parametrize("kind,S", [("bf16", 4), ("int8", 6), ("fp8", 6), ("crt", 14)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, True)])
def test_split_leading_dimensions_with_nan_gaps(kind, S, ta, tb):
    # operands and C are views into wider NaN-filled buffers: the gaps must be
    # neither read (a NaN would spread) nor written
    m, n, k = 150, 140, 130
    A, B, C = workloads.gemm_operands(m, n, k, kind="loguniform")
    if kind == "crt":
        want = ce.crt_gemm(A, B, S, C, 2.0, 0.5)
    else:
        want = se.split_gemm(A, B, S, kind, C, 2.0, 0.5)
    As = A.T.copy() if ta else A
    Bs = B.T.copy() if tb else B
    Abig = torch.full((As.shape[0], As.shape[1] + 7), float("nan"), dtype=torch.float64, device=DEV)
    Bbig = torch.full((Bs.shape[0], Bs.shape[1] + 3), float("nan"), dtype=torch.float64, device=DEV)
    Cbig = torch.full((m, n + 5), float("nan"), dtype=torch.float64, device=DEV)
    Abig[:, :As.shape[1]] = dev(As)
    Bbig[:, :Bs.shape[1]] = dev(Bs)
    Cbig[:, :n] = dev(C)
    mm.gemm_split(Abig[:, :As.shape[1]], Bbig[:, :Bs.shape[1]], Cbig[:, :n], alpha=2.0, beta=0.5, slices=S,
                  slice_type=kind, transA=ta, transB=tb)
    torch.cuda.synchronize()
    got = Cbig.cpu().numpy()
    np.testing.assert_array_equal(got[:, :n], want)
    assert np.isnan(got[:, n:]).all(), "wrote outside the leading-dimension gap"


def test_crt14_every_entry_within_1e13_at_8192():
    # m = n = k = 8192, signed log-uniform over [1e-8, 1e8]: the 14-moduli
    # product within 1e-13 of (|A||B|)_ij on all 67M entries.  The reference
    # is the 16-moduli product, pinned on sampled entries against the oracle
    # (its own error there is about 1e-16), so by the triangle inequality the
    # 14-moduli error is within 0.9e-13 + 1e-15 of |A||B| everywhere.
    m = n = k = 8192
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform", with_c=False)
    Ad, Bd = dev(A), dev(B)
    ref = mm.gemm_split(Ad, Bd, slices=16, slice_type="crt")
    rng = np.random.Generator(np.random.PCG64(9))
    rows = np.concatenate([rng.integers(0, m, 200), [0, m - 1, 255, 256]])
    cols = np.concatenate([rng.integers(0, n, 200), [n - 1, 0, 255, 256]])
    exact = oracle.gemm_entries(A, B, rows, cols)
    absab = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
    assert np.max(np.abs(ref[rows, cols].cpu().numpy() - exact) / absab) <= 1e-15
    got = mm.gemm_split(Ad, Bd, slices=14, slice_type="crt")
    absab_d = mm.gemm(Ad.abs(), Bd.abs())
    diff = (got - ref).abs_()
    del got, ref
    rel = torch.where(absab_d > 0, diff / absab_d, diff)
    assert float(rel.max().item()) <= 0.9e-13
