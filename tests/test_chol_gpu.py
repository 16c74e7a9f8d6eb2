"""Cholesky factorization on the device against its plain definition
(oracle/chol.py): residual bound, agreement with the row-by-row factor, exact
integer factors, the untouched lower triangle, failing pivots, block edges."""
import numpy as np
import pytest
import torch

import oracle
from oracle import chol

pytestmark = pytest.mark.gpu
mm = pytest.importorskip("paper_1904_05717_amd")
U53 = 2.0 ** -53


def spd(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    M = rng.uniform(-1, 1, (n, n))
    return M @ M.T + n * np.eye(n)


def factor(A):
    P = np.triu(A) + np.tril(np.full(A.shape, np.nan), -1)   # the lower triangle must not be read
    Ad = torch.from_numpy(P).to("cuda:0")
    info = mm.potrf(Ad)
    out = Ad.cpu().numpy()
    assert np.isnan(np.tril(out, -1)[np.tril_indices(A.shape[0], -1)]).all()   # nor written
    return np.triu(out), info


def assert_factor_within(U, want):
    """Per entry: a factor with U^T U = A + dA, |dA| <= g |U^T| |U| (g = 4 (n+2) u,
    the constant of the residual checks here), differs from the exact factor
    by dU = up(U^-T dA U^-1) U to first order (up: the upper triangle with the
    diagonal halved), so |dU| <= triu(|U^-T| g |U^T| |U| |U^-1|) |U|.  Both
    factors carry such an error; a further factor 2 covers second-order terms."""
    n = U.shape[0]
    g = 4 * (n + 2) * U53
    from scipy.linalg import lapack
    inv, info = lapack.dtrtri(want, lower=0)
    assert info == 0
    Ui = np.abs(inv)
    S = np.triu(Ui.T @ (np.abs(want.T) @ np.abs(want)) @ Ui)
    bound = 2 * 2 * g * (S @ np.abs(want))
    err = np.abs(U - want)
    assert np.all(err <= bound), f"n={n}: {(err > bound).sum()} entries over the per-entry bound"


@pytest.mark.parametrize("n", [1, 63, 64, 65, 96, 127, 128, 129, 192, 257, 300, 700])
def test_factor_matches_definition(n):
    A = spd(n, n)
    U, info = factor(A)
    assert info == 0
    R = oracle.gemm(U.T.copy(), U, A, 1.0, -1.0)
    assert np.all(np.abs(R) <= 4 * (n + 2) * U53 * (np.abs(U.T) @ np.abs(U) + np.abs(A)))
    want, winfo = chol.potrf_upper(A)
    assert winfo == 0
    assert_factor_within(U, want)


def test_integer_factor_exact():
    n = 200
    rng = np.random.Generator(np.random.PCG64(3))
    Ut = np.triu(rng.integers(-1, 2, (n, n)).astype(np.float64), 1) + np.eye(n)
    A = (Ut.T.astype(np.int64) @ Ut.astype(np.int64)).astype(np.float64)
    assert np.abs(A).max() < 2 ** 20
    U, info = factor(A)
    assert info == 0
    np.testing.assert_array_equal(U, Ut)


@pytest.mark.parametrize("bad_row", [0, 37, 64, 100, 127, 128, 150])
def test_indefinite_reports_first_failing_pivot(bad_row):
    n = 200
    A = spd(n, 4)
    # make the leading (bad_row + 1) minor indefinite and nothing earlier
    A[bad_row, bad_row] = -abs(A[bad_row, bad_row]) - 1e6
    U, info = factor(A)
    _, want = chol.potrf_upper(A)
    assert want == bad_row + 1
    assert info == want


def test_large_residual_sampled():
    n = 2048
    A = spd(n, 5)
    U, info = factor(A)
    assert info == 0
    rows = np.array([0, 1, 63, 64, 1023, 1024, 2047])
    R = oracle.gemm(U.T[rows].copy(), U, A[rows], 1.0, -1.0)
    bound = 4 * (n + 2) * U53 * (np.abs(U.T[rows]) @ np.abs(U) + np.abs(A[rows]))
    assert np.all(np.abs(R) <= bound)


def test_leading_dimension_with_nan_gap():
    n = 200
    A = spd(n, 8)
    big = np.full((n, n + 6), np.nan)
    big[:, :n] = np.triu(A) + np.tril(np.full((n, n), np.nan), -1)
    Ad = torch.from_numpy(big).to("cuda:0")
    info = mm.potrf(Ad[:, :n])
    out = Ad.cpu().numpy()
    assert info == 0 and np.isnan(out[:, n:]).all()
    want, _ = chol.potrf_upper(A)
    assert_factor_within(np.triu(out[:, :n]), want)


def test_benchmark_configuration_8192():
    # the matrix the benchmark factors: S S^T + I with S uniform / sqrt(n),
    # built by torch on the device; the residual U^T U - A on sampled rows by
    # the oracle, and on the whole upper triangle against the same bound
    import workloads
    n = 8192
    S = torch.from_numpy(workloads.uniform((n, n), 29) / np.sqrt(n)).to("cuda:0")
    Ad = S @ S.t() + torch.eye(n, dtype=torch.float64, device="cuda:0")
    del S
    A = Ad.cpu().numpy()
    Ud = Ad.clone()
    assert mm.potrf(Ud) == 0
    Ud = torch.triu(Ud)
    U = Ud.cpu().numpy()
    rows = np.array([0, 127, 128, 4096, 8191])
    Ut = np.ascontiguousarray(U.T[rows])
    R = oracle.gemm(Ut, U, np.ascontiguousarray(A[rows]), 1.0, -1.0)
    bound = 4 * (n + 2) * U53 * (np.abs(Ut) @ np.abs(U) + np.abs(A[rows]))
    keep = np.zeros((len(rows), n), dtype=bool)
    for r, i in enumerate(rows):
        keep[r, i:] = True   # the upper triangle: the part of A the factorization reads
    assert np.all(np.abs(R[keep]) <= bound[keep])
    full = mm.gemm(Ud, Ud, transA=True)
    babs = mm.gemm(Ud.abs(), Ud.abs(), transA=True)
    tri_mask = torch.ones(n, n, dtype=torch.bool, device="cuda:0").triu()
    excess = ((full - Ad).abs() - 4 * (n + 2) * U53 * (babs + Ad.abs())).masked_fill(~tri_mask, -1.0)
    assert float(excess.max().item()) <= 0.0
