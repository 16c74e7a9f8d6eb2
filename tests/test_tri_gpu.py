"""Triangular multiply and solve on the device against their plain
definitions (oracle/tri.py): every uplo / trans / diag combination, ragged
recursion, exact integer systems, the triangle and diagonal that must not be
read, alpha = 0, and a 2048-row case on sampled columns."""
import numpy as np
import pytest
import torch

import oracle
from oracle import tri

pytestmark = pytest.mark.gpu
mm = pytest.importorskip("paper_1904_05717_amd")
DEV = "cuda:0"
U = 2.0 ** -53
COMBOS = [(u, t, d) for u in "LU" for t in (False, True) for d in "NU"]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def well_conditioned(m, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.uniform(-1, 1, (m, m)) / np.sqrt(m)
    A[np.diag_indices(m)] = rng.uniform(1, 2, m) * np.sign(rng.uniform(-1, 1, m))
    return A


def poisoned(A, uplo, diag):
    """A copy with NaN wherever the operation must not read."""
    P = A.copy()
    m = A.shape[0]
    other = np.triu_indices(m, 1) if uplo == "L" else np.tril_indices(m, -1)
    P[other] = np.nan
    if diag == "U":
        P[np.diag_indices(m)] = np.nan
    return P


def abs_inverse(T):
    """|T^-1| of a triangular T (LAPACK's triangular inverse)."""
    from scipy.linalg import lapack
    lower = not np.any(np.triu(T, 1))
    inv, info = lapack.dtrtri(T, lower=int(lower))
    assert info == 0
    return np.abs(inv)


def assert_solve_within(X, want, T, B, alpha, what=""):
    """Per entry: a substitution or blocked solve with conventional products
    satisfies (T + dT) X = alpha B + dB with |dT| <= g |T| and |dB| <=
    u |alpha B| (g = 4 (m+2) u, the constant of the residual checks here), so
    X is within |T^-1| (g |T| |X| + u |alpha B|) of the exact solution; the
    device result and the oracle's are within twice that of each other."""
    m = T.shape[0]
    g = 4 * (m + 2) * U
    bound = 2 * abs_inverse(T) @ (g * (np.abs(T) @ np.abs(X)) + U * abs(alpha) * np.abs(B))
    err = np.abs(X - want)
    assert np.all(err <= bound), f"{what}: {(err > bound).sum()} entries over the per-entry bound"


@pytest.mark.parametrize("uplo,trans,diag", COMBOS)
def test_trsm_matches_substitution(uplo, trans, diag):
    m, n = 300, 170   # recursion 300 -> 192 + 108 -> ..., ragged diagonal blocks
    A = well_conditioned(m, 1)
    B = np.random.Generator(np.random.PCG64(2)).uniform(-1, 1, (m, n))
    Bd = dev(B)
    mm.trsm(dev(poisoned(A, uplo, diag)), Bd, alpha=0.75, uplo=uplo, trans=trans, diag=diag)
    torch.cuda.synchronize()
    X = Bd.cpu().numpy()
    T = tri.op_tri(A, uplo, trans, diag)
    R = oracle.gemm(T, X, B, 1.0, -0.75)
    assert np.all(np.abs(R) <= 4 * (m + 2) * U * (np.abs(T) @ np.abs(X) + 0.75 * np.abs(B)))
    want = tri.trsm(A, B, uplo, trans, diag, alpha=0.75)
    assert_solve_within(X, want, T, B, 0.75, f"{uplo} {trans} {diag}")


@pytest.mark.parametrize("uplo,trans,diag", COMBOS)
def test_trmm_within_product_bound(uplo, trans, diag):
    m, n = 300, 170
    rng = np.random.Generator(np.random.PCG64(3))
    A = rng.uniform(-1, 1, (m, m))
    B = rng.uniform(-1, 1, (m, n))
    C = dev(np.full((m, n), np.nan))
    mm.trmm(dev(poisoned(A, uplo, diag)), dev(B), C, alpha=-1.25, uplo=uplo, trans=trans, diag=diag)
    torch.cuda.synchronize()
    T = tri.op_tri(A, uplo, trans, diag)
    want = tri.trmm(A, B, uplo, trans, diag, alpha=-1.25)
    tol = 2 * (m + 2) * U * 1.25 * (np.abs(T) @ np.abs(B))
    assert np.all(np.abs(C.cpu().numpy() - want) <= tol)


@pytest.mark.parametrize("uplo,trans", [("L", False), ("U", True), ("U", False), ("L", True)])
def test_integer_unit_systems_exact(uplo, trans):
    m, n = 200, 90
    rng = np.random.Generator(np.random.PCG64(4))
    A = rng.integers(-1, 2, (m, m)).astype(np.float64)
    X = rng.integers(-2, 3, (m, n)).astype(np.float64)
    T = tri.op_tri(A, uplo, trans, "U")
    B = (T.astype(np.int64) @ X.astype(np.int64)).astype(np.float64)
    C = dev(np.zeros((m, n)))
    mm.trmm(dev(A), dev(X), C, uplo=uplo, trans=trans, diag="U")
    Bd = dev(B)
    mm.trsm(dev(A), Bd, uplo=uplo, trans=trans, diag="U")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(C.cpu().numpy(), B)
    # every value substitution and the block updates form is a partial sum of
    # small integers (the solution itself is X), so the solve is exact
    np.testing.assert_array_equal(Bd.cpu().numpy(), X)


def test_alpha_zero_and_empty():
    m, n = 70, 30
    A = np.full((m, m), np.nan)
    Bd = dev(np.ones((m, n)))
    mm.trsm(dev(A), Bd, alpha=0.0)
    C = dev(np.full((m, n), np.nan))
    mm.trmm(dev(A), dev(np.full((m, n), np.nan)), C, alpha=0.0)
    torch.cuda.synchronize()
    assert (Bd.cpu().numpy() == 0).all() and (C.cpu().numpy() == 0).all()
    E = dev(np.zeros((0, 5)))
    mm.trsm(dev(np.zeros((0, 0))), E)
    mm.trmm(dev(np.zeros((0, 0))), E, dev(np.zeros((0, 5))))


@pytest.mark.parametrize("m", [1, 63, 64, 65, 96, 127, 128, 129, 192, 257])
def test_block_edges(m):
    n = 33
    A = well_conditioned(m, 5)
    B = np.random.Generator(np.random.PCG64(6)).uniform(-1, 1, (m, n))
    Bd = dev(B)
    mm.trsm(dev(A), Bd, uplo="U", trans=True)
    C = dev(np.zeros((m, n)))
    mm.trmm(dev(A), dev(B), C, uplo="L")
    torch.cuda.synchronize()
    want = tri.trsm(A, B, "U", True)
    assert_solve_within(Bd.cpu().numpy(), want, tri.op_tri(A, "U", True), B, 1.0, f"m={m}")
    T = tri.op_tri(A, "L")
    assert np.all(np.abs(C.cpu().numpy() - tri.trmm(A, B, "L")) <= 2 * (m + 2) * U * (np.abs(T) @ np.abs(B)))


@pytest.mark.parametrize("uplo,trans,diag", COMBOS)
@pytest.mark.parametrize("m", [65, 100, 128, 150, 192, 193])
def test_multi_block_solve_every_combination(m, uplo, trans, diag):
    """Solves past one diagonal block: two and three 64-row blocks with the
    products between them (ragged last blocks, and uneven splits at 150 and
    193), on a ragged number of columns."""
    n = 70
    A = well_conditioned(m, 11)
    B = np.random.Generator(np.random.PCG64(12)).uniform(-1, 1, (m, n))
    Bd = dev(B)
    mm.trsm(dev(A), Bd, alpha=0.5, uplo=uplo, trans=trans, diag=diag)
    torch.cuda.synchronize()
    want = tri.trsm(A, B, uplo, trans, diag, alpha=0.5)
    assert_solve_within(Bd.cpu().numpy(), want, tri.op_tri(A, uplo, trans, diag), B, 0.5, f"m={m}")


def test_large_sampled_columns():
    m, n = 2048, 1024
    A = well_conditioned(m, 7)
    B = np.random.Generator(np.random.PCG64(8)).uniform(-1, 1, (m, n))
    Bd = dev(B)
    mm.trsm(dev(A), Bd, uplo="L", trans=False)
    C = dev(np.zeros((m, n)))
    mm.trmm(dev(A), dev(B), C, uplo="U", trans=True, alpha=2.0)
    torch.cuda.synchronize()
    cols = np.array([0, 1, 511, 512, 1023])
    want = tri.trsm(A, B[:, cols], "L")
    assert_solve_within(Bd.cpu().numpy()[:, cols], want, tri.op_tri(A, "L"), B[:, cols], 1.0, "2048")
    T = tri.op_tri(A, "U", True)
    wc = tri.trmm(A, B[:, cols], "U", True, alpha=2.0)
    assert np.all(np.abs(C.cpu().numpy()[:, cols] - wc) <= 2 * (m + 2) * U * 2.0 * (np.abs(T) @ np.abs(B[:, cols])))


def test_leading_dimensions_with_nan_gaps():
    m, n = 150, 90
    A = well_conditioned(m, 9)
    B = np.random.Generator(np.random.PCG64(10)).uniform(-1, 1, (m, n))
    Abig = torch.full((m, m + 5), float("nan"), dtype=torch.float64, device=DEV)
    Abig[:, :m] = dev(A)
    Bbig = torch.full((m, n + 3), float("nan"), dtype=torch.float64, device=DEV)
    Bbig[:, :n] = dev(B)
    Cbig = torch.full((m, n + 4), float("nan"), dtype=torch.float64, device=DEV)
    mm.trmm(Abig[:, :m], Bbig[:, :n], Cbig[:, :n], uplo="U", trans=True)
    mm.trsm(Abig[:, :m], Bbig[:, :n], uplo="L", trans=True, alpha=1.5)
    torch.cuda.synchronize()
    T = tri.op_tri(A, "U", True)
    gc = Cbig.cpu().numpy()
    assert np.all(np.abs(gc[:, :n] - tri.trmm(A, B, "U", True)) <= 2 * (m + 2) * U * (np.abs(T) @ np.abs(B)))
    assert np.isnan(gc[:, n:]).all()
    gb = Bbig.cpu().numpy()
    want = tri.trsm(A, B, "L", True, alpha=1.5)
    assert_solve_within(gb[:, :n], want, tri.op_tri(A, "L", True), B, 1.5, "nan gaps")
    assert np.isnan(gb[:, n:]).all()


def test_benchmark_configuration_8192_sampled_columns():
    # the shape and data the benchmark times: m = n = 8192, lower triangle,
    # off-diagonal U[-1, 1] / sqrt(m), diagonal 1.5
    import workloads
    m = n = 8192
    A = workloads.uniform((m, m), 27) / np.sqrt(m)
    A[np.diag_indices(m)] = 1.5
    B = workloads.uniform((m, n), 28)
    Ad, Bd = dev(A), dev(B)
    X = Bd.clone()
    mm.trsm(Ad, X, uplo="L")
    C = torch.empty_like(Bd)
    mm.trmm(Ad, Bd, C, uplo="L")
    torch.cuda.synchronize()
    cols = [0, 1, 63, 64, 4095, 8191]
    Bc = np.ascontiguousarray(B[:, cols])
    want = tri.trsm(A, Bc, "L")
    assert_solve_within(X[:, cols].cpu().numpy(), want, tri.op_tri(A, "L"), Bc, 1.0, "8192")
    T = tri.op_tri(A, "L")
    got = C[:, cols].cpu().numpy()
    assert np.all(np.abs(got - tri.trmm(A, Bc, "L")) <= 2 * (m + 2) * U * (np.abs(T) @ np.abs(Bc)))
