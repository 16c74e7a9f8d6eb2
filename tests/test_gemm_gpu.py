"""Parity of every FP64 family member with the CPU oracle, through the C ABI.

Bar: per entry |C_gpu - C_oracle| <= T_ij = 2 (k+2) 2^-53 (|alpha| (|A||B|)_ij
+ |beta| |C_ij|) for uniform data (the forward error bound of a k-term dot
product in any order; the oracle's own error is below 2^-53 |C_ij|, inside
the +2 margin), and bit-exact equality on integer data whose partial sums are
exact in every order.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

mm = pytest.importorskip("paper_1904_05717_amd")
FAMILY = mm.FAMILY
DEV = "cuda:0"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def run(A, B, C, alpha, beta, member, transA=False, transB=False, workspace=None):
    Cd = dev(C.copy()) if C is not None else None
    out = mm.gemm(dev(A), dev(B), Cd, alpha=alpha, beta=beta, member=member, transA=transA, transB=transB,
                  workspace=workspace)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def assert_within_bound(got, want, A, B, C, alpha, beta, what=""):
    k = A.shape[1]
    tol = oracle.error_bound(A, B, C, alpha, beta, k=k)
    err = np.abs(got - want)
    bad = err > tol
    assert not bad.any(), (f"{what}: {bad.sum()} entries over bound; worst err {err.max():.3e}, "
                           f"at {np.unravel_index(np.argmax(err - tol), err.shape)}")


@pytest.mark.parametrize("member", FAMILY + ["AUTO"])
def test_config1_uniform(member):
    m = n = k = 256
    A, B, _ = workloads.gemm_operands(m, n, k)
    C = np.zeros((m, n))
    want = oracle.gemm(A, B, C, 1.0, 1.0)
    got = run(A, B, C, 1.0, 1.0, member)
    assert_within_bound(got, want, A, B, C, 1.0, 1.0, member)


@pytest.mark.parametrize("member", FAMILY)
def test_config1_integer_bit_exact(member):
    m = n = k = 256
    A, B, _ = workloads.gemm_operands(m, n, k, kind="int")
    C = np.zeros((m, n))
    want = oracle.gemm(A, B, C, 1.0, 1.0)
    np.testing.assert_array_equal(run(A, B, C, 1.0, 1.0, member), want)


@pytest.mark.parametrize("shape", [(100, 3000, 500), (1000, 256, 1000)])
@pytest.mark.parametrize("trans", [(False, False), (True, True)])
def test_c3a2c0_shallow_chunks(shape, trans):
    # C3A2C0's chunk depth comes from its level-3 block (the chunk's A rows
    # and B columns must fit half an L2 beside the C block), so on these
    # shapes the A-resident kernel runs chunks shallower than its LDS block,
    # several of them, with a ragged last one
    m, n, k = shape
    p = mm.member_plan("C3A2C0", m, n, k)
    assert p["kc"] < 288 and k > 2 * p["kc"] and k % p["kc"] != 0, p
    ta, tb = trans
    A, B, C = workloads.gemm_operands(m, n, k)
    Ai, Bi, _ = workloads.gemm_operands(m, n, k, kind="int")
    for X, Y, Z, exact in ((A, B, C, False), (Ai, Bi, np.zeros((m, n)), True)):
        want = oracle.gemm(X, Y, Z, 1.5 if not exact else 1.0, -0.5 if not exact else 1.0)
        got = run(X.T.copy() if ta else X, Y.T.copy() if tb else Y, Z, 1.5 if not exact else 1.0,
                  -0.5 if not exact else 1.0, "C3A2C0", transA=ta, transB=tb)
        if exact:
            np.testing.assert_array_equal(got, want)
        else:
            assert_within_bound(got, want, X, Y, Z, 1.5, -0.5, f"C3A2C0 {shape} {trans}")


@pytest.mark.parametrize("trans", [(False, False), (True, True)])
def test_c3a2c0_one_workgroup_per_cu_block(trans):
    # C3A2C0 runs the 64-row, one-workgroup-per-CU form of the A-resident
    # kernel once its tiles fill the chip (the smaller shapes above run the
    # 32-row, two-per-CU form); here 2000 x 1100 gives 32 x 9 such tiles,
    # ragged in both directions, and k = 300 one full chunk and a ragged one
    m, n, k = 2000, 1100, 300
    p = mm.member_plan("C3A2C0", m, n, k)
    assert p["mt"] == 64 and p["workgroups"] >= 256 and k % p["kc"] != 0, p
    ta, tb = trans
    A, B, C = workloads.gemm_operands(m, n, k)
    Ai, Bi, _ = workloads.gemm_operands(m, n, k, kind="int")
    for X, Y, Z, exact in ((A, B, C, False), (Ai, Bi, np.zeros((m, n)), True)):
        alpha, beta = (1.0, 1.0) if exact else (1.5, -0.5)
        want = oracle.gemm(X, Y, Z, alpha, beta)
        got = run(X.T.copy() if ta else X, Y.T.copy() if tb else Y, Z, alpha, beta, "C3A2C0", transA=ta, transB=tb)
        if exact:
            np.testing.assert_array_equal(got, want)
        else:
            assert_within_bound(got, want, X, Y, Z, alpha, beta, f"C3A2C0 64-row {trans}")


def test_c4a2c0_chunks_per_launch():
    # C4A2C0's host loop steps k by kc3 (several chunks per launch) and the
    # kernel by kc inside: k = 2600 is two whole launches and a ragged third
    # (one whole chunk and an 8-deep one)
    m, n, k = 300, 700, 2600
    p = mm.member_plan("C4A2C0", m, n, k)
    assert p["kc3"] > p["kc"] and k % p["kc3"] > p["kc"] and k % p["kc3"] % p["kc"] != 0, p
    A, B, C = workloads.gemm_operands(m, n, k)
    Ai, Bi, _ = workloads.gemm_operands(m, n, k, kind="int")
    assert_within_bound(run(A, B, C, 1.5, -0.5, "C4A2C0"), oracle.gemm(A, B, C, 1.5, -0.5), A, B, C, 1.5, -0.5,
                        "C4A2C0")
    Z = np.zeros((m, n))
    np.testing.assert_array_equal(run(Ai, Bi, Z, 1.0, 1.0, "C4A2C0"), oracle.gemm(Ai, Bi, Z, 1.0, 1.0))


@pytest.mark.parametrize("member", FAMILY)
@pytest.mark.parametrize("shape", [(300, 280, 260), (129, 257, 131)])
def test_ragged_alpha_beta(member, shape):
    m, n, k = shape
    A, B, C = workloads.gemm_operands(m, n, k)
    want = oracle.gemm(A, B, C, 1.5, -0.5)
    got = run(A, B, C, 1.5, -0.5, member)
    assert_within_bound(got, want, A, B, C, 1.5, -0.5, f"{member} {shape}")


@pytest.mark.parametrize("member", ["C0", "C3C0", "A2C0"])
@pytest.mark.parametrize("shape", [(1, 1, 1), (15, 17, 3), (33, 65, 129), (64, 64, 64), (2, 300, 5)])
def test_small_shapes(member, shape):
    m, n, k = shape
    A, B, C = workloads.gemm_operands(m, n, k)
    want = oracle.gemm(A, B, C, 1.0, 1.0)
    assert_within_bound(run(A, B, C, 1.0, 1.0, member), want, A, B, C, 1.0, 1.0, f"{member} {shape}")


@pytest.mark.parametrize("member", FAMILY)
@pytest.mark.parametrize("ta,tb", [(False, True), (True, False), (True, True)])
def test_transposed_operands(member, ta, tb):
    m, n, k = 200, 150, 170
    A, B, C = workloads.gemm_operands(m, n, k)
    want = oracle.gemm(A, B, C, 1.0, 1.0)
    As = A.T.copy() if ta else A
    Bs = B.T.copy() if tb else B
    got = run(As, Bs, C, 1.0, 1.0, member, transA=ta, transB=tb)
    assert_within_bound(got, want, A, B, C, 1.0, 1.0, f"{member} ta={ta} tb={tb}")


@pytest.mark.parametrize("member", ["C0", "C3C0", "B3C0", "A2C0", "A3B2C0"])
def test_leading_dimensions(member):
    m, n, k = 130, 140, 150
    A, B, C = workloads.gemm_operands(m, n, k)
    want = oracle.gemm(A, B, C, 2.0, 0.5)
    Abig = torch.full((m, k + 7), float("nan"), dtype=torch.float64, device=DEV)
    Bbig = torch.full((k, n + 3), float("nan"), dtype=torch.float64, device=DEV)
    Cbig = torch.full((m, n + 5), float("nan"), dtype=torch.float64, device=DEV)
    Abig[:, :k] = dev(A)
    Bbig[:, :n] = dev(B)
    Cbig[:, :n] = dev(C)
    mm.gemm(Abig[:, :k], Bbig[:, :n], Cbig[:, :n], alpha=2.0, beta=0.5, member=member)
    torch.cuda.synchronize()
    got = Cbig.cpu().numpy()
    assert_within_bound(got[:, :n], want, A, B, C, 2.0, 0.5, member)
    assert np.isnan(got[:, n:]).all(), "wrote outside the leading-dimension gap"


def test_alpha_zero_k_zero_beta_zero():
    m, n, k = 70, 90, 40
    A, B, C = workloads.gemm_operands(m, n, k)
    np.testing.assert_array_equal(run(A, B, C, 0.0, 0.5, "C0"), 0.5 * C)
    np.testing.assert_array_equal(run(A, B, C, 0.0, 0.0, "C0"), np.zeros_like(C))
    Ak, Bk = np.zeros((m, 0)), np.zeros((0, n))
    np.testing.assert_array_equal(run(Ak, Bk, C, 1.0, -2.0, "C3C0"), -2.0 * C)
    Cn = np.full((m, n), np.nan)
    for member in FAMILY:
        got = run(A, B, Cn, 1.0, 0.0, member)
        assert np.isfinite(got).all(), member
        assert_within_bound(got, oracle.gemm(A, B), A, B, None, 1.0, 0.0, member)


def test_packed_goto_with_workspace():
    # n spans three n_c = 2048 panels (the last one ragged); k spans two
    # kc = 256 passes.
    m, n, k = 160, 4200, 300
    A, B, C = workloads.gemm_operands(m, n, k)
    ws = torch.empty(mm.workspace_size(m, n, k, "A2C0"), dtype=torch.uint8, device=DEV)
    got = run(A, B, C, 1.0, 1.0, "A2C0", workspace=ws)
    assert_within_bound(got, oracle.gemm(A, B, C, 1.0, 1.0), A, B, C, 1.0, 1.0, "A2C0 packed")
    Bt = B.T.copy()
    got = run(A, Bt, C, 1.0, 1.0, "A2C0", transB=True, workspace=ws)
    assert_within_bound(got, oracle.gemm(A, B, C, 1.0, 1.0), A, B, C, 1.0, 1.0, "A2C0 packed transB")


def sampled_check(m, n, k, member, npts=1500, alpha=1.0, beta=1.0, seed=0):
    A, B, C = workloads.gemm_operands(m, n, k)
    got = run(A, B, C, alpha, beta, member)
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = rng.integers(0, m, npts)
    cols = rng.integers(0, n, npts)
    # every tile boundary row/column (multiples of 64 and their predecessors) plus the last ones
    edges_r = np.unique(np.clip(np.concatenate([np.arange(0, m, 64), np.arange(63, m, 64), [m - 1]]), 0, m - 1))
    edges_c = np.unique(np.clip(np.concatenate([np.arange(0, n, 64), np.arange(63, n, 64), [n - 1]]), 0, n - 1))
    rows = np.concatenate([rows, edges_r, rng.integers(0, m, edges_c.size)])
    cols = np.concatenate([cols, rng.integers(0, n, edges_r.size), edges_c])
    want = oracle.gemm_entries(A, B, rows, cols, C, alpha, beta)
    absab = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
    tol = 2.0 * (k + 2) * 2.0 ** -53 * (abs(alpha) * absab + abs(beta) * np.abs(C[rows, cols]))
    err = np.abs(got[rows, cols] - want)
    assert (err <= tol).all(), f"{member} {m}x{n}x{k}: {(err > tol).sum()} sampled entries over bound"
    return got


@pytest.mark.parametrize("member", ["C0", "C3C0", "B3C0", "A3C0"])
def test_large_register_tile_sampled(member):
    # 128 x 128 register tiles are used once there are >= 512 tiles.
    sampled_check(3000, 2900, 384, member)


def test_bench_size_sampled():
    m = n = k = 8192
    sampled_check(m, n, k, "AUTO", npts=1024)


@pytest.mark.parametrize("member", ["A2C0", "B3A2C0", "A3B2C0", "C3A2C0", "C4A2C0"])
def test_lds_resident_members_bench_size_sampled(member):
    # the LDS-resident members at the size the member table and the
    # low-bandwidth experiments time them: every k chunk, granule and block
    # loop runs many times over
    sampled_check(8192, 8192, 8192, member, npts=512, seed=1)


@pytest.mark.parametrize("member", ["AUTO", "C0", "A2C0", "A3B2C0"])
@pytest.mark.parametrize("shape", [(16384, 16384, 256), (16384, 256, 16384)])
def test_sweep_thin_shapes_sampled(shape, member):
    # the rank-k and panel shapes of the sweep
    sampled_check(*shape, member, npts=512, seed=2)


@pytest.mark.parametrize("member", ["C0", "C3C0", "B3C0", "A3C0"])
def test_large_register_tile_integer_bit_exact(member):
    # 3072 x 3072 is 576 tiles of 128: the 128 x 128 register tile of the
    # benchmark's kernel (checked through the plan).  Integers in [-8, 8] with
    # k = 640 keep every partial sum an exact integer, so any summation order
    # gives the exact product; k = 640 also runs B3C0 and A3C0 over two k_c3
    # passes (512 + 128) and the staggered k start wraps in every tile.  The
    # exact product is the float64 BLAS product of the same integers (exact for
    # the same reason).
    m = n = 3072
    k = 640
    assert mm.member_plan(member, m, n, k)["mt"] == 128
    A, B, C = workloads.gemm_operands(m, n, k, kind="int")
    want = A @ B + C
    np.testing.assert_array_equal(run(A, B, C, 1.0, 1.0, member), want)


def test_momms_gemm_entry_point_on_the_set_stream():
    # The plain momms_gemm signature (no transposition, no workspace) on data,
    # on the stream installed by momms_set_stream: a side stream that waits on
    # an event recorded after C is filled on torch's stream.
    from paper_1904_05717_amd import _lib
    m, n, k = 517, 389, 700
    A, B, C = workloads.gemm_operands(m, n, k)
    want = oracle.gemm(A, B, C, -0.75, 1.25)
    Ad, Bd = dev(A), dev(B)
    side = torch.cuda.Stream()
    try:
        assert _lib.momms_set_stream(side.cuda_stream) == 0
        for member in ["AUTO", "C3C0", "A2C0", "B3A2C0"]:
            Cd = dev(C)
            ready = torch.cuda.Event()
            ready.record(torch.cuda.current_stream())
            side.wait_event(ready)
            st = _lib.momms_gemm(m, n, k, -0.75, Ad.data_ptr(), k, Bd.data_ptr(), n, 1.25, Cd.data_ptr(), n,
                                 mm.MEMBERS[member])
            assert st == 0, (member, st)
            side.synchronize()
            assert_within_bound(Cd.cpu().numpy(), want, A, B, C, -0.75, 1.25, f"momms_gemm {member}")
    finally:
        _lib.momms_set_stream(None)
