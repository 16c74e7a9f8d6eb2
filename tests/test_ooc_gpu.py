"""Out-of-core product (operands in host memory, Resident C blocks in device
memory, panels of A and B streamed in) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu
mm = pytest.importorskip("paper_1904_05717_amd")


def host(x, pinned=True):
    t = torch.from_numpy(np.ascontiguousarray(x))
    return t.pin_memory() if pinned else t.clone()


@pytest.mark.parametrize("block", [(256, 192, 200), (700, 650, 900), (128, 512, 64)])
@pytest.mark.parametrize("member", ["AUTO", "C0", "C3C0"])
def test_ragged_blocks_within_bound(block, member):
    m, n, k = 700, 650, 900
    A, B, C = workloads.gemm_operands(m, n, k)
    want = oracle.gemm(A, B, C, 1.5, 0.5)
    tol = oracle.error_bound(A, B, C, 1.5, 0.5)
    Ch = host(C)
    mm.gemm_ooc(host(A), host(B), Ch, alpha=1.5, beta=0.5, block=block, member=member)
    assert np.all(np.abs(Ch.numpy() - want) <= tol)


def test_integers_exact_and_pageable_memory():
    m, n, k = 300, 260, 500
    A, B, C = workloads.gemm_operands(m, n, k, kind="int")
    want = (A.astype(np.int64) @ B.astype(np.int64) + C.astype(np.int64)).astype(np.float64)
    Ch = host(C, pinned=False)
    mm.gemm_ooc(host(A, False), host(B, False), Ch, alpha=1.0, beta=1.0, block=(128, 100, 96))
    np.testing.assert_array_equal(Ch.numpy(), want)


def test_beta_zero_alpha_zero_and_k_zero():
    m, n, k = 200, 150, 120
    A, B, C = workloads.gemm_operands(m, n, k)
    Ch = host(np.full((m, n), np.nan))
    mm.gemm_ooc(host(A), host(B), Ch, alpha=1.0, beta=0.0, block=(64, 64, 50))
    assert np.all(np.abs(Ch.numpy() - oracle.gemm(A, B)) <= oracle.error_bound(A, B, None, 1.0, 0.0))
    Ch = host(C)
    mm.gemm_ooc(host(np.full((m, k), np.nan)), host(np.full((k, n), np.nan)), Ch, alpha=0.0, beta=-2.0,
                block=(64, 64, 50))
    np.testing.assert_array_equal(Ch.numpy(), -2.0 * C)
    Ch = host(C)
    mm.gemm_ooc(host(np.zeros((m, 0))), host(np.zeros((0, n))), Ch, alpha=1.0, beta=0.5, block=(64, 64, 50))
    np.testing.assert_array_equal(Ch.numpy(), 0.5 * C)


def test_one_block_equals_the_device_product():
    # with the whole problem in one block and one panel, the block product is
    # the device product of the same member: bit for bit
    m, n, k = 384, 320, 448
    A, B, C = workloads.gemm_operands(m, n, k)
    Ch = host(C)
    mm.gemm_ooc(host(A), host(B), Ch, alpha=1.0, beta=1.0, block=(m, n, k), member="C3C0")
    Cd = torch.from_numpy(C.copy()).to("cuda:0")
    mm.gemm(torch.from_numpy(A).to("cuda:0"), torch.from_numpy(B).to("cuda:0"), Cd, alpha=1.0, beta=1.0,
            member="C3C0")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Ch.numpy(), Cd.cpu().numpy())


def test_larger_problem_many_blocks_sampled():
    # 4096^3 through 1024 x 1024 blocks and 512-deep panels (16 blocks, 8 panels each)
    m = n = k = 4096
    A, B, C = workloads.gemm_operands(m, n, k)
    Ch = host(C)
    mm.gemm_ooc(host(A), host(B), Ch, alpha=1.0, beta=1.0, block=(1024, 1024, 512))
    rng = np.random.Generator(np.random.PCG64(9))
    rows = np.concatenate([rng.integers(0, m, 200), [0, 1023, 1024, m - 1]])
    cols = np.concatenate([rng.integers(0, n, 200), [n - 1, 1024, 1023, 0]])
    got = Ch.numpy()[rows, cols]
    want = oracle.gemm_entries(A, B, rows, cols, C, 1.0, 1.0)
    absab = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
    assert np.all(np.abs(got - want) <= 2 * (k + 2) * 2.0 ** -53 * (absab + np.abs(C[rows, cols])))
