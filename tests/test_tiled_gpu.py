"""Tile-major ("prepacked") storage mode through the C ABI: conversion round
trips are bit-exact, and the product on tiled operands equals the row-major
product of the same member bit for bit (same loop nest, k stagger and
micro-kernel; only the loads differ; Goto reads the tiled B in place instead
of packing it), within the FP64 bound of the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu
mm = pytest.importorskip("paper_1904_05717_amd")
DEV = "cuda:0"
MEMBERS = ["C0", "C3C0", "B3C0", "A3C0", "A2C0", "B3A2C0", "A3B2C0", "C3A2C0", "C4A2C0", "AUTO"]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("op", ["A", "B"])
@pytest.mark.parametrize("shape", [(1, 1), (130, 17), (17, 300), (256, 32), (301, 129)])
@pytest.mark.parametrize("trans", [False, True])
def test_round_trip_bit_exact(op, shape, trans):
    rows, cols = shape
    X = workloads.uniform((cols, rows) if trans else (rows, cols), 11)
    T = mm.to_tiled(dev(X), op, trans=trans)
    back = mm.from_tiled(T, op, rows, cols).cpu().numpy()
    np.testing.assert_array_equal(back, X.T if trans else X)


def test_layout_positions_and_padding():
    # A: element (r, c) at ((r // 128) * slabs + c // 16) * 2048 + (r % 128) * 16 + c % 16;
    # B: element (r, c) at ((c // 128) * kp + r) * 128 + c % 128; everything else zero.
    m, k, n = 200, 40, 150
    A = workloads.uniform((m, k), 12)
    B = workloads.uniform((k, n), 13)
    Ta = mm.to_tiled(dev(A), "A").cpu().numpy()
    Tb = mm.to_tiled(dev(B), "B").cpu().numpy()
    kp, slabs = 48, 3
    r, c = np.meshgrid(np.arange(m), np.arange(k), indexing="ij")
    ia = ((r // 128) * slabs + c // 16) * 2048 + (r % 128) * 16 + c % 16
    np.testing.assert_array_equal(Ta[ia], A)
    assert np.count_nonzero(np.delete(Ta, ia.ravel())) == 0
    r, c = np.meshgrid(np.arange(k), np.arange(n), indexing="ij")
    ib = ((c // 128) * kp + r) * 128 + c % 128
    np.testing.assert_array_equal(Tb[ib], B)
    assert np.count_nonzero(np.delete(Tb, ib.ravel())) == 0


@pytest.mark.parametrize("member", MEMBERS)
@pytest.mark.parametrize("shape", [(256, 256, 256), (300, 290, 700), (129, 65, 33), (1, 1, 1), (640, 1100, 1500),
                                   (1000, 256, 1000), (2000, 1100, 300)])
def test_equals_row_major_and_within_bound(member, shape):
    m, n, k = shape
    A, B, C = workloads.gemm_operands(m, n, k)
    Ad, Bd = dev(A), dev(B)
    got = mm.gemm_tiled(mm.to_tiled(Ad, "A"), mm.to_tiled(Bd, "B"), m, n, k, dev(C.copy()), 1.5, -0.5,
                        member=member).cpu().numpy()
    ref_member = member if member != "AUTO" else mm.select_member(m, n, k)
    if ref_member != "AUTO":
        # Goto on row-major operands packs B into the workspace; on tiled
        # operands it reads the same panel layout in place
        wsb = mm.workspace_size(m, n, k, ref_member)
        ws = torch.empty(wsb, dtype=torch.uint8, device=DEV) if wsb else None
        row = mm.gemm(Ad, Bd, dev(C.copy()), 1.5, -0.5, member=ref_member, workspace=ws).cpu().numpy()
        np.testing.assert_array_equal(got, row)
    want = oracle.gemm(A, B, C, 1.5, -0.5)
    bound = oracle.error_bound(A, B, C, 1.5, -0.5, k)
    assert np.all(np.abs(got - want) <= bound)


def test_transposed_sources_and_integers_exact():
    m, n, k = 260, 140, 300
    A, B, C = workloads.gemm_operands(m, n, k, kind="int")
    At = mm.to_tiled(dev(A.T.copy()), "A", trans=True)
    Bt = mm.to_tiled(dev(B.T.copy()), "B", trans=True)
    got = mm.gemm_tiled(At, Bt, m, n, k, dev(C.copy()), 1.0, 1.0).cpu().numpy()
    want = (A.astype(np.int64) @ B.astype(np.int64) + C.astype(np.int64)).astype(np.float64)
    np.testing.assert_array_equal(got, want)


def test_quick_returns_and_beta_zero():
    m, n, k = 130, 70, 50
    A, B, C = workloads.gemm_operands(m, n, k)
    At, Bt = mm.to_tiled(dev(A), "A"), mm.to_tiled(dev(B), "B")
    np.testing.assert_array_equal(mm.gemm_tiled(At, Bt, m, n, k, dev(C.copy()), 0.0, 2.0).cpu().numpy(), 2.0 * C)
    np.testing.assert_array_equal(mm.gemm_tiled(At, Bt, m, n, 0, dev(C.copy()), 1.0, -1.0).cpu().numpy(), -C)
    Cn = dev(np.full((m, n), np.nan))
    got = mm.gemm_tiled(At, Bt, m, n, k, Cn, 1.0, 0.0).cpu().numpy()
    assert np.all(np.abs(got - oracle.gemm(A, B)) <= oracle.error_bound(A, B, None, 1.0, 0.0, k))


def test_8192_sampled():
    m = n = k = 8192
    A, B, _ = workloads.gemm_operands(m, n, k, with_c=False)
    got = mm.gemm_tiled(mm.to_tiled(dev(A), "A"), mm.to_tiled(dev(B), "B"), m, n, k, member="C3C0")
    rng = np.random.Generator(np.random.PCG64(5))
    rows = np.concatenate([rng.integers(0, m, 200), [0, m - 1, 127, 128]])
    cols = np.concatenate([rng.integers(0, n, 200), [n - 1, 0, 128, 127]])
    g = got.cpu().numpy()[rows, cols]
    exact = oracle.gemm_entries(A, B, rows, cols)
    absab = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
    assert np.all(np.abs(g - exact) <= 2 * (k + 2) * 2.0 ** -53 * absab)
