"""Batched uneven GEMMs through the C ABI: every problem against the oracle,
graph replays against the eager result, and bitwise agreement with the
single-GEMM path when the register tile is the same."""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu
mm = pytest.importorskip("paper_1904_05717_amd")
DEV = "cuda:0"


def make_batch(shapes, seed0=100):
    host, dev = [], []
    for i, (m, n, k) in enumerate(shapes):
        A = workloads.uniform((m, k), seed0 + 3 * i)
        B = workloads.uniform((k, n), seed0 + 3 * i + 1)
        C = workloads.uniform((m, n), seed0 + 3 * i + 2)
        host.append((A, B, C))
        dev.append((torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV), torch.from_numpy(C).to(DEV)))
    return host, dev


SMALL = [(1, 1, 1), (7, 300, 65), (130, 129, 257), (64, 64, 64), (0, 5, 5), (5, 0, 5), (33, 17, 0),
         (200, 150, 170), (256, 256, 32), (129, 1, 400), (300, 280, 260)]


@pytest.mark.parametrize("tiles", [None, 64, 128])
def test_small_batch_against_oracle(tiles):
    host, dev = make_batch(SMALL)
    probs = [(A, B, C, 1.5, -0.5) for (A, B, C) in dev]
    plan = mm.BatchPlan(probs, tiles=None if tiles is None else [tiles] * len(SMALL))
    plan.run()
    torch.cuda.synchronize()
    for (A, B, C), (_, _, Cd) in zip(host, dev):
        want = oracle.gemm(A, B, C, 1.5, -0.5)
        tol = oracle.error_bound(A, B, C, 1.5, -0.5)
        assert np.all(np.abs(Cd.cpu().numpy() - want) <= tol), (A.shape, B.shape)
    info = plan.info()
    assert info["items"] > 0 and len(info["tiles"]) == len(SMALL)
    plan.close()


def test_graph_replays_match_eager_and_single_gemm():
    shapes = [(96, 80, 70), (130, 200, 90), (40, 300, 500), (257, 129, 64)]
    host, dev = make_batch(shapes, seed0=500)
    C0 = [C.clone() for (_, _, C) in dev]
    probs = [(A, B, C, 1.0, 1.0) for (A, B, C) in dev]
    plan = mm.BatchPlan(probs, tiles=[64] * len(shapes))
    # eager reference: the single-GEMM C0 member uses the same 64 x 64 tile
    # for problems this small, so results must agree bit for bit
    ref = []
    for (A, B, _), c0 in zip(dev, C0):
        Cr = c0.clone()
        mm.gemm(A, B, Cr, 1.0, 1.0, member="C0")
        ref.append(Cr)
    torch.cuda.synchronize()
    for rep in range(3):
        for (_, _, C), c0 in zip(dev, C0):
            C.copy_(c0)           # eager work between replays
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        for (_, _, C), r in zip(dev, ref):
            assert torch.equal(C, r), f"replay {rep} differs from the eager single-GEMM result"
    plan.close()


def test_config4_512_problems_sampled():
    shapes = workloads.batch_shapes(512)
    host, dev = make_batch(shapes, seed0=10_000)
    probs = [(A, B, C, 1.0, 1.0) for (A, B, C) in dev]
    plan = mm.BatchPlan(probs)
    plan.run()
    torch.cuda.synchronize()
    info = plan.info()
    assert abs(info["flops"] - sum(2.0 * m * n * k for (m, n, k) in shapes)) < 1.0
    rng = np.random.Generator(np.random.PCG64(5))
    for (A, B, C), (_, _, Cd) in zip(host, dev):
        m, n = C.shape
        rows = rng.integers(0, m, 24)
        cols = rng.integers(0, n, 24)
        want = oracle.gemm_entries(A, B, rows, cols, C, 1.0, 1.0)
        got = Cd.cpu().numpy()[rows, cols]
        absab = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
        tol = 2.0 * (A.shape[1] + 2) * 2.0 ** -53 * (absab + np.abs(C[rows, cols]))
        assert np.all(np.abs(got - want) <= tol), (m, n, A.shape[1])
    plan.close()


SPLIT = [(130, 129, 1300), (64, 64, 64), (300, 70, 700), (1, 5, 600), (200, 150, 513), (65, 300, 1024),
         (257, 129, 40), (33, 17, 0)]


@pytest.mark.parametrize("member", ["C0", "C3C0", "B3C0", "A3C0"])
def test_each_member_against_oracle_and_single_gemm(member):
    # Every batched member against the oracle, and bitwise against the single
    # product of the same member: these problems are small enough that the
    # single product uses the 64 x 64 register tile, so the batch is given the
    # same tile.  k up to 1300 runs B3C0 and A3C0 over up to three k_c3 = 512
    # chunks, added into C by the item that completes each tile.
    host, dev = make_batch(SPLIT, seed0=700)
    C0 = [C.clone() for (_, _, C) in dev]
    ref = []
    for (A, B, _), c0 in zip(dev, C0):
        Cr = c0.clone()
        mm.gemm(A, B, Cr, -0.5, 1.25, member=member)
        ref.append(Cr)
    plan = mm.BatchPlan([(A, B, C, -0.5, 1.25) for (A, B, C) in dev], members=member, tiles=64)
    info = plan.info()
    assert info["members"] == [member] * len(SPLIT)
    want_chunks = [(-(-k // 512) if member in ("B3C0", "A3C0") and k > 512 else 1) for (_, _, k) in SPLIT]
    assert info["chunks"] == [c if (m and n) else 1 for c, (m, n, _) in zip(want_chunks, SPLIT)]
    for rep in range(2):
        for (_, _, C), c0 in zip(dev, C0):
            C.copy_(c0)
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        for (A, B, C), (_, _, Cd), r in zip(host, dev, ref):
            got = Cd.cpu().numpy()
            want = oracle.gemm(A, B, C, -0.5, 1.25)
            tol = oracle.error_bound(A, B, C, -0.5, 1.25)
            assert np.all(np.abs(got - want) <= tol), (member, A.shape, B.shape)
            assert torch.equal(Cd, r), f"{member} {A.shape}x{B.shape[1]}: replay {rep} differs from momms_gemm"
    plan.close()


def test_auto_splits_a_long_tile_and_reports_members():
    # 200 small problems and one 64 x 64 x 8192 problem: one whole-k item of
    # the long one would take far longer than a slot's share, so AUTO splits
    # its k (B3C0, since it is one tile tall and one wide) and the partials are
    # reduced in chunk order; the small ones stay whole-k (C0: a single tile).
    shapes = [(48, 40, 64)] * 200 + [(64, 64, 8192), (400, 380, 96)]
    host, dev = make_batch(shapes, seed0=900)
    plan = mm.BatchPlan([(A, B, C, 1.0, 1.0) for (A, B, C) in dev])
    info = plan.info()
    assert info["members"][200] == "B3C0" and info["chunks"][200] > 1
    assert all(x == "C0" and c == 1 for x, c in zip(info["members"][:200], info["chunks"][:200]))
    assert info["members"][201] == "C3C0"
    assert info["padded_flops"] >= info["flops"]
    C0 = [C.clone() for (_, _, C) in dev]
    for rep in range(2):
        for (_, _, C), c0 in zip(dev, C0):
            C.copy_(c0)
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        for i in (0, 199, 200, 201):
            A, B, C = host[i]
            want = oracle.gemm(A, B, C, 1.0, 1.0)
            assert np.all(np.abs(dev[i][2].cpu().numpy() - want) <= oracle.error_bound(A, B, C, 1.0, 1.0)), i
    plan.close()


def test_alpha_zero_reads_neither_operand():
    # alpha == 0: C := beta C exactly, with NaN in A and B (never read) and
    # with NULL-free but NaN-filled operands of every member
    shapes = [(70, 90, 40), (130, 129, 1300), (64, 64, 64)]
    for member in ("AUTO", "C0", "B3C0"):
        dev = []
        Cs = []
        for i, (m, n, k) in enumerate(shapes):
            C = workloads.uniform((m, n), 40 + i)
            Cs.append(C)
            dev.append((torch.full((m, k), float("nan"), dtype=torch.float64, device=DEV),
                        torch.full((k, n), float("nan"), dtype=torch.float64, device=DEV),
                        torch.from_numpy(C.copy()).to(DEV)))
        plan = mm.BatchPlan([(A, B, C, 0.0, -1.5) for (A, B, C) in dev], members=member)
        plan.run()
        torch.cuda.synchronize()
        for (_, _, Cd), C in zip(dev, Cs):
            np.testing.assert_array_equal(Cd.cpu().numpy(), -1.5 * C)
        plan.close()
