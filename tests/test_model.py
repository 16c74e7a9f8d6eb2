"""Pins of the data-movement model (library, host-only) against an
independent brute-force simulation and the paper's printed numbers.

* The resident algorithms of Sec. 2.2 are run element by element through an
  LRU fast memory that holds the resident block plus two streamed rows and
  columns (Sec. 4.1: under LRU the panels a loop exposes must fit beside the
  block): when the blocks divide the matrices the simulated transfers equal
  the model's counts exactly; with ragged margins the spare room can only
  save transfers.
* Belady's optimal replacement never needs more than the model and never
  fewer than the I/O lower bound of Sec. 2.1, 2mnk/sqrt(M) - 2M reads.
* The paper's analysed intensities (Sec. 5.2, kept in
  tests/golden/paper_section5_2.json): Goto's algorithm with k_c = 192,
  n_c = 3000 reaches 23.26 flop/byte and B3A2C0 with a 768 x 768 block
  64 flop/byte; the balanced blocksizes of Sec. 2.4.
"""
import json
import math
import os

import pytest

import paper_1904_05717_amd as mm
from oracle import cache_sim as cs

CASES = [("C", (3, 2)), ("A", (3, 4)), ("B", (4, 2)), ("C", (4, 4)), ("A", (4, 3)), ("B", (2, 5))]


def model(res, shape, b, beta):
    return {k: int(v) for k, v in mm.model_resident(res, *shape, *b, beta).items()}


@pytest.mark.parametrize("res,b", CASES)
@pytest.mark.parametrize("beta", [1.0, 0.0])
def test_lru_equals_model_when_blocks_divide(res, b, beta):
    # shapes that are multiples of every block dimension involved
    b1, b2 = b
    if res == "C":
        shape = (2 * b1, 3 * b2, 5)
    elif res == "A":
        shape = (3 * b1, 4, 2 * b2)
    else:
        shape = (4, 3 * b2, 2 * b1)
    assert cs.simulate_lru(res, *shape, b1, b2, beta) == model(res, shape, b, beta)


@pytest.mark.parametrize("res,b", CASES)
@pytest.mark.parametrize("shape", [(7, 5, 6), (6, 4, 8), (12, 10, 9)])
def test_ragged_margins_never_exceed_model(res, b, shape):
    for beta in (1.0, 0.0):
        sim = cs.simulate_lru(res, *shape, *b, beta)
        mod = model(res, shape, b, beta)
        assert all(sim[x] <= mod[x] for x in sim), (sim, mod)


@pytest.mark.parametrize("res,b", CASES)
def test_optimal_replacement_between_lower_bound_and_model(res, b):
    shape = (12, 10, 9)
    sim = cs.simulate(res, *shape, *b, 1.0)
    mod = model(res, shape, b, 1.0)
    assert all(sim[x] <= mod[x] for x in sim)
    m, n, k = shape
    M = b[0] * b[1] + b[0] + b[1]
    reads = sim["a_reads"] + sim["b_reads"] + sim["c_reads"]
    assert reads >= 2 * m * n * k / math.sqrt(M) - 2 * M


def intensity(res, b1, b2, scale=200):
    # flops per byte of the model at large sizes (the paper counts 8-byte
    # elements; C read and written)
    if res == "B":
        m, n, k = 10 ** 7, b2 * scale, b1 * scale
    elif res == "C":
        m, n, k = b1 * scale, b2 * scale, 10 ** 7
    else:
        m, n, k = b1 * scale, 10 ** 7, b2 * scale
    c = mm.model_resident(res, m, n, k, b1, b2, 1.0)
    return 2.0 * m * n * k / (8.0 * sum(c.values()))


GOLDEN = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                     "paper_section5_2.json")))


def test_paper_intensities():
    # Goto: the B panel k_c x n_c sits in L3 and the rest streams -> Resident B
    g = GOLDEN["goto_blocksizes"]
    want = GOLDEN["goto_intensity_flop_per_byte"]
    assert intensity("B", g["k_c"], g["n_c"]) == pytest.approx(want["value"], abs=0.5 * 10 ** -want["digits"])
    # B3A2C0: 768 x 768 block of B in L3
    b = GOLDEN["b3a2c0_blocks"]["l3_block_of_B"]
    want = GOLDEN["b3a2c0_intensity_flop_per_byte"]
    assert intensity("B", b, b) == pytest.approx(want["value"], rel=2e-3)
    # derived the same way: C3A2C0 (624 x 624 block of C) and C4A2C0 (3600)
    assert intensity("C", 624, 624) == pytest.approx(78.0, rel=2e-3)
    assert intensity("C", 3600, 3600) == pytest.approx(450.0, rel=2e-3)


def test_balanced_blocks():
    M = 120 * 192
    mc, kc = mm.balanced_block(M, 1.0, 1.0)
    assert mc == pytest.approx(math.sqrt(M)) and kc == pytest.approx(math.sqrt(M))
    mc, kc = mm.balanced_block(M, 1.0, 2.0)   # C costs twice (read and written)
    assert mc / kc == pytest.approx(0.5) and mc * kc == pytest.approx(M)


def test_member_models_follow_resident_counts():
    # The level-3 models of the gfx950 members are resident counts with the
    # member's block sizes at the L2 boundary.
    m = n = k = 8192
    g = mm.member_plan("A2C0", m, n, k)
    for name, res, b in [("B3C0", "B", (512, 128)), ("A3C0", "A", (128, 512)), ("C3C0", "C", (1024, 1024)),
                         ("A2C0", "B", (g["kc"], g["nj"] * g["nt"]))]:
        got = mm.model_bytes(name, m, n, k, beta=1.0)
        want = mm.model_resident(res, m, n, k, *b, 1.0)
        assert got["a_reads"] == 8 * want["a_reads"], name
        assert got["b_reads"] == 8 * want["b_reads"], name
        assert got["c_reads"] == 8 * want["c_reads"] and got["c_writes"] == 8 * want["c_writes"], name


def test_lds_block_solver():
    # gfx950: 160 KiB of LDS, 8-deep slices of a 128-wide streamed panel; the
    # panel comes from the L2 (39 TB/s) and C is read and written in HBM
    # (8 TB/s), so a C element costs 2 * 39.3 / 8 streamed elements.
    lds, bc = 160 * 1024, 2 * 39.3 / 8
    # a block beside two 32-deep slices of a 128-wide streamed panel (the
    # B-resident kernel keeps its A slices in LDS, one workgroup per CU, two
    # columns of waves) ...
    assert mm.lds_block(lds, 32, 128, 64, 1.0, bc) == (64, 160)
    # ... and a block alone (the A-resident kernel streams B through
    # registers) in half of it (two workgroups per CU, one row of waves):
    # 32 x 288, since 32 x 319 is the most that fits and k_c steps by the
    # slice; the continuous optimum there has 32.3 rows
    assert mm.lds_block(lds / 2, 32, 0, 32, 1.0, bc) == (32, 288)
    mc, kc = mm.balanced_block(lds / 2 / 8, 1.0, bc)
    assert round(mc) == 32
    # with a CU to itself (C3A2C0, whose XCD's workgroups must stay in step
    # for its C block to stay in the L2) the same block has 64 rows
    assert mm.lds_block(lds, 32, 0, 64, 1.0, bc) == (64, 288)
    # the plans of the LDS-resident members use exactly those blocks, with
    # 32-deep streamed slices (C3A2C0 takes a shallower chunk of its block)
    for name in ("A2C0", "B3A2C0", "C4A2C0"):
        p = mm.member_plan(name, 8192, 8192, 8192)
        assert (p["mt"], p["kc"], p["ks"]) == (32, 288, 32), name
    p = mm.member_plan("C3A2C0", 8192, 8192, 8192)
    assert (p["mt"], p["kc"], p["ks"]) == (64, 256, 32)
    p = mm.member_plan("A3B2C0", 8192, 8192, 8192)
    assert (p["nt"], p["kc"], p["ks"]) == (64, 160, 32)
    # equal costs and thin slices: the block comes out nearly square
    # (Sec. 2.4), 128 x 136 within capacity, on either row grid
    assert mm.lds_block(lds, 8, 128, 64, 1.0, 1.0) == (128, 136)
    assert mm.lds_block(lds, 8, 128, 32, 1.0, 1.0) == (128, 136)
    # every answer fits: block (pitch kc + 1) plus two streamed slices
    for step in (32, 64):
        for b in (8 * 1024, 64 * 1024, 160 * 1024, 1 << 20):
            for ratio in (0.25, 1.0, 2.0, 10.0):
                r, k = mm.lds_block(b, 8, 128, step, 1.0, ratio)
                if r:
                    assert r % step == 0 and k % 8 == 0
                    assert 8 * (r * (k + 1) + 2 * 8 * 130) <= b
                r0, k0 = mm.lds_block(b, 8, 0, step, 1.0, ratio)
                if r0:
                    assert r0 % step == 0 and k0 % 8 == 0 and 8 * r0 * (k0 + 1) <= b
                    # with the slices gone the block can only grow
                    assert 2.0 * r0 * k0 / (k0 + ratio * r0) >= 2.0 * r * k / (k + ratio * r) - 1e-9 if r else True
    # C dearer -> the block deepens (kc / rows grows), never the reverse
    ratios = [mm.lds_block(1 << 20, 8, 128, 64, 1.0, c) for c in (0.5, 1.0, 4.0, 16.0)]
    depth = [k / r for r, k in ratios]
    assert depth == sorted(depth)
    with pytest.raises(Exception):
        mm.lds_block(-1, 8, 128, 64, 1.0, 1.0)
    with pytest.raises(Exception):
        mm.lds_block(1 << 20, 8, -1, 64, 1.0, 1.0)
    for bad_step in (0, 8, 40):
        with pytest.raises(Exception):
            mm.lds_block(1 << 20, 8, 0, bad_step, 1.0, 1.0)


L2_HALF = 0.5 * 4 * 1024 * 1024   # bytes: the Sec. 4.1 share of one XCD's L2 a block may take


def resident(res, shape, b1, b2, beta=1.0):
    return mm.model_resident(res, *shape, b1, b2, beta)


def member_counts(name, shape):
    """Element transfers each member's model must equal, written as the Sec.
    2.2 resident counts (pinned above against the LRU simulation) of the
    member's own planned blocks at the L2 boundary, plus the member's rule
    for C: C is read and written once per pass over its k range."""
    m, n, k = shape
    p = mm.member_plan(name, m, n, k)
    cdiv = lambda a, b: -(-a // b)  # noqa: E731
    passes = cdiv(k, p["k_range"]) if k else 1
    c = {"c_reads": m * n * passes, "c_writes": m * n * passes}
    t, tm, tn = p["mt"], cdiv(m, p["mt"]), cdiv(n, p["nt"])
    if name == "C0":
        # the tiles one XCD runs at once: every 8th tile of a run of
        # 8 * per_xcd consecutive row-major tiles, i.e. (with at least 8 tile
        # columns, so every XCD gets whole column sets) a C block of `rows`
        # tile rows by tn / 8 (strided) tile columns: Resident C on it
        per_xcd = 64 if t == 128 else 128
        if tn < 8 or tn % 8:
            pytest.skip("C0's every-8th-tile pattern on a grid not 8 tiles wide has no Resident C block form")
        rows = min(cdiv(8 * per_xcd, tn), tm)
        ab = resident("C", shape, rows * t, (tn // 8) * t)
    elif name == "C3C0":
        ab = resident("C", shape, p["mc3"], p["nc3"])
    elif name == "B3C0":
        r = resident("B", shape, p["kc3"], t)
        ab = {"a_reads": r["a_reads"] if 8 * m * p["kc3"] > L2_HALF else m * k * min(tn, 8), "b_reads": r["b_reads"]}
    elif name == "A3C0":
        r = resident("A", shape, t, p["kc3"])
        ab = {"a_reads": r["a_reads"], "b_reads": r["b_reads"] if 8 * p["kc3"] * n > L2_HALF else k * n * min(tm, 8)}
    elif name == "A2C0":
        # Resident B (kc x nj tiles) inside every n_c panel
        panels = [min(p["nc"], n - j) for j in range(0, n, p["nc"])]
        ab = {"a_reads": m * k * sum(cdiv(w, p["nj"] * p["nt"]) for w in panels),
              "b_reads": resident("B", shape, p["kc"], p["nj"] * p["nt"])["b_reads"]}
    elif name == "B3A2C0":
        r = resident("B", shape, p["kc3"], p["nc3"])
        jc3 = cdiv(n, p["nc3"])
        ab = {"a_reads": r["a_reads"] if 8 * m * p["kc3"] > L2_HALF else m * k * min(jc3, 8), "b_reads": r["b_reads"]}
    elif name == "A3B2C0":
        r = resident("A", shape, p["mc3"], p["kc3"])
        ic3 = cdiv(m, p["mc3"])
        ab = {"a_reads": r["a_reads"], "b_reads": r["b_reads"] if 8 * p["kc3"] * n > L2_HALF else k * n * min(ic3, 8)}
    elif name == "C3A2C0":
        # the C block of one XCD round (32 workgroups, one per CU, or 64 of
        # the 32-row block on problems that leave CUs without a 64-row tile:
        # group_m x per_xcd / group_m tiles) is Resident C; its lines stay
        # for reads (C read once) but are written back after every pass
        per_xcd = 32 if p["mt"] == 64 else 64
        cols = min(tn, cdiv(per_xcd, p["group_m"]))
        rows = min(tm, cdiv(per_xcd, cols))
        ab = resident("C", shape, rows * p["mt"], cols * p["nt"])
        c = {"c_reads": m * n, "c_writes": m * n * passes}
    elif name == "C4A2C0":
        # Resident C at level 4 (mc4 x nc4) for B; inside a C block A is
        # streamed once per n-granule of nj tiles (Goto's loop)
        panels = [min(p["nc4"], n - j) for j in range(0, n, p["nc4"])]
        ab = {"a_reads": m * k * sum(cdiv(w, p["nj"] * p["nt"]) for w in panels),
              "b_reads": resident("C", shape, p["mc4"], p["nc4"])["b_reads"]}
    else:
        raise ValueError(name)
    return {**{x: float(v) for x, v in ab.items() if x in ("a_reads", "b_reads")}, **c}


@pytest.mark.parametrize("name", ["C0", "C3C0", "B3C0", "A3C0", "A2C0", "B3A2C0", "A3B2C0", "C3A2C0", "C4A2C0"])
@pytest.mark.parametrize("shape", [(8192, 8192, 8192), (16384, 16384, 256), (16384, 256, 16384), (1000, 3000, 700)])
def test_every_member_model_is_its_resident_counts(name, shape):
    got = mm.model_bytes(name, *shape, beta=1.0)
    want = member_counts(name, shape)
    for x in ("a_reads", "b_reads", "c_reads", "c_writes"):
        assert got[x] == pytest.approx(8 * want[x], rel=1e-12), (name, x, got[x], 8 * want[x])


def test_c3a2c0_block_fits_l2():
    """Sec. 4.1 at level 3 for C3A2C0: the C block is the 32 tiles of 64 x 128
    one XCD runs at once (one per CU; 2 MiB, half of its 4 MiB L2), and the chunk's guests
    beside it, the block's A rows (rows x kc) and B columns (kc x cols), take
    at most the other half, with kc as deep as that allows (in 32-deep
    slices, at most the 288 of the LDS block)."""
    half = 2 * 1024 * 1024
    # hand-derived: a 512 x 512 block leaves 2 MiB / (8 B * 1024) = 256 of
    # depth; a 1024 x 256 block (two tile columns) 2 MiB / (8 * 1280) = 204.8
    p = mm.member_plan("C3A2C0", 8192, 8192, 8192)
    assert (p["mc3"], p["nc3"], p["kc"], p["k_range"]) == (512, 512, 256, 256)
    p = mm.member_plan("C3A2C0", 16384, 256, 16384)
    assert (p["mc3"], p["nc3"], p["kc"]) == (1024, 256, 192)
    # 1024^3: 128 tiles of 64 rows would leave half the CUs idle, so 256 of
    # 32 rows, two per CU; an XCD round of 64 is a 16 x 4 block, 512 x 512
    p = mm.member_plan("C3A2C0", 1024, 1024, 1024)
    assert (p["mt"], p["mc3"], p["nc3"], p["kc"], p["workgroups"]) == (32, 512, 512, 256, 256)
    # at the switch: 16 x 16 tiles of 64 rows fill the 256 CUs; 16 x 15 do
    # not, and their 32-row launch (at most twice the tiles) still fits the
    # chip at once, two workgroups per CU
    assert mm.member_plan("C3A2C0", 1024, 2048, 512)["mt"] == 64
    for m, n in [(1024, 1920), (1000, 1920), (993, 1917), (64, 128 * 255)]:
        p = mm.member_plan("C3A2C0", m, n, 512)
        assert p["mt"] == 32 and p["workgroups"] <= 2 * 256, (m, n, p)
    for shape in [(8192, 8192, 8192), (16384, 16384, 256), (16384, 256, 16384), (1024, 1024, 1024),
                  (100, 3000, 500), (3000, 100, 500), (64, 128, 4096), (4096, 8192, 2048)]:
        p = mm.member_plan("C3A2C0", *shape)
        m, n, k = shape
        edge = p["mc3"] + p["nc3"]
        assert p["kc"] % 32 == 0 and 32 <= p["kc"] <= 288
        assert 8 * p["kc"] * edge <= half, shape
        assert p["kc"] == 288 or 8 * (p["kc"] + 32) * edge > half, shape
        # the block is the tiles one XCD holds at once, clipped to the matrix
        # one 64-row workgroup per CU, or, where those tiles would leave CUs
        # idle, two 32-row ones per CU
        fill = -(-m // 64) * -(-n // 128) >= 256
        t, per_xcd = (64, 32) if fill else (32, 64)
        assert p["mt"] == t, shape
        assert p["mc3"] % t == 0 and p["nc3"] % 128 == 0
        assert (p["mc3"] // t) * (p["nc3"] // 128) <= per_xcd
        assert p["mc3"] <= max(t, -(-m // t) * t) and p["nc3"] <= max(128, -(-n // 128) * 128)
        assert p["k_range"] == min(p["kc"], k)
