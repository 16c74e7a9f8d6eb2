"""Host-only checks of the C ABI: the library loads, exports every function
declared in include/momms.h, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest

import paper_1904_05717_amd as mm
from paper_1904_05717_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(momms_[a-z0-9_]+)\s*\(", text))
    return names


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "momms_gemm" in names and "momms_gemm_ex" in names
    lib = _lib.library()
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_member_names_round_trip():
    assert mm.MEMBER_NAMES[0] == "AUTO"
    for i, name in enumerate(mm.MEMBER_NAMES):
        assert _lib.momms_member_id(name.encode()) == i
    assert _lib.momms_member_id(b"X9Y9") == -1
    assert _lib.momms_member_name(99) is None
    assert {"C0", "A2C0", "B3A2C0", "A3B2C0", "C3A2C0", "C4A2C0"} <= set(mm.FAMILY)


NULL = None
BIG = 1 << 20  # a fake non-null device address; never dereferenced on these paths


@pytest.mark.parametrize("args,code", [
    ((-1, 4, 4, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 4, 1), -1),
    ((4, -1, 4, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 4, 1), -2),
    ((4, 4, -1, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 4, 1), -3),
    ((4, 4, 4, 1.0, NULL, 4, BIG, 4, 0.0, BIG, 4, 1), -5),
    ((4, 4, 8, 1.0, BIG, 7, BIG, 4, 0.0, BIG, 4, 1), -6),
    ((4, 4, 4, 1.0, BIG, 4, NULL, 4, 0.0, BIG, 4, 1), -7),
    ((4, 6, 4, 1.0, BIG, 4, BIG, 5, 0.0, BIG, 6, 1), -8),
    ((4, 4, 4, 1.0, BIG, 4, BIG, 4, 0.0, NULL, 4, 1), -10),
    ((4, 6, 4, 1.0, BIG, 4, BIG, 6, 0.0, BIG, 5, 1), -11),
    ((4, 4, 4, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 4, 10), -12),
    ((4, 4, 4, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 4, -1), -12),
])
def test_argument_errors_reported_before_launch(args, code):
    assert _lib.momms_gemm(*args) == code


def test_ex_argument_errors():
    f = _lib.momms_gemm_ex
    # transA: A stored k x m, lda >= m
    assert f(1, 0, 8, 4, 4, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 4, 1, None, 0, None) == -8
    # transB: B stored n x k, ldb >= k
    assert f(0, 1, 4, 4, 8, 1.0, BIG, 8, BIG, 4, 0.0, BIG, 4, 1, None, 0, None) == -10
    # misaligned workspace
    assert f(0, 0, 4, 4, 4, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 4, 5, BIG + 8, 1 << 30, None) == -15
    # workspace too small for a packing member
    need = _lib.momms_workspace_size(64, 64, 64, mm.MEMBERS["A2C0"])
    assert need > 0
    assert f(0, 0, 64, 64, 64, 1.0, BIG, 64, BIG, 64, 0.0, BIG, 64, mm.MEMBERS["A2C0"], BIG, need - 8,
             None) == -16


def test_static_argument_errors_and_quick_returns_before_any_device_call():
    f = _lib.momms_gemm_static
    goto = mm.MEMBERS["A2C0"]
    assert f(0, 0, -1, 4, 4, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 4, goto, None) == -3
    assert f(0, 0, 4, -1, 4, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 4, goto, None) == -4
    assert f(0, 0, 4, 4, -1, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 4, goto, None) == -5
    assert f(0, 0, 4, 4, 4, 1.0, NULL, 4, BIG, 4, 0.0, BIG, 4, goto, None) == -7
    assert f(1, 0, 8, 4, 4, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 4, goto, None) == -8
    assert f(0, 0, 4, 4, 4, 1.0, BIG, 4, NULL, 4, 0.0, BIG, 4, goto, None) == -9
    assert f(0, 1, 4, 4, 8, 1.0, BIG, 8, BIG, 4, 0.0, BIG, 4, goto, None) == -10
    assert f(0, 0, 4, 4, 4, 1.0, BIG, 4, BIG, 4, 0.0, NULL, 4, goto, None) == -12
    assert f(0, 0, 4, 4, 4, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 3, goto, None) == -13
    assert f(0, 0, 4, 4, 4, 1.0, BIG, 4, BIG, 4, 0.0, BIG, 4, 99, None) == -14
    # quick returns: nothing launched, no scratch looked up
    assert f(0, 0, 0, 4, 4, 1.0, NULL, 4, NULL, 4, 0.0, NULL, 4, goto, None) == 0
    assert f(0, 0, 4, 4, 4, 0.0, NULL, 4, NULL, 4, 1.0, BIG, 4, goto, None) == 0
    # the largest panel any shape asks of Goto (k_c x n_c) fits the static array
    biggest = _lib.momms_workspace_size(64, 1 << 20, 64, goto)
    gp = mm.member_plan("A2C0", 64, 1 << 20, 64)
    assert biggest == 8 * gp["kc"] * gp["nc"] and biggest <= 4 << 20
    assert _lib.momms_status_string(1005) != _lib.momms_status_string(1004)


def test_quick_returns_do_not_touch_the_device():
    # m == 0, n == 0, or (alpha == 0 or k == 0) with beta == 1: nothing is launched
    assert _lib.momms_gemm(0, 4, 4, 1.0, NULL, 4, NULL, 4, 0.0, NULL, 4, 1) == 0
    assert _lib.momms_gemm(4, 0, 4, 1.0, NULL, 4, NULL, 1, 0.0, NULL, 1, 1) == 0
    assert _lib.momms_gemm(4, 4, 4, 0.0, NULL, 4, NULL, 4, 1.0, BIG, 4, 1) == 0
    assert _lib.momms_gemm(4, 4, 0, 1.0, NULL, 1, NULL, 4, 1.0, BIG, 4, 1) == 0


def test_plans_are_consistent():
    for name in mm.FAMILY:
        p = mm.member_plan(name, 8192, 8192, 8192)
        assert p["member"] == mm.MEMBERS[name]
        assert p["mt"] in (32, 64, 128) and p["nt"] in (64, 128)
        assert p["launches"] >= 1 and p["workgroups"] >= 1
        assert 1 <= p["k_range"] <= 8192
    assert mm.member_plan("AUTO", 8192, 8192, 8192)["member"] == mm.MEMBERS[mm.select_member(8192, 8192, 8192)]
    assert _lib.momms_member_plan(1, -1, 4, 4, mm.MommsPlan()) == -2
    assert _lib.momms_member_plan(1, 4, 4, 4, None) == -5


def test_member_table_overrides_prior_and_validates():
    import ctypes
    from paper_1904_05717_amd import tuner
    arr = ctypes.c_int * 1
    lib = _lib
    assert lib.momms_set_member_table(65, arr(0), arr(0), arr(0), arr(1)) == -1
    assert lib.momms_set_member_table(1, arr(5), arr(5), arr(5), arr(0)) == -5     # AUTO is not a member
    assert lib.momms_set_member_table(1, arr(5), arr(5), arr(5), arr(10)) == -5
    try:
        assert lib.momms_set_member_table(1, arr(5), arr(5), arr(5), arr(mm.MEMBERS["B3C0"])) == 0
        assert mm.select_member(32, 32, 32) == "B3C0"        # bucket (5, 5, 5)
        assert mm.select_member(64, 64, 64) == mm.MEMBER_NAMES[_lib.momms_select_member_prior(64, 64, 64)]
    finally:
        lib.momms_set_member_table(0, None, None, None, None)
        tuner.install()
    assert mm.select_member(8192, 8192, 8192) in mm.FAMILY


def test_member_table_is_ignored_when_measured_on_other_sources(tmp_path):
    import json
    from paper_1904_05717_amd import tuner
    entry = {"shape": [32, 32, 32], "bucket": [5, 5, 5], "best": "B3C0", "ms": {}, "prior": "C0"}
    stale = tmp_path / "stale.json"
    stale.write_text(json.dumps({"source_sha": "0000000000000000", "entries": [entry]}))
    fresh = tmp_path / "fresh.json"
    fresh.write_text(json.dumps({"source_sha": tuner.source_sha(), "entries": [entry]}))
    try:
        assert tuner.install(str(stale)) == 0
        assert mm.select_member(32, 32, 32) == mm.MEMBER_NAMES[_lib.momms_select_member_prior(32, 32, 32)]
        assert tuner.install(str(fresh)) == 1
        assert mm.select_member(32, 32, 32) == "B3C0"
    finally:
        _lib.momms_set_member_table(0, None, None, None, None)
        tuner.install()


def test_committed_measurements_belong_to_the_committed_sources():
    # The member table and the traffic profiles carry a hash of the kernel
    # and planner sources (comments stripped) they were measured on; AUTO and
    # the bench line use them only while it matches.  A source change that is
    # not re-measured shows here rather than as a silent fallback.
    import json
    import os
    from paper_1904_05717_amd import tuner
    import bench
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    table = json.load(open(os.path.join(root, "paper_1904_05717_amd", "tuned_members.json")))
    assert table["source_sha"] == tuner.source_sha()
    for shape in ("8192", "16384x16384x256", "16384x256x16384"):
        prof = json.load(open(os.path.join(root, "profiles", f"traffic_f64_{shape}.json")))
        assert prof["kernel_source_sha"] == bench.kernel_source_sha(), shape


def test_int8_and_fp8_exactness_limits():
    # slices * k (k rounded up to 128) must stay <= 2^17 so every INT32 sum
    # is exact; beyond it the call is refused before any launch.
    f = mm._lib.momms_gemm_split
    big = 1 << 20
    assert f(0, 0, 4, 4, 16385, 1.0, big, 16385, big, 4, 0.0, big, 4, 8, 2, 0, big, 1 << 40, None) == 1002
    assert f(0, 0, 4, 4, 18689, 1.0, big, 18689, big, 4, 0.0, big, 4, 7, 2, 0, big, 1 << 40, None) == 1002
    assert mm.split_workspace_size(4, 4, 16384, 8, "int8") > 0
    assert mm.split_workspace_size(4, 4, 4, 3, "fp8") > 0
    assert mm.split_workspace_size(4, 4, 4, 12, "fp8") > 0
    assert mm.split_workspace_size(4, 4, 4, 13, "fp8") == 0
    assert mm.split_workspace_size(4, 4, 4, 10, "int8") > 0
    assert mm.split_workspace_size(4, 4, 4, 11, "int8") == 0
    assert mm.split_workspace_size(4, 4, 4, 9, "bf16") == 0
    assert f(0, 0, 4, 4, 4, 1.0, big, 4, big, 4, 0.0, big, 4, 11, 2, 0, big, 1 << 30, None) == -14
    # FP8: slices * k <= 2^16 keeps every FP32 sum of products up to 16^2 exact
    assert f(0, 0, 4, 4, 8193, 1.0, big, 8193, big, 4, 0.0, big, 4, 8, 1, 0, big, 1 << 40, None) == 1002
    assert f(0, 0, 4, 4, 8192, 1.0, big, 8192, big, 4, 0.0, big, 4, 8, 1, 0, big, 0, None) == -18
    assert f(0, 0, 4, 4, 4, 1.0, big, 4, big, 4, 0.0, big, 4, 13, 1, 0, big, 1 << 30, None) == -14
    assert f(0, 0, 4, 4, 4, 1.0, big, 4, big, 4, 0.0, big, 4, 9, 0, 0, big, 1 << 30, None) == -14


def test_tiled_sizes_and_argument_errors():
    # A: m x k in 128 x 16 tiles, B: k x n in 16 x 128 tiles, zero-padded.
    assert mm.tiled_size("A", 300, 20) == 8 * 384 * 32
    assert mm.tiled_size("B", 20, 300) == 8 * 32 * 384
    assert mm.tiled_size("A", 0, 0) == 8 * 128 * 16
    assert _lib.momms_tiled_size(ord("C"), 4, 4) == 0
    assert _lib.momms_tiled_size(ord("A"), -1, 4) == 0
    big = 1 << 20
    assert _lib.momms_to_tiled(ord("C"), 0, 4, 4, big, 4, big, None) == -1
    assert _lib.momms_to_tiled(ord("A"), 2, 4, 4, big, 4, big, None) == -2
    assert _lib.momms_to_tiled(ord("A"), 0, -1, 4, big, 4, big, None) == -3
    assert _lib.momms_to_tiled(ord("A"), 0, 4, 4, None, 4, big, None) == -5
    assert _lib.momms_to_tiled(ord("A"), 0, 4, 8, big, 4, big, None) == -6    # ldx < cols
    assert _lib.momms_to_tiled(ord("A"), 1, 8, 4, big, 4, big, None) == -6    # transposed: ldx < rows
    assert _lib.momms_from_tiled(ord("B"), 4, 8, big, big, 4, None) == -6
    f = _lib.momms_gemm_tiled
    assert f(-1, 4, 4, 1.0, big, big, 0.0, big, 4, 0, None) == -1
    assert f(4, 4, 4, 1.0, None, big, 0.0, big, 4, 0, None) == -5
    assert f(4, 4, 4, 1.0, big, big, 0.0, big, 3, 0, None) == -9
    assert f(4, 4, 4, 1.0, big, big, 0.0, big, 4, 99, None) == -10
    assert f(4, 4, 4, 1.0, big, big, 0.0, big, 4, -1, None) == -10


def test_syrk_argument_errors():
    f = _lib.momms_syrk
    big = 1 << 20
    assert f(ord("X"), 0, 4, 4, 1.0, big, 4, 0.0, big, 4, 0, None) == -1
    assert f(ord("L"), 2, 4, 4, 1.0, big, 4, 0.0, big, 4, 0, None) == -2
    assert f(ord("L"), 0, -1, 4, 1.0, big, 4, 0.0, big, 4, 0, None) == -3
    assert f(ord("L"), 0, 4, -1, 1.0, big, 4, 0.0, big, 4, 0, None) == -4
    assert f(ord("L"), 0, 4, 4, 1.0, None, 4, 0.0, big, 4, 0, None) == -6
    assert f(ord("L"), 0, 4, 8, 1.0, big, 4, 0.0, big, 4, 0, None) == -7     # lda < k
    assert f(ord("U"), 1, 8, 4, 1.0, big, 4, 0.0, big, 8, 0, None) == -7     # transposed: lda < n
    assert f(ord("L"), 0, 4, 4, 1.0, big, 4, 0.0, None, 4, 0, None) == -9
    assert f(ord("L"), 0, 4, 4, 1.0, big, 4, 0.0, big, 3, 0, None) == -10
    assert f(ord("L"), 0, 4, 4, 1.0, big, 4, 0.0, big, 4, mm.MEMBERS["A2C0"], None) == -11


def test_crt_moduli_and_bits_match_the_definition():
    # the library's host computation against the oracle's independent one
    from oracle import crt_emul as ce
    for N in range(1, 17):
        for k in (1, 2, 31, 32, 260, 8192, 131072, 10 ** 6):
            t, p = mm.crt_bits(k, N)
            assert t == ce.bits(k, N) and p == ce.moduli(N), (N, k)
    f = mm._lib.momms_crt_bits
    assert f(-1, 4, None) == -1 and f(4, 0, None) == -2 and f(4, 17, None) == -2


def test_crt_limits():
    f = mm._lib.momms_gemm_split
    big = 1 << 20
    # k rounded up to 128 above 2^17: refused; too few moduli for k: refused
    assert f(0, 0, 4, 4, 131073, 1.0, big, 131073, big, 4, 0.0, big, 4, 16, 3, 0, big, 1 << 40, None) == 1002
    assert f(0, 0, 4, 4, 8192, 1.0, big, 8192, big, 4, 0.0, big, 4, 2, 3, 0, big, 1 << 40, None) == 1002
    assert f(0, 0, 4, 4, 4, 1.0, big, 4, big, 4, 0.0, big, 4, 17, 3, 0, big, 1 << 30, None) == -14
    assert mm.split_workspace_size(4, 4, 4, 16, "crt") > 0
    assert mm.split_workspace_size(4, 4, 4, 17, "crt") == 0


def test_ooc_argument_errors_before_any_device_call():
    f = mm._lib.momms_gemm_ooc
    big = 1 << 20
    ws = mm.ooc_workspace_size(64, 64, 32)
    assert ws >= 8 * (2 * 64 * 64 + 2 * (64 * 32 + 32 * 64))
    args = [100, 90, 80, 1.0, big, 80, big, 90, 1.0, big, 90, 64, 64, 32, 0, 1 << 30, ws, None, None]

    def call(i, v):
        a = list(args)
        a[i] = v
        return f(*a)

    assert call(0, -1) == -1 and call(1, -1) == -2 and call(2, -1) == -3
    assert call(4, None) == -5 and call(5, 79) == -6 and call(6, None) == -7 and call(7, 89) == -8
    assert call(9, None) == -10 and call(10, 89) == -11
    assert call(11, 0) == -12 and call(12, 0) == -13 and call(13, 0) == -14
    assert call(14, 99) == -15 and call(15, (1 << 30) + 8) == -16 and call(16, ws - 1) == -17
    assert call(15, None) == -17
    assert mm.ooc_workspace_size(0, 4, 4) == 0
    # quick returns: empty C, or nothing to add with beta = 1
    assert call(0, 0) == 0
    a = list(args)
    a[3] = 0.0
    a[8] = 1.0
    assert f(*a) == 0


def test_trmm_trsm_argument_errors():
    big = 1 << 20
    trmm, trsm = mm._lib.momms_trmm, mm._lib.momms_trsm
    L, N = ord("L"), ord("N")
    assert trmm(ord("X"), 0, N, 4, 4, 1.0, big, 4, big, 4, big, 4, None) == -1
    assert trmm(L, 2, N, 4, 4, 1.0, big, 4, big, 4, big, 4, None) == -2
    assert trmm(L, 0, ord("Z"), 4, 4, 1.0, big, 4, big, 4, big, 4, None) == -3
    assert trmm(L, 0, N, -1, 4, 1.0, big, 4, big, 4, big, 4, None) == -4
    assert trmm(L, 0, N, 4, -1, 1.0, big, 4, big, 4, big, 4, None) == -5
    assert trmm(L, 0, N, 4, 4, 1.0, None, 4, big, 4, big, 4, None) == -7
    assert trmm(L, 0, N, 4, 4, 1.0, big, 3, big, 4, big, 4, None) == -8
    assert trmm(L, 0, N, 4, 4, 1.0, big, 4, None, 4, big, 4, None) == -9
    assert trmm(L, 0, N, 4, 4, 1.0, big, 4, big, 3, big, 4, None) == -10
    assert trmm(L, 0, N, 4, 4, 1.0, big, 4, big, 4, None, 4, None) == -11
    assert trmm(L, 0, N, 4, 4, 1.0, big, 4, big, 4, big, 3, None) == -12
    assert trsm(L, 0, N, 4, 4, 1.0, None, 4, big, 4, None) == -7
    assert trsm(L, 0, N, 4, 4, 1.0, big, 4, None, 4, None) == -9
    assert trsm(L, 0, N, 4, 4, 1.0, big, 4, big, 3, None) == -10
    assert trsm(L, 0, N, 0, 4, 1.0, None, 1, None, 4, None) == 0


def test_potrf_argument_errors():
    f = mm._lib.momms_potrf
    big = 1 << 20
    assert f(ord("L"), 4, big, 4, None, None) == -1
    assert f(ord("U"), -1, big, 4, None, None) == -2
    assert f(ord("U"), 4, None, 4, None, None) == -3
    assert f(ord("U"), 4, big, 3, None, None) == -4
    assert f(ord("U"), 0, None, 1, None, None) == 0


def test_lowbw_sizes_and_argument_errors():
    L = mm._lib
    assert L.momms_lowbw_round_bytes() == 16384
    assert L.momms_lowbw_min_bytes(4) == 4 * 16 * 16384 and L.momms_lowbw_min_bytes(0) == 0
    assert L.momms_lowbw_record_words(4) == 4 * 16 * 4 and L.momms_lowbw_record_words(-1) == 0
    f = L.momms_lowbw_start
    buf, flag, rec = 1 << 20, 1 << 21, 1 << 22    # never dereferenced: every case fails its checks first
    need = L.momms_lowbw_min_bytes(8)
    assert f(2, buf, need, 8, flag, rec, 1.0, 100, None) == -1
    assert f(0, None, need, 8, flag, rec, 1.0, 100, None) == -2
    assert f(0, buf + 8, need, 8, flag, rec, 1.0, 100, None) == -2
    assert f(0, buf, need - 1, 8, flag, rec, 1.0, 100, None) == -3
    assert f(0, buf, need, 0, flag, rec, 1.0, 100, None) == -4
    assert f(0, buf, need, 8, None, rec, 1.0, 100, None) == -5
    assert f(1, None, 0, 8, flag, None, 1.0, 100, None) == -6
    assert f(1, None, 0, 8, flag, rec, 0.0, 100, None) == -7
    assert f(1, None, 0, 8, flag, rec, 61.0, 100, None) == -7
    assert f(1, None, 0, 8, flag, rec, 1.0, 0, None) == -8
    assert L.momms_lowbw_stop(None, None, None) == -1
    assert L.momms_lowbw_stamp(None, None) == -1
    with pytest.raises(ValueError):
        mm.BandwidthHog(8, mode="copy")


def _batch_args(**over):
    one = (ctypes.c_int64 * 1)
    ptr = (ctypes.c_void_p * 1)
    dbl = (ctypes.c_double * 1)
    a = dict(out=ctypes.byref(ctypes.c_void_p()), count=1, m=one(4), n=one(4), k=one(4), A=ptr(BIG), lda=one(4),
             B=ptr(BIG), ldb=one(4), C=ptr(BIG), ldc=one(4), alpha=dbl(1.0), beta=dbl(0.0), member=None, tile=None)
    a.update(over)
    return list(a.values())


def test_batch_argument_errors_before_any_device_call():
    one = (ctypes.c_int64 * 1)
    f = _lib.momms_batch_create
    assert f(*_batch_args(out=None)) == -1
    assert f(*_batch_args(count=-1)) == -2
    assert f(*_batch_args(m=one(-1))) == -3
    assert f(*_batch_args(lda=one(3))) == -7
    assert f(*_batch_args(A=(ctypes.c_void_p * 1)(None))) == -6
    assert f(*_batch_args(ldc=one(3))) == -11
    # members: only the register-resident ones are batched
    for bad in (mm.MEMBERS["A2C0"], mm.MEMBERS["C4A2C0"], 10, -1):
        assert f(*_batch_args(member=(ctypes.c_int * 1)(bad))) == -14
    assert f(*_batch_args(tile=(ctypes.c_int * 1)(96))) == -15


def test_batch_alpha_zero_accepts_null_operands():
    # alpha == 0: A and B are never read, so NULL operands pass validation (the
    # call then reaches the device query, which fails here without a GPU)
    dbl = (ctypes.c_double * 1)
    null = (ctypes.c_void_p * 1)(None)
    st = _lib.momms_batch_create(*_batch_args(A=null, B=null, alpha=dbl(0.0), beta=dbl(2.0)))
    assert st not in (-6, -8), st
    st = _lib.momms_batch_create(*_batch_args(A=null, alpha=dbl(1.0)))
    assert st == -6


def test_batch_set_rates_validates():
    f = _lib.momms_batch_set_rates
    assert f(0.0, 1.0, 0.0) == -1
    assert f(1.0, -1.0, 0.0) == -2
    assert f(1.0, 1.0, float("nan")) == -3
    assert f(66e12 / 512.0, 0.55 * 66e12 / 512.0, 1.5e-6) == 0
    assert mm.batch_select_tile(2048, 2048, 2048) == 128
    assert mm.batch_select_tile(40, 40, 64) == 64
