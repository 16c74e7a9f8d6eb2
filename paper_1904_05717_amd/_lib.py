"""ctypes binding of libmomms.so: the C ABI declared in include/momms.h.

Functions keep the C names and argument order.  Pointers are passed as
integers (device addresses); nothing here computes any part of the product.
The library must have been built (``python -m paper_1904_05717_amd.build``);
importing this module without it raises ImportError.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmomms.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1904_05717_amd.build` "
        "(hipcc for gfx950); there is no CPU fallback")

_L = ctypes.CDLL(LIB_PATH)

i32, i64, dbl, vp, sz = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class MommsPlan(ctypes.Structure):
    _fields_ = [
        ("member", i32), ("kernel", i32), ("mt", i32), ("nt", i32), ("ks", i32),
        ("nj", i32), ("mi", i32), ("group_m", i32), ("xcd_aware", i32), ("pack", i32),
        ("kc", i64), ("mc3", i64), ("nc3", i64), ("kc3", i64), ("mc4", i64), ("nc4", i64),
        ("nc", i64), ("k_range", i64), ("launches", i64), ("workgroups", i64),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class MommsBytes(ctypes.Structure):
    _fields_ = [(name, dbl) for name in (
        "flops", "compulsory", "l2_read", "l2_write", "hbm_read", "hbm_write", "lds_fill", "pack",
        "a_reads", "b_reads", "c_reads", "c_writes")]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def _fn(name, res, args):
    f = getattr(_L, name)
    f.restype = res
    f.argtypes = args
    return f


momms_gemm = _fn("momms_gemm", i32, [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, i32])
momms_gemm_ex = _fn("momms_gemm_ex", i32, [i32, i32, i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, i32,
                                           vp, sz, vp])
momms_gemm_static = _fn("momms_gemm_static", i32, [i32, i32, i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64,
                                                   i32, vp])
momms_workspace_size = _fn("momms_workspace_size", sz, [i64, i64, i64, i32])
momms_set_stream = _fn("momms_set_stream", i32, [vp])
momms_num_members = _fn("momms_num_members", i32, [])
momms_member_name = _fn("momms_member_name", ctypes.c_char_p, [i32])
momms_member_id = _fn("momms_member_id", i32, [ctypes.c_char_p])
momms_member_plan = _fn("momms_member_plan", i32, [i32, i64, i64, i64, ctypes.POINTER(MommsPlan)])
momms_model_bytes = _fn("momms_model_bytes", i32, [i32, i64, i64, i64, dbl, i32, ctypes.POINTER(MommsBytes)])
momms_select_member = _fn("momms_select_member", i32, [i64, i64, i64])
momms_status_string = _fn("momms_status_string", ctypes.c_char_p, [i32])
momms_split_workspace_size = _fn("momms_split_workspace_size", sz, [i64, i64, i64, i32, i32])
momms_crt_bits = _fn("momms_crt_bits", i32, [i64, i32, ctypes.POINTER(i32)])
momms_gemm_split = _fn("momms_gemm_split", i32, [i32, i32, i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64,
                                                 i32, i32, i32, vp, sz, vp])

_pp = ctypes.POINTER(ctypes.c_void_p)
_pi64 = ctypes.POINTER(i64)
_pdbl = ctypes.POINTER(dbl)
_pi32 = ctypes.POINTER(i32)
momms_batch_create = _fn("momms_batch_create", i32, [_pp, i32, _pi64, _pi64, _pi64, _pp, _pi64, _pp, _pi64, _pp,
                                                     _pi64, _pdbl, _pdbl, _pi32, _pi32])
momms_batch_run = _fn("momms_batch_run", i32, [vp, vp])
momms_batch_info = _fn("momms_batch_info", i32, [vp, _pi64, _pi64, _pdbl, _pdbl, _pi32, _pi32, _pi32])
momms_batch_destroy = _fn("momms_batch_destroy", i32, [vp])
momms_batch_select_tile = _fn("momms_batch_select_tile", i32, [i64, i64, i64])
momms_batch_set_rates = _fn("momms_batch_set_rates", i32, [dbl, dbl, dbl])

momms_model_resident = _fn("momms_model_resident", i32, [i32, i64, i64, i64, i64, i64, dbl, _pdbl])
momms_balanced_block = _fn("momms_balanced_block", i32, [dbl, dbl, dbl, _pdbl, _pdbl])
momms_lds_block = _fn("momms_lds_block", i32, [dbl, i32, i32, i32, dbl, dbl, ctypes.POINTER(i32), ctypes.POINTER(i32)])

momms_set_member_table = _fn("momms_set_member_table", i32, [i32, _pi32, _pi32, _pi32, _pi32])
momms_select_member_prior = _fn("momms_select_member_prior", i32, [i64, i64, i64])

momms_tiled_size = _fn("momms_tiled_size", sz, [i32, i64, i64])
momms_to_tiled = _fn("momms_to_tiled", i32, [i32, i32, i64, i64, vp, i64, vp, vp])
momms_from_tiled = _fn("momms_from_tiled", i32, [i32, i64, i64, vp, vp, i64, vp])
momms_gemm_tiled = _fn("momms_gemm_tiled", i32, [i64, i64, i64, dbl, vp, vp, dbl, vp, i64, i32, vp])
momms_trmm = _fn("momms_trmm", i32, [i32, i32, i32, i64, i64, dbl, vp, i64, vp, i64, vp, i64, vp])
momms_trsm = _fn("momms_trsm", i32, [i32, i32, i32, i64, i64, dbl, vp, i64, vp, i64, vp])
momms_potrf = _fn("momms_potrf", i32, [i32, i64, vp, i64, vp, vp])
momms_ooc_workspace_size = _fn("momms_ooc_workspace_size", sz, [i64, i64, i64])
momms_gemm_ooc = _fn("momms_gemm_ooc", i32, [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, i64, i64, i64, i32,
                                             vp, sz, vp, vp])
momms_syrk = _fn("momms_syrk", i32, [i32, i32, i64, i64, dbl, vp, i64, dbl, vp, i64, i32, vp])
momms_lowbw_min_bytes = _fn("momms_lowbw_min_bytes", sz, [i32])
momms_lowbw_record_words = _fn("momms_lowbw_record_words", sz, [i32])
momms_lowbw_round_bytes = _fn("momms_lowbw_round_bytes", i64, [])
momms_lowbw_clock_hz = _fn("momms_lowbw_clock_hz", i64, [])
momms_lowbw_start = _fn("momms_lowbw_start", i32, [i32, vp, sz, i32, vp, vp, dbl, i64, vp])
momms_lowbw_stop = _fn("momms_lowbw_stop", i32, [vp, vp, vp])
momms_lowbw_stamp = _fn("momms_lowbw_stamp", i32, [vp, vp])

EXPORTS = [
    "momms_gemm", "momms_gemm_ex", "momms_workspace_size", "momms_set_stream", "momms_num_members",
    "momms_member_name", "momms_member_id", "momms_member_plan", "momms_model_bytes",
    "momms_select_member", "momms_status_string", "momms_split_workspace_size", "momms_gemm_split",
    "momms_batch_create", "momms_batch_run", "momms_batch_info", "momms_batch_destroy", "momms_batch_select_tile",
    "momms_batch_set_rates",
    "momms_model_resident", "momms_balanced_block", "momms_set_member_table", "momms_select_member_prior",
    "momms_tiled_size", "momms_to_tiled", "momms_from_tiled", "momms_gemm_tiled", "momms_syrk", "momms_crt_bits",
    "momms_ooc_workspace_size", "momms_gemm_ooc", "momms_trmm", "momms_trsm", "momms_potrf",
    "momms_lowbw_min_bytes", "momms_lowbw_record_words", "momms_lowbw_round_bytes", "momms_lowbw_clock_hz",
    "momms_lowbw_start", "momms_lowbw_stop", "momms_lowbw_stamp", "momms_lds_block", "momms_gemm_static",
]


def bind_optional(name, res, args):
    """Bind a symbol added by a later source file; None if absent."""
    if not hasattr(_L, name):
        return None
    return _fn(name, res, args)


def library():
    return _L
