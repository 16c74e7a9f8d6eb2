"""MOMMS family of FP64 matrix multiplications on MI355X (gfx950).

Thin PyTorch-facing layer over the C ABI of libmomms.so (include/momms.h):
it checks tensor dtype/device/layout, reads leading dimensions and the
current HIP stream, and passes device pointers through.  Every arithmetic
step runs in the library's HIP kernels; there is no CPU fallback.
"""
import ctypes

import torch

from . import _lib
from ._lib import MommsBytes, MommsPlan

MEMBER_NAMES = [_lib.momms_member_name(i).decode() for i in range(_lib.momms_num_members())]
MEMBERS = {name: i for i, name in enumerate(MEMBER_NAMES)}
FAMILY = [name for name in MEMBER_NAMES if name != "AUTO"]

# the measured member table written by tuner.sweep on the device, if present
from . import tuner as _tuner  # noqa: E402

_tuner.install()


class MommsError(RuntimeError):
    pass


def member_id(member):
    if isinstance(member, str):
        if member not in MEMBERS:
            raise ValueError(f"unknown family member {member!r}; known: {MEMBER_NAMES}")
        return MEMBERS[member]
    return int(member)


def check_status(status, fn="momms"):
    if status == 0:
        return
    msg = _lib.momms_status_string(status).decode()
    if status < 0:
        raise ValueError(f"{fn}: argument {-status} is invalid ({msg})")
    raise MommsError(f"{fn}: status {status}: {msg}")


def _ld(t, name):
    if t.dim() != 2:
        raise ValueError(f"{name} must be a 2-D tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    rows, cols = t.shape
    if t.is_contiguous():
        return max(1, cols)
    if t.stride(1) != 1 or t.stride(0) < max(1, cols):
        raise ValueError(f"{name} must be row-major (unit column stride)")
    return t.stride(0)


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def gemm(A, B, C=None, alpha=1.0, beta=0.0, member="AUTO", transA=False, transB=False, workspace=None,
         stream=None):
    """C := alpha * op(A) @ op(B) + beta * C on the device, in place; returns C.

    A, B, C are float64 device tensors in row-major layout (unit column
    stride, any leading dimension).  op(X) = X.T when trans is set.  With
    C None a new zero tensor is created (beta is then irrelevant).
    `workspace` (a uint8 device tensor of at least workspace_size bytes)
    enables packing for members that pack.
    """
    m, k = (A.shape[1], A.shape[0]) if transA else (A.shape[0], A.shape[1])
    kb, n = (B.shape[1], B.shape[0]) if transB else (B.shape[0], B.shape[1])
    if k != kb:
        raise ValueError(f"inner dimensions differ: {k} vs {kb}")
    lda, ldb = _ld(A, "A"), _ld(B, "B")
    if C is None:
        C = torch.zeros((m, n), dtype=torch.float64, device=A.device)
        beta = 0.0
    if tuple(C.shape) != (m, n):
        raise ValueError(f"C has shape {tuple(C.shape)}, expected {(m, n)}")
    ldc = _ld(C, "C")
    mid = member_id(member)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        if not workspace.is_cuda:
            raise ValueError("workspace must be a device tensor")
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    st = _lib.momms_gemm_ex(int(bool(transA)), int(bool(transB)), m, n, k, float(alpha), A.data_ptr(), lda,
                            B.data_ptr(), ldb, float(beta), C.data_ptr(), ldc, mid, ws_ptr, ws_bytes,
                            _stream_handle(stream))
    check_status(st, "momms_gemm_ex")
    return C


def workspace_size(m, n, k, member="AUTO"):
    return int(_lib.momms_workspace_size(m, n, k, member_id(member)))


def member_plan(member, m, n, k):
    p = MommsPlan()
    check_status(_lib.momms_member_plan(member_id(member), m, n, k, p), "momms_member_plan")
    return p.as_dict()


def model_bytes(member, m, n, k, beta=1.0, packed=False):
    b = MommsBytes()
    check_status(_lib.momms_model_bytes(member_id(member), m, n, k, float(beta), int(bool(packed)), b),
                 "momms_model_bytes")
    return b.as_dict()


def select_member(m, n, k):
    return MEMBER_NAMES[_lib.momms_select_member(m, n, k)]


SLICE_TYPES = {"bf16": 0, "fp8": 1, "int8": 2, "crt": 3}
ERR_INFEASIBLE = 1002   # MOMMS_ERR_INFEASIBLE


def crt_bits(k, moduli):
    """(t, moduli list) of the modular split product at inner dimension k, or
    (None, moduli) when `moduli` moduli are too few for k."""
    out = (ctypes.c_int32 * 16)()
    t = int(_lib.momms_crt_bits(int(k), int(moduli), out))
    if t == ERR_INFEASIBLE:
        return None, [int(out[i]) for i in range(int(moduli))]
    check_status(min(t, 0), "momms_crt_bits")
    return t, [int(out[i]) for i in range(int(moduli))]


def split_workspace_size(m, n, k, slices, slice_type="bf16"):
    return int(_lib.momms_split_workspace_size(m, n, k, slices, SLICE_TYPES[slice_type]))


def gemm_split(A, B, C=None, alpha=1.0, beta=0.0, slices=7, slice_type="bf16", member="AUTO", transA=False,
               transB=False, workspace=None, stream=None):
    """FP64-accurate C := alpha op(A) op(B) + beta C from BF16, FP8 or INT8
    slice products, or (slice_type "crt") from INT8 products of residues
    modulo `slices` moduli.

    Same conventions as gemm().  `workspace` (uint8 device tensor of at
    least split_workspace_size bytes) is allocated through torch when None.
    """
    m, k = (A.shape[1], A.shape[0]) if transA else (A.shape[0], A.shape[1])
    kb, n = (B.shape[1], B.shape[0]) if transB else (B.shape[0], B.shape[1])
    if k != kb:
        raise ValueError(f"inner dimensions differ: {k} vs {kb}")
    lda, ldb = _ld(A, "A"), _ld(B, "B")
    if C is None:
        C = torch.zeros((m, n), dtype=torch.float64, device=A.device)
        beta = 0.0
    if tuple(C.shape) != (m, n):
        raise ValueError(f"C has shape {tuple(C.shape)}, expected {(m, n)}")
    ldc = _ld(C, "C")
    if slice_type not in SLICE_TYPES:
        raise ValueError(f"unknown slice type {slice_type!r}")
    need = split_workspace_size(m, n, k, slices, slice_type)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=A.device)
    st = _lib.momms_gemm_split(int(bool(transA)), int(bool(transB)), m, n, k, float(alpha), A.data_ptr(), lda,
                               B.data_ptr(), ldb, float(beta), C.data_ptr(), ldc, int(slices),
                               SLICE_TYPES[slice_type], member_id(member), workspace.data_ptr(),
                               workspace.numel() * workspace.element_size(), _stream_handle(stream))
    check_status(st, "momms_gemm_split")
    return C


class BatchPlan:
    """Batched uneven GEMMs C_i := alpha_i A_i B_i + beta_i C_i (C ABI momms_batch_*).

    `problems` is a list of (A, B, C, alpha, beta) with float64 row-major
    device tensors.  `members` optionally fixes each problem's family member
    ("AUTO", "C0", "C3C0", "B3C0" or "A3C0", or their ids); `tiles` its
    register tile (64 or 128; 0 = the library's prior).  The plan keeps
    references to the tensors so their memory stays valid while it exists.
    """

    def __init__(self, problems, members=None, tiles=None):
        import ctypes
        self._keep = list(problems)
        n = len(problems)
        I64 = ctypes.c_int64 * n
        P = ctypes.c_void_p * n
        D = ctypes.c_double * n
        ms, ns, ks, lda, ldb, ldc = [], [], [], [], [], []
        pa, pb, pc, al, be = [], [], [], [], []
        for (A, B, C, alpha, beta) in problems:
            m, k = A.shape
            k2, nn = B.shape
            if k != k2 or tuple(C.shape) != (m, nn):
                raise ValueError("batch problem shapes do not match")
            ms.append(m); ns.append(nn); ks.append(k)
            lda.append(_ld(A, "A")); ldb.append(_ld(B, "B")); ldc.append(_ld(C, "C"))
            pa.append(A.data_ptr()); pb.append(B.data_ptr()); pc.append(C.data_ptr())
            al.append(float(alpha)); be.append(float(beta))
        ml = None
        if members is not None:
            if isinstance(members, (str, int)):
                members = [members] * n
            ml = (ctypes.c_int * n)(*[member_id(x) for x in members])
        tl = None
        if tiles is not None:
            if isinstance(tiles, int):
                tiles = [tiles] * n
            tl = (ctypes.c_int * n)(*[int(t) for t in tiles])
        self.count = n
        self._h = ctypes.c_void_p()
        st = _lib.momms_batch_create(ctypes.byref(self._h), n, I64(*ms), I64(*ns), I64(*ks), P(*pa), I64(*lda),
                                     P(*pb), I64(*ldb), P(*pc), I64(*ldc), D(*al), D(*be), ml, tl)
        check_status(st, "momms_batch_create")

    def run(self, stream=None):
        check_status(_lib.momms_batch_run(self._h, _stream_handle(stream)), "momms_batch_run")

    def info(self):
        import ctypes
        items, wgs = ctypes.c_int64(), ctypes.c_int64()
        flops, padded = ctypes.c_double(), ctypes.c_double()
        n = max(self.count, 1)
        members, tiles, chunks = (ctypes.c_int * n)(), (ctypes.c_int * n)(), (ctypes.c_int * n)()
        check_status(_lib.momms_batch_info(self._h, ctypes.byref(items), ctypes.byref(wgs), ctypes.byref(flops),
                                           ctypes.byref(padded), members, tiles, chunks), "momms_batch_info")
        return {"items": items.value, "workgroups": wgs.value, "flops": flops.value,
                "padded_flops": padded.value, "members": [MEMBER_NAMES[x] for x in list(members)[:self.count]],
                "tiles": list(tiles)[:self.count], "chunks": list(chunks)[:self.count]}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.momms_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_set_rates(rate128, rate64, item_seconds):
    """Per-slot rates (flop/s) of the two register tiles and the fixed time of
    one work item, used by the batch planner's prior from now on."""
    check_status(_lib.momms_batch_set_rates(float(rate128), float(rate64), float(item_seconds)),
                 "momms_batch_set_rates")


def batch_select_tile(m, n, k):
    return int(_lib.momms_batch_select_tile(m, n, k))


def tiled_size(operand, rows, cols):
    """Bytes of a tile-major operand ('A': rows x cols = m x k, 'B': k x n)."""
    return int(_lib.momms_tiled_size(ord(operand), rows, cols))


def to_tiled(X, operand, trans=False, out=None, stream=None):
    """Tile-major copy of op(X) (float64 device tensor; op(X) = X.T if trans).

    Returns a flat float64 device tensor holding the layout of
    momms_to_tiled (A: [m/128][k/16][128][16], B: [n/128][k][128], zero-padded).
    """
    if operand not in ("A", "B"):
        raise ValueError("operand must be 'A' or 'B'")
    ld = _ld(X, "X")
    rows, cols = (X.shape[1], X.shape[0]) if trans else (X.shape[0], X.shape[1])
    need = tiled_size(operand, rows, cols) // 8
    if out is None:
        out = torch.empty(need, dtype=torch.float64, device=X.device)
    elif out.numel() < need or out.dtype != torch.float64 or not out.is_cuda:
        raise ValueError(f"out must be a float64 device tensor of at least {need} elements")
    check_status(_lib.momms_to_tiled(ord(operand), int(bool(trans)), rows, cols, X.data_ptr(), ld, out.data_ptr(),
                                     _stream_handle(stream)), "momms_to_tiled")
    return out


def from_tiled(T, operand, rows, cols, stream=None):
    """The rows x cols row-major matrix held in a tile-major buffer."""
    X = torch.empty((rows, cols), dtype=torch.float64, device=T.device)
    check_status(_lib.momms_from_tiled(ord(operand), rows, cols, T.data_ptr(), X.data_ptr(), max(1, cols),
                                       _stream_handle(stream)), "momms_from_tiled")
    return X


def gemm_tiled(At, Bt, m, n, k, C=None, alpha=1.0, beta=0.0, member="AUTO", stream=None):
    """C := alpha * A @ B + beta * C with A, B in tile-major storage (to_tiled)."""
    for T, op, rows, cols in ((At, "A", m, k), (Bt, "B", k, n)):
        if not T.is_cuda or T.dtype != torch.float64 or T.numel() * 8 < tiled_size(op, rows, cols):
            raise ValueError(f"{op} must be a tile-major float64 device buffer for {rows} x {cols}")
    if C is None:
        C = torch.zeros((m, n), dtype=torch.float64, device=At.device)
        beta = 0.0
    if tuple(C.shape) != (m, n):
        raise ValueError(f"C has shape {tuple(C.shape)}, expected {(m, n)}")
    ldc = _ld(C, "C")
    st = _lib.momms_gemm_tiled(m, n, k, float(alpha), At.data_ptr(), Bt.data_ptr(), float(beta), C.data_ptr(), ldc,
                               member_id(member), _stream_handle(stream))
    check_status(st, "momms_gemm_tiled")
    return C


def syrk(A, C=None, alpha=1.0, beta=0.0, uplo="L", trans=False, member="AUTO", stream=None):
    """C := alpha * op(A) @ op(A).T + beta * C on one triangle ('L' or 'U') of C.

    op(A) = A (n x k) or A.T when trans.  The other triangle of C is left
    untouched; a new C (None) starts from zeros.
    """
    n, k = (A.shape[1], A.shape[0]) if trans else (A.shape[0], A.shape[1])
    lda = _ld(A, "A")
    if C is None:
        C = torch.zeros((n, n), dtype=torch.float64, device=A.device)
        beta = 0.0
    if tuple(C.shape) != (n, n):
        raise ValueError(f"C has shape {tuple(C.shape)}, expected {(n, n)}")
    if uplo not in ("L", "U"):
        raise ValueError("uplo must be 'L' or 'U'")
    ldc = _ld(C, "C")
    st = _lib.momms_syrk(ord(uplo), int(bool(trans)), n, k, float(alpha), A.data_ptr(), lda, float(beta),
                         C.data_ptr(), ldc, member_id(member), _stream_handle(stream))
    check_status(st, "momms_syrk")
    return C


def trmm(A, B, C=None, alpha=1.0, uplo="L", trans=False, diag="N", stream=None):
    """C := alpha * op(T) @ B with T the uplo triangle of A (unit diagonal when
    diag == 'U'); out of place, returns C."""
    m, n = B.shape
    if tuple(A.shape) != (m, m):
        raise ValueError(f"A has shape {tuple(A.shape)}, expected {(m, m)}")
    if C is None:
        C = torch.empty((m, n), dtype=torch.float64, device=B.device)
    if tuple(C.shape) != (m, n):
        raise ValueError(f"C has shape {tuple(C.shape)}, expected {(m, n)}")
    if uplo not in ("L", "U") or diag not in ("N", "U"):
        raise ValueError("uplo must be 'L' or 'U' and diag 'N' or 'U'")
    st = _lib.momms_trmm(ord(uplo), int(bool(trans)), ord(diag), m, n, float(alpha), A.data_ptr(), _ld(A, "A"),
                         B.data_ptr(), _ld(B, "B"), C.data_ptr(), _ld(C, "C"), _stream_handle(stream))
    check_status(st, "momms_trmm")
    return C


def trsm(A, B, alpha=1.0, uplo="L", trans=False, diag="N", stream=None):
    """Solves op(T) X = alpha B in place (B becomes X); returns B."""
    m, n = B.shape
    if tuple(A.shape) != (m, m):
        raise ValueError(f"A has shape {tuple(A.shape)}, expected {(m, m)}")
    if uplo not in ("L", "U") or diag not in ("N", "U"):
        raise ValueError("uplo must be 'L' or 'U' and diag 'N' or 'U'")
    st = _lib.momms_trsm(ord(uplo), int(bool(trans)), ord(diag), m, n, float(alpha), A.data_ptr(), _ld(A, "A"),
                         B.data_ptr(), _ld(B, "B"), _stream_handle(stream))
    check_status(st, "momms_trsm")
    return B


def potrf(A, uplo="U", stream=None):
    """Cholesky A = U^T U in place on the upper triangle of the SPD device
    matrix A (the strictly lower triangle is not touched).  Returns info: 0,
    or the 1-based row of the first pivot that is not positive.  Waits for
    the stream to read info."""
    n = A.shape[0]
    if tuple(A.shape) != (n, n):
        raise ValueError("A must be square")
    if uplo != "U":
        raise ValueError("uplo must be 'U'")
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    st = stream if stream is not None else torch.cuda.current_stream(A.device)
    rc = _lib.momms_potrf(ord(uplo), n, A.data_ptr(), _ld(A, "A"), info.data_ptr(), st.cuda_stream)
    check_status(rc, "momms_potrf")
    st.synchronize()
    return int(info.item())


def _ld_host(t, name):
    if t.dim() != 2 or t.dtype != torch.float64 or t.is_cuda:
        raise ValueError(f"{name} must be a 2-D float64 host tensor")
    if t.is_contiguous():
        return max(1, t.shape[1])
    if t.stride(1) != 1 or t.stride(0) < max(1, t.shape[1]):
        raise ValueError(f"{name} must be row-major with unit column stride")
    return max(1, t.stride(0))


def ooc_workspace_size(mb, nb, kb):
    return int(_lib.momms_ooc_workspace_size(int(mb), int(nb), int(kb)))


def gemm_ooc(A, B, C, alpha=1.0, beta=0.0, block=(8192, 8192, 2048), member="AUTO", workspace=None,
             stream=None, copy_stream=None, device="cuda:0"):
    """Out-of-core C := alpha * A @ B + beta * C with A, B, C float64 HOST
    tensors (pin_memory() ones let copies overlap the products).  C is
    processed in mb x nb blocks resident in device memory while panels of A
    and B stream in; block = (mb, nb, kb).  Waits for the result before
    returning."""
    m, k = A.shape
    kb_, n = B.shape
    if k != kb_:
        raise ValueError(f"inner dimensions differ: {k} vs {kb_}")
    if tuple(C.shape) != (m, n):
        raise ValueError(f"C has shape {tuple(C.shape)}, expected {(m, n)}")
    lda, ldb, ldc = _ld_host(A, "A"), _ld_host(B, "B"), _ld_host(C, "C")
    mb, nb, kb = (int(x) for x in block)
    need = ooc_workspace_size(mb, nb, kb)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=device)
    if stream is None:
        stream = torch.cuda.current_stream(device)
    if copy_stream is None:
        copy_stream = torch.cuda.Stream(device=device)
    st = _lib.momms_gemm_ooc(m, n, k, float(alpha), A.data_ptr(), lda, B.data_ptr(), ldb, float(beta), C.data_ptr(),
                             ldc, mb, nb, kb, member_id(member), workspace.data_ptr(),
                             workspace.numel() * workspace.element_size(), stream.cuda_stream,
                             copy_stream.cuda_stream)
    check_status(st, "momms_gemm_ooc")
    stream.synchronize()
    return C


def model_resident(resident, m, n, k, b1, b2, beta=1.0):
    """Sec. 2.2 transfer counts: {a_reads, b_reads, c_reads, c_writes} in elements."""
    import ctypes
    out = (ctypes.c_double * 4)()
    check_status(_lib.momms_model_resident(ord(resident), m, n, k, b1, b2, float(beta), out),
                 "momms_model_resident")
    return {"a_reads": out[0], "b_reads": out[1], "c_reads": out[2], "c_writes": out[3]}


def balanced_block(M, beta_b, beta_c):
    import ctypes
    mc, kc = ctypes.c_double(), ctypes.c_double()
    check_status(_lib.momms_balanced_block(float(M), float(beta_b), float(beta_c), ctypes.byref(mc),
                                           ctypes.byref(kc)), "momms_balanced_block")
    return mc.value, kc.value


def lds_block(lds_bytes, slice_depth, tile_other, row_step, beta_stream, beta_c):
    """The planner's level-2 block solver: (rows, kc) of the resident block."""
    import ctypes
    rows, kc = ctypes.c_int(), ctypes.c_int()
    check_status(_lib.momms_lds_block(float(lds_bytes), int(slice_depth), int(tile_other), int(row_step),
                                      float(beta_stream), float(beta_c), ctypes.byref(rows), ctypes.byref(kc)),
                 "momms_lds_block")
    return rows.value, kc.value


class BandwidthHog:
    """The streaming kernel of the low-bandwidth experiments (Sec. 5), on a stream of its own.

    `workgroups` compute units are taken whole (all of their LDS).  mode
    "stream" reads a device buffer of `nbytes` with non-temporal loads, taking
    HBM bandwidth from a product run beside it; mode "sleep" takes the same
    compute units and reads nothing, the control.  Use:

        s = hog.concurrent_stream()
        hog.start(); hog.mark(s); <product on stream s>; hog.stop(s); hog.report()

    start() waits on the host for the hog stream's earlier work; the waves
    leave at stop(), after max_seconds, or after max_rounds rounds.
    """

    def __init__(self, workgroups, mode="stream", nbytes=4 << 30, device="cuda:0", stream=None):
        if mode not in ("stream", "sleep"):
            raise ValueError("mode is 'stream' or 'sleep'")
        self.workgroups, self.mode = int(workgroups), mode
        self.device = torch.device(device)
        need = _lib.momms_lowbw_min_bytes(self.workgroups)
        if need == 0:
            raise ValueError("workgroups must be positive")
        self.buf = None
        if mode == "stream":
            if nbytes < need:
                raise ValueError(f"the buffer needs at least {need} bytes for {workgroups} workgroups")
            self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.flag = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.rec = torch.zeros(_lib.momms_lowbw_record_words(self.workgroups), dtype=torch.int64, device=self.device)
        self.stamps = torch.zeros(2, dtype=torch.int64, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.max_seconds = None

    def concurrent_stream(self, tries=8, wait_s=0.05):
        """A new stream whose work runs while this hog's stream is busy.

        HIP multiplexes streams onto a few hardware queues, and two streams on
        one queue run one after the other: a product enqueued there would start
        only after the hog had ended.  Each candidate stream is tried beside a
        short sleeping hog (one workgroup, at most 0.25 s): it is kept if a
        stamp enqueued on it completes while that hog still runs."""
        import time
        for _ in range(tries):
            cand = torch.cuda.Stream(device=self.device)
            torch.cuda.current_stream(self.device).synchronize()
            check_status(_lib.momms_lowbw_start(1, None, 0, 1, self.flag.data_ptr(), self.rec.data_ptr(), 0.25,
                                                1 << 40, self.stream.cuda_stream), "momms_lowbw_start")
            check_status(_lib.momms_lowbw_stamp(self.stamps.data_ptr(), cand.cuda_stream), "momms_lowbw_stamp")
            ev = torch.cuda.Event()
            ev.record(cand)
            t0, ok = time.perf_counter(), False
            while time.perf_counter() - t0 < wait_s:
                if ev.query():
                    ok = True
                    break
                time.sleep(0.0005)
            check_status(_lib.momms_lowbw_stop(self.flag.data_ptr(), None, cand.cuda_stream), "momms_lowbw_stop")
            self.stream.synchronize()
            cand.synchronize()
            if ok:
                return cand
        raise MommsError("no stream found whose work runs beside the hog's stream")

    def start(self, max_seconds=5.0, max_rounds=1 << 40):
        buf_ptr = self.buf.data_ptr() if self.buf is not None else None
        nbytes = self.buf.numel() if self.buf is not None else 0
        self.rec.zero_()
        self.stamps.zero_()
        torch.cuda.current_stream(self.device).synchronize()   # the clears above, before the hog stream starts
        self.max_seconds = float(max_seconds)
        check_status(_lib.momms_lowbw_start(0 if self.mode == "stream" else 1, buf_ptr, nbytes, self.workgroups,
                                            self.flag.data_ptr(), self.rec.data_ptr(), self.max_seconds,
                                            int(max_rounds), self.stream.cuda_stream), "momms_lowbw_start")

    def mark(self, stream=None):
        """Stamp the wall clock on `stream` where the product starts."""
        check_status(_lib.momms_lowbw_stamp(self.stamps.data_ptr(), _stream_handle(stream)), "momms_lowbw_stamp")

    def stop(self, stream=None):
        """Enqueue the stop on `stream` (after the product)."""
        check_status(_lib.momms_lowbw_stop(self.flag.data_ptr(), self.stamps.data_ptr() + 8, _stream_handle(stream)),
                     "momms_lowbw_stop")

    def report(self):
        """Wait for the hog; its rounds, bytes, rate and whether it covered mark() .. stop()."""
        self.stream.synchronize()
        torch.cuda.synchronize(self.device)
        hz = float(_lib.momms_lowbw_clock_hz())
        rec = self.rec.view(-1, 4).cpu()
        mark, stop = (int(x) for x in self.stamps.cpu())
        rounds, t0, t1 = rec[:, 0], rec[:, 2], rec[:, 3]
        nbytes = int(rounds.sum()) * _lib.momms_lowbw_round_bytes() if self.mode == "stream" else 0
        span = (int(t1.max()) - int(t0.min())) / hz
        return {
            "mode": self.mode, "workgroups": self.workgroups, "waves": int(rec.shape[0]),
            "mark": mark, "stop": stop, "start_first": int(t0.min()), "start_last": int(t0.max()),
            "end_first": int(t1.min()), "end_last": int(t1.max()), "clock_hz": hz,
            "bytes": nbytes, "seconds": span, "GBps": nbytes / span / 1e9 if span > 0 else 0.0,
            "min_rounds": int(rounds.min()),
            "covered": bool(mark > 0 and stop > 0 and int(t0.max()) <= mark and int(t1.min()) >= stop),
            "timed_out": bool((t1 - t0).max() / hz >= 0.99 * self.max_seconds),
        }
