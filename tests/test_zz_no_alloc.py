"""The allocation-free entry point momms_gemm_static, through the C ABI.

It must give, bit for bit, what momms_gemm_ex gives with a caller-provided
workspace for the same member, stream and operands (the same kernels run; only
the packed panel's memory differs), and stay within the error bound against
the oracle.  Two calls in a row, the second smaller, show that what the first
call left in the shared array does not leak into the second.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

mm = pytest.importorskip("paper_1904_05717_amd")
from paper_1904_05717_amd import _lib  # noqa: E402

DEV = "cuda:0"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def call_static(A, B, C, alpha, beta, member, transA=False, transB=False):
    m, n = C.shape
    k = A.shape[0] if transA else A.shape[1]
    Ad, Bd, Cd = dev(A), dev(B), dev(C)
    st = torch.cuda.current_stream().cuda_stream
    r = _lib.momms_gemm_static(int(transA), int(transB), m, n, k, alpha, ptr(Ad), Ad.shape[1], ptr(Bd),
                               Bd.shape[1], beta, ptr(Cd), n, mm.member_id(member), ctypes.c_void_p(st))
    assert r == 0, _lib.momms_status_string(r)
    torch.cuda.synchronize()
    return Cd.cpu().numpy()


def call_ex(A, B, C, alpha, beta, member, transA=False, transB=False):
    m, n = C.shape
    k = A.shape[0] if transA else A.shape[1]
    Ad, Bd, Cd = dev(A), dev(B), dev(C)
    mid = mm.member_id(member)
    need = _lib.momms_workspace_size(m, n, k, mid)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=DEV)
    assert ws.data_ptr() % 256 == 0
    st = torch.cuda.current_stream().cuda_stream
    r = _lib.momms_gemm_ex(int(transA), int(transB), m, n, k, alpha, ptr(Ad), Ad.shape[1], ptr(Bd), Bd.shape[1],
                           beta, ptr(Cd), n, mid, ptr(ws), need, ctypes.c_void_p(st))
    assert r == 0, _lib.momms_status_string(r)
    torch.cuda.synchronize()
    return Cd.cpu().numpy()


def operands(m, n, k, transA=False, transB=False, seed_shift=0):
    A, B, C = workloads.gemm_operands(m, n, k)
    if seed_shift:
        A, B, C = -A, B[::-1].copy(), C[::-1].copy()
    if transA:
        A = np.ascontiguousarray(A.T)
    if transB:
        B = np.ascontiguousarray(B.T)
    return A, B, C


def check_pair(shape, member, transA=False, transB=False, seed_shift=0):
    m, n, k = shape
    A, B, C = operands(m, n, k, transA, transB, seed_shift)
    got = call_static(A, B, C, 1.25, -0.5, member, transA, transB)
    ref = call_ex(A, B, C, 1.25, -0.5, member, transA, transB)
    np.testing.assert_array_equal(got, ref)
    Aop = A.T if transA else A
    Bop = B.T if transB else B
    want = oracle.gemm(np.ascontiguousarray(Aop), np.ascontiguousarray(Bop), C, 1.25, -0.5)
    tol = oracle.error_bound(np.ascontiguousarray(Aop), np.ascontiguousarray(Bop), C, 1.25, -0.5, k=k)
    assert (np.abs(got - want) <= tol).all()


def test_goto_twice_second_smaller():
    # first call: two n_c panels (the whole 4 MiB array), ragged k; second:
    # a smaller problem whose panel covers only part of what the first wrote
    print("momms_gemm_static A2C0 (700, 4500, 300) then (130, 260, 70)", flush=True)
    check_pair((700, 4500, 300), "A2C0")
    check_pair((130, 260, 70), "A2C0", seed_shift=1)


def test_goto_transposed_twice():
    print("momms_gemm_static A2C0 transB (384, 1000, 257) then transA (96, 200, 129)", flush=True)
    check_pair((384, 1000, 257), "A2C0", transB=True)
    check_pair((96, 200, 129), "A2C0", transA=True, seed_shift=1)


@pytest.mark.parametrize("member", ["AUTO", "C3C0", "B3A2C0"])
def test_members_without_scratch(member):
    print(f"momms_gemm_static {member} (300, 200, 150) then (70, 50, 40)", flush=True)
    check_pair((300, 200, 150), member)
    check_pair((70, 50, 40), member, seed_shift=1)


def test_alpha_zero_and_quick_return_use_no_operands():
    m, n = 64, 48
    C = workloads.uniform((m, n), workloads.SEED_C)
    Cd = dev(C)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    r = _lib.momms_gemm_static(0, 0, m, n, 32, 0.0, None, 32, None, n, 2.0, ptr(Cd), n, mm.member_id("A2C0"), st)
    assert r == 0
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Cd.cpu().numpy(), 2.0 * C)
