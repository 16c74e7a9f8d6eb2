"""Differentiable GEMM: C = A @ B with a hand-written backward.

The backward products use the transposition flags of the C ABI instead of
materialised transposes:
    dA = dC @ B^T   -> gemm(dC, B, transB=True)   (m x n times (k x n)^T)
    dB = A^T @ dC   -> gemm(A, dC, transA=True)   ((m x k)^T times m x n)
Each product takes the family member the selector picks for its own shape
(the transposed shapes of a rectangular problem favour different members;
Sec. 2.3 of the MOMMS paper).

float64 tensors run on FP64 MFMA.  float32 tensors are widened exactly to
float64 and multiplied by the split-precision path with three BF16 slices
(8 + 9 + 9 bits, at least the 24-bit FP32 significand relative to each row and
column scale); the product is rounded once to float32.
"""
import torch

from . import gemm, gemm_split, select_member

FP32_SLICES = 3


def _mm(A, B, transA=False, transB=False):
    """op(A) @ op(B) for float64 (FP64 MFMA) or float32 (split path)."""
    m = A.shape[1] if transA else A.shape[0]
    k = A.shape[0] if transA else A.shape[1]
    n = B.shape[0] if transB else B.shape[1]
    if A.dtype == torch.float64:
        C = torch.empty((m, n), dtype=torch.float64, device=A.device)
        return gemm(A.contiguous(), B.contiguous(), C, 1.0, 0.0, member=select_member(m, n, k), transA=transA,
                    transB=transB)
    if A.dtype == torch.float32:
        A64 = A.contiguous().to(torch.float64)
        B64 = B.contiguous().to(torch.float64)
        C = torch.empty((m, n), dtype=torch.float64, device=A.device)
        gemm_split(A64, B64, C, 1.0, 0.0, slices=FP32_SLICES, transA=transA, transB=transB)
        return C.to(torch.float32)
    raise TypeError(f"MommsMatmul supports float64 and float32, got {A.dtype}")


class MommsMatmul(torch.autograd.Function):
    """C = A @ B for 2-D device tensors of one dtype (float64 or float32)."""

    @staticmethod
    def forward(ctx, A, B):
        if A.dim() != 2 or B.dim() != 2 or A.shape[1] != B.shape[0]:
            raise ValueError("MommsMatmul expects (m x k) @ (k x n)")
        if A.dtype != B.dtype:
            raise TypeError("A and B must have the same dtype")
        ctx.save_for_backward(A, B)
        return _mm(A, B)

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        dC = dC.to(A.dtype).contiguous()
        dA = dB = None
        if ctx.needs_input_grad[0]:
            dA = _mm(dC, B, transB=True)
        if ctx.needs_input_grad[1]:
            dB = _mm(A, dC, transA=True)
        return dA, dB


def matmul(A, B):
    return MommsMatmul.apply(A, B)
