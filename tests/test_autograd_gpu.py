"""The hand-written backward of MommsMatmul against finite differences,
torch.autograd.gradcheck and the oracle's gradients."""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu
mm = pytest.importorskip("paper_1904_05717_amd")
from paper_1904_05717_amd.autograd import MommsMatmul, matmul  # noqa: E402

DEV = "cuda:0"


def test_gradcheck_fp64_64():
    A = torch.from_numpy(workloads.uniform((64, 64), 1)).to(DEV).requires_grad_()
    B = torch.from_numpy(workloads.uniform((64, 64), 2)).to(DEV).requires_grad_()
    assert torch.autograd.gradcheck(MommsMatmul.apply, (A, B), eps=1e-6, atol=1e-9, rtol=1e-7)


def test_central_differences_64():
    # C is bilinear, so a central difference has no truncation error: only
    # rounding of order u |C| / h remains.
    m = n = k = 64
    A = torch.from_numpy(workloads.uniform((m, k), 3)).to(DEV)
    B = torch.from_numpy(workloads.uniform((k, n), 4)).to(DEV)
    W = torch.from_numpy(workloads.normal((m, n), workloads.SEED_DC)).to(DEV)   # upstream dC
    dA_dir = torch.from_numpy(workloads.uniform((m, k), 5)).to(DEV)
    dB_dir = torch.from_numpy(workloads.uniform((k, n), 6)).to(DEV)
    Ar, Br = A.clone().requires_grad_(), B.clone().requires_grad_()
    (matmul(Ar, Br) * W).sum().backward()
    h = 2.0 ** -10

    def f(a, b):
        return float((matmul(a, b) * W).sum())

    fd_a = (f(A + h * dA_dir, B) - f(A - h * dA_dir, B)) / (2 * h)
    fd_b = (f(A, B + h * dB_dir) - f(A, B - h * dB_dir)) / (2 * h)
    an_a = float((Ar.grad * dA_dir).sum())
    an_b = float((Br.grad * dB_dir).sum())
    assert abs(fd_a - an_a) <= 1e-9 * max(1.0, abs(an_a))
    assert abs(fd_b - an_b) <= 1e-9 * max(1.0, abs(an_b))


@pytest.mark.parametrize("shape", [(96, 80, 112), (200, 64, 300)])
def test_gradients_against_oracle_fp64(shape):
    m, k, n = shape
    A = workloads.uniform((m, k), 7)
    B = workloads.uniform((k, n), 8)
    dC = workloads.normal((m, n), workloads.SEED_DC)
    Ad = torch.from_numpy(A).to(DEV).requires_grad_()
    Bd = torch.from_numpy(B).to(DEV).requires_grad_()
    C = matmul(Ad, Bd)
    C.backward(torch.from_numpy(dC).to(DEV))
    np.testing.assert_array_less(np.abs(C.detach().cpu().numpy() - oracle.gemm(A, B)),
                                 oracle.error_bound(A, B) + 1e-300)
    dA_o = oracle.gemm(dC, B.T.copy())
    dB_o = oracle.gemm(A.T.copy(), dC)
    assert np.all(np.abs(Ad.grad.cpu().numpy() - dA_o) <= oracle.error_bound(dC, B.T))
    assert np.all(np.abs(Bd.grad.cpu().numpy() - dB_o) <= oracle.error_bound(A.T, dC))


def test_fp32_split_forward_and_backward():
    # FP32 via three BF16 slices: compare with the oracle on the FP32 inputs,
    # tolerance 2 (k+2) 2^-24 |A||B| (the FP32 analogue of the FP64 bound).
    m, k, n = 128, 96, 80
    A = workloads.uniform((m, k), 9).astype(np.float32)
    B = workloads.uniform((k, n), 10).astype(np.float32)
    dC = workloads.normal((m, n), workloads.SEED_DC).astype(np.float32)
    Ad = torch.from_numpy(A).to(DEV).requires_grad_()
    Bd = torch.from_numpy(B).to(DEV).requires_grad_()
    C = matmul(Ad, Bd)
    assert C.dtype == torch.float32
    C.backward(torch.from_numpy(dC).to(DEV))
    A64, B64, dC64 = A.astype(np.float64), B.astype(np.float64), dC.astype(np.float64)

    def check(got, X, Y):
        want = oracle.gemm(X, Y)
        tol = 2.0 * (X.shape[1] + 2) * 2.0 ** -24 * (np.abs(X) @ np.abs(Y))
        assert np.all(np.abs(got.astype(np.float64) - want) <= tol)

    check(C.detach().cpu().numpy(), A64, B64)
    check(Ad.grad.cpu().numpy(), dC64, B64.T.copy())
    check(Bd.grad.cpu().numpy(), A64.T.copy(), dC64)


def test_config5_shapes_sampled():
    # forward m=4096, k=8192, n=2048 in FP64; dC ~ N(0,1); sampled gradient entries
    m, k, n = 4096, 8192, 2048
    A = workloads.uniform((m, k), workloads.SEED_A)
    B = workloads.uniform((k, n), workloads.SEED_B)
    dC = workloads.normal((m, n), workloads.SEED_DC)
    Ad = torch.from_numpy(A).to(DEV).requires_grad_()
    Bd = torch.from_numpy(B).to(DEV).requires_grad_()
    C = matmul(Ad, Bd)
    C.backward(torch.from_numpy(dC).to(DEV))
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(11))
    r = rng.integers(0, m, 200)
    c = rng.integers(0, k, 200)
    dA_o = oracle.gemm_entries(dC, B.T.copy(), r, c)
    got = Ad.grad.cpu().numpy()[r, c]
    absab = np.einsum("ij,ji->i", np.abs(dC[r]), np.abs(B.T[:, c]))
    assert np.all(np.abs(got - dA_o) <= 2 * (n + 2) * 2.0 ** -53 * absab)
    r2 = rng.integers(0, k, 200)
    c2 = rng.integers(0, n, 200)
    AT = A.T.copy()
    dB_o = oracle.gemm_entries(AT, dC, r2, c2)
    got2 = Bd.grad.cpu().numpy()[r2, c2]
    absab2 = np.einsum("ij,ji->i", np.abs(AT[r2]), np.abs(dC[:, c2]))
    assert np.all(np.abs(got2 - dB_o) <= 2 * (m + 2) * 2.0 ** -53 * absab2)


def test_config5_fp32_split_sampled():
    # The FP32 form (three BF16 slices) at the config-5 shape: forward
    # m=4096, k=8192, n=2048 and both gradients on sampled entries plus the
    # first and last rows and columns, against the oracle on the FP32 inputs
    # widened exactly to FP64, within 2 (k+2) 2^-24 (|X||Y|)_ij.
    m, k, n = 4096, 8192, 2048
    A = workloads.uniform((m, k), workloads.SEED_A).astype(np.float32)
    B = workloads.uniform((k, n), workloads.SEED_B).astype(np.float32)
    dC = workloads.normal((m, n), workloads.SEED_DC).astype(np.float32)
    Ad = torch.from_numpy(A).to(DEV).requires_grad_()
    Bd = torch.from_numpy(B).to(DEV).requires_grad_()
    C = matmul(Ad, Bd)
    assert C.dtype == torch.float32
    C.backward(torch.from_numpy(dC).to(DEV))
    torch.cuda.synchronize()
    A64, B64, dC64 = A.astype(np.float64), B.astype(np.float64), dC.astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(12))

    def check(got, X, Y, what):
        rows_, cols_ = X.shape[0], Y.shape[1]
        r = np.concatenate([rng.integers(0, rows_, 150), [0, 0, rows_ - 1, rows_ - 1]])
        c = np.concatenate([rng.integers(0, cols_, 150), [0, cols_ - 1, 0, cols_ - 1]])
        want = oracle.gemm_entries(X, Y, r, c)
        absxy = np.einsum("ij,ji->i", np.abs(X[r]), np.abs(Y[:, c]))
        err = np.abs(got[r, c].astype(np.float64) - want)
        assert np.all(err <= 2.0 * (X.shape[1] + 2) * 2.0 ** -24 * absxy), what

    check(C.detach().cpu().numpy(), A64, B64, "C")
    check(Ad.grad.cpu().numpy(), dC64, B64.T.copy(), "dA")
    check(Bd.grad.cpu().numpy(), A64.T.copy(), dC64, "dB")
