"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds no arithmetic of the method: it only draws matrices and
problem shapes from numpy's PCG64 generator with fixed seeds.  The paper runs
on synthetic FP64 matrices of stated shapes and never states the entry
distribution, so the distributions below are this project's choice (uniform
[-1, 1] for plain GEMM, small integers for exact checks, signed log-uniform
magnitudes for the split-precision product, standard normal for upstream
gradients, log-uniform problem sizes for batches).
"""
import numpy as np

SEED_A = 190405717
SEED_B = 190405718
SEED_C = 190405719
SEED_DC = 190405720
SEED_BATCH = 190405721


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform(shape, seed, lo=-1.0, hi=1.0):
    """i.i.d. uniform[lo, hi) fp64 entries."""
    return _rng(seed).uniform(lo, hi, size=shape).astype(np.float64, copy=False)


def integers(shape, seed, lo=-8, hi=8):
    """i.i.d. integers in [lo, hi] stored as fp64 (exact in every summation order)."""
    return _rng(seed).integers(lo, hi + 1, size=shape).astype(np.float64)


def signed_log_uniform(shape, seed, lo=1e-8, hi=1e8):
    """Sign uniform on {-1, +1}, magnitude 10**U(log10 lo, log10 hi)."""
    g = _rng(seed)
    mag = 10.0 ** g.uniform(np.log10(lo), np.log10(hi), size=shape)
    sgn = np.where(g.integers(0, 2, size=shape) == 0, -1.0, 1.0)
    return (sgn * mag).astype(np.float64, copy=False)


def normal(shape, seed):
    """i.i.d. standard normal fp64 entries."""
    return _rng(seed).standard_normal(size=shape).astype(np.float64, copy=False)


def batch_shapes(count, seed=SEED_BATCH, lo=32, hi=2048):
    """(m, n, k) triples, each drawn as round(exp(U(ln lo, ln hi))) from one seed."""
    g = _rng(seed)
    x = np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), size=(count, 3)))).astype(np.int64)
    return [tuple(int(v) for v in row) for row in np.clip(x, lo, hi)]


def gemm_operands(m, n, k, kind="uniform", with_c=True):
    """A (m x k), B (k x n) and C (m x n) drawn with the standard seeds."""
    if kind == "uniform":
        A, B = uniform((m, k), SEED_A), uniform((k, n), SEED_B)
        C = uniform((m, n), SEED_C) if with_c else None
    elif kind == "int":
        A, B = integers((m, k), SEED_A), integers((k, n), SEED_B)
        C = integers((m, n), SEED_C) if with_c else None
    elif kind == "loguniform":
        A, B = signed_log_uniform((m, k), SEED_A), signed_log_uniform((k, n), SEED_B)
        C = uniform((m, n), SEED_C) if with_c else None
    else:
        raise ValueError(kind)
    return A, B, C
