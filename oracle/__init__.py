"""CPU oracle for the MOMMS GEMM family (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and the
two share no code: the oracle is a plain compensated triple loop in C
(``gemm_dot2.c``), a numpy step-by-step emulation of the split-precision
product (``split_emul.py``), the exact-integer definition of the modular split
product (``crt_emul.py``) and a brute-force transfer counter for blocked loop
nests (``cache_sim.py``).

Functions here marshal numpy arrays into the C oracle.  ``build()`` compiles it
with gcc.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gemm_dot2.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build():
    """Compile the C oracle (-O2, no contraction, no fast-math, OpenMP)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, dbl, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.oracle_dgemm.argtypes = [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64]
    lib.oracle_dgemm.restype = None
    lib.oracle_dgemm_entries.argtypes = [i64, vp, vp, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, vp]
    lib.oracle_dgemm_entries.restype = None
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _rowmajor(x):
    x = np.asarray(x, dtype=np.float64)
    if x.ndim != 2:
        raise ValueError("expected a 2-D array")
    if not x.flags.c_contiguous:
        x = np.ascontiguousarray(x)
    return x


def gemm(A, B, C=None, alpha=1.0, beta=0.0):
    """Return alpha*A@B + beta*C (fp64, compensated, rounded once per entry).

    A is m x k, B is k x n, C (optional) is m x n.  With beta == 0, C is not
    read.  Inputs are not modified.
    """
    A = _rowmajor(A)
    B = _rowmajor(B)
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    if C is None:
        out = np.zeros((m, n), dtype=np.float64)
    else:
        out = np.array(_rowmajor(C), dtype=np.float64, copy=True)
        if out.shape != (m, n):
            raise ValueError("C has the wrong shape")
    if m and n:
        _load().oracle_dgemm(m, n, k, float(alpha), _ptr(A), max(k, 1), _ptr(B), max(n, 1),
                             float(beta), _ptr(out), max(n, 1))
    return out


def gemm_entries(A, B, rows, cols, C=None, alpha=1.0, beta=0.0):
    """Entries (rows[t], cols[t]) of alpha*A@B + beta*C, computed one by one."""
    A = _rowmajor(A)
    B = _rowmajor(B)
    m, k = A.shape
    n = B.shape[1]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    if rows.shape != cols.shape:
        raise ValueError("rows and cols differ in length")
    if rows.size and (rows.min() < 0 or rows.max() >= m or cols.min() < 0 or cols.max() >= n):
        raise ValueError("entry index out of range")
    if C is None:
        Cc = np.zeros((1, 1), dtype=np.float64)
        ldc = 1
        beta = 0.0
    else:
        Cc = _rowmajor(C)
        ldc = Cc.shape[1]
    out = np.empty(rows.size, dtype=np.float64)
    if rows.size:
        _load().oracle_dgemm_entries(rows.size, _ptr(rows), _ptr(cols), k, float(alpha),
                                     _ptr(A), max(k, 1), _ptr(B), max(n, 1), float(beta),
                                     _ptr(Cc), ldc, _ptr(out))
    return out


def num_threads():
    """OpenMP threads the C oracle uses (OMP_NUM_THREADS or all cores)."""
    return int(_load().oracle_num_threads())


def error_bound(A, B, C=None, alpha=1.0, beta=0.0, k=None, u=2.0 ** -53):
    """Per-entry tolerance T_ij = 2 (k+2) u (|alpha| (|A||B|)_ij + |beta| |C_ij|).

    The dominant term is the forward error bound of a k-term floating-point dot
    product evaluated in any order (Higham, Accuracy and Stability, Sec. 3.1),
    widened by two terms for the alpha/beta update.  |A||B| is itself computed
    here in plain fp64; its own relative error (<= k u) is negligible at this
    scale.
    """
    A = np.abs(np.asarray(A, dtype=np.float64))
    B = np.abs(np.asarray(B, dtype=np.float64))
    if k is None:
        k = A.shape[1]
    t = abs(alpha) * (A @ B)
    if C is not None and beta != 0.0:
        t = t + abs(beta) * np.abs(np.asarray(C, dtype=np.float64))
    return 2.0 * (k + 2) * u * t
