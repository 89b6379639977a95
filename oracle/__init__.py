"""Plain FP64 CPU oracle for rpCholesky-QR (arXiv 2406.11751) -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports it and it
imports nothing from the GPU library.

The arithmetic lives in ``rpcholqr_oracle.c`` (compiled with gcc, no fast-math,
no fp contraction); this module only marshals numpy arrays through ctypes.
Every array is float64 in Fortran (column-major) order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rpcholqr_oracle.c")
_LIB = os.path.join(_HERE, "librpcholqr_oracle.so")

OK, ESKETCH, ECHOL, EINVAL = 0, 1, 2, -1

GCC_FLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (used by the build step)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        i64, u64, i32, dp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        L.orc_splitmix64_at.restype = u64
        L.orc_splitmix64_at.argtypes = [u64, u64]
        L.orc_sample_indices.restype = None
        L.orc_sample_indices.argtypes = [i64, i64, u64, dp]
        L.orc_gather.restype = None
        L.orc_gather.argtypes = [i64, i64, i64, dp, dp, i64, dp]
        L.orc_householder_r.restype = i32
        L.orc_householder_r.argtypes = [i64, i64, dp, i64, dp, i64, dp]
        L.orc_sign_normalize.restype = None
        L.orc_sign_normalize.argtypes = [i64, dp, i64]
        L.orc_trsm_rows.restype = None
        L.orc_trsm_rows.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, i32]
        L.orc_gram.restype = None
        L.orc_gram.argtypes = [i64, i64, dp, i64, dp, i64, i32]
        L.orc_cholesky_upper.restype = i32
        L.orc_cholesky_upper.argtypes = [i64, dp, i64, dp, i64, dp]
        L.orc_trmm_upper.restype = None
        L.orc_trmm_upper.argtypes = [i64, dp, i64, dp, i64, dp, i64]
        L.orc_alg1.restype = i32
        L.orc_alg1.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, dp, i64, dp, dp, dp, dp, i32]
        L.orc_rpcholqr.restype = i32
        L.orc_rpcholqr.argtypes = [i64, i64, i64, u64, dp, i64, dp, i64, dp, i64,
                                   dp, dp, dp, dp, dp, dp, dp, i32]
        L.orc_rpcholqr_ex.restype = i32
        L.orc_rpcholqr_ex.argtypes = [i64, i64, i64, u64, i32, dp, i64, dp, i64, dp, i64,
                                      dp, dp, dp, dp, dp, dp, dp, i32]
        L.orc_smooth_sample.restype = None
        L.orc_smooth_sample.argtypes = [i64, i64, i64, u64, dp, i64, dp, dp, i32]
        L.orc_smooth_rows.restype = i64
        L.orc_smooth_rows.argtypes = [i64]
        L.orc_smooth_chunk_rows.restype = i64
        L.orc_smooth_chunk_rows.argtypes = [i64]
        L.orc_scramble.restype = u64
        L.orc_scramble.argtypes = [u64, i64]
        L.orc_rademacher.restype = ctypes.c_double
        L.orc_rademacher.argtypes = [u64, i64]
        L.orc_max_threads.restype = i32
        L.orc_max_threads.argtypes = []
        _lib = L
    return _lib


def _f64(a: np.ndarray) -> np.ndarray:
    """float64, Fortran order: element (i, j) at offset i + j*rows (ld = rows)."""
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def _p(a):
    return None if a is None else a.ctypes.data


def max_threads() -> int:
    return int(lib().orc_max_threads())


def splitmix64_at(seed: int, r: int) -> int:
    return int(lib().orc_splitmix64_at(seed & (2**64 - 1), r))


def sample_indices(m: int, s: int, seed: int) -> np.ndarray:
    idx = np.empty(s, dtype=np.int64)
    lib().orc_sample_indices(m, s, seed & (2**64 - 1), _p(idx))
    return idx


def gather(A: np.ndarray, idx: np.ndarray) -> np.ndarray:
    A = _f64(A)
    m, n = A.shape
    s = idx.shape[0]
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    As = np.empty((s, n), dtype=np.float64, order="F")
    lib().orc_gather(m, n, s, _p(idx), _p(A), max(m, 1), _p(As))
    return As


def householder_r(As: np.ndarray, normalize: bool = True):
    """R factor of the Householder QR of As (s x n).  Returns (R, status, bad_k)."""
    W = np.array(As, dtype=np.float64, order="F", copy=True)
    s, n = W.shape
    R = np.zeros((n, n), dtype=np.float64, order="F")
    bad = ctypes.c_int32(-1)
    rc = lib().orc_householder_r(s, n, _p(W), s, _p(R), n, ctypes.addressof(bad))
    if rc == OK and normalize:
        lib().orc_sign_normalize(n, _p(R), n)
    return R, rc, bad.value


def trsm_rows(B: np.ndarray, U: np.ndarray, nthreads: int = 1) -> np.ndarray:
    B, U = _f64(B), _f64(U)
    m, n = B.shape
    X = np.empty((m, n), dtype=np.float64, order="F")
    lib().orc_trsm_rows(m, n, _p(B), max(m, 1), _p(U), n, _p(X), max(m, 1), nthreads)
    return X


def gram(X: np.ndarray, nthreads: int = 1) -> np.ndarray:
    X = _f64(X)
    m, n = X.shape
    G = np.empty((n, n), dtype=np.float64, order="F")
    lib().orc_gram(m, n, _p(X), max(m, 1), _p(G), n, nthreads)
    return G


def cholesky_upper(G: np.ndarray):
    G = _f64(G)
    n = G.shape[0]
    R = np.empty((n, n), dtype=np.float64, order="F")
    bad = ctypes.c_int32(-1)
    rc = lib().orc_cholesky_upper(n, _p(G), n, _p(R), n, ctypes.addressof(bad))
    return R, rc, bad.value


def trmm_upper(U: np.ndarray, V: np.ndarray) -> np.ndarray:
    U, V = _f64(U), _f64(V)
    n = U.shape[0]
    C = np.empty((n, n), dtype=np.float64, order="F")
    lib().orc_trmm_upper(n, _p(U), n, _p(V), n, _p(C), n)
    return C


class Result(dict):
    """Q, R and the intermediates of one oracle run (attribute access)."""

    __getattr__ = dict.__getitem__


def alg1(A: np.ndarray, Rs: np.ndarray, nthreads: int = 1, keep: bool = True) -> Result:
    """Algorithm "Preconditioned Cholesky-QR" with a given R_s (Section 3.1)."""
    A, Rs = _f64(A), _f64(Rs)
    m, n = A.shape
    Q = np.empty((m, n), dtype=np.float64, order="F")
    R = np.empty((n, n), dtype=np.float64, order="F")
    A1 = np.empty((m, n), dtype=np.float64, order="F") if keep else None
    G1 = np.empty((n, n), dtype=np.float64, order="F")
    R2 = np.empty((n, n), dtype=np.float64, order="F")
    bad = ctypes.c_int32(-1)
    rc = lib().orc_alg1(m, n, _p(A), max(m, 1), _p(Rs), n, _p(Q), m, _p(R), n,
                        _p(A1), _p(G1), _p(R2), ctypes.addressof(bad), nthreads)
    return Result(Q=Q, R=R, A1=A1, G1=G1, R2=R2, status=rc, index=bad.value)


def smooth_rows(m: int) -> int:
    return int(lib().orc_smooth_rows(m))


def smooth_chunk_rows(m: int) -> int:
    return int(lib().orc_smooth_chunk_rows(m))


def scramble(i: int, M: int) -> int:
    return int(lib().orc_scramble(i, M))


def rademacher(seed: int, i: int) -> float:
    return float(lib().orc_rademacher(seed & (2**64 - 1), i))


def smooth_sample(A: np.ndarray, s: int, seed: int, nthreads: int = 1):
    """Smoothed sample (Algorithm rpCholesky-QR line 2, F = H D P): (idx, As)."""
    A = _f64(A)
    m, n = A.shape
    idx = np.empty(s, dtype=np.int64)
    As = np.empty((s, n), dtype=np.float64, order="F")
    lib().orc_smooth_sample(m, n, s, seed & (2**64 - 1), _p(A), max(m, 1), _p(idx), _p(As), nthreads)
    return idx, As


def rpcholqr(A: np.ndarray, s: int, seed: int, nthreads: int = 1, keep: bool = True,
             smooth: bool = False) -> Result:
    """Algorithm "rpCholesky-QR" (Section 4); F = I, or F = H D P with smooth=True.

    Returns Q, R and the intermediates idx, As, Rs, A1 (if keep), G1, R2, plus
    status (OK / ESKETCH / ECHOL / EINVAL) and the failing index.
    """
    A = _f64(A)
    m, n = A.shape
    Q = np.empty((m, n), dtype=np.float64, order="F")
    R = np.empty((n, n), dtype=np.float64, order="F")
    idx = np.empty(s, dtype=np.int64)
    As = np.empty((s, n), dtype=np.float64, order="F")
    Rs = np.empty((n, n), dtype=np.float64, order="F")
    A1 = np.empty((m, n), dtype=np.float64, order="F") if keep else None
    G1 = np.empty((n, n), dtype=np.float64, order="F")
    R2 = np.empty((n, n), dtype=np.float64, order="F")
    bad = ctypes.c_int32(-1)
    rc = lib().orc_rpcholqr_ex(m, n, s, seed & (2**64 - 1), 1 if smooth else 0, _p(A), max(m, 1),
                               _p(Q), max(m, 1), _p(R), n, _p(idx), _p(As), _p(Rs), _p(A1), _p(G1),
                               _p(R2), ctypes.addressof(bad), nthreads)
    return Result(Q=Q, R=R, idx=idx, As=As, Rs=Rs, A1=A1, G1=G1, R2=R2, status=rc, index=bad.value)
