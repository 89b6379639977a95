"""Seeded synthetic inputs shaped like the paper's experiments.

This module holds no arithmetic of the factorization: it only draws test
matrices.  Both the oracle-side tests and the GPU-side tests and benchmark use
it, so that each side sees the same input bits.

``gen_usv(m, n, kappa, seed)`` builds A = U diag(sigma) V^T with
  * U = the Q factor of a Householder QR of an m x n standard Gaussian matrix
    (a Haar-distributed orthonormal basis, as the Haar premultiplier in the
    paper's Section 5.3 test matrices),
  * V = the Q factor of the QR of an n x n standard Gaussian matrix,
  * sigma_i = kappa^(-(i-1)/(n-1)), i = 1..n, geometric from 1 down to 1/kappa
    (the singular value profile of Matlab's randsvd in its default mode).
Hence ||A||_2 = 1, kappa_2(A) = kappa (up to rounding), and the rows of A have
low coherence (about n/m), so uniform row sampling without smoothing works.

The Gaussian draws use numpy's PCG64 seeded with ``seed``; the Gaussian matrix
is filled in column-major order.  ``backend="torch"`` draws on a torch device
with ``torch.Generator(device).manual_seed(seed)`` instead (for sizes the host
QR would take minutes on); the two backends give different matrices with the
same distribution.
"""
from __future__ import annotations

import hashlib

import numpy as np


def sigma_profile(n: int, kappa: float) -> np.ndarray:
    if n == 1 or kappa == 1.0:
        return np.ones(n)
    i = np.arange(n, dtype=np.float64)
    return kappa ** (-i / (n - 1))


def _haar_numpy(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    X = rng.standard_normal(m * n).reshape(n, m).T  # column-major fill
    Q, R = np.linalg.qr(X)
    # Fix the sign freedom so the distribution is Haar (Mezzadri 2007).
    Q = Q * np.sign(np.diag(R))[None, :]
    return Q


def gen_usv(m: int, n: int, kappa: float, seed: int, backend: str = "numpy", device=None):
    """A = U diag(sigma) V^T (m x n, float64, column-major); see module doc."""
    if backend == "numpy":
        rng = np.random.Generator(np.random.PCG64(seed))
        U = _haar_numpy(rng, m, n)
        V = _haar_numpy(rng, n, n)
        s = sigma_profile(n, kappa)
        return np.asfortranarray((U * s[None, :]) @ V.T)
    if backend == "torch":
        import torch

        dev = torch.device(device or "cuda")
        g = torch.Generator(device=dev)
        g.manual_seed(seed)
        X = torch.randn((n, m), generator=g, device=dev, dtype=torch.float64).t()
        U, RU = torch.linalg.qr(X)
        U = U * torch.sign(torch.diagonal(RU))[None, :]
        Y = torch.randn((n, n), generator=g, device=dev, dtype=torch.float64).t()
        V, RV = torch.linalg.qr(Y)
        V = V * torch.sign(torch.diagonal(RV))[None, :]
        s = torch.as_tensor(sigma_profile(n, kappa), device=dev, dtype=torch.float64)
        A = (U * s[None, :]) @ V.t()
        # column-major storage: (m, n) view with strides (1, m)
        return A.t().contiguous().t()
    raise ValueError(f"unknown backend {backend!r}")


def gen_usv_polar(m: int, n: int, kappa: float, seed: int, device=None, chunk_rows: int = 1 << 20):
    """A = U diag(sigma) V^T as gen_usv, for device-resident inputs too large for
    a QR of the Gaussian matrix next to A (the 16,000,000 x 512 workload is
    65.5 GB).  U is the orthonormal polar factor X (X^T X)^{-1/2} of the m x n
    standard Gaussian X, which is Haar-distributed like the Q factor of X (it
    differs from it by an n x n orthogonal factor that is independent of it);
    V is the Q factor of an n x n Gaussian matrix, sign-fixed.  A = X M with
    M = (X^T X)^{-1/2} diag(sigma) V^T is formed in place of X, chunk_rows rows
    at a time, so the input costs one m x n buffer.  Column-major (strides
    (1, m)); torch generator seeded with `seed`."""
    import torch

    dev = torch.device(device or "cuda")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    X = torch.randn((n, m), generator=g, device=dev, dtype=torch.float64).t()
    evals, evecs = torch.linalg.eigh(X.t() @ X)
    W = (evecs * evals.rsqrt()[None, :]) @ evecs.t()
    Y = torch.randn((n, n), generator=g, device=dev, dtype=torch.float64).t()
    V, RV = torch.linalg.qr(Y)
    V = V * torch.sign(torch.diagonal(RV))[None, :]
    sig = torch.as_tensor(sigma_profile(n, kappa), device=dev, dtype=torch.float64)
    M = (W * sig[None, :]) @ V.t()
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        X[r0:r1] = X[r0:r1] @ M
    return X


def checksum(A: np.ndarray) -> str:
    """SHA-256 of the column-major bytes of A."""
    return hashlib.sha256(np.asfortranarray(A, dtype=np.float64).tobytes(order="F")).hexdigest()


def batched_problem_list(count: int = 2048, seed: int = 0, m_lo: int = 2000, m_hi: int = 200000,
                         ns=(8, 16, 32, 64, 128), logk_lo: float = 2.0, logk_hi: float = 14.0):
    """Draw the (m_i, n_i, kappa_i, s_i, seed_i) list of the batched workload.

    m_i uniform on [m_lo, m_hi], n_i uniform on ``ns``, log10 kappa_i uniform on
    [logk_lo, logk_hi], s_i = 3 n_i, matrix and sampling seed = seed + i.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    nn = rng.choice(np.asarray(ns), size=count)
    lk = rng.uniform(logk_lo, logk_hi, size=count)
    return [dict(m=int(ms[i]), n=int(nn[i]), kappa=float(10.0 ** lk[i]), s=3 * int(nn[i]),
                 seed=seed + i) for i in range(count)]
