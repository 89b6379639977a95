"""Pins of the oracle's smoothed sample (Algorithm rpCholesky-QR line 2 with
F = F_T D: the remark after Theorem t_prob allows a Walsh-Hadamard F_T, D a
diagonal of independent random signs) against its definition, written here
independently of the oracle:

  M = smallest power of two >= m; H(k, i) = (-1)^popcount(k AND i) (Sylvester
  order); D_i = +1 if bit 63 of SplitMix64 output i seeded with
  seed XOR 0x5851f42d4c957f2d is 0, else -1; F = H D / sqrt(M) acts on A padded
  with zero rows; idx_r uniform on [0, M) (the pinned sampler with M);
  A_s = sqrt(M/c) (F [A; 0])(idx, :), computed as T / sqrt(c) with
  T(r, j) = sum_i D_i (-1)^popcount(idx_r AND i) A(i, j) summed in one fixed
  order: chunks of G * 4096 rows (G = max(1, ceil(ceil(m / 4096) / 256))),
  an fma chain in ascending i within a chunk, chunks added in ascending order,
  then T * (1 / sqrt(c)).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from workloads import gen_usv, metrics, sigma_profile

MASK = 2**64 - 1


def splitmix64(seed, r):
    z = (seed + (r + 1) * 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def signs(seed, m):
    return np.array([-1.0 if splitmix64(seed ^ 0x5851F42D4C957F2D, i) >> 63 else 1.0 for i in range(m)])


def padded_rows(m):
    return 1 << max(0, (m - 1).bit_length())


def dense_sample(A, idx, seed, s):
    """sqrt(M/s) (H D [A; 0] / sqrt(M))[idx] from dense matrices (any summation order)."""
    m, _ = A.shape
    M = padded_rows(m)
    H = scipy.linalg.hadamard(M)[:, :m] * signs(seed, m)[None, :]
    return math.sqrt(M / s) * (H[idx] @ A) / math.sqrt(M)


def test_sign_generator_and_padding(orc):
    for m in (1, 2, 3, 64, 65, 1000, 4097):
        assert orc.smooth_rows(m) == padded_rows(m)
    d = signs(12345, 200)
    assert all(orc.rademacher(12345, i) == d[i] for i in range(200))
    big = signs(7, 20000)
    assert abs(big.mean()) < 0.03  # balanced signs


def test_chunk_size_formula(orc):
    for m, want in [(1, 4096), (4096, 4096), (4097, 4096), (4096 * 256, 4096), (4096 * 256 + 1, 8192),
                    (16_000_000, 65536), (4_000_000, 16384)]:
        assert orc.smooth_chunk_rows(m) == want, m


@pytest.mark.parametrize("m,n,s,seed", [(37, 3, 10, 1), (64, 5, 20, 2), (1000, 4, 30, 3), (5000, 2, 7, 4)])
def test_integer_input_matches_the_dense_definition_exactly(orc, m, n, s, seed):
    rng = np.random.default_rng(seed)
    A = rng.integers(-1000, 1001, size=(m, n)).astype(np.float64)  # every partial sum exact
    idx, As = orc.smooth_sample(A, s, seed)
    assert np.array_equal(idx, orc.sample_indices(padded_rows(m), s, seed))
    M = padded_rows(m)
    H = scipy.linalg.hadamard(M)[:, :m].astype(np.int64) * signs(seed, m).astype(np.int64)[None, :]
    T = H[idx] @ A.astype(np.int64)  # exact integers
    sc = 1.0 / math.sqrt(s)
    assert np.array_equal(As, T.astype(np.float64) * sc)
    # and the same within rounding as the orthogonal transform written densely
    assert np.max(np.abs(As - dense_sample(A, idx, seed, s))) <= 1e-12 * np.max(np.abs(As))


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def test_summation_order_is_the_written_one(orc):
    """Two chunks (m > 4096), entries of mixed magnitude: the oracle's bits equal
    an exactly rounded re-derivation of the written order, and differ from a
    single fma chain over all rows."""
    m, n, s, seed = 4600, 2, 3, 9
    rng = np.random.default_rng(5)
    A = rng.standard_normal((m, n)) * np.exp2(rng.integers(-20, 21, size=(m, n)))
    idx, As = orc.smooth_sample(A, s, seed)
    d = signs(seed, m)
    chunk = 4096
    sc = 1.0 / math.sqrt(s)
    want = np.empty((s, n))
    chain = np.empty((s, n))
    for r in range(s):
        k = int(idx[r])
        sg = [(-d[i] if bin(k & i).count("1") & 1 else d[i]) for i in range(m)]
        for j in range(n):
            T = None
            for c0 in range(0, m, chunk):
                p = 0.0
                for i in range(c0, min(m, c0 + chunk)):
                    p = _fma(sg[i], float(A[i, j]), p)
                T = p if T is None else T + p
            want[r, j] = T * sc
            q = 0.0
            for i in range(m):
                q = _fma(sg[i], float(A[i, j]), q)
            chain[r, j] = q * sc
    assert np.array_equal(As, want)
    assert not np.array_equal(As, chain)


def test_sketch_gram_is_unbiased(orc):
    """F is orthogonal and rows are sampled uniformly from M with the sqrt(M/c)
    scale, so E[A_s^T A_s] = A^T A (the padding rows are zero)."""
    m, n, s = 300, 4, 40
    A = gen_usv(m, n, 10.0, 3)
    G = A.T @ A
    acc = np.zeros((n, n))
    trials = 400
    for t in range(trials):
        _, As = orc.smooth_sample(A, s, 1000 + t)
        acc += As.T @ As
    acc /= trials
    assert np.linalg.norm(acc - G) / np.linalg.norm(G) < 0.05


def coherent(m, n, kappa, seed):
    """The paper's Section 5.1 test matrices: A = Q_A R_A with Q_A = [I_n; 0]
    (coherence 1) and R_A with geometric singular values from 1 to 1/kappa and
    Haar singular vectors (as Matlab's randsvd)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    U, Ru = np.linalg.qr(rng.standard_normal((n, n)))
    U = U * np.sign(np.diag(Ru))[None, :]
    V, Rv = np.linalg.qr(rng.standard_normal((n, n)))
    V = V * np.sign(np.diag(Rv))[None, :]
    RA = (U * sigma_profile(n, kappa)[None, :]) @ V.T
    A = np.zeros((m, n))
    A[:n] = RA
    return np.asfortranarray(A)


def test_coherent_matrix_needs_smoothing(orc):
    """Section 5.1's worst-coherence matrix (m = 6000, n = 100, kappa = 1e15):
    sampling A's own rows leaves the sketch rank deficient; the smoothed sketch
    gives orthogonality below 1e-12 and a residual below 1e-15 at c = 3n."""
    m, n = 6000, 100
    A = coherent(m, n, 1e15, 1)
    plain = [orc.rpcholqr(A, 3 * n, seed, nthreads=4, keep=False).status for seed in range(4)]
    assert all(st == orc.ESKETCH for st in plain)
    for seed in range(3):
        r = orc.rpcholqr(A, 3 * n, seed, nthreads=4, keep=False, smooth=True)
        assert r.status == orc.OK
        assert metrics.orth_error(r.Q) < 1e-12
        assert metrics.residual(A, r.Q, r.R) < 1e-15


def test_lemma_l31_with_smoothing(orc):
    """sigma_i(sqrt(M/c) (F [Q; 0])(idx, :)) = 1 / sigma_{n-i+1}(A1)."""
    m, n, s = 3000, 20, 60
    A = coherent(m, n, 1e4, 2)
    r = orc.rpcholqr(A, s, 5, nthreads=4, smooth=True)
    assert r.status == orc.OK
    FQ = dense_sample(r.Q, r.idx, 5, s)
    sv = np.linalg.svd(FQ, compute_uv=False)
    sa = np.linalg.svd(r.A1, compute_uv=False)
    assert np.max(np.abs(sv - 1.0 / sa[::-1]) / sv) < 1e-10
