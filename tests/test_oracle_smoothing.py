"""Pins of the oracle's smoothed sample (Algorithm rpCholesky-QR line 2 with
F = F_T D: the remark after Theorem t_prob allows a Walsh-Hadamard F_T, D a
diagonal of independent random signs) against its definition, written here
independently of the oracle:

  M = smallest power of two >= m = 2^p; H(k, q) = (-1)^popcount(k AND q)
  (Sylvester order); pi(i) = the bijection of [0, M): x = i * 0x9e3779b97f4a7c15,
  x ^= x >> h, x *= 0xbf58476d1ce4e5b9, x ^= x >> h, everything mod M,
  h = max(1, floor(p / 2)); D_i = +1 if bit 63 of SplitMix64 output i seeded with
  seed XOR 0x5851f42d4c957f2d is 0, else -1; row i of A padded with zero rows
  goes to position pi(i) and is multiplied by D_i; F = H / sqrt(M) then mixes;
  idx_r uniform on [0, M) (the pinned sampler with M);
  A_s = sqrt(M/c) (F [A; 0])(idx, :), computed as T / sqrt(c) with
  T(r, j) = sum_i D_i (-1)^popcount(idx_r AND pi(i)) A(i, j) summed in one fixed
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


def scramble(i, M):
    p = M.bit_length() - 1
    h = max(1, p // 2)
    x = (i * 0x9E3779B97F4A7C15) % M
    x ^= x >> h
    x = (x * 0xBF58476D1CE4E5B9) % M
    x ^= x >> h
    return x


def signs(seed, m):
    return np.array([-1.0 if splitmix64(seed ^ 0x5851F42D4C957F2D, i) >> 63 else 1.0 for i in range(m)])


def padded_rows(m):
    return 1 << max(0, (m - 1).bit_length())


def permuted_signed(A, seed):
    """The M x n matrix with row i of A, times D_i, at position pi(i) (zeros elsewhere)."""
    m, n = A.shape
    M = padded_rows(m)
    B = np.zeros((M, n), dtype=A.dtype)
    d = signs(seed, m).astype(A.dtype)
    for i in range(m):
        B[scramble(i, M)] = d[i] * A[i]
    return B


def dense_sample(A, idx, seed, s):
    """sqrt(M/s) (H P D [A; 0] / sqrt(M))[idx] from dense matrices (any summation order)."""
    m, _ = A.shape
    M = padded_rows(m)
    H = scipy.linalg.hadamard(M)
    return math.sqrt(M / s) * (H[idx] @ permuted_signed(A, seed)) / math.sqrt(M)


def test_sign_generator_padding_and_scramble(orc):
    for m in (1, 2, 3, 64, 65, 1000, 4097):
        assert orc.smooth_rows(m) == padded_rows(m)
    for M in (1, 2, 8, 1024, 8192):
        pis = [orc.scramble(i, M) for i in range(M)]
        assert sorted(pis) == list(range(M))  # a permutation
        assert pis == [scramble(i, M) for i in range(M)]
    assert orc.scramble(123456, 1 << 24) == scramble(123456, 1 << 24)
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
    H = scipy.linalg.hadamard(M).astype(np.int64)
    T = H[idx] @ permuted_signed(A, seed).astype(np.int64)  # exact integers
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
    M = padded_rows(m)
    pis = [scramble(i, M) for i in range(m)]
    chunk = 4096
    sc = 1.0 / math.sqrt(s)
    want = np.empty((s, n))
    chain = np.empty((s, n))
    for r in range(s):
        k = int(idx[r])
        sg = [(-d[i] if bin(k & pis[i]).count("1") & 1 else d[i]) for i in range(m)]
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


def test_smoothed_sketch_of_a_coherent_matrix_is_well_conditioned(orc):
    """Section 5.1 at n = 300 (m = 6000, kappa = 1e15, c = 3n): kappa(A1) of the
    smoothed sketch is of the size of a Gaussian sketch's (about 4), and the
    orthogonality error follows the estimate 4 eps kappa(A1) of Section 5.2."""
    m, n = 6000, 300
    A = coherent(m, n, 1e15, 3)
    for seed in (1, 2):
        r = orc.rpcholqr(A, 3 * n, seed, nthreads=4, smooth=True)
        assert r.status == orc.OK
        sv = np.linalg.svd(r.A1, compute_uv=False)
        kap = sv[0] / sv[-1]
        assert kap < 10
        assert metrics.orth_error(r.Q) < 1e-12
        assert metrics.orth_error(r.Q) < 20 * 4 * 2.0 ** -52 * kap
