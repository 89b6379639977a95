"""Pins the rounding order of the oracle's sketch QR and row solves without
trusting the oracle or the GPU library.

Where the paper leaves the order of a computation free (the dot products of the
Householder QR of the sample, Algorithm rpCholesky-QR line 3; the row-wise
substitution A1 = A R_s^{-1} of Section 2.1), the oracle fixes one order so that
an independent implementation can reproduce its bits.  The orders, as written
down in words:

  * CR16 dot product of x and y over rows r = k..len-1: row r is added with a
    fused multiply-add into partial p[r mod 16], in ascending r; then
    p[i] = p[i] + p[i + h] for h = 1, 2, 4, 8 and i a multiple of 2h; result p[0].
  * Householder step k on column y = W[k:, k]: nu2 = CR16(y, y); nu = sqrt(nu2);
    alpha = y[0]; beta = -nu if alpha >= 0 else nu; d = 1/(alpha - beta);
    v = (1, y[1] d, y[2] d, ...); tau = (beta - alpha)/beta; R(k, k) = beta; for
    each later column w: t = tau * CR16(v, w); w[r] = fma(-t, v[r], w[r]) for
    r >= k; R(k, j) = w[k].  Afterwards rows of R with a negative diagonal are
    negated.
  * Row solve x U = b: rinv_k = 1/U(k, k) (one correctly rounded division);
    starting from t = b, for k = 0..n-1: x_k = t_k * rinv_k and
    t_j = fma(-x_k, U(k, j), t_j) for j > k.

This file re-derives every rounding from those sentences with exact rational
arithmetic (an fma is the exact a*b + c rounded once; Python's float() of a
Fraction rounds to nearest, ties to even) and IEEE scalar operations, and asks
the oracle for the same bits.  A different pairing of the tree, a different
partial count or a different accumulation order changes bits on these inputs
(checked below), so such a change in the oracle fails here, independently of
the GPU parity tests.
"""
import math
from fractions import Fraction

import numpy as np
import pytest


def fma(a: float, b: float, c: float) -> float:
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def tree16(p, pairs=((1,), (2,), (4,), (8,))):
    p = list(p)
    for (h,) in pairs:
        for i in range(0, 16, 2 * h):
            p[i] = p[i] + p[i + h]
    return p[0]


def cr16(x, y, k, length, tree=tree16):
    p = [0.0] * 16
    for r in range(k, length):
        p[r % 16] = fma(float(x[r]), float(y[r]), p[r % 16])
    return tree(p)


def householder_r(As, dot=cr16):
    W = [list(map(float, As[:, j])) for j in range(As.shape[1])]
    s, n = As.shape
    R = np.zeros((n, n))
    for k in range(n):
        y = W[k]
        nu2 = dot(y, y, k, s)
        assert nu2 > 0.0 and math.isfinite(nu2)
        nu = math.sqrt(nu2)
        alpha = y[k]
        beta = -nu if alpha >= 0.0 else nu
        d = 1.0 / (alpha - beta)
        v = [0.0] * s
        v[k] = 1.0
        for r in range(k + 1, s):
            v[r] = y[r] * d
        tau = (beta - alpha) / beta
        R[k, k] = beta
        for j in range(k + 1, n):
            w = W[j]
            t = tau * dot(v, w, k, s)
            for r in range(k, s):
                w[r] = fma(-t, v[r], w[r])
            R[k, j] = w[k]
    for k in range(n):
        if R[k, k] < 0.0:
            R[k, k:] = -R[k, k:]
    return R


def row_solve(B, U):
    m, n = B.shape
    rinv = [1.0 / float(U[k, k]) for k in range(n)]
    X = np.empty((m, n))
    for i in range(m):
        t = list(map(float, B[i]))
        for k in range(n):
            t[k] = t[k] * rinv[k]
            for j in range(k + 1, n):
                t[j] = fma(-t[k], float(U[k, j]), t[j])
        X[i] = t
    return X


def same_bits(a, b) -> bool:
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return a.shape == b.shape and bool(np.all(a.view(np.uint64) == b.view(np.uint64)))


# Sample shapes: fewer rows than the 16 partials, exactly 16, and several sweeps
# of them (s up to 40), for n up to 6.
SHAPES = [(3, 1), (5, 3), (9, 6), (15, 4), (16, 6), (17, 5), (23, 6), (31, 2), (33, 6), (40, 6)]


def sample(s, n, seed):
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    # entries of mixed magnitude, so that the order of additions shows in the bits
    return np.asfortranarray(rng.standard_normal((s, n)) * np.exp2(rng.integers(-6, 7, size=(s, n))))


@pytest.mark.parametrize("s,n", SHAPES)
def test_sketch_qr_bits_follow_the_written_order(orc, s, n):
    for seed in range(3):
        As = sample(s, n, 10 * s + n + seed)
        R_ref = householder_r(As)
        R_orc, rc, _ = orc.householder_r(As)
        assert rc == orc.OK
        assert same_bits(R_orc, R_ref), (s, n, seed)


@pytest.mark.parametrize("m,n", [(7, 1), (9, 3), (12, 6)])
def test_row_solve_bits_follow_the_written_order(orc, m, n):
    rng = np.random.Generator(np.random.PCG64(77 + n))
    for trial in range(3):
        B = rng.standard_normal((m, n)) * np.exp2(rng.integers(-5, 6, size=(m, n)))
        U = np.triu(rng.standard_normal((n, n))) + np.diag(rng.uniform(0.5, 2.0, n) * rng.choice([-1, 1], n))
        assert same_bits(orc.trsm_rows(B, U), row_solve(B, U)), (m, n, trial)


def test_other_orders_give_other_bits(orc):
    """The inputs above are sensitive to the order: a re-paired tree, a
    sequential sum of the partials, and a single running fma chain each change
    bits of R_s somewhere, so the pin above would catch such a change."""
    def tree_reversed(p):  # pairs far partials first: h = 8, 4, 2, 1
        return tree16(p, pairs=((8,), (4,), (2,), (1,)))

    def tree_sequential(p):
        acc = p[0]
        for v in p[1:]:
            acc = acc + v
        return acc

    def chain(x, y, k, length):
        acc = 0.0
        for r in range(k, length):
            acc = fma(float(x[r]), float(y[r]), acc)
        return acc

    variants = {
        "reversed tree": lambda x, y, k, L: cr16(x, y, k, L, tree=tree_reversed),
        "sequential partial sum": lambda x, y, k, L: cr16(x, y, k, L, tree=tree_sequential),
        "single fma chain": chain,
    }
    for name, dot in variants.items():
        differs = False
        for s, n in [(33, 6), (40, 6), (23, 6)]:
            As = sample(s, n, 10 * s + n)
            R_orc, _, _ = orc.householder_r(As)
            differs |= not same_bits(R_orc, householder_r(As, dot=dot))
        assert differs, name


def test_row_solve_other_orders_give_other_bits(orc):
    """Descending accumulation or division instead of the reciprocal changes bits."""
    rng = np.random.Generator(np.random.PCG64(5))
    B = rng.standard_normal((12, 6)) * np.exp2(rng.integers(-5, 6, size=(12, 6)))
    U = np.triu(rng.standard_normal((6, 6))) + np.diag(rng.uniform(0.5, 2.0, 6))
    X = orc.trsm_rows(B, U)
    m, n = B.shape

    def solve(order, divide):
        out = np.empty((m, n))
        for i in range(m):
            x = [0.0] * n
            for j in range(n):
                t = float(B[i, j])
                for k in order(j):
                    t = fma(-x[k], float(U[k, j]), t)
                x[j] = t / float(U[j, j]) if divide else t * (1.0 / float(U[j, j]))
            out[i] = x
        return out

    assert same_bits(X, solve(lambda j: range(j), False))
    assert not same_bits(X, solve(lambda j: reversed(range(j)), False))
    assert not same_bits(X, solve(lambda j: range(j), True))
