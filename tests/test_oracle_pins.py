"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a library
routine used as a textbook reference (LAPACK QR / Cholesky through numpy), a
high-precision brute-force computation, a closed form, an exact-arithmetic case,
an invariant the paper proves, or a magnitude the paper reports.
"""
import decimal
import math

import numpy as np
import pytest
import scipy.stats

from tests import _golden
from workloads import gen_usv, metrics

U = 2.0 ** -53
M64 = 2 ** 64 - 1


# ---------------------------------------------------------------------------
# Row sampling (Algorithm rpCholesky-QR, line 2; Section 4: uniform, independent,
# with replacement).
# ---------------------------------------------------------------------------

def _splitmix_sequential(seed, count):
    """The published sequential SplitMix64 (state += gamma, then mix)."""
    out, x = [], seed & M64
    for _ in range(count):
        x = (x + 0x9E3779B97F4A7C15) & M64
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        out.append(z ^ (z >> 31))
    return out


def test_indices_range_and_counter_form(orc):
    for m, s, seed in [(1, 5, 0), (7, 100, 3), (10_000, 150, 0), (2**40 + 17, 64, 2**63 + 5)]:
        idx = orc.sample_indices(m, s, seed)
        assert idx.dtype == np.int64 and idx.shape == (s,)
        assert idx.min() >= 0 and idx.max() < m
        z = _splitmix_sequential(seed, s)
        assert [orc.splitmix64_at(seed, r) for r in range(s)] == z
        assert idx.tolist() == [(zz * m) >> 64 for zz in z]


def test_indices_power_of_two_m_are_top_bits(orc):
    # floor(z * 2^k / 2^64) = z >> (64 - k): the multiply-high reduction keeps the top bits.
    for k in (1, 5, 20, 33):
        idx = orc.sample_indices(2**k, 500, 9)
        z = np.array([orc.splitmix64_at(9, r) for r in range(500)], dtype=np.uint64)
        assert np.array_equal(idx.astype(np.uint64), z >> np.uint64(64 - k))


def test_indices_uniform_chi2(orc):
    m, s = 97, 200_000
    idx = orc.sample_indices(m, s, 12345)
    counts = np.bincount(idx, minlength=m)
    assert scipy.stats.chisquare(counts).pvalue > 1e-4


def test_indices_pairs_independent_chi2(orc):
    m, s = 16, 200_001
    idx = orc.sample_indices(m, s, 777)
    pairs = idx[:-1] * m + idx[1:]
    counts = np.bincount(pairs, minlength=m * m)
    assert scipy.stats.chisquare(counts).pvalue > 1e-4


def test_indices_bits_balanced(orc):
    z = np.array([orc.splitmix64_at(2024, r) for r in range(20_000)], dtype=np.uint64)
    for b in range(64):
        frac = float(((z >> np.uint64(b)) & np.uint64(1)).mean())
        assert abs(frac - 0.5) < 0.02, b


def test_with_replacement_duplicates_at_birthday_rate(orc):
    # s draws from m with replacement: expected distinct = m (1 - (1-1/m)^s).
    m, s = 1000, 1000
    trials = [len(np.unique(orc.sample_indices(m, s, seed))) for seed in range(40)]
    expect = m * (1 - (1 - 1 / m) ** s)
    assert abs(np.mean(trials) - expect) < 5.0


# ---------------------------------------------------------------------------
# Scaled gather (Remark r_exp: A_s = sqrt(m/c) FA(rows,:)).
# ---------------------------------------------------------------------------

def test_gather_scale_makes_sketch_gram_unbiased(orc):
    # With the sqrt(m/c) scale, E[A_s^T A_s] = A^T A; over many draws the mean matches.
    rng = np.random.default_rng(1)
    A = np.asfortranarray(rng.standard_normal((200, 3)))
    acc = np.zeros((3, 3))
    trials = 400
    for seed in range(trials):
        As = orc.gather(A, orc.sample_indices(200, 50, seed))
        acc += As.T @ As
    G = A.T @ A
    assert np.linalg.norm(acc / trials - G) / np.linalg.norm(G) < 0.03


def test_gather_rows_exact(orc):
    rng = np.random.default_rng(2)
    A = np.asfortranarray(rng.standard_normal((64, 5)))
    idx = orc.sample_indices(64, 20, 4)
    As = orc.gather(A, idx)
    assert np.array_equal(As, np.sqrt(64 / 20) * A[idx, :])


# ---------------------------------------------------------------------------
# Thin QR of the sample (line 3), R only, positive diagonal.
# ---------------------------------------------------------------------------

def _lapack_r(X):
    R = np.linalg.qr(X, mode="r")
    return R * np.sign(np.diag(R))[:, None]


@pytest.mark.parametrize("s,n", [(5, 1), (10, 3), (63, 63), (64, 8), (65, 20), (150, 50), (192, 64), (300, 17)])
def test_householder_matches_lapack(orc, s, n):
    rng = np.random.default_rng(s * 1000 + n)
    X = np.asfortranarray(rng.standard_normal((s, n)) @ np.diag(np.logspace(0, -3, n)))
    R, rc, _ = orc.householder_r(X)
    assert rc == orc.OK
    assert np.all(np.diag(R) > 0) and np.array_equal(np.tril(R, -1), np.zeros((n, n)))
    Rl = _lapack_r(X)
    assert np.linalg.norm(R - Rl) / np.linalg.norm(Rl) < 1e-13
    # R^T R reproduces the Gram matrix to backward-error level.
    G = X.T @ X
    assert np.linalg.norm(R.T @ R - G) <= 20 * s * U * np.linalg.norm(X) ** 2


def test_householder_against_high_precision_cholesky(orc):
    # Brute force: R is the Cholesky factor of X^T X, computed exactly in 60-digit decimals.
    rng = np.random.default_rng(5)
    s, n = 9, 4
    X = np.asfortranarray(rng.standard_normal((s, n)))
    ctx = decimal.Context(prec=60)
    D = [[decimal.Decimal(float(v)) for v in row] for row in X]
    G = [[sum((D[r][i] * D[r][j] for r in range(s)), decimal.Decimal(0)) for j in range(n)] for i in range(n)]
    Rx = [[decimal.Decimal(0)] * n for _ in range(n)]
    for j in range(n):
        for i in range(j):
            t = G[i][j] - sum((Rx[k][i] * Rx[k][j] for k in range(i)), decimal.Decimal(0))
            Rx[i][j] = ctx.divide(t, Rx[i][i])
        d = G[j][j] - sum((Rx[k][j] ** 2 for k in range(j)), decimal.Decimal(0))
        Rx[j][j] = ctx.sqrt(d)
    Rref = np.array([[float(v) for v in row] for row in Rx])
    R, rc, _ = orc.householder_r(X)
    assert rc == orc.OK
    assert np.max(np.abs(R - Rref)) <= 50 * U * np.max(np.abs(Rref))


def test_householder_n1_is_norm(orc):
    rng = np.random.default_rng(6)
    for s in (1, 2, 7, 64, 65, 200):
        x = np.asfortranarray(rng.standard_normal((s, 1)))
        R, rc, _ = orc.householder_r(x)
        assert rc == orc.OK
        assert abs(R[0, 0] - math.sqrt(math.fsum(v * v for v in x[:, 0]))) <= 4 * U * R[0, 0]


def test_householder_exact_on_triangular_input(orc):
    # A_s = [R0; 0] with diag(R0) > 0: every reflection is exact (nu = |alpha|, tau = 2),
    # so the normalized factor equals R0 bit for bit.
    rng = np.random.default_rng(7)
    n = 12
    R0 = np.triu(rng.standard_normal((n, n)))
    np.fill_diagonal(R0, np.abs(np.diag(R0)) + 0.5)
    X = np.asfortranarray(np.vstack([R0, np.zeros((30, n))]))
    R, rc, _ = orc.householder_r(X)
    assert rc == orc.OK and np.array_equal(R, R0)


def test_householder_zero_column_is_esketch(orc):
    rng = np.random.default_rng(8)
    X = np.asfortranarray(rng.standard_normal((40, 6)))
    X[:, 3] = 0.0
    _, rc, k = orc.householder_r(X)
    assert rc == orc.ESKETCH and k == 3
    X = np.asfortranarray(rng.standard_normal((40, 6)))
    X[5, 2] = np.nan
    _, rc, k = orc.householder_r(X)
    # Column 0 is clean; the first reflection spreads the NaN through column 2, whose own
    # norm then is not finite.
    assert rc == orc.ESKETCH and k == 2


# ---------------------------------------------------------------------------
# Row-wise triangular solve (Section 2.1: Q = A R^{-1} as m triangular solves).
# ---------------------------------------------------------------------------

def test_trsm_componentwise_backward_error(orc):
    # Higham, Accuracy and Stability, Thm 8.5: (U + dU_i) x_i = b_i with |dU_i| <= gamma_n |U|.
    # Check |x U - b| <= gamma_{n+2} |x||U| row by row in extended precision.
    rng = np.random.default_rng(9)
    m, n = 300, 40
    Umat = np.triu(rng.standard_normal((n, n))) + np.diag(rng.uniform(0.1, 2.0, n))
    B = np.asfortranarray(rng.standard_normal((m, n)))
    X = orc.trsm_rows(B, Umat)
    Xl, Ul, Bl = X.astype(np.longdouble), Umat.astype(np.longdouble), B.astype(np.longdouble)
    res = np.abs(Xl @ Ul - Bl)
    gamma = (n + 2) * U / (1 - (n + 2) * U)
    bound = gamma * (np.abs(Xl) @ np.abs(Ul))
    assert np.all(res <= bound)


def test_trsm_exact_cases(orc):
    rng = np.random.default_rng(10)
    B = np.asfortranarray(rng.standard_normal((50, 7)))
    assert np.array_equal(orc.trsm_rows(B, np.eye(7)), B)
    D = np.diag(2.0 ** np.arange(-3, 4))
    assert np.array_equal(orc.trsm_rows(B, D), B / np.diag(D)[None, :])
    # integer unit-triangular U and X: B = X U exact, so the solve recovers X exactly.
    Xi = np.asfortranarray(rng.integers(-5, 6, size=(30, 6)).astype(np.float64))
    Ui = np.triu(rng.integers(-3, 4, size=(6, 6)).astype(np.float64), 1) + np.eye(6)
    assert np.array_equal(orc.trsm_rows(Xi @ Ui, Ui), Xi)


# ---------------------------------------------------------------------------
# Gram matrix (Algorithm Preconditioned Cholesky-QR, line 4).
# ---------------------------------------------------------------------------

def test_gram_matches_blas_and_exact_integers(orc):
    rng = np.random.default_rng(11)
    X = np.asfortranarray(rng.standard_normal((1000, 9)))
    G = orc.gram(X, nthreads=3)
    assert np.array_equal(np.tril(G, -1), np.zeros((9, 9)))
    ref = X.T @ X
    assert np.max(np.abs(np.triu(G) - np.triu(ref))) <= 1000 * U * np.max(np.abs(ref))
    Xi = np.asfortranarray(rng.integers(-50, 51, size=(500, 5)).astype(np.float64))
    assert np.array_equal(orc.gram(Xi), np.triu(Xi.T @ Xi))


def test_gram_thread_count_independent(orc):
    rng = np.random.default_rng(12)
    X = np.asfortranarray(rng.standard_normal((5000, 12)))
    assert np.array_equal(orc.gram(X, 1), orc.gram(X, 7))


# ---------------------------------------------------------------------------
# Cholesky (line 5) and triangular product (line 8).
# ---------------------------------------------------------------------------

def test_cholesky_matches_lapack(orc):
    rng = np.random.default_rng(13)
    n = 30
    Y = rng.standard_normal((80, n))
    G = Y.T @ Y
    R, rc, _ = orc.cholesky_upper(np.triu(G))
    assert rc == orc.OK
    Rl = np.linalg.cholesky(G).T
    assert np.linalg.norm(R - Rl) / np.linalg.norm(Rl) < 1e-13
    assert np.linalg.norm(R.T @ R - G) <= 10 * n * U * np.linalg.norm(G)


def test_cholesky_exact_and_breakdown(orc):
    R0 = np.array([[2.0, -1.0, 3.0, 0.5], [0, 4.0, 2.0, -2.0], [0, 0, 1.0, 6.0], [0, 0, 0, 8.0]])
    R, rc, _ = orc.cholesky_upper(np.triu(R0.T @ R0))
    assert rc == orc.OK and np.array_equal(R, R0)
    G = np.array([[4.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 1.0]])  # singular leading 2x2
    _, rc, j = orc.cholesky_upper(G)
    assert rc == orc.ECHOL and j == 1
    G = np.eye(3)
    G[2, 2] = np.nan
    _, rc, j = orc.cholesky_upper(G)
    assert rc == orc.ECHOL and j == 2


def test_trmm_matches_matmul(orc):
    rng = np.random.default_rng(14)
    A = np.triu(rng.integers(-9, 10, size=(11, 11)).astype(np.float64))
    B = np.triu(rng.integers(-9, 10, size=(11, 11)).astype(np.float64))
    assert np.array_equal(orc.trmm_upper(A, B), A @ B)


# ---------------------------------------------------------------------------
# End to end: rpCholesky-QR (Section 4).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", _golden.names())
def test_golden_closed_forms(orc, name):
    g = _golden.load(name)
    r = orc.rpcholqr(g["A"], g["s"], g["seed"])
    assert r.status == orc.OK
    assert np.max(np.abs(r.Q - g["Q"])) <= 1e-14
    assert np.max(np.abs(r.R - g["R"])) <= 1e-14 * np.max(np.abs(g["R"]))


def test_n1_closed_form(orc):
    rng = np.random.default_rng(15)
    a = np.asfortranarray(rng.standard_normal((5000, 1)))
    r = orc.rpcholqr(a, 3, 0)
    nrm = math.sqrt(math.fsum(v * v for v in a[:, 0]))
    assert abs(r.R[0, 0] - nrm) <= 1e-15 * nrm
    assert np.max(np.abs(r.Q[:, 0] - a[:, 0] / nrm)) <= 1e-15 * np.max(np.abs(a)) / nrm


@pytest.mark.parametrize("kappa", [1.0, 1e4, 1e8, 1e12, 1e15])
def test_paper_accuracy_claims(orc, kappa):
    # Section 5.1 summary: with c = 3n samples, orthogonality error <= 1e-12 and residual
    # below 1e-15, also for numerically singular A (kappa = 1e15).  Incoherent inputs (F = I).
    m, n = 20_000, 32
    A = gen_usv(m, n, kappa, 0)
    r = orc.rpcholqr(A, 3 * n, 0, nthreads=4)
    assert r.status == orc.OK
    orth = metrics.orth_error(r.Q)
    res = metrics.residual(A, r.Q, r.R)
    assert orth <= 1e-12
    assert res <= 1e-15
    # R is upper triangular with a positive diagonal.
    assert np.all(np.diag(r.R) > 0) and np.array_equal(np.tril(r.R, -1), np.zeros((n, n)))


def test_orthogonality_tracks_kappa_A1(orc):
    # Section 5.2, estimate e_ex1: ||Q^T Q - I||_2 ~ 4 eps kappa(A1), eps = 2^-52,
    # linear (not quadratic) in kappa(A1).  Sweep the sample count to vary kappa(A1).
    m, n = 20_000, 24
    A = gen_usv(m, n, 1e10, 3)
    eps = 2.0 ** -52
    ratios, kappas = [], []
    for c in (n + 1, n + 4, 2 * n, 3 * n, 6 * n):
        for seed in range(3):
            r = orc.rpcholqr(A, c, seed, nthreads=4)
            assert r.status == orc.OK
            k1 = np.linalg.cond(r.A1)
            orth = metrics.orth_error(r.Q)
            ratios.append(orth / (4 * eps * k1))
            kappas.append(k1)
    ratios = np.array(ratios)
    assert np.all(ratios > 0.02) and np.all(ratios < 20.0)
    assert max(kappas) / min(kappas) > 5.0  # the sweep really varied kappa(A1)


def test_lemma_l31_singular_values(orc):
    # Lemma l_31: sigma_i(S F Q) = 1 / sigma_{n-i+1}(A1).
    m, n, s = 5000, 10, 30
    A = gen_usv(m, n, 1e3, 4)
    r = orc.rpcholqr(A, s, 1)
    sq = np.linalg.svd(np.sqrt(m / s) * r.Q[r.idx, :], compute_uv=False)
    sa = np.linalg.svd(r.A1, compute_uv=False)
    assert np.max(np.abs(sq - 1.0 / sa[::-1]) / sq) < 1e-10


def test_remark_r_precond_invariances(orc):
    # Any nonsingular R_s gives the same Q and R: independent of seed and sample count,
    # and of the row order of A.
    m, n = 8000, 16
    A = gen_usv(m, n, 1e9, 5)
    base = orc.rpcholqr(A, 3 * n, 0)
    for seed, s in ((1, 3 * n), (2, 5 * n), (3, n + 2)):
        r = orc.rpcholqr(A, s, seed)
        assert metrics.rel_fro(r.R, base.R) < 1e-13
    perm = np.random.default_rng(0).permutation(m)
    r = orc.rpcholqr(np.asfortranarray(A[perm]), 3 * n, 0)
    assert metrics.rel_fro(r.R, base.R) < 1e-13


def test_power_of_two_column_scaling_is_exact(orc):
    # A D with D = diag(2^k): every step scales exactly, so Q is bit-identical and R -> R D.
    m, n = 3000, 9
    A = gen_usv(m, n, 1e6, 6)
    D = 2.0 ** np.array([3, -2, 0, 7, -5, 1, 0, 2, -1], dtype=np.float64)
    a = orc.rpcholqr(A, 27, 4)
    b = orc.rpcholqr(np.asfortranarray(A * D[None, :]), 27, 4)
    assert np.array_equal(a.Q, b.Q)
    assert np.array_equal(a.R * D[None, :], b.R)


@pytest.mark.parametrize("kappa", [1.0, 1e8, 1e15])
def test_against_lapack_qr(orc, kappa):
    m, n = 6000, 20
    A = gen_usv(m, n, kappa, 7)
    r = orc.rpcholqr(A, 3 * n, 2)
    Ql, Rl = np.linalg.qr(A)
    sg = np.sign(np.diag(Rl))
    Ql, Rl = Ql * sg[None, :], Rl * sg[:, None]
    assert metrics.rel_fro(r.R, Rl) < 1e-12
    assert metrics.rel_fro(r.Q, Ql) < max(100 * U * kappa, 1e-14)


def test_theorem_t_perturb2_bounds(orc):
    # Theorem t_perturb2 with the errors of this run measured in extended precision:
    # orthogonality and residual must lie below the rigorous bounds.
    m, n, s = 3000, 12, 36
    for kappa in (1e2, 1e6):
        A = gen_usv(m, n, kappa, 8)
        r = orc.rpcholqr(A, s, 0)
        L = np.longdouble
        Al, Rs, A1, G1, R2, Q, R = (x.astype(L) for x in (A, r.Rs, r.A1, r.G1, r.R2, r.Q, r.R))
        n2 = lambda M: float(np.linalg.norm(np.asarray(M, dtype=np.float64), 2))
        G1f = np.triu(G1) + np.triu(G1, 1).T
        Es = A1 @ Rs - Al
        E1 = G1f - A1.T @ A1
        E2 = R2.T @ R2 - G1f
        E3 = Q @ R2 - A1
        E4 = R - R2 @ Rs
        A1x = np.linalg.solve(Rs.astype(np.float64).T, A.T).T  # reference A R_s^{-1}
        k1 = np.linalg.cond(A1x)
        eA = 0.0
        es = n2(Es) / (n2(A1x) * n2(Rs))
        e1 = n2(E1) / n2(A1) ** 2
        e2 = n2(E2) / n2(G1f)
        e3 = n2(E3) / n2(A1)
        e4 = n2(E4) / n2(R2 @ Rs)
        eta = n2(A1x) * n2(Rs) / n2(A)
        eF = (eA + es) * np.linalg.cond(r.Rs)
        g1 = (1 + eF) ** 2 * (e1 + (1 + e1) * e2 + 2 * e3 + e3 ** 2)
        g2 = 2 * eF + eF ** 2 + (1 + eF) ** 2 * (e1 + (1 + e1) * e2)
        g3 = e4 * (1 + eF) * (1 + e3)
        assert k1 ** 2 * g2 < 1
        orth = n2(Q.T @ Q - np.eye(n, dtype=L))
        res = n2(Al - Q @ R) / n2(A)
        assert orth <= k1 ** 2 * g1 / (1 - k1 ** 2 * g2)
        bound = eA + (es + (1 + eF) * e3) * eta + g3 * np.sqrt((1 + g2) / (1 - k1 ** 2 * g2)) * eta * k1
        assert res <= bound


def test_basic_cholqr_breaks_down_where_rpcholqr_does_not(orc):
    # Algorithm Preconditioned Cholesky-QR with R_s = I is basic Cholesky-QR (Theorem
    # t_perturb1 is its special case); at kappa(A) = 1e15 its Gram matrix is numerically
    # indefinite, while rpCholesky-QR succeeds (Section 1.1, item 4).
    m, n = 4000, 16
    A = gen_usv(m, n, 1e15, 1)
    basic = orc.alg1(A, np.eye(n))
    assert basic.status == orc.ECHOL
    assert orc.rpcholqr(A, 3 * n, 0).status == orc.OK
    # Well conditioned: basic Cholesky-QR works, orthogonality ~ kappa^2 u (t_perturb1).
    A = gen_usv(m, n, 1e3, 1)
    basic = orc.alg1(A, np.eye(n))
    assert basic.status == orc.OK
    assert 1e-13 < metrics.orth_error(basic.Q) < 1e-7


def test_failure_codes(orc):
    rng = np.random.default_rng(16)
    A = np.asfortranarray(rng.standard_normal((500, 6)))
    A[:, 4] = 0.0
    r = orc.rpcholqr(A, 18, 0)
    assert r.status == orc.ESKETCH and r.index == 4
    A = np.asfortranarray(rng.standard_normal((500, 6)))
    idx = orc.sample_indices(500, 18, 0)
    A[idx[3], 2] = np.inf
    r = orc.rpcholqr(A, 18, 0)
    assert r.status == orc.ESKETCH and r.index == 2
    # A non-finite entry in a row the sample missed reaches the Gram matrix instead.
    A = np.asfortranarray(rng.standard_normal((500, 6)))
    missed = sorted(set(range(500)) - set(orc.sample_indices(500, 18, 0).tolist()))[0]
    A[missed, 1] = np.nan
    r = orc.rpcholqr(A, 18, 0)
    # Column 0 of A1 stays finite; the NaN enters column 1 and every later one.
    assert r.status == orc.ECHOL and r.index == 1
    for bad in [(0, 1, 1), (3, 4, 4), (10, 3, 2)]:
        m, n, s = bad
        assert orc.rpcholqr(np.zeros((max(m, 1), n), order="F")[:m], s, 0).status == orc.EINVAL
