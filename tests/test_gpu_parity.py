"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Bit-exact: sampled indices, the scaled sample A_s, the sketch factor R_s and the
preconditioned matrix A1 (the steps whose rounding is fixed by the operation
order both sides follow).  Within 1e-12 relative Frobenius error: Q and R (the
tolerance the target states), and the Gram matrix / Cholesky factor, whose
summation order is free.  Orthogonality and residual are checked for every
result.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle
from workloads import gen_usv, metrics

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-12
NTHREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def rq():
    import paper_2406_11751_amd

    return paper_2406_11751_amd


def dev(A_h):
    """Column-major device copy of a host matrix."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A_h).T)).to("cuda").t()


def host(t):
    return t.cpu().numpy()


def announce(*args):
    print("case:", *args, flush=True)


def check_case(A_h, s, seed, exact_a1=True, smooth=False):
    m, n = A_h.shape
    announce(f"m={m} n={n} s={s} seed={seed} smooth={smooth}")
    A = dev(A_h)
    Q, R, info, ex = rq().factor(A, s, seed, debug=True, precision=rq().SMOOTH if smooth else rq().FP64)
    ref = oracle.rpcholqr(A_h, s, seed, nthreads=NTHREADS, smooth=smooth)
    assert ref.status == oracle.OK
    assert np.array_equal(host(ex["idx"]), ref.idx), "sampled indices differ"
    assert np.array_equal(host(ex["As"]), ref.As), "A_s differs"
    assert np.array_equal(host(ex["Rs"]), ref.Rs), "R_s differs"
    if exact_a1:
        a1 = host(ex["A1"])
        if not np.array_equal(a1, ref.A1):
            bad = np.argwhere(a1 != ref.A1)
            raise AssertionError(f"A1 differs in {len(bad)} entries, first {bad[:3].tolist()}")
    assert metrics.rel_fro(np.triu(host(ex["G1"])), np.triu(ref.G1)) < TOL
    assert metrics.rel_fro(host(ex["R2"]), ref.R2) < TOL
    Qh, Rh = host(Q), host(R)
    eq, er = metrics.rel_fro(Qh, ref.Q), metrics.rel_fro(Rh, ref.R)
    orth, res = metrics.orth_error(Qh), metrics.residual(A_h, Qh, Rh)
    print(f"  |dQ|={eq:.2e} |dR|={er:.2e} orth={orth:.2e} res={res:.2e}", flush=True)
    assert eq < TOL and er < TOL
    assert np.array_equal(np.tril(Rh, -1), np.zeros((n, n)))
    assert np.all(np.diag(Rh) > 0)
    return Qh, Rh, orth, res


# (m, n, s, kappa, seed): several 64-row panels plus ragged tails, every NMAX
# bucket (8, 16, 32, 48, 64), s = n, s = 3n, s > 512 (generic sketch kernel),
# m = 2n, a single row panel, n = 1.  (A square A is not a case: sampling with
# replacement then misses rows with high probability and the sketch is rank
# deficient.)
CASES = [
    (1, 1, 1, 1.0, 0),
    (37, 1, 3, 1.0, 1),
    (100, 3, 9, 1e4, 2),
    (1000, 8, 24, 1e8, 3),
    (1037, 13, 39, 1e12, 4),
    (4099, 16, 48, 1e15, 5),
    (5000, 24, 72, 1e8, 6),
    (6001, 32, 96, 1e10, 7),
    (3000, 40, 120, 1e6, 8),
    (2500, 48, 144, 1e14, 9),
    (10000, 50, 150, 1e8, 0),   # the 10,000 x 50 workload, s = 3n
    (7777, 64, 192, 1e15, 11),
    (128, 64, 640, 1e3, 12),    # m = 2n, generic sketch kernel
    (100000, 20, 20, 1e5, 13),  # s = n
    (130, 20, 40, 1e5, 13),
    (20000, 64, 520, 1e12, 14),  # generic sketch kernel
    (3000, 5, 1536, 1e9, 15),   # generic sketch kernel, largest s
    (65, 33, 99, 1e2, 16),
]

# 64 < n <= 128: the two-half row solve (A1 bit-exact across the half boundary),
# the separate Gram pass and the LDS-resident pass B; ragged column counts, s = n,
# s = 3n, the largest s the generic sketch kernel takes, a single row-panel group.
WIDE_CASES = [
    (3000, 65, 195, 1e8, 20),
    (5001, 96, 288, 1e12, 21),
    (4099, 100, 300, 1e15, 22),
    (20000, 128, 384, 1e14, 23),
    (100000, 96, 96, 1e5, 24),      # s = n (m large, so the sample has no repeated rows)
    (2000, 128, 1536, 1e6, 25),     # largest s
    (200, 70, 210, 1e3, 26),        # a single row-panel group, m < 4 * 64
    (100003, 112, 336, 1e10, 27),
    (5000, 80, 160, 1e10, 28),      # s in 129..192: the 12-row register sketch of the wide class
]


# 128 < n <= 512: the panel sketch (32-column panels, reflectors applied column
# by column to the later panels), the MFMA row-panel solve (64-column panels,
# earlier panels of A1 read back), the 128 x 128 Gram groups, the Cholesky with
# G in global memory and the MFMA pass B.  Ragged n (129, 200, 300), every
# padded width (256, 384, 512), every sketch rows-per-lane class (32 .. 96),
# the largest s of the register sketch, a single row-panel group, s = 2n; and
# s = 1537 .. 6144 through the wave-per-column sketch (L = 32, 64, 96 rows per
# lane row) and s = 6145 .. 8192 through the streaming sketch.
BIG_CASES = [
    (3000, 129, 387, 1e8, 30),
    (20001, 200, 600, 1e12, 31),
    (12000, 256, 768, 1e15, 32),
    (5000, 300, 900, 1e6, 33),
    (4000, 384, 1152, 1e10, 34),
    (6000, 512, 1536, 1e10, 35),
    (40000, 256, 512, 1e5, 36),     # s = 2n
    (1000, 140, 1536, 1e3, 37),     # largest s, few rows
    (230, 130, 390, 1e4, 38),       # a single row-panel group
    (3001, 160, 260, 1e9, 39),      # s in 257..384 (24 rows per lane)
    # s > 1536: the streaming panel sketch (sample columns in the workspace)
    (20000, 150, 1537, 1e8, 50),    # one row past the register sketch
    (30000, 300, 3000, 1e12, 51),   # s = 10n
    (12000, 512, 5120, 1e10, 52),   # s = 10n at the largest n
    (9000, 130, 8192, 1e4, 53),     # largest s, ragged n
    (7000, 140, 6144, 1e7, 54),     # largest s of the wave-per-column sketch
    (7000, 140, 6145, 1e7, 55),     # one row past it (streaming sketch)
]


# 512 < n <= 1024: padded widths 640 .. 1024 (pass B on 32-row iterations, the
# Cholesky with G in global memory, up to 36 Gram groups), s = 3n through the
# wave-per-column sketch.
WIDER_CASES = [
    (4000, 513, 1539, 1e8, 60),
    (3000, 640, 1920, 1e12, 61),
    (5000, 768, 2304, 1e10, 62),
    (3001, 1000, 3000, 1e6, 63),
    (4000, 1024, 3072, 1e15, 64),
]


@pytest.mark.parametrize("m,n,s,kappa,seed", BIG_CASES + WIDER_CASES)
def test_parity_big(m, n, s, kappa, seed):
    A_h = gen_usv(m, n, kappa, 100 + seed)
    _, _, orth, res = check_case(A_h, s, seed)
    assert orth < (1e-12 if s >= 2 * n else 1e-10)
    assert res < 1e-15


# Smoothed sampling (F = H D): the sample of the transformed matrix is formed in
# a fixed order, so idx, A_s, R_s and A1 stay bit-exact; one chunk (m <= 4096),
# several chunks, chunks of two blocks (m > 4096 * 256), every column class.
SMOOTH_CASES = [
    (3000, 24, 72, 1e8, 40),
    (10000, 64, 192, 1e15, 41),
    (20001, 100, 300, 1e12, 42),
    (6000, 200, 600, 1e10, 43),
    (1_200_000, 16, 48, 1e6, 44),
    (5000, 5, 1536, 1e4, 45),
]


@pytest.mark.parametrize("m,n,s,kappa,seed", SMOOTH_CASES)
def test_parity_smoothed(m, n, s, kappa, seed):
    A_h = gen_usv(m, n, kappa, 100 + seed)
    _, _, orth, res = check_case(A_h, s, seed, smooth=True)
    assert orth < 1e-12 and res < 1e-15


def coherent(m, n, kappa, seed):
    """Section 5.1's test matrices A = [I_n; 0] R_A, R_A with geometric singular
    values and Haar singular vectors (Matlab's randsvd)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    U, Ru = np.linalg.qr(rng.standard_normal((n, n)))
    V, Rv = np.linalg.qr(rng.standard_normal((n, n)))
    U, V = U * np.sign(np.diag(Ru))[None, :], V * np.sign(np.diag(Rv))[None, :]
    from workloads import sigma_profile

    A = np.zeros((m, n))
    A[:n] = (U * sigma_profile(n, kappa)[None, :]) @ V.T
    return np.asfortranarray(A)


@pytest.mark.parametrize("m,n", [(6000, 100), (6000, 300)])
def test_coherent_matrix_with_and_without_smoothing(m, n):
    A_h = coherent(m, n, 1e15, 3)
    announce(f"coherent [I;0] R_A {m}x{n}")
    # Without smoothing the sample holds few of the n informative rows: the sketch
    # is rank deficient, which shows as an exactly zero Householder column
    # (ESKETCH) or, when rounding leaves residue there, as a failed Cholesky
    # pivot of the then useless preconditioner (ECHOL); the oracle fails alike.
    ref = oracle.rpcholqr(A_h, 3 * n, 1, nthreads=NTHREADS, keep=False)
    assert ref.status in (oracle.ESKETCH, oracle.ECHOL)
    with pytest.raises(rq().RpCholQRError) as e:
        rq().factor(dev(A_h), 3 * n, 1)
    assert e.value.code == ref.status
    if ref.status == oracle.ESKETCH:
        assert e.value.index == ref.index
    Qh, Rh, orth, res = check_case(A_h, 3 * n, 1, smooth=True)
    assert orth < 1e-12 and res < 1e-15


@pytest.mark.parametrize("m,n,s,kappa,seed", CASES)
def test_parity_small(m, n, s, kappa, seed):
    A_h = gen_usv(m, n, kappa, 100 + seed)
    _, _, orth, res = check_case(A_h, s, seed)
    # Section 5.1: orth <= 1e-12 and residual below 1e-15 with c = 3n samples; with
    # fewer samples kappa(A1) grows and so does the orthogonality error (Section 5.2).
    assert orth < (1e-12 if s >= 2 * n else 1e-10)
    assert res < 1e-15


@pytest.mark.parametrize("m,n,s,kappa,seed", WIDE_CASES)
def test_parity_wide(m, n, s, kappa, seed):
    A_h = gen_usv(m, n, kappa, 100 + seed)
    _, _, orth, res = check_case(A_h, s, seed)
    assert orth < (1e-12 if s >= 2 * n else 1e-10)
    assert res < 1e-15


def test_deterministic_bits():
    A_h = gen_usv(20000, 64, 1e12, 3)
    A = dev(A_h)
    announce("determinism 20000x64")
    Q1, R1, _ = rq().factor(A, 192, 5)
    Q2, R2, _ = rq().factor(A, 192, 5)
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)


# One case per register-sketch class (4, 8, 12, 16 and 24 sample rows per lane)
# and a ragged s: the debug entry point (which also copies out the
# intermediates) must give the same Q and R bits as the plain one.
@pytest.mark.parametrize("m,n,s", [(5000, 20, 60), (7001, 40, 120), (100000, 64, 192), (9000, 48, 250),
                                   (20000, 64, 384), (3000, 7, 21)])
def test_debug_entry_matches_plain_entry(m, n, s):
    A = dev(gen_usv(m, n, 1e9, 17))
    announce(f"debug vs plain {m}x{n} s={s}")
    Q1, R1, _ = rq().factor(A, s, 4)
    Q2, R2, _, _ = rq().factor(A, s, 4, debug=True)
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)


def test_deterministic_bits_wide():
    A_h = gen_usv(30000, 112, 1e10, 4)
    A = dev(A_h)
    announce("determinism 30000x112")
    Q1, R1, _ = rq().factor(A, 336, 5)
    Q2, R2, _ = rq().factor(A, 336, 5)
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)


@pytest.mark.parametrize("m,n,s", [(50000, 64, 192), (20000, 100, 300), (20000, 300, 900), (8000, 200, 2000)])
def test_single_call_graph_capture(m, n, s):
    # rpcholqr_factor issues kernels only (no allocation, no memset), so a call
    # can be captured; every replay must give the eager result.
    A = dev(gen_usv(m, n, 1e8, 9))
    announce(f"graph capture {m}x{n}")
    Q0, R0, _ = rq().factor(A, s, 3)
    Q = rq().colmajor_empty(m, n, "cuda")
    R = rq().colmajor_empty(n, n, "cuda")
    ws = torch.empty(rq().workspace_bytes(m, n, s), dtype=torch.uint8, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    st = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        rq().factor(A, s, 3, Q=Q, R=R, workspace=ws, info=info, stream=st.cuda_stream, check=False)
        st.synchronize()
        with torch.cuda.graph(g, stream=st):
            rq().factor(A, s, 3, Q=Q, R=R, workspace=ws, info=info, stream=st.cuda_stream, check=False)
    for rep in range(3):
        Q.zero_()
        R.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert info.cpu().tolist() == [0, -1]
        assert torch.equal(Q, Q0) and torch.equal(R, R0), f"replay {rep}"


@pytest.mark.parametrize("pad,off,n", [(13, 0, 24), (14, 0, 24), (14, 1, 24), (13, 0, 100), (14, 1, 100),
                                       (13, 0, 300), (14, 1, 300)])
def test_leading_dimensions(pad, off, n):
    # Odd and even leading dimensions, and an A that starts 8 bytes into its
    # allocation, for a 64-column class, the 128-column class and n > 128.
    m = 3001
    s = 3 * n
    A_h = gen_usv(m, n, 1e6, 4)
    announce(f"padded leading dimensions pad={pad} off={off}")
    big = torch.full((n, m + pad), float("nan"), dtype=torch.float64, device="cuda").t()
    big[off:off + m] = dev(A_h)
    A = big[off:off + m]                            # lda = m + pad
    Q = torch.zeros((n, m + 5), dtype=torch.float64, device="cuda").t()[:m]
    R = torch.zeros((n + 3, n + 3), dtype=torch.float64, device="cuda").t()[:n, :n]
    rq().factor(A, s, 9, Q=Q, R=R)
    ref = oracle.rpcholqr(A_h, s, 9)
    assert metrics.rel_fro(host(Q), ref.Q) < TOL and metrics.rel_fro(host(R), ref.R) < TOL


@pytest.mark.parametrize("n,col", [(12, 7), (100, 90), (300, 250)])
def test_esketch_zero_column(n, col):
    A_h = gen_usv(2000, n, 1e3, 1)
    A_h[:, col] = 0.0
    announce(f"ESKETCH zero column {col} of {n}")
    with pytest.raises(rq().RpCholQRError) as e:
        rq().factor(dev(A_h), 3 * n, 0)
    assert e.value.code == 1 and e.value.index == col
    assert oracle.rpcholqr(A_h, 3 * n, 0).index == col


# Two zero columns: the first failure must end the sweep.  The second column lies
# in a later 16-step block (and, for n = 100, in phase 3 of the 128-column
# sketch), where a sweep that went on would report it instead.  s = 400 takes
# the generic sketch kernel.
@pytest.mark.parametrize("n,s,cols", [(24, 72, (3, 17)), (40, 120, (17, 33)), (24, 400, (3, 17)),
                                      (100, 300, (3, 17)), (100, 300, (65, 81)), (100, 300, (33, 99)),
                                      (200, 400, (3, 17)), (200, 400, (40, 150))])
def test_esketch_first_of_two_zero_columns(n, s, cols):
    A_h = gen_usv(3000, n, 1e3, 5)
    for c in cols:
        A_h[:, c] = 0.0
    announce(f"ESKETCH zero columns {cols} of {n}, s={s}")
    ref = oracle.rpcholqr(A_h, s, 0)
    assert ref.status == oracle.ESKETCH and ref.index == cols[0]
    with pytest.raises(rq().RpCholQRError) as e:
        rq().factor(dev(A_h), s, 0)
    assert e.value.code == 1 and e.value.index == cols[0]


@pytest.mark.parametrize("n,col", [(12, 3), (80, 70), (260, 200)])
def test_echol_nonfinite_unsampled_row(n, col):
    m, s = 2000, 3 * n
    A_h = gen_usv(m, n, 1e3, 2)
    missed = sorted(set(range(m)) - set(oracle.sample_indices(m, s, 0).tolist()))[5]
    A_h[missed, col] = np.nan
    announce(f"ECHOL NaN row, column {col} of {n}")
    with pytest.raises(rq().RpCholQRError) as e:
        rq().factor(dev(A_h), s, 0)
    ref = oracle.rpcholqr(A_h, s, 0)
    assert ref.status == oracle.ECHOL
    assert e.value.code == 2 and e.value.index == ref.index == col


def test_esketch_inf_in_sample():
    m, n, s = 2000, 12, 36
    A_h = gen_usv(m, n, 1e3, 3)
    A_h[oracle.sample_indices(m, s, 1)[4], 5] = np.inf
    announce("ESKETCH inf in sample")
    with pytest.raises(rq().RpCholQRError) as e:
        rq().factor(dev(A_h), s, 1)
    ref = oracle.rpcholqr(A_h, s, 1)
    assert e.value.code == 1 and e.value.index == ref.index


def test_argument_errors():
    lib = rq().load_library()
    m, n, s = 1000, 8, 24
    A = dev(gen_usv(m, n, 10.0, 1))
    Q = rq().colmajor_empty(m, n, "cuda")
    R = rq().colmajor_empty(n, n, "cuda")
    ws = torch.empty(rq().workspace_bytes(m, n, s), dtype=torch.uint8, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    nb = ws.numel()
    announce("argument errors")

    def call(m_=m, n_=n, s_=s, A_=A, lda=m, Q_=Q, ldq=m, R_=R, ldr=n, prec=0, ws_=P(ws), wsb=nb):
        return lib.rpcholqr_factor(m_, n_, s_, 0, P(A_), lda, P(Q_), ldq, P(R_), ldr, prec, ws_, wsb, P(info), st)

    assert call(lda=m - 1) == -1
    assert call(ldq=m - 1) == -1
    assert call(ldr=n - 1) == -1
    assert call(s_=n - 1) == -1
    assert call(m_=n - 1, lda=n - 1, ldq=n - 1) == -1
    assert call(Q_=A) == -1                       # Q overlaps A
    assert call(wsb=nb - 8) == -3
    assert call(prec=1) == -3                    # FP32_REFINE needs a larger workspace
    assert call(prec=2) == -3                    # BF16X2_REFINE likewise
    assert call(prec=7) == -4
    big_n = rq().max_n() + 1
    assert lib.rpcholqr_factor(10 * big_n, big_n, 3 * big_n, 0, P(A), 10 * big_n, P(Q), 10 * big_n, P(R), big_n,
                               0, P(ws), nb, P(info), st) == -4
    torch.cuda.synchronize()
    assert call() == 0
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, -1]


def test_factor_on_a_caller_stream():
    # The workspace allocated inside factor() is used on the caller's stream and
    # freed on return (check=False); the result must still be the plain call's.
    m, n, s = 200000, 48, 144
    A_h = gen_usv(m, n, 1e6, 13)
    A = dev(A_h)
    announce("caller stream")
    Q0, R0, _ = rq().factor(A, s, 3)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    outs = []
    for _ in range(3):
        outs.append(rq().factor(A, s, 3, stream=side.cuda_stream, check=False))
        torch.empty(1 << 22, dtype=torch.uint8, device="cuda").fill_(255)  # reuse freed memory on the default stream
    side.synchronize()
    for Q, R, info in outs:
        assert info.cpu().tolist() == [0, -1]
        assert torch.equal(Q, Q0) and torch.equal(R, R0)


def test_timing_api_counts_calls():
    m, n, s = 50000, 32, 96
    A = dev(gen_usv(m, n, 1e4, 2))
    announce("timing API")
    rq().timing_enable(True)
    for _ in range(3):
        rq().factor(A, s, 1, check=False)
    calls, ms = rq().timing_read()
    rq().timing_enable(False)
    assert calls == 3 and all(v > 0 for v in ms.values())


KAPPAS = [1.0, 1e4, 1e8, 1e12, 1e15]


@pytest.mark.parametrize("kappa", KAPPAS)
def test_parity_full_size_1e6x64(kappa):
    # The 1,000,000 x 64 workload with s = 3n = 192: full comparison against the oracle,
    # bit-exact A1 on every row, and the paper's accuracy claims (Section 5.1 summary).
    m, n, s = 1_000_000, 64, 192
    A_h = gen_usv(m, n, kappa, 0)
    Qh, Rh, orth, res = check_case(A_h, s, 0)
    print(f"  kappa={kappa:.0e}: orth={orth:.3e} residual={res:.3e}", flush=True)
    assert orth <= 1e-12 and res <= 1e-15


@pytest.mark.parametrize("kappa", [1e8, 1e15])
def test_parity_full_size_1e6x128(kappa):
    # The 128-column class at 1,000,000 rows (s = 3n = 384): bit-exact idx, A_s,
    # R_s and A1 across the half boundary of the row solve on every row.
    m, n, s = 1_000_000, 128, 384
    A_h = gen_usv(m, n, kappa, 0)
    Qh, Rh, orth, res = check_case(A_h, s, 0)
    print(f"  kappa={kappa:.0e}: orth={orth:.3e} residual={res:.3e}", flush=True)
    assert orth <= 1e-12 and res <= 1e-15


def test_parity_small_reference_configuration():
    # The small single-matrix workload exactly: 10,000 x 50, s = 3n = 150,
    # kappa = 1e8, matrix seed 0, sampling seed 0.
    A_h = gen_usv(10_000, 50, 1e8, 0)
    _, _, orth, res = check_case(A_h, 150, 0)
    assert orth <= 1e-12 and res <= 1e-15
