"""GPU parity of rpcholqr_precond_factor (Algorithm "Preconditioned Cholesky-QR",
Section 3.1, with a caller-supplied R_s) against the oracle's alg1, and its
consistency with rpcholqr_factor when given the sketch's R_s."""
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
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A_h).T)).to("cuda").t()


def host(t):
    return t.cpu().numpy()


def announce(*args):
    print("case:", *args, flush=True)


@pytest.mark.parametrize("m,n,s,kappa,seed", [(5000, 24, 72, 1e8, 1), (20000, 64, 192, 1e12, 2),
                                              (3001, 100, 300, 1e10, 3), (1000, 128, 384, 1e6, 4),
                                              (4000, 300, 900, 1e12, 5)])
def test_sketch_preconditioner_reproduces_factor(m, n, s, kappa, seed):
    # Given the sketch's own R_s, Algorithm 1 is the rest of rpCholesky-QR: the
    # same A1, G1, R2 and R to the bit.  Line 6 differs in method (substitution
    # here, the explicit R2^{-1} in rpcholqr_factor), so Q agrees to rounding.
    A_h = gen_usv(m, n, kappa, 300 + seed)
    A = dev(A_h)
    announce(f"precond = factor, m={m} n={n}")
    Q1, R1, _, ex = rq().factor(A, s, seed, debug=True)
    Q2, R2, _ = rq().precond_factor(A, ex["Rs"])
    assert torch.equal(R1, R2)
    assert metrics.rel_fro(host(Q2), host(Q1)) < 1e-14
    ref = oracle.alg1(A_h, host(ex["Rs"]), nthreads=NTHREADS)
    assert metrics.rel_fro(host(Q2), ref.Q) < TOL and metrics.rel_fro(host(R2), ref.R) < TOL


@pytest.mark.parametrize("m,n,kappa,seed", [(4000, 16, 1e6, 5), (10000, 50, 1e8, 6), (2500, 96, 1e10, 7),
                                            (3000, 200, 1e10, 8), (3000, 700, 1e8, 9)])
def test_against_oracle_alg1_with_signed_preconditioner(m, n, kappa, seed):
    # A preconditioner that is not sign-normalized: the sketch's R_s with every
    # third row negated (Algorithm 1 takes any nonsingular upper triangular R_s).
    A_h = gen_usv(m, n, kappa, 400 + seed)
    Rs = oracle.rpcholqr(A_h, 3 * n, seed, nthreads=NTHREADS).Rs.copy()
    Rs[::3, :] *= -1.0
    announce(f"alg1 m={m} n={n}")
    Q, R, _ = rq().precond_factor(dev(A_h), dev(Rs))
    ref = oracle.alg1(A_h, Rs, nthreads=NTHREADS)
    assert ref.status == oracle.OK
    assert metrics.rel_fro(host(Q), ref.Q) < TOL and metrics.rel_fro(host(R), ref.R) < TOL
    assert metrics.orth_error(host(Q)) < 1e-12 and metrics.residual(A_h, host(Q), host(R)) < 1e-15
    assert np.any(np.diag(host(R)) < 0)  # the signs of R_s carry over to R = R2 R_s


# Algorithm "Basic Cholesky-QR" (Section 2.1) is Preconditioned Cholesky-QR with
# R_s = I: A1 = A, G1 = A^T A.  Theorem t_perturb1 (Section 2.2) puts its loss of
# orthogonality at the scale u kappa(A)^2 and needs kappa(A)^2 u well below one;
# at kappa = 1e15 the Cholesky of A^T A breaks down, while the randomized
# preconditioner of rpCholesky-QR keeps kappa(A1) small (Section 5.1).
U64 = 2.0 ** -53


@pytest.mark.parametrize("n", [16, 64, 100, 160])
def test_basic_cholqr_loses_orthogonality_as_kappa_squared(n):
    m, kappa = 20000, 1e3
    A_h = gen_usv(m, n, kappa, 11)
    eye = np.eye(n)
    announce(f"basic Cholesky-QR m={m} n={n} kappa={kappa:.0e}")
    Q, R, _ = rq().precond_factor(dev(A_h), dev(eye))
    ref = oracle.alg1(A_h, eye, nthreads=NTHREADS)
    assert ref.status == oracle.OK
    scale = kappa ** 2 * U64
    orth = metrics.orth_error(host(Q))
    # far above rpCholesky-QR's 1e-15, at most a modest multiple of u kappa^2
    assert 1e-13 < orth < 100 * scale, orth
    assert metrics.orth_error(ref.Q) < 100 * scale
    # the two results are both correct to the perturbation scale of the theorem
    assert metrics.rel_fro(host(R), ref.R) < scale and metrics.rel_fro(host(Q), ref.Q) < scale
    assert metrics.residual(A_h, host(Q), host(R)) < 1e-15
    # R_s = I makes A1 = A, so R = R2 and Q R reproduces A to rounding
    assert np.all(np.diag(host(R)) > 0)


def test_basic_cholqr_breaks_down_where_rpcholqr_does_not():
    m, n, kappa = 20000, 64, 1e15
    A_h = gen_usv(m, n, kappa, 12)
    announce(f"basic Cholesky-QR breakdown m={m} n={n} kappa={kappa:.0e}")
    ref = oracle.alg1(A_h, np.eye(n), nthreads=NTHREADS)
    assert ref.status == oracle.ECHOL
    with pytest.raises(rq().RpCholQRError) as e:
        rq().precond_factor(dev(A_h), dev(np.eye(n)))
    # which pivot fails first depends on rounding in A^T A; that one fails does not
    assert e.value.code == 2 and 0 <= e.value.index < n
    Q, R, _ = rq().factor(dev(A_h), 3 * n, 0)
    assert metrics.orth_error(host(Q)) < 1e-12
    assert metrics.residual(A_h, host(Q), host(R)) < 1e-15


def test_refined_precision_with_given_preconditioner():
    m, n = 20000, 48
    A_h = gen_usv(m, n, 1e12, 8)
    Rs = oracle.rpcholqr(A_h, 3 * n, 8, nthreads=NTHREADS).Rs
    ref = oracle.alg1(A_h, Rs, nthreads=NTHREADS)
    for prec in (rq().FP32_REFINE, rq().BF16X2_REFINE):
        announce(f"alg1 precision {prec}")
        Q, R, _ = rq().precond_factor(dev(A_h), dev(Rs), precision=prec)
        assert metrics.rel_fro(host(Q), ref.Q) < TOL and metrics.rel_fro(host(R), ref.R) < TOL


def test_precond_argument_errors():
    lib = rq().load_library()
    m, n = 1000, 8
    A = dev(gen_usv(m, n, 10.0, 1))
    Rs = dev(np.triu(np.eye(n) + 0.1))
    Q = rq().colmajor_empty(m, n, "cuda")
    R = rq().colmajor_empty(n, n, "cuda")
    ws = torch.empty(rq().workspace_bytes(m, n, n), dtype=torch.uint8, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    announce("precond argument errors")

    def call(Rs_=P(Rs), ldrs=n, wsb=ws.numel()):
        return lib.rpcholqr_precond_factor(m, n, P(A), m, Rs_, ldrs, P(Q), m, P(R), n, 0, P(ws), wsb, P(info), st)

    assert call(Rs_=None) == -1
    assert call(ldrs=n - 1) == -1
    assert call(wsb=ws.numel() - 8) == -3
    assert call() == 0
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, -1]
