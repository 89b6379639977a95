"""rpcholqr_factor_noalloc (the entry point that allocates nothing, with its
workspace in a static device array) against rpcholqr_factor with a caller's
workspace, called through the C ABI: several calls in a row on the one array,
each later one smaller than the one before, so that a call that depended on the
array's leftover contents would show.  The first (n = 300) needs fewer Gram
partials to fit the array, so it agrees to rounding rather than to the bit."""
import ctypes

import numpy as np
import pytest

from workloads import gen_usv, metrics

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-12


def lib():
    import paper_2406_11751_amd as rq

    return rq.load_library()


def dev(A_h):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A_h).T)).to("cuda").t()


def P(t):
    return ctypes.c_void_p(t.data_ptr())


def colmajor(m, n):
    return torch.empty((n, m), dtype=torch.float64, device="cuda").t()


def stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def with_workspace(A, s, seed, prec):
    m, n = A.shape
    Q, R = colmajor(m, n), colmajor(n, n)
    info = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    wsb = lib().rpcholqr_workspace_bytes(m, n, s, prec)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    rc = lib().rpcholqr_factor(m, n, s, seed, P(A), m, P(Q), m, P(R), n, prec, P(ws), wsb, P(info), stream())
    assert rc == 0
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, -1]
    return Q, R


def no_alloc(A, s, seed, prec):
    m, n = A.shape
    # outputs pre-filled with NaN: every entry must be written by the call
    Q = colmajor(m, n).fill_(float("nan"))
    R = colmajor(n, n).fill_(float("nan"))
    info = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    rc = lib().rpcholqr_factor_noalloc(m, n, s, seed, P(A), m, P(Q), m, P(R), n, prec, P(info), stream())
    assert rc == 0
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, -1]
    return Q, R


# (m, n, s, kappa, precision): decreasing sizes; the 128-column class, the
# 64-column class, a refined precision and a small ragged case.
CALLS = [(60_000, 300, 900, 1e10, 0), (400_000, 100, 300, 1e10, 0), (300_001, 64, 192, 1e12, 0),
         (100_003, 48, 144, 1e8, 1), (5_000, 24, 72, 1e6, 0)]


def test_no_alloc_matches_workspace_entry_point():
    for i, (m, n, s, kappa, prec) in enumerate(CALLS):
        print(f"case: no-alloc call {i}: m={m} n={n} s={s} precision={prec}", flush=True)
        A = dev(gen_usv(m, n, kappa, 50 + i))
        Qw, Rw = with_workspace(A, s, 9 + i, prec)
        Qn, Rn = no_alloc(A, s, 9 + i, prec)
        assert metrics.rel_fro(Qn.cpu().numpy(), Qw.cpu().numpy()) < TOL
        assert metrics.rel_fro(Rn.cpu().numpy(), Rw.cpu().numpy()) < TOL
        if n <= 128:  # these fit the array with the usual partial count: the same bits
            assert torch.equal(Qn, Qw) and torch.equal(Rn, Rw)
        assert metrics.orth_error(Qn) < 1e-12


def test_no_alloc_argument_errors():
    m, n, s = 1000, 8, 24
    A = dev(gen_usv(m, n, 10.0, 1))
    Q, R = colmajor(m, n), colmajor(n, n)
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    f = lib().rpcholqr_factor_noalloc
    print("case: no-alloc argument errors", flush=True)
    assert f(m, n, s, 0, P(A), m - 1, P(Q), m, P(R), n, 0, P(info), stream()) == -1  # lda < m
    assert f(m, n, n - 1, 0, P(A), m, P(Q), m, P(R), n, 0, P(info), stream()) == -1  # s < n
    assert f(m, n, s, 0, P(A), m, P(A), m, P(R), n, 0, P(info), stream()) == -1      # Q overlaps A
    assert f(m, n, s, 0, P(A), m, P(Q), m, P(R), n, 7, P(info), stream()) == -4      # unknown precision
    big = lib().rpcholqr_max_n() + 1
    assert f(10 * big, big, 3 * big, 0, P(A), 10 * big, P(Q), 10 * big, P(R), big, 0, P(info), stream()) == -4
    torch.cuda.synchronize()
