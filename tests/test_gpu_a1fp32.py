"""GPU checks of RPCHOLQR_A1_FP32: A1 computed in FP64 (bit-identical to the
oracle's) and kept in FP32 inside the Q buffer between the two passes.

What is fixed exactly: idx, A_s and R_s equal the oracle's; the stored A1 equals
the oracle's A1 rounded to float (round to nearest on both sides).  What follows
from it within rounding: G1 is the FP64 Gram of those float values, R2 its
Cholesky factor, Q = A1_f32 R2^{-1} and R = R2 R_s.  The accuracy claims: Q as
orthogonal as in FP64 (<= 1e-13), and ||A - QR|| / ||A|| at the float level
(the rounding of A1 enters the residual only; Theorem t_perturb2)."""
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from workloads import gen_usv, metrics

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NTHREADS = max(1, min(16, len(os.sched_getaffinity(0))))
U32 = 2.0 ** -24


def rq():
    import paper_2406_11751_amd

    return paper_2406_11751_amd


def dev(A_h):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A_h).T)).to("cuda").t()


def host(t):
    return t.cpu().numpy()


def announce(*args):
    print("case:", *args, flush=True)


CASES = [
    (1, 1, 1, 1.0, 0), (37, 1, 3, 1.0, 1), (1000, 8, 24, 1e8, 3), (4099, 16, 48, 1e15, 5),
    (6001, 32, 96, 1e10, 7), (2500, 48, 144, 1e14, 9), (10000, 50, 150, 1e8, 0), (7777, 64, 192, 1e15, 11),
    (20000, 64, 520, 1e12, 14), (65, 33, 99, 1e2, 16), (20001, 64, 192, 1.0, 17),
]


def check(A_h, s, seed, smooth=False):
    m, n = A_h.shape
    announce(f"A1_FP32 m={m} n={n} s={s} seed={seed} smooth={smooth}")
    prec = rq().A1_FP32 | (rq().SMOOTH if smooth else 0)
    Q, R, _, ex = rq().factor(dev(A_h), s, seed, debug=True, precision=prec)
    ref = oracle.rpcholqr(A_h, s, seed, nthreads=NTHREADS, smooth=smooth)
    assert ref.status == oracle.OK
    assert np.array_equal(host(ex["idx"]), ref.idx)
    assert np.array_equal(host(ex["As"]), ref.As)
    assert np.array_equal(host(ex["Rs"]), ref.Rs)
    a1 = host(ex["A1"])
    assert np.array_equal(a1, ref.A1.astype(np.float32).astype(np.float64)), "stored A1 is not fl32(A1)"
    G1, R2 = host(ex["G1"]), host(ex["R2"])
    Gx = a1.T @ a1
    assert metrics.rel_fro(np.triu(G1), np.triu(Gx)) < 1e-13
    assert metrics.rel_fro(R2.T @ R2, Gx) < 1e-13
    Qh, Rh = host(Q), host(R)
    Qx = scipy.linalg.solve_triangular(R2, a1.T, trans="T", lower=False).T
    assert metrics.rel_fro(Qh, Qx) < 1e-12
    assert metrics.rel_fro(Rh, R2 @ ref.Rs) < 1e-12
    assert np.array_equal(np.tril(Rh, -1), np.zeros((n, n))) and np.all(np.diag(Rh) > 0)
    orth, res = metrics.orth_error(Qh), metrics.residual(A_h, Qh, Rh)
    # R against the FP64 oracle: the float rounding of A1 moves R at the float level
    dR = metrics.rel_fro(Rh, ref.R)
    print(f"  orth={orth:.2e} residual={res:.2e} |dR| vs FP64 oracle={dR:.2e}", flush=True)
    assert orth < 1e-13
    assert res < 8 * U32 * max(1.0, np.sqrt(n))
    assert dR < 1e-5
    return orth, res


@pytest.mark.parametrize("m,n,s,kappa,seed", CASES)
def test_a1_fp32(m, n, s, kappa, seed):
    check(gen_usv(m, n, kappa, 500 + seed), s, seed)


def test_a1_fp32_smoothed():
    check(gen_usv(30000, 40, 1e12, 77), 120, 3, smooth=True)


@pytest.mark.parametrize("kappa", [1e8, 1e15])
def test_a1_fp32_full_size_1e6x64(kappa):
    check(gen_usv(1_000_000, 64, kappa, 0), 192, 0)


def test_a1_fp32_is_faster_in_place_and_unsupported_sizes():
    # the float copy is written inside Q's own rows: a Q with ldq > m (padding
    # rows never touched) gives the same result as a tight one
    m, n, s = 5003, 40, 120
    A_h = gen_usv(m, n, 1e9, 3)
    A = dev(A_h)
    Q1, R1, _ = rq().factor(A, s, 2, precision=rq().A1_FP32)
    Qpad = torch.full((n, m + 77), float("nan"), dtype=torch.float64, device="cuda").t()
    Q2, R2, _ = rq().factor(A, s, 2, Q=Qpad[:m], precision=rq().A1_FP32)
    assert np.array_equal(host(Q1), host(Q2)) and np.array_equal(host(R1), host(R2))
    assert torch.isnan(Qpad[m:]).all()
    for n_bad in (65, 200):
        with pytest.raises(rq().RpCholQRError) as e:
            rq().factor(dev(gen_usv(3000, n_bad, 10.0, 1)), 3 * n_bad, 0, precision=rq().A1_FP32)
        assert e.value.status == -4
