"""GPU parity of the batched entry points (rpcholqr_batched_*, rpcholqr_factor_batched).

Every problem of a batch is checked against the CPU oracle (Q and R within
1e-12 relative Frobenius error, orthogonality and residual) and against the
single-problem entry point; failures of single problems must stay confined to
their own info entry.
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
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A_h).T)).to("cuda").t()


def host(t):
    return t.cpu().numpy()


def announce(*args):
    print("case:", *args, flush=True)


# (m, n, s, kappa): every column class (16, 32, 48, 64), several sketch kernels
# (s <= 64 ... s > 384), ragged row tails, a single partial row panel, n = 1,
# s = n, and sizes that give one and many pass-A workgroups per problem.
MIXED = [
    (1, 1, 1, 1.0), (37, 1, 3, 1.0), (100, 3, 9, 1e4), (1000, 8, 24, 1e8), (1037, 13, 39, 1e12),
    (4099, 16, 48, 1e15), (5000, 24, 72, 1e8), (6001, 32, 96, 1e10), (3000, 40, 120, 1e6),
    (2500, 48, 144, 1e14), (10000, 50, 150, 1e8), (7777, 64, 192, 1e15), (128, 64, 640, 1e3),
    (60000, 20, 20, 1e5), (130, 20, 40, 1e5), (20000, 64, 520, 1e12), (3000, 5, 1536, 1e9),
    (65, 33, 99, 1e2), (150000, 64, 192, 1e8), (70000, 17, 51, 1e13),
    (5001, 96, 288, 1e12), (20000, 128, 384, 1e14), (300, 65, 195, 1e4), (2000, 128, 1536, 1e6),
]


def run_batch(problems, seeds):
    As_h = [gen_usv(m, n, k, 1000 + i) for i, (m, n, s, k) in enumerate(problems)]
    As = [dev(A) for A in As_h]
    plan = rq().BatchedPlan(As, [p[2] for p in problems], seeds)
    return As_h, As, plan


def test_batched_mixed_sizes_against_oracle():
    seeds = [7 * i + 1 for i in range(len(MIXED))]
    announce(f"mixed batch of {len(MIXED)}")
    As_h, As, plan = run_batch(MIXED, seeds)
    info = plan.execute()
    assert np.array_equal(host(info), np.tile([0, -1], (len(MIXED), 1)))
    for i, ((m, n, s, k), A_h) in enumerate(zip(MIXED, As_h)):
        announce(f"problem {i}: m={m} n={n} s={s}")
        ref = oracle.rpcholqr(A_h, s, seeds[i], nthreads=NTHREADS)
        Qh, Rh = host(plan.Qs[i]), host(plan.Rs[i])
        eq, er = metrics.rel_fro(Qh, ref.Q), metrics.rel_fro(Rh, ref.R)
        orth, res = metrics.orth_error(Qh), metrics.residual(A_h, Qh, Rh)
        print(f"  |dQ|={eq:.2e} |dR|={er:.2e} orth={orth:.2e} res={res:.2e}", flush=True)
        assert eq < TOL and er < TOL
        assert orth < (1e-12 if s >= 2 * n else 1e-10) and res < 1e-15
        assert np.array_equal(np.tril(Rh, -1), np.zeros((n, n)))
        # the single-problem entry point on the same input
        Q1, R1, _ = rq().factor(As[i], s, seeds[i])
        assert metrics.rel_fro(host(Q1), Qh) < 1e-13 and metrics.rel_fro(host(R1), Rh) < 1e-13
    plan.close()


def test_batched_reexecution_is_deterministic():
    probs = MIXED[3:12]
    announce("re-execution")
    _, _, plan = run_batch(probs, list(range(len(probs))))
    plan.execute()
    Q0 = [q.clone() for q in plan.Qs]
    R0 = [r.clone() for r in plan.Rs]
    for q in plan.Qs:
        q.zero_()
    plan.execute()
    for a, b in zip(Q0, plan.Qs):
        assert torch.equal(a, b)
    for a, b in zip(R0, plan.Rs):
        assert torch.equal(a, b)
    plan.close()


def test_batched_failures_stay_in_their_problem():
    m, n, s = 2000, 12, 36
    good = [gen_usv(3000, 16, 1e6, 50 + i) for i in range(3)]
    bad_sketch = gen_usv(m, n, 1e3, 1)
    bad_sketch[:, 7] = 0.0
    bad_chol = gen_usv(m, n, 1e3, 2)
    missed = sorted(set(range(m)) - set(oracle.sample_indices(m, s, 5).tolist()))[5]
    bad_chol[missed, 3] = np.nan
    As_h = [good[0], bad_sketch, good[1], bad_chol, good[2]]
    ss = [48, s, 48, s, 48]
    seeds = [1, 4, 2, 5, 3]
    announce("failure isolation")
    plan = rq().BatchedPlan([dev(A) for A in As_h], ss, seeds)
    info = host(plan.execute(check=False))
    refs = [oracle.rpcholqr(A, si, sd, nthreads=NTHREADS) for A, si, sd in zip(As_h, ss, seeds)]
    assert refs[1].status == oracle.ESKETCH and refs[3].status == oracle.ECHOL
    assert info[1].tolist() == [1, refs[1].index] and info[3].tolist() == [2, refs[3].index]
    for i in (0, 2, 4):
        assert info[i].tolist() == [0, -1]
        assert metrics.rel_fro(host(plan.Qs[i]), refs[i].Q) < TOL
        assert metrics.rel_fro(host(plan.Rs[i]), refs[i].R) < TOL
    with pytest.raises(rq().RpCholQRError):
        plan.execute(check=True)
    plan.close()


def test_batched_failures_in_the_wide_class():
    # ESKETCH (a zero column beyond 64) and ECHOL (NaN in an unsampled row, column
    # beyond 64) in 128-column-class problems next to good ones of both classes.
    m, n, s = 3000, 100, 300
    good = [gen_usv(m, n, 1e6, 60), gen_usv(4000, 40, 1e4, 61)]
    bad_sketch = gen_usv(m, n, 1e3, 62)
    bad_sketch[:, 90] = 0.0
    bad_chol = gen_usv(m, n, 1e3, 63)
    missed = sorted(set(range(m)) - set(oracle.sample_indices(m, s, 8).tolist()))[3]
    bad_chol[missed, 70] = np.nan
    As_h = [good[0], bad_sketch, good[1], bad_chol]
    ss = [s, s, 120, s]
    seeds = [6, 7, 9, 8]
    announce("failure isolation, 128-column class")
    plan = rq().BatchedPlan([dev(A) for A in As_h], ss, seeds)
    info = host(plan.execute(check=False))
    refs = [oracle.rpcholqr(A, si, sd, nthreads=NTHREADS) for A, si, sd in zip(As_h, ss, seeds)]
    assert refs[1].status == oracle.ESKETCH and refs[3].status == oracle.ECHOL
    assert info[1].tolist() == [1, refs[1].index] and info[3].tolist() == [2, refs[3].index]
    for i in (0, 2):
        assert info[i].tolist() == [0, -1]
        assert metrics.rel_fro(host(plan.Qs[i]), refs[i].Q) < TOL
        assert metrics.rel_fro(host(plan.Rs[i]), refs[i].R) < TOL
    plan.close()


def test_batched_factor_convenience_and_graph_capture():
    probs = MIXED[5:9]
    As_h = [gen_usv(m, n, k, 300 + i) for i, (m, n, s, k) in enumerate(probs)]
    As = [dev(A) for A in As_h]
    ss = [p[2] for p in probs]
    announce("factor_batched + graph capture")
    Qs, Rs, info = rq().factor_batched(As, ss, 11)
    plan = rq().BatchedPlan(As, ss, 11)
    info2 = torch.zeros((len(probs), 2), dtype=torch.int32, device="cuda")
    st = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        plan.execute(info=info2, stream=st.cuda_stream, check=False)  # warm-up outside capture
        st.synchronize()
        for q in plan.Qs:
            q.zero_()
        with torch.cuda.graph(g, stream=st):
            plan.execute(info=info2, stream=st.cuda_stream, check=False)
    for rep in range(3):
        for q in plan.Qs:
            q.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert host(info2).tolist() == [[0, -1]] * len(probs)
        for a, b in zip(Qs, plan.Qs):
            assert torch.equal(a, b), f"replay {rep}"
        for a, b in zip(Rs, plan.Rs):
            assert torch.equal(a, b), f"replay {rep}"
    plan.close()


def test_batched_argument_errors():
    lib = rq().load_library()
    A = dev(gen_usv(1000, 8, 10.0, 1))
    Q = rq().colmajor_empty(1000, 8, "cuda")
    R = rq().colmajor_empty(8, 8, "cuda")
    big = rq().colmajor_empty(1000, 129, "cuda")
    Qb = rq().colmajor_empty(1000, 129, "cuda")
    Rb = rq().colmajor_empty(129, 129, "cuda")
    I64 = ctypes.c_int64 * 2
    P = ctypes.c_void_p * 2

    def create(n1=8, ldq1=1000, A1=A, s1=24):
        h = ctypes.c_void_p()
        bad = ctypes.c_int64(-9)
        rc = lib.rpcholqr_batched_plan_create(
            2, I64(1000, 1000), I64(8, n1), I64(24, s1), (ctypes.c_uint64 * 2)(1, 2),
            P(A.data_ptr(), A1.data_ptr()), I64(1000, 1000), P(Q.data_ptr(), Qb.data_ptr()), I64(1000, ldq1),
            P(R.data_ptr(), Rb.data_ptr()), I64(8, 129), 0, ctypes.byref(h), ctypes.byref(bad))
        if rc == 0:
            lib.rpcholqr_batched_plan_destroy(h)
        return rc, bad.value

    announce("batched argument errors")
    assert create() == (0, -1)
    assert create(n1=129, A1=big, s1=400) == (-4, 1)     # n beyond the supported maximum
    assert create(ldq1=999) == (-1, 1)                    # ldq < m
    assert create(s1=4) == (-1, 1)                        # s < n
    assert lib.rpcholqr_batched_execute(None, None, None) == -1
    assert lib.rpcholqr_batched_plan_destroy(None) == 0


def test_batched_config3_like_sample():
    """A reduced instance of the 2048-problem workload: m ~ U{2000..20000},
    n ~ U{8, 16, 32, 64}, log10 kappa ~ U[2, 14], s = 3n, seed i; every problem
    checked for orthogonality and residual, every 16th against the oracle."""
    rng = np.random.default_rng(0)
    B = 128
    ms = rng.integers(2000, 20001, size=B)
    ns = rng.choice([8, 16, 32, 64], size=B)
    ks = 10.0 ** rng.uniform(2, 14, size=B)
    As_h = [gen_usv(int(m), int(n), float(k), i) for i, (m, n, k) in enumerate(zip(ms, ns, ks))]
    announce(f"config-3-like batch of {B}")
    plan = rq().BatchedPlan([dev(A) for A in As_h], [3 * int(n) for n in ns], list(range(B)))
    plan.execute()
    for i in range(B):
        Qh, Rh = host(plan.Qs[i]), host(plan.Rs[i])
        orth, res = metrics.orth_error(Qh), metrics.residual(As_h[i], Qh, Rh)
        assert orth < 1e-12 and res < 1e-15, (i, orth, res)
        if i % 16 == 0:
            ref = oracle.rpcholqr(As_h[i], 3 * int(ns[i]), i, nthreads=NTHREADS)
            assert metrics.rel_fro(Qh, ref.Q) < TOL and metrics.rel_fro(Rh, ref.R) < TOL
    plan.close()


def test_batched_tuning_shapes_agree():
    """Launch shapes from rpcholqr_batched_set_tuning: one Gram partial and
    16-row pass-B workgroups for the 64-column class, many small partials for the
    128-column class; every problem still matches the oracle, and a malformed
    table is rejected without changing the installed one."""
    probs = [(30000, 64, 192, 1e10), (45000, 100, 300, 1e8), (2100, 20, 60, 1e12), (70000, 128, 384, 1e6)]
    As_h = [gen_usv(m, n, k, 900 + i) for i, (m, n, s, k) in enumerate(probs)]
    As = [dev(A) for A in As_h]
    ss = [p[2] for p in probs]
    refs = [oracle.rpcholqr(A, p[2], 21 + i, nthreads=NTHREADS) for i, (A, p) in enumerate(zip(As_h, probs))]
    announce("batched tuning shapes")
    table = [dict(nmax=64, m_max=10**9, pa_rows=256, pa_max=1, pb_rows=16),
             dict(nmax=128, m_max=50000, pa_rows=512, pa_max=128, pb_rows=4096),
             dict(nmax=128, m_max=10**9, pa_rows=16384, pa_max=3, pb_rows=32),
             dict(nmax=32, m_max=10**9, pa_rows=256, pa_max=128, pb_rows=64)]
    try:
        rq().set_batched_tuning(table)
        with pytest.raises(rq().RpCholQRError):
            rq().set_batched_tuning([dict(nmax=40, m_max=10, pa_rows=256, pa_max=1, pb_rows=16)])
        with pytest.raises(rq().RpCholQRError):
            rq().set_batched_tuning([dict(nmax=64, m_max=10, pa_rows=300, pa_max=1, pb_rows=16)])
        with pytest.raises(rq().RpCholQRError):
            rq().set_batched_tuning([dict(nmax=64, m_max=10, pa_rows=256, pa_max=129, pb_rows=16)])
        plan = rq().BatchedPlan(As, ss, [21 + i for i in range(len(As))])
        plan.execute()
        for i, ref in enumerate(refs):
            assert metrics.rel_fro(host(plan.Qs[i]), ref.Q) < TOL and metrics.rel_fro(host(plan.Rs[i]), ref.R) < TOL
        plan.close()
    finally:
        rq().set_batched_tuning([])
        rq().load_batched_tuning()
