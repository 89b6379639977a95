"""GPU: matrices with more than 2^31 elements (every element offset past 32 bits).

A is k stacked copies of a small well-conditioned A0 (m0 rows): A^T A = k A0^T A0,
so the thin QR with positive diagonal is exactly R = sqrt(k) R0 and Q = copies of
Q0 / sqrt(k), with A0 = Q0 R0 (uniqueness of the thin QR with positive diagonal,
paper Section 2).  R and the first copy of Q are compared with LAPACK's QR of A0.
Every row of Q is computed from its own row of A with the same arithmetic in the
row solve and in Q = A1 R2^{-1}, so all copies of Q must be equal to the bit: an
offset computed wrongly anywhere in the m x n range shows up as a mismatch.
"""
import numpy as np
import pytest

from workloads import gen_usv, metrics

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-12


def rq():
    import paper_2406_11751_amd

    return paper_2406_11751_amd


def exact_qr(A0_h):
    Q0, R0 = np.linalg.qr(A0_h)
    d = np.sign(np.diag(R0))
    return Q0 * d, R0 * d[:, None]


def stacked(A0_h, k):
    m0, n = A0_h.shape
    A0 = torch.from_numpy(np.ascontiguousarray(A0_h.T)).to("cuda")  # (n, m0)
    A = rq().colmajor_empty(m0 * k, n, "cuda")
    A.t().view(n, k, m0).copy_(A0.unsqueeze(1).expand(n, k, m0))
    return A


def check_copies(Q, m0, k, n):
    Qv = Q.t().view(n, k, m0)
    assert torch.equal(Qv, Qv[:, :1, :].expand(n, k, m0)), "copies of Q differ"


@pytest.mark.parametrize("n,k", [(64, 34_000), (128, 17_000)])
def test_beyond_2_31_elements(n, k):
    m0 = 1000
    m = m0 * k
    assert m * n > 2**31
    s = 3 * n
    print(f"case: stacked {k} x ({m0} x {n}), m = {m}, s = {s}", flush=True)
    A0_h = gen_usv(m0, n, 1e2, 31)
    Q0, R0 = exact_qr(A0_h)
    A = stacked(A0_h, k)
    Q, R, _ = rq().factor(A, s, 7)
    torch.cuda.synchronize()
    check_copies(Q, m0, k, n)
    Rh, Qh = R.cpu().numpy(), Q[:m0].cpu().numpy()
    er, eq = metrics.rel_fro(Rh, np.sqrt(k) * R0), metrics.rel_fro(Qh, Q0 / np.sqrt(k))
    print(f"  |dR|={er:.2e} |dQ|={eq:.2e}", flush=True)
    assert er < TOL and eq < TOL
    assert np.array_equal(np.tril(Rh, -1), np.zeros((n, n)))

    # The batched entry point with the same large problem next to a small one.
    A_small = stacked(A0_h, 1)
    plan = rq().BatchedPlan([A, A_small], [s, s], [7, 8])
    try:
        plan.execute()
        torch.cuda.synchronize()
        check_copies(plan.Qs[0], m0, k, n)
        Rb, Qb = plan.Rs[0].cpu().numpy(), plan.Qs[0][:m0].cpu().numpy()
        assert metrics.rel_fro(Rb, np.sqrt(k) * R0) < TOL and metrics.rel_fro(Qb, Q0 / np.sqrt(k)) < TOL
        assert metrics.rel_fro(plan.Rs[1].cpu().numpy(), R0) < TOL
        assert metrics.rel_fro(plan.Qs[1].cpu().numpy(), Q0) < TOL
    finally:
        plan.close()
    del A, Q, R, plan
    torch.cuda.empty_cache()
