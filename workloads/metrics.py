"""Accuracy measures used in the paper's experiments (Section 5).

* orthogonality  ||Q^T Q - I||_2
* residual       ||A - Q R||_2 / ||A||_2
* kappa(A1)      via Lemma l_31: sigma_i(S F Q) = 1/sigma_{n-i+1}(A1), so kappa(A1)
                 is the condition number of the scaled sampled rows of Q.

All are evaluated in float64.  The 2-norm of a tall matrix M is taken as
sqrt(lambda_max(M^T M)); M^T M is formed in float64 (numpy on the host, or
torch on the device for large GPU-resident matrices).
"""
from __future__ import annotations

import numpy as np


def _sym_norm2(S: np.ndarray) -> float:
    return float(np.max(np.abs(np.linalg.eigvalsh(np.asarray(S, dtype=np.float64)))))


def orth_error(Q) -> float:
    if _is_torch(Q):
        G = (Q.t() @ Q).cpu().numpy()
    else:
        Q = np.asarray(Q, dtype=np.float64)
        G = Q.T @ Q
    return _sym_norm2(G - np.eye(G.shape[0]))


def _tall_norm2(M) -> float:
    if _is_torch(M):
        S = (M.t() @ M).cpu().numpy()
    else:
        S = M.T @ M
    return float(np.sqrt(max(_sym_norm2(S), 0.0)))


def residual(A, Q, R, chunk_rows: int = 1 << 20) -> float:
    if _is_torch(A):
        # (A - QR)^T (A - QR) summed over row chunks: no m x n temporary
        S = None
        for r0 in range(0, A.shape[0], chunk_rows):
            D = A[r0:r0 + chunk_rows] - Q[r0:r0 + chunk_rows] @ R
            P = D.t() @ D
            S = P if S is None else S + P
        res2 = max(_sym_norm2(S.cpu().numpy()), 0.0)
        return float(np.sqrt(res2)) / _tall_norm2(A)
    A = np.asarray(A, dtype=np.float64)
    return _tall_norm2(A - Q @ R) / _tall_norm2(A)


def kappa_A1_via_sample(Q, idx, m: int) -> float:
    """kappa(A1) = kappa(sqrt(m/s) Q[idx,:]) (Lemma l_31)."""
    Q = Q.cpu().numpy() if _is_torch(Q) else np.asarray(Q)
    idx = idx.cpu().numpy() if _is_torch(idx) else np.asarray(idx)
    s = idx.shape[0]
    sv = np.linalg.svd(np.sqrt(m / s) * Q[idx, :], compute_uv=False)
    return float(sv[0] / sv[-1])


def rel_fro(X, Y) -> float:
    X = X.cpu().numpy() if _is_torch(X) else np.asarray(X)
    Y = Y.cpu().numpy() if _is_torch(Y) else np.asarray(Y)
    d = np.linalg.norm(Y)
    return float(np.linalg.norm(X - Y) / (d if d > 0 else 1.0))


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")
