"""Accuracy study of rpCholesky-QR on the GPU, shaped like the paper's
Section 5 experiments.

Test matrices (Section 5.1): A = [I_n; 0] R_A, m = 6000, with R_A an n x n
matrix of geometric singular values from 1 to 1/kappa (kappa = 1e15) and Haar
singular vectors, as Matlab's randsvd; worst-case coherence, so the smoothed
sample (F = F_T D, here the RPCHOLQR_SMOOTH option) is used, as in the paper.

  sweep-c:  n = 100 and n = 1000, 10 trials (sampling seeds) for each
            sampling amount c from n + 10 to 6n; reports the smallest, mean and
            largest orthogonality error ||Q^T Q - I||_2, residual
            ||A - QR||_2/||A||_2 and kappa(A1) (Figures ErrorRange3 and
            ErrorRange1);
  sweep-n:  c = 3n for n = 100 .. 1024 (Figure ErrorRangeG, n = 100 .. 2000 in
            the paper; this library takes n <= 1024);
  estimate: for every run, the orthogonality error over the estimate
            4 eps kappa(A1) of Section 5.2 (eps = 2^-52).

kappa(A1) is taken from the singular values of A1 (debug output).  Lemma l_31
(the sampled, smoothed rows of Q, sqrt(M/c) (F [Q; 0])(idx), have singular
values 1/sigma(A1), reversed) is checked on each c with the library's own
smoothed sample of the computed Q (same seed), on the same kind of matrix with
kappa = 1e6: the lemma is an identity of exact arithmetic, and the computed R_s
factors the sketch only up to a backward error of order eps ||A_s||, so the
sample of A1 is orthonormal only to about eps kappa(A) (1e-1 at kappa = 1e15).

    python -m paper_2406_11751_amd.study [--trials 10] [--out study.json]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

EPS = 2.0 ** -52


def coherent(m, n, kappa, seed):
    """[I_n; 0] R_A with R_A = U diag(sigma) V^T, Haar U and V (seeded)."""
    import numpy as np

    from workloads import sigma_profile

    rng = np.random.Generator(np.random.PCG64(seed))
    U, Ru = np.linalg.qr(rng.standard_normal((n, n)))
    V, Rv = np.linalg.qr(rng.standard_normal((n, n)))
    U, V = U * np.sign(np.diag(Ru))[None, :], V * np.sign(np.diag(Rv))[None, :]
    A = np.zeros((m, n))
    A[:n] = (U * sigma_profile(n, kappa)[None, :]) @ V.T
    return np.asfortranarray(A)


def lemma_l31_deviation(rq, torch, A, c, seed):
    """max_i |sigma_i(sample of Q) - 1/sigma_{n-i+1}(A1)| / sigma_i(sample of Q)."""
    import numpy as np

    Q, _, _, ex = rq.factor(A, c, seed, debug=True, precision=rq.SMOOTH)
    sv = torch.linalg.svdvals(ex["A1"]).cpu().numpy()
    _, _, _, exq = rq.factor(Q, c, seed, debug=True, precision=rq.SMOOTH)
    sq = np.linalg.svd(exq["As"].cpu().numpy(), compute_uv=False)
    return float(np.max(np.abs(sq - 1.0 / sv[::-1]) / sq))


def run_one(rq, torch, metrics, A, c, seed):
    try:
        Q, R, info, ex = rq.factor(A, c, seed, debug=True, precision=rq.SMOOTH)
    except rq.RpCholQRError as e:
        return dict(c=c, seed=seed, ok=False, code=e.code, index=e.index)
    sv = torch.linalg.svdvals(ex["A1"]).cpu().numpy()
    kap = float(sv[0] / sv[-1])
    orth = metrics.orth_error(Q)
    res = metrics.residual(A, Q, R)
    out = dict(c=c, seed=seed, ok=True, orth=orth, residual=res, kappa_A1=kap,
               orth_over_estimate=orth / (4 * EPS * kap))
    return out


def summarize(runs):
    ok = [r for r in runs if r["ok"]]
    s = dict(trials=len(runs), failures=len(runs) - len(ok))
    for key in ("orth", "residual", "kappa_A1", "orth_over_estimate"):
        v = [r[key] for r in ok]
        if v:
            s[key] = dict(min=min(v), mean=sum(v) / len(v), max=max(v))
    return s


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trials", type=int, default=10)
    ap.add_argument("--m", type=int, default=6000)
    ap.add_argument("--kappa", type=float, default=1e15)
    ap.add_argument("--out", default=None)
    ap.add_argument("--quick", action="store_true", help="a reduced sweep (n = 100, fewer c)")
    a = ap.parse_args(argv)
    import torch

    import paper_2406_11751_amd as rq
    from workloads import metrics

    dev = torch.device("cuda:0")
    t0 = time.time()
    report = dict(m=a.m, kappa=a.kappa, trials=a.trials, smoothing="RPCHOLQR_SMOOTH", sweep_c={}, sweep_n={})
    sweeps = [(100, (110, 150, 200, 300, 400, 600))]
    if not a.quick:
        sweeps.append((1000, (1010, 1500, 2000, 3000, 4000, 6000)))
    for n, cs in sweeps:
        A_h = coherent(a.m, n, a.kappa, 1)
        A = torch.from_numpy(A_h.T.copy()).to(dev).t()
        A_mod = torch.from_numpy(coherent(a.m, n, 1e6, 1).T.copy()).to(dev).t()
        rows = {}
        for c in cs:
            runs = [run_one(rq, torch, metrics, A, c, seed) for seed in range(a.trials)]
            try:
                dev_l31 = lemma_l31_deviation(rq, torch, A_mod, c, 0)
            except rq.RpCholQRError:
                dev_l31 = None
            rows[str(c)] = dict(summary=summarize(runs), lemma_l31_rel_dev_kappa1e6=dev_l31)
            s = rows[str(c)]["summary"]
            print(f"# n={n} c={c}: failures {s['failures']}/{s['trials']}"
                  + (f", orth {s['orth']['min']:.1e}..{s['orth']['max']:.1e}, residual <= {s['residual']['max']:.1e}, "
                     f"kappa(A1) {s['kappa_A1']['min']:.1f}..{s['kappa_A1']['max']:.1f}, "
                     f"orth/(4 eps kappa(A1)) {s['orth_over_estimate']['min']:.2f}..{s['orth_over_estimate']['max']:.2f}"
                     if "orth" in s else "") + f", Lemma l_31 deviation (kappa 1e6) {dev_l31}" + f" [{time.time() - t0:.0f}s]", flush=True)
        report["sweep_c"][str(n)] = rows
    for n in ((100, 200, 300) if a.quick else (100, 200, 300, 500, 750, 1000, 1024)):
        A_h = coherent(a.m, n, a.kappa, 2)
        A = torch.from_numpy(A_h.T.copy()).to(dev).t()
        runs = [run_one(rq, torch, metrics, A, 3 * n, seed) for seed in range(a.trials)]
        report["sweep_n"][str(n)] = summarize(runs)
        s = report["sweep_n"][str(n)]
        print(f"# c=3n, n={n}: failures {s['failures']}/{s['trials']}"
              + (f", orth <= {s['orth']['max']:.1e}, residual <= {s['residual']['max']:.1e}, "
                 f"kappa(A1) <= {s['kappa_A1']['max']:.1f}" if "orth" in s else "") + f" [{time.time() - t0:.0f}s]",
              flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(report, f, indent=1)
    return report


if __name__ == "__main__":
    main()
