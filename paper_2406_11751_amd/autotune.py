"""Autotuner for the batched launch shapes (rpcholqr_batched_set_tuning).

For every column class (n rounded up to 16, 32, 48, 64, or the 128-column
class) and m bucket, builds a synthetic batch shaped like the block-method
workload (m uniform in the bucket, A = U diag(sigma) V^T with log10 kappa
uniform in [2, 14], s = 3n), and times candidate shapes as HIP-graph replays
of the batched plan:

  pass A: the panel height (rows per workgroup, pa_rows) and the largest
          number of workgroups of one problem (pa_max), swept together with
          pass B at its built-in shape;
  pass B: the rows per workgroup (pb_rows), with pass A at its best shape.

The fastest shape of each (class, bucket) goes into a JSON table, which
BatchedPlan installs by default (paper_2406_11751_amd/tuning/).  Run on the GPU
the table is for:

    python -m paper_2406_11751_amd.autotune [--out PATH] [--problems 48]
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

CLASSES = (16, 32, 48, 64, 128)
BUCKETS = ((2_000, 20_000), (20_001, 60_000), (60_001, 200_000))
PA_ROWS = (512, 1024, 2048, 4096, 8192)
PA_MAX = (16, 32, 64, 128)
PB_ROWS = (128, 256, 512, 1024, 2048, 4096)


def log(*a):
    print(*a, flush=True)


def time_plan(rq, torch, As, ss, seeds, replays):
    """ms per execution of one plan, timed over graph replays."""
    plan = rq.BatchedPlan(As, ss, seeds)
    info = torch.zeros((len(As), 2), dtype=torch.int32, device=As[0].device)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        plan.execute(info=info, stream=st.cuda_stream)  # warm-up and check
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            plan.execute(info=info, stream=st.cuda_stream, check=False)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(replays):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    assert int((info[:, 0] != 0).sum()) == 0
    ms = e0.elapsed_time(e1) / replays
    del g
    plan.close()
    return ms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--problems", type=int, default=48, help="problems per synthetic batch")
    ap.add_argument("--replays", type=int, default=8)
    args = ap.parse_args()
    import numpy as np
    import torch

    import paper_2406_11751_amd as rq
    from workloads import gen_usv

    out = args.out or rq.native.TUNING_PATH
    dev = torch.device("cuda:0")
    rng = np.random.Generator(np.random.PCG64(2024))
    entries, report = [], []
    t_start = time.time()
    for nmax in CLASSES:
        n = 8 if nmax == 16 else (100 if nmax == 128 else nmax)
        for lo, hi in BUCKETS:
            ms = rng.integers(lo, hi + 1, size=args.problems)
            ks = 10.0 ** rng.uniform(2, 14, size=args.problems)
            As = [gen_usv(int(m), n, float(k), 7000 + i, backend="torch", device=dev) for i, (m, k) in
                  enumerate(zip(ms, ks))]
            ss, seeds = [3 * n] * len(As), list(range(len(As)))
            base = dict(nmax=nmax, m_max=hi, pa_rows=2048, pa_max=64,
                        pb_rows=(2048 if nmax == 128 else 1024))

            def run(e):
                rq.set_batched_tuning([e])
                return time_plan(rq, torch, As, ss, seeds, args.replays)

            t_default = run(base)
            best, t_best = dict(base), t_default
            for pa_rows in PA_ROWS:
                for pa_max in PA_MAX:
                    e = dict(base, pa_rows=pa_rows, pa_max=pa_max)
                    t = run(e)
                    if t < t_best:
                        best, t_best = e, t
            for pb_rows in PB_ROWS:
                e = dict(best, pb_rows=pb_rows)
                t = run(e)
                if t < t_best:
                    best, t_best = e, t
            entries.append(best)
            report.append(dict(nmax=nmax, n=n, m_range=[lo, hi], problems=len(As), ms_builtin=t_default,
                               ms_tuned=t_best, speedup=t_default / t_best, shape=best))
            log(f"# nmax={nmax} m in [{lo},{hi}]: built-in {t_default:.3f} ms -> tuned {t_best:.3f} ms "
                f"(pa_rows={best['pa_rows']} pa_max={best['pa_max']} pb_rows={best['pb_rows']}) "
                f"[{time.time() - t_start:.0f}s]")
            del As
            torch.cuda.empty_cache()
    rq.set_batched_tuning([])
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        json.dump(dict(device=torch.cuda.get_device_name(0), problems_per_batch=args.problems,
                       entries=entries, report=report), f, indent=1)
    log(f"wrote {out}")


if __name__ == "__main__":
    main()
