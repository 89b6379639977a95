#!/usr/bin/env python3
"""Throughput of rpCholesky-QR on one MI355X.

One step = one full factorization (sample, gather, sketch QR, pass A, Gram
reduction, Cholesky, R product, pass B) of the 1,000,000 x 64 workload with
s = 3n = 192 sampled rows: A = U diag(sigma) V^T, kappa = 1e8, seed 0, FP64,
resident in HBM before the timed region starts.

value = algorithmic bytes per factorization / time per factorization, in GB/s;
factorizations/s is reported beside it.  The algorithmic bytes are 24 m n: the
method must read A twice (once before and once after the Gram matrix exists)
and write Q once.  This implementation instead reads A once, writes A1 into the
Q buffer, reads A1 back and overwrites it with Q: 32 m n bytes moved, whose rate
is reported as well (bytes_moved_GBps).  Time per factorization is the mean over
the timed steps (the contract's value), with the median, p10 and p90 of the
per-step times beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rpCholQR GB/s & factorizations/s; mixed/batched vs FP64 at orth err<=1e-12"
HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP64_PEAK_TFS = 78.6       # MI355X FP64 (vector and matrix share this rate)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--m", type=int, default=1_000_000)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--s", type=int, default=None)
    ap.add_argument("--kappa", type=float, default=1e8)
    ap.add_argument("--no-accuracy", action="store_true", help="skip the per-kappa accuracy sweep")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="bounded CPU sample: repeat oracle factorizations for about this long")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-workload measurement")
    ap.add_argument("--no-mixed", action="store_true", help="skip the refined-precision measurement")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--no-large", action="store_true", help="skip the 1e6 x 128, 4e6 x 256 and 1.6e7 x 512 workloads")
    ap.add_argument("--large-only", default="", help="comma-separated subset of the large workloads")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy three times (for counter calibration)")
    return ap.parse_args()


def host_cores() -> int:
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_traffic(pass_name: str, m: int, n: int):
    """HBM bytes per launch from the committed rocprofv3 counter record of this
    pass at this size, or None when there is none or the kernel sources changed
    since it was taken."""
    from paper_2406_11751_amd import profiling

    path = os.path.join(ROOT, "profiles", f"traffic_{pass_name}_fp64_{m}x{n}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_digest") != profiling.source_digest():
        return None
    return rec["traffic_bytes"]


def per_pass_roofline_s(m, n):
    """Sum over the two streaming passes of max(bytes / HBM peak, flops / FP64 peak):
    pass A reads A (8mn B) and does m n^2 + m n (n+1) flops; pass B reads and
    writes (16mn B) and does m n^2 flops."""
    a = max(8.0 * m * n / (HBM_PEAK_GBS * 1e9), m * (2.0 * n * n + n) / (FP64_PEAK_TFS * 1e12))
    b = max(16.0 * m * n / (HBM_PEAK_GBS * 1e9), 1.0 * m * n * n / (FP64_PEAK_TFS * 1e12))
    return a + b


def batched_measurement(args, torch, rq, gen_usv, metrics):
    """Batched workload: the 2048-problem list (m ~ U{2000..200000}, n ~ U{8, 16,
    32, 64, 128}, log10 kappa ~ U[2, 14], s = 3n, seed i), generated on the GPU.
    One plan (launch shapes from the autotuned table) is captured in a HIP graph;
    the replays are timed.  For comparison: the eager execute, and the same
    problems factored one call at a time with the single-problem entry point."""
    import numpy as np
    from workloads import batched_problem_list

    dev = torch.device("cuda:0")
    plist = batched_problem_list(2048, 0)
    keep = [p for p in plist if p["n"] <= 128]
    t0 = time.time()
    As = []
    for i, p in enumerate(keep):
        As.append(gen_usv(p["m"], p["n"], p["kappa"], p["seed"], backend="torch", device=dev))
        if (i + 1) % 256 == 0:
            print(f"# batched inputs: {i + 1}/{len(keep)} ({time.time() - t0:.0f}s)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    print(f"# batched inputs generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    tuned = rq.load_batched_tuning()
    plan = rq.BatchedPlan(As, [p["s"] for p in keep], [p["seed"] for p in keep])
    info = torch.zeros((len(keep), 2), dtype=torch.int32, device=dev)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        plan.execute(info=info, stream=st.cuda_stream)  # warm-up and check
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            plan.execute(info=info, stream=st.cuda_stream, check=False)
    g.replay()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.batched_steps + 1)]
    evs[0].record()
    for k in range(args.batched_steps):
        g.replay()
        evs[k + 1].record()
    torch.cuda.synchronize()
    rep = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.batched_steps)])
    ms = float(np.median(rep))
    assert int((info[:, 0] != 0).sum()) == 0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.batched_steps):
        plan.execute(info=info, check=False)
    e1.record()
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / args.batched_steps
    orth = max(metrics.orth_error(plan.Qs[i]) for i in range(0, len(keep), 64))
    # the same problems one call at a time (single-problem entry point, its own workspace each)
    ws = torch.empty(max(rq.workspace_bytes(p["m"], p["n"], p["s"]) for p in keep), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    e0.record()
    for A, Q, R, p in zip(As, plan.Qs, plan.Rs, keep):
        rq.factor(A, p["s"], p["seed"], Q=Q, R=R, workspace=ws, info=info[0], check=False)
    e1.record()
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1)
    bytes_alg = sum(24.0 * p["m"] * p["n"] for p in keep)
    roof_ms = sum(per_pass_roofline_s(p["m"], p["n"]) for p in keep) * 1e3
    out = dict(workload="2048-problem list (m ~ U{2000..200000}, n ~ U{8,16,32,64,128}, log10 kappa ~ U[2,14], "
                        "s = 3n, seed i)", problems=len(keep), ms_per_batch=ms,
               ms_p10=float(np.percentile(rep, 10)), ms_p90=float(np.percentile(rep, 90)),
               timing="median over HIP-graph replays of one captured plan execution",
               eager_ms_per_batch=eager_ms, autotuned_shapes=tuned,
               factorizations_per_s=len(keep) / (ms * 1e-3), value_GBps=bytes_alg / (ms * 1e-3) / 1e9,
               roofline_ms=roof_ms, roofline_frac=roof_ms / ms,
               roofline_model="sum over problems and passes of max(bytes / 8 TB/s, flops / 78.6 TF/s)",
               sequential_single_calls_ms=seq_ms, speedup_vs_single_calls=seq_ms / ms,
               max_orth_every_64th=orth, device_bytes=plan.device_bytes)
    del g
    plan.close()
    del As
    torch.cuda.empty_cache()
    print(f"# batched: {len(keep)} problems in {ms:.2f} ms (graph replay; eager {eager_ms:.2f} ms; "
          f"{out['factorizations_per_s']:.0f} fact/s, {out['roofline_frac']:.2f} of roofline); "
          f"one call at a time {seq_ms:.1f} ms", file=sys.stderr, flush=True)
    return out


def large_measurement(args, torch, rq, metrics):
    """The 1,000,000 x 128 (kappa 1e8, s = 384), 4,000,000 x 256 (kappa 1e12, s = 768)
    and 16,000,000 x 512 (kappa 1e10, s = 1536 and s = 5120) workloads in FP64,
    generated on the GPU (the largest with the
    polar-factor construction, which needs no second m x n buffer).  Reports time
    per factorization, GB/s on 24mn, TFLOP/s on 3mn^2 and its fraction of the
    FP64 peak, orthogonality and residual at full size, and parity against the
    oracle on the first 100,000 rows (same seed and s)."""
    import numpy as np

    import oracle
    from workloads import gen_usv, gen_usv_polar

    dev = torch.device("cuda:0")
    res = {}
    A, made = None, None
    for name, m, n, s, kappa, steps in (("1e6x128", 1_000_000, 128, 384, 1e8, 20),
                                        ("4e6x256", 4_000_000, 256, 768, 1e12, 10),
                                        ("1.6e7x512", 16_000_000, 512, 1536, 1e10, 3),
                                        ("1.6e7x512_s10n", 16_000_000, 512, 5120, 1e10, 3)):
        if args.large_only and name not in args.large_only.split(","):
            continue
        if made != (m, n, kappa):  # the s = 10n run factors the same matrix
            A = None
            torch.cuda.empty_cache()
            t0 = time.time()
            if m * n > 10**9:
                A = gen_usv_polar(m, n, kappa, 0, device=dev)
            else:
                A = gen_usv(m, n, kappa, 0, backend="torch", device=dev)
            made = (m, n, kappa)
            torch.cuda.synchronize()
            print(f"# {name}: input generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
        Q = rq.colmajor_empty(m, n, dev)
        R = rq.colmajor_empty(n, n, dev)
        ws = torch.empty(rq.workspace_bytes(m, n, s), dtype=torch.uint8, device=dev)
        info = torch.zeros(2, dtype=torch.int32, device=dev)
        rq.factor(A, s, 0, Q=Q, R=R, workspace=ws, info=info)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        evs[0].record()
        for k in range(steps):
            rq.factor(A, s, 0, Q=Q, R=R, workspace=ws, info=info, check=False)
            evs[k + 1].record()
        torch.cuda.synchronize()
        t = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(steps)])
        ms = float(np.median(t))
        rq.timing_enable(True)
        rq.factor(A, s, 0, Q=Q, R=R, workspace=ws, info=info, check=False)
        _, stage_ms = rq.timing_read()
        rq.timing_enable(False)
        assert info.cpu().tolist() == [0, -1]
        orth, resid = metrics.orth_error(Q), metrics.residual(A, Q, R)
        # parity on a row subsample the oracle finishes quickly
        msub = 100_000
        A_sub = A[:msub].cpu().numpy()
        Qs, Rs, _ = rq.factor(A[:msub], s, 0)
        ref = oracle.rpcholqr(A_sub, s, 0, nthreads=host_cores(), keep=False)
        assert ref.status == oracle.OK
        tf = 3.0 * m * n * n / (ms * 1e-3) / 1e12
        res[name] = dict(m=m, n=n, s=s, kappa=kappa, dtype="f64", ms_per_factorization=ms,
                         ms_p10=float(np.percentile(t, 10)), ms_p90=float(np.percentile(t, 90)),
                         factorizations_per_s=1e3 / ms, value_GBps=24.0 * m * n / (ms * 1e-3) / 1e9,
                         tflops=tf, frac_fp64_peak=tf / FP64_PEAK_TFS,
                         stage_ms=stage_ms, orth=orth, residual=resid,
                         parity_subsample=dict(rows=msub, rel_fro_Q=metrics.rel_fro(Qs, ref.Q),
                                               rel_fro_R=metrics.rel_fro(Rs, ref.R)))
        print(f"# {name}: {ms:.2f} ms ({tf:.1f} TF/s = {tf / FP64_PEAK_TFS:.2f} of FP64 peak), orth {orth:.1e}, "
              f"residual {resid:.1e}, subsample |dQ| {res[name]['parity_subsample']['rel_fro_Q']:.1e}",
              file=sys.stderr, flush=True)
        del Q, R, ws, Qs, Rs
        torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.copy_calibration:
        import torch

        x = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(f"copied {x.numel() * 8} bytes three times", flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: the factorization runs on one GPU; --gpus {args.gpus} is not supported "
              "(row sharding over several GPUs is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2406_11751_amd as rq
    from workloads import gen_usv, metrics

    m, n = args.m, args.n
    s = args.s or 3 * n
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    bytes_alg = 24.0 * m * n            # A read twice + Q written once
    flops_alg = 3.0 * m * n * n         # TRSM (m n^2) + SYRK (m n (n+1)) + TRSM (m n^2), to leading order

    def to_dev(A_h):
        return torch.from_numpy(np.ascontiguousarray(A_h.T)).to(dev).t()

    t0 = time.time()
    A_h = gen_usv(m, n, args.kappa, 0)
    A = to_dev(A_h)
    print(f"# input {m}x{n} kappa={args.kappa:.0e} generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    Q = rq.colmajor_empty(m, n, dev)
    R = rq.colmajor_empty(n, n, dev)
    ws = torch.empty(rq.workspace_bytes(m, n, s), dtype=torch.uint8, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)

    def step():
        rq.factor(A, s, 0, Q=Q, R=R, workspace=ws, info=info, check=False)

    for _ in range(max(args.warmup, 1)):  # at least one call, whose status is checked
        step()
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, -1], info
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    step_ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    e0.record(stream)
    step_ev[0].record(stream)
    for i in range(args.steps):
        step()
        step_ev[i + 1].record(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    step_ms = np.array([step_ev[i].elapsed_time(step_ev[i + 1]) for i in range(args.steps)])
    dist = dict(mean_ms=ms, median_ms=float(np.median(step_ms)), p10_ms=float(np.percentile(step_ms, 10)),
                p90_ms=float(np.percentile(step_ms, 90)))

    # Per-kernel durations: HIP events recorded by the library between its kernels on
    # the same stream, over a second loop of the same length.  They are not taken in
    # the timed loop above because each recorded event adds a small gap between two
    # kernels, which would inflate the time that loop reports.
    rq.timing_enable(True)
    for _ in range(args.steps):
        step()
    calls, stage_ms = rq.timing_read()
    rq.timing_enable(False)
    stage_avg = {k: v / calls for k, v in stage_ms.items()}
    print(f"# {ms * 1e3:.1f} us/factorization; stages (us): "
          + " ".join(f"{k}={v * 1e3:.1f}" for k, v in stage_avg.items()), file=sys.stderr, flush=True)

    # Accuracy of this run and of the kappa sweep (the metric is quoted at orth <= 1e-12).
    acc = {}
    Qh_orth = metrics.orth_error(Q)
    acc[f"{args.kappa:.0e}"] = dict(orth=Qh_orth, residual=metrics.residual(A, Q, R))
    if not args.no_accuracy:
        for kappa in (1.0, 1e4, 1e12, 1e15):
            Ak = to_dev(gen_usv(m, n, kappa, 0))
            Qk, Rk, _ = rq.factor(Ak, s, 0)
            acc[f"{kappa:.0e}"] = dict(orth=metrics.orth_error(Qk), residual=metrics.residual(Ak, Qk, Rk))
            del Ak, Qk, Rk
    print("# accuracy " + json.dumps(acc), file=sys.stderr, flush=True)

    pa_us, pb_us = stage_avg["passA"] * 1e3, stage_avg["passB"] * 1e3
    # Algorithmic work of the two streaming passes (Algorithm 2, lines 4-6):
    #   pass A: read A (8mn bytes); A1 = A R_s^{-1} (m n^2 flops) and G1 = A1^T A1 upper (m n (n+1) flops);
    #   pass B: read A1, write Q (16mn bytes); Q = A1 R2^{-1} (m n^2 flops).
    # Storing A1 in pass A is this implementation's choice and is not counted.
    # For 64 < n <= 128 pass A is three kernels (two half-row solves and the Gram
    # pass) and pass B keeps R2^{-1} in LDS.
    wide = n > 64
    passes = {
        "passA": dict(kernel="k_passW + k_gramW" if wide else "k_passA_mfma", us=pa_us,
                      bytes=8.0 * m * n, flops=m * (2.0 * n * n + n)),
        "passB": dict(kernel="k_passB128" if wide else "k_passB", us=pb_us, bytes=16.0 * m * n,
                      flops=1.0 * m * n * n),
    }
    dom_name = max(passes, key=lambda k: passes[k]["us"])
    dom = passes[dom_name]
    t_bytes = dom["bytes"] / (HBM_PEAK_GBS * 1e9)
    t_flops = dom["flops"] / (FP64_PEAK_TFS * 1e12)
    if t_flops >= t_bytes:
        achieved = dom["flops"] / (dom["us"] * 1e-6) / 1e12
        roofline = dict(kernel=dom["kernel"], bound="alu", achieved=achieved, peak=FP64_PEAK_TFS, unit="TFLOP/s",
                        frac=achieved / FP64_PEAK_TFS)
    else:
        achieved = dom["bytes"] / (dom["us"] * 1e-6) / 1e9
        roofline = dict(kernel=dom["kernel"], bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=achieved / HBM_PEAK_GBS)
    roofline["traffic"] = measured_traffic(dom_name, m, n)
    roofline["algorithmic_bytes"] = dom["bytes"]
    roofline["algorithmic_flops"] = dom["flops"]
    roofline["launch_us"] = dom["us"]
    t_roof = sum(max(p["bytes"] / (HBM_PEAK_GBS * 1e9), p["flops"] / (FP64_PEAK_TFS * 1e12)) for p in passes.values())

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        cores = host_cores()

        def time_oracle(nthreads, budget_s, max_runs):
            runs, t0 = 0, time.perf_counter()
            while runs < 1 or (time.perf_counter() - t0 < budget_s and runs < max_runs):
                r = oracle.rpcholqr(A_h, s, 0, nthreads=nthreads, keep=True)
                runs += 1
            assert r.status == oracle.OK
            return runs, (time.perf_counter() - t0) / runs

        runs, dt = time_oracle(cores, args.cpu_seconds, 50)
        runs1, dt1 = time_oracle(1, 0.0, 1)
        cpu = dict(value=bytes_alg / dt / 1e9, unit="GB/s", cores=cores, kind="oracle",
                   cpu_model=cpu_model(), factorizations_per_s=1.0 / dt, seconds_per_factorization=dt,
                   sample=f"{runs} full oracle factorizations of the same {m}x{n} input, s={s}, on {cores} "
                          f"threads ({runs * dt:.1f} s), and one on 1 thread ({dt1:.1f} s)",
                   one_thread=dict(value=bytes_alg / dt1 / 1e9, unit="GB/s", cores=1,
                                   seconds_per_factorization=dt1, factorizations_per_s=1.0 / dt1))

    # Mixed precisions on the same input: the refined ones (lower-precision Gram
    # in pass 1, FP64 Cholesky-QR second pass) and A1 kept in binary32 between
    # the passes.
    ws_r = torch.empty(rq.workspace_bytes(m, n, s, rq.FP32_REFINE), dtype=torch.uint8, device=dev)
    mixed = None if args.no_mixed else {}
    for pname in () if args.no_mixed else ("A1_FP32", "FP32_REFINE", "BF16X2_REFINE"):
        prec = getattr(rq, pname)

        def step_refine():
            rq.factor(A, s, 0, Q=Q, R=R, workspace=ws_r, info=info, check=False, precision=prec)

        for _ in range(max(args.warmup, 1)):
            step_refine()
        torch.cuda.synchronize()
        assert info.cpu().tolist() == [0, -1], info
        e0.record(stream)
        for _ in range(args.steps):
            step_refine()
        e1.record(stream)
        torch.cuda.synchronize()
        ms_r = e0.elapsed_time(e1) / args.steps
        mixed[pname] = dict(ms_per_factorization=ms_r, value_GBps=bytes_alg / (ms_r * 1e-3) / 1e9,
                            factorizations_per_s=1e3 / ms_r, speed_vs_fp64=ms / ms_r,
                            orth=metrics.orth_error(Q), residual=metrics.residual(A, Q, R))
        print(f"# {pname}: {ms_r * 1e3:.1f} us/factorization, orth {mixed[pname]['orth']:.1e}, "
              f"residual {mixed[pname]['residual']:.1e}", file=sys.stderr, flush=True)
    del ws_r
    step()  # leave the FP64 result in Q, R

    batched = None if args.no_batched else batched_measurement(args, torch, rq, gen_usv, metrics)
    large = None if args.no_large else large_measurement(args, torch, rq, metrics)

    out = {
        "metric": METRIC,
        "value": bytes_alg / (ms * 1e-3) / 1e9,
        "unit": "GB/s",
        "factorizations_per_s": 1e3 / ms,
        "bytes_moved_GBps": (32.0 if n <= 64 else 40.0) * m * n / (ms * 1e-3) / 1e9,
        "step_time": dist,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"rpCholesky-QR FP64, A {m}x{n} = U diag(sigma) V^T, kappa={args.kappa:.0e}, "
                               f"s={s} sampled rows, seed 0", "m": m, "n": n, "s": s, "kappa": args.kappa,
                   "parallelism": "single GPU"},
        "gflops": flops_alg / (ms * 1e-3) / 1e9,
        "stage_us": {k: v * 1e3 for k, v in stage_avg.items()},
        "roofline": roofline,
        "roofline_whole_path": dict(t_roof_us=t_roof * 1e6, frac=t_roof / (ms * 1e-3),
                                    model="sum over passes of max(bytes/8 TB/s, flops/78.6 TF)"),
        "accuracy": acc,
        "cpu_baseline": cpu,
        "mixed": mixed,
        "batched": batched,
        "large": large,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
