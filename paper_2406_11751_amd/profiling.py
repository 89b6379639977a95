"""Summaries of rocprofv3 runs of the library's kernels.

Reads the CSV output of
  rocprofv3 --kernel-trace --stats --output-format csv ...   (kernel statistics)
  rocprofv3 --pmc FETCH_SIZE --output-format csv ...          (HBM bytes read)
  rocprofv3 --pmc WRITE_SIZE --output-format csv ...          (HBM bytes written)
and the same two counters taken on a plain device copy of known size
(`python bench.py --copy-calibration`), which fixes the factor between what the
counters report and the bytes that actually moved.  Writes a Markdown summary
and a JSON record of the traffic of one kernel, stamped with a digest of the
kernel sources so that a later change to them invalidates the record.

    python -m paper_2406_11751_amd.profiling --stats DIR --fetch DIR --write DIR \\
        --copy-fetch DIR --copy-write DIR --kernel k_passA --tag passA_fp64_1e6x64 \\
        --workload "..." --command-stats "..." --command-fetch "..." ... --out profiles
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# Sources that define the streaming-pass kernels (their traffic records go stale
# when these change).
KERNEL_SOURCES = ("csrc/passes.h", "csrc/device_common.h")
COPY_BYTES = 64 * 1024 * 1024 * 8  # the calibration copy moves 512 MiB each way per call


def source_digest(files=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(PKG, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _one(pattern: str, root: str) -> str:
    hits = sorted(glob.glob(os.path.join(root, "**", pattern), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no {pattern} under {root}")
    return hits[0]


def kernel_stats(root: str):
    rows = list(csv.DictReader(open(_one("*kernel_stats.csv", root))))
    out = []
    for r in rows:
        out.append(dict(name=r["Name"], calls=int(r["Calls"]), avg_us=float(r["AverageNs"]) / 1e3,
                        min_us=float(r["MinNs"]) / 1e3, max_us=float(r["MaxNs"]) / 1e3))
    return out


def counter_per_dispatch(root: str, counter: str):
    """{kernel name: (dispatches, counter summed over a dispatch, averaged over dispatches)}."""
    rows = list(csv.DictReader(open(_one("*counter_collection.csv", root))))
    total = collections.defaultdict(float)
    ids = collections.defaultdict(set)
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        total[r["Kernel_Name"]] += float(r["Counter_Value"])
        ids[r["Kernel_Name"]].add(r["Dispatch_Id"])
    return {k: (len(ids[k]), total[k] / len(ids[k])) for k in total}


def counter_by_kernel(root: str, counter: str):
    """{kernel name: mean of the counter over its dispatches}."""
    rows = list(csv.DictReader(open(_one("*counter_collection.csv", root))))
    vals = collections.defaultdict(list)
    for r in rows:
        if r["Counter_Name"] == counter:
            vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in vals.items()}


def counter_max_dispatch(root: str, counter: str):
    """{kernel name: the counter summed over one dispatch, largest dispatch}."""
    rows = list(csv.DictReader(open(_one("*counter_collection.csv", root))))
    per = collections.defaultdict(float)
    for r in rows:
        if r["Counter_Name"] == counter:
            per[(r["Kernel_Name"], r["Dispatch_Id"])] += float(r["Counter_Value"])
    out = {}
    for (k, _), v in per.items():
        out[k] = max(out.get(k, 0.0), v)
    return out


def mfma_summary(stats_dir, mfma_dir, workload, command_stats, command_mfma, out_path, traffic=None):
    """Markdown table of the library's kernels: calls, average time, and the
    derived MfmaUtil counter (MFMA busy cycles over active cycles of all SIMDs).
    With traffic = (fetch_dir, write_dir, fetch_scale, write_scale, commands),
    also the HBM bytes read and written by the largest dispatch of each kernel."""
    stats = [s for s in kernel_stats(stats_dir) if "rpq::" in s["name"]]
    util = counter_by_kernel(mfma_dir, "MfmaUtil")
    cmds = [command_stats, command_mfma] + (list(traffic[4]) if traffic else [])
    head = "| kernel | calls | average us | total ms | MfmaUtil % |"
    rule = "|---|---|---|---|---|"
    if traffic:
        fetch = counter_max_dispatch(traffic[0], "FETCH_SIZE")
        write = counter_max_dispatch(traffic[1], "WRITE_SIZE")
        head += " HBM read, largest dispatch (GB) | HBM written (GB) |"
        rule += "---|---|"
    lines = [f"# rocprofv3: {workload}", "", "Kernel statistics and MFMA utilization, commands (repository root, MI355X):",
             "", "```", *cmds, "```", ""]
    if traffic:
        lines += [f"HBM bytes are FETCH_SIZE x {traffic[2]:.3f} and WRITE_SIZE x {traffic[3]:.3f} (the factors "
                  "that make the counters of a plain 512 MiB device copy read 512 MiB).", ""]
    lines += [head, rule]
    for s in sorted(stats, key=lambda s: -s["avg_us"] * s["calls"]):
        u = util.get(s["name"])
        row = (f"| `{s['name']}` | {s['calls']} | {s['avg_us']:.1f} | {s['avg_us'] * s['calls'] / 1e3:.2f} | "
               + (f"{u:.1f}" if u is not None else "-") + " |")
        if traffic:
            f, w = fetch.get(s["name"]), write.get(s["name"])
            row += (f" {f * 1024 * traffic[2] / 1e9:.2f} |" if f is not None else " - |")
            row += (f" {w * 1024 * traffic[3] / 1e9:.2f} |" if w is not None else " - |")
        lines.append(row)
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _pick(table: dict, needle: str):
    keys = [k for k in table if needle in k]
    if not keys:
        raise KeyError(f"no kernel matching {needle!r}")
    return keys[0], table[keys[0]]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mfma", default=None,
                    help="MfmaUtil counter run: write only a kernel table with MFMA utilization to --out/--tag.md")
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--kernel", required=True, help="substring of the kernel to record traffic for")
    ap.add_argument("--copy-kernel", default="copyBuffer", help="substring of the calibration copy kernel")
    ap.add_argument("--tag", required=True, help="file stem, named for the kernel and workload")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command-stats", required=True)
    ap.add_argument("--command-fetch", required=True)
    ap.add_argument("--command-write", required=True)
    ap.add_argument("--command-copy", required=True)
    ap.add_argument("--command-mfma", default="")
    ap.add_argument("--algorithmic-bytes", type=float, required=True,
                    help="bytes the kernel must move per launch (for comparison)")
    ap.add_argument("--out", required=True)
    if "--mfma" in os.sys.argv:
        for req in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--kernel", "--command-fetch",
                    "--command-write", "--command-copy", "--algorithmic-bytes"):
            for act in ap._actions:
                if req in act.option_strings:
                    act.required = False
    a = ap.parse_args()
    if a.mfma:
        os.makedirs(a.out, exist_ok=True)
        traffic = None
        if a.fetch and a.write and a.copy_fetch and a.copy_write:
            _, (_, cf_kib) = _pick(counter_per_dispatch(a.copy_fetch, "FETCH_SIZE"), a.copy_kernel)
            _, (_, cw_kib) = _pick(counter_per_dispatch(a.copy_write, "WRITE_SIZE"), a.copy_kernel)
            traffic = (a.fetch, a.write, COPY_BYTES / (cf_kib * 1024.0), COPY_BYTES / (cw_kib * 1024.0),
                       (a.command_fetch, a.command_write, a.command_copy))
        mfma_summary(a.stats, a.mfma, a.workload, a.command_stats, a.command_mfma,
                     os.path.join(a.out, f"{a.tag}.md"), traffic)
        return

    stats = kernel_stats(a.stats)
    lib = [s for s in stats if "rpq::" in s["name"]]
    fetch = counter_per_dispatch(a.fetch, "FETCH_SIZE")
    write = counter_per_dispatch(a.write, "WRITE_SIZE")
    cfetch = counter_per_dispatch(a.copy_fetch, "FETCH_SIZE")
    cwrite = counter_per_dispatch(a.copy_write, "WRITE_SIZE")
    kname, (nf, f_kib) = _pick(fetch, a.kernel)
    _, (nw, w_kib) = _pick(write, a.kernel)
    _, (_, cf_kib) = _pick(cfetch, a.copy_kernel)
    _, (_, cw_kib) = _pick(cwrite, a.copy_kernel)
    fetch_scale = COPY_BYTES / (cf_kib * 1024.0)
    write_scale = COPY_BYTES / (cw_kib * 1024.0)
    traffic = f_kib * 1024.0 * fetch_scale + w_kib * 1024.0 * write_scale
    rec = dict(kernel=kname, workload=a.workload, fetch_kib_per_dispatch=f_kib, write_kib_per_dispatch=w_kib,
               dispatches=dict(fetch=nf, write=nw), copy_fetch_kib=cf_kib, copy_write_kib=cw_kib,
               copy_bytes=COPY_BYTES, fetch_scale=fetch_scale, write_scale=write_scale,
               traffic_bytes=traffic, algorithmic_bytes=a.algorithmic_bytes,
               source_digest=source_digest(), sources=list(KERNEL_SOURCES))
    os.makedirs(a.out, exist_ok=True)
    with open(os.path.join(a.out, f"traffic_{a.tag}.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    lines = [f"# rocprofv3: {a.workload}", "",
             "Kernel statistics, command (repository root, MI355X):", "", "```", a.command_stats, "```", "",
             "| kernel | calls | average us | min us | max us |", "|---|---|---|---|---|"]
    for s in sorted(lib, key=lambda s: -s["avg_us"] * s["calls"]):
        lines.append(f"| `{s['name']}` | {s['calls']} | {s['avg_us']:.1f} | {s['min_us']:.1f} | {s['max_us']:.1f} |")
    lines += ["", f"HBM traffic of `{kname}` per dispatch (`FETCH_SIZE`, `WRITE_SIZE` in KiB), commands:", "",
              "```", a.command_fetch, a.command_write, a.command_copy, "```", "",
              "| quantity | value |", "|---|---|",
              f"| FETCH_SIZE per dispatch | {f_kib:.0f} KiB |",
              f"| WRITE_SIZE per dispatch | {w_kib:.0f} KiB |",
              f"| plain copy of {COPY_BYTES >> 20} MiB: FETCH_SIZE / WRITE_SIZE | {cf_kib:.0f} / {cw_kib:.0f} KiB |",
              f"| scale factors (bytes per counted byte) read / write | {fetch_scale:.3f} / {write_scale:.3f} |",
              f"| traffic per dispatch (scaled) | {traffic / 1e6:.1f} MB |",
              f"| algorithmic bytes per dispatch | {a.algorithmic_bytes / 1e6:.1f} MB |",
              f"| kernel source digest | `{rec['source_digest']}` |", ""]
    with open(os.path.join(a.out, f"{a.tag}.md"), "w") as fh:
        fh.write("\n".join(lines))
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
