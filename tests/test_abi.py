"""The C-ABI library loads and exports every function include/rpcholqr.h declares.

CPU only: no compute call is made (there may be no GPU here).
"""
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "rpcholqr.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int32_t|size_t|void)\s+(rpcholqr_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    names = header_functions()
    for want in ("rpcholqr_factor", "rpcholqr_factor_debug", "rpcholqr_workspace_bytes", "rpcholqr_max_n",
                 "rpcholqr_timing_enable", "rpcholqr_timing_read"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_2406_11751_amd as rq
    from paper_2406_11751_amd import native

    lib = rq.load_library()
    for name in header_functions():
        assert hasattr(lib, name), name
        assert name in native.SIGNATURES, f"binding lacks {name}"


def test_workspace_query_host_logic():
    import paper_2406_11751_amd as rq

    assert rq.max_n() >= 64
    assert rq.workspace_bytes(10_000, 50, 150) > 0
    assert rq.workspace_bytes(1_000_000, 64, 192) > 0
    # invalid or unsupported sizes -> 0
    assert rq.workspace_bytes(10, 20, 40) == 0       # m < n
    assert rq.workspace_bytes(100, 10, 5) == 0       # s < n
    assert rq.workspace_bytes(100, 0, 5) == 0        # n < 1
    assert rq.workspace_bytes(1000, rq.max_n() + 1, 500) == 0
    assert rq.workspace_bytes(100, 10, 30, precision=7) == 0
    # the workspace holds the s x n scaled sample and grows with s
    for s in (96, 384, 385, 1536):
        assert rq.workspace_bytes(100_000, 32, s) >= s * 32 * 8
    assert rq.workspace_bytes(100_000, 32, 1536) > rq.workspace_bytes(100_000, 32, 96)
    assert rq.workspace_bytes(100_000, 32, 1537) == 0  # beyond the largest supported sample
    # 64 < n <= 128: FP64 only; the generic sketch kernel bounds s
    assert rq.max_n() == 1024
    assert rq.workspace_bytes(100_000, 128, 384) >= 384 * 128 * 8 + 128 * 128 * 8
    assert rq.workspace_bytes(100_000, 65, 1536) > 0
    assert rq.workspace_bytes(100_000, 65, 1537) == 0
    assert rq.workspace_bytes(100_000, 100, 300, precision=rq.FP32_REFINE) == 0
    # binary32 A1: the FP64 plan, n <= 64 only
    assert rq.workspace_bytes(100_000, 64, 192, precision=rq.A1_FP32) == rq.workspace_bytes(100_000, 64, 192)
    assert rq.workspace_bytes(100_000, 65, 195, precision=rq.A1_FP32) == 0
    assert rq.workspace_bytes(100_000, 300, 900, precision=rq.A1_FP32) == 0
    assert rq.workspace_bytes(100_000, 64, 192, precision=rq.FP32_REFINE) > 0
    # 128 < n <= 1024: the register panel sketch takes s <= 1536, the streaming
    # one s <= 8192; columns padded to 128k
    for n in (129, 256, 300, 512):
        assert rq.workspace_bytes(1_000_000, n, 3 * n) >= 3 * n * n * 8
    assert rq.workspace_bytes(1_000_000, 512, 1536) > rq.workspace_bytes(1_000_000, 256, 768)
    assert rq.workspace_bytes(1_000_000, 300, 1537) >= 1537 * 300 * 8
    assert rq.workspace_bytes(16_000_000, 512, 5120) >= 5120 * 512 * 8
    assert rq.workspace_bytes(1_000_000, 300, 8192) > 0
    assert rq.workspace_bytes(1_000_000, 300, 8193) == 0
    assert rq.workspace_bytes(100, 129, 387) == 0       # m < n
    assert rq.workspace_bytes(1_000_000, 513, 1539) > 0
    assert rq.workspace_bytes(1_000_000, 1024, 3072) >= 3072 * 1024 * 8 + 4 * 1024 * 1024 * 8
    assert rq.workspace_bytes(1_000_000, 1025, 3075) == 0
    # smoothing adds the chunk sums: ceil(m / chunk) * s * n doubles
    for m, n, s in ((1_000_000, 64, 192), (3000, 300, 900), (20_000_000, 16, 48)):
        chunk = 4096 * max(1, -(-(-(-m // 4096)) // 256))
        extra = rq.workspace_bytes(m, n, s, rq.SMOOTH) - rq.workspace_bytes(m, n, s)
        assert extra >= -(-m // chunk) * s * n * 8, (m, n, s)


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2406_11751_amd import native

    monkeypatch.setattr(native, "LIB_PATH", "/nonexistent/librpcholqr.so")
    monkeypatch.setattr(native, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        native.load_library()


def test_host_sample_indices_match_the_oracle():
    import numpy as np

    import oracle
    import paper_2406_11751_amd as rq

    for m, s, seed in [(1, 5, 0), (1_000_000, 192, 0), (2**40 + 3, 100, 123456789), (7, 0, 1),
                       (10**12, 50, 2**64 - 1), (13, 400, 42)]:
        got = rq.sample_indices(m, s, seed)
        assert np.array_equal(got, oracle.sample_indices(m, s, seed)), (m, s, seed)
        assert got.dtype == np.int64 and (s == 0 or (got.min() >= 0 and got.max() < m))
    with pytest.raises(rq.RpCholQRError):
        rq.sample_indices(0, 3, 1)



def test_bench_rejects_several_gpus():
    # The benchmark measures one GPU; asking for more exits with a message
    # (before touching any device).
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_batched_tuning_table_is_well_formed():
    """The autotuner's committed table (if present) has one entry per column
    class and m bucket, with shapes the library accepts."""
    import json
    import os

    import paper_2406_11751_amd as rq

    path = rq.native.TUNING_PATH
    if not os.path.exists(path):
        return
    t = json.load(open(path))
    for e in t["entries"]:
        assert e["nmax"] in (16, 32, 48, 64, 128)
        assert e["pa_rows"] % 256 == 0 and 1 <= e["pa_max"] <= 128 and e["pb_rows"] % 16 == 0
    assert {e["nmax"] for e in t["entries"]} == {16, 32, 48, 64, 128}
