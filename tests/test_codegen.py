"""Code-generation properties of the HIP library that its speed depends on,
checked on the gfx950 assembly (hipcc cross-compiles without a GPU):

- The batched kernels read their pointers from a device table.  Unless those
  pointers are re-read as global-memory pointers, the compiler accesses memory
  through them with flat instructions, which also count against the LDS
  counter and serialize mixed traffic.
- The operand prefetches of the TRSM panels and of pass B for n > 128 must not
  wait for each load before issuing the next: a conditional load
  (`c ? p[i] : 0`) compiles to a zero written into the load's destination and
  a wait for the loads in flight, which turns a prefetch into one load at a
  time.  The sign in the assembly is a load, `s_waitcnt vmcnt(0)`, then the
  next load.
- The Householder sweeps of the sketch for n > 128 read the reflector from LDS
  a chunk at a time, not one read and one wait per fma.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2406_11751_amd import build as libbuild

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(libbuild.HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("asm") / "rpcholqr.s"
    flags = [f for f in libbuild.FLAGS if f not in ("-fPIC", "-shared")]
    cmd = [libbuild.HIPCC, *flags, "--cuda-device-only", "-S", "-o", str(out), *libbuild.SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    text = out.read_text()
    shutil.rmtree(out.parent, ignore_errors=True)
    return text


def kernels(text, pattern):
    """{mangled name: body} of the kernels whose name matches pattern."""
    out = {}
    for name in re.findall(r"\.amdhsa_kernel (\S+)", text):
        if re.search(pattern, name):
            i = text.index(name + ":")
            out[name] = text[i:text.index(".Lfunc_end", i)]
    return out


def serialized_loads(body):
    """Loads followed by a full vmcnt wait and then another load."""
    ev = []
    for line in body.split("\n"):
        line = line.strip()
        if re.match(r"(global|buffer|flat)_load", line):
            ev.append("L")
        elif line.startswith("s_waitcnt") and "vmcnt(0)" in line:
            ev.append("W")
    return sum(1 for i in range(len(ev) - 2) if ev[i:i + 3] == ["L", "W", "L"])


def test_batched_kernels_use_global_memory_instructions(asm):
    ks = kernels(asm, r"^_ZN3rpq\d+kb_")
    assert len(ks) >= 20
    for name, body in ks.items():
        assert not re.search(r"\n\s+flat_(load|store)", body), name


def test_large_n_prefetches_are_not_serialized(asm):
    passb = kernels(asm, r"k_passB_big")
    assert len(passb) == 7  # nmax = 256, 384, ..., 1024
    for name, body in passb.items():
        assert serialized_loads(body) == 0, name
    (trsm,) = kernels(asm, r"k_trsm_panel").values()
    # the copy of the next U block into LDS is a short load / store sequence
    # per block; the A1 prefetch in the k-chunk loop must stay pipelined
    assert serialized_loads(trsm) <= 8
    assert re.search(r"s_waitcnt vmcnt\((8|9|10|11)\)", trsm)


def lds_reads_waited_one_by_one(body):
    ev = []
    for line in body.split("\n"):
        line = line.strip()
        if line.startswith("ds_read"):
            ev.append("R")
        elif line.startswith("s_waitcnt") and "lgkmcnt(0)" in line:
            ev.append("W")
        elif line.startswith("s_waitcnt"):
            ev.append("w")
    return sum(1 for i in range(len(ev) - 1) if ev[i] == "R" and ev[i + 1] == "W")


def test_large_n_sketch_reads_the_reflector_in_chunks(asm):
    ks = kernels(asm, r"k_sketch_(panel|trail)(_w)?ILi")
    assert len(ks) == 18  # RPT = 16 ... 96 and L = 32, 64, 96, panel and trail each
    for name, body in ks.items():
        reads = len(re.findall(r"\n\s+ds_read", body))
        assert lds_reads_waited_one_by_one(body) <= max(8, reads // 16), name
