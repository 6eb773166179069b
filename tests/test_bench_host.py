"""Host-side behaviour of bench.py (no GPU): more than one GPU is refused
with a message, and the committed counters are only attached when their
code hash matches the kernel sources."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_code_hash_ignores_comments_only():
    b = load_bench()
    csrc = os.path.join(ROOT, "paper_2602_17494_amd", "csrc")
    read = {}
    for n in os.listdir(csrc):
        with open(os.path.join(csrc, n), encoding="utf-8") as f:
            read[n] = f.read()
    h = b.kernel_source_hash(read=read)
    edited = dict(read)
    edited["green.hip"] = "// a comment\n/* and a block\n comment */\n" + read["green.hip"].replace("\n", "\n  ", 3)
    assert b.kernel_source_hash(read=edited) == h
    # the host orchestration decides frame pitch and box geometry: it counts
    host = dict(read)
    host["api.hip"] = read["api.hip"] + "\nint unused_host_symbol;\n"
    assert b.kernel_source_hash(read=host) != h
    edited["kernels.hip"] = read["kernels.hip"] + "\nint changed;\n"
    assert b.kernel_source_hash(read=edited) != h


def test_committed_counters_match_the_sources():
    b = load_bench()
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        traffic = json.load(f)
    with open(os.path.join(ROOT, "profiles", "sq_counters.json")) as f:
        sq = json.load(f)
    assert traffic["source_hash"] == sq["source_hash"]
    if traffic["source_hash"] != b.kernel_source_hash():
        # the kernels changed since the counters were taken: bench reports null
        assert b.read_traffic("s1_local_cols") is None and b.read_valu_issue("s1_local_cols") is None
        pytest.skip("the committed counters were taken on other kernel code")
    assert b.read_traffic("s1_local_cols") > 0 and b.read_valu_issue("s1_local_cols") > 0
