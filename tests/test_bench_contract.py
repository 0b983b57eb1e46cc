"""bench.py's command-line contract, checked on the CPU: one GPU only, the
counter summary is read back, and the summary ties traffic to the sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run("--gpus", "2")
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_help_lists_the_contract_flags():
    r = run("--help")
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup"):
        assert flag in r.stdout


def test_traffic_summary_matches_sources_or_is_ignored():
    sys.path.insert(0, ROOT)
    import bench

    path = os.path.join(ROOT, bench.TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        pytest.skip("no counter summary committed")
    fields = dict(l.split(": ", 1) for l in open(path).read().splitlines() if ": " in l)
    t = bench.measured_traffic()
    if fields["source_hash"].strip() == bench.kernel_source_hash():
        assert t == float(fields["traffic_bytes_per_launch"]) and t > 0
    else:
        assert t is None
