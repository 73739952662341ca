"""Host-side logic of bench.py (no GPU): the one-GPU contract, the lookup of the
profiled HBM traffic and its source-hash guard, and the oracle CPU-baseline leg.
"""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_profiled_traffic_follows_the_kernel_source_hash(tmp_path):
    b = _bench()
    src = os.path.join(ROOT, "paper_2512_03277_amd", "csrc", "scc_kernel.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for key, path in b.PROFILES.items():
        lines = dict(l.split(":", 1) for l in open(path) if l.startswith(("traffic_bytes_per_launch",
                                                                          "kernel_source_sha256_16")))
        expect = float(lines["traffic_bytes_per_launch"]) if lines["kernel_source_sha256_16"].strip() == sha else None
        assert b.profiled_traffic(*key) == expect
    assert b.profiled_traffic(99, "mulliken") is None
    for key in b.PROFILES:
        ex = b.profiled_value(*key, "executed_per_algorithmic_fp64")
        assert ex is None or 0.5 < ex < 3.0
    assert b.profiled_value(2, "mulliken", "no_such_figure") is None
    # a summary for another source is not used
    fake = tmp_path / "p.md"
    fake.write_text("traffic_bytes_per_launch: 123\nkernel_source_sha256_16: 0000000000000000\n")
    b.PROFILES[(7, "x")] = str(fake)
    assert b.profiled_traffic(7, "x") is None


def test_cpu_baseline_leg_reports_the_oracle_on_one_thread():
    b = _bench()
    from cavgen import make_params, make_system
    out = b.cpu_baseline(make_params(), make_system(1), 1e-8, seconds=0.5, min_units=2)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "unit-evals/s"
    assert out["value"] > 0 and "units of the workload" in out["sample"]
