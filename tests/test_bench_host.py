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


def test_cpu_baseline_leg_reports_the_oracle_on_one_and_all_cores():
    b = _bench()
    from cavgen import make_params, make_system
    out = b.cpu_baseline(make_params(), make_system(1), "mulliken", 1e-8, 0.0, seconds=0.5, max_workers=2)
    assert out["kind"] == "oracle" and out["unit"] == "unit-evals/s"
    assert out["value_1core"] > 0 and out["nproc"] >= 1 and out["cpu_model"]
    assert out["cores"] in (1, 2) and out["value"] > 0 and "first units" in out["sample"]
    if out["value_all_cores"] is not None:
        assert out["cores"] == min(2, out["cpus_allowed"]) and out["value"] == out["value_all_cores"]


def test_launch_table_json_schema():
    # the library applies every flat object holding "bucket" (with "arch"); the
    # timing records must not carry that key, or they would be read as entries
    import json
    from paper_2512_03277_amd import autotune
    entries = [{"arch": "gfx950", "bucket": 48, "wg_per_cu": 2, "job_queue": 1, "eig_mode": 0},
               {"arch": "gfx950", "bucket": 192, "wg_per_cu": 1, "job_queue": 0, "eig_mode": 2}]
    timings = [{"tried_bucket": None, "setting": None, "ms_per_eval": 3.0},
               {"tried_bucket": 48, "setting": {"wg_per_cu": 1, "job_queue": 1, "eig_mode": 0}, "ms_per_eval": 3.1}]
    text = autotune.table_json(entries, timings, 4, "mulliken", 3.0, 2.9)
    assert text.count('"bucket"') == len(entries)
    d = json.loads(text)
    assert d["entries"] == entries and d["tuned_on"] == {"workload": 4, "born": "mulliken"}
