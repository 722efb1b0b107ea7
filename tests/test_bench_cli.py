"""Host logic of bench.py: the one-GPU refusal, the record's contract
fields and the CPU-baseline leg (the oracle on a small sample)."""
import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [0, 2, 8])
def test_more_than_one_gpu_is_refused_with_a_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and f"--gpus {n}" in r.stderr
    assert not any(line.startswith("{") for line in r.stdout.splitlines())  # no result line


def test_record_carries_the_contract_fields():
    args = types.SimpleNamespace(steps=7, warmup=2)
    rec = bench.base_record(args, 1234.56, 3.21, "bulk build", {"probe_both": 0})
    assert json.loads(json.dumps(rec)) == rec
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config"):
        assert k in rec, k
    assert rec["n_gpus"] == 1 and rec["steps"] == 7 and rec["warmup"] == 2
    assert rec["value"] == 1234.6 and rec["unit"] == "Mops/s" and rec["higher_is_better"] is True
    assert rec["scaling"] == "weak" and rec["vs_baseline"] is None and rec["data"] == "synthetic"
    assert rec["config"] == {"workload": "bulk build", "probe_both": 0}


def test_source_digest_covers_the_kernel_sources():
    d = bench.source_digest()
    assert len(d) == 16 and int(d, 16) >= 0
    assert d == bench.source_digest()


def test_cpu_baseline_leg_runs_the_oracle_on_a_small_sample():
    rec = bench.cpu_baseline(12)
    assert rec["kind"] == "oracle" and rec["cores"] == 1 and rec["unit"] == "Mops/s"
    assert rec["value"] > 0
    assert "2^12 keys" in rec["sample"]
