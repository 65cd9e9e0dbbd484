"""The benchmark's command-line contract, checked without a GPU: one GPU
only (a clear refusal for more), a loud failure where there is no GPU (never
a CPU fallback), and the keys of its JSON line."""

import argparse
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _run(*args):
    return subprocess.run([sys.executable, BENCH, *args], capture_output=True, text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_no_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        import pytest
        pytest.skip("a GPU is present")
    r = _run("--steps", "1", "--warmup", "0", "--cpu-sample", "0")
    assert r.returncode != 0
    assert "needs a GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_modes_listed():
    r = _run("--help")
    assert r.returncode == 0
    for mode in ("single", "batch", "surrogate", "decomposed", "graph", "copy"):
        assert mode in r.stdout


def test_json_record_has_the_contract_keys():
    sys.path.insert(0, ROOT)
    import bench
    args = argparse.Namespace(steps=10, warmup=2)
    rec = bench.base_record(args, 123.4567, 1.25, "f64", {"workload": "orszag_tang_8000x8000_fp64_hd"})
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config"):
        assert key in rec, key
    assert rec["n_gpus"] == 1 and rec["higher_is_better"] is True and rec["vs_baseline"] is None
    assert rec["config"]["workload"].startswith("orszag_tang_8000x8000")
    assert rec["metric"] == bench.METRIC
