"""Host-side parts of the benchmark's contract (CPU only): one GPU only,
argument checks, and the rule that measured HBM traffic is reported only
for the kernel sources and launch shape the counters were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    out = _run("--gpus", "2")
    assert out.returncode == 2
    assert "one GPU" in out.stderr


@pytest.mark.parametrize("args", [("--steps", "0"), ("--warmup", "-1")])
def test_bad_step_counts_are_refused(args):
    out = _run(*args)
    assert out.returncode == 2
    assert "--steps" in out.stderr


def test_traffic_only_for_the_profiled_sources_and_launch(tmp_path, monkeypatch):
    rec = {"source_sha256": bench.kernel_source_hash(), "launch": [256, 65536],
           "traffic_bytes_per_launch": 3.63e9}
    path = tmp_path / "counters.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "COUNTERS", str(path))
    assert bench.measured_traffic((256, 65536)) == 3.63e9
    assert bench.measured_traffic((128, 65536)) is None
    path.write_text(json.dumps({**rec, "source_sha256": "0" * 64}))
    assert bench.measured_traffic((256, 65536)) is None
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "missing.json"))
    assert bench.measured_traffic((256, 65536)) is None


def test_source_hash_covers_every_step_source():
    for rel in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, rel)), rel
    names = {os.path.basename(r) for r in bench.KERNEL_SOURCES}
    assert {"cmflb_step.h", "cmflb_step_pull.hip", "cmflb_device.h", "cmflb_internal.h",
            "cmflb_d3q19.h"} <= names
