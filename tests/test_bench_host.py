"""CPU checks of bench.py's host logic (no GPU is touched): it refuses more
than one GPU, and a committed counter record is used only for its own
workload and only while the kernel sources hash to the recorded value."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


@pytest.mark.parametrize("family", ["sr", "lr_gemm"])
def test_traffic_record_follows_the_sources(family, monkeypatch):
    path = os.path.join(ROOT, "profiles", bench.TRAFFIC_FILES[family].format("c3"))
    with open(path) as fh:
        rec = json.load(fh)
    assert rec["workload"] == "C3"
    # fetch and write scaled by the copy-kernel calibration, and their sum
    assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0
    assert rec["hbm_bytes_per_launch"] == pytest.approx(rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"])
    assert rec["hbm_bytes_per_launch"] > rec["algorithmic_bytes_per_launch"] > 0
    monkeypatch.setattr(bench, "source_hash", lambda fam, h=rec["source_hash"]: h)
    assert bench.recorded_traffic(family, "C3") == rec["hbm_bytes_per_launch"]
    assert bench.recorded_traffic(family, "C5") is None  # no record for that workload
    monkeypatch.setattr(bench, "source_hash", lambda fam: "0" * 16)
    assert bench.recorded_traffic(family, "C3") is None  # the kernel changed since


def test_source_hash_covers_the_kernel_files():
    for fam, files in bench.KERNEL_SOURCES.items():
        for f in files:
            assert os.path.exists(os.path.join(ROOT, f)), (fam, f)
        assert len(bench.source_hash(fam)) == 16
