"""bench.py host logic: the algorithmic-bytes models, the guard that drops a
stored HBM-traffic figure once the kernel sources or the iteration count no
longer match it, and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bytes_models():
    # rods: 80-byte D record read twice + 8 incidence + 48 gamma/g/q per
    # contact; U written and read + axis per particle
    assert bench.iteration_bytes(1, 0, True) == 2 * 80 + 8 + 48
    assert bench.iteration_bytes(0, 1, True) == 2 * 48 + 24
    assert bench.iteration_bytes(1, 0, False) == 2 * 32 + 8 + 48
    assert bench.iteration_bytes(0, 1, False) == 2 * 24 + 8
    # a mixture reduces to the pure models
    assert bench.mixed_iteration_bytes(7, 0, 5, 0) == bench.iteration_bytes(7, 5, True)
    assert bench.mixed_iteration_bytes(0, 7, 0, 5) == bench.iteration_bytes(7, 5, False)
    assert bench.operator_bytes(3, 10) == 12 * 10 + 44 * 3


def test_traffic_record_guard(tmp_path):
    rec = {"iters": 1304, "bytes_per_launch": 123, "kernel_sha256": bench.kernel_digest()}
    f = tmp_path / "t.json"
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic(1304, str(f)) == 123
    assert bench.measured_traffic(1305, str(f)) is None   # another launch
    rec["kernel_sha256"] = "0" * 64                      # other kernel sources
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic(1304, str(f)) is None
    assert bench.measured_traffic(1304, str(tmp_path / "missing.json")) is None


def test_host_cpu_report():
    model, nproc, usable = bench.host_cpu()
    assert isinstance(model, str) and model
    assert 1 <= usable <= nproc


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
