"""Host-side checks of bench.py: the one-GPU contract and the rule that a
committed HBM-traffic record is reported only for the kernel source it was
measured on."""
import importlib.util
import json
import os
import re
import shutil
import subprocess
import sys

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
    assert "one" in r.stderr and "GPU" in r.stderr
    assert r.stdout == ""


def test_source_fingerprints_cover_their_sections():
    b = _bench()
    shas = [b.kernel_source_sha(), b.eigen_source_sha(), b.wave2_source_sha()]
    assert all(re.fullmatch(r"[0-9a-f]{16}", s) for s in shas)
    assert len(set(shas)) == 3


def test_traffic_record_needs_the_same_kernel_source(tmp_path, monkeypatch):
    b = _bench()
    os.makedirs(tmp_path / "profiles")
    os.makedirs(tmp_path / "paper_1203_4587_amd" / "csrc")
    shutil.copy(os.path.join(ROOT, "paper_1203_4587_amd", "csrc", "iterate.hip"),
                tmp_path / "paper_1203_4587_amd" / "csrc" / "iterate.hip")
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    rec = {"workload": "tv256", "kernel_sha": b.kernel_source_sha(), "bytes_per_launch": 12345}
    path = tmp_path / "profiles" / "x_update_wave_tv256_traffic.json"
    path.write_text(json.dumps(rec))
    assert b.measured_traffic("x_update_wave", "tv256", 100) == 12345
    assert b.measured_traffic("x_update_wave", "dft192", 100) is None          # other workload
    assert b.measured_traffic("x_update_eigen2", "tv256", 1, b.eigen_source_sha) is None   # no record
    # a changed kernel source invalidates the record
    src = tmp_path / "paper_1203_4587_amd" / "csrc" / "iterate.hip"
    src.write_text("// changed\n" + src.read_text())
    assert b.measured_traffic("x_update_wave", "tv256", 100) is None
    # a per-iteration record of the single-launch solve scales with the iteration count
    rec = {"workload": "tv256", "kernel_sha": b.kernel_source_sha(), "bytes_per_iteration": 10}
    (tmp_path / "profiles" / "column_solve_tv256_traffic.json").write_text(json.dumps(rec))
    assert b.measured_traffic("column_solve", "tv256", 7) == 70
