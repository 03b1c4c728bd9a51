"""Host-side behaviour of bench.py that needs no GPU: it refuses more than
one GPU, and it reports the recorded force-kernel HBM traffic only while the
kernel source still has the hash the counters were taken on."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_recorded_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    src = tmp_path / "paper_1907_02290_amd" / "csrc" / "nb_force.hip"
    src.parent.mkdir(parents=True)
    src.write_bytes(b"// kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "profiles" / "disk_4m_hbm_counters.md"
    prof.parent.mkdir()
    prof.write_text("Force kernel, per launch: traffic_bytes_per_launch="
                    "2.5e+09 source_sha256=%s\n" % sha)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic() == 2.5e9
    src.write_bytes(b"// kernel source, changed\n")
    assert bench.recorded_traffic() is None
    prof.unlink()
    assert bench.recorded_traffic() is None
