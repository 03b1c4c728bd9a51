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


def test_recorded_valu_busy_follows_the_kernel_source(tmp_path, monkeypatch):
    src = tmp_path / "paper_1907_02290_amd" / "csrc" / "nb_force.hip"
    src.parent.mkdir(parents=True)
    src.write_bytes(b"// kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "profiles" / "force_disk_4m_valu_counters.md"
    prof.parent.mkdir()
    prof.write_text("valu_busy=0.8125 source_sha256=%s\n" % sha)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_valu_busy() == 0.8125
    src.write_bytes(b"// changed\n")
    assert bench.recorded_valu_busy() is None


def test_quadrupole_flop_count():
    """The quadrupole superparticle term, counted as the paper counts its 23
    flops of a monopole term (FMA = 2, reciprocal square root = 4)."""
    parts = dict(offsets=3, r2=6, rsqrt=4, powers=4, sd=15, dsd=5, coef=7,
                 f53=1, acc=12, pot=8)
    assert sum(parts.values()) == bench.N_OP_QUAD == 65
    mono = dict(offsets=3, r2=6, rsqrt=4, mr=1, mr3=2, acc=6, pot=1)
    assert sum(mono.values()) == bench.N_OP == 23
