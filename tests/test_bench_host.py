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


def test_direct_check_errors_and_energy():
    """The policy comparison's error check: zero error for the oracle's own
    direct-sum forces, errors per system for batched sets, and the energy
    of a circular two-body orbit (velocities half a step behind, as the
    kick-drift leaves them) equal to the closed form -G m1 m2 / (2 r)."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(3)
    n = 300
    d = dict(x=rng.standard_normal(n), y=rng.standard_normal(n),
             z=rng.standard_normal(n), m=rng.uniform(0.5, 1.5, n),
             offsets=np.array([0, 120, n]))
    p = dict(eps=0.05, dt=0.01)
    chk = bench.DirectCheck(d, p, 100)
    f = [np.zeros(n) for _ in range(4)]
    for a, b in ((0, 120), (120, n)):
        r = oracle.force_direct(d["x"][a:b], d["y"][a:b], d["z"][a:b],
                                d["m"][a:b], p["eps"], 1.0)
        for q in range(4):
            f[q][a:b] = r[q]
    med, p99 = chk.errors(d["x"], d["y"], d["z"], f)
    assert med == 0.0 and p99 == 0.0
    # forces over all particles (ignoring the split) are wrong per system
    whole = oracle.force_direct(d["x"], d["y"], d["z"], d["m"], p["eps"], 1.0)
    assert chk.errors(d["x"], d["y"], d["z"], whole)[0] > 1e-3
    # two equal masses on a circle of radius 1/2 about their centre, no
    # softening worth the name: E = -1/(2 r) with r = 1
    m = np.array([1.0, 1.0])
    two = dict(x=np.array([-0.5, 0.5]), y=np.zeros(2), z=np.zeros(2), m=m)
    q = dict(eps=1e-9, dt=1e-3)
    c2 = bench.DirectCheck(two, q, 2)
    v = np.sqrt(0.5)   # circular speed: v^2 / 0.5 = 1 / r^2
    acc = oracle.force_direct(two["x"], two["y"], two["z"], m, q["eps"], 1.0)
    # counter-clockwise motion; the velocities half a step behind are the
    # current ones turned back by omega dt / 2
    w = v / 0.5 * q["dt"] / 2
    vx = np.array([-v * np.sin(w), v * np.sin(w)])
    vy = np.array([-v * np.cos(w), v * np.cos(w)])
    st = (two["x"], two["y"], two["z"], vx, vy, np.zeros(2))
    e = c2.energy(st, acc)
    assert abs(e - (-0.5)) < 1e-6
