"""Sanity of the seeded synthetic systems: determinism, masses, shapes and a
few textbook properties (Plummer half-mass radius and virial ratio, ring
radii, disk + halo mass split)."""
import numpy as np
import pytest

import workloads


def test_seeded_and_deterministic():
    a = workloads.plummer(1000, workloads.seed_for(1))
    b = workloads.plummer(1000, workloads.seed_for(1))
    c = workloads.plummer(1000, workloads.seed_for(1, 1))
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
    assert not np.array_equal(a["x"], c["x"])
    assert workloads.seed_for(3, 2) == 0x1907022900000302


def test_plummer_half_mass_radius_and_virial(orc):
    d = workloads.plummer(4096, workloads.seed_for(1))
    r = np.sqrt(d["x"] ** 2 + d["y"] ** 2 + d["z"] ** 2)
    rh = np.median(r)
    assert abs(rh - 1.0 / np.sqrt(0.5 ** (-2 / 3) - 1)) < 0.06
    _, _, _, pot = orc.force_direct(d["x"], d["y"], d["z"], d["m"], 0.0, 1.0)
    W = 0.5 * (d["m"] * pot).sum()
    K = 0.5 * (d["m"] * (d["vx"] ** 2 + d["vy"] ** 2 + d["vz"] ** 2)).sum()
    assert 0.9 < 2 * K / abs(W) < 1.1
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert abs((d["m"] * d[k]).sum()) < 1e-12


def test_disk_halo_masses_and_extent():
    d = workloads.disk_halo(1 << 12, 1 << 12, workloads.seed_for(3))
    m = d["m"]
    assert m.size == 1 << 13
    assert m[:4096].sum() == pytest.approx(1.0)
    assert m[4096:].sum() == pytest.approx(10.0)
    assert np.all(m[4096:] == 10 * m[0])
    R = np.hypot(d["x"][:4096], d["y"][:4096])
    zd = d["z"][:4096]
    # sech^2 profile, z0 = 0.1: median |z - z_mid| = z0 atanh(1/2) ~ 0.055
    assert abs(np.median(np.abs(zd - np.median(zd))) - 0.0549) < 0.01
    assert np.ptp(R) < 10.5 + 2.0
    # the disk rotates
    L = (d["x"][:4096] * d["vy"][:4096] - d["y"][:4096] * d["vx"][:4096])
    assert np.mean(L > 0) > 0.9


def test_ring_geometry():
    d = workloads.ring(5000, workloads.seed_for(4))
    r = np.sqrt(d["x"] ** 2 + d["y"] ** 2)
    assert r.min() > 0.89 and r.max() < 1.11
    assert np.abs(d["z"]).max() < 0.01
    v = np.sqrt(d["vx"] ** 2 + d["vy"] ** 2 + d["vz"] ** 2)
    np.testing.assert_allclose(v, 1 / np.sqrt(r), rtol=0.01)
    assert d["m"].sum() == pytest.approx(1e-5)


def test_uniform_sphere_cold():
    d = workloads.uniform_sphere(2000, 3)
    r = np.sqrt(d["x"] ** 2 + d["y"] ** 2 + d["z"] ** 2)
    assert r.max() <= 1.05  # recentred on the centre of mass
    assert np.all(d["vx"] == 0)


def test_king_model_virial_and_tidal_radius(orc):
    d = workloads.king(3000, 21)
    r = np.sqrt(d["x"] ** 2 + d["y"] ** 2 + d["z"] ** 2)
    # W0 = 6: tidal radius about 17.8 King radii (concentration c = 1.25)
    assert 14.0 < r.max() < 18.5
    _, _, _, pot = orc.force_direct(d["x"], d["y"], d["z"], d["m"], 0.0, 1.0)
    W = 0.5 * (d["m"] * pot).sum()
    K = 0.5 * (d["m"] * (d["vx"] ** 2 + d["vy"] ** 2 + d["vz"] ** 2)).sum()
    assert 0.9 < 2 * K / abs(W) < 1.1


def test_clusters_offsets():
    c = workloads.clusters(6, 3, lo_exp=6, hi_exp=9)
    off = c["offsets"]
    assert off[0] == 0 and off[-1] == c["x"].size and np.all(np.diff(off) > 0)
    assert np.all(np.diff(off) >= 2 ** 6 - 1)
