"""Pins of the oracle's short-range part (section 2: group walk with a
different opening criterion; section 4.2: lists reused over steps): the SPH
kernel against its closed-form values and its normalisation, the neighbour
lists against a definition without a walk and against brute-force neighbour
sets, the list density against the all-pairs density, and list reuse
within the skin."""
import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads


def test_kernel_values_and_normalisation():
    h = 0.37
    c = 8.0 / (np.pi * h ** 3)
    assert oracle.sph_w(0.0, h) == pytest.approx(c, rel=1e-15)
    assert oracle.sph_w(0.5 * h, h) == pytest.approx(0.25 * c, rel=1e-14)
    assert oracle.sph_w(h, h) == 0.0
    assert oracle.sph_w(1.5 * h, h) == 0.0
    # continuous at q = 1/2 and at q = 1
    e = 1e-9 * h
    assert oracle.sph_w(0.5 * h - e, h) == pytest.approx(
        oracle.sph_w(0.5 * h + e, h), rel=1e-7)
    assert oracle.sph_w(h - e, h) < 1e-20 * c + 1e-12
    # unit integral over space
    val, err = integrate.quad(lambda r: 4 * np.pi * r * r * oracle.sph_w(r, h),
                              0.0, h, points=[0.5 * h], epsabs=1e-13)
    assert val == pytest.approx(1.0, abs=1e-10)
    # decreasing in r
    r = np.linspace(0.0, h, 200)
    w = np.array([oracle.sph_w(v, h) for v in r])
    assert np.all(np.diff(w) <= 1e-12 * c)


def _tree(d, n_leaf=8, n_grp=32):
    return oracle.Tree(d["x"], d["y"], d["z"], d["m"], n_leaf, n_grp)


def _sorted_xyz(t, d):
    _, perm = t.keys()
    return (d["x"][perm], d["y"][perm], d["z"][perm], d["m"][perm])


def _lists_without_walk(t, h):
    """Particles of every leaf whose cube overlaps the group's box grown by
    h, leaves in pre-order, from the cell table alone."""
    c = t.cells()
    g = t.groups()
    leaves = np.nonzero(c["leaf"])[0]
    half = np.ldexp(1.0, t.k - c["level"][leaves].astype(int) - 1)
    ctr = c["ctr"][leaves]
    out = []
    for gi in range(t.n_groups):
        lo, hi = g["lo"][gi], g["hi"][gi]
        gap = np.maximum(0.0, np.maximum(lo - ctr, ctr - hi))
        ok = np.all(gap <= (half + h)[:, None], axis=1)
        # a leaf that holds the group is opened whatever its distance
        b, n = int(g["begin"][gi]), int(g["count"][gi])
        holds = (c["begin"][leaves] <= b) & \
            (c["begin"][leaves].astype(np.int64) + c["count"][leaves] >= b + n)
        sel = leaves[ok | holds]
        ids = [np.arange(c["begin"][k], c["begin"][k] + c["count"][k])
               for k in sel]
        out.append(np.concatenate(ids) if ids else np.zeros(0, np.int64))
    return out


@pytest.mark.parametrize("kind,n,h", [("plummer", 1500, 0.05),
                                      ("plummer", 1500, 0.3),
                                      ("disk", 2000, 0.02),
                                      ("plummer", 300, 0.0)])
def test_lists_match_definition_without_walk(kind, n, h):
    d = workloads.plummer(n, 3) if kind == "plummer" else \
        workloads.disk_halo(n // 2, n - n // 2, 5)
    t = _tree(d)
    off, ids = t.neighbour_lists(h)
    want = _lists_without_walk(t, h)
    for gi in range(t.n_groups):
        np.testing.assert_array_equal(ids[off[gi]:off[gi + 1]], want[gi])


@pytest.mark.parametrize("h", [0.02, 0.1, 0.4])
def test_lists_hold_every_neighbour(h):
    d = workloads.plummer(1200, 4)
    t = _tree(d, n_leaf=4, n_grp=16)
    off, ids = t.neighbour_lists(h)
    x, y, z, _ = _sorted_xyz(t, d)
    g = t.groups()
    for gi in range(t.n_groups):
        b, n = int(g["begin"][gi]), int(g["count"][gi])
        lst = set(ids[off[gi]:off[gi + 1]].tolist())
        for i in range(b, b + n):
            r2 = (x - x[i]) ** 2 + (y - y[i]) ** 2 + (z - z[i]) ** 2
            need = np.nonzero(r2 <= h * h)[0]
            assert set(need.tolist()) <= lst
            assert i in lst


@pytest.mark.parametrize("kind,h", [("plummer", 0.08), ("disk", 0.03),
                                    ("sphere", 0.15)])
def test_list_density_equals_all_pairs(kind, h):
    n = 2500
    d = {"plummer": lambda: workloads.plummer(n, 8),
         "disk": lambda: workloads.disk_halo(n // 2, n - n // 2, 9),
         "sphere": lambda: workloads.uniform_sphere(n, 10)}[kind]()
    t = _tree(d, n_leaf=8, n_grp=64)
    t.neighbour_lists(h)
    got = t.sph_density(h)
    want = oracle.sph_density_direct(d["x"], d["y"], d["z"], d["m"], h)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)
    # every particle feels at least itself
    assert np.all(got >= d["m"] * oracle.sph_w(0.0, h) * (1 - 1e-12))


def test_uniform_lattice_density():
    """Interior particles of a cubic lattice of spacing a and particle mass
    m get the lattice density m / a^3 to the kernel's accuracy."""
    a, m = 0.1, 1e-3
    k = np.arange(20) * a
    X, Y, Z = np.meshgrid(k, k, k, indexing="ij")
    x, y, z = X.ravel(), Y.ravel(), Z.ravel()
    d = dict(x=x, y=y, z=z, m=np.full(x.size, m))
    t = _tree(d)
    h = 2.5 * a
    t.neighbour_lists(h)
    rho = t.sph_density(h)
    inner = np.all(np.abs(np.stack([x, y, z]) - 0.95) < 0.55, axis=0)
    assert inner.sum() > 100
    np.testing.assert_allclose(rho[inner], m / a ** 3, rtol=0.02)


def test_reuse_within_the_skin():
    """Lists built with h (1 + s) still give the all-pairs density for h
    after every particle moved by less than s h / 2."""
    h, s = 0.06, 0.3
    d = workloads.plummer(2000, 12)
    t = _tree(d)
    t.neighbour_lists(h * (1 + s))
    rng = np.random.default_rng(13)
    step = rng.standard_normal((3, d["x"].size))
    step *= (0.49 * s * h / np.sqrt(3)) / np.abs(step).max()
    x2, y2, z2 = d["x"] + step[0], d["y"] + step[1], d["z"] + step[2]
    t.refresh(x2, y2, z2, d["m"])
    got = t.sph_density(h)
    want = oracle.sph_density_direct(x2, y2, z2, d["m"], h)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)
