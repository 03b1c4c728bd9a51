"""Pins of the oracle's list forces and direct forces: all-open list sum
equals the direct sum, two-body closed form, momentum conservation, error
falling with theta, the quadrupole's error order, the isotropic-quadrupole
identity, and a ~ -grad(phi) of the superparticle expansion."""
import numpy as np
import pytest


def _rel_err(a, b):
    ax, ay, az = a[:3]
    bx, by, bz = b[:3]
    num = np.sqrt((ax - bx) ** 2 + (ay - by) ** 2 + (az - bz) ** 2)
    return num / np.sqrt(bx ** 2 + by ** 2 + bz ** 2)


def test_two_body_closed_form(orc):
    eps, G = 0.3, 2.0
    x = np.array([0.0, 1.5])
    y = np.array([0.0, 2.0])
    z = np.array([0.0, 0.0])
    m = np.array([3.0, 5.0])
    ax, ay, az, pot = orc.force_direct(x, y, z, m, eps, G)
    r2 = 1.5 ** 2 + 2.0 ** 2
    f = G / (r2 + eps * eps) ** 1.5
    assert ax[0] == pytest.approx(f * 5.0 * 1.5, rel=1e-15)
    assert ay[0] == pytest.approx(f * 5.0 * 2.0, rel=1e-15)
    assert ax[1] == pytest.approx(-f * 3.0 * 1.5, rel=1e-15)
    assert az[0] == 0.0
    assert pot[0] == pytest.approx(-G * 5.0 / np.sqrt(r2 + eps * eps), rel=1e-15)
    # the same through the tree with every cell opened
    t = orc.Tree(x, y, z, m, n_leaf=1, n_grp=1)
    t.make_lists(0.0)
    lx, ly, lz, lp = t.force_lists(1, eps, G)
    np.testing.assert_allclose([lx, ly, lz, lp], [ax, ay, az, pot], rtol=1e-15)


def test_direct_sum_conserves_momentum(orc):
    rng = np.random.default_rng(4)
    n = 600
    x, y, z = rng.standard_normal((3, n))
    m = rng.uniform(0.2, 3.0, n)
    ax, ay, az, _ = orc.force_direct(x, y, z, m, 0.05, 1.0)
    for a in (ax, ay, az):
        assert abs((m * a).sum()) <= 1e-13 * np.abs(m * a).sum()


@pytest.mark.parametrize("order", [1, 2])
def test_all_open_list_sum_equals_direct(orc, order):
    rng = np.random.default_rng(5)
    n = 1500
    x, y, z = rng.standard_normal((3, n))
    m = rng.uniform(0.2, 3.0, n)
    t = orc.Tree(x, y, z, m, n_leaf=8, n_grp=32)
    t.make_lists(0.0)
    got = t.force_lists(order, 0.02, 1.0)
    ref = orc.force_direct(x, y, z, m, 0.02, 1.0)
    assert _rel_err(got, ref).max() < 1e-13
    np.testing.assert_allclose(got[3], ref[3], rtol=1e-13)


def test_error_falls_with_theta_and_quadrupole_helps(orc):
    import workloads
    d = workloads.plummer(4096, 123)
    x, y, z, m = d["x"], d["y"], d["z"], d["m"]
    ref = orc.force_direct(x, y, z, m, 1 / 64, 1.0)
    t = orc.Tree(x, y, z, m, n_leaf=8, n_grp=64)
    med = {}
    for theta in (0.3, 0.5, 0.7):
        t.make_lists(theta)
        for order in (1, 2):
            med[(theta, order)] = np.median(
                _rel_err(t.force_lists(order, 1 / 64, 1.0), ref))
    for order in (1, 2):
        assert med[(0.3, order)] < med[(0.5, order)] < med[(0.7, order)]
    for theta in (0.3, 0.5, 0.7):
        assert med[(theta, 2)] < 0.5 * med[(theta, 1)]


def _clump_probe(rng, d, K=8, s=1.0, iso=False):
    """K particles inside [0, s]^3 and one probe at distance ~d on +x, with d
    just below a power of two so that the clump's octant of the root is a
    single accepted superparticle for theta = 1."""
    if iso:
        c = 0.5 * s
        h = 0.3 * s
        pts = np.array([[c + h, c, c], [c - h, c, c], [c, c + h, c],
                        [c, c - h, c], [c, c, c + h], [c, c, c - h]])
        m = np.full(6, 0.7)
    else:
        pts = rng.uniform(0.0, s, (K, 3))
        m = rng.uniform(0.5, 1.5, K)
    probe = np.array([[d, 0.31 * s, 0.17 * s]])
    P = np.vstack([pts, probe])
    return P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy(), np.append(m, 1e-3)


def _probe_force(orc, x, y, z, m, order, eps=0.0):
    n = x.size
    t = orc.Tree(x, y, z, m, n_leaf=n - 1, n_grp=n - 1)
    t.make_lists(1.0)
    eo, e, so, s = t.lists()
    key, perm = t.keys()
    probe_pos = int(np.nonzero(perm == n - 1)[0][0])
    g = t.groups()
    gi = int(np.nonzero((g["begin"] <= probe_pos) &
                        (g["begin"] + g["count"] > probe_pos))[0][0])
    assert so[gi + 1] - so[gi] == 1  # the whole clump is one superparticle
    assert list(e[eo[gi]:eo[gi + 1]]) == [probe_pos]
    f = t.force_lists(order, eps, 1.0)
    return np.array([f[0][n - 1], f[1][n - 1], f[2][n - 1], f[3][n - 1]])


def test_quadrupole_error_order(orc):
    rng = np.random.default_rng(31)
    ds = np.array([0.9 * 2.0 ** k for k in range(4, 10)])
    errs = {1: [], 2: []}
    base = _clump_probe(rng, 0.0)
    for d in ds:
        x, y, z, m = base
        x = x.copy()
        x[-1] = d
        ref = orc.force_direct(x, y, z, m, 0.0, 1.0, targets=[x.size - 1])
        a_ref = np.array([ref[0][0], ref[1][0], ref[2][0]])
        for order in (1, 2):
            a = _probe_force(orc, x, y, z, m, order)[:3]
            errs[order].append(np.linalg.norm(a - a_ref) / np.linalg.norm(a_ref))
    sl1 = np.polyfit(np.log(ds), np.log(errs[1]), 1)[0]
    sl2 = np.polyfit(np.log(ds), np.log(errs[2]), 1)[0]
    assert -2.3 < sl1 < -1.7, sl1
    assert -3.3 < sl2 < -2.7, sl2


def test_isotropic_quadrupole_adds_nothing(orc):
    rng = np.random.default_rng(1)
    x, y, z, m = _clump_probe(rng, 0.9 * 64, iso=True)
    mono = _probe_force(orc, x, y, z, m, 1)
    quad = _probe_force(orc, x, y, z, m, 2)
    np.testing.assert_allclose(quad, mono, rtol=1e-13)


@pytest.mark.parametrize("eps", [0.0, 0.7])
def test_superparticle_force_is_minus_gradient(orc, eps):
    rng = np.random.default_rng(2)
    x, y, z, m = _clump_probe(rng, 0.9 * 16)
    a = _probe_force(orc, x, y, z, m, 2, eps)
    h = 1e-4
    grad = []
    for ax_i, arr in enumerate((x, y, z)):
        ph = []
        for sgn in (1, -1):
            arr2 = arr.copy()
            arr2[-1] += sgn * h
            args = [x, y, z]
            args[ax_i] = arr2
            ph.append(_probe_force(orc, *args, m, 2, eps)[3])
        grad.append((ph[0] - ph[1]) / (2 * h))
    np.testing.assert_allclose(a[:3], -np.array(grad), rtol=1e-6)


def test_self_term_excluded(orc):
    # a lone particle feels nothing and has zero potential
    t = orc.Tree(np.array([0.3]), np.array([0.1]), np.array([-0.2]),
                 np.array([2.0]), n_leaf=8, n_grp=8)
    t.make_lists(0.5)
    f = t.force_lists(1, 0.1, 1.0)
    assert [float(v[0]) for v in f] == [0.0, 0.0, 0.0, 0.0]


def test_reuse_refresh_matches_rebuild_when_unmoved(orc):
    rng = np.random.default_rng(8)
    n = 2000
    x, y, z = rng.standard_normal((3, n))
    m = rng.uniform(0.5, 1.5, n)
    t = orc.Tree(x, y, z, m, n_leaf=8, n_grp=32)
    t.make_lists(0.5)
    f0 = t.force_lists(2, 0.01, 1.0)
    t.refresh(x, y, z, m)
    f1 = t.force_lists(2, 0.01, 1.0)
    for a, b in zip(f0, f1):
        np.testing.assert_array_equal(a, b)
    # doubling every mass doubles every force on frozen lists
    t.refresh(x, y, z, 2 * m)
    f2 = t.force_lists(2, 0.01, 1.0)
    for a, b in zip(f0, f2):
        np.testing.assert_allclose(b, 2 * a, rtol=1e-12)
