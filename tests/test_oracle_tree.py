"""Pins of the oracle's octree link and particle groups (section 4.3, local
tree step 4; Barnes' vectorisation, section 2): invariants, and brute-force
enumeration of every cell on tiny inputs."""
import numpy as np
import pytest

MAXL = 21


def _systems():
    rng = np.random.default_rng(3)
    out = []
    for n in (1, 2, 9, 37, 64):
        out.append(rng.standard_normal((3, n)))
    # clustered + duplicated points (level-21 leaves with many particles)
    p = rng.standard_normal((3, 50)) * 1e-9
    p[:, :20] = 0.0
    out.append(p)
    return out


def _brute_cells(key, n_leaf):
    """Every (level, prefix) whose ancestors all hold > n_leaf particles,
    ordered by (begin, level): the DFS pre-order by definition."""
    key = np.asarray(key, dtype=np.uint64)
    n = key.size
    cells = []
    alive = {0: {0}}  # level -> prefixes that exist
    for lev in range(0, MAXL + 1):
        sh = np.uint64(3 * (MAXL - lev))
        pre = key >> sh
        for p in sorted(alive.get(lev, ())):
            idx = np.nonzero(pre == np.uint64(p))[0]
            if idx.size == 0:
                continue
            cnt = idx.size
            split = cnt > n_leaf and lev < MAXL
            cells.append((int(idx[0]), lev, p, cnt, not split))
            if split:
                kids = set(int(v) for v in (key[idx] >> np.uint64(3 * (MAXL - lev - 1))))
                alive.setdefault(lev + 1, set()).update(kids)
    cells.sort(key=lambda c: (c[0], c[1]))
    return cells


@pytest.mark.parametrize("case", range(6))
@pytest.mark.parametrize("n_leaf", [1, 4, 8])
def test_brute_force_cell_enumeration(orc, case, n_leaf):
    x, y, z = _systems()[case]
    n = x.size
    t = orc.Tree(x, y, z, np.ones(n), n_leaf=n_leaf, n_grp=8)
    key, _ = t.keys()
    ref = _brute_cells(key, n_leaf)
    c = t.cells()
    assert t.n_cell == len(ref)
    got = list(zip(c["begin"].tolist(), c["level"].tolist(),
                   c["prefix"].tolist(), c["count"].tolist(),
                   [bool(v) for v in c["leaf"]]))
    assert got == [(b, l, p, k, lf) for (b, l, p, k, lf) in ref]


def _check_tree(orc, t, n_leaf):
    key, _ = t.keys()
    c = t.cells()
    nc = t.n_cell
    begin = c["begin"].astype(np.int64)
    count = c["count"].astype(np.int64)
    end = begin + count
    lev = c["level"].astype(np.int64)
    # root
    assert begin[0] == 0 and count[0] == t.n and lev[0] == 0
    # members share the prefix
    for i in range(nc):
        sh = np.uint64(3 * (MAXL - lev[i]))
        ks = key[begin[i]:end[i]] >> sh
        assert np.all(ks == c["prefix"][i])
    # leaf rule
    leaf = c["leaf"].astype(bool)
    assert np.all(count[leaf & (lev < MAXL)] <= n_leaf)
    assert np.all(count[~leaf] > n_leaf)
    # leaves partition [0, n) in order
    lb, le = begin[leaf], end[leaf]
    assert lb[0] == 0 and le[-1] == t.n and np.all(lb[1:] == le[:-1])
    # children partition the parent, in octant order
    par = c["parent"].astype(np.int64)
    for p in np.nonzero(~leaf)[0]:
        kids = np.nonzero(par == p)[0]
        assert kids.size >= 1
        assert begin[kids[0]] == begin[p] and end[kids[-1]] == end[p]
        assert np.all(begin[kids[1:]] == end[kids[:-1]])
        assert np.all(lev[kids] == lev[p] + 1)
        assert kids[0] == p + 1  # first child follows in pre-order
    # pre-order: sorted by (begin, level); skip = end of subtree
    order = np.lexsort((lev, begin))
    np.testing.assert_array_equal(order, np.arange(nc))
    for i in range(nc):
        s = int(c["skip"][i])
        sub = np.arange(i + 1, s)
        assert np.all(begin[sub] >= begin[i]) and np.all(end[sub] <= end[i])
        assert s == nc or begin[s] >= end[i]
    return c


def test_tree_invariants_and_geometry(orc):
    rng = np.random.default_rng(9)
    n = 5000
    x, y, z = rng.standard_normal((3, n)) ** 3  # strongly clustered
    m = rng.uniform(0.5, 1.5, n)
    t = orc.Tree(x, y, z, m, n_leaf=8, n_grp=64)
    key, perm = t.keys()
    t_pos = (x[perm], y[perm], z[perm])
    c = _check_tree(orc, t, 8)
    # every member inside [ctr - s/2, ctr + s/2]
    for i in range(0, t.n_cell, 7):
        side = 2.0 ** (t.k - int(c["level"][i]))
        b, e = int(c["begin"][i]), int(c["begin"][i] + c["count"][i])
        for a in range(3):
            lo = c["ctr"][i, a] - side / 2
            hi = c["ctr"][i, a] + side / 2
            pa = t_pos[a][b:e]
            assert np.all(pa >= lo - 1e-12 * abs(lo)) and np.all(pa <= hi)


def test_moments_definition(orc):
    rng = np.random.default_rng(21)
    n = 400
    x, y, z = rng.standard_normal((3, n))
    m = rng.uniform(0.1, 2.0, n)
    t = orc.Tree(x, y, z, m, n_leaf=4, n_grp=16)
    key, perm = t.keys()
    c = t.cells()
    M, X, S = t.moments()
    P = np.stack([x[perm], y[perm], z[perm]], 1)
    ms = m[perm]
    # root: whole-system moments; leaves: brute force over members
    for i in [0] + list(range(1, t.n_cell, 5)):
        b, e = int(c["begin"][i]), int(c["begin"][i] + c["count"][i])
        mm, pp = ms[b:e], P[b:e]
        assert M[i] == pytest.approx(mm.sum(), rel=1e-14)
        com = (mm[:, None] * pp).sum(0) / mm.sum()
        np.testing.assert_allclose(X[i], com, rtol=1e-12, atol=1e-14)
        d = pp - com
        full = (mm[:, None, None] * d[:, :, None] * d[:, None, :]).sum(0)
        want = [full[0, 0], full[1, 1], full[2, 2], full[0, 1], full[0, 2],
                full[1, 2]]
        np.testing.assert_allclose(S[i], want, rtol=1e-10, atol=1e-14)
    # parallel-axis identity: parent second moment = sum over children
    par = c["parent"].astype(np.int64)
    for p in np.nonzero(c["leaf"] == 0)[0][:50]:
        kids = np.nonzero(par == p)[0]
        tot = np.zeros((3, 3))
        for kk in kids:
            s6 = S[kk]
            Sk = np.array([[s6[0], s6[3], s6[4]], [s6[3], s6[1], s6[5]],
                           [s6[4], s6[5], s6[2]]])
            dd = X[kk] - X[p]
            tot += Sk + M[kk] * np.outer(dd, dd)
        s6 = S[p]
        Sp = np.array([[s6[0], s6[3], s6[4]], [s6[3], s6[1], s6[5]],
                       [s6[4], s6[5], s6[2]]])
        np.testing.assert_allclose(Sp, tot, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("n_grp", [1, 8, 64, 512])
def test_groups_partition_and_maximality(orc, n_grp):
    rng = np.random.default_rng(17)
    n = 3000
    x, y, z = rng.standard_normal((3, n))
    t = orc.Tree(x, y, z, np.ones(n), n_leaf=8, n_grp=n_grp)
    key, perm = t.keys()
    c = t.cells()
    g = t.groups()
    gb = g["begin"].astype(np.int64)
    ge = gb + g["count"]
    assert gb[0] == 0 and ge[-1] == n and np.all(gb[1:] == ge[:-1])
    for i in range(t.n_groups):
        cell = int(g["cell"][i])
        assert c["begin"][cell] == gb[i] and c["count"][cell] == g["count"][i]
        assert g["count"][i] <= n_grp or c["leaf"][cell]
        if cell != 0:
            assert c["count"][c["parent"][cell]] > n_grp
        np.testing.assert_array_equal(g["ctr"][i], c["ctr"][cell])
        pts = np.stack([x[perm[gb[i]:ge[i]]], y[perm[gb[i]:ge[i]]],
                        z[perm[gb[i]:ge[i]]]], 1)
        np.testing.assert_array_equal(g["lo"][i], pts.min(0))
        np.testing.assert_array_equal(g["hi"][i], pts.max(0))


def test_single_group_when_small(orc):
    rng = np.random.default_rng(2)
    x, y, z = rng.standard_normal((3, 40))
    t = orc.Tree(x, y, z, np.ones(40), n_leaf=8, n_grp=64)
    g = t.groups()
    assert t.n_groups == 1 and g["cell"][0] == 0 and g["count"][0] == 40
