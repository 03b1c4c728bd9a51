"""Pins of the oracle's rebuild-predictor pieces: the perceptron (closed
forms, finite-difference gradients, convergence), the Adam step (closed form
of the first step), the opening-test margins and the staleness flags
(against a brute-force recursive walk with the current boxes)."""
import numpy as np
import pytest

NP = 12 * 64 + 64 + 64 * 64 + 64 + 64 + 1


def test_parameter_count(orc):
    assert orc.mlp_nparam() == NP


def test_zero_weights_closed_form(orc):
    rng = np.random.default_rng(0)
    x = rng.standard_normal((50, 12))
    y = (rng.uniform(size=50) > 0.3).astype(float)
    w = np.zeros(NP)
    p = orc.mlp_forward(w, x)
    np.testing.assert_array_equal(p, 0.5)
    loss, g = orc.mlp_loss_grad(w, x, y)
    assert loss == pytest.approx(np.log(2.0), rel=1e-14)
    assert g[-1] == pytest.approx(np.mean(0.5 - y), rel=1e-13)
    assert np.all(g[:-1] == 0.0)


def test_zero_weights_positive_weight(orc):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((40, 12))
    y = (rng.uniform(size=40) > 0.6).astype(float)
    w = np.zeros(NP)
    loss, g = orc.mlp_loss_grad(w, x, y, pos_weight=3.0)
    yb = y.mean()
    assert loss == pytest.approx(np.log(2.0) * (3.0 * yb + 1.0 - yb),
                                 rel=1e-14)
    assert g[-1] == pytest.approx(np.mean(0.5 * (3 * y + 1 - y) - 3 * y),
                                  rel=1e-13)


def test_output_bias_only(orc):
    w = np.zeros(NP)
    w[-1] = 1.3
    p = orc.mlp_forward(w, np.ones((3, 12)))
    np.testing.assert_allclose(p, 1.0 / (1.0 + np.exp(-1.3)), rtol=1e-15)


def test_single_path_closed_form(orc):
    # one input -> one hidden unit -> one hidden unit -> output
    w = np.zeros(NP)
    w[0 * 12 + 3] = 0.7            # W1[0][3]
    w[768 + 0] = -0.2              # b1[0]
    w[832 + 5 * 64 + 0] = 1.1      # W2[5][0]
    w[832 + 4096 + 5] = 0.05       # b2[5]
    w[832 + 4096 + 64 + 5] = 2.0   # w3[5]
    w[-1] = -0.4
    x = np.zeros((1, 12))
    x[0, 3] = 0.9
    h1 = np.tanh(0.7 * 0.9 - 0.2)
    h2 = np.tanh(1.1 * h1 + 0.05)
    want = 1.0 / (1.0 + np.exp(-(2.0 * h2 - 0.4)))
    assert orc.mlp_forward(w, x)[0] == pytest.approx(want, rel=1e-15)


@pytest.mark.parametrize("pw", [1.0, 4.0])
def test_gradient_matches_finite_differences(orc, pw):
    rng = np.random.default_rng(3)
    w = rng.standard_normal(NP) * 0.3
    x = rng.standard_normal((20, 12))
    y = (rng.uniform(size=20) > 0.5).astype(float)
    _, g = orc.mlp_loss_grad(w, x, y, pw)
    idx = np.concatenate([rng.choice(768, 40, replace=False),
                          768 + np.arange(0, 64, 9),
                          832 + rng.choice(4096, 40, replace=False),
                          4928 + np.arange(0, 64, 9),
                          4992 + np.arange(0, 64, 9), [NP - 1]])
    h = 1e-6
    for k in idx:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (orc.mlp_loss_grad(wp, x, y, pw)[0] -
              orc.mlp_loss_grad(wm, x, y, pw)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-9, k


def test_adam_first_step_closed_form(orc):
    rng = np.random.default_rng(4)
    w = rng.standard_normal(NP)
    g = rng.standard_normal(NP)
    m = np.zeros(NP)
    v = np.zeros(NP)
    w0 = w.copy()
    orc.adam(w, g, m, v, 1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(w, w0 - 0.01 * np.sign(g), rtol=0, atol=1e-9)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)


def test_training_learns_a_separable_rule(orc):
    rng = np.random.default_rng(5)
    x = rng.standard_normal((400, 12))
    y = (x[:, 0] + 0.5 * x[:, 1] - x[:, 2] > 0).astype(float)
    w = rng.standard_normal(NP) * 0.1
    m = np.zeros(NP)
    v = np.zeros(NP)
    loss0 = orc.mlp_loss_grad(w, x, y)[0]
    for t in range(1, 301):
        loss, g = orc.mlp_loss_grad(w, x, y)
        orc.adam(w, g, m, v, t, lr=0.01)
    acc = np.mean((orc.mlp_forward(w, x) > 0.5) == (y > 0.5))
    assert loss < 0.2 * loss0 and acc > 0.97


def _children(c):
    par = c["parent"].astype(np.int64)
    kids = {}
    for i in range(1, par.size):
        kids.setdefault(int(par[i]), []).append(i)
    return kids


def _sides(t, c, shift, pos):
    """Brute-force opening-test sides: max(geometric side, twice the largest
    per-axis distance from the moved centre to a member particle)."""
    key, perm = t.keys()
    p = np.stack([a[perm] for a in pos], axis=1)   # sorted order
    out = np.empty(t.n_cell)
    for cc in range(t.n_cell):
        b, n = int(c["begin"][cc]), int(c["count"][cc])
        ctr = c["ctr"][cc] + shift[cc]
        h = np.abs(p[b:b + n] - ctr).max()
        out[cc] = max(2.0 ** (t.k - int(c["level"][cc])), 2.0 * h)
    return out


def _brute_walk(t, c, kids, shift, gb, gn, lo, hi, theta, sides=None):
    """Recursive walk (an independent restatement of the stackless one):
    returns EPJ ids, SPJ ids and the two opening-test slacks."""
    epj, spj, sa, so = [], [], [np.inf], [np.inf]

    def visit(cc):
        cb, cn = int(c["begin"][cc]), int(c["count"][cc])
        if not (cb <= gb and cb + cn >= gb + gn):
            side = (2.0 ** (t.k - int(c["level"][cc])) if sides is None
                    else sides[cc])
            ctr = c["ctr"][cc] + shift[cc]
            d = np.maximum(0.0, np.maximum(lo - ctr, ctr - hi))
            dist = float(np.sqrt(d @ d))
            r = side / theta
            if dist > r:
                spj.append(cc)
                sa[0] = min(sa[0], dist - r)
                return
            so[0] = min(so[0], r - dist)
        if c["leaf"][cc]:
            epj.extend(range(cb, cb + cn))
            return
        for k in kids.get(cc, []):
            visit(k)

    visit(0)
    return epj, spj, sa[0], so[0]


def _setup(orc, n=300, seed=8, theta=0.6):
    rng = np.random.default_rng(seed)
    x, y, z = rng.standard_normal((3, n))
    m = np.full(n, 1.0 / n)
    t = orc.Tree(x, y, z, m, n_leaf=4, n_grp=8)
    t.make_lists(theta)
    return rng, (x, y, z, m), t


def test_slacks_against_brute_force(orc):
    theta = 0.6
    _, _, t = _setup(orc, theta=theta)
    c, g = t.cells(), t.groups()
    kids = _children(c)
    sa, so = t.margins()
    zero = np.zeros((t.n_cell, 3))
    eo, e, so_, s = t.lists()
    for gi in range(t.n_groups):
        b, cnt = int(g["begin"][gi]), int(g["count"][gi])
        pe, ps, a, o = _brute_walk(t, c, kids, zero, b, cnt, g["lo"][gi],
                                   g["hi"][gi], theta)
        assert pe == e[eo[gi]:eo[gi + 1]].tolist()
        assert ps == s[so_[gi]:so_[gi + 1]].tolist()
        assert sa[gi] == pytest.approx(a, rel=1e-12, abs=1e-15)
        assert so[gi] == pytest.approx(o, rel=1e-12, abs=1e-15)
        assert sa[gi] > 0.0 and so[gi] >= 0.0


def test_cell_sides_are_geometric_until_particles_spread(orc):
    _, (x, y, z, m), t = _setup(orc)
    c = t.cells()
    geo = 2.0 ** (t.k - c["level"].astype(float))
    np.testing.assert_array_equal(t.cell_sides(), geo)
    # a rigid shift keeps every cell's particles about its moved centre
    t.refresh(x + 0.5, y - 0.25, z + 0.125, m)
    np.testing.assert_allclose(t.cell_sides(), geo, rtol=1e-12)
    # stretching by 3 along x: the top cell's particles reach 3x as far
    t.refresh(3.0 * x, y, z, m)
    s = t.cells()
    sides = t.cell_sides()
    assert sides[0] > geo[0]


def test_unmoved_particles_are_not_stale(orc):
    _, (x, y, z, m), t = _setup(orc)
    t.refresh(x, y, z, m)
    st, lo, _ = t.stale(0.6)
    assert not st.any()
    # tau = 0 fires exactly where a kept superparticle fails the test: none
    # right after construction
    np.testing.assert_array_equal(lo, t.groups()["lo"])
    f = t.features(8, np.full(t.n_groups, 3))
    np.testing.assert_array_equal(f[:, 0], 3.0 / 8.0)
    # no box change and no cell shift: the motion features vanish
    np.testing.assert_array_equal(f[:, [1, 2, 3, 4, 5, 6, 9]], 0.0)


def test_rigid_motion_changes_no_list(orc):
    # coordinates on a 2^-30 grid, a shift on the same grid: every shifted
    # position is exact, so only the centre-of-mass division rounds
    rng = np.random.default_rng(11)
    n = 400
    q = lambda a: np.round(a * 2.0**30) / 2.0**30
    x, y, z = q(rng.standard_normal((3, n)))
    m = np.full(n, 2.0**-9)
    t = orc.Tree(x, y, z, m, n_leaf=4, n_grp=8)
    t.make_lists(0.5)
    v = np.array([0.25, -0.375, 0.125])
    t.refresh(x + v[0], y + v[1], z + v[2], m)
    st, _, _ = t.stale(0.5)
    assert not st.any()
    f = t.features(4, np.ones(t.n_groups, np.int32))
    g = t.groups()
    c = t.cells()
    side = 2.0 ** (t.k - c["level"][g["cell"]].astype(float))
    assert np.all(f[:, [1, 2, 5, 9]] < 1e-12)
    np.testing.assert_allclose(f[:, 6], np.log1p(np.linalg.norm(v) / side),
                               rtol=1e-12)


def _violations(t, sides, shift, lo, hi, theta, tau, eo_so):
    """Direct check of every kept superparticle (vectorised restatement)."""
    c = t.cells()
    _, so, s = eo_so
    side = sides
    r2 = (side / (theta * (1.0 + tau))) ** 2
    ctr = c["ctr"] + shift
    out = np.zeros(t.n_groups, bool)
    for g in range(t.n_groups):
        cs = s[so[g]:so[g + 1]].astype(np.int64)
        d = np.maximum(0.0, np.maximum(lo[g] - ctr[cs], ctr[cs] - hi[g]))
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        out[g] = bool(np.any(~(d2 > r2[cs])))
    return out


def test_stale_and_refresh_against_brute_force(orc):
    theta = 0.6
    rng, (x, y, z, m), t = _setup(orc, theta=theta)
    _, com0, _ = t.moments()
    c, g = t.cells(), t.groups()
    kids = _children(c)
    eo0, e0, so0, s0 = t.lists()
    # a shear flow plus noise: some lists go stale, not all
    xn = x + 0.15 * y + 0.03 * rng.standard_normal(x.size)
    yn, zn = y.copy(), z + 0.03 * rng.standard_normal(x.size)
    t.refresh(xn, yn, zn, m)
    _, com, _ = t.moments()
    shift = com - com0
    key, perm = t.keys()
    sides = _sides(t, c, shift, (xn, yn, zn))
    np.testing.assert_allclose(t.cell_sides(), sides, rtol=1e-13)
    geo = 2.0 ** (t.k - c["level"].astype(float))
    assert np.all(sides >= geo) and np.any(sides > geo)
    st, lo, hi = t.stale(theta)
    st1, _, _ = t.stale(theta, 0.1)
    assert st.any() and not st.all()
    assert st1.any() and not np.array_equal(st1, st)
    assert not np.any(st1 & ~st)               # monotone in tau
    assert not t.stale(theta, 1e6)[0].any()
    np.testing.assert_array_equal(
        st, _violations(t, sides, shift, lo, hi, theta, 0.0, (eo0, so0, s0)))
    np.testing.assert_array_equal(
        st1, _violations(t, sides, shift, lo, hi, theta, 0.1, (eo0, so0, s0)))
    walked = {}
    for gi in range(t.n_groups):
        b, cnt = int(g["begin"][gi]), int(g["count"][gi])
        members = perm[b:b + cnt]
        np.testing.assert_array_equal(lo[gi], [xn[members].min(),
                                               yn[members].min(),
                                               zn[members].min()])
        pe, ps, a, o = _brute_walk(t, c, kids, shift, b, cnt, lo[gi], hi[gi],
                                   theta, sides)
        walked[gi] = (pe, ps, a, o)
        same = (pe == e0[eo0[gi]:eo0[gi + 1]].tolist() and
                ps == s0[so0[gi]:so0[gi + 1]].tolist())
        # a violated superparticle means a fresh walk opens it
        if st[gi]:
            assert not same, gi
    # refresh every other stale group and a few fresh ones
    sel = np.union1d(np.flatnonzero(st)[::2], np.arange(0, t.n_groups, 7))
    t.refresh_lists(theta, sel)
    eo, e, so_, s = t.lists()
    sa, so = t.margins()
    gg = t.groups()
    for gi in range(t.n_groups):
        if gi in set(sel.tolist()):
            pe, ps, a, o = walked[gi]
            assert pe == e[eo[gi]:eo[gi + 1]].tolist()
            assert ps == s[so_[gi]:so_[gi + 1]].tolist()
            assert sa[gi] == pytest.approx(a, rel=1e-12, abs=1e-15)
            assert so[gi] == pytest.approx(o, rel=1e-12, abs=1e-15)
            np.testing.assert_array_equal(gg["lo"][gi], lo[gi])
        else:
            assert e[eo[gi]:eo[gi + 1]].tolist() == \
                e0[eo0[gi]:eo0[gi + 1]].tolist()
            assert s[so_[gi]:so_[gi + 1]].tolist() == \
                s0[so0[gi]:so0[gi + 1]].tolist()
    st2, _, _ = t.stale(theta)
    np.testing.assert_array_equal(st2, st & ~np.isin(np.arange(t.n_groups),
                                                     sel))
    # refreshed groups start from their new box: no box change, no shift
    f = t.features(8, np.zeros(t.n_groups, np.int32))
    assert np.all(f[sel][:, [1, 2, 3, 4, 5, 6, 9]] == 0.0)


def test_feature_counts_and_caps(orc):
    _, _, t = _setup(orc)
    g = t.groups()
    eo, _, so, _ = t.lists()
    sa, so_ = t.margins()
    f = t.features(4, np.array([0, 9] * (t.n_groups // 2) +
                               [2] * (t.n_groups % 2), np.int32))
    np.testing.assert_allclose(f[:, 10], np.log2(g["count"]) / 6, rtol=1e-15)
    nl = np.diff(eo) + np.diff(so)
    np.testing.assert_allclose(f[:, 11], np.log2(1.0 + nl) / 16, rtol=1e-15)
    assert set(np.unique(f[:, 0])) <= {0.0, 0.5, 1.0}
    # slacks of +inf (no accepted / no opened cell) hit the cap
    cap = np.log1p(1e6)
    assert np.all(f[np.isinf(sa), 7] == cap)
    assert np.all(f[np.isinf(so_), 8] == cap)
    assert np.all(f[:, 7:9] <= cap)


def test_slack_and_shift_features_by_hand(orc):
    """f3, f4, f7, f8 at non-trivial values: a rigid translation v of a
    tree on a 2^-30 grid gives every cell the shift v (B = |v|, E = 0);
    the slacks come from the brute-force walk above, not from the oracle.
    Rows with finite, distinct sa and so tell the four inputs apart (a swap
    of sa and so, or of B and E, fails)."""
    rng = np.random.default_rng(21)
    n = 400
    q = lambda a: np.round(a * 2.0**30) / 2.0**30
    x, y, z = q(rng.standard_normal((3, n)))
    m = np.full(n, 2.0**-9)
    theta = 0.55
    t = orc.Tree(x, y, z, m, n_leaf=4, n_grp=8)
    t.make_lists(theta)
    c, g = t.cells(), t.groups()
    kids = _children(c)
    zero = np.zeros((t.n_cell, 3))
    v = np.array([0.0625, -0.09375, 0.03125])
    t.refresh(x + v[0], y + v[1], z + v[2], m)
    f = t.features(4, np.full(t.n_groups, 2, np.int32))
    B = float(np.linalg.norm(v))
    cap = 1e6
    rows = 0
    for gi in range(t.n_groups):
        b, cnt = int(g["begin"][gi]), int(g["count"][gi])
        _, _, sa, so = _brute_walk(t, c, kids, zero, b, cnt, g["lo"][gi],
                                   g["hi"][gi], theta)
        if not (np.isfinite(sa) and np.isfinite(so) and sa > 0 and so > 0
                and abs(sa - so) > 0.1 * max(sa, so)):
            continue
        rows += 1
        s = 2.0 ** (t.k - int(c["level"][int(g["cell"][gi])]))
        want = {3: np.log1p(min(B / sa, cap)), 4: np.log1p(min(B / so, cap)),
                7: np.log1p(min(sa / s, cap)), 8: np.log1p(min(so / s, cap))}
        for k, w in want.items():
            assert f[gi, k] == pytest.approx(w, rel=1e-9), (gi, k)
        # no deformation: E = 0, so the box-motion inputs vanish
        assert f[gi, 1] < 1e-12 and f[gi, 2] < 1e-12
        assert f[gi, 0] == 0.5
    assert rows >= 10, rows
