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


def test_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(3)
    w = rng.standard_normal(NP) * 0.3
    x = rng.standard_normal((20, 12))
    y = (rng.uniform(size=20) > 0.5).astype(float)
    _, g = orc.mlp_loss_grad(w, x, y)
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
        fd = (orc.mlp_loss_grad(wp, x, y)[0] - orc.mlp_loss_grad(wm, x, y)[0]) / (2 * h)
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


def _brute_walk_box(t, c, gb, gn, lo, hi, theta):
    kids = _children(c)
    epj, spj, rat_a, rat_o = [], [], [], []

    def visit(cc):
        cb, cn = int(c["begin"][cc]), int(c["count"][cc])
        holds = cb <= gb and cb + cn >= gb + gn
        if not holds:
            side = 2.0 ** (t.k - int(c["level"][cc]))
            d = np.maximum(0.0, np.maximum(lo - c["ctr"][cc], c["ctr"][cc] - hi))
            d2 = float((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
            r2 = (side / theta) ** 2
            if d2 > r2:
                spj.append(cc)
                rat_a.append(d2 / r2)
                return
            rat_o.append(d2 / r2)
        if c["leaf"][cc]:
            epj.extend(range(cb, cb + cn))
            return
        for k in kids.get(cc, []):
            visit(k)

    visit(0)
    return epj, spj, min(rat_a, default=np.inf), max(rat_o, default=-np.inf)


def test_margins_and_staleness_against_brute_force(orc):
    rng = np.random.default_rng(8)
    n = 300
    x, y, z = rng.standard_normal((3, n))
    m = np.ones(n)
    t = orc.Tree(x, y, z, m, n_leaf=4, n_grp=8)
    theta = 0.6
    t.make_lists(theta)
    c, g = t.cells(), t.groups()
    key, perm = t.keys()
    amin, omax = t.margins(theta)
    for gi in range(t.n_groups):
        b, cnt = int(g["begin"][gi]), int(g["count"][gi])
        _, _, a, o = _brute_walk_box(t, c, b, cnt, g["lo"][gi], g["hi"][gi],
                                     theta)
        assert amin[gi] == pytest.approx(a, rel=1e-12) or amin[gi] == a
        assert omax[gi] == pytest.approx(o, rel=1e-12) or omax[gi] == o
        assert amin[gi] > 1.0 and omax[gi] <= 1.0
    # unmoved particles: nothing is stale
    st, lo, hi = t.stale(theta, x, y, z)
    assert not st.any()
    np.testing.assert_array_equal(lo, g["lo"])
    # moved particles: the flag says whether a walk with the new box differs
    v = rng.standard_normal((3, n)) * 0.05
    xn, yn, zn = x + v[0], y + v[1], z + v[2]
    st, lo, hi = t.stale(theta, xn, yn, zn)
    eo, e, so, s = t.lists()
    assert st.any() and not st.all()
    for gi in range(t.n_groups):
        b, cnt = int(g["begin"][gi]), int(g["count"][gi])
        pe, ps, _, _ = _brute_walk_box(t, c, b, cnt, lo[gi], hi[gi], theta)
        same = (pe == e[eo[gi]:eo[gi + 1]].tolist() and
                ps == s[so[gi]:so[gi + 1]].tolist())
        assert st[gi] == (not same), gi
        members = perm[b:b + cnt]
        np.testing.assert_array_equal(lo[gi], [xn[members].min(),
                                               yn[members].min(),
                                               zn[members].min()])
