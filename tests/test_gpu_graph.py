"""Reuse steps replayed from a captured HIP graph give exactly the results of
the same steps launched one by one: every replay is checked, with readbacks
(eager work and synchronisation) between replays, across construction steps
and a change of time step.  Every step's forces are also checked against the
FP64 oracle: its tree is built on the GPU's own positions at each
construction step and refreshed with them at each reuse step (section 4.2:
moments over the frozen tree), then summed over the same lists."""
import numpy as np
import pytest

import oracle
import workloads
import paper_1907_02290_amd as nb
from test_gpu_parity import check_forces

pytestmark = pytest.mark.gpu


def _pair(d, **kw):
    out = []
    for graph in (True, False):
        ctx = nb.Context(theta=0.5, eps=0.01, n_leaf=8, graph=graph, **kw)
        ctx.set_particles(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"],
                          d["m"])
        out.append(ctx)
    return out


class OracleRun:
    """The oracle following a run of one system (or a batch of independent
    systems, offsets `off`) on the GPU's positions."""

    def __init__(self, m, off, n_grp, order, eps=0.01):
        self.m, self.off, self.n_grp = m, off, n_grp
        self.order, self.eps = order, eps
        self.trees = None

    def step(self, state, construct):
        x, y, z = state[:3]
        parts = range(self.off.size - 1)
        if construct or self.trees is None:
            self.trees = []
            for s in parts:
                b, e = int(self.off[s]), int(self.off[s + 1])
                t = oracle.Tree(x[b:e], y[b:e], z[b:e], self.m[b:e], 8,
                                self.n_grp)
                t.make_lists(0.5)
                self.trees.append(t)
        else:
            for s, t in zip(parts, self.trees):
                b, e = int(self.off[s]), int(self.off[s + 1])
                t.refresh(x[b:e], y[b:e], z[b:e], self.m[b:e])
        refs = [t.force_lists(self.order, self.eps, 1.0) for t in self.trees]
        return tuple(np.concatenate([r[k] for r in refs]) for k in range(4))


@pytest.mark.parametrize("order,n_grp", [(1, 64), (2, 256)])
def test_graph_replays_match_eager_steps(order, n_grp):
    print("case graph order=%d n_grp=%d" % (order, n_grp), flush=True)
    d = workloads.plummer(20000, workloads.seed_for(1, 9))
    orc = OracleRun(d["m"], np.array([0, d["x"].size]), n_grp, order)
    g, e = _pair(d, order=order, n_grp=n_grp)
    with g, e:
        for c in (g, e):
            c.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        check_forces(g.get_forces(), orc.step(g.get_state(), True),
                     what="step 0")
        dt = 1 / 128
        for step in range(1, 14):
            if step == 9:
                dt = 1 / 256  # a new time step drops and recaptures the graph
            mode = nb.NB_MAKE_LIST_FOR_REUSE if step % 4 == 0 else \
                nb.NB_REUSE_LIST
            for c in (g, e):
                c.step(mode, dt, dt)
            fg, fe = g.get_forces(internal=True), e.get_forces(internal=True)
            for a, b in zip(fg, fe):
                np.testing.assert_array_equal(a, b, err_msg="step %d" % step)
            sg, se = g.get_state(internal=True), e.get_state(internal=True)
            for a, b in zip(sg, se):
                np.testing.assert_array_equal(a, b, err_msg="step %d" % step)
            check_forces(g.get_forces(),
                         orc.step(g.get_state(),
                                  mode == nb.NB_MAKE_LIST_FOR_REUSE),
                         what="step %d" % step)
        ig, ie = g.get_info(), e.get_info()
        assert ig["force_evals"] == ie["force_evals"] == 14
        assert ig["total_inter"] == ie["total_inter"]


def test_graph_with_batched_systems():
    print("case graph batch", flush=True)
    d = workloads.clusters(6, 5, lo_exp=8, hi_exp=12)
    orc = OracleRun(d["m"], d["offsets"], 64, 1)
    g, e = _pair(d)
    with g, e:
        for c in (g, e):
            c.set_systems(d["offsets"])
            c.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        orc.step(g.get_state(), True)
        for step in range(1, 9):
            mode = nb.NB_MAKE_LIST_FOR_REUSE if step % 4 == 0 else \
                nb.NB_REUSE_LIST
            for c in (g, e):
                c.step(mode, 1 / 128, 1 / 128)
            for a, b in zip(g.get_state(), e.get_state()):
                np.testing.assert_array_equal(a, b)
            check_forces(g.get_forces(),
                         orc.step(g.get_state(),
                                  mode == nb.NB_MAKE_LIST_FOR_REUSE),
                         what="batch step %d" % step)


@pytest.mark.parametrize("mode,n,n_grp,steps", [("check", 6000, 32, 8),
                                                ("refresh", 6000, 32, 8),
                                                ("refresh", 200000, 8, 4)])
def test_graph_replays_refresh_steps(mode, n, n_grp, steps):
    """Refresh mode: NB_REUSE_CHECK / NB_REUSE_REFRESH steps, whose
    selection, walk and in-place list refresh run without the host, are
    captured in a HIP graph; every replay gives exactly the eager steps'
    lists, forces, state and counts (readbacks between replays), across a
    construction step.  With the exact check (pure drifts, so the oracle
    follows the positions) the lists after every step are the oracle's
    refresh of the groups it flags at tau or by age.  The large case
    refreshes thousands of groups per step; its shear
    grows some lists past their slots by the third step (the oracle's
    refresh of every group shows it), and those groups keep their lists
    alike in both."""
    from test_gpu_learn import THETA, drift, sheared
    print("case graph refresh mode %s n=%d n_grp=%d" % (mode, n, n_grp),
          flush=True)
    d = sheared(n, 5)
    dt, tau, k_max = 1 / 64, 0.05, 5
    nbm = nb.NB_REUSE_CHECK if mode == "check" else nb.NB_REUSE_REFRESH
    rng = np.random.default_rng(3)
    w = (rng.standard_normal(nb.MLP_NPARAM) * 0.3).astype(np.float32)
    ctxs = []
    for graph in (True, False):
        c = nb.Context(theta=THETA, eps=0.01, n_leaf=8, n_grp=n_grp,
                       refresh=True, tau=tau, k_max=k_max, p_star=0.5,
                       graph=graph)
        c.set_particles(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"],
                        d["m"])
        c.mlp_set(w)
        ctxs.append(c)
    g, e = ctxs
    if mode == "check":
        t = oracle.Tree(d["x"], d["y"], d["z"], d["m"], 8, n_grp)
        t.make_lists(THETA)
        age = np.zeros(t.n_groups, int)
    with g, e:
        for c in (g, e):
            c.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        refreshed = 0
        for s in range(1, steps + 1):
            for c in (g, e):
                c.step(nbm, 0.0, dt)
            ig, ie = g.get_info(), e.get_info()
            for k in ("n_epj", "n_spj", "n_inter", "last_refreshed",
                      "total_refreshed", "total_inter", "last_overflow"):
                assert ig[k] == ie[k], (s, k, ig[k], ie[k])
            if n <= 6000:
                assert ig["last_overflow"] == 0
            refreshed += ig["last_refreshed"]
            for a, b in zip(g.get_lists(), e.get_lists()):
                np.testing.assert_array_equal(a, b, err_msg="step %d" % s)
            for a, b in zip(g.get_forces(internal=True),
                            e.get_forces(internal=True)):
                np.testing.assert_array_equal(a, b, err_msg="step %d" % s)
            for a, b in zip(g.get_state(internal=True),
                            e.get_state(internal=True)):
                np.testing.assert_array_equal(a, b, err_msg="step %d" % s)
            if mode == "check":
                x, y, z = drift(d, dt, s)
                t.refresh(x, y, z, d["m"])
                age += 1
                sel = np.flatnonzero(t.stale(THETA, tau)[0] | (age >= k_max))
                t.refresh_lists(THETA, sel)
                age[sel] = 0
                assert ig["last_refreshed"] == sel.size
                eo, ev, so, sv = g.get_lists()
                oeo, oe, oso, os_ = t.lists()
                np.testing.assert_array_equal(eo, oeo)
                np.testing.assert_array_equal(ev, oe)
                np.testing.assert_array_equal(so, oso)
                np.testing.assert_array_equal(sv, os_)
        assert refreshed > 0
        assert g.get_info()["total_refreshed"] == refreshed
