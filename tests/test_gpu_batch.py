"""Batched independent systems (one context, one set of launches): every
system of a batch gets the keys, tree, groups and lists it gets when run
alone (bit-exact, ids shifted by the system's first slot / first cell), the
same forces, and matches the FP64 oracle run on that system alone."""
import numpy as np
import pytest

import oracle
import workloads
import paper_1907_02290_amd as nb
from test_gpu_graph import OracleRun
from test_gpu_parity import check_forces

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _batch(seed=7, n_sys=7, lo=6, hi=13):
    return workloads.clusters(n_sys, seed, lo_exp=lo, hi_exp=hi)


def _ctx(d, order=1, n_grp=64):
    ctx = nb.Context(theta=0.5, eps=0.01, n_leaf=8, n_grp=n_grp, order=order)
    ctx.set_particles(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"],
                      d["m"])
    return ctx


def _sub(d, b, e):
    return {k: d[k][b:e].copy() for k in ("x", "y", "z", "vx", "vy", "vz",
                                           "m")}


@pytest.mark.parametrize("order", [1, 2])
def test_batch_equals_systems_run_alone(order):
    say("case batch vs alone order=%d" % order)
    d = _batch()
    off = d["offsets"]
    with _ctx(d, order) as ctx:
        ctx.set_systems(off)
        ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        key, orig = ctx.get_keys()
        c = ctx.get_cells()
        g = ctx.get_groups()
        eo, e, so, s = ctx.get_lists()
        f = ctx.get_forces()
        lo, k = ctx.get_roots()
    roots = np.nonzero(c["level"] == 0)[0]
    assert roots.size == off.size - 1
    ncell = np.append(roots, c["level"].size)
    for si in range(off.size - 1):
        b, en = int(off[si]), int(off[si + 1])
        sub = _sub(d, b, en)
        with _ctx(sub, order) as one:
            one.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
            k1, o1 = one.get_keys()
            c1 = one.get_cells()
            g1 = one.get_groups()
            eo1, e1, so1, s1 = one.get_lists()
            f1 = one.get_forces()
            lo1, kk1 = one.get_root()
        np.testing.assert_array_equal(lo[si], lo1)
        assert k[si] == kk1
        np.testing.assert_array_equal(key[b:en], k1)
        np.testing.assert_array_equal(orig[b:en], o1 + b)
        c0, c_end = int(ncell[si]), int(ncell[si + 1])
        assert c_end - c0 == c1["level"].size
        for fld in ("level", "begin", "count", "skip", "leaf", "ctr"):
            got = c[fld][c0:c_end]
            want = c1[fld]
            if fld == "begin":
                want = want + b
            if fld == "skip":
                want = want + c0
            np.testing.assert_array_equal(got, want, err_msg=fld)
        par = c["parent"][c0:c_end].astype(np.int64)
        par1 = c1["parent"].astype(np.int64)
        np.testing.assert_array_equal(par[1:], par1[1:] + c0)
        # groups of this system
        gs = np.nonzero((g["begin"] >= b) & (g["begin"] < en))[0]
        np.testing.assert_array_equal(g["begin"][gs], g1["begin"] + b)
        np.testing.assert_array_equal(g["cell"][gs], g1["cell"] + c0)
        np.testing.assert_array_equal(g["lo"][gs], g1["lo"])
        for j, gi in enumerate(gs):
            np.testing.assert_array_equal(e[eo[gi]:eo[gi + 1]],
                                          e1[eo1[j]:eo1[j + 1]] + b)
            np.testing.assert_array_equal(s[so[gi]:so[gi + 1]],
                                          s1[so1[j]:so1[j + 1]] + c0)
        for a, a1 in zip(f, f1):
            np.testing.assert_array_equal(a[b:en], a1)


def test_batch_matches_oracle_per_system():
    say("case batch vs oracle")
    d = _batch(seed=11, n_sys=5, lo=8, hi=12)
    off = d["offsets"]
    with _ctx(d) as ctx:
        ctx.set_systems(off)
        ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        key, orig = ctx.get_keys()
        eo, e, so, s = ctx.get_lists()
        g = ctx.get_groups()
        c = ctx.get_cells()
        f = ctx.get_forces()
    roots = np.nonzero(c["level"] == 0)[0]
    for si in range(off.size - 1):
        b, en = int(off[si]), int(off[si + 1])
        sub = _sub(d, b, en)
        t = oracle.Tree(sub["x"], sub["y"], sub["z"], sub["m"], 8, 64)
        t.make_lists(0.5)
        ok, op = t.keys()
        np.testing.assert_array_equal(key[b:en], ok)
        np.testing.assert_array_equal(orig[b:en], op + b)
        oeo, oe, oso, os_ = t.lists()
        gs = np.nonzero((g["begin"] >= b) & (g["begin"] < en))[0]
        assert gs.size == t.n_groups
        for j, gi in enumerate(gs):
            np.testing.assert_array_equal(e[eo[gi]:eo[gi + 1]],
                                          oe[oeo[j]:oeo[j + 1]] + b)
            np.testing.assert_array_equal(s[so[gi]:so[gi + 1]],
                                          os_[oso[j]:oso[j + 1]] + roots[si])
        ref = t.force_lists(1, 0.01, 1.0)
        num = np.sqrt(sum((a[b:en] - r) ** 2 for a, r in zip(f[:3], ref[:3])))
        den = np.sqrt(sum(r ** 2 for r in ref[:3]))
        assert np.median(num / den) < 1e-5


def test_batch_many_groups_two_lane_walk_and_slabs():
    """Enough groups for the walk on two lanes per group; the second
    construction (same positions) writes its tokens into per-group slabs in
    one pass.  Both give every system the oracle's lists."""
    say("case batch many groups")
    d = _batch(seed=13, n_sys=4, lo=13, hi=15)
    off = d["offsets"]
    with _ctx(d, n_grp=4) as ctx:
        ctx.set_systems(off)
        ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        assert ctx.get_info()["n_groups"] >= 8192
        first = ctx.get_lists()
        ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)  # one pass, slabs
        eo, e, so, s = ctx.get_lists()
        for a, b in zip(first, (eo, e, so, s)):
            np.testing.assert_array_equal(a, b)
        g = ctx.get_groups()
        c = ctx.get_cells()
    roots = np.nonzero(c["level"] == 0)[0]
    for si in range(off.size - 1):
        b, en = int(off[si]), int(off[si + 1])
        sub = _sub(d, b, en)
        t = oracle.Tree(sub["x"], sub["y"], sub["z"], sub["m"], 8, 4)
        t.make_lists(0.5)
        oeo, oe, oso, os_ = t.lists()
        gs = np.nonzero((g["begin"] >= b) & (g["begin"] < en))[0]
        assert gs.size == t.n_groups
        for j, gi in enumerate(gs):
            np.testing.assert_array_equal(e[eo[gi]:eo[gi + 1]],
                                          oe[oeo[j]:oeo[j + 1]] + b)
            np.testing.assert_array_equal(s[so[gi]:so[gi + 1]],
                                          os_[oso[j]:oso[j + 1]] + roots[si])


def test_batch_reuse_steps_stay_independent():
    say("case batch reuse")
    d = _batch(seed=3, n_sys=4, lo=8, hi=11)
    off = d["offsets"]
    dt = 1 / 64
    with _ctx(d) as ctx:
        ctx.set_systems(off)
        ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        for step in range(3):
            ctx.kick_drift(dt, dt)
            ctx.compute_forces(nb.NB_REUSE_LIST)
        st = ctx.get_state()
    for si in range(off.size - 1):
        b, en = int(off[si]), int(off[si + 1])
        with _ctx(_sub(d, b, en)) as one:
            one.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
            for step in range(3):
                one.kick_drift(dt, dt)
                one.compute_forces(nb.NB_REUSE_LIST)
            st1 = one.get_state()
        for a, a1 in zip(st, st1):
            np.testing.assert_array_equal(a[b:en], a1)


def test_set_systems_rejects_bad_offsets():
    say("case bad offsets")
    d = _batch(seed=1, n_sys=3, lo=6, hi=7)
    with _ctx(d) as ctx:
        n = d["x"].size
        for bad in ([0, 5, 5, n], [1, 5, n], [0, 5, n - 1], [0, n + 1]):
            with pytest.raises(nb.NbError) as err:
                ctx.set_systems(bad)
            assert err.value.code == nb.NB_ERR_INPUT


@pytest.mark.parametrize("order", [1, 2])
def test_persistent_force_launch_is_bit_identical(order):
    """Resident workgroups pulling work items from per-XCD counters compute
    each work item exactly as the one-workgroup-per-item launch does, and
    both match the oracle on the construction and the reuse step."""
    say("case persistent force order=%d" % order)
    d = _batch(seed=7, n_sys=6, lo=9, hi=14)
    out = []
    for persistent in (False, True):
        orc = OracleRun(d["m"], d["offsets"], 64, order)
        ctx = nb.Context(theta=0.5, eps=0.01, n_leaf=8, n_grp=64, order=order,
                         persistent=persistent)
        ctx.set_particles(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"],
                          d["m"])
        ctx.set_systems(d["offsets"])
        ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        f0 = ctx.get_forces()
        check_forces(f0, orc.step(ctx.get_state(), True),
                     what="persistent=%d construction" % persistent)
        ctx.kick_drift(1 / 128, 1 / 128)
        ctx.compute_forces(nb.NB_REUSE_LIST)
        f1 = ctx.get_forces()
        check_forces(f1, orc.step(ctx.get_state(), False),
                     what="persistent=%d reuse" % persistent)
        out.append((f0, f1))
        ctx.close()
    for step in (0, 1):
        for a, b in zip(out[0][step], out[1][step]):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("n_grp", [8, 64, 256])
def test_copied_lists_give_the_same_forces(n_grp):
    """Lists of copied j-data (the paper's method G1) give the forces of
    index lists (G2) bit for bit, on a construction and a reuse step, and
    both match the oracle's FP64 sums over the same lists."""
    say("case copied lists n_grp=%d" % n_grp)
    d = _batch(seed=9, n_sys=5, lo=9, hi=14)
    out = []
    for copied in (False, True):
        orc = OracleRun(d["m"], d["offsets"], n_grp, 1)
        ctx = nb.Context(theta=0.5, eps=0.01, n_leaf=8, n_grp=n_grp, order=1,
                         copied_lists=copied)
        ctx.set_particles(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"],
                          d["m"])
        ctx.set_systems(d["offsets"])
        ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        f0 = ctx.get_forces()
        check_forces(f0, orc.step(ctx.get_state(), True),
                     what="copied=%d construction" % copied)
        ctx.kick_drift(1 / 128, 1 / 128)
        ctx.compute_forces(nb.NB_REUSE_LIST)
        f1 = ctx.get_forces()
        check_forces(f1, orc.step(ctx.get_state(), False),
                     what="copied=%d reuse" % copied)
        out.append((f0, f1))
        ctx.close()
    for step in (0, 1):
        for a, b in zip(out[0][step], out[1][step]):
            np.testing.assert_array_equal(a, b)


def test_copied_lists_config_errors():
    for kw in (dict(order=2), dict(refresh=True), dict(persistent=True)):
        with pytest.raises(nb.NbError):
            nb.Context(copied_lists=True, **kw)
