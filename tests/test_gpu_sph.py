"""GPU parity of the short-range path (section 2: the group walk with the
short-range opening rule; section 4.2: list reuse) against the FP64 oracle,
through the C ABI: neighbour lists bit-exact, SPH densities within the FP32
tolerance (median relative error <= 1e-5), reuse within the skin, batched
systems, error paths, and a full-size sampled check."""
import numpy as np
import pytest

import oracle
import workloads
import paper_1907_02290_amd as nb

pytestmark = pytest.mark.gpu

RHO_MEDIAN_TOL = 1e-5
RHO_MAX_TOL = 1e-3


def say(*a):
    print(*a, flush=True)


def _system(kind, n, seed=0):
    if kind == "plummer":
        return workloads.plummer(n, workloads.seed_for(1, seed))
    if kind == "disk":
        return workloads.disk_halo(n // 2, n - n // 2, workloads.seed_for(3, seed))
    if kind == "sphere":
        return workloads.uniform_sphere(n, workloads.seed_for(6, seed))
    if kind == "ring":
        return workloads.ring(n, workloads.seed_for(4, seed))
    raise KeyError(kind)


def _ctx(d, n_leaf=8, n_grp=64):
    ctx = nb.Context(theta=0.5, eps=0.01, n_leaf=n_leaf, n_grp=n_grp)
    ctx.set_particles(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"],
                      d["m"])
    return ctx


def _check_rho(got, want, what):
    err = np.abs(got - want) / np.abs(want)
    say("  %s rho rel err: median %.2e max %.2e" % (what, np.median(err),
                                                     err.max()))
    assert np.median(err) <= RHO_MEDIAN_TOL
    assert err.max() <= RHO_MAX_TOL


CASES = [("plummer", 4096, 0.05), ("plummer", 4096, 0.4), ("disk", 20000, 0.02),
         ("sphere", 5000, 0.12), ("ring", 12345, 0.003), ("plummer", 9, 0.5),
         ("plummer", 1, 0.1), ("plummer", 3000, 0.0)]


@pytest.mark.parametrize("kind,n,h", CASES)
def test_neighbour_lists_and_density(kind, n, h):
    say("case neighbour lists %s n=%d h=%g" % (kind, n, h))
    d = _system(kind, n)
    t = oracle.Tree(d["x"], d["y"], d["z"], d["m"], 8, 64)
    off, ids = t.neighbour_lists(h)
    with _ctx(d) as ctx:
        ctx.build_tree()
        ctx.neighbour_lists(h)
        goff, gids = ctx.get_neighbour_lists()
        np.testing.assert_array_equal(goff, off)
        np.testing.assert_array_equal(gids, ids)
        if h > 0:
            ctx.sph_density(h)
            _check_rho(ctx.get_density(), t.sph_density(h), kind)


@pytest.mark.parametrize("n_leaf,n_grp", [(1, 1), (16, 100), (8, 512)])
def test_neighbour_lists_leaf_and_group_sizes(n_leaf, n_grp):
    say("case neighbour lists n_leaf=%d n_grp=%d" % (n_leaf, n_grp))
    d = _system("plummer", 3000, seed=2)
    h = 0.1
    t = oracle.Tree(d["x"], d["y"], d["z"], d["m"], n_leaf, n_grp)
    off, ids = t.neighbour_lists(h)
    with _ctx(d, n_leaf, n_grp) as ctx:
        ctx.build_tree()
        ctx.neighbour_lists(h)
        goff, gids = ctx.get_neighbour_lists()
        np.testing.assert_array_equal(goff, off)
        np.testing.assert_array_equal(gids, ids)
        ctx.sph_density(h)
        _check_rho(ctx.get_density(), t.sph_density(h), "sizes")


def test_reuse_after_drift_within_the_skin():
    """Lists built with h (1 + s) before a drift of less than s h / 2 give
    the density of all pairs at the drifted positions."""
    say("case neighbour list reuse")
    d = _system("plummer", 8192, seed=5)
    h, s = 0.05, 0.3
    vmax = np.sqrt(d["vx"] ** 2 + d["vy"] ** 2 + d["vz"] ** 2).max()
    dt = 0.45 * s * h / vmax
    x1 = d["x"] + d["vx"] * dt
    y1 = d["y"] + d["vy"] * dt
    z1 = d["z"] + d["vz"] * dt
    t = oracle.Tree(d["x"], d["y"], d["z"], d["m"], 8, 64)
    t.neighbour_lists(h * (1 + s))
    t.refresh(x1, y1, z1, d["m"])
    want = t.sph_density(h)
    direct = oracle.sph_density_direct(x1, y1, z1, d["m"], h)
    np.testing.assert_allclose(want, direct, rtol=1e-12)
    with _ctx(d) as ctx:
        ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        ctx.neighbour_lists(h * (1 + s))
        ctx.kick_drift(0.0, dt)   # a pure drift, bit-exact with x + v dt
        ctx.sph_density(h)
        _check_rho(ctx.get_density(), want, "after drift")


def test_batched_systems_equal_systems_alone():
    say("case neighbour lists batched")
    d = workloads.clusters(5, 17, lo_exp=8, hi_exp=12)
    off = d["offsets"]
    h = 0.05
    with _ctx(d) as ctx:
        ctx.set_systems(off)
        ctx.build_tree()
        ctx.neighbour_lists(h)
        goff, gids = ctx.get_neighbour_lists()
        g = ctx.get_groups()
        ctx.sph_density(h)
        rho = ctx.get_density()
    first_group = 0
    for s in range(off.size - 1):
        b, e = int(off[s]), int(off[s + 1])
        sub = {k: d[k][b:e].copy() for k in ("x", "y", "z", "vx", "vy", "vz",
                                             "m")}
        with _ctx(sub) as one:
            one.build_tree()
            one.neighbour_lists(h)
            o1, i1 = one.get_neighbour_lists()
            one.sph_density(h)
            r1 = one.get_density()
        ng = o1.size - 1
        got_off = goff[first_group:first_group + ng + 1]
        np.testing.assert_array_equal(got_off - got_off[0], o1)
        np.testing.assert_array_equal(gids[got_off[0]:got_off[-1]], i1 + b)
        np.testing.assert_array_equal(rho[b:e], r1)
        assert g["begin"][first_group] == b
        first_group += ng
    assert first_group == goff.size - 1


def test_errors():
    d = _system("plummer", 500)
    with _ctx(d) as ctx:
        with pytest.raises(nb.NbError):
            ctx.neighbour_lists(0.1)        # no tree yet
        ctx.build_tree()
        with pytest.raises(nb.NbError):
            ctx.sph_density(0.1)            # no lists yet
        with pytest.raises(nb.NbError):
            ctx.neighbour_lists(-1.0)
        with pytest.raises(nb.NbError):
            ctx.neighbour_lists(float("nan"))
        ctx.neighbour_lists(0.1)
        with pytest.raises(nb.NbError):
            ctx.sph_density(0.2)            # beyond the lists' radius
        with pytest.raises(nb.NbError):
            ctx.sph_density(0.0)
        with pytest.raises(nb.NbError):
            ctx.get_density()               # nothing computed
        ctx.sph_density(0.1)
        ctx.build_tree()                    # a new tree drops the lists
        with pytest.raises(nb.NbError):
            ctx.sph_density(0.1)


@pytest.mark.parametrize("name", ["sphere_4m", "disk_4m"])
def test_full_size_sampled(name):
    """N = 2^22 (the cold sphere, leaf 16, n_grp 64; the disk, leaf 8,
    n_grp 256) with h for about 64 neighbours in a unit ball: lists of
    sampled groups and every density."""
    say("case neighbour lists full size %s" % name)
    d, p = workloads.make(name)
    n = d["x"].size
    h = (64 / n) ** (1 / 3)   # unit ball of n particles: 64 within h
    t = oracle.Tree(d["x"], d["y"], d["z"], d["m"], p["n_leaf"], p["n_grp"])
    off, ids = t.neighbour_lists(h)
    rho_o = t.sph_density(h)
    with _ctx(d, p["n_leaf"], p["n_grp"]) as ctx:
        ctx.build_tree()
        ctx.neighbour_lists(h)
        goff, gids = ctx.get_neighbour_lists()
        ctx.sph_density(h)
        rho = ctx.get_density()
    np.testing.assert_array_equal(goff, off)
    rng = np.random.default_rng(3)
    for g in rng.choice(off.size - 1, 256, replace=False):
        np.testing.assert_array_equal(gids[goff[g]:goff[g + 1]],
                                      ids[off[g]:off[g + 1]])
    _check_rho(rho, rho_o, name)
