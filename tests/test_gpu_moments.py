"""The two-launch moment pass (subtree blocks in LDS, then the cells above
them through a child table) against the one-launch-per-level pass: the same
moments bit for bit, and so the same forces, at construction and at reuse
steps; and both within the FP32 tolerance of the FP64 oracle.

The two passes run in two contexts that are alive at the same time, so that
neither reads memory the other wrote."""
import numpy as np
import pytest

import oracle
import workloads
import paper_1907_02290_amd as nb
from test_gpu_parity import system

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _pair(d, order, n_leaf, n_grp=64, offsets=None):
    ctxs = []
    for level in (False, True):
        ctx = nb.Context(theta=0.5, eps=1 / 64, n_leaf=n_leaf, n_grp=n_grp,
                         order=order, level_moments=level)
        ctx.set_particles(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"],
                          d["m"])
        if offsets is not None:
            ctx.set_systems(offsets)
        ctxs.append(ctx)
    return ctxs


def _same_moments(a, b):
    for u, v, what in zip(a.get_moments(), b.get_moments(),
                          ("mass", "com", "quad")):
        np.testing.assert_array_equal(u, v, err_msg=what)


def _same_forces(a, b):
    for u, v in zip(a.get_forces(), b.get_forces()):
        np.testing.assert_array_equal(u, v)


CASES = [("plummer", 1), ("plummer", 2), ("plummer", 9), ("plummer", 1000),
         ("plummer", 65537), ("clustered", 3000), ("disk", 20000),
         ("ring", 12345), ("sphere", 5000)]


@pytest.mark.parametrize("kind,n", CASES)
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("n_leaf", [1, 8, 64])
def test_two_launch_moments_equal_level_launches(kind, n, order, n_leaf):
    say("case moments two-launch vs levels %s n=%d order=%d n_leaf=%d"
        % (kind, n, order, n_leaf))
    d = system(kind, n)
    a, b = _pair(d, order, n_leaf)
    try:
        for ctx in (a, b):
            ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        _same_moments(a, b)
        _same_forces(a, b)
        # a reuse step: the moments over the frozen tree at moved positions
        for ctx in (a, b):
            ctx.kick_drift(1 / 256, 1 / 128)
            ctx.compute_forces(nb.NB_REUSE_LIST)
        _same_moments(a, b)
        _same_forces(a, b)
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("order", [1, 2])
def test_two_launch_moments_batched_systems(order):
    """Systems from 2^6 to 2^15 particles: some are single blocks, others
    have cells above the blocks; every system root is level 0."""
    say("case moments two-launch vs levels, batch order=%d" % order)
    d = workloads.clusters(9, 5, lo_exp=6, hi_exp=15)
    a, b = _pair(d, order, 8, offsets=d["offsets"])
    try:
        for ctx in (a, b):
            ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        _same_moments(a, b)
        _same_forces(a, b)
    finally:
        a.close()
        b.close()


def test_two_launch_moments_full_size_disk():
    """disk_4m (2^22 particles, 1.8 million cells): blocks and cells above
    them over ten levels."""
    say("case moments two-launch vs levels, disk_4m")
    d, p = workloads.make("disk_4m")
    a, b = _pair(d, 1, p["n_leaf"], n_grp=p["n_grp"])
    try:
        for ctx in (a, b):
            ctx.build_tree()
        _same_moments(a, b)
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("order", [1, 2])
def test_two_launch_moments_match_oracle(order):
    """65537 Plummer particles (cells above the blocks at several levels):
    the two-launch moments within the FP32 tolerance of the oracle's."""
    say("case moments two-launch vs oracle order=%d" % order)
    d = system("plummer", 65537, seed=3)
    with nb.Context(theta=0.5, eps=1 / 64, n_leaf=8, n_grp=64,
                    order=order) as ctx:
        ctx.set_particles(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"],
                          d["m"])
        ctx.build_tree()
        M, X, S = ctx.get_moments()
    t = oracle.Tree(d["x"], d["y"], d["z"], d["m"], 8, 64)
    oM, oX, oS = t.moments()
    lev = t.cells()["level"].astype(np.int64)
    side = 2.0 ** (t.k - lev)
    np.testing.assert_allclose(M, oM, rtol=1e-6)
    assert np.all(np.abs(X - oX).max(1) <= 1e-5 * side)
    if order == 2:
        scale = (oM * side ** 2)[:, None]
        assert np.all(np.abs(S - oS) <= 1e-5 * scale + 1e-30)


@pytest.mark.parametrize("kind,n,n_leaf,order", [
    # 1447 cells above the blocks (one-particle leaves): more than one per
    # thread of the top launch, which keeps them in LDS
    ("plummer", 1 << 21, 1, 1),
    # more than 2048: the top launch works from global memory
    ("plummer", 1 << 22, 1, 1),
    # more than 1024 with quadrupoles: the same
    ("ring", 1 << 22, 8, 2)])
def test_two_launch_moments_many_top_cells(kind, n, n_leaf, order):
    say("case moments two-launch vs levels, many top cells %s n=%d" % (kind, n))
    d = system(kind, n)
    a, b = _pair(d, order, n_leaf)
    try:
        for ctx in (a, b):
            ctx.build_tree()
        _same_moments(a, b)
    finally:
        a.close()
        b.close()
