"""Pins of the oracle's root cell, Morton keys and key sort (section 4.3,
local tree steps 1-2) against closed forms and a library sort."""
import numpy as np
import pytest


def test_root_power_of_two_strictly_above_extent(orc):
    # extent 1.0 -> L = 2 (strictly larger), 0.75 -> 1, 3 -> 4, 0.3 -> 0.5
    for ext, k in [(1.0, 1), (0.75, 0), (3.0, 2), (0.3, -1), (1e-3, -9)]:
        x = np.array([5.0, 5.0 + ext])
        lo, kk = orc.root(x, np.zeros(2), np.zeros(2))
        assert kk == k, (ext, kk)
        assert lo[0] == 5.0
        assert 2.0 ** kk > ext >= 2.0 ** (kk - 1)


def test_root_degenerate_single_point(orc):
    lo, k = orc.root(np.array([2.0]), np.array([3.0]), np.array([-1.0]))
    assert k == 0 and list(lo) == [2.0, 3.0, -1.0]


def test_root_uses_largest_axis(orc):
    x = np.array([0.0, 0.1])
    y = np.array([-2.0, 1.5])
    z = np.array([0.0, 0.0])
    lo, k = orc.root(x, y, z)
    assert k == 2 and list(lo) == [0.0, -2.0, 0.0]


def test_key_corner_is_zero(orc):
    lo = np.array([-1.0, -1.0, -1.0])
    key = orc.keys(np.array([-1.0]), np.array([-1.0]), np.array([-1.0]), lo, 1)
    assert int(key[0]) == 0


def test_key_far_corner_is_all_ones(orc):
    # extent just below L: every axis quantises to 2^21 - 1
    e = 1.0 - 2.0 ** -22
    key = orc.keys(np.array([e]), np.array([e]), np.array([e]),
                   np.zeros(3), 0)
    assert int(key[0]) == (1 << 63) - 1


def test_key_cube_centre(orc):
    # centre of the root cube: q = 2^20 on every axis -> top digit 0b111
    key = orc.keys(np.array([0.5]), np.array([0.5]), np.array([0.5]),
                   np.zeros(3), 0)
    assert int(key[0]) == 7 << 60


def test_key_digit_order_x_most_significant(orc):
    assert orc.interleave(1, 0, 0) == 4
    assert orc.interleave(0, 1, 0) == 2
    assert orc.interleave(0, 0, 1) == 1
    # a point in the upper-x half only: first digit 0b100
    key = orc.keys(np.array([0.5]), np.array([0.25]), np.array([0.0]),
                   np.zeros(3), 0)
    assert int(key[0]) >> 60 == 0b100
    assert (int(key[0]) >> 57) & 7 == 0b010  # y = 0.25 -> second digit has y


def test_key_quantisation_floor(orc):
    # q = floor((x - lo) * 2^(21-k)); just below a cell boundary stays below
    h = 2.0 ** -21
    xs = np.array([3 * h, 3 * h - 2.0 ** -60, 3.5 * h])
    key = orc.keys(xs, np.zeros(3), np.zeros(3), np.zeros(3), 0)
    qx = [orc.deinterleave(int(k), 21)[0] for k in key]
    assert qx == [3, 2, 3]


def test_interleave_roundtrip(orc):
    rng = np.random.default_rng(5)
    for _ in range(200):
        q = rng.integers(0, 1 << 21, 3)
        key = orc.interleave(*q)
        assert key < (1 << 63)
        assert orc.deinterleave(key, 21) == tuple(int(v) for v in q)
        # a coarser level keeps the top bits of each coordinate
        for lev in (0, 1, 7, 20):
            assert orc.deinterleave(key, lev) == tuple(
                int(v) >> (21 - lev) for v in q)


def test_sorted_keys_match_stable_library_sort(orc):
    rng = np.random.default_rng(7)
    n = 3000
    # many duplicates: positions on a coarse lattice
    x, y, z = (rng.integers(0, 4, (3, n)) * 0.25).astype(np.float64)
    m = np.ones(n)
    t = orc.Tree(x, y, z, m, n_leaf=8, n_grp=64)
    key, perm = t.keys()
    raw = orc.keys(x, y, z, t.lo, t.k)
    ref = np.argsort(raw, kind="stable")
    np.testing.assert_array_equal(perm, ref)
    np.testing.assert_array_equal(key, raw[ref])
    assert np.all(np.diff(key.astype(np.uint64)) >= 0)


def test_quantised_point_inside_its_key_cell(orc):
    rng = np.random.default_rng(11)
    x, y, z = rng.standard_normal((3, 500))
    lo, k = orc.root(x, y, z)
    key = orc.keys(x, y, z, lo, k)
    h = 2.0 ** (k - 21)
    for i in range(500):
        q = orc.deinterleave(int(key[i]), 21)
        for a, p in enumerate((x, y, z)):
            assert lo[a] + q[a] * h <= p[i] < lo[a] + (q[a] + 1) * h + 1e-12
