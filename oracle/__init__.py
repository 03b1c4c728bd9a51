"""FP64 CPU oracle of the Barnes-Hut step of "Accelerated FDPS".

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
product (``paper_1907_02290_amd``) never imports it and it never imports the
product.  The arithmetic lives in ``orc.c`` (plain C, FP64, no FMA
contraction); this module only marshals numpy arrays through ctypes.

Stage map (paper sections):
  root / keys ...... section 4.3, local tree step 1 (root cell, Morton keys)
  Tree(...) ........ section 4.3, steps 2-4 (stable sort, reorder, link),
                     the moment pass, and the particle groups of section 2
  make_lists ....... section 4.3 list construction, indices per section 4.1
  refresh .......... section 4.2 reuse step (moments over frozen ranges)
  force_lists ...... the kernel's sum over EPJ and SPJ of each list
  force_direct ..... direct summation (what the tree approximates)
  kick_drift ....... orbit integration (KDK leapfrog)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_SRC_MLP = os.path.join(_HERE, "mlp.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def build_lib(force: bool = True) -> str:
    """Compile ``orc.c`` into ``liborc.so`` with gcc (FP64, no contraction)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-Wno-unused-parameter", _SRC, _SRC_MLP, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_lib()
    lib = C.CDLL(_LIB)
    p = C.c_void_p
    i64 = C.c_int64
    d = C.c_double
    lib.orc_root.argtypes = [i64, p, p, p, p, p]
    lib.orc_keys.argtypes = [i64, p, p, p, p, C.c_int, p]
    lib.orc_interleave.argtypes = [C.c_uint32] * 3
    lib.orc_interleave.restype = C.c_uint64
    lib.orc_deinterleave.argtypes = [C.c_uint64, C.c_int, p]
    lib.orc_deinterleave.restype = None
    lib.orc_build.argtypes = [i64, p, p, p, p, C.c_int, C.c_int]
    lib.orc_build.restype = p
    lib.orc_free.argtypes = [p]
    lib.orc_free.restype = None
    lib.orc_info.argtypes = [p, p, p]
    lib.orc_get_keys.argtypes = [p, p, p]
    lib.orc_get_cells.argtypes = [p] + [p] * 8
    lib.orc_get_moments.argtypes = [p, p, p, p]
    lib.orc_get_groups.argtypes = [p] + [p] * 6
    lib.orc_make_lists.argtypes = [p, d, i64, p, p]
    lib.orc_get_lists.argtypes = [p, p, p, p, p]
    lib.orc_refresh.argtypes = [p, p, p, p, p]
    lib.orc_force_lists.argtypes = [p, C.c_int, d, d, p, p, p, p]
    lib.orc_force_direct.argtypes = [i64, p, p, p, p, d, d, i64, p, p, p, p, p]
    lib.orc_kick_drift.argtypes = [i64, p, p, p, p, p, p, p, p, p, d, d, d, d]
    lib.orc_num_threads.argtypes = []
    lib.orc_group_margins.argtypes = [p, p, p]
    lib.orc_group_stale.argtypes = [p, d, d, p, p, p]
    lib.orc_refresh_lists.argtypes = [p, d, i64, p, p]
    lib.orc_cell_sides.argtypes = [p, p]
    lib.orc_group_features.argtypes = [p, C.c_int, p, p]
    lib.orc_mlp_nparam.argtypes = []
    lib.orc_mlp_forward.argtypes = [p, i64, p, p]
    lib.orc_mlp_loss_grad.argtypes = [p, i64, p, p, d, p, p]
    lib.orc_adam.argtypes = [p, p, p, p, i64, d, d, d, d]
    lib.orc_neighbour_lists.argtypes = [p, d, p]
    lib.orc_get_neighbour_lists.argtypes = [p, p, p]
    lib.orc_sph_w.argtypes = [d, d]
    lib.orc_sph_w.restype = d
    lib.orc_sph_density.argtypes = [p, d, p]
    lib.orc_sph_density_direct.argtypes = [i64, p, p, p, p, d, p]
    for f in ("orc_root", "orc_keys", "orc_info", "orc_get_keys",
              "orc_get_cells", "orc_get_moments", "orc_get_groups",
              "orc_make_lists", "orc_get_lists", "orc_refresh",
              "orc_force_lists", "orc_force_direct", "orc_kick_drift",
              "orc_num_threads", "orc_group_margins", "orc_group_stale",
              "orc_refresh_lists", "orc_group_features", "orc_cell_sides",
              "orc_mlp_nparam", "orc_mlp_forward", "orc_mlp_loss_grad",
              "orc_adam", "orc_neighbour_lists", "orc_get_neighbour_lists",
              "orc_sph_density", "orc_sph_density_direct"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("oracle %s failed (rc=%d)" % (what, rc))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def root(x, y, z):
    """Root corner ``lo`` and exponent ``k`` (side ``L = 2**k``)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    lo = np.zeros(3)
    k = C.c_int(0)
    _check(_load().orc_root(x.size, _ptr(x), _ptr(y), _ptr(z), _ptr(lo),
                            C.byref(k)), "root")
    return lo, int(k.value)


def keys(x, y, z, lo, k):
    x, y, z = _f64(x), _f64(y), _f64(z)
    lo = _f64(lo)
    out = np.zeros(x.size, dtype=np.uint64)
    _check(_load().orc_keys(x.size, _ptr(x), _ptr(y), _ptr(z), _ptr(lo),
                            int(k), _ptr(out)), "keys")
    return out


def interleave(qx, qy, qz) -> int:
    return int(_load().orc_interleave(int(qx), int(qy), int(qz)))


def deinterleave(key, level):
    q = np.zeros(3, dtype=np.uint32)
    _load().orc_deinterleave(int(key), int(level), _ptr(q))
    return tuple(int(v) for v in q)


class Tree:
    """One construction step of the oracle: root, keys, sort, reorder,
    link, moments and groups over FP64 particle arrays (input order)."""

    def __init__(self, x, y, z, m, n_leaf=8, n_grp=64):
        lib = _load()
        self._x, self._y, self._z, self._m = (_f64(x), _f64(y), _f64(z),
                                              _f64(m))
        n = self._x.size
        self._h = lib.orc_build(n, _ptr(self._x), _ptr(self._y),
                                _ptr(self._z), _ptr(self._m), int(n_leaf),
                                int(n_grp))
        if not self._h:
            raise RuntimeError("oracle build failed")
        info = np.zeros(6, dtype=np.int64)
        lo = np.zeros(3)
        lib.orc_info(self._h, _ptr(info), _ptr(lo))
        self.n, self.n_cell, self.n_groups, self.k = (int(v) for v in info[:4])
        self.n_leaf, self.n_grp = int(info[4]), int(info[5])
        self.lo = lo
        self._sel = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().orc_free(h)
            self._h = None

    def keys(self):
        key = np.zeros(self.n, dtype=np.uint64)
        perm = np.zeros(self.n, dtype=np.uint32)
        _check(_load().orc_get_keys(self._h, _ptr(key), _ptr(perm)), "keys")
        return key, perm

    def cells(self):
        nc = self.n_cell
        out = dict(prefix=np.zeros(nc, np.uint64), level=np.zeros(nc, np.uint8),
                   begin=np.zeros(nc, np.uint32), count=np.zeros(nc, np.uint32),
                   parent=np.zeros(nc, np.uint32), skip=np.zeros(nc, np.uint32),
                   leaf=np.zeros(nc, np.uint8), ctr=np.zeros((nc, 3)))
        _check(_load().orc_get_cells(self._h, *(_ptr(out[k]) for k in (
            "prefix", "level", "begin", "count", "parent", "skip", "leaf",
            "ctr"))), "cells")
        return out

    def moments(self):
        nc = self.n_cell
        mass, com, quad = np.zeros(nc), np.zeros((nc, 3)), np.zeros((nc, 6))
        _check(_load().orc_get_moments(self._h, _ptr(mass), _ptr(com),
                                       _ptr(quad)), "moments")
        return mass, com, quad

    def groups(self):
        ng = self.n_groups
        out = dict(cell=np.zeros(ng, np.uint32), begin=np.zeros(ng, np.uint32),
                   count=np.zeros(ng, np.uint32), lo=np.zeros((ng, 3)),
                   hi=np.zeros((ng, 3)), ctr=np.zeros((ng, 3)))
        _check(_load().orc_get_groups(self._h, *(_ptr(out[k]) for k in (
            "cell", "begin", "count", "lo", "hi", "ctr"))), "groups")
        return out

    def make_lists(self, theta, sel=None):
        """Walk the selected groups (all when ``sel`` is None)."""
        sizes = np.zeros(3, dtype=np.int64)
        if sel is None:
            rc = _load().orc_make_lists(self._h, float(theta), 0, None,
                                        _ptr(sizes))
        else:
            s = np.ascontiguousarray(sel, dtype=np.int64)
            rc = _load().orc_make_lists(self._h, float(theta), s.size,
                                        _ptr(s), _ptr(sizes))
        _check(rc, "make_lists")
        self._sizes = sizes.copy()
        return int(sizes[0]), int(sizes[1]), int(sizes[2])

    def lists(self):
        ns, ne, nsp = (int(v) for v in self._sizes)
        eo = np.zeros(ns + 1, np.int64)
        so = np.zeros(ns + 1, np.int64)
        e = np.zeros(ne, np.uint32)
        s = np.zeros(nsp, np.uint32)
        _check(_load().orc_get_lists(self._h, _ptr(eo), _ptr(e), _ptr(so),
                                     _ptr(s)), "lists")
        return eo, e, so, s

    def refresh(self, x, y, z, m):
        """Reuse step: new positions (input order), frozen topology."""
        self._x, self._y, self._z, self._m = (_f64(x), _f64(y), _f64(z),
                                              _f64(m))
        _check(_load().orc_refresh(self._h, _ptr(self._x), _ptr(self._y),
                                   _ptr(self._z), _ptr(self._m)), "refresh")

    def margins(self):
        """Opening-test slacks (sa, so) of the walk that made each group's
        list, in length units (+inf where no cell of that kind)."""
        sa = np.zeros(self.n_groups)
        so = np.zeros(self.n_groups)
        _check(_load().orc_group_margins(self._h, _ptr(sa), _ptr(so)),
               "margins")
        return sa, so

    def stale(self, theta, tau=0.0):
        """Groups with a kept superparticle that fails the opening test at
        angle theta (1 + tau) from the current box; also the boxes."""
        st = np.zeros(self.n_groups, np.uint8)
        lo = np.zeros((self.n_groups, 3))
        hi = np.zeros((self.n_groups, 3))
        _check(_load().orc_group_stale(self._h, float(theta), float(tau),
                                       _ptr(st), _ptr(lo), _ptr(hi)), "stale")
        return st.astype(bool), lo, hi

    def refresh_lists(self, theta, sel):
        """Walk the listed groups again with their current boxes."""
        sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
        sizes = np.zeros(3, np.int64)
        _check(_load().orc_refresh_lists(self._h, float(theta), sel.size,
                                         _ptr(sel), _ptr(sizes)),
               "refresh_lists")
        self._sizes = sizes.copy()
        return int(sizes[0]), int(sizes[1]), int(sizes[2])

    def cell_sides(self):
        """Side of every cell in the opening test at the current positions
        (the geometric side unless the cell's particles spread further)."""
        out = np.zeros(self.n_cell)
        _check(_load().orc_cell_sides(self._h, _ptr(out)), "cell_sides")
        return out

    def features(self, kmax, age):
        """The 12 rebuild-predictor inputs per group (FP64, [G, 12])."""
        age = np.ascontiguousarray(np.asarray(age, dtype=np.int32))
        assert age.shape == (self.n_groups,)
        f = np.zeros((self.n_groups, 12))
        _check(_load().orc_group_features(self._h, int(kmax), _ptr(age),
                                          _ptr(f)), "features")
        return f

    def neighbour_lists(self, h):
        """Neighbour lists of every group for search radius h (short-range
        walk, section 2); returns (offsets, sorted-order ids)."""
        n = np.zeros(1, np.int64)
        _check(_load().orc_neighbour_lists(self._h, float(h), _ptr(n)),
               "neighbour_lists")
        off = np.zeros(self.n_groups + 1, np.int64)
        ids = np.zeros(int(n[0]), np.uint32)
        _check(_load().orc_get_neighbour_lists(self._h, _ptr(off), _ptr(ids)),
               "get_neighbour_lists")
        return off, ids

    def sph_density(self, h):
        """FP64 SPH density over the neighbour lists, input order."""
        rho = np.zeros(self.n)
        _check(_load().orc_sph_density(self._h, float(h), _ptr(rho)),
               "sph_density")
        return rho

    def force_lists(self, order=1, eps=0.0, G=1.0):
        """FP64 sum over the saved lists; NaN for particles of groups that
        were not walked.  Input order."""
        out = [np.full(self.n, np.nan) for _ in range(4)]
        _check(_load().orc_force_lists(self._h, int(order), float(eps),
                                       float(G), *(_ptr(a) for a in out)),
               "force_lists")
        return tuple(out)


def mlp_nparam() -> int:
    return int(_load().orc_mlp_nparam())


def mlp_forward(w, x):
    w = _f64(w)
    x = _f64(x).reshape(-1, 12)
    p = np.zeros(x.shape[0])
    _check(_load().orc_mlp_forward(_ptr(w), x.shape[0], _ptr(x), _ptr(p)),
           "mlp_forward")
    return p


def mlp_loss_grad(w, x, y, pos_weight=1.0):
    w = _f64(w)
    x = _f64(x).reshape(-1, 12)
    y = _f64(y)
    loss = np.zeros(1)
    g = np.zeros(mlp_nparam())
    _check(_load().orc_mlp_loss_grad(_ptr(w), x.shape[0], _ptr(x), _ptr(y),
                                     float(pos_weight), _ptr(loss), _ptr(g)),
           "mlp_loss_grad")
    return float(loss[0]), g


def adam(w, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place on w, m, v (FP64 arrays)."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    _check(_load().orc_adam(_ptr(w), _ptr(g), _ptr(m), _ptr(v), int(t),
                            float(lr), float(beta1), float(beta2), float(eps)),
           "adam")


def force_direct(x, y, z, m, eps=0.0, G=1.0, targets=None):
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    n = x.size
    tgt = np.arange(n, dtype=np.int64) if targets is None else \
        np.ascontiguousarray(targets, dtype=np.int64)
    out = [np.zeros(tgt.size) for _ in range(4)]
    _check(_load().orc_force_direct(n, _ptr(x), _ptr(y), _ptr(z), _ptr(m),
                                    float(eps), float(G), tgt.size, _ptr(tgt),
                                    *(_ptr(a) for a in out)), "force_direct")
    return tuple(out)


def sph_w(r, h):
    """The SPH kernel W(r, h) (cubic spline of compact support h)."""
    return float(_load().orc_sph_w(float(r), float(h)))


def sph_density_direct(x, y, z, m, h):
    """SPH density over all pairs, FP64."""
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    rho = np.zeros(x.size)
    _check(_load().orc_sph_density_direct(x.size, _ptr(x), _ptr(y), _ptr(z),
                                          _ptr(m), float(h), _ptr(rho)),
           "sph_density_direct")
    return rho


def kick_drift(pos, vel, acc, dt_kick, dt_drift, ext_mass=0.0, G=1.0):
    """In place on ``pos`` and ``vel`` (lists of three FP64 arrays)."""
    for a in list(pos) + list(vel):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    acc = [_f64(a) for a in acc]
    n = pos[0].size
    _check(_load().orc_kick_drift(n, *(_ptr(a) for a in pos),
                                  *(_ptr(a) for a in vel),
                                  *(_ptr(a) for a in acc), float(dt_kick),
                                  float(dt_drift), float(ext_mass), float(G)),
           "kick_drift")
