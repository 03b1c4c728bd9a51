"""ctypes binding of ``libnbody_hip.so`` (declared in ``include/nbody.h``).

Argument marshalling only: every stage of the step runs in the library's
HIP kernels.  There is no CPU fallback -- if the library is missing the
import of a context raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbody_hip.so")

NB_OK = 0
NB_ERR_INPUT = -1
NB_ERR_OOM = -2
NB_ERR_LIST = -3
NB_ERR_STATE = -4
NB_ERR_HIP = -5

NB_MAKE_LIST = 0
NB_MAKE_LIST_FOR_REUSE = 1
NB_REUSE_LIST = 2
NB_REUSE_REFRESH = 3
NB_REUSE_CHECK = 4

PHASES = ("root", "keys", "sort", "reorder", "link", "moments", "groups",
          "walk", "force", "kick", "graph", "refresh")
NB_FLAG_TIMING = 1
NB_FLAG_GRAPH = 2
NB_FLAG_REFRESH = 4
NB_FLAG_PERSISTENT = 8
NB_FLAG_COPIED_LISTS = 16
NB_FLAG_LEVEL_MOMENTS = 32
MLP_NIN = 12
MLP_NPARAM = 5057
MLP_STATIC_MAX_ROWS = 8192

STATUS = {NB_OK: "NB_OK", NB_ERR_INPUT: "NB_ERR_INPUT",
          NB_ERR_OOM: "NB_ERR_OOM", NB_ERR_LIST: "NB_ERR_LIST",
          NB_ERR_STATE: "NB_ERR_STATE", NB_ERR_HIP: "NB_ERR_HIP"}


class NbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class nb_config(C.Structure):
    _fields_ = [("theta", C.c_double), ("eps", C.c_double), ("G", C.c_double),
                ("ext_mass", C.c_double), ("n_leaf", C.c_int32),
                ("n_grp", C.c_int32), ("order", C.c_int32),
                ("flags", C.c_int32), ("k_max", C.c_int32),
                ("p_star", C.c_double), ("tau", C.c_double),
                ("tile_j", C.c_int32), ("waves_per_simd", C.c_int32),
                ("stream", C.c_void_p)]


_lib = None


def load():
    """Load the library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "libnbody_hip.so is not built (%s); run __graft_entry__.build()"
            % LIB_PATH)
    # PyTorch ships its own HIP runtime under the same soname as the one the
    # library links.  Loading torch first makes the dynamic linker bind the
    # library to torch's runtime, so the process holds a single HIP runtime
    # and torch's streams and device pointers are valid in the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    p, i64, i32, d = C.c_void_p, C.c_int64, C.c_int, C.c_double
    sig = {
        "nb_create": ([p, p], i32),
        "nb_destroy": ([p], None),
        "nb_set_config": ([p, p], i32),
        "nb_set_particles": ([p, i64] + [p] * 7 + [i32], i32),
        "nb_build_tree": ([p], i32),
        "nb_make_lists": ([p, i32], i32),
        "nb_compute_forces": ([p, i32], i32),
        "nb_kick_drift": ([p, d, d], i32),
        "nb_step": ([p, i32, d, d], i32),
        "nb_get_forces": ([p, p, p, p, p, i32], i32),
        "nb_get_state": ([p] + [p] * 6 + [i32], i32),
        "nb_get_info": ([p, p], i32),
        "nb_get_root": ([p, p, p], i32),
        "nb_get_roots": ([p, p, p], i32),
        "nb_set_systems": ([p, i64, p], i32),
        "nb_neighbour_lists": ([p, d], i32),
        "nb_sph_density": ([p, d], i32),
        "nb_get_density": ([p, p, i32], i32),
        "nb_get_neighbour_lists": ([p, p, p, p], i32),
        "nb_get_keys": ([p, p, p], i32),
        "nb_get_cells": ([p] + [p] * 7, i32),
        "nb_get_moments": ([p, p, p, p], i32),
        "nb_get_groups": ([p] + [p] * 6, i32),
        "nb_get_lists": ([p, p, p, p, p], i32),
        "nb_upload_lists": ([p, i64, p, i64, p, p, i64, p, i32], i32),
        "nb_get_timing": ([p, p, p, i32], i32),
        "nb_group_features": ([p, p, i32], i32),
        "nb_group_stale": ([p, d, p, p, i32], i32),
        "nb_refresh_lists": ([p, i64, p], i32),
        "nb_get_group_state": ([p, p, p, p], i32),
        "nb_get_cell_sides": ([p, p], i32),
        "nb_mlp_set": ([p, p, i64], i32),
        "nb_mlp_get": ([p, p, i64], i32),
        "nb_mlp_forward": ([p, i64, p, p, i32], i32),
        "nb_mlp_grad": ([p, i64, p, p, C.c_float, p, p, i32], i32),
        "nb_mlp_grad_static": ([p, i64, p, p, C.c_float, p, p], i32),
        "nb_mlp_adam": ([p, p, C.c_float, C.c_float, C.c_float, C.c_float,
                         i32], i32),
        "nb_mlp_train": ([p, i64, p, p, i32, i32, i64, C.c_float, C.c_float,
                          p], i32),
        "nb_last_error": ([p], C.c_char_p),
        "nb_version": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def version() -> str:
    return load().nb_version().decode()


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _is_torch(a):
    return type(a).__module__.startswith("torch")


class Context:
    """One GPU-resident particle system (``nb_ctx``)."""

    def __init__(self, theta=0.5, eps=0.01, G=1.0, n_leaf=8, n_grp=64,
                 order=1, ext_mass=0.0, timing=False, graph=False,
                 refresh=False, k_max=8, p_star=0.5, tau=0.0,
                 persistent=False, copied_lists=False, tile_j=0,
                 waves_per_simd=0, stream=None, level_moments=False):
        self._lib = load()
        flags = (NB_FLAG_TIMING if timing else 0) | \
            (NB_FLAG_GRAPH if graph else 0) | \
            (NB_FLAG_REFRESH if refresh else 0) | \
            (NB_FLAG_PERSISTENT if persistent else 0) | \
            (NB_FLAG_COPIED_LISTS if copied_lists else 0) | \
            (NB_FLAG_LEVEL_MOMENTS if level_moments else 0)
        self._cfg = nb_config(theta, eps, G, ext_mass, n_leaf, n_grp, order,
                              flags, k_max, p_star, tau, tile_j,
                              waves_per_simd, stream)
        h = C.c_void_p()
        rc = self._lib.nb_create(C.byref(self._cfg), C.byref(h))
        if rc != NB_OK:
            raise NbError(rc, "nb_create failed")
        self._h = h
        self.n = 0
        self.n_sys = 1

    def close(self):
        if getattr(self, "_h", None):
            self._lib.nb_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, rc):
        if rc != NB_OK:
            raise NbError(rc, self.last_error())
        return rc

    def last_error(self) -> str:
        return self._lib.nb_last_error(self._h).decode()

    @property
    def config(self):
        c = self._cfg
        return dict(theta=c.theta, eps=c.eps, G=c.G, ext_mass=c.ext_mass,
                    n_leaf=c.n_leaf, n_grp=c.n_grp, order=c.order,
                    k_max=c.k_max, p_star=c.p_star, tau=c.tau,
                    tile_j=c.tile_j, waves_per_simd=c.waves_per_simd,
                    refresh=bool(c.flags & NB_FLAG_REFRESH))

    def set_config(self, **kw):
        for k, v in kw.items():
            if k == "timing":
                self._cfg.flags = (self._cfg.flags & ~NB_FLAG_TIMING) | \
                    (NB_FLAG_TIMING if v else 0)
            elif k == "graph":
                self._cfg.flags = (self._cfg.flags & ~NB_FLAG_GRAPH) | \
                    (NB_FLAG_GRAPH if v else 0)
            elif k == "refresh":
                self._cfg.flags = (self._cfg.flags & ~NB_FLAG_REFRESH) | \
                    (NB_FLAG_REFRESH if v else 0)
            elif k == "persistent":
                self._cfg.flags = (self._cfg.flags & ~NB_FLAG_PERSISTENT) | \
                    (NB_FLAG_PERSISTENT if v else 0)
            elif k == "copied_lists":
                self._cfg.flags = (self._cfg.flags & ~NB_FLAG_COPIED_LISTS) | \
                    (NB_FLAG_COPIED_LISTS if v else 0)
            elif k == "level_moments":
                self._cfg.flags = (self._cfg.flags & ~NB_FLAG_LEVEL_MOMENTS) | \
                    (NB_FLAG_LEVEL_MOMENTS if v else 0)
            else:
                setattr(self._cfg, k, v)
        self._chk(self._lib.nb_set_config(self._h, C.byref(self._cfg)))

    # ---- particles ----
    def set_particles(self, x, y, z, vx, vy, vz, m):
        arrs = [x, y, z, vx, vy, vz, m]
        if _is_torch(x) and x.is_cuda:
            import torch
            arrs = [a.to(torch.float64).contiguous() for a in arrs]
            self._keep = arrs  # alive until the copy has completed
            ptrs = [C.c_void_p(a.data_ptr()) for a in arrs]
            n = arrs[0].numel()
            rc = self._lib.nb_set_particles(self._h, n, *ptrs, 1)
            self._keep = None
        else:
            arrs = [np.ascontiguousarray(np.asarray(a), dtype=np.float64)
                    for a in arrs]
            n = arrs[0].size
            if any(a.size != n for a in arrs):
                raise ValueError("particle arrays differ in length")
            rc = self._lib.nb_set_particles(self._h, n,
                                            *(_ptr(a) for a in arrs), 0)
        self._chk(rc)
        self.n = n
        self.n_sys = 1

    def set_systems(self, offsets):
        """Independent systems: particles [off[s], off[s+1]) form system s."""
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        self._chk(self._lib.nb_set_systems(self._h, off.size - 1, _ptr(off)))
        self.n_sys = off.size - 1

    # ---- the step ----
    def build_tree(self):
        self._chk(self._lib.nb_build_tree(self._h))

    def make_lists(self, mode=NB_MAKE_LIST_FOR_REUSE):
        self._chk(self._lib.nb_make_lists(self._h, int(mode)))

    def compute_forces(self, mode=NB_MAKE_LIST):
        self._chk(self._lib.nb_compute_forces(self._h, int(mode)))

    def step(self, mode, dt_kick, dt_drift):
        """Kick-drift then forces; reuse steps may replay a HIP graph."""
        self._chk(self._lib.nb_step(self._h, int(mode), float(dt_kick),
                                    float(dt_drift)))

    def kick_drift(self, dt_kick, dt_drift):
        self._chk(self._lib.nb_kick_drift(self._h, float(dt_kick),
                                          float(dt_drift)))

    # ---- readback ----
    def get_forces(self, internal=False):
        out = [np.empty(self.n) for _ in range(4)]
        self._chk(self._lib.nb_get_forces(self._h, *(_ptr(a) for a in out),
                                          1 if internal else 0))
        return tuple(out)

    def get_state(self, internal=False):
        out = [np.empty(self.n) for _ in range(6)]
        self._chk(self._lib.nb_get_state(self._h, *(_ptr(a) for a in out),
                                         1 if internal else 0))
        return tuple(out)

    def get_info(self):
        a = np.zeros(17, dtype=np.int64)
        self._chk(self._lib.nb_get_info(self._h, _ptr(a)))
        keys = ("n", "n_cell", "n_groups", "n_epj", "n_spj", "n_inter",
                "force_evals", "total_inter", "k", "n_wi", "n_sys",
                "last_refreshed", "total_refreshed", "n_inter_spj",
                "total_inter_spj", "last_overflow", "total_overflow")
        return {k: int(v) for k, v in zip(keys, a)}

    def get_root(self):
        lo = np.zeros(3)
        k = C.c_int32(0)
        self._chk(self._lib.nb_get_root(self._h, _ptr(lo), C.byref(k)))
        return lo, int(k.value)

    def get_roots(self):
        ns = self.get_info()["n_sys"]
        lo = np.zeros((ns, 3))
        k = np.zeros(ns, np.int32)
        self._chk(self._lib.nb_get_roots(self._h, _ptr(lo), _ptr(k)))
        return lo, k

    def get_keys(self):
        key = np.zeros(self.n, np.uint64)
        orig = np.zeros(self.n, np.uint32)
        self._chk(self._lib.nb_get_keys(self._h, _ptr(key), _ptr(orig)))
        return key, orig

    def get_cells(self):
        nc = self.get_info()["n_cell"]
        out = dict(level=np.zeros(nc, np.uint8), begin=np.zeros(nc, np.uint32),
                   count=np.zeros(nc, np.uint32),
                   parent=np.zeros(nc, np.uint32),
                   skip=np.zeros(nc, np.uint32), leaf=np.zeros(nc, np.uint8),
                   ctr=np.zeros((nc, 3)))
        self._chk(self._lib.nb_get_cells(self._h, *(_ptr(out[k]) for k in (
            "level", "begin", "count", "parent", "skip", "leaf", "ctr"))))
        return out

    def get_moments(self):
        nc = self.get_info()["n_cell"]
        mass, com, quad = np.zeros(nc), np.zeros((nc, 3)), np.zeros((nc, 6))
        self._chk(self._lib.nb_get_moments(self._h, _ptr(mass), _ptr(com),
                                           _ptr(quad)))
        return mass, com, quad

    def get_groups(self):
        ng = self.get_info()["n_groups"]
        out = dict(cell=np.zeros(ng, np.uint32), begin=np.zeros(ng, np.uint32),
                   count=np.zeros(ng, np.uint32), lo=np.zeros((ng, 3)),
                   hi=np.zeros((ng, 3)), ctr=np.zeros((ng, 3)))
        self._chk(self._lib.nb_get_groups(self._h, *(_ptr(out[k]) for k in (
            "cell", "begin", "count", "lo", "hi", "ctr"))))
        return out

    def get_lists(self):
        info = self.get_info()
        ng, ne, ns = info["n_groups"], info["n_epj"], info["n_spj"]
        eo = np.zeros(ng + 1, np.int64)
        so = np.zeros(ng + 1, np.int64)
        e = np.zeros(ne, np.uint32)
        s = np.zeros(ns, np.uint32)
        self._chk(self._lib.nb_get_lists(self._h, _ptr(eo), _ptr(e), _ptr(so),
                                         _ptr(s)))
        return eo, e, so, s

    def upload_lists(self, epj_off, epj, spj_off, spj):
        """Install caller-made CSR index lists for the current tree (see
        nb_upload_lists); numpy arrays or CUDA tensors (int64 offsets,
        uint32/int32 ids), all on the same side."""
        dev = _is_torch(epj_off)
        if dev:
            for a in (epj_off, epj, spj_off, spj):
                assert a.is_cuda and a.is_contiguous()
            ng = epj_off.numel() - 1
            ne, ns = epj.numel(), spj.numel()
            ptrs = [a.data_ptr() if a.numel() else None
                    for a in (epj_off, epj, spj_off, spj)]
        else:
            eo = np.ascontiguousarray(epj_off, np.int64)
            so = np.ascontiguousarray(spj_off, np.int64)
            e = np.ascontiguousarray(epj, np.uint32)
            s = np.ascontiguousarray(spj, np.uint32)
            ng, ne, ns = eo.size - 1, e.size, s.size
            keep = (eo, e, so, s)
            ptrs = [_ptr(a) if a.size else None for a in keep]
        self._chk(self._lib.nb_upload_lists(self._h, ng, ptrs[0], ne, ptrs[1],
                                            ptrs[2], ns, ptrs[3],
                                            1 if dev else 0))

    # ---- short-range interactions ----
    def neighbour_lists(self, h_list):
        """Neighbour lists of every group for search radius h_list."""
        self._chk(self._lib.nb_neighbour_lists(self._h, float(h_list)))

    def sph_density(self, h):
        self._chk(self._lib.nb_sph_density(self._h, float(h)))

    def get_density(self, internal=False):
        rho = np.zeros(self.n)
        self._chk(self._lib.nb_get_density(self._h, _ptr(rho),
                                           1 if internal else 0))
        return rho

    def get_neighbour_lists(self):
        ne = np.zeros(1, np.int64)
        self._chk(self._lib.nb_get_neighbour_lists(self._h, _ptr(ne), None,
                                                   None))
        ng = self.get_info()["n_groups"]
        off = np.zeros(ng + 1, np.int64)
        ids = np.zeros(int(ne[0]), np.uint32)
        self._chk(self._lib.nb_get_neighbour_lists(self._h, None, _ptr(off),
                                                   _ptr(ids)))
        return off, ids

    def get_timing(self, reset=False):
        ms = np.zeros(len(PHASES))
        calls = np.zeros(len(PHASES), np.int64)
        self._chk(self._lib.nb_get_timing(self._h, _ptr(ms), _ptr(calls),
                                          1 if reset else 0))
        return {p: (float(t), int(c)) for p, t, c in zip(PHASES, ms, calls)}

    # ---- per-group list refresh and its predictor ----
    def group_features(self, out=None):
        """Predictor inputs [groups, 12] FP32; ``out`` may be a CUDA tensor
        (filled on the device), else a numpy array is returned."""
        if out is not None and _is_torch(out) and out.is_cuda:
            self._chk(self._lib.nb_group_features(
                self._h, C.c_void_p(out.data_ptr()), 1))
            return out
        ng = self.get_info()["n_groups"]
        f = np.zeros((ng, MLP_NIN), np.float32)
        self._chk(self._lib.nb_group_features(self._h, _ptr(f), 0))
        return f

    def group_stale(self, tau=0.0, label_out=None):
        """Stale flags at tolerance ``tau`` (bool array); with a CUDA tensor
        ``label_out`` the labels (0.0 / 1.0) are written there instead."""
        if label_out is not None and _is_torch(label_out) and label_out.is_cuda:
            self._chk(self._lib.nb_group_stale(
                self._h, float(tau), None, C.c_void_p(label_out.data_ptr()),
                1))
            return label_out
        ng = self.get_info()["n_groups"]
        st = np.zeros(ng, np.uint8)
        self._chk(self._lib.nb_group_stale(self._h, float(tau), _ptr(st),
                                           None, 0))
        return st.astype(bool)

    def refresh_lists(self, sel):
        sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
        self._chk(self._lib.nb_refresh_lists(self._h, sel.size, _ptr(sel)))

    def group_state(self):
        ng = self.get_info()["n_groups"]
        sa, so = np.zeros(ng), np.zeros(ng)
        age = np.zeros(ng, np.int32)
        self._chk(self._lib.nb_get_group_state(self._h, _ptr(sa), _ptr(so),
                                               _ptr(age)))
        return sa, so, age

    def cell_sides(self):
        nc = self.get_info()["n_cell"]
        out = np.zeros(nc)
        self._chk(self._lib.nb_get_cell_sides(self._h, _ptr(out)))
        return out

    def mlp_set(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._chk(self._lib.nb_mlp_set(self._h, _ptr(w), w.size))

    def mlp_get(self):
        w = np.zeros(MLP_NPARAM, np.float32)
        self._chk(self._lib.nb_mlp_get(self._h, _ptr(w), w.size))
        return w

    def _in(self, a, cols=None):
        """(pointer, rows, on_device) of an FP32 input array or tensor."""
        if _is_torch(a) and a.is_cuda:
            import torch
            if a.dtype != torch.float32 or not a.is_contiguous():
                raise ValueError("device inputs must be contiguous float32")
            return C.c_void_p(a.data_ptr()), a.shape[0], 1, a
        a = np.ascontiguousarray(a, dtype=np.float32)
        if cols is not None:
            a = a.reshape(-1, cols)
        return _ptr(a), a.shape[0], 0, a

    def mlp_forward(self, x):
        px, n, dev, keep = self._in(x, MLP_NIN)
        if dev:
            import torch
            p = torch.empty(n, dtype=torch.float32, device=x.device)
            self._chk(self._lib.nb_mlp_forward(self._h, n, px,
                                               C.c_void_p(p.data_ptr()), 1))
            return p
        p = np.zeros(n, np.float32)
        self._chk(self._lib.nb_mlp_forward(self._h, n, px, _ptr(p), 0))
        return p

    def mlp_grad(self, x, y, pos_weight=1.0):
        px, n, dev, kx = self._in(x, MLP_NIN)
        py, ny, dev2, ky = self._in(y)
        if ny != n or dev != dev2:
            raise ValueError("x and y disagree")
        loss = C.c_float(0.0)
        if dev:
            import torch
            g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=x.device)
            self._chk(self._lib.nb_mlp_grad(self._h, n, px, py,
                                            float(pos_weight), C.byref(loss),
                                            C.c_void_p(g.data_ptr()), 1))
            return float(loss.value), g
        g = np.zeros(MLP_NPARAM, np.float32)
        self._chk(self._lib.nb_mlp_grad(self._h, n, px, py, float(pos_weight),
                                        C.byref(loss), _ptr(g), 0))
        return float(loss.value), g

    def mlp_grad_static(self, x, y, grad, loss=None, pos_weight=1.0):
        """nb_mlp_grad_static: device tensors in and out (grad holds
        MLP_NPARAM floats, loss one float or None); only enqueued on the
        context's stream, no allocation, no synchronisation."""
        px, n, dev, kx = self._in(x, MLP_NIN)
        py, ny, dev2, ky = self._in(y)
        pg, ng, dev3, kg = self._in(grad)
        if not (dev and dev2 and dev3):
            raise ValueError("x, y and grad must be device tensors")
        if ny != n or ng != MLP_NPARAM:
            raise ValueError("x, y and grad disagree")
        pl = None
        if loss is not None:
            pl, nl, dev4, kl = self._in(loss)
            if not dev4 or nl < 1:
                raise ValueError("loss must be a device tensor")
        self._chk(self._lib.nb_mlp_grad_static(self._h, n, px, py,
                                               float(pos_weight), pl, pg))

    def mlp_adam(self, grad=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        if grad is None:
            self._chk(self._lib.nb_mlp_adam(self._h, None, lr, beta1, beta2,
                                            eps, 0))
            return
        pg, n, dev, keep = self._in(grad)
        self._chk(self._lib.nb_mlp_adam(self._h, pg, lr, beta1, beta2, eps,
                                        dev))

    def mlp_train(self, x, y, epochs=1, batch=4096, lr=1e-3, pos_weight=1.0):
        px, n, dev, kx = self._in(x, MLP_NIN)
        py, ny, dev2, ky = self._in(y)
        if ny != n or dev != dev2:
            raise ValueError("x and y disagree")
        loss = C.c_float(0.0)
        self._chk(self._lib.nb_mlp_train(self._h, n, px, py, dev, int(epochs),
                                         int(batch), float(lr),
                                         float(pos_weight), C.byref(loss)))
        return float(loss.value)
