"""Learned per-group list refresh: label collection, training of the
staleness predictor on the GPU, threshold choice, and runs of the reuse
policies that the predictor is compared with.

Every computation goes through the library's C ABI (``nbody.Context``); this
module only sequences the calls and keeps the training rows in device
tensors.  It measures no accuracy itself: callers pass a check function
(``bench.py --policies`` passes errors against the FP64 oracle's direct sum
on sampled particles).

Policies (``run_policy``):
  * ``fixed``   -- the paper's reuse (section 4.2): a construction step every
                   ``k`` steps, the kept lists in between;
  * ``learned`` -- a construction step every ``k`` steps, and in between each
                   group's list is walked again when the predictor's p exceeds
                   ``p_star`` or the list is ``k_max`` steps old
                   (NB_REUSE_REFRESH);
  * ``checked`` -- the same with the exact staleness check instead of the
                   predictor (the check reads every kept superparticle each
                   step; a reference for what the predictor approximates).
"""
from __future__ import annotations

import time

import numpy as np

from . import nbody as nb


def _torch():
    import torch
    return torch


def make_context(d, theta, eps, n_leaf=8, n_grp=64, order=1, ext_mass=0.0,
                 k_max=16, p_star=0.5, tau=0.1, offsets=None, timing=False,
                 graph=False):
    ctx = nb.Context(theta=theta, eps=eps, n_leaf=n_leaf, n_grp=n_grp,
                     order=order, ext_mass=ext_mass, refresh=True,
                     k_max=k_max, p_star=p_star, tau=tau, timing=timing,
                     graph=graph)
    ctx.set_particles(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"],
                      d["m"])
    if offsets is not None:
        ctx.set_systems(offsets)
    return ctx


def collect(ctx, steps, dt, tau, rebuild_every, device="cuda"):
    """Leapfrog steps with the paper's fixed reuse (construction every
    ``rebuild_every`` steps); after every reuse step the predictor inputs and
    the staleness labels at tolerance ``tau`` of all groups are appended.
    Returns (X [rows, 12], Y [rows]) as device tensors."""
    torch = _torch()
    xs, ys = [], []
    ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
    for s in range(1, steps + 1):
        dtk = dt / 2 if s == 1 else dt
        if s % rebuild_every == 0:
            ctx.step(nb.NB_MAKE_LIST_FOR_REUSE, dtk, dt)
            continue
        ctx.step(nb.NB_REUSE_LIST, dtk, dt)
        ng = ctx.get_info()["n_groups"]
        x = torch.empty((ng, nb.MLP_NIN), dtype=torch.float32, device=device)
        y = torch.empty(ng, dtype=torch.float32, device=device)
        ctx.group_features(out=x)
        ctx.group_stale(tau, label_out=y)
        xs.append(x)
        ys.append(y)
    return torch.cat(xs), torch.cat(ys)


def init_weights(seed, scale=None):
    """Glorot-style random weights (W1, W2, w3 scaled by fan-in), zero
    biases, FP32."""
    rng = np.random.default_rng(seed)
    w = np.zeros(nb.MLP_NPARAM, np.float32)
    o = 0
    for rows, cols in ((64, 12), (64, 64), (1, 64)):
        k = rows * cols
        sc = scale if scale is not None else 1.0 / np.sqrt(cols)
        w[o:o + k] = rng.standard_normal(k) * sc
        o += k
        o += rows  # biases stay zero
    return w


def train(ctx, X, Y, epochs=20, batch=8192, lr=2e-3, pos_weight=None,
          seed=0):
    """Shuffle the rows once (seeded), then train on the GPU.  pos_weight
    defaults to the negative/positive ratio (capped at 50).  Returns the
    final loss."""
    torch = _torch()
    n = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(n, generator=g).to(X.device)
    Xs = X[perm].contiguous()
    Ys = Y[perm].contiguous()
    if pos_weight is None:
        pos = float(Ys.sum().item())
        pos_weight = min(50.0, max(1.0, (n - pos) / max(pos, 1.0)))
    return ctx.mlp_train(Xs, Ys, epochs=epochs, batch=batch, lr=lr,
                         pos_weight=pos_weight)


def choose_threshold(p, y, recall=0.98):
    """Largest p* such that the rows with p > p* hold at least ``recall`` of
    the positive labels (host arrays)."""
    p = np.asarray(p, np.float64)
    y = np.asarray(y) > 0.5
    if not y.any():
        return 1.0
    ps = np.sort(p[y])
    # p* just below the (1 - recall) quantile of the positives' scores
    k = int(np.floor((1.0 - recall) * ps.size))
    return float(np.nextafter(ps[k], -np.inf)) if k < ps.size else 0.0


def classify(p, y, p_star):
    p = np.asarray(p)
    y = np.asarray(y) > 0.5
    flag = p > p_star
    tp = int(np.sum(flag & y))
    return dict(recall=tp / max(1, int(y.sum())),
                flagged=float(flag.mean()), positives=float(y.mean()),
                precision=tp / max(1, int(flag.sum())))


def force_error(got, ref):
    """Per-particle |a - a_ref| / |a_ref| of two (ax, ay, az, ...) tuples."""
    ax, ay, az = got[:3]
    rx, ry, rz = ref[:3]
    num = np.sqrt((ax - rx) ** 2 + (ay - ry) ** 2 + (az - rz) ** 2)
    den = np.sqrt(rx * rx + ry * ry + rz * rz)
    ok = den > 0
    return num[ok] / den[ok]


def run_policy(ctx, policy, steps, dt, k, tau=None, check=None,
               check_every=4, rebuild_frac=None):
    """Run ``steps`` leapfrog steps under a policy (see the module doc) from
    a construction step at the initial state.  The wall time of every step
    is taken around device synchronisations.  With ``tau`` the fraction of
    groups whose list fails the relaxed test at tolerance tau is recorded
    after every reuse step; with ``check`` (a function of the context that
    returns a dict of numbers, for example errors against a reference) it is
    called at step 0, at every ``check_every``-th step and at the last one.
    Both happen outside the timed steps.  ``rebuild_frac`` (refresh
    policies): when a step walks more than that fraction of the groups
    again, or a walked-again list did not fit its group's list slot, the
    next step is a construction step.  Returns ms/step, list walks
    per step (all groups at a construction step, refreshed groups
    otherwise), construction steps, the rebuilds each trigger asked for,
    the refreshed and overflowed groups of every step, stale fractions and
    the check results (a list of dicts)."""
    import torch
    times = []
    stale = []
    checks = []
    walks = refreshed = constructions = 0

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)

    timed(lambda: ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE))
    ng = ctx.get_info()["n_groups"]
    walks += ng
    constructions += 1
    if check is not None:
        checks.append(dict(step=0, **check(ctx)))
    since = 0
    rebuild_next = False
    by_frac = by_overflow = 0
    per_step = []
    reuse_mode = {"fixed": nb.NB_REUSE_LIST, "learned": nb.NB_REUSE_REFRESH,
                  "checked": nb.NB_REUSE_CHECK}[policy]
    for s in range(1, steps + 1):
        dtk = dt / 2 if s == 1 else dt
        since += 1
        build = since >= k or rebuild_next
        mode = nb.NB_MAKE_LIST_FOR_REUSE if build else reuse_mode
        timed(lambda: ctx.step(mode, dtk, dt))
        info = ctx.get_info()
        if build:
            since = 0
            rebuild_next = False
            walks += info["n_groups"]
            constructions += 1
        elif policy != "fixed":
            r = info["last_refreshed"]
            ovf = info["last_overflow"]
            walks += r
            refreshed += r
            per_step.append((s, r, ovf))
            if rebuild_frac is not None:
                # too many lists to walk again, or a walked list that no
                # longer fits its slot: the tree has aged, build a new one
                frac = r > rebuild_frac * info["n_groups"]
                rebuild_next = frac or ovf > 0
                by_frac += int(frac)
                by_overflow += int(ovf > 0 and not frac)
            if tau is not None:
                stale.append(float(np.mean(ctx.group_stale(tau))))
        elif tau is not None:
            stale.append(float(np.mean(ctx.group_stale(tau))))
        if check is not None and (s % check_every == 0 or s == steps):
            checks.append(dict(step=s, **check(ctx)))
    return dict(policy=policy, k=k, steps=steps,
                ms_per_step=1e3 * float(np.sum(times)) / len(times),
                construction_steps=constructions,
                rebuilds_by_fraction=by_frac, rebuilds_by_overflow=by_overflow,
                refresh_steps=per_step,
                walks_per_step=walks / len(times),
                walk_fraction=walks / len(times) / max(1, ng),
                refreshed=refreshed,
                stale_mean=float(np.mean(stale)) if stale else 0.0,
                stale_max=float(np.max(stale)) if stale else 0.0,
                checks=checks)
