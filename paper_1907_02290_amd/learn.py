"""Learned per-group list refresh: label collection, training of the
staleness predictor on the GPU, threshold choice, and runs of the reuse
policies that the predictor is compared with.

Every computation goes through the library's C ABI (``nbody.Context``); this
module only sequences the calls and keeps the training rows in device
tensors.

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
                 k_max=16, p_star=0.5, tau=0.1, offsets=None, timing=False):
    ctx = nb.Context(theta=theta, eps=eps, n_leaf=n_leaf, n_grp=n_grp,
                     order=order, ext_mass=ext_mass, refresh=True,
                     k_max=k_max, p_star=p_star, tau=tau, timing=timing)
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


class Reference:
    """Direct-sum forces (theta = 0: every list holds every particle of the
    system) through the same library, for the error of a policy's forces at
    the positions it reached."""

    def __init__(self, eps, G=1.0, ext_mass=0.0, n_grp=256, offsets=None):
        self.ctx = nb.Context(theta=0.0, eps=eps, G=G, n_leaf=8, n_grp=n_grp,
                              order=1, ext_mass=ext_mass)
        self.offsets = offsets
        self.ext_mass = ext_mass
        self.G = G

    def close(self):
        self.ctx.close()

    def forces(self, x, y, z, m):
        zero = np.zeros_like(x)
        self.ctx.set_particles(x, y, z, zero, zero, zero, m)
        if self.offsets is not None:
            self.ctx.set_systems(self.offsets)
        self.ctx.compute_forces(nb.NB_MAKE_LIST)
        return self.ctx.get_forces()

    def energy(self, x, y, z, vx, vy, vz, m, pot):
        kin = 0.5 * np.sum(m * (vx * vx + vy * vy + vz * vz))
        e = kin + 0.5 * np.sum(m * pot)
        if self.ext_mass:
            e -= self.G * self.ext_mass * np.sum(m / np.sqrt(x * x + y * y +
                                                             z * z))
        return float(e)


def force_error(got, ref):
    ax, ay, az = got[:3]
    rx, ry, rz = ref[:3]
    num = np.sqrt((ax - rx) ** 2 + (ay - ry) ** 2 + (az - rz) ** 2)
    den = np.sqrt(rx * rx + ry * ry + rz * rz)
    ok = den > 0
    return num[ok] / den[ok]


def run_policy(ctx, policy, steps, dt, k, tau, measure=True, ref=None,
               m=None, err_every=4):
    """Run ``steps`` leapfrog steps under a policy (see module doc).  With
    ``measure`` the staleness of the lists the force kernel used is checked
    after every reuse step, and with ``ref`` (a Reference) the forces are
    compared with the direct sum every ``err_every`` steps and the energy
    is evaluated; all of that outside the timed region.  Returns a dict with
    the wall time of the steps, list walks per step (all groups at a
    construction step, refreshed groups otherwise), stale fractions, force
    errors and the relative energy change."""
    import torch
    walks = 0
    stale = []
    errs = []
    energies = []
    t_run = 0.0
    refreshed = 0

    def check(s):
        if ref is None or s % err_every:
            return
        x, y, z, vx, vy, vz = ctx.get_state()
        got = ctx.get_forces()
        r = ref.forces(x, y, z, m)
        e = force_error(got, r)
        errs.append((float(np.median(e)), float(np.percentile(e, 99))))
        energies.append(ref.energy(x, y, z, vx, vy, vz, m, r[3]))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
    walks += ctx.get_info()["n_groups"]
    torch.cuda.synchronize()
    t_run += time.perf_counter() - t0
    check(0)
    for s in range(1, steps + 1):
        dtk = dt / 2 if s == 1 else dt
        t0 = time.perf_counter()
        if s % k == 0:
            ctx.step(nb.NB_MAKE_LIST_FOR_REUSE, dtk, dt)
            walks += ctx.get_info()["n_groups"]
        elif policy == "fixed":
            ctx.step(nb.NB_REUSE_LIST, dtk, dt)
        elif policy == "learned":
            ctx.step(nb.NB_REUSE_REFRESH, dtk, dt)
            r = ctx.get_info()["last_refreshed"]
            walks += r
            refreshed += r
        elif policy == "checked":
            ctx.step(nb.NB_REUSE_CHECK, dtk, dt)
            r = ctx.get_info()["last_refreshed"]
            walks += r
            refreshed += r
        else:
            raise ValueError(policy)
        torch.cuda.synchronize()
        t_run += time.perf_counter() - t0
        if measure and s % k != 0:
            stale.append(float(np.mean(ctx.group_stale(tau))))
        check(s)
    ng = ctx.get_info()["n_groups"]
    out = dict(policy=policy, k=k, steps=steps, seconds=t_run,
               ms_per_step=1e3 * t_run / (steps + 1),
               walks_per_step=walks / (steps + 1),
               walk_fraction=walks / (steps + 1) / max(1, ng),
               refreshed=refreshed,
               stale_mean=float(np.mean(stale)) if stale else 0.0,
               stale_max=float(np.max(stale)) if stale else 0.0)
    if errs:
        e = np.array(errs)
        out.update(force_err_median=float(e[:, 0].mean()),
                   force_err_p99=float(e[:, 1].mean()),
                   force_err_p99_max=float(e[:, 1].max()),
                   energy_rel_change=abs(energies[-1] - energies[0]) /
                   abs(energies[0]))
    return out


def evaluate(workload="disk_4m", n=1 << 18, tau=0.1, k_tree=16,
             collect_cycles=3, recall=0.98, epochs=30, batch=8192, lr=2e-3,
             steps=64, fixed=(1, 2, 4, 8, 16), k_trees=None,
             fixed_thetas=(), log=print):
    """Train the predictor on one realisation of a workload (seed 0) and
    compare the reuse policies on another (seed 1).  Returns a list of
    result dicts: the training summary, then one per policy."""
    import torch
    import workloads
    d0, p = workloads.make(workload, n=n, replicate=0)
    d1, _ = workloads.make(workload, n=n, replicate=1)
    common = dict(theta=p["theta"], eps=p["eps"], n_leaf=p["n_leaf"],
                  n_grp=p["n_grp"], order=p["order"],
                  ext_mass=p.get("ext_mass", 0.0), tau=tau)
    dt = p["dt"]
    out = []
    with make_context(d0, k_max=k_tree, offsets=d0.get("offsets"),
                      **common) as ctx:
        ctx.mlp_set(init_weights(0))
        t0 = time.perf_counter()
        X, Y = collect(ctx, collect_cycles * k_tree, dt, tau, k_tree)
        torch.cuda.synchronize()
        t_collect = time.perf_counter() - t0
        n_rows = X.shape[0]
        cut = (2 * n_rows) // 3
        t0 = time.perf_counter()
        loss = train(ctx, X[:cut].contiguous(), Y[:cut].contiguous(),
                     epochs=epochs, batch=batch, lr=lr)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        pv = ctx.mlp_forward(X[cut:].contiguous()).cpu().numpy()
        yv = Y[cut:].cpu().numpy()
        p_star = choose_threshold(pv, yv, recall)
        w = ctx.mlp_get()
    stats = classify(pv, yv, p_star)
    summary = dict(kind="training", workload=workload, n=int(d0["x"].size),
                   tau=tau, k_tree=k_tree, rows=int(n_rows),
                   train_rows=int(cut), positives=float(Y.mean().item()),
                   loss=loss, p_star=p_star, collect_s=t_collect,
                   train_s=t_train, validation=stats)
    log(summary)
    out.append(summary)
    # fixed intervals at the workload's theta and at smaller angles (the
    # equal-error comparison), then the refresh policies
    runs = [("fixed", k, p["theta"]) for k in fixed]
    runs += [("fixed", k, th) for th in fixed_thetas for k in (2, 4, 8)]
    for kt in (k_trees or (k_tree,)):
        runs += [("checked", kt, p["theta"]), ("learned", kt, p["theta"])]
    ref = Reference(p["eps"], ext_mass=p.get("ext_mass", 0.0),
                    offsets=d1.get("offsets"))
    for policy, k, th in runs:
        cfg = dict(common, theta=th)
        with make_context(d1, k_max=k_tree, p_star=min(1.0, max(0.0, p_star)),
                          offsets=d1.get("offsets"), **cfg) as ctx:
            ctx.mlp_set(w)
            r = run_policy(ctx, policy, steps, dt, k, tau, ref=ref,
                           m=d1["m"])
        r.update(kind="policy", workload=workload, n=int(d1["x"].size),
                 tau=tau, theta=th)
        log(r)
        out.append(r)
    ref.close()
    return out


def main(argv=None):
    import argparse
    import json
    import os
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="disk_4m")
    ap.add_argument("--n", type=int, default=1 << 18)
    ap.add_argument("--tau", type=float, default=0.1)
    ap.add_argument("--k-tree", type=int, default=16)
    ap.add_argument("--cycles", type=int, default=3)
    ap.add_argument("--recall", type=float, default=0.98)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--fixed-thetas", default="",
                    help="comma list of smaller opening angles for extra "
                         "fixed-interval runs (K = 2, 4, 8)")
    ap.add_argument("--k-trees", default=None,
                    help="comma list of construction intervals for the "
                         "refresh policies (default: --k-tree)")
    a = ap.parse_args(argv)
    kts = tuple(int(v) for v in a.k_trees.split(",")) if a.k_trees else None
    fth = tuple(float(v) for v in a.fixed_thetas.split(",") if v)
    res = evaluate(a.workload, a.n, a.tau, a.k_tree, a.cycles, a.recall,
                   a.epochs, steps=a.steps, k_trees=kts, fixed_thetas=fth,
                   log=lambda r: print(json.dumps(r), file=sys.stderr,
                                       flush=True))
    for r in res:
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
