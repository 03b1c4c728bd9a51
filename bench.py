"""Benchmark: GPU-resident Barnes-Hut leapfrog steps with list reuse.

Workload (default): disk galaxy, N = 2^22 (2^21 exponential-disk particles +
2^21 Hernquist-halo particles, halo particles 10x heavier), theta = 0.5,
eps = 0.01, dt = 1/128, interaction lists rebuilt every 4 steps (a
construction step every 4 steps, reuse steps in between).

One timed step = kick-drift + (construction step: root, keys, sort, reorder,
link, moments, groups, walk | reuse step: moments) + multiwalk force kernel.
Inputs are resident in HBM before timing starts.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--n-grp G]
                  [--no-cpu-baseline] [--copy-probe MiB]

``--sph`` times the short-range path instead (neighbour lists and SPH
densities on them, ``paper_1907_02290_amd.sph``) with the FP64 oracle's
lists and densities on the same workload as its CPU baseline:

  python bench.py --sph --workload sphere_4m [--neighbours 64] [--skin 0.3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_OP = 23              # flops per interaction (the paper's convention)
# flops of one quadrupole superparticle interaction counted the same way
# (FMA = 2, rsqrt = 4): 3 sub, r^2 6, rsqrt 4, f^2..f^7 4, S d 15, d.S.d 5,
# coefficient 7, 3 f^5 1, acceleration 12, potential 8
N_OP_QUAD = 65
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector peak
WORKLOAD = "disk_4m"


def recorded_traffic():
    """Force-kernel HBM bytes per launch from the committed counter summary,
    or None when the kernel source changed since the counters were taken."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_1907_02290_amd", "csrc", "nb_force.hip")
    prof = os.path.join(ROOT, "profiles", "disk_4m_hbm_counters.md")
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch=([0-9.eE+-]+) source_sha256=(\w+)",
                  text)
    if not m or m.group(2) != sha:
        return None
    return float(m.group(1))


def recorded_valu_busy():
    """VALU-busy fraction of the force kernel from the committed counter
    summary, or None when the kernel source changed since."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_1907_02290_amd", "csrc", "nb_force.hip")
    prof = os.path.join(ROOT, "profiles", "force_disk_4m_valu_counters.md")
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"valu_busy=([0-9.eE+-]+) source_sha256=(\w+)", text)
    if not m or m.group(2) != sha:
        return None
    return float(m.group(1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def direct_error(d, p, targets, seed=4242):
    """Accuracy guard of the autotuner: a function of the forces (original
    order) giving the 99th percentile of the relative acceleration error
    against the FP64 oracle's direct sum on `targets` sampled particles of
    the initial state (computed once here)."""
    import oracle
    n = d["x"].size
    rng = np.random.default_rng(seed)
    tgt = np.sort(rng.choice(n, size=min(targets, n), replace=False))
    ref = oracle.force_direct(d["x"], d["y"], d["z"], d["m"], p["eps"], 1.0,
                              tgt)
    den = np.sqrt(ref[0] ** 2 + ref[1] ** 2 + ref[2] ** 2)

    def err(forces):
        num = np.sqrt((forces[0][tgt] - ref[0]) ** 2 +
                      (forces[1][tgt] - ref[1]) ** 2 +
                      (forces[2][tgt] - ref[2]) ** 2)
        return float(np.percentile(num / den, 99))
    return err


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--n-grp", default=None,
                    help="group size, or 'auto' to run the autotuner first "
                         "(untimed)")
    ap.add_argument("--n-leaf", type=int, default=None)
    ap.add_argument("--theta", type=float, default=None,
                    help="opening angle (default: the workload's)")
    ap.add_argument("--tile-j", type=int, default=0,
                    help="force kernel tile (list entries per LDS tile; 0: "
                         "the library's default)")
    ap.add_argument("--waves", type=int, default=0,
                    help="force kernel occupancy target, waves per SIMD "
                         "(0: the library's default)")
    ap.add_argument("--reuse", type=int, default=None)
    ap.add_argument("--graph", action="store_true",
                    help="replay reuse steps from a captured HIP graph")
    ap.add_argument("--persistent", action="store_true",
                    help="persistent work-queue force launch")
    ap.add_argument("--copied-lists", action="store_true",
                    help="lists of copied j-data (the paper's G1) instead "
                         "of indices, for comparison")
    ap.add_argument("--latency-steps", type=int, default=32,
                    help="steps timed one by one afterwards (p50/p99)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--direct-targets", type=int, default=4096,
                    help="sampled targets of the FP64 direct-sum error "
                         "check (0: skip)")
    ap.add_argument("--sph", action="store_true",
                    help="time the short-range path (neighbour lists and "
                         "SPH densities) instead of the gravity step")
    ap.add_argument("--neighbours", type=float, default=64)
    ap.add_argument("--skin", type=float, default=0.3)
    ap.add_argument("--policies", action="store_true",
                    help="compare list-reuse policies at equal error: fixed "
                         "intervals against the learned per-group refresh "
                         "(errors against the FP64 oracle's direct sum)")
    ap.add_argument("--fixed", default="4,8,16",
                    help="construction intervals of the fixed policies")
    ap.add_argument("--fixed-thetas", default="0.45",
                    help="smaller opening angles for more fixed policies")
    ap.add_argument("--fixed-small", default="8,16",
                    help="intervals used with --fixed-thetas")
    ap.add_argument("--k-trees", default="16,32",
                    help="construction intervals of the learned policy")
    ap.add_argument("--tau", type=float, default=1.0,
                    help="staleness tolerance of the predictor's labels")
    ap.add_argument("--rebuild-frac", type=float, default=0.25,
                    help="learned policy: a construction step replaces a "
                         "refresh once this fraction of the groups is "
                         "flagged")
    ap.add_argument("--err-every", type=int, default=0,
                    help="policy runs: steps between error checks (0: 8 "
                         "checks per run)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run a plain device copy of this many MiB "
                         "(reference kernel for HBM counters)")
    return ap.parse_args()


def sph_main(args):
    """Short-range path: the library's neighbour lists and densities, and
    the FP64 oracle's on the same workload (CPU baseline)."""
    import torch
    from paper_1907_02290_amd import sph
    torch.cuda.set_device(0)
    workload = args.workload if args.workload != WORKLOAD else "sphere_4m"
    res = sph.measure(workload, args.n, args.neighbours, args.skin,
                      max(args.steps, 1),
                      int(args.n_grp) if args.n_grp else None, args.n_leaf)
    if not args.no_cpu_baseline:
        import oracle
        import workloads
        d, p = workloads.make(workload, n=args.n)
        h = res["h"]
        t = oracle.Tree(d["x"], d["y"], d["z"], d["m"], res["n_leaf"],
                        res["n_grp"])
        t0 = time.perf_counter()
        t.neighbour_lists(h * (1 + args.skin))
        t1 = time.perf_counter()
        t.sph_density(h)
        t2 = time.perf_counter()
        res["cpu_baseline"] = {
            "kind": "oracle", "cores": oracle.num_threads(),
            "list_s": t1 - t0, "density_s": t2 - t1,
            "value": res["pairs_per_eval"] / (t2 - t1),
            "unit": "candidate pairs/s",
            "sample": "FP64 oracle neighbour lists and densities of every "
                      "group of the same tree"}
    print(json.dumps(res), flush=True)


class DirectCheck:
    """Force errors against the FP64 oracle's direct sum (over each
    particle's own system) on a fixed sample of target particles, and the
    energy of a state from the run's own potentials."""

    def __init__(self, d, p, targets, seed=4242):
        n = d["x"].size
        off = d.get("offsets")
        self.off = off if off is not None else np.array([0, n])
        self.m = d["m"]
        self.eps = p["eps"]
        self.ext = p.get("ext_mass", 0.0)
        self.dt = p["dt"]
        rng = np.random.default_rng(seed)
        k = min(targets, n)
        self.tgt = np.sort(rng.choice(n, size=k, replace=False))
        self.seconds = 0.0

    def errors(self, x, y, z, forces):
        import oracle
        t0 = time.perf_counter()
        rel = []
        for s in range(self.off.size - 1):
            a, b = int(self.off[s]), int(self.off[s + 1])
            sel = self.tgt[(self.tgt >= a) & (self.tgt < b)]
            if sel.size == 0:
                continue
            r = oracle.force_direct(x[a:b], y[a:b], z[a:b], self.m[a:b],
                                    self.eps, 1.0, sel - a)
            num = np.sqrt((forces[0][sel] - r[0]) ** 2 +
                          (forces[1][sel] - r[1]) ** 2 +
                          (forces[2][sel] - r[2]) ** 2)
            den = np.sqrt(r[0] ** 2 + r[1] ** 2 + r[2] ** 2)
            rel.append(num[den > 0] / den[den > 0])
        self.seconds += time.perf_counter() - t0
        e = np.concatenate(rel)
        return float(np.median(e)), float(np.percentile(e, 99))

    def __call__(self, ctx):
        """Errors and energy of a context's current state and forces."""
        st = ctx.get_state()
        f = ctx.get_forces()
        med, p99 = self.errors(st[0], st[1], st[2], f)
        return dict(err_median=med, err_p99=p99, energy=self.energy(st, f))

    def energy(self, state, forces):
        """Total energy with the velocities brought to the positions' time
        (the kick-drift leaves them half a step behind)."""
        x, y, z, vx, vy, vz = state
        ax, ay, az, pot = forces
        if self.ext:
            r3 = (x * x + y * y + z * z) ** 1.5
            ax = ax - self.ext * x / r3
            ay = ay - self.ext * y / r3
            az = az - self.ext * z / r3
        h = 0.5 * self.dt
        ux, uy, uz = vx + h * ax, vy + h * ay, vz + h * az
        m = self.m
        e = 0.5 * np.sum(m * (ux * ux + uy * uy + uz * uz)) + \
            0.5 * np.sum(m * pot)
        if self.ext:
            e -= self.ext * np.sum(m / np.sqrt(x * x + y * y + z * z))
        return float(e)


def policies_main(args):
    """Equal-error comparison of list-reuse policies on one workload at full
    size: the paper's fixed reuse interval (section 4.2) at the workload's
    opening angle and at smaller ones, against the learned per-group
    refresh (predictor trained on another realisation of the workload).
    Errors are against the FP64 oracle's direct sum on sampled targets;
    the energy uses each run's own potentials."""
    import torch
    import workloads
    import paper_1907_02290_amd as nb
    from paper_1907_02290_amd import learn
    torch.cuda.set_device(0)
    wl = args.workload
    d0, p = workloads.make(wl, n=args.n, replicate=0)
    d1, _ = workloads.make(wl, n=args.n, replicate=1)
    theta, dt = p["theta"], p["dt"]
    steps = args.steps
    err_every = args.err_every or max(1, steps // 8)
    n_grp = int(args.n_grp) if args.n_grp and args.n_grp != "auto" \
        else p["n_grp"]
    n_leaf = args.n_leaf or p["n_leaf"]
    common = dict(eps=p["eps"], n_leaf=n_leaf, n_grp=n_grp, order=p["order"],
                  ext_mass=p.get("ext_mass", 0.0))
    ints = lambda v: [int(u) for u in v.split(",") if u]
    k_trees = ints(args.k_trees)
    tau = args.tau
    # training on replicate 0: labels after every reuse step of fixed
    # reuse with the first construction interval
    kt0 = k_trees[0] if k_trees else 16
    t0 = time.perf_counter()
    with learn.make_context(d0, theta=theta, k_max=kt0, tau=tau,
                            offsets=d0.get("offsets"), **common) as ctx:
        ctx.mlp_set(learn.init_weights(0))
        X, Y = learn.collect(ctx, 2 * kt0, dt, tau, kt0)
        cut = (2 * X.shape[0]) // 3
        loss = learn.train(ctx, X[:cut].contiguous(), Y[:cut].contiguous(),
                           epochs=30)
        pv = ctx.mlp_forward(X[cut:].contiguous()).cpu().numpy()
        yv = Y[cut:].cpu().numpy()
        p_star = learn.choose_threshold(pv, yv, 0.98)
        w = ctx.mlp_get()
    train = dict(rows=int(X.shape[0]), positives=float(Y.mean().item()),
                 loss=loss, p_star=p_star,
                 validation=learn.classify(pv, yv, p_star),
                 seconds=time.perf_counter() - t0)
    log("training: " + json.dumps(train))
    del X, Y
    check = DirectCheck(d1, p, args.direct_targets or 4096)
    runs = [("fixed", k, theta) for k in ints(args.fixed)]
    for th in (float(v) for v in args.fixed_thetas.split(",") if v):
        runs += [("fixed", k, th) for k in ints(args.fixed_small)]
    runs += [("learned", k, theta) for k in k_trees]
    results = []
    for policy, k, th in runs:
        kw = dict(common, theta=th)
        if policy == "fixed":
            ctx = nb.Context(graph=args.graph, **kw)
            ctx.set_particles(d1["x"], d1["y"], d1["z"], d1["vx"], d1["vy"],
                              d1["vz"], d1["m"])
            if "offsets" in d1:
                ctx.set_systems(d1["offsets"])
        else:
            ctx = learn.make_context(d1, k_max=k, p_star=p_star, tau=tau,
                                     offsets=d1.get("offsets"),
                                     graph=args.graph, **kw)
            ctx.mlp_set(w)
        with ctx:
            r = learn.run_policy(ctx, policy, steps, dt, k, check=check,
                                 check_every=err_every,
                                 rebuild_frac=(args.rebuild_frac
                                               if policy != "fixed" else None))
        c = r.pop("checks")
        e0, e1 = c[0]["energy"], c[-1]["energy"]
        r.update(theta=th,
                 force_err_median=float(np.mean([q["err_median"] for q in c])),
                 force_err_p99=float(np.mean([q["err_p99"] for q in c])),
                 force_err_p99_max=float(np.max([q["err_p99"] for q in c])),
                 energy_rel_change=abs(e1 - e0) / abs(e0), checks=len(c))
        log(json.dumps(r))
        results.append(r)
    out = dict(kind="policies", workload=wl, n=int(d1["x"].size),
               steps=steps, dt=dt, tau=tau, rebuild_frac=args.rebuild_frac,
               graph=bool(args.graph),
               n_grp=n_grp, n_leaf=n_leaf, training=train,
               error_reference="FP64 oracle direct sum over each particle's "
                               "system, %d sampled targets"
                               % check.tgt.size,
               oracle_seconds=check.seconds, results=results)
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU "
              "path (requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world),
              file=sys.stderr)
        sys.exit(2)
    if args.sph:
        sph_main(args)
        return
    if args.policies:
        policies_main(args)
        return

    import torch
    import workloads
    import paper_1907_02290_amd as nb

    d, p = workloads.make(args.workload, n=args.n)
    if args.theta is not None:
        p = dict(p, theta=args.theta)
    tuned = None
    tile_j, waves = args.tile_j, args.waves
    n_leaf = args.n_leaf or p["n_leaf"]
    if args.n_grp == "auto":
        from paper_1907_02290_amd import tune
        guard = None
        if args.direct_targets > 0 and "offsets" not in d:
            guard = direct_error(d, p, min(args.direct_targets, 1024))
        tuned = tune.tune(args.workload, args.n, n_leafs=(n_leaf,),
                          theta=p["theta"], error=guard, log=log)
        n_grp = tuned["best"]["n_grp"]
        tile_j = tuned["best"]["tile_j"]
        waves = tuned["best"]["waves_per_simd"]
        log("autotuner: n_grp %d tile_j %d waves %d (%.3f ms/step)"
            % (n_grp, tile_j, waves, tuned["best_ms_per_step"]))
    else:
        n_grp = int(args.n_grp) if args.n_grp else p["n_grp"]
    reuse = args.reuse or p.get("reuse", 4)
    dt = p["dt"]
    n = d["x"].size
    log("workload %s n=%d theta=%g eps=%g n_leaf=%d n_grp=%d reuse=%d"
        % (args.workload, n, p["theta"], p["eps"], n_leaf, n_grp, reuse))

    torch.cuda.set_device(0)
    dev = {k: torch.from_numpy(d[k]).cuda()
           for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
    ctx = nb.Context(theta=p["theta"], eps=p["eps"], n_leaf=n_leaf,
                     n_grp=n_grp, order=p["order"],
                     ext_mass=p.get("ext_mass", 0.0), timing=True,
                     graph=args.graph, persistent=args.persistent,
                     copied_lists=args.copied_lists, tile_j=tile_j,
                     waves_per_simd=waves)
    ctx.set_particles(dev["x"], dev["y"], dev["z"], dev["vx"], dev["vy"],
                      dev["vz"], dev["m"])
    del dev
    n_sys = 1
    if "offsets" in d:
        ctx.set_systems(d["offsets"])
        n_sys = d["offsets"].size - 1

    # KDK leapfrog with merged half kicks.  Step g (g >= 1): kick (dt/2 for
    # g = 1, else dt), drift dt, forces; a construction step when g is a
    # multiple of `reuse`, a reuse step otherwise.  Forces at t = 0 come
    # from an untimed construction step.
    step_no = [1]

    def step():
        g = step_no[0]
        mode = nb.NB_MAKE_LIST_FOR_REUSE if g % reuse == 0 else \
            nb.NB_REUSE_LIST
        ctx.step(mode, dt / 2 if g == 1 else dt, dt)
        step_no[0] += 1
        return mode

    ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
    # forces of the initial (seeded) state, checked against the FP64 oracle
    # at the end
    gx, gy, gz, gp = ctx.get_forces()
    info_first = ctx.get_info()
    # warm up, then start timing on a construction step so the timed steps
    # hold whole reuse cycles
    warm = 0
    while warm < args.warmup or step_no[0] % reuse != 0:
        step()
        warm += 1
    torch.cuda.synchronize()
    ctx.get_timing(reset=True)
    info0 = ctx.get_info()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    info1 = ctx.get_info()
    timing = ctx.get_timing(reset=True)
    elapsed = t1 - t0
    inter = info1["total_inter"] - info0["total_inter"]
    inter_spj = info1["total_inter_spj"] - info0["total_inter_spj"]
    evals = info1["force_evals"] - info0["force_evals"]
    value = inter / elapsed
    ms_step = elapsed / args.steps * 1e3
    f_ms, f_calls = timing["force"]
    f_avg_s = f_ms / max(f_calls, 1) * 1e-3
    inter_per_launch = inter / max(evals, 1)
    # quadrupole superparticle interactions carry their own flop count
    quad_share = inter_spj / max(inter, 1) if p["order"] == 2 else 0.0
    flops_per_inter = N_OP * (1 - quad_share) + N_OP_QUAD * quad_share
    flops_per_launch = flops_per_inter * inter_per_launch
    achieved = flops_per_launch / f_avg_s / 1e12 if f_avg_s > 0 else 0
    log("timed %d steps in %.3f s: %.3f ms/step, %.3e interactions/s"
        % (args.steps, elapsed, ms_step, value))
    log("phase ms: " + ", ".join("%s %.2f/%d" % (k, v[0], v[1])
                                 for k, v in timing.items()))

    # latency: steps timed one by one (host clock around a device-wide
    # synchronisation), construction and reuse steps apart
    lat = {"construction": [], "reuse": []}
    for _ in range(args.latency_steps):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        mode = step()
        torch.cuda.synchronize()
        kind = "reuse" if mode == nb.NB_REUSE_LIST else "construction"
        lat[kind].append((time.perf_counter() - ta) * 1e3)
    every = lat["construction"] + lat["reuse"]
    latency = {"steps": len(every)}
    for k, v in (("all", every), ("construction", lat["construction"]),
                 ("reuse", lat["reuse"])):
        if v:
            latency[k] = {"p50_ms": float(np.percentile(v, 50)),
                          "p99_ms": float(np.percentile(v, 99)),
                          "count": len(v)}
    if n_sys > 1:
        latency["note"] = ("the %d systems advance together, so every "
                           "system's step latency is the batch step time"
                           % n_sys)
    log("latency: " + json.dumps(latency))

    if args.copy_probe:
        a = torch.empty(args.copy_probe * (1 << 20) // 4, dtype=torch.float32,
                        device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: %d MiB" % args.copy_probe)

    # force error of the first construction step vs the FP64 oracle, and
    # the CPU baseline on a bounded sample of groups (both on the seeded
    # initial state)
    info_last = info_first
    ctx.close()

    force_err = None
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        tb = time.perf_counter()
        t = oracle.Tree(d["x"], d["y"], d["z"], d["m"], n_leaf, n_grp)
        t_build = time.perf_counter() - tb
        rng = np.random.default_rng(12345)
        gcount = t.groups()["count"].astype(np.int64)

        def run(sel):
            ta = time.perf_counter()
            ng, ne, ns = t.make_lists(p["theta"], sel)
            f = t.force_lists(p["order"], p["eps"], 1.0)
            eo, e, so, s = t.lists()
            it = int((gcount[sel] * (np.diff(eo) + np.diff(so))).sum())
            return time.perf_counter() - ta, it, f

        probe = np.sort(rng.choice(t.n_groups, size=min(64, t.n_groups),
                                   replace=False))
        tp, ip, _ = run(probe)
        rate = ip / max(tp, 1e-6)
        per_group = ip / probe.size
        want = int(min(t.n_groups, max(64, args.cpu_seconds * rate /
                                       max(per_group, 1))))
        sel = np.sort(rng.choice(t.n_groups, size=want, replace=False))
        tc, ic, f = run(sel)
        mask = np.isfinite(f[0])
        num = np.sqrt((gx - f[0]) ** 2 + (gy - f[1]) ** 2 +
                      (gz - f[2]) ** 2)[mask]
        den = np.sqrt(f[0] ** 2 + f[1] ** 2 + f[2] ** 2)[mask]
        ea = num[den > 0] / den[den > 0]
        ep = (np.abs(gp - f[3])[mask] / np.abs(f[3])[mask])
        force_err = {"median": float(np.median(ea)),
                     "p99": float(np.percentile(ea, 99)),
                     "max": float(ea.max()),
                     "pot_median": float(np.median(ep)),
                     "particles": int(mask.sum()),
                     "reference": "FP64 oracle sum over the same lists"}
        cpu = {"value": ic / tc, "unit": "interactions/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "FP64 oracle walk + list-force sum over %d of %d "
                         "groups (%d particles, %.3e interactions) of the "
                         "construction step of the seeded initial state of "
                         "the same workload; oracle tree build (%.1f s, all "
                         "N) not counted"
                         % (sel.size, t.n_groups, int(gcount[sel].sum()),
                            ic, t_build),
               "seconds": tc}
        log("cpu baseline: %.3e interactions/s on %d threads (%.1f s); "
            "force err median %.2e" % (cpu["value"], cpu["cores"], tc,
                                       force_err["median"]))

    # Barnes-Hut error: the same initial forces against the oracle's FP64
    # direct sum over all N on sampled targets
    force_err_direct = None
    if args.direct_targets > 0 and n_sys == 1:
        import oracle
        rng = np.random.default_rng(4242)
        tgt = np.sort(rng.choice(n, size=min(args.direct_targets, n),
                                 replace=False))
        td = time.perf_counter()
        ref = oracle.force_direct(d["x"], d["y"], d["z"], d["m"], p["eps"],
                                  1.0, tgt)
        td = time.perf_counter() - td
        num = np.sqrt((gx[tgt] - ref[0]) ** 2 + (gy[tgt] - ref[1]) ** 2 +
                      (gz[tgt] - ref[2]) ** 2)
        den = np.sqrt(ref[0] ** 2 + ref[1] ** 2 + ref[2] ** 2)
        ea = num / den
        ep = np.abs(gp[tgt] - ref[3]) / np.abs(ref[3])
        force_err_direct = {
            "median": float(np.median(ea)), "p99": float(np.percentile(ea, 99)),
            "max": float(ea.max()), "pot_median": float(np.median(ep)),
            "targets": int(tgt.size),
            "reference": "FP64 oracle direct sum over all N particles "
                         "(softened, self term excluded) on sampled targets; "
                         "the error of the Barnes-Hut lists at this theta "
                         "plus the FP32 kernel's",
            "oracle_seconds": td}
        log("force err vs direct sum: median %.2e p99 %.2e (%d targets, "
            "%.1f s)" % (force_err_direct["median"], force_err_direct["p99"],
                         tgt.size, td))

    out = {
        "metric": "interactions/s at N=2^22, theta=0.5 (lists reused every "
                  "4 steps); ms/step and rel force err vs FP64 oracle beside",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warm,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (force kernel); f64 (keys, tree, walk, integration)",
        "data": "synthetic",
        "config": {
            "workload": "%s: exponential disk 2^21 + Hernquist halo 2^21 "
                        "(halo particles 10x heavier), eps 0.01, dt 1/128"
                        % args.workload if args.workload == "disk_4m"
                        else args.workload,
            "n": n, "theta": p["theta"], "eps": p["eps"], "n_leaf": n_leaf,
            "n_grp": n_grp, "order": p["order"], "reuse_every": reuse,
            "groups": info_last["n_groups"], "cells": info_last["n_cell"],
            "mean_n_i": n / max(info_last["n_groups"], 1),
            "mean_list": (info_last["n_epj"] + info_last["n_spj"]) /
                         max(info_last["n_groups"], 1),
            "force_evals": evals,
            "force_work_items": info_last["n_wi"],
            "n_grp_autotuned": tuned is not None,
            "tile_j": tile_j, "waves_per_simd": waves,
            "systems": n_sys,
            "graph": bool(args.graph),
            "persistent_force": bool(args.persistent),
            "lists": "copied j-data" if args.copied_lists else "indices",
        },
        "step_latency": latency,
        "roofline": {
            "kernel": "k_force (multiwalk force, %s)" % (
                "monopole" if p["order"] == 1 else
                "monopole particles + quadrupole superparticles"),
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": (recorded_traffic()
                        if args.workload == WORKLOAD and n_grp == 256 and
                        args.n is None else None),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + "
                            "WRITE_SIZE x 1.0, scaled on a 1 GiB copy)",
            "flops_per_launch": flops_per_launch,
            "flops_per_interaction": flops_per_inter,
            "avg_launch_ms": f_avg_s * 1e3,
            "valu_busy": (recorded_valu_busy()
                          if args.workload == WORKLOAD and n_grp == 256 and
                          args.n is None else None),
        },
        "cpu_baseline": cpu,
        "force_err": force_err,
        "force_err_direct": force_err_direct,
        "phase_ms_per_step": {k: v[0] / args.steps for k, v in timing.items()},
        "interactions_per_s_frac_of_fp32_peak": value * flops_per_inter /
                                                (FP32_PEAK_TFLOPS * 1e12),
        "superparticle_interactions_per_s": inter_spj / elapsed,
        "superparticle_share": inter_spj / max(inter, 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
