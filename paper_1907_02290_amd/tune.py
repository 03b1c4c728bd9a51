"""Autotuner for the group size n_grp, the leaf size n_leaf and the tile
shape of the force kernel.

The paper picks the group size by hand from a sweep (its n_grp study of
section 6.1); here the sweep runs on the device the library will use: for
every candidate it times whole reuse cycles of the real step (construction
step plus reuse steps, inputs resident on the GPU) and keeps the fastest.

Stage 1 sweeps n_grp x n_leaf at the default tile shape.  Stage 2 sweeps the
force kernel's instances (tile_j list entries per LDS tile, and the
occupancy its registers are allotted for, waves_per_simd) at the stage-1
choice.  An optional accuracy guard keeps the tuner from buying time with
error: ``error(forces)`` (supplied by the caller, for example the p99
relative force error against a direct sum on sampled particles) is taken on
the forces of each candidate's first construction step, and a candidate is
admissible only when that error is at most ``max_err`` or, without it,
``guard`` times the error of the workload's own (n_grp, n_leaf).  Larger
groups open more cells (their boxes are larger) and so are more accurate;
the tile shape does not change which interactions are summed.

The result is a small JSON record that ``bench.py --n-grp auto`` and users
can pass back as configuration.

  python -m paper_1907_02290_amd.tune --workload disk_4m [--n N]
         [--n-grp 32,48,64,96,128,192,256,384,512] [--n-leaf 8]
         [--tile-j 64,128,192,256]
         [--waves 4,6,8] [--cycles 2] [--theta T] [--out F]
"""
from __future__ import annotations

import json
import time

from . import nbody as nb


def time_config(d_dev, p, n_grp, n_leaf, reuse, cycles, offsets=None,
                tile_j=0, waves_per_simd=0, theta=None, error=None):
    """Mean ms per step over `cycles` reuse cycles after one warm-up cycle
    (construction step at the start of each cycle), the interactions of the
    last construction step, and error(forces of the first construction
    step) when an error function is given."""
    import torch
    dt = p["dt"]
    with nb.Context(theta=p["theta"] if theta is None else theta,
                    eps=p["eps"], n_leaf=n_leaf, n_grp=n_grp,
                    order=p["order"], ext_mass=p.get("ext_mass", 0.0),
                    tile_j=tile_j, waves_per_simd=waves_per_simd) as ctx:
        ctx.set_particles(d_dev["x"], d_dev["y"], d_dev["z"], d_dev["vx"],
                          d_dev["vy"], d_dev["vz"], d_dev["m"])
        if offsets is not None:
            ctx.set_systems(offsets)
        ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
        err = error(ctx.get_forces()) if error is not None else None

        def cycle():
            for s in range(reuse):
                mode = nb.NB_REUSE_LIST if s else nb.NB_MAKE_LIST_FOR_REUSE
                ctx.step(mode, dt, dt)

        cycle()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(cycles):
            cycle()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / (cycles * reuse)
        info = ctx.get_info()
    return ms, info, err


def tune(workload, n=None, n_grps=(32, 48, 64, 96, 128, 192, 256, 384, 512),
         n_leafs=(8,),
         tiles=(64, 128, 192, 256), waves=(4, 6, 8), cycles=2, reuse=None,
         theta=None, error=None, guard=1.05, max_err=None, log=None):
    import torch
    import workloads
    d, p = workloads.make(workload, n=n)
    reuse = reuse or p.get("reuse", 4)
    dev = {k: torch.from_numpy(d[k]).cuda()
           for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
    offsets = d.get("offsets")

    def run(ng, nl, tj, w, stage):
        ms, info, err = time_config(dev, p, ng, nl, reuse, cycles, offsets,
                                    tj, w, theta, error)
        r = dict(stage=stage, n_grp=ng, n_leaf=nl, tile_j=tj,
                 waves_per_simd=w, ms_per_step=ms, groups=info["n_groups"],
                 interactions=info["n_inter"])
        if err is not None:
            r["err"] = err
        if log:
            log(r)
        return r

    grid = [(ng, nl) for nl in n_leafs for ng in n_grps]
    home = (p["n_grp"], p["n_leaf"])
    if error is not None and max_err is None and home not in grid:
        grid.append(home)
    stage1 = [run(ng, nl, 0, 0, 1) for ng, nl in grid]
    bound = max_err
    if error is not None and bound is None:
        ref = next(r for r in stage1 if (r["n_grp"], r["n_leaf"]) == home)
        bound = guard * ref["err"]

    def ok(r):
        return bound is None or r["err"] <= bound

    for r in stage1:
        r["admissible"] = ok(r)
    cand = [r for r in stage1 if r["admissible"]] or stage1
    b1 = min(cand, key=lambda r: r["ms_per_step"])
    stage2 = [run(b1["n_grp"], b1["n_leaf"], tj, w, 2)
              for tj in tiles for w in waves]
    for r in stage2:
        r["admissible"] = ok(r)
    cand = [r for r in stage2 if r["admissible"]] + [b1]
    best = min(cand, key=lambda r: r["ms_per_step"])
    return dict(workload=workload, n=int(d["x"].size),
                theta=p["theta"] if theta is None else theta, reuse=reuse,
                cycles=cycles, error_bound=bound,
                best=dict(n_grp=best["n_grp"], n_leaf=best["n_leaf"],
                          tile_j=best["tile_j"],
                          waves_per_simd=best["waves_per_simd"]),
                best_ms_per_step=best["ms_per_step"],
                results=stage1 + stage2)


def main(argv=None):
    import argparse
    import os
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    ap = argparse.ArgumentParser(description="n_grp / n_leaf / tile autotuner")
    ap.add_argument("--workload", default="disk_4m")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--n-grp", default="32,48,64,96,128,192,256,384,512")
    ap.add_argument("--n-leaf", default="8")
    ap.add_argument("--tile-j", default="64,128,192,256")
    ap.add_argument("--waves", default="4,6,8")
    ap.add_argument("--cycles", type=int, default=2)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    def ints(s):
        return [int(v) for v in s.split(",") if v]

    res = tune(a.workload, a.n, ints(a.n_grp), ints(a.n_leaf),
               ints(a.tile_j), ints(a.waves), a.cycles, theta=a.theta,
               log=lambda r: print(json.dumps(r), file=sys.stderr,
                                   flush=True))
    text = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text, flush=True)


if __name__ == "__main__":
    main()
