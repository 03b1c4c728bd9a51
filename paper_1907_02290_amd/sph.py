"""Timing of the short-range path: neighbour lists (the group walk with the
short-range opening rule, section 2) and SPH densities on them, reused over
several evaluations (section 4.2).

For a workload of N particles the smoothing length h is chosen so that a
uniform ball of unit radius would hold ``--neighbours`` particles within h;
the lists are built for h (1 + skin).  The tool builds the tree and the
lists once, evaluates the density ``--evals`` times, and reports the list
and density times from the library's HIP-event timers and the candidate
pairs per evaluation (sum over groups of members x list length).  The
FP64 CPU timing of the same lists and densities is a leg of the repository's
benchmark script (``bench.py --sph``), which is allowed to run the oracle;
this module never loads it.

  python -m paper_1907_02290_amd.sph --workload sphere_4m [--neighbours 64]
         [--skin 0.3] [--evals 20]
"""
from __future__ import annotations

import json
import time

import numpy as np


def smoothing_length(n, neighbours):
    """h such that a uniform ball of unit radius and n particles holds
    `neighbours` of them within h: n h^3 = neighbours."""
    return (neighbours / n) ** (1.0 / 3.0)


def measure(workload, n=None, neighbours=64, skin=0.3, evals=20, n_grp=None,
            n_leaf=None):
    import torch
    import workloads
    from . import nbody as nb
    d, p = workloads.make(workload, n=n)
    n = int(d["x"].size)
    h = smoothing_length(n, neighbours)
    dev = {k: torch.from_numpy(d[k]).cuda()
           for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
    n_grp = n_grp or p["n_grp"]
    n_leaf = n_leaf or p["n_leaf"]
    with nb.Context(theta=p["theta"], eps=p["eps"], n_leaf=n_leaf,
                    n_grp=n_grp, timing=True) as ctx:
        ctx.set_particles(dev["x"], dev["y"], dev["z"], dev["vx"],
                          dev["vy"], dev["vz"], dev["m"])
        ctx.build_tree()
        ctx.neighbour_lists(h * (1 + skin))     # warm-up
        ctx.sph_density(h)
        torch.cuda.synchronize()
        ctx.get_timing(reset=True)
        ctx.neighbour_lists(h * (1 + skin))
        torch.cuda.synchronize()
        t_list = ctx.get_timing(reset=True)["walk"]
        t0 = time.perf_counter()
        for _ in range(evals):
            ctx.sph_density(h)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / evals
        t_rho = ctx.get_timing(reset=True)["force"]
        off, ids = ctx.get_neighbour_lists()
        g = ctx.get_groups()
        rho = ctx.get_density()
    count = g["count"].astype(np.int64)
    pairs = int((count * np.diff(off)).sum())
    return dict(workload=workload, n=n, h=h, skin=skin, n_grp=n_grp,
                n_leaf=n_leaf, neighbours_target=neighbours,
                n_groups=int(count.size),
                list_entries=int(off[-1]), pairs_per_eval=pairs,
                list_ms=t_list[0], density_ms=t_rho[0] / t_rho[1],
                density_wall_ms=wall,
                pairs_per_s=pairs / (t_rho[0] / t_rho[1] * 1e-3),
                mean_rho=float(rho.mean()))


def main(argv=None):
    import argparse
    import os
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    ap = argparse.ArgumentParser(description="short-range path timing")
    ap.add_argument("--workload", default="sphere_4m")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--neighbours", type=float, default=64)
    ap.add_argument("--skin", type=float, default=0.3)
    ap.add_argument("--evals", type=int, default=20)
    ap.add_argument("--n-grp", default=None,
                    help="group sizes to try, comma-separated (default: the "
                         "workload's)")
    ap.add_argument("--n-leaf", default=None,
                    help="leaf sizes to try, comma-separated")
    a = ap.parse_args(argv)
    grps = [int(v) for v in a.n_grp.split(",")] if a.n_grp else [None]
    leafs = [int(v) for v in a.n_leaf.split(",")] if a.n_leaf else [None]
    for nl in leafs:
        for ng in grps:
            res = measure(a.workload, a.n, a.neighbours, a.skin, a.evals, ng,
                          nl)
            print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
