"""Autotuner for the group size n_grp and the leaf size n_leaf.

The paper picks the group size by hand from a sweep (its n_grp study);
here the sweep runs on the device the library will use: for every
candidate it times whole reuse cycles of the real step (construction step
plus reuse steps, inputs resident on the GPU) and keeps the fastest.  The
result is a small JSON record that ``bench.py --n-grp auto`` and users can
pass back as configuration.

  python -m paper_1907_02290_amd.tune --workload disk_4m [--n N]
         [--n-grp 32,64,128,256,512] [--n-leaf 8] [--cycles 2] [--out F]
"""
from __future__ import annotations

import json
import time

from . import nbody as nb


def time_config(d_dev, p, n_grp, n_leaf, reuse, cycles, offsets=None):
    """Mean ms per step over `cycles` reuse cycles after one warm-up cycle
    (construction step at the start of each cycle), and the interactions of
    the last construction step."""
    import torch
    dt = p["dt"]
    with nb.Context(theta=p["theta"], eps=p["eps"], n_leaf=n_leaf,
                    n_grp=n_grp, order=p["order"],
                    ext_mass=p.get("ext_mass", 0.0)) as ctx:
        ctx.set_particles(d_dev["x"], d_dev["y"], d_dev["z"], d_dev["vx"],
                          d_dev["vy"], d_dev["vz"], d_dev["m"])
        if offsets is not None:
            ctx.set_systems(offsets)
        ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)

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
    return ms, info


def tune(workload, n=None, n_grps=(32, 64, 128, 256, 512), n_leafs=(8,),
         cycles=2, reuse=None, log=None):
    import torch
    import workloads
    d, p = workloads.make(workload, n=n)
    reuse = reuse or p.get("reuse", 4)
    dev = {k: torch.from_numpy(d[k]).cuda()
           for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
    results = []
    for nl in n_leafs:
        for ng in n_grps:
            ms, info = time_config(dev, p, ng, nl, reuse, cycles,
                                   d.get("offsets"))
            r = dict(n_grp=ng, n_leaf=nl, ms_per_step=ms,
                     groups=info["n_groups"], interactions=info["n_inter"])
            if log:
                log(r)
            results.append(r)
    best = min(results, key=lambda r: r["ms_per_step"])
    return dict(workload=workload, n=int(d["x"].size), reuse=reuse,
                cycles=cycles, best=dict(n_grp=best["n_grp"],
                                         n_leaf=best["n_leaf"]),
                best_ms_per_step=best["ms_per_step"], results=results)


def main(argv=None):
    import argparse
    import os
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    ap = argparse.ArgumentParser(description="n_grp / n_leaf autotuner")
    ap.add_argument("--workload", default="disk_4m")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--n-grp", default="32,64,128,256,512")
    ap.add_argument("--n-leaf", default="8")
    ap.add_argument("--cycles", type=int, default=2)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = tune(a.workload, a.n, [int(v) for v in a.n_grp.split(",")],
               [int(v) for v in a.n_leaf.split(",")], a.cycles,
               log=lambda r: print(json.dumps(r), file=sys.stderr,
                                   flush=True))
    text = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text, flush=True)


if __name__ == "__main__":
    main()
