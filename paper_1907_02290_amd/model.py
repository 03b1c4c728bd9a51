"""Performance model of the step, refitted on the device the library runs on.

The paper models the force kernel (its appendix A) as

    T_kernel = n <n_list> (alpha_calc n_op / F + alpha_transfer (b_EPJ + b_ID)
                           / (<n_i> B))

with F the peak FP32 rate, B the device memory bandwidth, n_op = 23 flops
per interaction, b_EPJ = 32 bytes (FP64 position and mass) and b_ID = 4
bytes (one list index); on its GPU it found alpha_calc = 1.7 and
alpha_transfer = 2.7 by measuring the time per interaction against the mean
group size <n_i> at theta = 1, 0.5 and 0.25.  Every other part of its step
(section 6.2) is a bandwidth term, alpha times the bytes the part moves
divided by the bandwidth of the memory it runs from.

Here the whole step runs on one GPU, so every part is a term of the second
kind over device memory (B = 8 TB/s), and the kernel keeps the paper's two
terms (F = 157.3 TFLOP/s).  ``sweep`` measures the phases of whole steps
(construction every ``reuse`` steps) over a grid of theta and n_grp;
``fit`` finds alpha_calc and alpha_transfer by least squares in 1/<n_i> on
the time per interaction, and one alpha per phase from the calibration
points; ``predict`` gives the phase times and ms/step of any point from its
sizes (N, groups, interactions, list entries).

  python -m paper_1907_02290_amd.model --workload sphere_4m \
      [--thetas 0.25,0.5,1.0] [--n-grps 16,32,...] [--calibrate 0.5] [--out F]
"""
from __future__ import annotations

import json
import time

import numpy as np

# the paper's constants (force-model coefficient tables of section 6.2 and
# appendix A; size table of section 6.2)
N_OP = 23
B_EPJ = 32
B_ID = 4
PAPER_ALPHA_CALC = 1.7
PAPER_ALPHA_TRANSFER = 2.7

# MI355X published peaks
F_PEAK = 157.3e12      # FP32 vector flop/s
B_PEAK = 8.0e12        # HBM bytes/s

# Algorithmic bytes of the other phases, per particle of the step that runs
# them (construction phases once per reuse cycle); the walk per list entry
# (one index written).  Their alphas absorb latency and launch costs.
PHASE_BYTES = {
    "root": 24.0,      # x, y, z read for the bounding box
    "keys": 32.0,      # x, y, z read, key written
    "sort": 256.0,     # 8 radix passes over (key, index) pairs + histograms
    "reorder": 116.0,  # gather of position, velocity, mass, index
    "link": 8.0,       # sorted keys read
    "moments": 32.0,   # position and mass read (reuse steps too)
    "groups": 32.0,    # member positions read for the tight boxes
    "kick": 128.0,     # position, velocity, acceleration read; x, v written
}
CONSTRUCTION = ("root", "keys", "sort", "reorder", "link", "groups", "walk")
EVERY_STEP = ("moments", "force", "kick")


def n_list_model(n, n_i, theta):
    """The paper's estimate of the mean list length (section 6.2,
    equation for <n_list>)."""
    return (n_i + 14.0 * n_i ** (2.0 / 3.0) / theta
            + 21.0 * np.pi * n_i ** (1.0 / 3.0) / theta ** 2
            + 28.0 * np.pi / (3.0 * theta ** 3)
            * np.log2(theta / 2.8 * (n ** (1.0 / 3.0) - n_i ** (1.0 / 3.0))))


def kernel_time(n_inter, n_i, alpha_calc, alpha_transfer, F=F_PEAK,
                B=B_PEAK):
    """Force-kernel seconds for n_inter = n <n_list> interactions at mean
    group size n_i (appendix A)."""
    return n_inter * (alpha_calc * N_OP / F
                      + alpha_transfer * (B_EPJ + B_ID) / (n_i * B))


def fit_kernel(n_i, t_int, F=F_PEAK, B=B_PEAK):
    """alpha_calc, alpha_transfer from times per interaction t_int (s) at
    mean group sizes n_i: least squares of t_int = a + b / n_i weighted by
    1 / t_int (relative residuals)."""
    n_i = np.asarray(n_i, float)
    t = np.asarray(t_int, float)
    w = 1.0 / t
    A = np.stack([np.ones_like(n_i), 1.0 / n_i], axis=1) * w[:, None]
    (a, b), *_ = np.linalg.lstsq(A, t * w, rcond=None)
    return a * F / N_OP, b * B / (B_EPJ + B_ID)


def phase_bytes(point):
    """Bytes per step of every non-kernel phase of a measured point (a dict
    with n, reuse, n_epj, n_spj)."""
    n, reuse = point["n"], point["reuse"]
    out = {}
    for ph, b in PHASE_BYTES.items():
        per = n * b
        out[ph] = per / reuse if ph in CONSTRUCTION else per
    out["walk"] = (point["n_epj"] + point["n_spj"]) * B_ID / reuse
    return out


def fit(points, B=B_PEAK, F=F_PEAK):
    """Model coefficients from calibration points (see ``sweep``)."""
    a_calc, a_tr = fit_kernel([p["n_i"] for p in points],
                              [p["t_int"] for p in points], F, B)
    alphas = {}
    for ph in list(PHASE_BYTES) + ["walk"]:
        r = [p["phase_ms"][ph] * 1e-3 * B / phase_bytes(p)[ph]
             for p in points if phase_bytes(p)[ph] > 0]
        alphas[ph] = float(np.mean(r)) if r else 0.0
    return dict(alpha_calc=float(a_calc), alpha_transfer=float(a_tr),
                alpha=alphas, F=F, B=B)


def predict(point, coef):
    """Phase ms per step and total ms/step of a point from its sizes."""
    B = coef["B"]
    ms = {ph: coef["alpha"][ph] * x / B * 1e3
          for ph, x in phase_bytes(point).items()}
    ms["force"] = 1e3 * kernel_time(point["n_inter"], point["n_i"],
                                    coef["alpha_calc"],
                                    coef["alpha_transfer"], coef["F"], B)
    return ms, float(sum(ms.values()))


def measure(d_dev, p, theta, n_grp, reuse, cycles):
    """One point: whole steps (construction every `reuse` steps) timed by
    phase with HIP events, and wall ms per step."""
    import torch
    from . import nbody as nb
    dt = p["dt"]
    with nb.Context(theta=theta, eps=p["eps"], n_leaf=p["n_leaf"],
                    n_grp=n_grp, order=p["order"],
                    ext_mass=p.get("ext_mass", 0.0), timing=True) as ctx:
        ctx.set_particles(d_dev["x"], d_dev["y"], d_dev["z"], d_dev["vx"],
                          d_dev["vy"], d_dev["vz"], d_dev["m"])
        ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)

        def cycle():
            for s in range(reuse):
                ctx.step(nb.NB_REUSE_LIST if s else nb.NB_MAKE_LIST_FOR_REUSE,
                         dt, dt)

        cycle()
        torch.cuda.synchronize()
        ctx.get_timing(reset=True)
        t0 = time.perf_counter()
        for _ in range(cycles):
            cycle()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / (cycles * reuse)
        timing = ctx.get_timing(reset=True)
        info = ctx.get_info()
    steps = cycles * reuse
    phase_ms = {k: v[0] / steps for k, v in timing.items()
                if k in PHASE_BYTES or k in ("walk", "force")}
    f_ms, f_calls = timing["force"]
    n = int(info["n"])
    return dict(theta=theta, n_grp=n_grp, n=n, reuse=reuse,
                n_groups=int(info["n_groups"]),
                n_i=n / info["n_groups"], n_inter=int(info["n_inter"]),
                n_list=info["n_inter"] / n, n_epj=int(info["n_epj"]),
                n_spj=int(info["n_spj"]),
                n_list_model=float(n_list_model(n, n / info["n_groups"],
                                                theta)),
                t_int=f_ms * 1e-3 / f_calls / info["n_inter"],
                force_ms=f_ms / f_calls, phase_ms=phase_ms,
                ms_per_step=wall)


def sweep(workload, thetas, n_grps, n=None, reuse=4, cycles=2, log=None):
    import torch
    import workloads
    d, p = workloads.make(workload, n=n)
    dev = {k: torch.from_numpy(d[k]).cuda()
           for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
    out = []
    for theta in thetas:
        for ng in n_grps:
            r = measure(dev, p, theta, ng, reuse, cycles)
            if log:
                log(r)
            out.append(r)
    return out


def main(argv=None):
    import argparse
    import os
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    ap = argparse.ArgumentParser(description="step model refit")
    ap.add_argument("--workload", default="sphere_4m")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--thetas", default="0.25,0.5,1.0")
    ap.add_argument("--n-grps", default="32,64,128,256,512,1024")
    ap.add_argument("--calibrate", type=float, default=0.5,
                    help="theta of the calibration points; the others are "
                         "predicted")
    ap.add_argument("--reuse", type=int, default=4)
    ap.add_argument("--cycles", type=int, default=2)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    thetas = [float(v) for v in a.thetas.split(",")]
    n_grps = [int(v) for v in a.n_grps.split(",")]
    pts = sweep(a.workload, thetas, n_grps, a.n, a.reuse, a.cycles,
                log=lambda r: print(json.dumps(r), file=sys.stderr,
                                    flush=True))
    cal = [q for q in pts if abs(q["theta"] - a.calibrate) < 1e-12]
    coef = fit(cal)
    kall = fit_kernel([q["n_i"] for q in pts], [q["t_int"] for q in pts])
    rows = []
    for q in pts:
        ms, total = predict(q, coef)
        rows.append(dict(theta=q["theta"], n_grp=q["n_grp"], n_i=q["n_i"],
                         n_list=q["n_list"], n_list_model=q["n_list_model"],
                         t_int_ns=q["t_int"] * 1e9,
                         force_ms=q["force_ms"],
                         force_ms_model=1e3 * kernel_time(
                             q["n_inter"], q["n_i"], coef["alpha_calc"],
                             coef["alpha_transfer"]),
                         phases_ms=sum(q["phase_ms"].values()),
                         ms_per_step=q["ms_per_step"],
                         ms_per_step_model=total,
                         calibration=q in cal))
    res = dict(workload=a.workload, coef=coef,
               kernel_fit_all_thetas=dict(alpha_calc=kall[0],
                                          alpha_transfer=kall[1]),
               paper=dict(alpha_calc=PAPER_ALPHA_CALC,
                          alpha_transfer=PAPER_ALPHA_TRANSFER),
               points=rows)
    text = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text, flush=True)


if __name__ == "__main__":
    main()
