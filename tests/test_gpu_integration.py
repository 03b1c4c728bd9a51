"""Integration run on the 2^20-particle Plummer workload (quadrupole
superparticles, eps 1/256): one force evaluation per opening angle checked
against the oracle's FP64 direct sum on a sample of particles, then ten KDK
leapfrog steps of dt = 1/128 with lists rebuilt every 4 steps and the energy
compared before and after (velocities synchronised by a closing half
kick)."""
import numpy as np
import pytest

import oracle
import workloads
import paper_1907_02290_amd as nb

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _energy(ctx, m):
    x, y, z, vx, vy, vz = ctx.get_state()
    _, _, _, pot = ctx.get_forces()
    return 0.5 * np.sum(m * (vx * vx + vy * vy + vz * vz)) + \
        0.5 * np.sum(m * pot)


@pytest.fixture(scope="module")
def plummer():
    return workloads.make("plummer_1m")


def test_force_error_grows_with_theta_and_energy_is_kept(plummer):
    d, p = plummer
    n = d["x"].size
    rng = np.random.default_rng(20)
    sample = np.sort(rng.choice(n, 256, replace=False))
    ref = oracle.force_direct(d["x"], d["y"], d["z"], d["m"], p["eps"], 1.0,
                              sample)
    med = {}
    dt = p["dt"]
    for theta in (0.3, 0.5, 0.7):
        say("case plummer 2^20 theta=%.1f" % theta)
        with nb.Context(theta=theta, eps=p["eps"], n_leaf=p["n_leaf"],
                        n_grp=p["n_grp"], order=p["order"]) as ctx:
            ctx.set_particles(d["x"], d["y"], d["z"], d["vx"], d["vy"],
                              d["vz"], d["m"])
            ctx.compute_forces(nb.NB_MAKE_LIST_FOR_REUSE)
            ax, ay, az, pot = ctx.get_forces()
            num = np.sqrt((ax[sample] - ref[0]) ** 2 + (ay[sample] - ref[1]) ** 2
                          + (az[sample] - ref[2]) ** 2)
            den = np.sqrt(ref[0] ** 2 + ref[1] ** 2 + ref[2] ** 2)
            err = num / den
            med[theta] = float(np.median(err))
            e0 = _energy(ctx, d["m"])
            for s in range(1, 11):
                mode = nb.NB_MAKE_LIST_FOR_REUSE if s % 4 == 0 else \
                    nb.NB_REUSE_LIST
                ctx.step(mode, dt / 2 if s == 1 else dt, dt)
            ctx.kick_drift(dt / 2, 0.0)
            e1 = _energy(ctx, d["m"])
            de = abs(e1 - e0) / abs(e0)
            say("  force err vs direct: median %.2e p99 %.2e; |dE/E| over "
                "10 steps %.2e" % (med[theta], np.percentile(err, 99), de))
            assert de < 5e-4
    assert med[0.3] < med[0.5] < med[0.7]
    assert med[0.5] < 2e-3
