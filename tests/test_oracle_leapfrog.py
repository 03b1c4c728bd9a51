"""Pins of the oracle's kick-drift (KDK leapfrog) and reuse steps: Kepler
orbit closure with second-order energy error, dt^2 energy scaling of an
N-body run, and time reversibility with frozen lists (section 4.2)."""
import numpy as np
import pytest


def _kepler_run(orc, dt, n_steps, e=0.5):
    # one test particle around a fixed unit mass, apocentre start
    a = 1.0
    ra = a * (1 + e)
    va = np.sqrt((1 - e) / ra)
    pos = [np.array([ra]), np.array([0.0]), np.array([0.0])]
    vel = [np.array([0.0]), np.array([va]), np.array([0.0])]
    zero = [np.zeros(1)] * 3

    def energy():
        r = np.sqrt(pos[0] ** 2 + pos[1] ** 2 + pos[2] ** 2)[0]
        v2 = (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)[0]
        return 0.5 * v2 - 1.0 / r

    e0 = energy()
    # KDK with merged half kicks: the pull of the central mass is applied by
    # kick_drift itself (acceleration argument zero)
    orc.kick_drift(pos, vel, zero, dt / 2, dt, ext_mass=1.0)
    emax = 0.0
    for s in range(1, n_steps):
        orc.kick_drift(pos, vel, zero, dt, dt, ext_mass=1.0)
        # synchronise a copy for the energy check
        p2 = [p.copy() for p in pos]
        v2 = [v.copy() for v in vel]
        orc.kick_drift(p2, v2, zero, dt / 2, 0.0, ext_mass=1.0)
        r = np.sqrt(p2[0] ** 2 + p2[1] ** 2 + p2[2] ** 2)[0]
        en = 0.5 * (v2[0] ** 2 + v2[1] ** 2 + v2[2] ** 2)[0] - 1.0 / r
        emax = max(emax, abs(en - e0))
    orc.kick_drift(pos, vel, zero, dt / 2, 0.0, ext_mass=1.0)
    return pos, vel, abs(energy() - e0), emax


def test_kepler_orbit_closes_second_order(orc):
    period = 2 * np.pi
    res = []
    for nsteps in (2000, 4000):
        dt = period / nsteps
        pos, vel, de_end, de_max = _kepler_run(orc, dt, nsteps)
        res.append((pos, de_max))
        # back near the apocentre after one period
        assert abs(pos[0][0] - 1.5) < 1e-3 and abs(pos[1][0]) < 2e-2
    ratio = res[0][1] / res[1][1]
    assert 3.5 < ratio < 4.5, ratio


def _nbody_energy_error(orc, dt, t_end, x, y, z, vx, vy, vz, m, eps):
    pos = [x.copy(), y.copy(), z.copy()]
    vel = [vx.copy(), vy.copy(), vz.copy()]

    def acc():
        ax, ay, az, pot = orc.force_direct(*pos, m, eps, 1.0)
        return [ax, ay, az], pot

    def energy(pot):
        v2 = vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2
        return (0.5 * m * v2).sum() + 0.5 * (m * pot).sum()

    a, pot = acc()
    e0 = energy(pot)
    n = int(round(t_end / dt))
    for s in range(n):
        orc.kick_drift(pos, vel, a, dt / 2, dt)
        a, pot = acc()
        orc.kick_drift(pos, vel, a, dt / 2, 0.0)
    return abs(energy(pot) - e0) / abs(e0)


def test_nbody_energy_error_scales_as_dt_squared(orc):
    import workloads
    d = workloads.plummer(128, 77)
    args = (d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["m"], 0.05)
    e1 = _nbody_energy_error(orc, 1 / 32, 1.0, *args)
    e2 = _nbody_energy_error(orc, 1 / 64, 1.0, *args)
    assert e1 < 1e-3
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)


def test_time_reversal_with_frozen_lists(orc):
    import workloads
    d = workloads.plummer(1024, 5)
    m = d["m"]
    pos = [d["x"].copy(), d["y"].copy(), d["z"].copy()]
    vel = [d["vx"].copy(), d["vy"].copy(), d["vz"].copy()]
    t = orc.Tree(*pos, m, n_leaf=8, n_grp=32)
    t.make_lists(0.5)
    dt, eps = 1 / 128, 1 / 64

    def acc():
        t.refresh(*pos, m)
        f = t.force_lists(2, eps, 1.0)
        return list(f[:3])

    a = acc()
    for sgn in (1, -1):
        if sgn < 0:
            for v in vel:
                v *= -1.0
        for s in range(20):
            orc.kick_drift(pos, vel, a, dt / 2, dt)
            a = acc()
            orc.kick_drift(pos, vel, a, dt / 2, 0.0)
    for p, p0 in zip(pos, (d["x"], d["y"], d["z"])):
        np.testing.assert_allclose(p, p0, rtol=0, atol=1e-12)


def test_kick_drift_order(orc):
    pos = [np.array([1.0]), np.array([0.0]), np.array([0.0])]
    vel = [np.array([0.0]), np.array([2.0]), np.array([0.0])]
    acc = [np.array([-3.0]), np.array([0.0]), np.array([1.0])]
    orc.kick_drift(pos, vel, acc, 0.5, 0.25)
    # kick first: v = (-1.5, 2, 0.5); then drift with the new v
    assert [v[0] for v in vel] == [-1.5, 2.0, 0.5]
    assert [p[0] for p in pos] == [1.0 - 0.375, 0.5, 0.125]
