"""Seeded synthetic particle systems shared by the oracle tests, the GPU
tests and the benchmark.

This module holds initial-condition recipes only (no keys, trees, lists or
forces of the tree method).  Every array is FP64 and every generator takes an
explicit integer seed fed to numpy's PCG64.  The recipes and the readings
behind them are listed in the repository's design notes.

Systems
  plummer        Plummer sphere, radii by inverse mass CDF truncated at a
                 mass fraction, speeds by von Neumann rejection from the
                 isotropic distribution function (Aarseth, Henon & Wielen
                 1974).
  uniform_sphere cold uniform sphere (the paper's benchmark system,
                 section 6.1).
  disk_halo      exponential disk (sech^2 vertical profile) inside a
                 Hernquist halo; disk kinematics from the circular speed,
                 a Toomre-Q radial dispersion, the epicyclic ratio and an
                 isothermal-sheet vertical dispersion; halo speeds Gaussian
                 with the isotropic Jeans dispersion of the Hernquist model.
  ring           planetesimal ring on Keplerian orbits around a unit central
                 mass at the origin, Rayleigh-distributed e and i.
  king           King (1966) model with central potential W0: the
                 dimensionless Poisson equation integrated to the tidal
                 radius, radii from the enclosed mass, speeds by rejection
                 from the lowered-isothermal distribution function.
  clusters       many independent Plummer / King systems (separate trees).
"""
from __future__ import annotations

import functools

import numpy as np
from scipy import special

SEED_BASE = 0x1907022900000000


def seed_for(config: int, replicate: int = 0) -> int:
    """Seed of configuration ``config`` (1-based), replicate ``replicate``."""
    return SEED_BASE | (int(config) << 8) | int(replicate)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def _isotropic(rng, n):
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - cz * cz)
    return s * np.cos(ph), s * np.sin(ph), cz


def _pack(x, y, z, vx, vy, vz, m, recentre=True):
    out = dict(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, m=m)
    if recentre:
        M = m.sum()
        for a in ("x", "y", "z", "vx", "vy", "vz"):
            out[a] = out[a] - (m * out[a]).sum() / M
    return {k: np.ascontiguousarray(v, dtype=np.float64)
            for k, v in out.items()}


def plummer(n, seed, a=1.0, M=1.0, G=1.0, mcut=0.999):
    """Equal-mass Plummer sphere with scale ``a`` and mass ``M``."""
    rng = _rng(seed)
    X = rng.uniform(0.0, mcut, n)
    X = np.maximum(X, 1e-12)
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    ux, uy, uz = _isotropic(rng, n)
    # speed fraction q of the local escape speed, g(q) = q^2 (1-q^2)^3.5
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = rng.uniform(0.0, 1.0, todo.size)
        yy = rng.uniform(0.0, 0.1, todo.size)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0 * G * M / a) * (1.0 + (r / a) ** 2) ** (-0.25)
    v = q * vesc
    wx, wy, wz = _isotropic(rng, n)
    m = np.full(n, M / n)
    return _pack(r * ux, r * uy, r * uz, v * wx, v * wy, v * wz, m)


def uniform_sphere(n, seed, R=1.0, M=1.0):
    """Cold (v = 0) uniform sphere of radius ``R``."""
    rng = _rng(seed)
    r = R * rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    ux, uy, uz = _isotropic(rng, n)
    zero = np.zeros(n)
    return _pack(r * ux, r * uy, r * uz, zero, zero.copy(), zero.copy(),
                 np.full(n, M / n))


def _hernquist_sigma2(r, M, a, G):
    """Isotropic Jeans radial dispersion of the Hernquist model."""
    s = r / a
    t1 = 12.0 * s * (1.0 + s) ** 3 * np.log1p(1.0 / s)
    t2 = s / (1.0 + s) * (25.0 + 52.0 * s + 42.0 * s * s + 12.0 * s ** 3)
    return np.maximum(G * M / (12.0 * a) * (t1 - t2), 0.0)


def disk_halo(n_disk, n_halo, seed, R_d=1.0, z0=0.1, M_d=1.0, R_max=10.0,
              a_h=5.0, halo_over_disk=10.0, r_max=50.0, Q=1.5, G=1.0):
    """Exponential disk + Hernquist halo.  The halo particles carry
    ``halo_over_disk`` times the disk mass in total inside ``r_max``."""
    rng = _rng(seed)
    M_h_in = halo_over_disk * M_d
    frac = (r_max / (r_max + a_h)) ** 2        # Hernquist M(<r_max)/M
    M_H = M_h_in / frac                          # untruncated halo mass

    # --- halo positions (inverse CDF of M(r) = M r^2/(r+a)^2)
    u = rng.uniform(0.0, frac, n_halo)
    su = np.sqrt(u)
    rh = a_h * su / (1.0 - su)
    hx, hy, hz = _isotropic(rng, n_halo)
    sig = np.sqrt(_hernquist_sigma2(np.maximum(rh, 1e-8), M_H, a_h, G))
    vesc = np.sqrt(2.0 * G * M_H / (rh + a_h))
    hv = rng.normal(size=(3, n_halo)) * sig
    sp = np.sqrt((hv ** 2).sum(0))
    cap = 0.95 * vesc
    hv = np.where(sp > cap, hv * (cap / np.maximum(sp, 1e-300)), hv)

    # --- disk positions
    R = np.empty(n_disk)
    todo = np.arange(n_disk)
    while todo.size:
        rr = -R_d * np.log(rng.uniform(1e-300, 1.0, todo.size) *
                           rng.uniform(1e-300, 1.0, todo.size))
        ok = rr <= R_max
        R[todo[ok]] = rr[ok]
        todo = todo[~ok]
    ph = rng.uniform(0.0, 2.0 * np.pi, n_disk)
    zz = z0 * np.arctanh(rng.uniform(-1.0, 1.0, n_disk) * (1.0 - 1e-12))

    # --- disk kinematics on a radial grid
    Rg = np.geomspace(1e-4, R_max * 1.01, 4096)
    Sig0 = M_d / (2.0 * np.pi * R_d ** 2)
    yv = Rg / (2.0 * R_d)
    vd2 = 4.0 * np.pi * G * Sig0 * R_d * yv ** 2 * (
        special.i0(yv) * special.k0(yv) - special.i1(yv) * special.k1(yv))
    vh2 = G * M_H * Rg / (Rg + a_h) ** 2
    vc2 = np.maximum(vd2 + vh2, 0.0)
    Om2 = vc2 / Rg ** 2
    kap2 = np.gradient(Rg ** 2 * vc2, Rg) / Rg ** 3
    kap2 = np.maximum(kap2, 1e-12)
    Sig = Sig0 * np.exp(-Rg / R_d)
    sR = Q * 3.36 * G * Sig / np.sqrt(kap2)
    sP2 = sR ** 2 * kap2 / (4.0 * Om2)
    vphi2 = vc2 + sR ** 2 * (1.0 - kap2 / (4.0 * Om2) - 2.0 * Rg / R_d)
    vphi = np.sqrt(np.maximum(vphi2, 0.0))
    sZ = np.sqrt(np.pi * G * Sig * z0)
    i_R = lambda f: np.interp(R, Rg, f)
    vR = rng.normal(size=n_disk) * i_R(sR)
    vP = i_R(vphi) + rng.normal(size=n_disk) * np.sqrt(i_R(sP2))
    vZ = rng.normal(size=n_disk) * i_R(sZ)
    cph, sph = np.cos(ph), np.sin(ph)
    dx, dy = R * cph, R * sph
    dvx = vR * cph - vP * sph
    dvy = vR * sph + vP * cph

    x = np.concatenate([dx, rh * hx])
    y = np.concatenate([dy, rh * hy])
    z = np.concatenate([zz, rh * hz])
    vx = np.concatenate([dvx, hv[0]])
    vy = np.concatenate([dvy, hv[1]])
    vz = np.concatenate([vZ, hv[2]])
    m = np.concatenate([np.full(n_disk, M_d / n_disk),
                        np.full(n_halo, M_h_in / n_halo)])
    return _pack(x, y, z, vx, vy, vz, m)


def ring(n, seed, a_lo=0.9, a_hi=1.1, sigma_e=1e-3, sigma_i=1e-3,
         total_mass=1e-5, M_c=1.0, G=1.0):
    """Equal-mass planetesimal ring on Keplerian orbits around a fixed
    central mass ``M_c`` at the origin (not recentred)."""
    rng = _rng(seed)
    a = rng.uniform(a_lo, a_hi, n)
    e = np.minimum(rng.rayleigh(sigma_e, n), 0.5)
    inc = rng.rayleigh(sigma_i, n)
    Om = rng.uniform(0.0, 2.0 * np.pi, n)
    w = rng.uniform(0.0, 2.0 * np.pi, n)
    Mn = rng.uniform(0.0, 2.0 * np.pi, n)
    E = Mn.copy()
    for _ in range(30):  # Kepler's equation by Newton iterations
        E = E - (E - e * np.sin(E) - Mn) / (1.0 - e * np.cos(E))
    cE, sE = np.cos(E), np.sin(E)
    sq = np.sqrt(1.0 - e * e)
    nn = np.sqrt(G * M_c / a ** 3)
    xo = a * (cE - e)
    yo = a * sq * sE
    den = 1.0 - e * cE
    vxo = -a * nn * sE / den
    vyo = a * nn * sq * cE / den
    cw, sw = np.cos(w), np.sin(w)
    cO, sO = np.cos(Om), np.sin(Om)
    ci, si = np.cos(inc), np.sin(inc)
    # rotation R_z(Om) R_x(inc) R_z(w)
    r11 = cO * cw - sO * sw * ci
    r12 = -cO * sw - sO * cw * ci
    r21 = sO * cw + cO * sw * ci
    r22 = -sO * sw + cO * cw * ci
    r31 = sw * si
    r32 = cw * si
    x = r11 * xo + r12 * yo
    y = r21 * xo + r22 * yo
    z = r31 * xo + r32 * yo
    vx = r11 * vxo + r12 * vyo
    vy = r21 * vxo + r22 * vyo
    vz = r31 * vxo + r32 * vyo
    m = np.full(n, total_mass / n)
    return _pack(x, y, z, vx, vy, vz, m, recentre=False)


@functools.lru_cache(maxsize=8)
def _king_profile(W0):
    """Dimensionless King (1966) model: radius grid r (King radius 1),
    potential W(r) >= 0 and enclosed mass mu(r) = r^2 (-dW/dr), integrated
    out to the tidal radius where W = 0."""
    from scipy.integrate import solve_ivp
    from scipy.special import erf

    def rho(W):
        W = np.maximum(W, 0.0)
        return np.exp(W) * erf(np.sqrt(W)) - np.sqrt(4.0 * W / np.pi) * (
            1.0 + 2.0 * W / 3.0)

    rho0 = rho(np.array(W0))

    def rhs(r, y):
        W, dW = y
        return [dW, -9.0 * rho(np.array(W)) / rho0 - 2.0 * dW / r]

    def edge(r, y):
        return y[0]
    edge.terminal = True
    edge.direction = -1
    r0 = 1e-6
    sol = solve_ivp(rhs, (r0, 1e3), [W0 - 1.5 * r0 * r0, -3.0 * r0],
                    events=edge, max_step=0.01, rtol=1e-9, atol=1e-12,
                    dense_output=True)
    rt = sol.t_events[0][0]
    r = np.linspace(r0, rt, 20001)
    W, dW = sol.sol(r)
    return r, np.maximum(W, 0.0), r * r * (-dW)


def king(n, seed, W0=6.0, M=1.0, r0=1.0, G=1.0):
    """Equal-mass King model with central potential W0 and King radius r0:
    radii from the enclosed-mass profile, speeds by rejection from the
    lowered-isothermal distribution function f ~ exp(W - v^2/2) - 1."""
    rng = _rng(seed)
    r, W, mu = _king_profile(W0)
    mu_t = mu[-1]
    sigma = np.sqrt(G * M / (r0 * mu_t))       # velocity unit
    u = rng.uniform(0.0, mu_t, n)
    rad = np.interp(u, mu, r)
    Wr = np.interp(rad, r, W)
    ux, uy, uz = _isotropic(rng, n)
    v = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        w = Wr[todo]
        vmax = np.sqrt(2.0 * w)
        vv = rng.uniform(0.0, 1.0, todo.size) * vmax
        # bound of v^2 (e^(W - v^2/2) - 1) on [0, vmax]: below W e^W
        g = vv * vv * np.expm1(w - 0.5 * vv * vv)
        ok = rng.uniform(0.0, 1.0, todo.size) * (2.0 * w * np.exp(w) + 1e-300) < g
        v[todo[ok]] = vv[ok]
        todo = todo[~ok]
    wx, wy, wz = _isotropic(rng, n)
    m = np.full(n, M / n)
    return _pack(r0 * rad * ux, r0 * rad * uy, r0 * rad * uz,
                 sigma * v * wx, sigma * v * wy, sigma * v * wz, m)


def clusters(n_sys, seed, lo_exp=10, hi_exp=18):
    """Independent clusters: N_k = round(2^U), U ~ U[lo_exp, hi_exp]; each
    a Plummer or a King (W0 = 6) model by a fair coin, mass 1, scale 1.
    Returns the concatenated arrays and the system offsets."""
    rng = _rng(seed)
    sizes = np.round(2.0 ** rng.uniform(lo_exp, hi_exp, n_sys)).astype(int)
    kinds = rng.integers(0, 2, n_sys)
    parts = []
    for k in range(n_sys):
        sub = int(rng.integers(0, 2 ** 62))
        parts.append(plummer(int(sizes[k]), sub) if kinds[k] == 0 else
                     king(int(sizes[k]), sub))
    out = {key: np.concatenate([p[key] for p in parts]) for key in parts[0]}
    out["offsets"] = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    out["kinds"] = np.where(kinds == 0, "plummer", "king")
    return out


def near_faces(n, seed):
    """Tiny adversarial input for the key quantisation: a corner particle at
    a non-dyadic lo (about 0.1 per axis), one at lo + 0.9 (so the root side
    is 1), and n - 2 particles at lo + j/16 (j = 1..15 per axis) moved by
    -2..2 units in the last place.  The subtraction x - lo that gives a key
    rounds, so some of them land in a cell whose cube they lie just outside
    of.  Equal masses 1/n, zero velocities."""
    rng = _rng(seed)
    lo = 0.1 + rng.uniform(0.0, 1e-3, 3)
    pos = np.empty((3, n))
    pos[:, 0] = lo
    pos[:, 1] = lo + 0.9
    for a in range(3):
        v = lo[a] + rng.integers(1, 16, n - 2) / 16.0
        for i, k in enumerate(rng.integers(-2, 3, n - 2)):
            for _ in range(abs(int(k))):
                v[i] = np.nextafter(v[i], np.inf if k > 0 else -np.inf)
        pos[a, 2:] = v
    z = np.zeros(n)
    return dict(x=pos[0].copy(), y=pos[1].copy(), z=pos[2].copy(), vx=z,
                vy=z.copy(), vz=z.copy(), m=np.full(n, 1.0 / n))


# Named workloads: (generator, kwargs) plus run parameters.
def make(name, n=None, seed=None, replicate=0):
    """Build one of the named workloads.

    plummer_4k   Plummer N=4096 (eps 1/64, theta 0.5, monopole, leaf 8, n_grp 64)
    plummer_1m   Plummer N=2^20 (eps 1/256, dt 1/128)
    disk_4m      disk 2^21 + halo 2^21 (eps 0.01, theta 0.5, lists reused
                 every 4 steps, dt 1/128; n_grp 256, the fastest step of a
                 sweep over 32..1024 on MI355X)
    ring_8m      ring N=2^23 (eps 1e-4, dt 2 pi/256, central mass 1; n_grp
                 256, the autotuner's pick on MI355X: the thin ring's cells
                 of <= 64 particles hold 11 on average)
    clusters_64  64 independent Plummer / King(W0 = 6) clusters, N log-uniform
                 in [2^10, 2^18] (eps 0.01, dt 1/128)
    sphere_4m    cold uniform sphere N=2^22 (leaf 16)
    ``n`` overrides the particle count (same recipe, smaller system).
    """
    if name == "plummer_4k":
        nn = n or 4096
        s = seed if seed is not None else seed_for(1, replicate)
        return plummer(nn, s), dict(eps=1.0 / 64, theta=0.5, order=1,
                                    n_leaf=8, n_grp=64, dt=1.0 / 128)
    if name == "plummer_1m":
        nn = n or (1 << 20)
        s = seed if seed is not None else seed_for(2, replicate)
        return plummer(nn, s), dict(eps=1.0 / 256, theta=0.5, order=2,
                                    n_leaf=8, n_grp=64, dt=1.0 / 128)
    if name == "disk_4m":
        nn = n or (1 << 22)
        s = seed if seed is not None else seed_for(3, replicate)
        return disk_halo(nn // 2, nn - nn // 2, s), dict(
            eps=0.01, theta=0.5, order=1, n_leaf=8, n_grp=256, dt=1.0 / 128,
            reuse=4)
    if name == "ring_8m":
        nn = n or (1 << 23)
        s = seed if seed is not None else seed_for(4, replicate)
        return ring(nn, s), dict(eps=1e-4, theta=0.5, order=1, n_leaf=8,
                                 n_grp=256, dt=2.0 * np.pi / 256,
                                 ext_mass=1.0)
    if name == "clusters_64":
        s = seed if seed is not None else seed_for(5, replicate)
        return clusters(64, s), dict(eps=0.01, theta=0.5, order=1, n_leaf=8,
                                     n_grp=64, dt=1.0 / 128, reuse=4)
    if name == "sphere_4m":
        nn = n or (1 << 22)
        s = seed if seed is not None else seed_for(6, replicate)
        return uniform_sphere(nn, s), dict(eps=1.0 / 256, theta=0.5,
                                           order=1, n_leaf=16, n_grp=64,
                                           dt=1.0 / 128)
    raise KeyError(name)
