"""Seeded synthetic workloads: grids, physical parameters and initial states.

This module holds only input generation (grid shapes, parameter sets and
initial fields); none of the scheme's arithmetic lives here.  It is shared by
the GPU package's tests/benchmark and by the oracle-side tests, which is why it
depends on numpy only.

Shapes and parameters follow the paper's experiments (sec. 8: capillary wave,
rising droplet, Rayleigh-Taylor), scaled to the workloads named below.  Fluid 1
is the phase c = 1 (its density is rho1, sec. 2.1).

Field arrays have shape (m2, m1): row j, column i.  u[j, i] is the x-velocity
on the west face of cell (i, j); v[j, i] the y-velocity on its south face.
"""
import math

import numpy as np

WALL, PERIODIC = 0, 1


def eta_of(rho1, rho2):
    """Interface ratio parameter of sec. 8.1 (sharp-interface matching) for
    the density pair; the equal-density limit of the same expression is
    3/(2 sqrt 2 rho1)."""
    if abs(rho2 - rho1) < 1e-6 * rho1:
        return 3.0 / (2.0 * math.sqrt(2.0) * rho1)
    d = rho2 - rho1
    return d ** 3 / (2.0 * math.sqrt(2.0) * rho1 * rho2 * (rho2 ** 2 - rho1 ** 2 - 2.0 * rho1 * rho2 * math.log(rho2 / rho1)))


def splitmix64(seed, n):
    """n uniform doubles in [0,1) from the SplitMix64 generator (Steele, Lea,
    Flood 2014), top 53 bits of each output."""
    out = np.empty(n, dtype=np.float64)
    mask = (1 << 64) - 1
    s = seed & mask
    for k in range(n):
        s = (s + 0x9E3779B97F4A7C15) & mask
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        z = z ^ (z >> 31)
        out[k] = (z >> 11) * (1.0 / 9007199254740992.0)
    return out


def _centres(m1, m2, h):
    x = (np.arange(m1) + 0.5) * h
    y = (np.arange(m2) + 0.5) * h
    return np.meshgrid(x, y)  # (m2, m1)


SMOOTH_SEGREGATED, SMOOTH_COUPLED = 0, 1
PRIMITIVE, PROJECTION = 0, 1


def default_opts(tol=1e-10):
    return dict(tol=tol, max_vcycles=50, nu1=2, nu2=2, nu_coarse=0, vanka_omega=1.0, smoother=SMOOTH_COUPLED,
                coarse_omega=0.0, accel=2, blocking=1)


def params(rho1, rho2, visc1, visc2, Re, We, inv_Fr, eps, M=None, Pe=None, eta=None, mob_reg=None, rho_ref=0.0):
    return dict(rho1=rho1, rho2=rho2, visc1=visc1, visc2=visc2, Re=Re, We=We, inv_Fr=inv_Fr,
                Pe=(1.0 / eps) if Pe is None else Pe, M=eps if M is None else M, eps=eps,
                eta=eta_of(rho1, rho2) if eta is None else eta,
                mob_reg=eps if mob_reg is None else mob_reg, rho_ref=rho_ref)


def capillary(m1=32, m2=64, eps=0.02, levels=4):
    """Capillary wave on [0,1]x[0,2], periodic in x, walls in y; interface at
    y = 1 + 0.01 cos(2 pi x) with fluid 1 (c = 1) above; no gravity."""
    h = 1.0 / m1
    grid = dict(m1=m1, m2=m2, Lx=1.0, Ly=m2 * h, bcx=PERIODIC, bcy=WALL, levels=levels)
    par = params(1.0, 3.0, 1.0, 1.0, Re=100.0, We=100.0, inv_Fr=0.0, eps=eps)
    X, Y = _centres(m1, m2, h)
    c = 0.5 * (1.0 + np.tanh((Y - 1.0 - 0.01 * np.cos(2 * np.pi * X)) / (2.0 * math.sqrt(2.0) * eps)))
    return dict(name="capillary_%dx%d" % (m1, m2), grid=grid, params=par, dt=1e-3, state=dict(c=c))


def rising_drop(m1=256, m2=512, eps=0.01, levels=0, radius=0.25, rho_ratio=10.0, visc_ratio=10.0,
                Re=35.0, We=10.0, inv_Fr=1.0, dt=5e-4):
    """Light drop (fluid 1, c = 1) of the given radius centred at (0.5, 0.5)
    in [0,1]x[0,2] with walls on all sides and gravity along -y."""
    h = 1.0 / m1
    grid = dict(m1=m1, m2=m2, Lx=1.0, Ly=m2 * h, bcx=WALL, bcy=WALL, levels=levels)
    par = params(1.0, rho_ratio, 1.0, visc_ratio, Re=Re, We=We, inv_Fr=inv_Fr, eps=eps)
    X, Y = _centres(m1, m2, h)
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2)
    c = 0.5 * (1.0 - np.tanh((r - radius) / (2.0 * math.sqrt(2.0) * eps)))
    return dict(name="rising_drop_%dx%d" % (m1, m2), grid=grid, params=par, dt=dt, state=dict(c=c))


def rayleigh_taylor(m1=512, m2=2048, eps=0.005, levels=0, seed=1703, noise=1e-3):
    """Heavy fluid (c = 0, rho2 = 3) above light fluid (c = 1, rho1 = 1) in
    [0,1]x[0,4], periodic in x, walls in y, interface y = 2 + 0.1 cos(2 pi x)
    plus seeded uniform noise of the given amplitude on c."""
    h = 1.0 / m1
    grid = dict(m1=m1, m2=m2, Lx=1.0, Ly=m2 * h, bcx=PERIODIC, bcy=WALL, levels=levels)
    par = params(1.0, 3.0, 1.0, 1.0, Re=3000.0, We=200.0, inv_Fr=1.0, eps=eps)
    X, Y = _centres(m1, m2, h)
    c = 0.5 * (1.0 - np.tanh((Y - 2.0 - 0.1 * np.cos(2 * np.pi * X)) / (2.0 * math.sqrt(2.0) * eps)))
    xi = (splitmix64(seed, m1 * m2).reshape(m2, m1) * 2.0 - 1.0) * noise
    return dict(name="rayleigh_taylor_%dx%d" % (m1, m2), grid=grid, params=par, dt=2.5e-4, state=dict(c=c + xi))


def random_state(grid, seed, amp=(0.05, 0.1, 0.1, 0.2, 0.2), base_c=0.5):
    """Smooth-ish random state (c, mu, p, u, v) for operator and identity tests:
    c = base_c + noise, the rest zero-mean noise, wall faces zeroed."""
    rng = np.random.default_rng(seed)
    m1, m2 = grid["m1"], grid["m2"]
    st = {}
    for k, (name, a) in enumerate(zip(("c", "mu", "p", "u", "v"), amp)):
        f = rng.uniform(-a, a, size=(m2, m1))
        if name == "c":
            f = f + base_c
        st[name] = f
    if grid["bcx"] == WALL:
        st["u"][:, 0] = 0.0
    if grid["bcy"] == WALL:
        st["v"][0, :] = 0.0
    return st


def serving_requests(n=64, rate_hz=20.0, seed=6606, nsteps=50, dt=5e-4,
                     sizes=((64, 128), (128, 256), (256, 512), (512, 1024))):
    """Independent rising-droplet requests arriving as a seeded Poisson stream:
    grid drawn uniformly from sizes on [0,1]x[0,2] (walls), drop radius
    U[0.15, 0.3], density ratio U[2, 20], viscosity ratio U[1, 10], Re = 35,
    We = 10, 1/Fr = 1, eps = 2.56 h (the interface resolution of the 256x512
    droplet), nsteps steps of dt each.  Returns a list of dicts with the
    arrival time (s) and a workload."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += rng.exponential(1.0 / rate_hz)
        m1, m2 = sizes[rng.integers(len(sizes))]
        radius = rng.uniform(0.15, 0.3)
        rr = rng.uniform(2.0, 20.0)
        vr = rng.uniform(1.0, 10.0)
        eps = 2.56 / m1
        w = rising_drop(m1, m2, eps=eps, radius=radius, rho_ratio=rr, visc_ratio=vr, dt=dt)
        w["name"] = "request_%d_%dx%d" % (k, m1, m2)
        out.append(dict(arrival=t, work=w, nsteps=nsteps))
    return out


def _periodic_drops(m, ndrops, r_lo, r_hi, eps, rng):
    """c on an m x m periodic unit box: the maximum over ndrops circular drops
    (fluid 1) of the tanh profile, radii U[r_lo, r_hi], centres uniform,
    accepted only if the periodic distance to every earlier drop is at least
    the sum of the radii plus 4 eps"""
    centres, radii = [], []
    while len(centres) < ndrops:
        x, y, R = rng.uniform(), rng.uniform(), rng.uniform(r_lo, r_hi)
        ok = True
        for (a, b), Rb in zip(centres, radii):
            dx = min(abs(x - a), 1 - abs(x - a))
            dy = min(abs(y - b), 1 - abs(y - b))
            if math.hypot(dx, dy) < R + Rb + 4 * eps:
                ok = False
                break
        if ok:
            centres.append((x, y))
            radii.append(R)
    # each profile is evaluated within R + 30 eps of its centre (beyond that it
    # is below 1e-9 and taken as 0)
    h = 1.0 / m
    c = np.zeros((m, m))
    for (a, b), R in zip(centres, radii):
        w = int(math.ceil((R + 30 * eps) / h)) + 1
        ia = int(a / h)
        jb = int(b / h)
        ii = np.arange(ia - w, ia + w + 1) if 2 * w + 1 < m else np.arange(m)
        jj = np.arange(jb - w, jb + w + 1) if 2 * w + 1 < m else np.arange(m)
        xi, yj = (ii + 0.5) * h, (jj + 0.5) * h
        dx = np.abs(xi - a)
        dx = np.minimum(dx % 1.0, 1 - dx % 1.0)
        dy = np.abs(yj - b)
        dy = np.minimum(dy % 1.0, 1 - dy % 1.0)
        r = np.sqrt(dx[None, :] ** 2 + dy[:, None] ** 2)
        prof = 0.5 * (1.0 - np.tanh((r - R) / (2.0 * math.sqrt(2.0) * eps)))
        sub = np.ix_(jj % m, ii % m)
        c[sub] = np.maximum(c[sub], prof)
    return c


def drops_box(m, ndrops, r_lo, r_hi, eps, seed, rho_ratio=100.0, visc_ratio=50.0, Re=500.0, We=50.0,
              inv_Fr=1.0, dt=1e-4):
    """Light drops (fluid 1, c = 1) in a heavy fluid on the periodic unit box
    (seeded rejection sampling, see _periodic_drops); gravity along -y in
    buoyancy form: the force is measured against the mean density of the box,
    which the scheme conserves, so that a fully periodic box has no net body
    force."""
    grid = dict(m1=m, m2=m, Lx=1.0, Ly=1.0, bcx=PERIODIC, bcy=PERIODIC, levels=0)
    c = _periodic_drops(m, ndrops, r_lo, r_hi, eps, np.random.default_rng(seed))
    par = params(1.0, rho_ratio, 1.0, visc_ratio, Re=Re, We=We, inv_Fr=inv_Fr, eps=eps)
    rho = par["rho1"] * par["rho2"] / ((par["rho2"] - par["rho1"]) * c + par["rho1"])
    par["rho_ref"] = float(rho.mean())
    return dict(name="drops_box_%dx%d_%d" % (m, m, ndrops), grid=grid, params=par, dt=dt, state=dict(c=c))


def serving_at_scale(nbig=16, big=2048, nsteps=20, bg_rate_hz=20.0, bg_size=256, duration_s=None, seed_bg=6607):
    """nbig periodic boxes of big x big cells with 40 drops each (R U[0.02,
    0.05], eps = 0.002, seeds 1000 + k) submitted at time 0, and a background
    Poisson stream of bg_size x bg_size boxes with 5 drops (R U[0.05, 0.1],
    eps = 0.01) at bg_rate_hz; all nsteps steps of dt = 1e-4, density ratio
    100, viscosity ratio 50, Re = 500, We = 50, 1/Fr = 1.  Background arrivals
    cover duration_s seconds (None: the caller stops submitting when the big
    runs are done).  Returns (big requests, background request generator)."""
    bigs = [dict(arrival=0.0, work=drops_box(big, 40, 0.02, 0.05, 0.002, 1000 + k), nsteps=nsteps)
            for k in range(nbig)]
    for k, r in enumerate(bigs):
        r["work"]["name"] = "box_%d_%dx%d" % (k, big, big)

    def background():
        rng = np.random.default_rng(seed_bg)
        t, k = 0.0, 0
        while duration_s is None or t < duration_s:
            t += rng.exponential(1.0 / bg_rate_hz)
            w = drops_box(bg_size, 5, 0.05, 0.1, 0.01, int(rng.integers(1 << 30)))
            w["name"] = "bg_%d_%dx%d" % (k, bg_size, bg_size)
            yield dict(arrival=t, work=w, nsteps=nsteps)
            k += 1

    return bigs, background()


def convergence_case(m, amp=0.2, eps=0.1, T=0.25, rho_ratio=3.0, visc_ratio=3.0):
    """Cauchy convergence study of sec. 9 on the unit square with walls:
    c = 0.5 + amp (cos 2 pi x + cos 2 pi y) (bounded away from the density
    pole, unlike the printed cos 2 pi x + cos 2 pi y), everything else zero,
    density and viscosity ratios 3 (the paper does not state them), Re = We =
    10, gravity 1/Fr = 1, M = eps, Pe = 1/eps; time step dt = (1/16)(16/m)^2 as
    in the printed schedule, run to time T."""
    h = 1.0 / m
    grid = dict(m1=m, m2=m, Lx=1.0, Ly=1.0, bcx=WALL, bcy=WALL, levels=0)
    par = params(1.0, rho_ratio, 1.0, visc_ratio, Re=10.0, We=10.0, inv_Fr=1.0, eps=eps)
    X, Y = _centres(m, m, h)
    c = 0.5 + amp * (np.cos(2 * np.pi * X) + np.cos(2 * np.pi * Y))
    dt = (1.0 / 16.0) * (16.0 / m) ** 2
    return dict(name="convergence_%dx%d" % (m, m), grid=grid, params=par, dt=dt, nsteps=int(round(T / dt)),
                state=dict(c=c))
