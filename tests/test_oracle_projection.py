"""Pins of the oracle's projection scheme (sec. 6.2, eqs. (pj-num-mx)-
(pj-num-chem); smoother of sec. 7.2) against what the paper and mathematics
fix: the discrete mass and energy theorems of sec. 6.2, the pointwise
continuity identity behind the mass theorem, a hydrostatic closed form, the
root of a dense Newton solve of the same system, and the exactness of the
pressure step of the smoother.

Reading pinned here: gravity acts in the projection equation (as in the
time-discrete scheme (pj-pj)) and not in the intermediate momentum equation;
with it the energy identity of the theorem of sec. 6.2 holds to round-off,
with it in the momentum equation it would miss the work of gravity on
u^{n+1} - u~.
"""
import numpy as np
import pytest

import oracle as OR
from paper_1703_06606_amd import workloads as W

FIELDS = ("c", "mu", "p", "u", "v")


def pj(tol=1e-10, **kw):
    return dict(W.default_opts(tol), scheme=W.PROJECTION, **kw)


def grid_(m1, m2, bcx, bcy, levels=0, L=1.0):
    return dict(m1=m1, m2=m2, Lx=L, Ly=L * m2 / m1, bcx=bcx, bcy=bcy, levels=levels)


def par_O1(**kw):
    p = dict(rho1=1.0, rho2=2.5, visc1=1.0, visc2=1.8, Re=3.0, We=2.0, inv_Fr=0.7, Pe=2.0, M=0.8,
             eps=0.5, eta=0.9, mob_reg=0.05, rho_ref=0.0)
    p.update(kw)
    return p


def _periodic_drop():
    c = W.rising_drop(32, 32, eps=0.04)
    c["grid"] = grid_(32, 32, 1, 1)
    c["params"] = dict(c["params"], inv_Fr=0.0)
    return c


CASES = {
    "capillary": W.capillary,
    "drop_gravity": lambda: W.rising_drop(32, 64, eps=0.04),
    "periodic": _periodic_drop,
}


@pytest.mark.parametrize("name", list(CASES))
def test_projection_mass_and_energy_law(name):
    """Theorems of sec. 6.2 on converged steps: the total mass (rho, 1) is
    conserved, and E^{n+1} - E^n = -D with D = dt/Re |grad u~|^2 + dt/(3Re)
    |div u~|^2 + dt/(M Pe) |grad mu_c|^2 + 1/2 |sqrt(rho^n)(u~ - u^n)|^2 +
    1/2 |sqrt(rho^{n+1})(u^{n+1} - u~)|^2, every part non-negative"""
    c = CASES[name]()
    o = OR.Oracle(c["grid"], c["params"], pj())
    o.set_state(c["state"]["c"])
    for _ in range(3):
        M0, E0 = o.mass(), o.energy()
        assert o.step(c["dt"]) == OR.OK
        M1, E1, D = o.mass(), o.energy(), o.dissipation()
        assert abs(M1.sum() - M0.sum()) <= 1e-12 * max(1.0, abs(M0.sum()))
        assert (D >= 0).all()
        dE = E1[0] - E0[0]
        assert dE <= 0.0
        assert abs(dE + D.sum()) < 1e-12, (dE, D)
    # the projection part is active: u^{n+1} differs from u~
    assert D[4] > 0.0


@pytest.mark.parametrize("bc", [(0, 0), (1, 0), (1, 1)])
def test_projection_pointwise_continuity(bc):
    """(rho(c) - rho^n)/dt + d_x(A_x rho(c) u) + d_y(A_y rho(c) v) equals
    rho(c) (N_p - alpha N_c) at every cell for any iterate, u the velocity of
    time n+1 (the identity behind the mass theorem of sec. 6.2: the phase
    equation's rho^n (c - c^n)/dt and advection at time n+1 pair with the
    mass equation through rho(c) = rho^{n+1})"""
    grid = grid_(8, 12, *bc)
    P, dt = par_O1(rho2=4.0), 0.3
    o = OR.Oracle(grid, P, pj())
    w, wn = W.random_state(grid, 1), W.random_state(grid, 2)
    o.set_time_n_and_iterate(wn, w, dt)
    r, _ = o.residual()
    N = -r
    u, v = o.velocity_np1()
    rho = lambda c: P["rho1"] * P["rho2"] / ((P["rho2"] - P["rho1"]) * c + P["rho1"])
    al = (P["rho2"] - P["rho1"]) / (P["rho1"] * P["rho2"])
    h = grid["Lx"] / grid["m1"]
    rs, rn = rho(w["c"]), rho(wn["c"])
    Fx = 0.5 * (rs + np.roll(rs, 1, axis=1)) * u
    Fy = 0.5 * (rs + np.roll(rs, 1, axis=0)) * v
    if bc[0] == W.PERIODIC:
        Fe = np.roll(Fx, -1, axis=1)
    else:
        assert np.all(Fx[:, 0] == 0.0)
        Fe = np.concatenate([Fx[:, 1:], np.zeros((grid["m2"], 1))], axis=1)
    if bc[1] == W.PERIODIC:
        Fn = np.roll(Fy, -1, axis=0)
    else:
        assert np.all(Fy[0, :] == 0.0)
        Fn = np.concatenate([Fy[1:, :], np.zeros((1, grid["m1"]))], axis=0)
    lhs = (rs - rn) / dt + (Fe - Fx) / h + (Fn - Fy) / h
    rhs = rs * (N[2] - al * N[0])
    assert np.abs(lhs - rhs).max() < 1e-11 * np.abs(lhs).max()


def test_projection_velocity_is_the_projection():
    """the velocity of time n+1 satisfies (pj-num-pjx) face by face:
    A rho (u - u~)/dt = -D pbar/M + A(rho_ew mubar) D c/M (- gravity on v),
    written out here from its definition (App. A.6 for the surface term)"""
    grid = grid_(8, 10, 0, 0)
    P, dt = par_O1(rho2=3.0, rho_ref=0.4), 0.2
    o = OR.Oracle(grid, P, pj())
    w, wn = W.random_state(grid, 5), W.random_state(grid, 6)
    o.set_time_n_and_iterate(wn, w, dt)
    u, v = o.velocity_np1()
    rho = lambda c: P["rho1"] * P["rho2"] / ((P["rho2"] - P["rho1"]) * c + P["rho1"])
    h = grid["Lx"] / grid["m1"]
    c, mu, p = w["c"], w["mu"], w["p"]
    r = rho(c)
    for j in range(grid["m2"]):
        for i in range(1, grid["m1"]):
            Ar = 0.5 * (r[j, i] + r[j, i - 1])
            st = 0.5 * (r[j, i] * mu[j, i - 1] + r[j, i - 1] * mu[j, i]) * (c[j, i] - c[j, i - 1]) / h
            rhs = (-(p[j, i] - p[j, i - 1]) / h + st) / P["M"]
            assert abs(Ar * (u[j, i] - w["u"][j, i]) / dt - rhs) < 1e-12 * (1 + abs(rhs))
    for j in range(1, grid["m2"]):
        for i in range(grid["m1"]):
            Ar = 0.5 * (r[j, i] + r[j - 1, i])
            st = 0.5 * (r[j, i] * mu[j - 1, i] + r[j - 1, i] * mu[j, i]) * (c[j, i] - c[j - 1, i]) / h
            rhs = (-(p[j, i] - p[j - 1, i]) / h + st) / P["M"] - P["inv_Fr"] * (Ar - P["rho_ref"])
            assert abs(Ar * (v[j, i] - w["v"][j, i]) / dt - rhs) < 1e-12 * (1 + abs(rhs))
    assert np.all(u[:, 0] == 0.0) and np.all(v[0, :] == 0.0)


def test_projection_hydrostatic_closed_form():
    """Equal densities, uniform c, fluid at rest, walls: u~ = u = 0,
    mubar = K1 f(c0) / 1 (rho^n mubar with rho^n = rho), and the hydrostatic
    pressure (1/M) D_y pbar = -(1/Fr) rho from the projection equation"""
    m1, m2 = 16, 32
    grid = grid_(m1, m2, 0, 0)
    P = par_O1(rho1=2.0, rho2=2.0, inv_Fr=1.5, M=0.4)
    o = OR.Oracle(grid, P, pj(1e-12))
    c0 = 0.3
    o.set_state(np.full((m2, m1), c0))
    assert o.step(0.05) == OR.OK
    s = o.get_state()
    h = 1.0 / m1
    K1 = P["M"] * P["eta"] / (P["eps"] * P["We"])
    y = (np.arange(m2) + 0.5) * h
    p_exact = -P["M"] * P["inv_Fr"] * 2.0 * (y - y.mean())
    assert np.abs(s["u"]).max() < 1e-12 and np.abs(s["v"]).max() < 1e-12
    assert np.abs(s["c"] - c0).max() < 1e-13
    assert np.abs(s["mu"] - K1 * c0 * (c0 - 1) * (c0 - 0.5)).max() < 1e-12
    assert np.abs(s["p"] - p_exact[:, None]).max() < 1e-11


def _unknown_blocks(grid):
    """dense ordering of the oracle: per cell c, mu, p, then u, v where they
    are unknowns"""
    idx = {k: [] for k in FIELDS}
    n = 0
    for j in range(grid["m2"]):
        for i in range(grid["m1"]):
            for k in ("c", "mu", "p"):
                idx[k].append(n); n += 1
            if grid["bcx"] == W.PERIODIC or i >= 1:
                idx["u"].append(n); n += 1
            if grid["bcy"] == W.PERIODIC or j >= 1:
                idx["v"].append(n); n += 1
    return idx, n


@pytest.mark.parametrize("case", ["walls", "periodic_x"])
def test_projection_multigrid_root_equals_dense_newton(case):
    """the V-cycles of sec. 7.2 reach the root of the projection system found
    by a dense Newton iteration (pbar mean bordered), compared on c, mubar,
    pbar and the velocity of time n+1"""
    if case == "walls":
        c = W.rising_drop(8, 16, eps=0.1)
    else:
        c = W.capillary(8, 16, eps=0.1, levels=0)
    P = dict(c["params"], inv_Fr=1.0)
    dt = 0.01
    o = OR.Oracle(c["grid"], P, pj(1e-12))
    o.set_state(c["state"]["c"])
    assert o.step(dt) == OR.OK
    smg = o.get_state()
    on = OR.Oracle(c["grid"], P, pj())
    on.set_state(c["state"]["c"])
    on.begin_step(dt)
    B, n = _unknown_blocks(c["grid"])
    assert n == on.dense(jacobian=False)[0].size
    b = np.zeros(n)
    b[B["p"]] = 1.0
    for it in range(30):
        N, J = on.dense()
        st = on.get_state()
        K = np.zeros((n + 1, n + 1))
        K[:n, :n] = J
        K[:n, n] = b
        K[n, :n] = b
        dx = np.linalg.solve(K, -np.concatenate([N, [st["p"].sum()]]))
        on.add_unknowns(dx[:n])
        if np.abs(dx[:n]).max() < 1e-14 and np.abs(N).max() < 1e-11:
            break
    N, _ = on.dense(jacobian=False)
    assert np.abs(N).max() < 1e-10
    snt = on.get_state()
    un, vn = on.velocity_np1()
    snt["u"], snt["v"] = un, vn
    for k in FIELDS:
        scale = max(np.abs(snt[k]).max(), 1e-3)
        assert np.abs(smg[k] - snt[k]).max() < 1e-9 * scale, k


def test_projection_pressure_step_is_exact():
    """sec. 7.2, step 3: after a half-sweep the mass equation holds at every
    cell of the colour (it depends on pbar of the cell linearly, through the
    mobility term and through the projected velocity of its four faces, and
    on nothing a later box of the colour changes)"""
    grid = grid_(12, 8, 1, 0)
    P = par_O1(rho2=3.0)
    o = OR.Oracle(grid, P, pj())
    w, wn = W.random_state(grid, 11), W.random_state(grid, 12)
    o.set_time_n_and_iterate(wn, w, 0.2)
    _, n0 = o.residual()
    for colour in (0, 1):
        o.halfsweep(colour)
        r, _ = o.residual()
        J, I = np.indices((grid["m2"], grid["m1"]))
        own = ((I + J) & 1) == colour
        assert np.abs(r[2][own]).max() < 1e-11 * max(1.0, n0[2]), colour
        assert np.abs(r[2][~own]).max() > 1e-6


def test_projection_vcycle_contracts():
    """V-cycles of the projection scheme converge on the parity workloads
    (the paper prints no iteration counts: parity unpinned for the factor)"""
    for c in (W.capillary(), W.rising_drop(32, 64, eps=0.04), _periodic_drop()):
        o = OR.Oracle(c["grid"], c["params"], pj())
        o.set_state(c["state"]["c"])
        assert o.step(c["dt"]) == OR.OK
        nv, hist = o.stats()
        assert nv <= 12
        f = (hist[-1].max() / hist[0].max()) ** (1.0 / nv)
        assert f < 0.25, f
