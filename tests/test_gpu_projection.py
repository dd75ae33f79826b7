"""Parity of the HIP projection scheme (sec. 6.2, smoother of sec. 7.2)
with the FP64 CPU oracle through the C ABI: residuals, half-sweeps, V-cycles
and converged steps element by element, mass, energy and the five parts of
the dissipation, the discrete energy law on the GPU's own steps, and the
256 x 512 rising droplet checked by the oracle's residual.  Tolerances as for
the primitive scheme: 1e-12 relative for a residual evaluation, 1e-11 for
half-sweeps, 1e-10 for V-cycles and converged steps."""
import sys

import numpy as np
import pytest

import oracle as OR
from paper_1703_06606_amd import qnsch as Q
from paper_1703_06606_amd import workloads as W

pytestmark = pytest.mark.gpu
FIELDS = ("c", "mu", "p", "u", "v")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pj(tol=1e-10, **kw):
    return dict(W.default_opts(tol), scheme=W.PROJECTION, **kw)


def pair(cfg, opts):
    return Q.Solver(cfg["grid"], cfg["params"], opts), OR.Oracle(cfg["grid"], cfg["params"], opts)


def rel(a, b, floor=1e-12):
    return np.abs(a - b).max() / max(np.abs(b).max(), floor)


def grid_(m1, m2, bcx, bcy, levels=0):
    return dict(m1=m1, m2=m2, Lx=1.0, Ly=m2 / m1, bcx=bcx, bcy=bcy, levels=levels)


def par_O1(**kw):
    p = dict(rho1=1.0, rho2=2.5, visc1=1.0, visc2=1.8, Re=3.0, We=2.0, inv_Fr=0.7, Pe=2.0, M=0.8,
             eps=0.5, eta=0.9, mob_reg=0.05, rho_ref=0.0)
    p.update(kw)
    return p


SHAPES = [(16, 24, 0, 0), (16, 24, 1, 0), (16, 16, 1, 1), (40, 24, 0, 0), (72, 40, 1, 1), (8, 8, 1, 1)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d_bc%d%d" % s)
def test_projection_residual_matches_oracle(shape):
    m1, m2, bx, by = shape
    say("projection residual parity", shape)
    cfg = dict(grid=grid_(m1, m2, bx, by), params=par_O1(rho2=3.0, rho_ref=0.3))
    g, o = pair(cfg, pj())
    w, wn = W.random_state(cfg["grid"], 21), W.random_state(cfg["grid"], 22)
    for s in (g, o):
        s.set_time_n_and_iterate(wn, w, 0.3)
    rg, ng = g.residual()
    ro, no = o.residual()
    for q, k in enumerate(FIELDS):
        assert rel(rg[q], ro[q]) < 1e-12, (k, rel(rg[q], ro[q]))
    assert np.allclose(ng, no, rtol=1e-12, atol=0)


@pytest.mark.parametrize("smoother", [W.SMOOTH_COUPLED, W.SMOOTH_SEGREGATED], ids=["coupled", "segregated"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d_bc%d%d" % s)
def test_projection_halfsweeps_match_oracle(shape, smoother):
    m1, m2, bx, by = shape
    say("projection halfsweep parity", shape, "smoother", smoother)
    cfg = dict(grid=grid_(m1, m2, bx, by), params=par_O1(rho2=3.0))
    g, o = pair(cfg, pj(smoother=smoother))
    w, wn = W.random_state(cfg["grid"], 23), W.random_state(cfg["grid"], 24)
    for s in (g, o):
        s.set_time_n_and_iterate(wn, w, 0.3)
    for colour in (0, 1, 0):
        g.halfsweep(colour)
        o.halfsweep(colour)
        a, b = g.get_state(), o.get_state()
        for k in FIELDS:
            assert rel(a[k], b[k]) < 1e-11, (colour, k, rel(a[k], b[k]))


def _periodic_drop():
    c = W.rising_drop(32, 32, eps=0.04)
    c["grid"] = grid_(32, 32, 1, 1)
    c["params"] = dict(c["params"], inv_Fr=0.0)
    return c


def _cases():
    return {
        "capillary_32x64": W.capillary(),
        "drop_32x64": W.rising_drop(32, 64, eps=0.04),
        "drop_40x24_ragged": W.rising_drop(40, 24, eps=0.05, radius=0.2),
        "periodic_box_32x32": _periodic_drop(),
        "rayleigh_taylor_16x64": W.rayleigh_taylor(16, 64, eps=0.08),
    }


@pytest.mark.parametrize("smoother", [W.SMOOTH_COUPLED, W.SMOOTH_SEGREGATED], ids=["coupled", "segregated"])
@pytest.mark.parametrize("name", list(_cases()))
def test_projection_vcycles_match_oracle(name, smoother):
    cfg = _cases()[name]
    say("projection vcycle parity", name, "smoother", smoother)
    g, o = pair(cfg, pj(smoother=smoother))
    for s in (g, o):
        s.set_state(cfg["state"]["c"])
        s.begin_step(cfg["dt"])
    for it in range(3):
        g.vcycle()
        o.vcycle()
        a, b = g.get_state(), o.get_state()
        for k in FIELDS:
            assert rel(a[k], b[k], 1e-9) < 1e-10, (it, k, rel(a[k], b[k], 1e-9))
        _, ng = g.residual()
        _, no = o.residual()
        assert np.allclose(ng, no, rtol=1e-6, atol=1e-14), (ng, no)
    # end of the step by phases: the velocity of time n+1 replaces u~
    un, vn = o.velocity_np1()
    g.end_step()
    a = g.get_state()
    assert rel(a["u"], un, 1e-9) < 1e-10 and rel(a["v"], vn, 1e-9) < 1e-10


@pytest.mark.parametrize("name", list(_cases()))
def test_projection_converged_step_matches_oracle(name):
    cfg = _cases()[name]
    say("projection step parity", name)
    g, o = pair(cfg, pj())
    for s in (g, o):
        s.set_state(cfg["state"]["c"])
    for step in range(2):
        mg0, eg0 = g.mass(), g.energy()
        assert g.step(cfg["dt"]) == Q.OK
        assert o.step(cfg["dt"]) == OR.OK
        a, b = g.get_state(), o.get_state()
        for k in FIELDS:
            assert rel(a[k], b[k], 1e-9) < 1e-10, (step, k, rel(a[k], b[k], 1e-9))
        assert abs(g.stats()["vcycles"] - o.stats()[0]) <= 1
        mg = g.mass()
        assert abs(mg.sum() - mg0.sum()) <= 1e-12 * max(1.0, abs(mg0.sum()))
        eg = g.energy()
        assert np.allclose(eg, o.energy(), rtol=1e-10, atol=1e-14)
        dg, do = g.dissipation(), o.dissipation()
        assert np.allclose(dg, do, rtol=1e-9, atol=1e-15), (dg, do)
        assert (dg >= 0).all()
        if cfg["grid"]["bcy"] == W.WALL or cfg["params"]["inv_Fr"] == 0.0:
            assert abs(eg[0] - eg0[0] + dg.sum()) < 1e-12, (eg[0] - eg0[0], dg)


def test_projection_full_size_rising_drop():
    """256 x 512 rising droplet in the projection scheme: one V-cycle field
    by field against the oracle, then V-cycles on the GPU to 1e-10 and the
    oracle's own residual at the GPU's iterate, and the step's mass and
    energy law"""
    cfg = W.rising_drop()
    say("projection full size", cfg["name"])
    opts = pj()
    g, o = pair(cfg, opts)
    for s in (g, o):
        s.set_state(cfg["state"]["c"])
        s.begin_step(cfg["dt"])
    g.vcycle()
    o.vcycle()
    a, b = g.get_state(), o.get_state()
    for k in FIELDS:
        assert rel(a[k], b[k], 1e-9) < 1e-10, (k, rel(a[k], b[k], 1e-9))
    for _ in range(30):
        _, n = g.residual()
        if n.max() <= 1e-10:
            break
        g.vcycle()
    st = g.get_state()
    o2 = OR.Oracle(cfg["grid"], cfg["params"], opts)
    o2.set_time_n_and_iterate(dict(c=cfg["state"]["c"]), st, cfg["dt"])
    _, no = o2.residual()
    assert no.max() <= 2e-10, no
    g.end_step()
    un, vn = o2.velocity_np1()
    a = g.get_state()
    assert rel(a["u"], un, 1e-9) < 1e-10 and rel(a["v"], vn, 1e-9) < 1e-10
    g.set_state(cfg["state"]["c"])
    m0, e0 = g.mass(), g.energy()
    assert g.step(cfg["dt"]) == Q.OK
    m1, e1 = g.mass(), g.energy()
    assert abs(m1.sum() - m0.sum()) <= 1e-12 * abs(m0.sum())
    assert abs(e1[0] - e0[0] + g.dissipation().sum()) < 1e-10
    say("projection full size V-cycles", g.stats()["vcycles"])


def test_projection_rayleigh_taylor_full_size_vcycle():
    """512 x 2048 Rayleigh-Taylor grid in the projection scheme (4096 finest
    tiles, 9 levels down to a 2 x 8 level periodic in x), moving with a
    discretely divergence-free velocity (u = D_y psi, v = -D_x psi from a
    stream function at the vertices, zero on the walls): one V-cycle field by
    field against the oracle (1e-10)"""
    cfg = W.rayleigh_taylor()
    m2, m1 = cfg["state"]["c"].shape
    h = 1.0 / m1
    xv, yv = np.arange(m1 + 1) * h, np.arange(m2 + 1) * h
    psi = 0.05 * np.sin(np.pi * yv / (m2 * h))[:, None] ** 2 * np.cos(2 * np.pi * xv)[None, :]
    u0 = (psi[1:, :m1] - psi[:-1, :m1]) / h
    v0 = -(psi[:m2, 1:] - psi[:m2, :-1]) / h
    say("projection full size", cfg["name"])
    g, o = pair(cfg, pj())
    for s in (g, o):
        s.set_state(cfg["state"]["c"], None, None, u0, v0)
        s.begin_step(cfg["dt"])
    g.vcycle()
    say("oracle V-cycle at 512 x 2048")
    o.vcycle()
    a, b = g.get_state(), o.get_state()
    for k in FIELDS:
        say(k, rel(a[k], b[k], 1e-9))
        assert rel(a[k], b[k], 1e-9) < 1e-10, (k, rel(a[k], b[k], 1e-9))


def test_projection_rejections():
    cfg = W.rising_drop(16, 32, eps=0.08)
    with pytest.raises(Q.QnschError):
        Q.Solver(cfg["grid"], cfg["params"], pj(precision=Q.MIXED))
    srv = Q.Server(hbm_budget=1 << 30, max_slots=2)
    with pytest.raises(Q.QnschError):
        srv.submit(cfg["grid"], cfg["params"], pj(), cfg["state"]["c"], 1, cfg["dt"])
