"""Temporal blocking of the smoother (a red and a black half-sweep in one
launch on the levels smoothed by many workgroups): parity with the FP64
oracle, which runs the plain half-sweeps of sec. 7.1, and with the GPU's own
unfused path, through the C ABI.

Cases span walls, periodic axes, ragged tiles, an odd number of sweeps (the
last sweep unfused) and the benchmark's 256 x 512 droplet, whose three
coarse multi-workgroup levels are the ones fused by default (blocking 1,
which also fuses a finest level of at most one tile per compute unit, as on
the small cases; blocking 2 fuses the finest level in any case).  Tolerances:
1e-10 relative against the oracle (FP64 parity), 1e-12 against the unfused
GPU path (same arithmetic; only the compiler's contraction of the two
instances may differ).
"""
import sys

import numpy as np
import pytest

import oracle as OR
from paper_1703_06606_amd import qnsch as Q
from paper_1703_06606_amd import workloads as W

FIELDS = ("c", "mu", "p", "u", "v")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b, floor=1e-9):
    return np.abs(a - b).max() / max(np.abs(b).max(), floor)


def _periodic_box():
    c = W.rising_drop(32, 32, eps=0.04)
    c["grid"] = dict(m1=32, m2=32, Lx=1.0, Ly=1.0, bcx=W.PERIODIC, bcy=W.PERIODIC, levels=0)
    c["params"] = dict(c["params"], inv_Fr=0.0)
    return c


def _cases():
    return {
        "drop_32x64": (W.rising_drop(32, 64, eps=0.04), {}),
        "capillary_32x64": (W.capillary(), {}),
        "drop_40x24_ragged": (W.rising_drop(40, 24, eps=0.05, radius=0.2), {}),
        "periodic_box_32x32": (_periodic_box(), {}),
        "drop_32x64_nu3": (W.rising_drop(32, 64, eps=0.04), dict(nu1=3, nu2=1)),
    }


def test_fused_footprint_adds_a_cell_set():
    """host only: a second set of c, mubar, pbar on every level (64 x 128,
    automatic hierarchy of 5 levels down to 4 x 8; the same for the
    projection scheme), of the FP32 corrections in mixed precision"""
    cfg = W.rising_drop(64, 128, eps=0.04)
    base = dict(W.default_opts(), blocking=0)
    f0 = Q.footprint(cfg["grid"], base)
    f1 = Q.footprint(cfg["grid"], dict(base, blocking=1))
    cells = sum((64 >> l) * (128 >> l) for l in range(5))
    assert 24 * cells <= f1 - f0 <= 24 * cells + 3 * 256 * 5, (f0, f1)
    g0 = Q.footprint(cfg["grid"], dict(base, precision=Q.MIXED))
    g1 = Q.footprint(cfg["grid"], dict(base, blocking=1, precision=Q.MIXED))
    assert 12 * cells <= g1 - g0 <= 12 * cells + 3 * 256 * 5, (g0, g1)
    p0 = Q.footprint(cfg["grid"], dict(base, scheme=1))
    assert Q.footprint(cfg["grid"], dict(base, blocking=2, scheme=1)) - p0 == f1 - f0


def _start(s, cfg):
    s.set_state(cfg["state"]["c"])
    s.begin_step(cfg["dt"])


@pytest.mark.gpu
@pytest.mark.parametrize("smoother", [W.SMOOTH_COUPLED, W.SMOOTH_SEGREGATED], ids=["coupled", "segregated"])
@pytest.mark.parametrize("name", list(_cases()))
def test_fused_vcycles_match_oracle(name, smoother):
    cfg, extra = _cases()[name]
    say("fused vcycle parity", name, "smoother", smoother)
    base = dict(W.default_opts(), smoother=smoother, blocking=0, **extra)
    fused = Q.Solver(cfg["grid"], cfg["params"], dict(base, blocking=2))
    plain = Q.Solver(cfg["grid"], cfg["params"], base)
    o = OR.Oracle(cfg["grid"], cfg["params"], base)
    for s in (fused, plain, o):
        _start(s, cfg)
    for it in range(3):
        for s in (fused, plain, o):
            s.vcycle()
        a, b, r = fused.get_state(), plain.get_state(), o.get_state()
        for k in FIELDS:
            assert rel(a[k], r[k]) < 1e-10, (it, k, rel(a[k], r[k]))
            assert rel(a[k], b[k]) < 1e-12, (it, k, rel(a[k], b[k]))
        for s in (fused, plain, o):
            s.accelerate()
    _, nf = fused.residual()
    _, no = o.residual()
    assert np.allclose(nf, no, rtol=1e-6, atol=1e-14), (nf, no)


@pytest.mark.gpu
@pytest.mark.parametrize("blocking", [1, 2])
def test_fused_full_size_rising_drop(blocking):
    """The benchmark's 256 x 512 droplet: one V-cycle with fused coarse
    levels (and the finest one) against the oracle's and the unfused GPU
    cycle, then a converged step whose V-cycle count and oracle residual
    match the unfused path."""
    cfg = W.rising_drop()
    say("fused full size, blocking", blocking)
    base = dict(W.default_opts(1e-10), blocking=0)
    fused = Q.Solver(cfg["grid"], cfg["params"], dict(base, blocking=blocking))
    plain = Q.Solver(cfg["grid"], cfg["params"], base)
    o = OR.Oracle(cfg["grid"], cfg["params"], base)
    for s in (fused, plain, o):
        _start(s, cfg)
        s.vcycle()
    a, b, r = fused.get_state(), plain.get_state(), o.get_state()
    for k in FIELDS:
        assert rel(a[k], r[k]) < 1e-10, (k, rel(a[k], r[k]))
        assert rel(a[k], b[k]) < 1e-12, (k, rel(a[k], b[k]))
    for s in (fused, plain):
        s.set_state(cfg["state"]["c"])
        assert s.step(cfg["dt"]) == Q.OK
    assert abs(fused.stats()["vcycles"] - plain.stats()["vcycles"]) <= 1
    st = fused.get_state()
    o2 = OR.Oracle(cfg["grid"], cfg["params"], base)
    o2.set_time_n_and_iterate(dict(c=cfg["state"]["c"]), st, cfg["dt"])
    _, no = o2.residual()
    assert no.max() <= 2e-10, no
    say("fused full size vcycles", fused.stats()["vcycles"], plain.stats()["vcycles"])


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["drop_32x64", "capillary_32x64", "periodic_box_32x32", "drop_40x24_ragged"])
def test_fused_mixed_matches_unfused_and_oracle(name):
    """Mixed precision with the FP32 correction smoother fused on every
    level that qualifies (the finest included): after each of three outer
    iterations the FP64 iterate agrees with the unfused mixed path (the same
    FP32 arithmetic; 1e-6 of the field maxima), and the converged step with
    the oracle's converged FP64 step (1e-6, the mixed-precision bar)."""
    cfg, _ = _cases()[name]
    say("fused mixed", name)
    base = dict(W.default_opts(1e-10), blocking=0, precision=Q.MIXED)
    fused = Q.Solver(cfg["grid"], cfg["params"], dict(base, blocking=2))
    plain = Q.Solver(cfg["grid"], cfg["params"], base)
    for s in (fused, plain):
        _start(s, cfg)
    for it in range(3):
        for s in (fused, plain):
            s.vcycle()
        a, b = fused.get_state(), plain.get_state()
        for k in FIELDS:
            assert rel(a[k], b[k]) < 1e-6, (it, k, rel(a[k], b[k]))
    o = OR.Oracle(cfg["grid"], cfg["params"], dict(base, precision=Q.FP64))
    fused.set_state(cfg["state"]["c"])
    o.set_state(cfg["state"]["c"])
    assert fused.step(cfg["dt"]) == Q.OK
    assert o.step(cfg["dt"]) == OR.OK
    a, r = fused.get_state(), o.get_state()
    for k in FIELDS:
        assert rel(a[k], r[k]) < 1e-6, (k, rel(a[k], r[k]))


@pytest.mark.gpu
@pytest.mark.parametrize("smoother", [W.SMOOTH_COUPLED, W.SMOOTH_SEGREGATED], ids=["coupled", "segregated"])
@pytest.mark.parametrize("name", ["drop_32x64", "capillary_32x64", "periodic_box_32x32", "drop_40x24_ragged"])
def test_fused_projection_matches_oracle(name, smoother):
    """The projection scheme's smoother (sec. 7.2) fused on every qualifying
    level: three V-cycles with combinations against the oracle's (1e-10) and
    the unfused GPU path (1e-12), then the velocity of time n+1."""
    cfg, _ = _cases()[name]
    say("fused projection", name, "smoother", smoother)
    base = dict(W.default_opts(), smoother=smoother, blocking=0, scheme=Q.PROJECTION)
    fused = Q.Solver(cfg["grid"], cfg["params"], dict(base, blocking=2))
    plain = Q.Solver(cfg["grid"], cfg["params"], base)
    o = OR.Oracle(cfg["grid"], cfg["params"], base)
    for s in (fused, plain, o):
        _start(s, cfg)
    for it in range(3):
        for s in (fused, plain, o):
            s.vcycle()
        a, b, r = fused.get_state(), plain.get_state(), o.get_state()
        for k in FIELDS:
            assert rel(a[k], r[k]) < 1e-10, (it, k, rel(a[k], r[k]))
            assert rel(a[k], b[k]) < 1e-12, (it, k, rel(a[k], b[k]))
        for s in (fused, plain, o):
            s.accelerate()
    # end of the step: the velocity of time n+1 replaces u~
    un, vn = o.velocity_np1()
    fused.end_step()
    a = fused.get_state()
    assert rel(a["u"], un) < 1e-10 and rel(a["v"], vn) < 1e-10
