"""Replayed cycle graphs (qnsch_graphs): a context that replays each cycle's
fixed launches from a captured HIP graph gives bitwise the iterates of a
context that launches them one by one (the default), step after step and cycle after
cycle, with the programme's own eager work (reductions, state reads, the
acceleration's combination) and host synchronisations between the replays.

Cases: the primitive scheme with the default options (acceleration,
temporal blocking of the coarse levels), plain cycles, blocking of every
level, the segregated smoother, the projection scheme (whose step end flips
the finest level's face buffer, so its cycles start from two buffer
patterns), mixed precision, a periodic box, and the 256 x 512 benchmark
droplet.
"""
import sys

import numpy as np
import pytest

from paper_1703_06606_amd import qnsch as Q
from paper_1703_06606_amd import workloads as W

pytestmark = pytest.mark.gpu
FIELDS = ("c", "mu", "p", "u", "v")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _periodic_box():
    c = W.rising_drop(32, 32, eps=0.04)
    c["grid"] = dict(m1=32, m2=32, Lx=1.0, Ly=1.0, bcx=W.PERIODIC, bcy=W.PERIODIC, levels=0)
    c["params"] = dict(c["params"], inv_Fr=0.0)
    return c


def _cases():
    d = W.default_opts(1e-10)
    return {
        "drop_64x128_default": (W.rising_drop(64, 128, eps=0.02), d),
        "drop_64x128_plain": (W.rising_drop(64, 128, eps=0.02), dict(d, accel=0)),
        "drop_64x128_blocking2": (W.rising_drop(64, 128, eps=0.02), dict(d, blocking=2)),
        "drop_32x64_segregated": (W.rising_drop(32, 64, eps=0.04), dict(d, smoother=W.SMOOTH_SEGREGATED, accel=0)),
        "drop_64x128_projection": (W.rising_drop(64, 128, eps=0.02), dict(d, scheme=W.PROJECTION)),
        "drop_64x128_mixed": (W.rising_drop(64, 128, eps=0.02), dict(W.default_opts(1e-8), precision=Q.MIXED)),
        "periodic_box_32x32": (_periodic_box(), d),
        "capillary_32x64": (W.capillary(), d),
    }


def _pair(cfg, opts):
    a = Q.Solver(cfg["grid"], cfg["params"], opts)
    b = Q.Solver(cfg["grid"], cfg["params"], opts)
    a.graphs(True)
    for s in (a, b):
        s.set_state(cfg["state"]["c"])
    return a, b


def _same(a, b, what):
    sa, sb = a.get_state(), b.get_state()
    for k in FIELDS:
        assert np.array_equal(sa[k], sb[k]), (what, k, np.abs(sa[k] - sb[k]).max())


@pytest.mark.parametrize("name", list(_cases()))
def test_replayed_steps_equal_direct_launches(name):
    cfg, opts = _cases()[name]
    say("graph replay steps", name)
    g, d = _pair(cfg, opts)
    for step in range(3):
        assert g.step(cfg["dt"]) == Q.OK
        assert d.step(cfg["dt"]) == Q.OK
        sg, sd = g.stats(), d.stats()
        assert sg["vcycles"] == sd["vcycles"], (step, sg["vcycles"], sd["vcycles"])
        assert np.array_equal(sg["hist"], sd["hist"]), step
        _same(g, d, "step %d" % step)
        # eager work of the programme between replays
        assert np.array_equal(g.mass(), d.mass())
        assert np.array_equal(g.energy(), d.energy())
    say("graph replay steps", name, "V-cycles of the last step", g.stats()["vcycles"])


@pytest.mark.parametrize("name", ["drop_64x128_default", "drop_64x128_projection", "drop_64x128_mixed"])
def test_replayed_cycles_by_phases(name):
    """begin_step / vcycle / accelerate, with a residual read and, on FP64
    contexts, a single half-sweep between cycles (it flips the finest level's
    buffer, so the next cycle starts from a new pattern and is captured anew)"""
    cfg, opts = _cases()[name]
    say("graph replay phases", name)
    g, d = _pair(cfg, opts)
    for s in (g, d):
        s.begin_step(cfg["dt"])
    for it in range(4):
        for s in (g, d):
            s.vcycle()
            s.accelerate()
        _same(g, d, "cycle %d" % it)
        rg, ng = g.residual()
        rd, nd = d.residual()
        assert np.array_equal(ng, nd) and all(np.array_equal(x, y) for x, y in zip(rg, rd))
        if it == 1 and opts.get("precision", Q.FP64) == Q.FP64:
            for s in (g, d):
                s.halfsweep(0)
            _same(g, d, "half-sweep")
    for s in (g, d):
        s.end_step()
    _same(g, d, "end of step")


def test_replayed_steps_benchmark_droplet():
    """the 256 x 512 droplet of the benchmark, two steps, and a third after
    switching the replaying context to direct launches and back"""
    cfg = W.rising_drop()
    opts = W.default_opts(1e-8)
    say("graph replay", cfg["name"])
    g, d = _pair(cfg, opts)
    for step in range(3):
        if step == 2:
            g.graphs(False)
            g.graphs(True)
        assert g.step(cfg["dt"]) == Q.OK
        assert d.step(cfg["dt"]) == Q.OK
        assert g.stats()["vcycles"] == d.stats()["vcycles"]
        _same(g, d, "step %d" % step)
