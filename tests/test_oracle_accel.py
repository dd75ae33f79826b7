"""Pins of the oracle's acceleration of the cycle iteration (the nonlinear
Krylov acceleration of multigrid of Washio and Oosterlee; the paper's sec. 7.1
asks only for FAS V-cycles, so this is a solver choice that must leave the
root of the discrete system of sec. 6.1 unchanged).

The combination is checked against an independent computation: numpy's
least-squares solver (QR/SVD, not the oracle's normal equations) applied to
the cycle results and residuals read back through the oracle's public calls.
The root itself is pinned by the dense Newton test of test_oracle_pins.py,
which runs with and without acceleration.
"""
import numpy as np
import pytest

import oracle as OR
from paper_1703_06606_amd import workloads as W

FIELDS = ("c", "mu", "p", "u", "v")


def _stack(st):
    return np.stack([st[k] for k in FIELDS])


def _case(name):
    if name == "drop_walls":
        return W.rising_drop(16, 32, eps=0.08)
    if name == "box_ratio100":
        return W.drops_box(32, 3, 0.08, 0.15, 0.03, 11)
    return W.rayleigh_taylor(16, 64, eps=0.08)


@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("name", ["drop_walls", "box_ratio100", "rt_periodic_x"])
def test_combination_is_the_least_squares_one(name, m):
    c = _case(name)
    o = OR.Oracle(c["grid"], c["params"], dict(W.default_opts(1e-14), accel=m))
    o.set_state(c["state"]["c"])
    o.begin_step(c["dt"])
    ws, rs = [], []
    for k in range(m + 3):
        o.vcycle()
        ws.append(_stack(o.get_state()))
        r, _ = o.residual()
        rs.append(r.copy())
        g = o.accel_coeffs()
        # results are kept from the second cycle of the step on
        n = max(0, min(k - 1, m))
        if n == 0:
            assert g.size == 0
        else:
            # columns r_0 - r_a of the newest result against the a-th earlier one
            A = np.stack([(rs[-1] - rs[-1 - a]).ravel() for a in range(1, n + 1)], 1)
            gl, *_ = np.linalg.lstsq(A, -rs[-1].ravel(), rcond=None)
            assert g.size == n
            assert np.allclose(g, gl, rtol=1e-7, atol=1e-9 * max(1.0, np.abs(gl).max())), (g, gl)
            # optimality: the linearised residual is orthogonal to the columns
            z = rs[-1].ravel() + A @ g
            assert np.abs(A.T @ z).max() <= 1e-8 * np.abs(A).max() * np.abs(rs[-1]).max() * A.shape[0]
            # the linearised residual is no larger than the plain result's
            assert np.linalg.norm(z) <= np.linalg.norm(rs[-1]) * (1 + 1e-12)
        o.accelerate()
        new = _stack(o.get_state())
        expect = ws[-1].copy()
        for a in range(1, n + 1):
            expect += g[a - 1] * (ws[-1] - ws[-1 - a])
        scale = np.abs(ws[-1]).reshape(5, -1).max(1)[:, None, None] + 1e-300
        assert (np.abs(new - expect) / scale).max() < 1e-13
        # the next cycle restarts from the combination; a pbar of zero mean
        # stays so (up to rounding)
        assert abs(new[2].mean()) < 1e-12 * max(1.0, np.abs(new[2]).max())


def test_first_cycle_is_the_plain_cycle():
    """Nothing is combined before two results exist: the first cycle of an
    accelerated step is bitwise the plain one"""
    c = W.capillary()
    out = []
    for m in (0, 2):
        o = OR.Oracle(c["grid"], c["params"], dict(W.default_opts(1e-10), accel=m))
        o.set_state(c["state"]["c"])
        o.begin_step(c["dt"])
        o.vcycle()
        o.accelerate()
        out.append(o.get_state())
    for k in FIELDS:
        assert np.array_equal(out[0][k], out[1][k])


def test_acceleration_reaches_the_same_root_in_fewer_cycles():
    """On the periodic drop box at density ratio 100 (slow plain cycles), the
    accelerated step converges to the same state in fewer cycles"""
    c = W.drops_box(64, 5, 0.06, 0.12, 0.015, 3)
    res = {}
    for m in (0, 2):
        o = OR.Oracle(c["grid"], c["params"], dict(W.default_opts(1e-10), accel=m, max_vcycles=80))
        o.set_state(c["state"]["c"])
        assert o.step(c["dt"]) == OR.OK
        res[m] = (o.stats()[0], o.get_state())
    assert res[2][0] < res[0][0], (res[0][0], res[2][0])
    for k in FIELDS:
        scale = max(np.abs(res[0][1][k]).max(), 1e-3)
        assert np.abs(res[0][1][k] - res[2][1][k]).max() < 1e-8 * scale, k


def test_history_restarts_when_a_result_does_not_improve():
    """A cycle result whose largest residual norm is not below its
    predecessor's starts a new history: no combination after it, and the next
    one uses that result and its successor only (checked against numpy's
    least squares on the two)"""
    c = W.rising_drop(16, 32, eps=0.08)
    o = OR.Oracle(c["grid"], c["params"], dict(W.default_opts(1e-14), accel=2))
    o.set_state(c["state"]["c"])
    o.begin_step(c["dt"])
    for _ in range(4):
        o.vcycle()
        o.accelerate()
    _, n_before = o.residual()
    # disturb the iterate (time-n data and the history stay)
    st = o.get_state()
    rng = np.random.default_rng(5)
    o.set_state(*[st[k] + (0.05 * rng.standard_normal(st[k].shape) if k in ("u", "v") else 0.0)
                  for k in FIELDS])
    o.vcycle()
    _, n_after = o.residual()
    assert n_after.max() >= n_before.max()
    assert o.accel_coeffs().size == 0
    o.accelerate()
    w1, (r1, _) = _stack(o.get_state()), o.residual()
    o.vcycle()
    w2, (r2, _) = _stack(o.get_state()), o.residual()
    g = o.accel_coeffs()
    assert g.size == 1
    A = (r2 - r1).ravel()[:, None]
    gl, *_ = np.linalg.lstsq(A, -r2.ravel(), rcond=None)
    assert np.allclose(g, gl, rtol=1e-7)
    o.accelerate()
    assert np.allclose(_stack(o.get_state()), w2 + g[0] * (w2 - w1), rtol=0, atol=1e-13 * np.abs(w2).max())
