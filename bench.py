#!/usr/bin/env python3
"""Benchmark of the multigrid time step on one MI355X.

Main line (``value``): the 256 x 512 rising droplet on [0,1] x [0,2] (walls on
all sides, density ratio 10, viscosity ratio 10, Re = 35, We = 10, Fr = 1,
eps = 0.01, dt = 5e-4, 7 multigrid levels), FP64, each step solved to a
residual of 1e-8.  A step is one call of qnsch_step (all V-cycles of the time
step).  The timed region starts from the initial droplet after W untimed
warm-up steps, with all inputs resident in HBM, and covers exactly K steps,
run as they run for any caller (no launch carries timing events).

Beside it, on the same JSON line:
  projection -- the same droplet steps in the projection scheme of sec. 6.2
             (FP64), with its speedup over the primitive scheme, V-cycles,
             total-mass drift and the energy law of its theorem;
  mixed   -- the 512 x 2048 Rayleigh-Taylor run in FP64 and in mixed
             precision (FP32 correction cycles inside FP64 defect correction),
             the same number of steps each, with the mixed/FP64 speedup and
             the difference of the final states;
  served  -- 64 droplet requests of four sizes arriving as a seeded Poisson
             stream at 20 per second, 50 steps each, through the continuous-
             batching server in mixed precision; throughput and p50/p99 step
             latency against the same requests run one after another;
  roofline   -- of the kernel that takes the most time in the step (by a
             breakdown of two untimed steps, every launch between HIP
             events), measured by HIP events that carry that kernel's own
             start and end over a second pass of the same K steps (launches
             that carry events take longer to issue, so the timed region
             carries none; the kernels and their arguments are the same),
             against its algorithmic bytes; the same for the
             finest-level half-sweep; the whole step's algorithmic bytes
             over the timed region's time;
  capillary -- the 32 x 64 capillary wave, FP64 to 1e-10: 100 repeats of
             one step, p50/p99 latency;
  paper_smoother -- the droplet with the printed smoother of sec. 7.1 and
             plain cycles;
  paper_table2 -- the GPU's seconds per step on the grids of the paper's
             Table 2 (the convergence-study workload) beside the paper's own
             CPU seconds per step, quoted with its hardware as context;
  cpu_baseline -- the FP64 CPU oracle on the host's cores: the capillary
             step in full and full droplet steps.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1703_06606_amd import qnsch as Q  # noqa: E402
from paper_1703_06606_amd import workloads as W  # noqa: E402

METRIC = "cell-steps/s to MG residual 1e-8, mixed vs FP64; p50/p99 step latency"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes (what the method must move, FP64, per cell of the level
# a launch works on).  One smoothing sweep reads the five unknowns and the
# three time-n fields and writes the five unknowns: 13 doubles = 104 B per
# cell; a coarse level also reads the five FAS right-hand sides: 144 B.  A
# colour half-sweep is half a sweep (52 / 72 B).  A residual moves as much
# as a sweep; a restriction or a prolongation about 100 B per fine cell.
SWEEP_B = {True: 104.0, False: 144.0}      # finest level: True
RESID_B = {True: 104.0, False: 144.0}
TRANSFER_B = 100.0
# FP32 correction smoother (mixed precision): per sweep it reads the
# linearisation point (4), the five corrections, the three time-n fields
# and the five right-hand sides and writes the five corrections, in FP32:
# 22 floats = 88 B per cell
MX_SWEEP_B = 88.0
TRAFFIC_WORKLOAD = "rising_drop_256x512"
# vector issue capacity: 256 CUs x 4 SIMDs, one wave64 VALU instruction per SIMD
# every 4 cycles at 2.4 GHz; FP64 vector peak 78.6 TFLOP/s
VALU_WAVE_INSTS_PER_S = 1024 * 2.4e9 / 4
FP64_PEAK_TFLOPS = 78.6

# kernel launched by each operation of the library's breakdown, on the finest
# level and on coarser ones (the residual operations also launch the
# reduction's finalisation and, after a cycle, the pbar shift)
OP_KERNEL = {
    "halfsweep": ("k_halfsweep_fine", "k_halfsweep"), "fused_sweep": ("k_hs_fused", "k_hs_fused"),
    "smooth": ("k_coarse_solve", "k_coarse_solve"), "coarse_solve": ("k_coarse_solve", "k_coarse_solve"),
    "restrict": ("k_restrict", "k_restrict"),
    "prolong": ("k_prolong", "k_prolong"), "residual": ("k_resid_norm",) * 2, "residual0": ("k_resid_norm",) * 2,
    "residual_acc": ("k_resid_norm",) * 2, "accelerate": ("k_accel",) * 2, "begin": ("k_begin",) * 2,
    "restrict_n": ("k_restrict_n",) * 2, "mx_halfsweep": ("k_mx_halfsweep_fine", "k_mx_halfsweep"),
    "mx_fused_sweep": ("k_mx_fused",) * 2, "mx_smooth": ("k_mx_coarse_solve",) * 2,
    "mx_coarse_solve": ("k_mx_coarse_solve",) * 2, "mx_restrict": ("k_mx_restrict",) * 2,
    "mx_prolong": ("k_mx_prolong",) * 2, "mx_update": ("k_mx_update",) * 2, "mx_restrict_n": ("k_mx_restrict_n",) * 2,
    "pj_final": ("k_pj_final",) * 2,
}


# kernels one operation launches (the residual reductions: the residual with
# partial sums, their finalisation and, after a cycle, the pbar shift)
KERNELS_PER_OP = {"residual": 3, "residual_acc": 3, "residual0": 2, "step_end": 2, "dissipation": 2,
                  "diagnostics": 2}


def kernel_of(op, lev):
    k = OP_KERNEL.get(op)
    return (k[0] if lev == 0 else k[1]) if k else op


def class_bytes(op, lev, launches, cells, opts):
    """algorithmic bytes of `launches` launches of operation op on level lev
    (cells[l] = cells of level l); None for operations outside a step's
    arithmetic"""
    n, fine = cells[lev], lev == 0
    if op == "halfsweep":
        return launches * 0.5 * SWEEP_B[fine] * n
    if op == "fused_sweep":
        return launches * SWEEP_B[fine] * n
    if op == "smooth":
        # level-resident smoothing: pre- and post-smoothing launches alternate,
        # nu1 and nu2 sweeps, the post-smoothing taking the prolongation too
        half = launches / 2.0
        return (half * opts["nu1"] + half * opts["nu2"]) * SWEEP_B[False] * n + half * TRANSFER_B * n
    if op == "coarse_solve":
        # the coarsest solve's sweeps (0 in the options: the library's
        # automatic 4 for the primitive scheme on 6 levels or more, else 6)
        nu_c = opts["nu_coarse"] or (4 if opts.get("scheme", 0) != Q.PROJECTION and len(cells) >= 6 else 6)
        return launches * nu_c * SWEEP_B[False] * n
    if op == "restrict":
        # the residual and the restriction (per fine cell), then the coarse
        # right-hand side, a residual of the coarse level
        return launches * (TRANSFER_B * n + RESID_B[False] * cells[lev + 1])
    if op == "prolong":
        return launches * TRANSFER_B * n
    if op in ("residual", "residual0", "residual_acc"):
        return launches * RESID_B[True] * n
    if op == "accelerate":
        return launches * 8.0 * 5 * (2 + opts.get("accel", 2)) * n
    if op == "begin":
        return launches * 80.0 * n
    if op == "restrict_n":
        return launches * 48.0 * n
    if op == "mx_halfsweep":
        return launches * 0.5 * MX_SWEEP_B * n
    if op == "mx_fused_sweep":
        return launches * MX_SWEEP_B * n
    return None


def level_cells(cfg, nlev):
    return [(cfg["grid"]["m1"] >> l) * (cfg["grid"]["m2"] >> l) for l in range(nlev)]


def kernel_table(bd, cells, opts):
    """{kernel: {launches, ms, alg_bytes}} from a per-(operation, level)
    breakdown; alg_bytes None if some class of it has no algorithmic count"""
    out = {}
    for (op, lev), (n, ms) in bd.items():
        k = kernel_of(op, lev)
        e = out.setdefault(k, {"launches": 0, "ms": 0.0, "alg_bytes": 0.0, "ops": set()})
        e["launches"] += n
        e["ms"] += ms
        e["ops"].add(op)
        b = class_bytes(op, lev, n, cells, opts)
        e["alg_bytes"] = None if (b is None or e["alg_bytes"] is None) else e["alg_bytes"] + b
    return out

# depth of the acceleration of the cycle iteration for every leg (--accel)
ACCEL = 2
# temporal blocking of the smoothing (--blocking): 0 off, 1 coarse levels, 2 all
BLOCKING = None


def base_opts(tol):
    o = dict(W.default_opts(tol), accel=ACCEL)
    if BLOCKING is not None:
        o["blocking"] = BLOCKING
    return o


def source_hash():
    from paper_1703_06606_amd.build import device_source_hash
    return device_source_hash()


def _profile_values(path):
    """key: value lines of a committed counter summary, only if it was taken
    on the current kernel source"""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv if kv.get("source_hash") == source_hash() else None


def traffic_file(kernel):
    return os.path.join(ROOT, "profiles", "%s_%s_traffic.txt" % (kernel, TRAFFIC_WORKLOAD))


def traffic_from_profile(kernel):
    """HBM bytes per launch of the kernel (mean over its dispatches, every
    level) from the committed counter summary"""
    kv = _profile_values(traffic_file(kernel))
    try:
        return float(kv["hbm_bytes_per_launch"]) if kv else None
    except (KeyError, ValueError):
        return None


def valu_from_profile(kernel, avg_launch_us):
    """vector-ALU view of the same kernel from the committed SQ counter
    summary: wave instructions per launch, the issue time they need at full
    rate, and the executed FP64 rate against the FP64 vector peak"""
    kv = _profile_values(os.path.join(ROOT, "profiles", "%s_%s_valu.txt" % (kernel, TRAFFIC_WORKLOAD)))
    if not kv:
        return None
    try:
        insts, flops = float(kv["valu_wave_insts_per_launch"]), float(kv["fp64_flops_per_launch"])
    except (KeyError, ValueError):
        return None
    floor_us = insts / VALU_WAVE_INSTS_PER_S * 1e6
    tf = flops / (avg_launch_us * 1e-6) / 1e12
    return {"valu_wave_insts_per_launch": insts, "issue_floor_us": floor_us, "issue_frac": floor_us / avg_launch_us,
            "fp64_flops_per_launch": flops, "fp64_tflops": tf, "fp64_frac": tf / FP64_PEAK_TFLOPS}


def host_cpu():
    """CPU model and the cores this process may run on"""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count()
    return model, ncpu


def cpu_baseline(c1_repeats=3, c2_steps=2):
    """The FP64 oracle as it stands on the host's cores (its cells of a
    colour and residuals spread over OpenMP threads, sums sequential): the
    capillary 32 x 64 step (tol 1e-10) in full, c1_repeats times from the
    same state, and c2_steps full steps of the 256 x 512 droplet at the
    metric's tolerance 1e-8 from its initial state.  value: droplet
    cell-steps/s."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as OR
    model, ncpu = host_cpu()
    threads = OR.threads()
    c1 = W.capillary()
    o = OR.Oracle(c1["grid"], c1["params"], W.default_opts(1e-10))
    lat1, nv1 = [], []
    for _ in range(c1_repeats):
        o.set_state(c1["state"]["c"])
        t0 = time.perf_counter()
        assert o.step(c1["dt"]) == OR.OK
        lat1.append(time.perf_counter() - t0)
        nv1.append(o.stats()[0])
    # the same step on one thread (the oracle's arithmetic does not depend on
    # the thread count)
    OR.threads(1)
    o.set_state(c1["state"]["c"])
    t0 = time.perf_counter()
    assert o.step(c1["dt"]) == OR.OK
    t1s = time.perf_counter() - t0
    OR.threads(threads)
    c2 = W.rising_drop()
    o = OR.Oracle(c2["grid"], c2["params"], dict(W.default_opts(1e-8), accel=ACCEL))
    o.set_state(c2["state"]["c"])
    t0 = time.perf_counter()
    nv2 = []
    for _ in range(c2_steps):
        assert o.step(c2["dt"]) == OR.OK
        nv2.append(o.stats()[0])
    t2 = time.perf_counter() - t0
    cells = c2["grid"]["m1"] * c2["grid"]["m2"]
    return {"value": cells * c2_steps / t2, "unit": "cell-steps/s", "cores": threads, "kind": "oracle",
            "cpu": model, "cpus_available": ncpu,
            "sample": "FP64 C oracle on %d OpenMP threads of a %s (%d cpus available): %d full steps of the %dx%d "
                      "droplet from its initial state at tol 1e-8 (%.2f s, %s V-cycles), and the capillary 32x64 "
                      "step at tol 1e-10 in full, %d times (%s V-cycles)"
                      % (threads, model, ncpu, c2_steps, c2["grid"]["m1"], c2["grid"]["m2"], t2, nv2, c1_repeats,
                         nv1),
            "capillary_32x64": {"p50_ms": 1e3 * float(np.percentile(lat1, 50)),
                                "cell_steps_per_s": 2048 / float(np.mean(lat1)),
                                "single_thread_ms": 1e3 * t1s},
            "rising_drop_256x512": {"s_per_step": t2 / c2_steps, "vcycles": nv2}}


def note(*a):
    """progress on stderr (the JSON line is the only stdout output)"""
    print(*a, file=sys.stderr, flush=True)


def timed_steps(g, cfg, steps):
    """K steps from the configuration's initial state; wall seconds, per-step
    latencies, V-cycle counts"""
    g.set_state(cfg["state"]["c"])
    g.synchronize()
    lat, nv = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        g.step(cfg["dt"])
        lat.append(time.perf_counter() - ts)
        nv.append(g.stats()["vcycles"])
    g.synchronize()
    return time.perf_counter() - t0, lat, nv


def timed_then_profiled(g, cfg, steps):
    """the steps timed as they run, then the same steps again with the finest
    smoother's launches carrying HIP events (which take longer to issue):
    wall seconds, latencies and V-cycle counts of the first pass, timed
    launches and their milliseconds of the second"""
    el, lat, nv = timed_steps(g, cfg, steps)
    g.profile(1)
    timed_steps(g, cfg, steps)
    launches, kms = g.profile_read()
    g.profile(0)
    return el, lat, nv, launches, kms


def run_mixed(steps, tol):
    """Rayleigh-Taylor 512 x 2048: FP64 against mixed precision, same steps"""
    cfg = W.rayleigh_taylor()
    cells = cfg["grid"]["m1"] * cfg["grid"]["m2"]
    out = {"workload": cfg["name"], "steps": steps, "tol": tol}
    res = {}
    for name, prec in (("fp64", Q.FP64), ("mixed", Q.MIXED)):
        note("mixed-precision comparison:", cfg["name"], name, steps, "steps")
        g = Q.Solver(cfg["grid"], cfg["params"], dict(base_opts(tol), precision=prec))
        g.set_state(cfg["state"]["c"])
        g.step(cfg["dt"])  # warm-up
        g.set_state(cfg["state"]["c"])
        m0, e0 = g.mass(), g.energy()
        el, lat, nv, launches, kms = timed_then_profiled(g, cfg, steps)
        m1, e1 = g.mass(), g.energy()
        res[name] = (g.get_state(), e1)
        bpc = 0.5 * (MX_SWEEP_B if prec == Q.MIXED else SWEEP_B[True])
        avg_ms = kms / max(launches, 1)
        out[name] = {"cell_steps_per_s": cells * steps / el, "ms_per_step": 1e3 * el / steps,
                     "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                     "vcycles_per_step": float(np.mean(nv)),
                     "mass_drift": float(np.abs(m1 - m0).max() / np.abs(m0).max()),
                     "energy_first_last": [float(e0[0]), float(e1[0])],
                     "finest_halfsweep_us": 1e3 * avg_ms,
                     "finest_halfsweep_GBps": bpc * cells / (avg_ms * 1e-3) / 1e9}
        del g
    out["speedup_mixed_vs_fp64"] = out["mixed"]["cell_steps_per_s"] / out["fp64"]["cell_steps_per_s"]
    a, b = res["mixed"][0], res["fp64"][0]
    out["mixed_vs_fp64_rel_err"] = {k: float(np.abs(a[k] - b[k]).max() / max(np.abs(b[k]).max(), 1e-300))
                                    for k in ("c", "mu", "p", "u", "v")}
    out["mixed_vs_fp64_rel_err"]["energy"] = float(abs(res["mixed"][1][0] - res["fp64"][1][0]) / abs(res["fp64"][1][0]))
    return out


# the paper's own timings of the primitive method (Table 2: average CPU time
# per time step on the convergence test of sec. 9, one desktop with a 4.0 GHz
# AMD FX-8350; thread count, physical parameters and multigrid tolerance not
# stated): context for the GPU's time per step on the same grids, not a target
PAPER_TABLE2_S_PER_STEP = {16: 2.913e-2, 32: 1.659e-1, 64: 2.659e-1, 128: 1.027, 256: 2.622}


def run_paper_table2(steps=20):
    """the convergence-study workload of sec. 9 (walls, the bounded initial
    condition, density ratio 3, dt = (1/16)(16/m)^2) on the grids of the
    paper's Table 2, FP64 to 1e-8: GPU seconds per step beside the paper's CPU
    seconds per step"""
    out = {"source": "Table 2 of the paper: primitive method, average CPU time per step on the convergence "
                     "test of sec. 9, one 4.0 GHz AMD FX-8350 desktop (threads, parameters and tolerance not "
                     "stated); the GPU runs this repository's reading of that workload (its printed initial "
                     "condition crosses the density pole), FP64, tol 1e-8, %d steps from the initial state" % steps,
           "grids": {}}
    for m in sorted(PAPER_TABLE2_S_PER_STEP):
        cfg = W.convergence_case(m)
        note("paper Table 2 grid:", cfg["name"], steps, "steps")
        g = Q.Solver(cfg["grid"], cfg["params"], base_opts(1e-8))
        g.set_state(cfg["state"]["c"])
        g.step(cfg["dt"])
        g.set_state(cfg["state"]["c"])
        g.synchronize()
        nv = []
        t0 = time.perf_counter()
        for _ in range(steps):
            g.step(cfg["dt"])
            nv.append(g.stats()["vcycles"])
        g.synchronize()
        s_gpu = (time.perf_counter() - t0) / steps
        s_cpu = PAPER_TABLE2_S_PER_STEP[m]
        out["grids"]["%dx%d" % (m, m)] = {"gpu_s_per_step": s_gpu, "gpu_vcycles_per_step": float(np.mean(nv)),
                                          "paper_cpu_s_per_step": s_cpu, "paper_cpu_cell_steps_per_s": m * m / s_cpu,
                                          "gpu_cell_steps_per_s": m * m / s_gpu, "ratio": s_cpu / s_gpu}
        del g
    return out


def run_capillary(repeats=100, warmup=3):
    """capillary 32 x 64 (periodic in x, walls in y, 4 levels), FP64 to a
    residual of 1e-10: the same step from the same state `repeats` times after
    `warmup` untimed ones; latency percentiles of one step"""
    cfg = W.capillary()
    note("capillary:", cfg["name"], repeats, "repeats of one step")
    g = Q.Solver(cfg["grid"], cfg["params"], base_opts(1e-10))
    lat, nv = [], []
    for k in range(warmup + repeats):
        g.set_state(cfg["state"]["c"])
        g.synchronize()
        t0 = time.perf_counter()
        g.step(cfg["dt"])
        t = time.perf_counter() - t0
        if k >= warmup:
            lat.append(t)
            nv.append(g.stats()["vcycles"])
    cells = cfg["grid"]["m1"] * cfg["grid"]["m2"]
    return {"workload": cfg["name"], "precision": "fp64", "tol": 1e-10, "levels": g.levels, "repeats": repeats,
            "warmup": warmup, "p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)), "mean_ms": 1e3 * float(np.mean(lat)),
            "cell_steps_per_s": cells / float(np.mean(lat)), "vcycles_per_step": float(np.mean(nv))}


def run_paper_smoother(steps, warmup, tol, primitive_value):
    """the droplet with the smoother of sec. 7.1 as printed (the Newton step
    on (c, mubar), then the Vanka box) and plain V-cycles (no acceleration):
    what the coupled box and the acceleration buy"""
    cfg = W.rising_drop()
    cells = cfg["grid"]["m1"] * cfg["grid"]["m2"]
    note("paper's smoother:", cfg["name"], steps, "steps")
    g = Q.Solver(cfg["grid"], cfg["params"], dict(base_opts(tol), smoother=W.SMOOTH_SEGREGATED, accel=0))
    g.set_state(cfg["state"]["c"])
    for _ in range(warmup):
        g.step(cfg["dt"])
    el, lat, nv, launches, kms = timed_then_profiled(g, cfg, steps)
    value = cells * steps / el
    avg_ms = kms / max(launches, 1)
    return {"workload": cfg["name"], "smoother": "segregated (sec. 7.1)", "accel": 0, "steps": steps, "tol": tol,
            "cell_steps_per_s": value, "ms_per_step": 1e3 * el / steps,
            "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
            "vcycles_per_step": float(np.mean(nv)), "headline_speedup_over_it": primitive_value / value,
            "finest_halfsweep_us": 1e3 * avg_ms,
            "finest_halfsweep_GBps": 0.5 * SWEEP_B[True] * cells / (avg_ms * 1e-3) / 1e9}


def run_projection(steps, warmup, tol, primitive_value):
    """the same droplet workload in the projection scheme of sec. 6.2 (FP64):
    throughput against the primitive scheme, V-cycles, the finest smoother's
    launch time, total-mass drift and the energy law over the timed steps"""
    cfg = W.rising_drop()
    cells = cfg["grid"]["m1"] * cfg["grid"]["m2"]
    note("projection scheme:", cfg["name"], steps, "steps")
    g = Q.Solver(cfg["grid"], cfg["params"], dict(base_opts(tol), scheme=Q.PROJECTION))
    g.set_state(cfg["state"]["c"])
    for _ in range(warmup):
        g.step(cfg["dt"])
    el, lat, nv, launches, kms = timed_then_profiled(g, cfg, steps)
    # untimed: mass and the energy law E^{n+1} - E^n + D = 0 step by step
    g.set_state(cfg["state"]["c"])
    m0 = g.mass()
    law = 0.0
    for _ in range(5):
        e0 = g.energy()[0]
        g.step(cfg["dt"])
        law = max(law, abs(g.energy()[0] - e0 + g.dissipation().sum()))
    drift = abs(g.mass().sum() - m0.sum()) / abs(m0.sum())
    value = cells * steps / el
    return {"workload": cfg["name"], "scheme": "projection (sec. 6.2)", "steps": steps, "tol": tol,
            "cell_steps_per_s": value, "ms_per_step": 1e3 * el / steps,
            "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
            "vcycles_per_step": float(np.mean(nv)), "speedup_vs_primitive": value / primitive_value,
            "finest_halfsweep_us": 1e3 * kms / max(launches, 1),
            "total_mass_drift_5_steps": drift, "energy_law_max_abs_5_steps": law}


# Served requests run plain cycles: in launches batched over many requests the
# step is throughput-bound, and the acceleration's recording and combination
# traffic costs more than the cycles it saves on these droplets (3 % less
# throughput measured with depth 2); requests run alone are latency-bound and
# keep the default acceleration.
SERVED_ACCEL = 0


def run_served(n, nsteps, tol, seq_steps, lanes):
    """the request stream through the server (mixed precision), and the same
    requests one after another alone (FP64 and mixed) on a sample of steps"""
    reqs = W.serving_requests(n=n, nsteps=nsteps)
    mixed = dict(base_opts(tol), precision=Q.MIXED)
    fp64 = base_opts(tol)
    served = dict(mixed, accel=SERVED_ACCEL)
    # sequential baselines: every request alone for all its steps (the first
    # steps of a request take the most cycles, so a shorter sample would
    # overstate the sequential time)
    seq = {"fp64": float("nan"), "mixed": float("nan")}
    for name, opts in (("fp64", fp64), ("mixed", mixed)) if seq_steps else ():
        note("serving: sequential baseline", name)
        cs, t = 0.0, 0.0
        for r in reqs:
            w = r["work"]
            g = Q.Solver(w["grid"], w["params"], opts)
            g.set_state(w["state"]["c"])
            g.synchronize()
            t0 = time.perf_counter()
            for _ in range(seq_steps):
                g.step(w["dt"])
            g.synchronize()
            t += time.perf_counter() - t0
            cs += w["grid"]["m1"] * w["grid"]["m2"] * seq_steps
            del g
        seq[name] = cs / t
    def serve(burst):
        note("serving: %d requests through the server%s" % (n, ", all at once" if burst else ""))
        srv = Q.Server(hbm_budget=64 << 30, max_slots=n, lanes=lanes)
        t0 = time.perf_counter()
        k = 0
        while True:
            now = time.perf_counter() - t0
            while k < len(reqs) and (burst or reqs[k]["arrival"] <= now):
                w = reqs[k]["work"]
                srv.submit(w["grid"], w["params"], served, w["state"]["c"], reqs[k]["nsteps"], w["dt"])
                k += 1
            left = srv.progress(32)
            if left == 0 and k == len(reqs):
                break
            if left == 0:
                time.sleep(min(1e-3, max(0.0, reqs[k]["arrival"] - (time.perf_counter() - t0))))
        st = srv.stats()
        del srv
        return st

    s = serve(False)
    b = serve(True)
    return {"workload": "%d rising-droplet requests, sizes 64x128..512x1024, Poisson 20/s, %d steps each, mixed "
                        "precision, tol %g" % (n, nsteps, tol),
            "lanes": lanes, "accel_served": SERVED_ACCEL, "accel_sequential": ACCEL,
            "cell_steps_per_s": s["cell_steps_per_s"], "p50_step_ms": s["p50_ms"], "p99_step_ms": s["p99_ms"],
            "wall_s": s["wall_s"], "steps": int(s["steps"]), "launches": int(s["launches"]),
            "contexts_created": int(s["contexts_created"]),
            "host_ms": {"admit": s["host_admit_ms"], "finish": s["host_finish_ms"], "wait": s["host_wait_ms"]},
            "sequential_fp64_cell_steps_per_s": seq["fp64"], "sequential_mixed_cell_steps_per_s": seq["mixed"],
            "sequential_sample": "each request alone, %d steps from its initial state" % seq_steps,
            "speedup_vs_sequential_fp64": s["cell_steps_per_s"] / seq["fp64"],
            "speedup_vs_sequential_mixed": s["cell_steps_per_s"] / seq["mixed"],
            # the stream above is paced by its arrivals (the last one at ~2.2 s);
            # the same requests submitted at once show the server's capacity
            "burst": {"cell_steps_per_s": b["cell_steps_per_s"], "wall_s": b["wall_s"], "p50_step_ms": b["p50_ms"],
                      "p99_step_ms": b["p99_ms"], "launches": int(b["launches"]),
                      "speedup_vs_sequential_fp64": b["cell_steps_per_s"] / seq["fp64"],
                      "speedup_vs_sequential_mixed": b["cell_steps_per_s"] / seq["mixed"]}}


def run_served_at_scale(nbig, big, nsteps, tol, lanes, max_vcycles):
    """nbig periodic drop boxes of big x big cells submitted at once, with a
    Poisson background stream of 256 x 256 boxes while they run, through the
    server in mixed precision; the plain-FP64 sequential baseline is each kind
    of request alone for all its steps (one big box, one background box; the
    first steps of a box take the most cycles, so a shorter sample would
    overstate the sequential time)"""
    bigs, bg = W.serving_at_scale(nbig=nbig, big=big, nsteps=nsteps)
    mixed = dict(base_opts(tol), precision=Q.MIXED, max_vcycles=max_vcycles)
    fp64 = dict(base_opts(tol), max_vcycles=max_vcycles)
    seq = {}
    for name, r, k in (("big", bigs[0], nsteps), ("background", next(W.serving_at_scale(1, 64, nsteps)[1]), nsteps)):
        note("serving at scale: sequential FP64 baseline,", name)
        w = r["work"]
        g = Q.Solver(w["grid"], w["params"], fp64)
        g.set_state(w["state"]["c"])
        g.step(w["dt"])
        g.set_state(w["state"]["c"])
        g.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            g.step(w["dt"])
        g.synchronize()
        seq[name] = w["grid"]["m1"] * w["grid"]["m2"] * k / (time.perf_counter() - t0)
        del g
    note("serving at scale: %d boxes of %dx%d with a background stream" % (nbig, big, big))
    srv = Q.Server(hbm_budget=128 << 30, max_slots=nbig + 64, lanes=lanes)
    ids_big = [srv.submit(r["work"]["grid"], r["work"]["params"], mixed, r["work"]["state"]["c"], r["nsteps"],
                          r["work"]["dt"]) for r in bigs]
    ids_bg, shapes = [], {}
    nxt = next(bg)
    t0 = time.perf_counter()
    while True:
        now = time.perf_counter() - t0
        while nxt["arrival"] <= now:
            w = nxt["work"]
            ids_bg.append(srv.submit(w["grid"], w["params"], mixed, w["state"]["c"], nxt["nsteps"], w["dt"]))
            nxt = next(bg)
        srv.progress(32)
        if all(srv.poll(i)[0] == 2 for i in ids_big):
            break
    # let the background requests already admitted finish; stop arrivals
    while srv.progress(32) > 0:
        pass
    s = srv.stats()
    rb = [srv.result(i) for i in ids_big]
    rg = [srv.result(i) for i in ids_bg]
    big_cells = big * big * nsteps * nbig
    bg_cells = sum(256 * 256 * nsteps for _ in rg)
    seq_s = big_cells / seq["big"] + bg_cells / seq["background"]
    return {"workload": "%d periodic %dx%d boxes with 40 drops (density ratio 100) at t=0 + 256x256 5-drop boxes "
                        "arriving Poisson 20/s, %d steps each, mixed precision, tol %g, at most %d V-cycles"
                        % (nbig, big, big, nsteps, tol, max_vcycles),
            "lanes": lanes, "status_ok": all(r["status"] == Q.OK for r in rb + rg),
            "cell_steps_per_s": s["cell_steps_per_s"], "wall_s": s["wall_s"], "steps": int(s["steps"]),
            "p50_step_ms": s["p50_ms"], "p99_step_ms": s["p99_ms"],
            "big_done_s": max(r["total_ms"] for r in rb) / 1e3,
            "background_requests": len(rg),
            "background_p50_total_ms": float(np.percentile([r["total_ms"] for r in rg], 50)) if rg else None,
            "background_p99_total_ms": float(np.percentile([r["total_ms"] for r in rg], 99)) if rg else None,
            "mass_drift_max": float(max(np.abs(r["mass"][-1] - r["mass"][0]).max() / np.abs(r["mass"][0]).max()
                                        for r in rb + rg)),
            "vcycles_per_step_big": float(np.mean([r["vcycles"].mean() for r in rb])),
            "sequential_fp64_estimate_s": seq_s,
            "speedup_vs_sequential_fp64": seq_s / s["wall_s"] if s["wall_s"] > 0 else None,
            "sequential_sample": "one %dx%d box and one background box alone for %d steps each, FP64"
                                 % (big, big, nsteps)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--accel", type=int, default=2, help="acceleration depth of the cycle iteration (0 = plain cycles)")
    ap.add_argument("--blocking", type=int, default=None,
                    help="temporal blocking of the smoothing: 0 off, 1 coarse levels, 2 all (default: the library's)")
    ap.add_argument("--mixed-steps", type=int, default=200)
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=50)
    ap.add_argument("--serve-lanes", type=int, default=3)
    ap.add_argument("--no-seq", action="store_true", help="skip the sequential baselines of the served run")
    ap.add_argument("--no-serve-scale", action="store_true", help="skip the serving-at-scale workload")
    ap.add_argument("--scale-boxes", type=int, default=16)
    ap.add_argument("--scale-size", type=int, default=2048)
    ap.add_argument("--scale-steps", type=int, default=20)
    ap.add_argument("--scale-max-vcycles", type=int, default=150)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-projection", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-capillary", action="store_true")
    ap.add_argument("--no-paper-smoother", action="store_true")
    ap.add_argument("--no-paper-table2", action="store_true")
    ap.add_argument("--event-pass-only", action="store_true",
                    help="skip the plain timed pass (for a profiler's trace of the event-timed pass alone, "
                         "whose kernel averages the roofline uses); value is then the event pass's rate")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the time step of one simulation is a single-GPU "
              "kernel pipeline here (how it would shard over several GPUs is documented, not built)", file=sys.stderr)
        sys.exit(2)

    cfg = W.rising_drop()
    global ACCEL, BLOCKING
    ACCEL = args.accel
    BLOCKING = args.blocking
    opts = base_opts(args.tol)
    g = Q.Solver(cfg["grid"], cfg["params"], dict(opts, precision=Q.FP64))
    cells = cfg["grid"]["m1"] * cfg["grid"]["m2"]
    lc = level_cells(cfg, g.levels)
    copy_gbs, _ = Q.copy_probe(64 << 20, 10)  # 512 MiB copy: calibration and sanity figure

    # which kernel dominates the step: every launch of two untimed steps
    # bracketed by events, grouped by kernel
    note("main: breakdown of", cfg["name"])
    g.set_state(cfg["state"]["c"])
    for _ in range(args.warmup):
        g.step(cfg["dt"])
    g.set_state(cfg["state"]["c"])
    g.profile(2)
    nv_bd = []
    for _ in range(2):
        g.step(cfg["dt"])
        nv_bd.append(g.stats()["vcycles"])
    bd = g.profile_breakdown(by_level=True)
    g.profile(0)
    ktab = kernel_table(bd, lc, opts)
    smoothers = [k for k in ktab if ktab[k]["alg_bytes"] is not None]
    dominant = max(smoothers, key=lambda k: ktab[k]["ms"])
    # the finest level's smoothing kernel: fused sweeps where blocking covers
    # the finest level, else the half-sweeps
    finest = "k_halfsweep_fine" if ("halfsweep", 0) in bd else "k_hs_fused"
    timed_ops = sorted(ktab[dominant]["ops"] | (ktab[finest]["ops"] if finest in ktab else set()))

    # the timed region: the steps as they run for any caller
    note("main:", cfg["name"], args.steps, "steps")
    g.set_state(cfg["state"]["c"])
    for _ in range(args.warmup):
        g.step(cfg["dt"])
    if not args.event_pass_only:
        elapsed, lat, nv = timed_steps(g, cfg, args.steps)
    # the kernels' durations: the same steps again, the launches of the
    # dominant and the finest smoothing kernels carrying HIP events (the
    # kernel's own start and end; such launches take longer to issue, which
    # the timed region above does not pay)
    note("main: the same", args.steps, "steps; launches of", dominant, "and", finest, "carry HIP events")
    g.profile_ops(timed_ops)
    elapsed_direct, lat_direct, nv_direct = timed_steps(g, cfg, args.steps)
    tbd = g.profile_breakdown(by_level=True)
    g.profile(0)
    if args.event_pass_only:
        elapsed, lat, nv = elapsed_direct, lat_direct, nv_direct
    value = cells * args.steps / elapsed
    ttab = kernel_table(tbd, lc, opts)

    def roof(k):
        e = ttab[k]
        avg_us = 1e3 * e["ms"] / e["launches"]
        per_launch = e["alg_bytes"] / e["launches"]
        ach = e["alg_bytes"] / (e["ms"] * 1e-3) / 1e9
        tr = traffic_from_profile(k)
        r = {"bound": "hbm", "kernel": k, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": ach / HBM_PEAK_GBS, "traffic": tr, "traffic_vs_algorithmic": tr / per_launch if tr else None,
             "launches": e["launches"], "avg_launch_us": avg_us, "alg_bytes_per_launch": per_launch,
             "levels": sorted({lev for (op, lev) in tbd if kernel_of(op, lev) == k})}
        v = valu_from_profile(k, avg_us)
        if v:
            r["valu"] = v
        return r

    rf = roof(dominant)
    rf["share_of_step"] = ktab[dominant]["ms"] / sum(e["ms"] for e in ktab.values())
    if finest != dominant and finest in ttab:
        rf["finest"] = roof(finest)
    # the whole step against the same bytes: the algorithmic bytes of every
    # operation of the two breakdown steps per V-cycle, times the timed
    # steps' mean V-cycle count, over the timed ms_per_step
    per_cycle = sum(e["alg_bytes"] for e in ktab.values() if e["alg_bytes"] is not None) / max(1, sum(nv_bd))
    step_bytes = per_cycle * float(np.mean(nv))
    ms_step = 1e3 * elapsed / args.steps
    rf["step"] = {"alg_bytes_per_vcycle": per_cycle, "alg_bytes_per_finest_cell_per_vcycle": per_cycle / cells,
                  "alg_bytes_per_step": step_bytes, "alg_GBps": step_bytes / (ms_step * 1e-3) / 1e9,
                  "frac": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS}
    tot = sum(e["ms"] for e in ktab.values())
    kernels = {k: {"launches": e["launches"], "ms_per_step": e["ms"] / 2.0, "share": e["ms"] / tot,
                   "avg_us": 1e3 * e["ms"] / e["launches"],
                   "alg_GBps": (e["alg_bytes"] / (e["ms"] * 1e-3) / 1e9) if e["alg_bytes"] else None}
               for k, e in sorted(ktab.items(), key=lambda kv: -kv[1]["ms"])}
    out = {
        "metric": METRIC, "value": value, "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": [cfg["grid"]["m1"], cfg["grid"]["m2"]], "levels": g.levels,
                   "dt": cfg["dt"], "tol": args.tol, "precision": "fp64", "cycle": "V(2,2)", "accel": ACCEL,
                   "parallelism": "none"},
        "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "vcycles_per_step": float(np.mean(nv)),
        "timed_region": "event pass (profiling run)" if args.event_pass_only else "plain steps",
        "event_timed_pass": {"ms_per_step": 1e3 * elapsed_direct / args.steps,
                             "vcycles_per_step": float(np.mean(nv_direct))},
        "roofline": rf,
        "copy_probe_GBps": copy_gbs,
        "step_breakdown": kernels,
        "kernel_launches_per_vcycle": sum(n * KERNELS_PER_OP.get(op, 1) for (op, lev), (n, _) in bd.items())
                                      / max(1, sum(nv_bd)),
    }
    del g
    if not args.no_capillary:
        out["capillary"] = run_capillary()
    if not args.no_paper_smoother:
        out["paper_smoother"] = run_paper_smoother(min(args.steps, 30), args.warmup, args.tol, value)
    if not args.no_paper_table2:
        out["paper_table2"] = run_paper_table2()
    if not args.no_projection:
        out["projection"] = run_projection(args.steps, args.warmup, args.tol, value)
    if not args.no_mixed:
        out["mixed"] = run_mixed(args.mixed_steps, args.tol)
    if not args.no_serve:
        out["served"] = run_served(args.serve_requests, args.serve_steps, args.tol, seq_steps=0 if args.no_seq else args.serve_steps,
                                   lanes=args.serve_lanes)
    if not args.no_serve_scale:
        out["served_at_scale"] = run_served_at_scale(args.scale_boxes, args.scale_size, args.scale_steps, args.tol,
                                                     args.serve_lanes, args.scale_max_vcycles)
    if not args.no_cpu_baseline:
        note("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
