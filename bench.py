#!/usr/bin/env python3
"""Benchmark of the multigrid time step on one MI355X.

Workload: the 256 x 512 rising droplet on [0,1] x [0,2] (walls on all sides,
density ratio 10, viscosity ratio 10, Re = 35, We = 10, Fr = 1, eps = 0.01,
dt = 5e-4, 7 multigrid levels), FP64, each step solved to a residual of 1e-8.
A step is one call of qnsch_step (all V-cycles of the time step).  The timed
region starts from the initial droplet after W untimed warm-up steps, with all
inputs resident in HBM, and covers exactly K steps.

Prints one JSON line: cell-steps/s, p50/p99 step latency, the roofline of the
finest-level half-sweep kernel (HIP-event timing of its launches inside the
timed region) and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
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
# algorithmic bytes of one half-sweep launch per cell of the level: it reads
# the five unknowns and the three time-n fields of every cell (the stencils of
# the cells of one colour cover all cells), writes c, mubar, pbar of the half
# of the cells it relaxes and both face velocities of every face (ping-pong)
HALFSWEEP_BYTES_PER_CELL = 8 * 8 + 3 * 8 / 2 + 2 * 8
KERNEL = "k_halfsweep_fine"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_halfsweep_fine_rising_drop_256x512_traffic.txt")
SOURCES = [os.path.join(ROOT, "paper_1703_06606_amd", "csrc", f) for f in ("qnsch_dev.hpp", "qnsch_kern.hpp", "qnsch_lib.hip")]


def source_hash():
    h = hashlib.sha256()
    for f in SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per launch of the kernel from the committed counter summary,
    only if it was taken on the current kernel source"""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(cfg, opts, vcycles_per_step):
    """The FP64 oracle as it stands, single-threaded, on a bounded sample of
    the same workload: one residual evaluation and one V-cycle of the first
    step, extrapolated to a step with the mean V-cycle count of the GPU run
    (same algorithm, same count)."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as OR
    o = OR.Oracle(cfg["grid"], cfg["params"], opts)
    o.set_state(cfg["state"]["c"])
    o.begin_step(cfg["dt"])
    t0 = time.perf_counter()
    o.residual()
    t_res = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.vcycle()
    t_vc = time.perf_counter() - t0
    t_step = t_res + vcycles_per_step * (t_vc + t_res)
    cells = cfg["grid"]["m1"] * cfg["grid"]["m2"]
    return {"value": cells / t_step, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
            "sample": "one residual (%.2f s) and one V-cycle (%.2f s) of the first %dx%d step on the FP64 C oracle, "
                      "single thread, extrapolated to %.2f V-cycles per step (the GPU run's mean)"
                      % (t_res, t_vc, cfg["grid"]["m1"], cfg["grid"]["m2"], vcycles_per_step)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the time step of one simulation is a single-GPU "
              "kernel pipeline here (multi-GPU sharding is described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    cfg = W.rising_drop()
    opts = W.default_opts(args.tol)
    g = Q.Solver(cfg["grid"], cfg["params"], dict(opts, precision=Q.FP64))
    cells = cfg["grid"]["m1"] * cfg["grid"]["m2"]
    c0 = cfg["state"]["c"]
    copy_gbs, _ = Q.copy_probe(64 << 20, 10)  # 512 MiB copy: calibration and sanity figure

    g.set_state(c0)
    for _ in range(args.warmup):
        g.step(cfg["dt"])
    g.set_state(c0)
    g.synchronize()
    g.profile(True)
    lat, nv = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        g.step(cfg["dt"])
        lat.append(time.perf_counter() - ts)
        nv.append(g.stats()["vcycles"])
    g.synchronize()
    elapsed = time.perf_counter() - t0
    launches, kms = g.profile_read()
    g.profile(False)

    value = cells * args.steps / elapsed
    avg_ms = kms / max(launches, 1)
    alg_bytes = HALFSWEEP_BYTES_PER_CELL * cells
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": [cfg["grid"]["m1"], cfg["grid"]["m2"]], "levels": g.levels,
                   "dt": cfg["dt"], "tol": args.tol, "precision": "fp64", "cycle": "V(2,2)",
                   "parallelism": "none"},
        "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "vcycles_per_step": float(np.mean(nv)),
        "roofline": {"bound": "hbm", "kernel": KERNEL, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profile(),
                     "launches": launches, "avg_launch_us": 1e3 * avg_ms,
                     "alg_bytes_per_launch": alg_bytes},
        "copy_probe_GBps": copy_gbs,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, opts, float(np.mean(nv)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
