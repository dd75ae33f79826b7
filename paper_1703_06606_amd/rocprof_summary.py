"""Summaries of rocprofv3 runs of bench.py for one kernel and workload.

Reads the CSV output of three rocprofv3 runs of the same bench command
(``--kernel-trace --stats``, ``--pmc FETCH_SIZE``, ``--pmc WRITE_SIZE``, each
``-f csv -d <dir>``) and writes, for each named kernel:

* ``<kernel>_<workload>.md``: the trace statistics of the kernel per grid
  size (one grid size per level), the kernel's average duration over all its
  dispatches, its HBM bytes per dispatch from the counters, and the table of
  every kernel of the run by total time;
* ``<kernel>_<workload>_traffic.txt``: ``hbm_bytes_per_launch`` (mean over
  the kernel's dispatches of FETCH_SIZE and WRITE_SIZE, KiB, each scaled by
  what the counter reads for the copy-probe kernel that bench.py runs first:
  it reads and writes 512 MiB), and the hash of the device code the counters
  were taken on (bench.py ignores a summary of other device code);
* with ``--busy-tail SECONDS``, ``busy_<workload>.md``: the share of the
  last SECONDS of kernel activity in which some kernel ran, and the kernels
  of that window;
* with ``--valu DIR`` (a ``--pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VALU_ADD_F64
  SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64`` run),
  ``<kernel>_<workload>_valu.txt``: waves, vector-ALU wave instructions and
  FP64 wave instructions per dispatch (means over the kernel's dispatches)
  and the FP64 flops they execute with every lane counted.

Usage: python -m paper_1703_06606_amd.rocprof_summary [--trace DIR --fetch DIR
--write DIR] [--valu DIR] --workload NAME --out DIR --command "..." KERNEL
[KERNEL ...]
"""
import argparse
import csv
import glob
import os
import re
import statistics

from paper_1703_06606_amd.build import device_source_hash

COPY_BYTES = 64 << 23  # k_copy_probe: 64 Mi doubles read and as many written


def _rows(d, suffix):
    out = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def _name(row):
    return row.get("Kernel_Name") or row.get("Name") or ""


def _match(kernel):
    return re.compile(r"\b%s\b(?!_)" % re.escape(kernel))


def _grid(row):
    for k in ("Grid_Size", "Grid_Size_X"):
        if row.get(k):
            g = int(row[k])
            for k2 in ("Grid_Size_Y", "Grid_Size_Z"):
                if row.get(k2):
                    g *= int(row[k2])
            return g
    return 0


def short(name):
    m = re.search(r"\b(k_[a-z0-9_]+)", name)
    return m.group(1) if m else name


def counters(d, counter):
    """{dispatch id: (kernel name, grid, value)} of one counter"""
    out = {}
    for r in _rows(d, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        key = (r.get("Process_Id"), r.get("Dispatch_Id"))
        v = float(r["Counter_Value"])
        if key in out:
            out[key] = (out[key][0], out[key][1], out[key][2] + v)
        else:
            out[key] = (_name(r), _grid(r), v)
    return out


def copy_scale(c, factor_bytes):
    vals = [v for (n, g, v) in c.values() if _match("k_copy_probe").search(n)]
    if not vals:
        return None
    return factor_bytes / (statistics.median(vals) * 1024.0)


VALU_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64",
                 "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64")


def valu_summaries(a):
    c = {n: counters(a.valu, n) for n in VALU_COUNTERS}
    h = device_source_hash()
    for kern in a.kernels:
        rx = _match(kern)
        m = {n: [v for (name, g, v) in c[n].values() if rx.search(name)] for n in VALU_COUNTERS}
        if not all(m.values()):
            continue
        mean = {n: statistics.mean(v) for n, v in m.items()}
        f64 = mean["SQ_INSTS_VALU_ADD_F64"] + mean["SQ_INSTS_VALU_MUL_F64"] + mean["SQ_INSTS_VALU_FMA_F64"] \
            + mean["SQ_INSTS_VALU_TRANS_F64"]
        flops = 64.0 * (mean["SQ_INSTS_VALU_ADD_F64"] + mean["SQ_INSTS_VALU_MUL_F64"]
                        + 2.0 * mean["SQ_INSTS_VALU_FMA_F64"] + mean["SQ_INSTS_VALU_TRANS_F64"])
        with open(os.path.join(a.out, "%s_%s_valu.txt" % (kern, a.workload)), "w") as fh:
            fh.write("# SQ counters of %s on %s, mean per dispatch over %d dispatches (every level);\n"
                     % (kern, a.workload, len(m["SQ_WAVES"])))
            for cmd in a.command:
                fh.write("# command: %s\n" % cmd)
            fh.write("# summarised by: python -m paper_1703_06606_amd.rocprof_summary --valu;\n"
                     "# FP64 flops = 64 lanes x (ADD + MUL + 2 FMA + TRANS wave instructions), every lane counted;\n"
                     "# valid for the device code with this hash\n")
            fh.write("source_hash: %s\nwaves_per_launch: %.0f\nvalu_wave_insts_per_launch: %.0f\n"
                     "valu_wave_insts_per_wave: %.1f\nfp64_wave_insts_per_launch: %.0f\nfp64_flops_per_launch: %.0f\n"
                     "dispatches: %d\n" % (h, mean["SQ_WAVES"], mean["SQ_INSTS_VALU"],
                                          mean["SQ_INSTS_VALU"] / max(mean["SQ_WAVES"], 1.0), f64, flops,
                                          len(m["SQ_WAVES"])))


def busy_summary(a, trace):
    """busy_<workload>.md: the share of the last busy_tail seconds of kernel
    activity in which at least one kernel ran (the union of the kernels'
    intervals), and the kernels of that window"""
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short(_name(r))) for r in trace)
    t1 = max(e for _, e, _ in iv)
    t0 = t1 - int(a.busy_tail * 1e9)
    busy, cur_s, cur_e = 0, None, None
    per = {}
    for s0, e0, k in iv:
        if e0 <= t0:
            continue
        per.setdefault(k, []).append((e0 - s0) * 1e-3)
        s0, e0 = max(s0, t0), min(e0, t1)
        if e0 <= s0:
            continue
        if cur_e is None or s0 > cur_e:
            if cur_e is not None:
                busy += cur_e - cur_s
            cur_s, cur_e = s0, e0
        else:
            cur_e = max(cur_e, e0)
    if cur_e is not None:
        busy += cur_e - cur_s
    n = sum(len(v) for v in per.values())
    lines = ["# kernel activity of %s" % a.workload, ""]
    lines += ["command: `%s`" % c for c in a.command]
    lines += ["summarised by: `python -m paper_1703_06606_amd.rocprof_summary --busy-tail %.3f` (device code %s)"
              % (a.busy_tail, device_source_hash()), "",
              "window: the last %.3f s of kernel activity in the trace" % a.busy_tail,
              "dispatches_in_window: %d" % n,
              "busy_fraction: %.4f (share of the window in which at least one kernel ran)" % (busy / (t1 - t0)), "",
              "| kernel | dispatches | avg us | total ms |", "|---|---|---|---|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        lines.append("| %s | %d | %.2f | %.3f |" % (k, len(v), statistics.mean(v), sum(v) * 1e-3))
    with open(os.path.join(a.out, "busy_%s.md" % a.workload), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--valu", help="directory of the SQ counter run (see above)")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", action="append", default=[], help="commands that made the runs (repeatable)")
    ap.add_argument("--busy-tail", type=float, default=0.0,
                    help="also report the share of the last SECONDS of kernel activity in which some kernel ran")
    ap.add_argument("kernels", nargs="*")
    a = ap.parse_args()
    os.makedirs(a.out, exist_ok=True)
    if a.valu:
        valu_summaries(a)
    if not a.trace:
        return
    trace = _rows(a.trace, "kernel_trace.csv")
    durs = {}
    for r in trace:
        n = _name(r)
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        durs.setdefault((short(n), _grid(r)), []).append(d)
    if a.busy_tail > 0:
        busy_summary(a, trace)
    if not (a.fetch and a.write and a.kernels):
        return
    fetch, write = counters(a.fetch, "FETCH_SIZE"), counters(a.write, "WRITE_SIZE")
    fs, ws = copy_scale(fetch, COPY_BYTES), copy_scale(write, COPY_BYTES)
    table = sorted(((k, g, len(v), statistics.mean(v), statistics.median(v), min(v), sum(v) * 1e-3)
                    for (k, g), v in durs.items()), key=lambda t: -t[6])
    h = device_source_hash()
    for kern in a.kernels:
        rx = _match(kern)
        mine = [(g, v) for (k, g), v in durs.items() if k == kern]
        alld = [x for _, v in mine for x in v]
        fv = [(g, v) for (n, g, v) in fetch.values() if rx.search(n)]
        wv = [(g, v) for (n, g, v) in write.values() if rx.search(n)]
        lines = ["# %s, %s" % (kern, a.workload), ""]
        lines += ["command: `%s`" % c for c in a.command]
        lines += ["summarised by: `python -m paper_1703_06606_amd.rocprof_summary` (device code %s)" % h, ""]
        if alld:
            lines.append("%s over all its dispatches in the trace run: %d dispatches, average %.2f us, median %.2f us"
                         % (kern, len(alld), statistics.mean(alld), statistics.median(alld)))
        hbm = None
        if fv and wv and fs and ws:
            hbm = statistics.mean(v for _, v in fv) * 1024 * fs + statistics.mean(v for _, v in wv) * 1024 * ws
            lines.append("HBM bytes per dispatch (mean of FETCH_SIZE x %.4f + WRITE_SIZE x %.4f over %d / %d "
                         "dispatches, KiB -> bytes): %.0f" % (fs, ws, len(fv), len(wv), hbm))
        lines += ["", "## %s per grid size (work-items; one per level)" % kern, "",
                  "| grid | dispatches | avg us | median us | FETCH_SIZE KiB | WRITE_SIZE KiB |", "|---|---|---|---|---|---|"]
        for g, v in sorted(mine, key=lambda t: -t[0]):
            f1 = [x for gg, x in fv if gg == g]
            w1 = [x for gg, x in wv if gg == g]
            lines.append("| %d | %d | %.2f | %.2f | %s | %s |" % (
                g, len(v), statistics.mean(v), statistics.median(v),
                "%.0f" % statistics.mean(f1) if f1 else "-", "%.0f" % statistics.mean(w1) if w1 else "-"))
        lines += ["", "## every kernel of the trace run, by total time", "",
                  "| kernel | grid | dispatches | avg us | median us | min us | total ms |", "|---|---|---|---|---|---|---|"]
        for k, g, n, av, med, mn, tot in table:
            lines.append("| %s | %d | %d | %.2f | %.2f | %.2f | %.3f |" % (k, g, n, av, med, mn, tot))
        if fs and ws:
            lines += ["", "counter calibration: k_copy_probe reads and writes %d bytes; FETCH_SIZE scale %.4f, "
                      "WRITE_SIZE scale %.4f" % (COPY_BYTES, fs, ws)]
        with open(os.path.join(a.out, "%s_%s.md" % (kern, a.workload)), "w") as fh:
            fh.write("\n".join(lines) + "\n")
        if hbm is not None:
            with open(os.path.join(a.out, "%s_%s_traffic.txt" % (kern, a.workload)), "w") as fh:
                fh.write("# HBM bytes per dispatch of %s on %s, mean over its dispatches (every level), FETCH_SIZE\n"
                         "# and WRITE_SIZE copy-kernel scaled; from the runs of %s_%s.md;\n"
                         "# valid for the device code with this hash\n" % (kern, a.workload, kern, a.workload))
                fh.write("source_hash: %s\nhbm_bytes_per_launch: %.0f\nfetch_scale: %.4f\nwrite_scale: %.4f\n"
                         "dispatches: %d\n" % (h, hbm, fs, ws, len(fv)))


if __name__ == "__main__":
    main()
