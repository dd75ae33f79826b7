"""Host logic of the measurement (CPU only): the algorithmic byte counts
bench.py divides by kernel time (per launch, per level, per kernel), and the
rocprofv3 summaries (trace averages, HBM bytes from FETCH_SIZE / WRITE_SIZE
scaled by the copy kernel, the busy share of a window, the SQ vector-ALU
figures) on synthetic CSV files whose answers are worked out by hand here."""
import csv
import os
import subprocess
import sys

import pytest

import bench as B
from paper_1703_06606_amd import qnsch as Q
from paper_1703_06606_amd import rocprof_summary as RS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CELLS = [131072, 32768, 8192, 2048, 512, 128, 32]  # the 256 x 512 droplet's 7 levels
OPTS = {"nu1": 2, "nu2": 2, "nu_coarse": 0, "accel": 2, "scheme": 0}


def test_sweep_and_transfer_bytes():
    # a half-sweep of the finest level moves half of 104 B per cell
    assert B.class_bytes("halfsweep", 0, 3, CELLS, OPTS) == 3 * 52.0 * 131072
    # coarse half-sweeps also read the five right-hand sides: 72 B
    assert B.class_bytes("halfsweep", 2, 1, CELLS, OPTS) == 72.0 * 8192
    assert B.class_bytes("fused_sweep", 1, 2, CELLS, OPTS) == 2 * 144.0 * 32768
    # restriction: 100 B per fine cell and the coarse residual of the next level
    assert B.class_bytes("restrict", 0, 1, CELLS, OPTS) == 100.0 * 131072 + 144.0 * 32768
    assert B.class_bytes("prolong", 0, 2, CELLS, OPTS) == 2 * 100.0 * 131072
    assert B.class_bytes("residual_acc", 0, 1, CELLS, OPTS) == 104.0 * 131072
    # level-resident smoothing: pre- and post-smoothing launches alternate
    # (nu1 + nu2 sweeps of 144 B per pair of launches, and the prolongation)
    assert B.class_bytes("smooth", 4, 2, CELLS, OPTS) == (2 + 2) * 144.0 * 512 + 100.0 * 512
    assert B.class_bytes("mx_halfsweep", 0, 1, CELLS, OPTS) == 44.0 * 131072
    assert B.class_bytes("pj_final", 0, 1, CELLS, OPTS) is None


def test_coarsest_solve_bytes_follow_the_automatic_rule():
    """nu_coarse = 0: 4 sweeps for the primitive scheme on 6 or more levels,
    else 6 (the library's rule)"""
    n = CELLS[-1]
    assert B.class_bytes("coarse_solve", 6, 1, CELLS, OPTS) == 4 * 144.0 * n
    assert B.class_bytes("coarse_solve", 6, 1, CELLS, dict(OPTS, scheme=Q.PROJECTION)) == 6 * 144.0 * n
    assert B.class_bytes("coarse_solve", 4, 1, CELLS[:5], OPTS) == 6 * 144.0 * CELLS[4]
    assert B.class_bytes("coarse_solve", 6, 1, CELLS, dict(OPTS, nu_coarse=5)) == 5 * 144.0 * n


def test_kernel_table_groups_operations_by_kernel():
    bd = {("halfsweep", 0): (8, 0.08), ("halfsweep", 1): (8, 0.05), ("fused_sweep", 1): (4, 0.05),
          ("fused_sweep", 2): (4, 0.05), ("residual_acc", 0): (1, 0.02), ("pj_final", 0): (1, 0.01)}
    t = B.kernel_table(bd, CELLS, OPTS)
    assert set(t) == {"k_halfsweep_fine", "k_halfsweep", "k_hs_fused", "k_resid_norm", "k_pj_final"}
    e = t["k_hs_fused"]
    assert e["launches"] == 8 and abs(e["ms"] - 0.10) < 1e-15
    assert e["alg_bytes"] == 4 * 144.0 * 32768 + 4 * 144.0 * 8192
    assert e["ops"] == {"fused_sweep"}
    assert t["k_halfsweep_fine"]["alg_bytes"] == 8 * 52.0 * 131072
    assert t["k_pj_final"]["alg_bytes"] is None


def _write(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def _kname(k):
    return "void qn::%s<qn::Item1>(qn::Item1, int, double)" % k


def test_rocprof_summary_trace_counters_and_busy(tmp_path):
    t0 = 10 ** 9
    # trace: k_a twice (10 and 20 us, two grids), k_b once (5 us) overlapping
    # k_a's first run, then a gap: busy union over the last 60 us
    trace = [
        dict(Kernel_Name=_kname("k_a"), Start_Timestamp=t0, End_Timestamp=t0 + 10000, Grid_Size=512),
        dict(Kernel_Name=_kname("k_b"), Start_Timestamp=t0 + 5000, End_Timestamp=t0 + 10000, Grid_Size=256),
        dict(Kernel_Name=_kname("k_a"), Start_Timestamp=t0 + 40000, End_Timestamp=t0 + 60000, Grid_Size=1024),
    ]
    _write(str(tmp_path / "trace" / "run_kernel_trace.csv"), trace)
    copy = RS.COPY_BYTES / 1024.0
    fetch, write = [], []
    for d, (k, f, w) in enumerate([("k_copy_probe", copy / 2.0, copy), ("k_a", 100.0, 50.0), ("k_a", 300.0, 150.0)]):
        fetch.append(dict(Counter_Name="FETCH_SIZE", Process_Id=1, Dispatch_Id=d, Counter_Value=f,
                          Kernel_Name=_kname(k), Grid_Size=512))
        write.append(dict(Counter_Name="WRITE_SIZE", Process_Id=1, Dispatch_Id=d, Counter_Value=w,
                          Kernel_Name=_kname(k), Grid_Size=512))
    _write(str(tmp_path / "fetch" / "run_counter_collection.csv"), fetch)
    _write(str(tmp_path / "write" / "run_counter_collection.csv"), write)
    out = tmp_path / "out"
    subprocess.run([sys.executable, "-m", "paper_1703_06606_amd.rocprof_summary", "--trace", str(tmp_path / "trace"),
                    "--fetch", str(tmp_path / "fetch"), "--write", str(tmp_path / "write"), "--workload", "w",
                    "--out", str(out), "--command", "cmd", "--busy-tail", "60e-6", "k_a"], check=True, cwd=ROOT)
    md = (out / "k_a_w.md").read_text()
    assert "2 dispatches, average 15.00 us" in md
    kv = dict(l.split(": ", 1) for l in (out / "k_a_w_traffic.txt").read_text().splitlines() if not l.startswith("#"))
    # fetch scale 2 (the copy kernel reads COPY_BYTES), write scale 1
    assert abs(float(kv["fetch_scale"]) - 2.0) < 1e-4 and abs(float(kv["write_scale"]) - 1.0) < 1e-4
    assert int(kv["hbm_bytes_per_launch"]) == int(200.0 * 1024 * 2.0 + 100.0 * 1024 * 1.0)
    busy = (out / "busy_w.md").read_text()
    # window [t0, t0 + 60 us]: kernels cover [0, 10] and [40, 60] us
    assert "busy_fraction: 0.5000" in busy and "dispatches_in_window: 3" in busy


def test_rocprof_summary_valu(tmp_path):
    rows = []
    for d in range(2):
        for n, v in (("SQ_WAVES", 100), ("SQ_INSTS_VALU", 1000 + 200 * d), ("SQ_INSTS_VALU_ADD_F64", 10),
                     ("SQ_INSTS_VALU_MUL_F64", 20), ("SQ_INSTS_VALU_FMA_F64", 30), ("SQ_INSTS_VALU_TRANS_F64", 4)):
            rows.append(dict(Counter_Name=n, Process_Id=1, Dispatch_Id=d, Counter_Value=v, Kernel_Name=_kname("k_a"),
                             Grid_Size=512))
    _write(str(tmp_path / "valu" / "run_counter_collection.csv"), rows)
    out = tmp_path / "out"
    subprocess.run([sys.executable, "-m", "paper_1703_06606_amd.rocprof_summary", "--valu", str(tmp_path / "valu"),
                    "--workload", "w", "--out", str(out), "--command", "cmd", "k_a"], check=True, cwd=ROOT)
    kv = dict(l.split(": ", 1) for l in (out / "k_a_w_valu.txt").read_text().splitlines() if not l.startswith("#"))
    assert float(kv["valu_wave_insts_per_launch"]) == 1100
    assert float(kv["valu_wave_insts_per_wave"]) == pytest.approx(11.0)
    assert float(kv["fp64_wave_insts_per_launch"]) == 64
    # 64 lanes x (ADD + MUL + 2 FMA + TRANS)
    assert float(kv["fp64_flops_per_launch"]) == 64 * (10 + 20 + 60 + 4)


def test_profile_values_ignore_other_device_code(tmp_path, monkeypatch):
    p = tmp_path / "x_traffic.txt"
    p.write_text("# comment\nsource_hash: %s\nhbm_bytes_per_launch: 123\n" % B.source_hash())
    assert B._profile_values(str(p))["hbm_bytes_per_launch"] == "123"
    p.write_text("source_hash: 0000000000000000\nhbm_bytes_per_launch: 123\n")
    assert B._profile_values(str(p)) is None
