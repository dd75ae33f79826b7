"""The C-ABI library loads and exports every function include/qnsch.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1703_06606_amd import qnsch as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "qnsch.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qnsch_[a-z_0-9]+)\s*\(", txt)))


# the calls of the boundary: context, state, step, mass and energy of sec.
# 6.1, step statistics, and the serving calls with their latency figures
BOUNDARY = ("qnsch_create", "qnsch_set_state", "qnsch_get_state", "qnsch_step", "qnsch_mass", "qnsch_energy",
            "qnsch_stats", "qnsch_last_error", "qnsch_destroy", "qnsch_default_eta", "qnsch_server_create",
            "qnsch_server_submit", "qnsch_server_progress", "qnsch_server_result", "qnsch_server_latency",
            "qnsch_server_destroy")


def test_header_declares_the_boundary():
    names = declared()
    for n in BOUNDARY:
        assert n in names, n


def test_struct_layouts_match_the_binding(tmp_path):
    """the binding's ctypes structures have the sizes and field offsets the C
    compiler gives the header's structs (host gcc, no GPU)"""
    import subprocess
    structs = {"qnsch_grid": Q.Grid, "qnsch_params": Q.Params, "qnsch_opts": Q.Opts,
               "qnsch_step_stats": Q.StepStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "qnsch.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ['printf("QNSCH_HIST %d\\n", QNSCH_HIST);', "return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n") if l)
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[cname + "." + f]) == getattr(py, f).offset, (cname, f)
    assert int(got["QNSCH_HIST"]) == Q.HIST


@pytest.mark.skipif(not os.path.exists(Q.LIB), reason="HIP library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(Q.LIB)
    for n in declared():
        assert hasattr(lib, n), n
    assert set(Q.SYMBOLS) == set(declared())


def test_binding_refuses_to_run_without_the_library(tmp_path, monkeypatch):
    monkeypatch.setattr(Q, "LIB", str(tmp_path / "missing.so"))
    monkeypatch.setattr(Q, "_lib", None)
    with pytest.raises(RuntimeError):
        Q.lib()


@pytest.mark.skipif(not os.path.exists(Q.LIB), reason="HIP library not built")
def test_default_eta_is_the_matching_formula():
    """qnsch_default_eta (host only) against the formula of sec. 8.1 written
    out here, its equal-density limit 3/(2 sqrt2 rho1), and continuity across
    the switch to the series (|rho2/rho1 - 1| = 0.05)"""
    import math

    def direct(r1, r2):
        d = r2 - r1
        return d ** 3 / (2 * math.sqrt(2) * r1 * r2 * (r2 * r2 - r1 * r1 - 2 * r1 * r2 * math.log(r2 / r1)))

    for r1, r2 in ((1.0, 3.0), (1.0, 10.0), (1.0, 100.0), (2.0, 0.5), (1.0, 1.3)):
        assert math.isclose(Q.default_eta(r1, r2), direct(r1, r2), rel_tol=1e-13)
    # the workloads' values at ratios 3, 10 and 100
    assert abs(Q.default_eta(1.0, 3.0) - 0.66945) < 5e-6
    assert abs(Q.default_eta(1.0, 10.0) - 0.48678) < 5e-6
    assert abs(Q.default_eta(1.0, 100.0) - 0.37790) < 5e-6
    for r1 in (1.0, 2.5):
        assert math.isclose(Q.default_eta(r1, r1), 3 / (2 * math.sqrt(2) * r1), rel_tol=1e-15)
    # on both sides of the switch: the series and the direct form agree
    # (the direct form loses about 6 digits to cancellation there)
    for x in (0.0499999, 0.0500001, -0.0499999, -0.0500001):
        assert math.isclose(Q.default_eta(1.0, 1.0 + x), direct(1.0, 1.0 + x), rel_tol=1e-9)
    assert math.isnan(Q.default_eta(0.0, 1.0))
