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


def test_header_declares_the_boundary():
    names = declared()
    for n in ("qnsch_create", "qnsch_step", "qnsch_mass", "qnsch_energy", "qnsch_destroy"):
        assert n in names


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
