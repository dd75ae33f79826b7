"""Values the paper prints, kept as fixtures under tests/golden/ (each names
its passage).  Only Table 1 of sec. 9 prints solver results; its errors come
from an initial condition the scheme cannot run as printed (it reaches the
density pole), so the study here uses a bounded one and compares rates, not
errors.  This file checks the transcription against the table's own
arithmetic: each printed rate is log2 of the ratio of successive errors, and
the finest rates are the paper's claim of second order."""
import json
import math
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def table1():
    return json.load(open(os.path.join(HERE, "golden", "table1_cauchy_convergence.json")))


@pytest.mark.parametrize("scheme", ["primitive", "projection"])
def test_table1_rates_are_the_error_ratios(scheme):
    t = table1()[scheme]
    e, r = t["error"], t["rate"]
    assert r[0] is None and len(e) == len(r) == 4
    for k in range(1, 4):
        # printed with two decimals from errors printed with four digits
        assert abs(math.log2(e[k - 1] / e[k]) - r[k]) < 0.015, (scheme, k)
    assert abs(r[-1] - 2.0) < 0.1
