"""The Table 2 readings report (tests/golden/table2_readings.txt) is what the
committed script computes from the oracle now, and its conclusions hold:
under the reading the search uses (reject out-of-gamut pairs, peak-to-peak
change, r <= 100) every present cell is checked in the paper; the reading with
the fewest wrong cells is the clip reading with a one-sided change."""
from __future__ import annotations

import importlib.util
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def _script():
    spec = importlib.util.spec_from_file_location("table2_readings", os.path.join(HERE, "golden", "table2_readings.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_report_is_current(oracle):
    mod = _script()
    with open(mod.OUT) as f:
        stored = f.read()
    assert mod.report() == stored


def test_report_conclusions():
    with open(os.path.join(HERE, "golden", "table2_readings.txt")) as f:
        rows = [ln.split() for ln in f if ln.startswith("union ")]
    union = {(r[1], r[2], int(r[3])): tuple(int(x) for x in r[4:]) for r in rows}
    m, e, x, w = union[("reject", "p2p", 100)]
    assert (m, e, x, w) == (15, 0, 22, 22)  # sound: no cell outside the paper's checks
    best = min(union.items(), key=lambda kv: kv[1][3])
    assert best[0][:2] == ("clip", "one-sided") and best[1][3] == 5
