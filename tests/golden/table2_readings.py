"""Table 2 under every combination of the readings the paper leaves open.

Writes tests/golden/table2_readings.txt (run from the repository root:
`python tests/golden/table2_readings.py`); tests/test_table2_readings.py
recomputes it and compares.  Calls only the FP64 oracle (for the 8-bit codes
and gamut flags of every candidate); the predicate of Section 3 is then applied
here under each reading:

- gamut: "reject" (a pair counts only when every linear channel of both
  colours lies in [0, 1]) or "clip" (codes clamped to [0, 255], no rejection);
- change of a channel: "p2p", the peak-to-peak |V+ - V-| of the two colours
  that alternate, or "one-sided", max(|V+ - T|, |V- - T|), the larger move of
  either colour away from the target's own 8-bit code T;
- the largest radius searched, r_max (Delta E 1976 units);
- the setting: any of Table 1's twelve (V_th, R_novib), or each one alone.

Grid: r = 0.25 .. 100 in steps of 0.25 (400 radii) x theta = 0 .. 359 deg in
steps of 1 deg; the nine Table 1 colours.  A cell (colour, information) is
present when some pair encodes that pattern.  Against Table 2: matched = cells
checked both here and in the paper, extra = present here but empty in the
paper, missed = checked in the paper but absent here; wrong = extra + missed.
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

GRID = (0.25, 400, 1.0, 360)
R_MAX = (5, 10, 20, 30, 50, 75, 100)
OUT = os.path.join(HERE, "table2_readings.txt")


def paper_table() -> np.ndarray:
    """Table 2 as printed: [9 colours, 7 patterns] (pattern p at column p - 1)."""
    pres = np.zeros((9, 7), dtype=bool)
    with open(os.path.join(HERE, "table2_presence.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            pres[:, int(parts[0], 2) - 1] = [bool(int(x)) for x in parts[1:]]
    return pres


def first_radius(nthreads: int = 0):
    """For every reading (gamut, change), setting and (colour, pattern): the
    smallest radius index with a pair of that pattern (nr if none)."""
    cols = W.PAPER_COLOUR_ARRAY
    nr = GRID[1]
    out = {}
    target = cols.astype(np.int64)
    for gamut, flags in (("reject", 0), ("clip", 1)):
        # codes and gamut flags do not depend on the thresholds
        ev = oracle.eval_all(cols, GRID, (50, 0.5, 0x7F, flags), nthreads=nthreads)
        Vp = ev["Vp"].astype(np.int64)
        Vm = ev["Vm"].astype(np.int64)
        ok = np.ones(ev.shape, bool) if flags else ev["gamut"] == 3
        for change in ("p2p", "one-sided"):
            if change == "p2p":
                d = np.abs(Vp - Vm)
            else:
                T = target[:, None, None, :]
                d = np.maximum(np.abs(Vp - T), np.abs(Vm - T))
            for v_th, rn in W.TABLE1_RULES:
                hi = d > v_th
                lo = d < v_th * rn
                every = (hi | lo).all(-1) & ok
                p = (hi[..., 0] * 4 + hi[..., 1] * 2 + hi[..., 2]) * every
                first = np.full((9, 7), nr, dtype=np.int64)
                for q in range(1, 8):
                    rows = (p == q).any(-1)  # [colour, i]
                    has = rows.any(-1)
                    first[has, q - 1] = rows[has].argmax(-1)
                out[(gamut, change, v_th, rn)] = first
    return out


def score(pres: np.ndarray, paper: np.ndarray):
    matched = int((pres & paper).sum())
    extra = int((pres & ~paper).sum())
    missed = int((~pres & paper).sum())
    return matched, extra, missed


def report(nthreads: int = 0) -> str:
    paper = paper_table()
    first = first_radius(nthreads)
    dr = GRID[0]
    lines = ["# Table 2 (Section 3) against the readings the paper leaves open; written by",
             "# tests/golden/table2_readings.py from the FP64 oracle's codes.  Grid r = 0.25..100",
             "# step 0.25 x theta = 0..359 deg step 1; nine Table 1 colours.  The paper checks",
             f"# {int(paper.sum())} of 63 cells.",
             "#",
             "# union of the twelve settings: gamut change r_max matched extra missed wrong"]
    best = None
    for gamut in ("reject", "clip"):
        for change in ("p2p", "one-sided"):
            for rmax in R_MAX:
                imax = int(round(rmax / dr)) - 1
                pres = np.zeros((9, 7), dtype=bool)
                for v_th, rn in W.TABLE1_RULES:
                    pres |= first[(gamut, change, v_th, rn)] <= imax
                m, e, x = score(pres, paper)
                lines.append(f"union {gamut} {change} {rmax} {m} {e} {x} {e + x}")
                if best is None or e + x < best[0]:
                    best = (e + x, gamut, change, rmax, m, e, x)
    lines.append(f"# fewest wrong cells over the union: {best[1]} {best[2]} r_max {best[3]}: {best[0]} wrong "
                 f"({best[4]} matched, {best[5]} extra, {best[6]} missed)")
    lines.append("#")
    lines.append("# each setting alone: gamut change r_max v_th r_novib matched extra missed wrong")
    best1 = None
    for gamut in ("reject", "clip"):
        for change in ("p2p", "one-sided"):
            for rmax in R_MAX:
                imax = int(round(rmax / dr)) - 1
                for v_th, rn in W.TABLE1_RULES:
                    pres = first[(gamut, change, v_th, rn)] <= imax
                    m, e, x = score(pres, paper)
                    lines.append(f"setting {gamut} {change} {rmax} {v_th} {rn} {m} {e} {x} {e + x}")
                    if best1 is None or e + x < best1[0]:
                        best1 = (e + x, gamut, change, rmax, v_th, rn, m, e, x)
    lines.append(f"# fewest wrong cells for one setting: {best1[1]} {best1[2]} r_max {best1[3]} "
                 f"V_th {best1[4]} R_novib {best1[5]}: {best1[0]} wrong ({best1[6]} matched, {best1[7]} extra, "
                 f"{best1[8]} missed)")
    lines.append("#")
    lines.append("# presence tables (rows = information 100 010 001 110 101 011 111, columns = the nine")
    lines.append("# colours in Table 1's order), reject / p2p / r_max 100, the union and each setting")
    imax = int(round(100 / dr)) - 1

    def table(tag, pres):
        lines.append(f"table {tag}")
        for q in range(7):
            lines.append("  " + W.PATTERNS[q] + " " + "".join("x" if c else "." for c in pres[:, int(W.PATTERNS[q], 2) - 1]))

    union = np.zeros((9, 7), dtype=bool)
    for v_th, rn in W.TABLE1_RULES:
        union |= first[("reject", "p2p", v_th, rn)] <= imax
    table("union", union)
    for v_th, rn in W.TABLE1_RULES:
        table(f"{v_th} {rn}", first[("reject", "p2p", v_th, rn)] <= imax)
    bu = np.zeros((9, 7), dtype=bool)
    for v_th, rn in W.TABLE1_RULES:
        bu |= first[(best[1], best[2], v_th, rn)] <= int(round(best[3] / dr)) - 1
    table(f"union {best[1]} {best[2]} r_max {best[3]} (fewest wrong)", bu)
    table("paper", paper)
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    text = report()
    with open(OUT, "w") as f:
        f.write(text)
    print(text)
