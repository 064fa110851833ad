"""The per-candidate parity checks (tests/parity.py) on the CPU: the oracle's
own reduced outputs pass them, and outputs with a planted mistake (a count off
by one, a best pair moved along its ray, a wrong code, a per-ray maximum one
step short, a per-pattern best of another pattern) fail them."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W

import parity

GRID = (0.5, 60, 2.0, 180)
RULE = (50, 0.5, 0x7F)


@pytest.fixture(scope="module")
def case(oracle):
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(12, 15)])
    summ = oracle.reduce(cols, GRID, RULE)
    recs, offs, _ = oracle.search(cols, GRID, RULE)
    r = oracle.reduce_bounds(cols, GRID, RULE, bins=True, rays=True)
    return cols, summ, recs, offs, r


def _pattern_bests(recs, offs, n):
    dt = np.dtype([("i", "<u2"), ("j", "<u2"), ("plus", "u1", 3), ("minus", "u1", 3),
                   ("pattern", "u1"), ("flags", "u1")])
    pb = np.zeros((n, 7), dt)
    for c in range(n):
        seg = recs[offs[c]:offs[c + 1]]
        for p in range(1, 8):
            sp = seg[seg["pattern"] == p]
            if len(sp):
                b = sp[np.lexsort((sp["j"], -sp["i"].astype(np.int64)))[0]]
                pb[c, p - 1] = (b["i"], b["j"], b["plus"], b["minus"], p, 1)
    return pb


def _rays(recs, offs, n, nt):
    rays = np.zeros((n, nt), np.int64)
    col = np.repeat(np.arange(n), np.diff(offs))
    np.maximum.at(rays, (col, recs["j"].astype(np.int64)), recs["i"].astype(np.int64) + 1)
    return rays


def test_oracle_outputs_pass(oracle, case):
    cols, summ, recs, offs, r = case
    parity.check_summaries(oracle, cols, GRID, RULE, summ, bounds=r["bounds"])
    parity.check_rays(oracle, cols, GRID, RULE, _rays(recs, offs, len(cols), GRID[3]), r)
    parity.check_pattern_bests(oracle, cols, GRID, RULE, _pattern_bests(recs, offs, len(cols)),
                               bounds=r["bounds"])
    _, tc, tb = oracle.reduce(cols, GRID, RULE, table=True)
    t = np.zeros(len(cols), np.dtype([("count", "<u4"), ("bin_ridx", "u1", 36)]))
    t["count"], t["bin_ridx"] = tc, tb
    parity.check_table(oracle, cols, GRID, RULE, t)


def _colour_with_best(summ):
    c = np.nonzero((summ["best_i"] != 0xFFFF) & (summ["best_i"] > 0))[0]
    assert len(c)
    return int(c[0])


def test_planted_summary_mistakes_fail(oracle, case):
    cols, summ, recs, offs, r = case
    c = _colour_with_best(summ)
    mutations = []
    m = summ.copy(); m["count"][c] += 1; m["per_pattern"][c, m["best_p"][c] - 1] += 1
    mutations.append(m)
    m = summ.copy(); m["per_pattern"][c, 0] += 1; m["count"][c] += 1
    mutations.append(m)
    m = summ.copy(); m["best_i"][c] -= 1
    mutations.append(m)
    m = summ.copy(); m["best_j"][c] = (int(m["best_j"][c]) + 1) % GRID[3]
    mutations.append(m)
    m = summ.copy(); m["best_plus"][c, 0] ^= 1
    mutations.append(m)
    m = summ.copy(); m["best_p"][c] = 7 if m["best_p"][c] != 7 else 1
    mutations.append(m)
    m = summ.copy(); m["n_gamut"][c] += int(r["bounds"]["n_boundary"][c]) + 1
    mutations.append(m)
    for k, m in enumerate(mutations):
        with pytest.raises(AssertionError):
            parity.check_summaries(oracle, cols, GRID, RULE, m, bounds=r["bounds"])
            print("mutation", k, "passed")


def test_planted_ray_and_pattern_mistakes_fail(oracle, case):
    cols, summ, recs, offs, r = case
    rays = _rays(recs, offs, len(cols), GRID[3])
    c, j = np.argwhere(rays > 1)[0]
    bad = rays.copy(); bad[c, j] -= 1
    with pytest.raises(AssertionError):
        parity.check_rays(oracle, cols, GRID, RULE, bad, r)
    pb = _pattern_bests(recs, offs, len(cols))
    c, p = np.argwhere(pb["flags"] == 1)[0]
    bad = pb.copy(); bad["i"][c, p] -= 1
    with pytest.raises(AssertionError):
        parity.check_pattern_bests(oracle, cols, GRID, RULE, bad, bounds=r["bounds"])
    bad = pb.copy(); bad["pattern"][c, p] = (p + 1) % 7 + 1
    with pytest.raises(AssertionError):
        parity.check_pattern_bests(oracle, cols, GRID, RULE, bad, bounds=r["bounds"])
    bad = pb.copy(); bad["flags"][c, p] = 0
    with pytest.raises(AssertionError):
        parity.check_pattern_bests(oracle, cols, GRID, RULE, bad, bounds=r["bounds"])
    _, tc, tb = oracle.reduce(cols, GRID, RULE, table=True)
    t = np.zeros(len(cols), np.dtype([("count", "<u4"), ("bin_ridx", "u1", 36)]))
    t["count"], t["bin_ridx"] = tc, tb
    k = np.argwhere(tb > 1)[0]
    t["bin_ridx"][k[0], k[1]] -= 1
    with pytest.raises(AssertionError):
        parity.check_table(oracle, cols, GRID, RULE, t)
