"""Per-candidate parity checks of reduced outputs against the FP64 oracle.

Section 3's predicate decides each candidate from its 8-bit codes.  A
candidate whose unrounded channel lies within 1e-3 codes of a rounding tie or
of the gamut edge (the band) may be decided either way by an FP32 device path;
the oracle gives, per band candidate, the set of decisions reachable inside
the band, and per colour the range every reduced output can take when each
such candidate ends either way (oracle.reduce_bounds).  The checks below hold
every reduced output of every colour to that range: where no band candidate
can move a field the range is a single value and the check is equality.
Every pair a device path reports (best pair, per-pattern best, per-ray
maximum) is also re-evaluated by the oracle at its own (i, j): it must be a
candidate that can survive with the reported pattern, and its 8-bit codes must
equal the oracle's unless a channel lies in the band.
"""
from __future__ import annotations

import numpy as np

NONE_I = 0xFFFF


def _key(i, j):
    """Order of 'maximum amplitude': larger i first, then smaller j (0 = none)."""
    i = np.asarray(i, np.int64)
    j = np.asarray(j, np.int64)
    return np.where(i == NONE_I, 0, (i << 16) | (0xFFFF - j))


def _check_pairs(oracle, colours, grid, rule, cidx, i, j, plus, minus, pattern, what):
    """Each reported pair (colour index, i, j, codes, pattern) can survive
    under the oracle with that pattern, and its codes are the oracle's unless
    a channel lies in the band.  Returns the number of band pairs."""
    if len(cidx) == 0:
        return 0
    idx = np.stack([np.asarray(cidx, np.int64), np.asarray(i, np.int64),
                    np.asarray(j, np.int64)], axis=1)
    ev = oracle.eval_list(colours, idx, grid, rule)
    pattern = np.asarray(pattern, np.int64)
    reach = (ev["dset"].astype(np.int64) >> pattern) & 1
    bad = np.nonzero(reach == 0)[0]
    assert len(bad) == 0, (f"{what}: {len(bad)} reported pairs cannot survive with their pattern, "
                           f"first {idx[bad[0]].tolist()} p={pattern[bad[0]]} dset={ev['dset'][bad[0]]:#x}")
    clear = (ev["boundary"] & 1) == 0
    assert np.array_equal(np.asarray(plus)[clear], ev["Vp"][clear]), what
    assert np.array_equal(np.asarray(minus)[clear], ev["Vm"][clear]), what
    return int((~clear).sum())


def within(lo, x, hi, what):
    lo, x, hi = (np.asarray(a, np.int64) for a in (lo, x, hi))
    bad = np.nonzero((x < lo) | (x > hi))
    assert len(bad[0]) == 0, (f"{what}: {len(bad[0])} values outside the oracle's range, first at "
                              f"{tuple(int(b[0]) for b in bad)}: {x[bad][0]} not in "
                              f"[{lo[bad][0]}, {hi[bad][0]}]")


def check_summaries(oracle, colours, grid, rule, g, bounds=None, ngamut=True):
    """GPU per-colour summaries (SUMMARY_DTYPE records) against the oracle's
    ranges, per candidate.  Returns (bounds, stats)."""
    b = oracle.reduce_bounds(colours, grid, rule)["bounds"] if bounds is None else bounds
    n = len(b)
    assert len(g) == n
    within(b["count_lo"], g["count"], b["count_hi"], "count")
    within(b["pat_lo"], g["per_pattern"], b["pat_hi"], "per_pattern")
    assert np.array_equal(g["count"].astype(np.int64), g["per_pattern"].astype(np.int64).sum(1))
    kg = _key(g["best_i"], g["best_j"])
    within(b["key_lo"], kg, b["key_hi"], "best (i, j)")
    has = kg > 0
    nb = _check_pairs(oracle, colours, grid, rule, np.nonzero(has)[0], g["best_i"][has],
                      g["best_j"][has], g["best_plus"][has], g["best_minus"][has], g["best_p"][has],
                      "best pair")
    if ngamut:
        # n_gamut counts in-gamut candidates; only those at the gamut edge can differ
        within(b["n_gamut"].astype(np.int64) - b["n_boundary"], g["n_gamut"],
               b["n_gamut"].astype(np.int64) + b["n_boundary"], "n_gamut")
    else:
        assert np.all(g["n_gamut"] == 0)
    moved = int(((b["count_lo"] != b["count_hi"]) | (b["key_lo"] != b["key_hi"])).sum())
    return b, {"colours": n, "fields_movable": moved, "band_best_pairs": nb,
               "ambiguous": int(b["n_ambiguous"].sum())}


def check_table(oracle, colours, grid, rule, t, b=None):
    """Angle-bin table rows (TABLE_DTYPE) against the oracle's ranges."""
    r = oracle.reduce_bounds(colours, grid, rule, bins=True)
    bb = r["bounds"]
    within(bb["count_lo"], t["count"], bb["count_hi"], "table count")
    within(r["bins_lo"], t["bin_ridx"], r["bins_hi"], "table bins")
    return r


def check_rays(oracle, colours, grid, rule, rays, r=None):
    """Per-ray maxima (largest i + 1 per (colour, j), 0 = none) against the
    oracle's ranges."""
    if r is None:
        r = oracle.reduce_bounds(colours, grid, rule, rays=True)
    within(r["rays_lo"], rays, r["rays_hi"], "per-ray maxima")
    return r


def check_pattern_bests(oracle, colours, grid, rule, pb, bounds=None):
    """Per-pattern best pairs (PATTERN_PAIR_DTYPE [n, 7]; flags bit 0 = a pair)
    against the oracle's ranges, each reported pair re-evaluated."""
    b = oracle.reduce_bounds(colours, grid, rule)["bounds"] if bounds is None else bounds
    have = (pb["flags"] & 1) == 1
    kg = np.where(have, _key(pb["i"], pb["j"]), 0)
    within(b["pkey_lo"], kg, b["pkey_hi"], "per-pattern best (i, j)")
    c, p = np.nonzero(have)
    assert np.all(pb["pattern"][have] == p + 1)
    sel = pb[have]
    return _check_pairs(oracle, colours, grid, rule, c, sel["i"], sel["j"], sel["plus"],
                        sel["minus"], sel["pattern"], "per-pattern best")


def check_ray_records(oracle, colours, grid, rule, recs, offsets, r=None):
    """A per-ray list (PAIR_DTYPE in (colour, j) order, CSR offsets): its
    maxima against the oracle's ranges and every record re-evaluated."""
    n = len(colours)
    nt = grid[3]
    rays = np.zeros((n, nt), np.int64)
    col = np.repeat(np.arange(n), np.diff(offsets))
    assert np.array_equal(recs["colour"].astype(np.int64), col)
    rays[col, recs["j"].astype(np.int64)] = recs["i"].astype(np.int64) + 1
    r = check_rays(oracle, colours, grid, rule, rays, r)
    nb = _check_pairs(oracle, colours, grid, rule, col, recs["i"], recs["j"], recs["plus"],
                      recs["minus"], recs["pattern"], "per-ray record")
    return r, nb
