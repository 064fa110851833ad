"""Pins of the oracle's boundary band and decision-ambiguity classifier.

Every GPU parity test excuses a candidate only when the oracle flags it: bit 0
of `boundary` when a channel lies within 1e-3 codes of a rounding tie (k + 1/2)
or of the gamut edges 0 / 255 (and no channel of the pair is clearly out of
gamut), bit 1 when moving values inside that band can change the candidate's
decision, with `dset` the set of decisions it can reach (bit 0 = not a
survivor, bit p = survivor of pattern p; Section 3's predicate under Table 1's
thresholds).  A classifier that over-flags would silently widen every
exemption, so it is pinned here against an independent model:

- the channel values v+ and v- come from the 50-digit model of the colour
  conversions (dec_model.py), not from the oracle;
- the reachable decisions come from a different formulation: each of the six
  channels moves on its own by any amount below 1e-3, its code is the
  round-half-even of the moved value and its colour is in gamut when all
  three moved values lie in [0, 255]; the open interval of each channel is cut
  at the ties and edges it contains and one point of every piece is tried,
  every combination of the six channels is decided.

Candidates: band candidates of seeded grids (ambiguous ones, and ones whose
tie flip changes nothing), near misses just outside the band, clearly
out-of-gamut candidates with a channel at a tie, and hand-built candidates at
the gamut edge, placed by bisection on the radius where a channel of one
colour meets 0 or 255 near the edge of the ray's in-gamut range.  Mistakes
planted in a copy of the oracle's source (over-flagging, no gamut flips, a
wider band, no tie flips, ties at the wrong point, no out-of-gamut exclusion)
must each fail the comparison.
"""
from __future__ import annotations

import itertools
import math
import os
import shutil
from decimal import ROUND_FLOOR

import numpy as np
import pytest

import workloads as W
from dec_model import D, d_encode, d_lab_to_linear, d_rgb8_to_lab, d_round, d_sincos_deg

BAND = D("0.001")
HALF = D("0.5")
RULES = [(50, 0.5, 0x7F, 0), (100, 0.25, 0x55, 0), (50, 0.5, 0x7F, 1)]
HARVEST_GRID = (0.37, 120, 1.0, 360)


# --------------------------------------------------------------------------
# The independent model.

_lab_cache: dict = {}


def model_values(rgb, r, deg):
    """The six unrounded code values (+R, +G, +B, -R, -G, -B) at 50 digits."""
    if rgb not in _lab_cache:
        _lab_cache[rgb] = d_rgb8_to_lab(rgb)
    L, a, b = _lab_cache[rgb]
    s, c = d_sincos_deg(deg)
    Da, Db = r * s, r * c
    v = []
    for sg in (1, -1):
        lin = d_lab_to_linear((L, a + sg * Da, b + sg * Db))
        v += [255 * d_encode(x) for x in lin]
    return v


def decide(codes, gp, gm, rule):
    """Section 3 with Table 1's thresholds: 0 = not a survivor, else p."""
    v_th, rn, mask, clip = rule
    if not (clip or (gp and gm)):
        return 0
    p, ok = 0, True
    for k in range(3):
        d = abs(codes[k] - codes[k + 3])
        hi, lo = d > v_th, D(d) < D(v_th) * D(str(rn))
        ok = ok and (hi or lo)
        p = 2 * p + int(hi)
    return p if ok and p and (mask >> (p - 1)) & 1 else 0


def _clamp(u):
    return min(max(u, D(0)), D(255))


def channel_options(x, clip):
    """(code, in range) pairs the channel reaches when moved by less than the band."""
    lo, hi = x - BAND, x + BAND
    cuts = {lo, hi}
    for m in range(int((lo - HALF).to_integral_value(ROUND_FLOOR)), int(hi.to_integral_value(ROUND_FLOOR)) + 1):
        t = D(m) + HALF
        if lo < t < hi:
            cuts.add(t)
    for e in (D(0), D(255)):
        if lo < e < hi:
            cuts.add(e)
    cuts = sorted(cuts)
    opts = set()
    for a, b in zip(cuts, cuts[1:]):
        u = (a + b) / 2
        opts.add((d_round(_clamp(u) if clip else u), D(0) <= u <= D(255)))
    return sorted(opts)


def model_classify(v, rule):
    """(band flag, ambiguity flag, reachable decision set as a bit mask)."""
    clip = rule[3] & 1

    def near_tie(a):
        return abs(a - (a.to_integral_value(ROUND_FLOOR) + HALF)) < BAND

    if clip:
        band = any(near_tie(_clamp(x)) for x in v)
    else:
        out = any(x < -BAND or x > 255 + BAND for x in v)
        edge = any(abs(x) < BAND or abs(x - 255) < BAND for x in v)
        band = not out and (edge or any(near_tie(x) for x in v))
    dset = 0
    for combo in itertools.product(*[channel_options(x, clip) for x in v]):
        codes = [c for c, _ in combo]
        inr = [f for _, f in combo]
        dset |= 1 << decide(codes, all(inr[:3]), all(inr[3:]), rule)
    return band, bin(dset).count("1") > 1, dset


# --------------------------------------------------------------------------
# Candidates.  Each is (rgb, dr, i, j): radius (i + 1) dr on ray j (1 deg steps).

def _tie_dist(v):
    return np.abs(v - (np.floor(v) + 0.5))


def harvest(oracle, rule, rng):
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(613, 6)])
    allc = oracle.eval_all(cols, HARVEST_GRID, rule)
    v = np.concatenate([allc["vp"], allc["vm"]], axis=-1)
    bnd = allc["boundary"]
    clip = rule[3] & 1
    vv = np.clip(v, 0, 255) if clip else v
    dist = _tie_dist(vv).min(-1)
    out = ((v < -1e-3) | (v > 255 + 1e-3)).any(-1)
    picks = []

    def take(mask, k):
        idx = np.argwhere(mask)
        if len(idx) > k:
            idx = idx[rng.choice(len(idx), k, replace=False)]
        picks.extend((tuple(int(x) for x in cols[c]), HARVEST_GRID[0], int(i), int(j)) for c, i, j in idx)
        return len(idx)

    counts = {
        "ambiguous": take((bnd & 2) != 0, 50),
        "band, decision fixed": take(bnd == 1, 50),
        "near miss": take((bnd == 0) & (dist >= 1e-3) & (dist < 1.6e-3) & ~out, 30),
        "out, at a tie": take((bnd == 0) & (dist < 1e-3) & out, 15 if not clip else 0),
    }
    return picks, counts


EDGE_COLOURS = [(255, 120, 30), (0, 200, 90), (250, 250, 250), (255, 255, 255), (6, 6, 6), (240, 100, 240),
                (100, 240, 240), (30, 255, 180)]


def edge_candidates(oracle, rule):
    """Near the edge of each ray's in-gamut range: the radius where a channel of
    one colour meets 0 or 255, then 4e-4 codes inside and outside of it."""
    cands = []
    dr0 = 0.05
    for rgb in EDGE_COLOURS:
        for j in (0, 33, 75, 140, 222, 300):
            idx = np.array([[0, i, j] for i in range(1600)])
            ev = oracle.eval_list([rgb], idx, (dr0, 1600, 1.0, 360), rule)
            v = np.concatenate([ev["vp"], ev["vm"]], axis=-1)
            both = (ev["gamut"] == 3)
            # the last radius in gamut before the pair leaves it
            exits = np.nonzero(both[:-1] & ~both[1:])[0]
            for i in exits[:2]:
                k = int(np.argmax(np.minimum(np.abs(v[i + 1]), np.abs(v[i + 1] - 255)) *
                                  ((v[i + 1] < 0) | (v[i + 1] > 255))))
                edge = 0.0 if v[i + 1][k] < 0 else 255.0

                def f(r):
                    c = oracle.eval_one(rgb, (r, 1, 1.0, 360), rule, 0, j)
                    return np.concatenate([c["vp"], c["vm"]])[k] - edge

                a, b = dr0 * (i + 1), dr0 * (i + 2)
                fa = f(a)
                for _ in range(80):
                    m = 0.5 * (a + b)
                    if (f(m) > 0) == (fa > 0):
                        a, fa = m, f(m)
                    else:
                        b = m
                slope = (f(b + 1e-6) - f(b - 1e-6)) / 2e-6
                if not math.isfinite(slope) or slope == 0:
                    continue
                for off in (-4e-4, 4e-4, -1.5e-3):
                    cands.append((rgb, b + off / slope, 0, j))
    return cands


@pytest.fixture(scope="module")
def cases(oracle):
    rng = np.random.default_rng(77)
    out = []
    report = {}
    for rule in RULES:
        picks, counts = harvest(oracle, rule, rng)
        if not rule[3]:
            picks += edge_candidates(oracle, rule)
        model = []
        for rgb, dr, i, j in picks:
            r = D((i + 1) * dr)  # the oracle's FP64 radius, exactly
            model.append(model_classify(model_values(rgb, r, D(j)), rule))
        out.append((rule, picks, model))
        report[rule] = counts
    print("band pin candidates:", report)
    return out


def compare(oracle, cases, L=None):
    """Candidates on which the oracle build L disagrees with the model."""
    bad = []
    for rule, picks, model in cases:
        for (rgb, dr, i, j), (band, amb, dset) in zip(picks, model):
            c = oracle.eval_one(rgb, (dr, i + 1, 1.0, 360), rule, i, j, L=L)
            got = (bool(c["boundary"] & 1), bool(c["boundary"] & 2), int(c["dset"]))
            if got != (band, amb, dset):
                bad.append((rule, rgb, dr, i, j, got, (band, amb, dset)))
    return bad


# --------------------------------------------------------------------------

def test_classifier_matches_the_perturbation_model(oracle, cases):
    bad = compare(oracle, cases)
    assert not bad, bad[:5]
    # the pin covers every kind of candidate
    kinds = {"ambiguous": 0, "fixed": 0, "edge": 0, "edge ambiguous": 0, "gamut flip only": 0, "clean": 0}
    for rule, picks, model in cases:
        for (rgb, dr, i, j), (band, amb, dset) in zip(picks, model):
            v = model_values(rgb, D((i + 1) * dr), D(j))
            near_edge = any(abs(x) < BAND or abs(x - 255) < BAND for x in v)
            kinds["ambiguous"] += amb
            kinds["fixed"] += band and not amb
            kinds["edge"] += band and near_edge
            kinds["edge ambiguous"] += amb and near_edge
            kinds["clean"] += not band
            # a decision that only a gamut flip changes: no channel near a tie
            if amb and near_edge and not any(abs(x - (x.to_integral_value(ROUND_FLOOR) + HALF)) < BAND for x in v):
                kinds["gamut flip only"] += 1
    print("kinds:", kinds)
    assert kinds["ambiguous"] >= 20 and kinds["fixed"] >= 20 and kinds["clean"] >= 20
    assert kinds["edge"] >= 10 and kinds["edge ambiguous"] >= 3 and kinds["gamut flip only"] >= 1


MUTATIONS = {
    "over-flagging": ("if (c->dset & (c->dset - 1)) c->boundary |= 2;", "c->boundary |= 2;"),
    "no gamut flips": ("const int gp_alt = (edge_p && !out_p) ? !gp : gp;", "const int gp_alt = gp;"),
    "band twice as wide": ("static const double BAND = 1e-3;", "static const double BAND = 2e-3;"),
    "no tie flips": ("alt[k] = (nom[k] == f) ? f + 1 : f;", "alt[k] = nom[k];"),
    "ties at integers": ("double t = floor(v) + 0.5;", "double t = floor(v);"),
    "no out-of-gamut exclusion": ("static int clearly_out(double v) { return v < -BAND || v > 255.0 + BAND; }",
                                  "static int clearly_out(double v) { (void)v; return 0; }"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_classifier_mistakes_are_caught(oracle, cases, tmp_path, name):
    old, new = MUTATIONS[name]
    srcs = []
    for src in oracle.sources():
        dst = tmp_path / os.path.basename(src)
        shutil.copy(src, dst)
        srcs.append(str(dst))
    text = open(srcs[0]).read()
    assert text.count(old) == 1, name
    open(srcs[0], "w").write(text.replace(old, new))
    L = oracle.load_library(oracle.compile_library(srcs, str(tmp_path / "mutant.so")))
    assert compare(oracle, cases, L=L), f"the planted mistake '{name}' went unnoticed"


def test_reduce_bounds_follow_the_decision_sets(oracle):
    """orc_reduce_bounds against the per-candidate decision sets of eval_all:
    must-survivors (dset = {p}) give the lower ends, may-survivors (some p in
    dset) the upper ends, of counts, pattern counts, best keys, bins and rays;
    a partial turn of 80 rays of N = 90, two rules."""
    nt = 80
    g = (0.5, 40, 4.0, nt)
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(617, 5)])
    for rule in ((50, 0.5, 0x7F), (100, 0.25, 0x2D)):
        allc = oracle.eval_all(cols, g, rule)
        out = oracle.reduce_bounds(cols, g, rule, bins=True, rays=True)
        b = out["bounds"]
        summ = oracle.reduce(cols, g, rule)
        for k in range(len(cols)):
            ds = allc[k]["dset"].astype(np.int64)
            may = (ds & 0xFE) != 0
            must = (ds & 1) == 0
            ii, jj = np.meshgrid(np.arange(40), np.arange(nt), indexing="ij")
            key = (ii << 16) | (0xFFFF - jj)
            assert b["count_lo"][k] == must.sum() and b["count_hi"][k] == may.sum()
            assert b["count_lo"][k] <= summ["count"][k] <= b["count_hi"][k]
            assert b["n_ambiguous"][k] == summ["n_ambiguous"][k] == ((allc[k]["boundary"] & 2) != 0).sum()
            assert b["key_lo"][k] == (key[must].max() if must.any() else 0)
            assert b["key_hi"][k] == (key[may].max() if may.any() else 0)
            for p in range(1, 8):
                one = ds == (1 << p)
                some = ((ds >> p) & 1) == 1
                assert b["pat_lo"][k][p - 1] == one.sum() and b["pat_hi"][k][p - 1] == some.sum()
                assert b["pkey_lo"][k][p - 1] == (key[one].max() if one.any() else 0)
                assert b["pkey_hi"][k][p - 1] == (key[some].max() if some.any() else 0)
            for j in range(nt):
                lo = ii[:, j][must[:, j]]
                hi = ii[:, j][may[:, j]]
                assert out["rays_lo"][k][j] == (lo.max() + 1 if len(lo) else 0)
                assert out["rays_hi"][k][j] == (hi.max() + 1 if len(hi) else 0)
            for q in range(36):
                sel = (4 * jj) // 10 == q
                lo = ii[must & sel]
                hi = ii[may & sel]
                assert out["bins_lo"][k][q] == (lo.max() + 1 if len(lo) else 0)
                assert out["bins_hi"][k][q] == (hi.max() + 1 if len(hi) else 0)
