"""Adaptive per-ray search (cv_ray_search) on the GPU: its per-ray maxima and
records against the exhaustive per-ray search of the same library (bit for
bit) and against the FP64 oracle's per-ray ranges (per candidate), on the
batched-frames grid and on grids that exercise every tiling of the kernel."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import workloads as W

import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cv():
    import paper_2507_22901_amd as cv
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cv.lib()
    return cv


def _dense_per_ray(cv, res, n, nt):
    """The exhaustive per-ray list (CV_PER_RAY) as dense [n, nt] maxima and records."""
    g = cv.as_records(res.pairs, cv.PAIR_DTYPE)
    rays = np.zeros((n, nt), np.int64)
    recs = np.zeros((n, nt), cv.PAIR_DTYPE)
    recs["colour"] = np.arange(n)[:, None]
    c, j = g["colour"].astype(np.int64), g["j"].astype(np.int64)
    rays[c, j] = g["i"].astype(np.int64) + 1
    recs[c, j] = g
    return rays, recs


CASES = [
    ("frames grid", (0.1, 500, 1.0, 360), (50, 0.5, 0x7F, 0)),
    ("partial turn", (0.5, 90, 2.0, 131), (50, 0.5, 0x7F, 0)),
    ("cube grid, mask", (0.25, 200, 2.0, 180), (100, 0.25, 0x15, 0)),
    ("clip reading", (0.5, 120, 2.0, 180), (50, 0.5, 0x7F, 1)),
    ("long rays", (0.02, 5000, 6.0, 60), (50, 0.5, 0x7F, 0)),
    ("one ray block", (1.5, 40, 10.0, 36), (50, 0.5, 0x7F, 0)),
]


@pytest.mark.parametrize("name,grid,rule", CASES, ids=[c[0] for c in CASES])
def test_rays_equal_exhaustive_per_ray(cv, name, grid, rule):
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(120, 55),
                           np.array([[0, 0, 0], [255, 255, 255], [1, 254, 3]], np.uint8)])
    x = torch.from_numpy(cols).cuda()
    g, r = cv.Grid(*grid), cv.Rule(*rule)
    ad = cv.ray_search(x, g, r, records=True)
    ex = cv.pair_search(x, g, r, per_ray=True)
    torch.cuda.synchronize()
    rays_e, recs_e = _dense_per_ray(cv, ex, len(cols), grid[3])
    rays_a = ad.rays.cpu().numpy().view(np.uint16).astype(np.int64)
    assert np.array_equal(rays_a, rays_e), name
    recs_a = cv.as_records(ad.records.reshape(-1, 16), cv.PAIR_DTYPE).reshape(len(cols), grid[3])
    has = rays_e > 0
    assert np.array_equal(recs_a[has], recs_e[has]), name
    assert np.all(recs_a["flags"][~has] == 0) and np.all(recs_a["i"][~has] == 0)
    assert np.array_equal(recs_a["colour"], np.broadcast_to(np.arange(len(cols))[:, None], rays_a.shape))
    ev, tested, closed = (int(v) for v in ad.counts.cpu().numpy())
    total = len(cols) * grid[1] * grid[3]
    print(f"{name}: {int(has.sum())} rays with a survivor of {has.size}; evaluated {ev} of {total} "
          f"candidates ({ev / total:.3f}); {closed} of {tested} row blocks closed by the bound")
    assert 0 < ev <= total
    if rule[3] & 1:
        assert closed == 0
    else:
        assert closed > 0


def test_rays_match_oracle_on_frame_colours(cv, oracle):
    """A sample of a synthetic 4K frame's distinct colours on the batched
    frames grid (r = 0.1..50 x 1 deg): every per-ray maximum within the
    oracle's range and every record re-evaluated by the oracle."""
    f = W.frames([0])
    ids = oracle.distinct_colours(f)
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(len(ids), 300, replace=False))
    cols = np.concatenate([W.cube_colours(ids[sample]), W.PAPER_COLOUR_ARRAY])
    grid = W.GRID_FRAMES.astuple()
    rule = W.DEFAULT_RULE
    ad = cv.ray_search(torch.from_numpy(cols).cuda(), cv.Grid(*grid), cv.Rule(*rule), records=True)
    torch.cuda.synchronize()
    rays = ad.rays.cpu().numpy().view(np.uint16)
    recs = cv.as_records(ad.records.reshape(-1, 16), cv.PAIR_DTYPE)
    r = parity.check_rays(oracle, cols, grid, rule, rays)
    have = recs["flags"] != 0
    offs = np.concatenate([[0], np.cumsum(have.reshape(len(cols), -1).sum(1))])
    parity.check_ray_records(oracle, cols, grid, rule, recs[have], offs, r)
    ev = int(ad.counts[0].item())
    total = len(cols) * grid[1] * grid[3]
    print(f"frame colours: {int(have.sum())} rays with a survivor; "
          f"{int((r['rays_lo'] != r['rays_hi']).sum())} of {r['rays_lo'].size} rays movable; "
          f"evaluated {ev / total:.4f} of the candidates")


@pytest.mark.parametrize("grid", [(0.1, 500, 1.0, 360), (0.5, 90, 2.0, 131)])
def test_best_key_is_the_maximum_amplitude_pair(cv, grid):
    """The per-colour best key of the adaptive search (an exact one-pair
    resolve from the outermost radius inward) equals the exhaustive reduce's
    maximum-amplitude pair."""
    cols = torch.from_numpy(np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(122, 2500)])).cuda()
    g, r = cv.Grid(*grid), cv.Rule(50, 0.5)
    ad = cv.ray_search(cols, g, r, best=True)
    summ, _ = cv.pair_reduce(cols, g, r)
    torch.cuda.synchronize()
    s = cv.as_records(summ, cv.SUMMARY_DTYPE)
    key = ad.best.cpu().numpy().view(np.uint32).astype(np.int64)
    want = np.where(s["best_i"] == 0xFFFF, 0,
                    (s["best_i"].astype(np.int64) << 16) | (0xFFFF - s["best_j"].astype(np.int64)))
    assert np.array_equal(key, want)


def test_rays_degenerate(cv):
    g, r = cv.Grid(0.5, 80, 2.0, 180), cv.Rule(50, 0.5)
    empty = torch.zeros((0, 3), dtype=torch.uint8, device="cuda")
    res = cv.ray_search(empty, g, r)
    assert res.rays.numel() == 0 and int(res.counts.sum()) == 0
    # one radius, one angle
    cols = torch.from_numpy(W.random_colours(121, 40)).cuda()
    for grid in ((30.0, 1, 180.0, 1), (40.0, 2, 180.0, 2), (0.5, 1, 1.0, 360)):
        a = cv.ray_search(cols, cv.Grid(*grid), r)
        e = cv.pair_search(cols, cv.Grid(*grid), r, per_ray=True)
        torch.cuda.synchronize()
        rays_e, _ = _dense_per_ray(cv, e, 40, grid[3])
        assert np.array_equal(a.rays.cpu().numpy().view(np.uint16).astype(np.int64), rays_e), grid
