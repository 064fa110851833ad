"""Exact one-pair resolve with a global early exit (cv_best_pair_search): each
colour's maximum-amplitude survivor equals the exhaustive reduce's best pair
and the adaptive per-ray search's best key bit for bit (the same arithmetic on
every candidate it evaluates), and stays within the FP64 oracle's per-colour
range, with every reported pair re-evaluated by the oracle."""
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


CASES = [
    ("frames grid", (0.1, 500, 1.0, 360), (50, 0.5, 0x7F, 0)),
    ("partial turn", (0.5, 90, 2.0, 131), (50, 0.5, 0x7F, 0)),
    ("cube grid, mask", (0.25, 200, 2.0, 180), (100, 0.25, 0x15, 0)),
    ("clip reading", (0.5, 120, 2.0, 180), (50, 0.5, 0x7F, 1)),
    ("long rays", (0.02, 5000, 6.0, 60), (50, 0.5, 0x7F, 0)),
    ("one level", (1.5, 40, 10.0, 36), (50, 0.5, 0x7F, 0)),
    ("wide turn", (0.5, 70, 0.5, 720), (50, 0.5, 0x7F, 0)),
]


def _colours(n_random, seed):
    return np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(seed, n_random),
                           np.array([[0, 0, 0], [255, 255, 255], [1, 254, 3], [128, 128, 128]], np.uint8)])


@pytest.mark.parametrize("name,grid,rule", CASES, ids=[c[0] for c in CASES])
def test_best_pair_equals_the_exhaustive_best(cv, name, grid, rule):
    cols = _colours(400, 131)
    x = torch.from_numpy(cols).cuda()
    g, r = cv.Grid(*grid), cv.Rule(*rule)
    bp = cv.best_pair_search(x, g, r)
    summ, _ = cv.pair_reduce(x, g, r)
    ray = cv.ray_search(x, g, r, best=True)
    torch.cuda.synchronize()
    s = cv.as_records(summ, cv.SUMMARY_DTYPE)
    key = bp.best.cpu().numpy().view(np.uint32).astype(np.int64)
    want = parity._key(s["best_i"], s["best_j"])
    assert np.array_equal(key, want), name
    assert np.array_equal(key, ray.best.cpu().numpy().view(np.uint32).astype(np.int64)), name
    p = cv.as_records(bp.pairs.reshape(-1, 16), cv.PAIR_DTYPE)
    assert np.array_equal(p["colour"], np.arange(len(cols)))
    has = key > 0
    assert np.all(p["flags"][has] & 4) and np.all(p["flags"][~has] == 0)
    assert np.array_equal(p["i"][has], s["best_i"][has]) and np.array_equal(p["j"][has], s["best_j"][has])
    assert np.array_equal(p["plus"][has], s["best_plus"][has])
    assert np.array_equal(p["minus"][has], s["best_minus"][has])
    assert np.array_equal(p["pattern"][has], s["best_p"][has])
    assert np.all(p["i"][~has] == 0) and np.all(p["pattern"][~has] == 0)
    ev, tested, closed = (int(v) for v in bp.counts.cpu().numpy())
    ev_ray = int(ray.counts[0].item())
    total = len(cols) * grid[1] * grid[3]
    print(f"{name}: {int(has.sum())} of {len(cols)} colours with a pair; evaluated {ev} candidates "
          f"({ev / total:.4f} of the grid; the per-ray search {ev_ray}); {closed} of {tested} blocks closed")
    assert 0 < ev <= ev_ray
    if rule[3] & 1:
        assert closed == 0


def test_best_pair_within_the_oracle_range(cv, oracle):
    """Distinct colours of a synthetic 4K frame on the batched-frames grid:
    the key within the oracle's per-colour range (a single value where no
    band candidate can move it) and every pair re-evaluated by the oracle."""
    f = cv.frames_generate([3], 2160, 3840).cpu().numpy()
    ids = oracle.distinct_colours(f)
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(len(ids), 400, replace=False))
    cols = np.concatenate([W.cube_colours(ids[sample]), W.PAPER_COLOUR_ARRAY])
    grid, rule = W.GRID_FRAMES.astuple(), W.DEFAULT_RULE
    bp = cv.best_pair_search(torch.from_numpy(cols).cuda(), cv.Grid(*grid), cv.Rule(*rule))
    torch.cuda.synchronize()
    b = oracle.reduce_bounds(cols, grid, rule)["bounds"]
    key = bp.best.cpu().numpy().view(np.uint32).astype(np.int64)
    parity.within(b["key_lo"], key, b["key_hi"], "best (i, j)")
    p = cv.as_records(bp.pairs.reshape(-1, 16), cv.PAIR_DTYPE)
    has = key > 0
    parity._check_pairs(oracle, cols, grid, rule, np.nonzero(has)[0], p["i"][has], p["j"][has],
                        p["plus"][has], p["minus"][has], p["pattern"][has], "best pair")
    assert int((b["key_lo"] == b["key_hi"]).sum()) > len(cols) // 2


def test_best_pair_degenerate(cv):
    g, r = cv.Grid(0.5, 80, 2.0, 180), cv.Rule(50, 0.5)
    empty = torch.zeros((0, 3), dtype=torch.uint8, device="cuda")
    res = cv.best_pair_search(empty, g, r)
    torch.cuda.synchronize()
    assert int(res.counts.sum()) == 0
    cols = torch.from_numpy(W.random_colours(121, 40)).cuda()
    for grid in ((30.0, 1, 180.0, 1), (40.0, 2, 180.0, 2), (0.5, 1, 1.0, 360), (0.3, 65, 1.0, 360)):
        a = cv.best_pair_search(cols, cv.Grid(*grid), r)
        summ, _ = cv.pair_reduce(cols, cv.Grid(*grid), r)
        torch.cuda.synchronize()
        s = cv.as_records(summ, cv.SUMMARY_DTYPE)
        assert np.array_equal(a.best.cpu().numpy().view(np.uint32).astype(np.int64),
                              parity._key(s["best_i"], s["best_j"])), grid
