"""Full-size configurations on the GPU, checked on sampled outputs against the
FP64 oracle and through properties that hold at any size:

- the whole RGB cube (2^24 colours) on the 200 x 180 grid -> angle-bin table;
- eight synthetic 3840 x 2160 frames on the 500 x 360 grid -> de-duplicated
  colours, per-colour results and the two rendered frames.
"""
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


def cube_ids_device():
    ids = torch.arange(1 << 24, dtype=torch.int32, device="cuda")
    return torch.stack([(ids >> 16) & 255, (ids >> 8) & 255, ids & 255], dim=1).to(torch.uint8)


def test_cube_table_full(cv, oracle):
    grid = W.GRID_CUBE.astuple()
    rule = W.DEFAULT_RULE
    cols = cube_ids_device()
    summ, tab = cv.pair_reduce(cols, cv.Grid(*grid), cv.Rule(*rule), table=True)
    torch.cuda.synchronize()
    # properties over all 2^24 rows: half-turn symmetry (bin k and k + 18 hold
    # mirrored pairs) and agreement of the table count with the summary count
    bins = tab[:, 4:40]
    assert torch.equal(bins[:, :18], bins[:, 18:])
    cnt = tab[:, :4].contiguous().view(torch.int32)
    assert torch.equal(cnt, summ[:, :4].contiguous().view(torch.int32))
    assert int((cnt & 1).sum()) == 0
    assert int((bins.max(dim=1).values > 0).sum()) == int((cnt > 0).sum())
    # sampled rows against the oracle
    rng = np.random.default_rng(4)
    ids = np.unique(np.concatenate([rng.integers(0, 1 << 24, 1536),
                                    [0, 0xFF, 0xFF00, 0xFFFF, 0xFF0000, 0xFF00FF, 0xFFFF00, 0xFFFFFF],
                                    (W.PAPER_COLOUR_ARRAY.astype(np.int64) << [16, 8, 0]).sum(1)]))
    sub = W.cube_colours(ids)
    t = cv.as_records(tab[torch.from_numpy(ids).cuda()], cv.TABLE_DTYPE)
    r = parity.check_table(oracle, sub, grid, rule, t)
    s_g = cv.as_records(summ[torch.from_numpy(ids).cuda()], cv.SUMMARY_DTYPE)
    _, st = parity.check_summaries(oracle, sub, grid, rule, s_g, bounds=r["bounds"])
    fixed = (r["bins_lo"] == r["bins_hi"]).all(1) & (r["bounds"]["count_lo"] == r["bounds"]["count_hi"])
    print(f"cube: {len(ids)} sampled rows, {int(fixed.sum())} with no movable field; {st}; "
          f"{int((cnt > 0).sum())} of 2^24 colours feasible")


def test_frames_4k_full(cv, oracle):
    f = W.frames(range(8))
    info = W.info_map(0)
    npix_frame = f.shape[1] * f.shape[2]
    grid = W.GRID_FRAMES.astuple()
    rule = W.DEFAULT_RULE
    px = torch.from_numpy(f).cuda()
    inf = torch.from_numpy(np.tile(info.reshape(-1), len(f))).cuda()
    res = cv.frames_resolve(px, cv.Grid(*grid), cv.Rule(*rule), info=inf, rays=True, graph=True)
    torch.cuda.synchronize()
    n = int(res.ncolours.item())
    ids = oracle.distinct_colours(f)
    assert n == len(ids)
    cols = res.colours[:n]
    assert np.array_equal(cols.cpu().numpy(), W.cube_colours(ids))
    # every pixel's index points at its own colour
    idx = res.pixel_index.long()
    assert torch.equal(cols[idx], px.reshape(-1, 3))
    # rendering against a composition of the GPU's own per-colour pairs
    pb = res.pbest.reshape(-1, 7, 12)[idx, inf.long() - 1]     # [npix, 12]
    has = (pb[:, 11] & 1).bool()
    ref_a = torch.where(has[:, None], pb[:, 4:7], px.reshape(-1, 3))
    ref_b = torch.where(has[:, None], pb[:, 7:10], px.reshape(-1, 3))
    assert torch.equal(res.frame_a, ref_a) and torch.equal(res.frame_b, ref_b)
    assert int(res.resolved.item()) == int(has.sum())
    # sampled colours against the oracle
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(n, 1024, replace=False))
    sc = W.cube_colours(ids[sample])
    s_g = cv.as_records(res.summaries[torch.from_numpy(sample).cuda()], cv.SUMMARY_DTYPE)
    r = oracle.reduce_bounds(sc, grid, rule, rays=True)
    _, st = parity.check_summaries(oracle, sc, grid, rule, s_g, bounds=r["bounds"])
    # per-ray maxima and per-pattern best pairs of the same colours
    rays_g = res.rays[torch.from_numpy(sample).cuda()].cpu().numpy().view(np.uint16)
    parity.check_rays(oracle, sc, grid, rule, rays_g, r)
    pb_g = cv.as_records(res.pbest[torch.from_numpy(sample).cuda()].reshape(-1, 12),
                         cv.PATTERN_PAIR_DTYPE).reshape(-1, 7)
    nb = parity.check_pattern_bests(oracle, sc, grid, rule, pb_g, bounds=r["bounds"])
    print(f"frames sample: {st}; {nb} band pattern-best pairs; "
          f"{int((r['rays_lo'] != r['rays_hi']).sum())} of {r['rays_lo'].size} rays movable")
    print(f"frames: {n} distinct colours in {len(f)} frames of {npix_frame} pixels; "
          f"{int(has.sum())} pixels carry a pair")
