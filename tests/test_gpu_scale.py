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
    s_o, tc, tb = oracle.reduce(sub, grid, rule, table=True)
    ok = s_o["n_ambiguous"] == 0
    assert ok.mean() > 0.5
    assert np.array_equal(t["count"][ok], tc[ok])
    assert np.array_equal(t["bin_ridx"][ok], tb[ok])
    assert np.all(np.abs(t["count"].astype(np.int64) - tc) <= s_o["n_ambiguous"])
    print(f"cube: {ok.sum()} of {len(ids)} sampled rows exact, "
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
    s_o = oracle.reduce(sc, grid, rule)
    s_g = cv.as_records(res.summaries[torch.from_numpy(sample).cuda()], cv.SUMMARY_DTYPE)
    ok = s_o["n_ambiguous"] == 0  # on this fine grid most colours have a few
    assert ok.sum() > 100
    for k in ("count", "n_gamut", "best_i", "per_pattern"):
        assert np.array_equal(s_g[k][ok], s_o[k][ok]), k
    some = ok & (s_o["count"] > 0)  # best_j, best_p and the codes exist only with a survivor
    for k in ("best_j", "best_p"):
        assert np.array_equal(s_g[k][some], s_o[k][some]), k
    assert np.all(np.abs(s_g["count"].astype(np.int64) - s_o["count"]) <= s_o["n_ambiguous"])
    # per-ray maxima and per-pattern best pairs on a smaller sample
    small = sample[:400]
    recs, offs, _ = oracle.search(W.cube_colours(ids[small]), grid, rule)
    rays_g = res.rays[torch.from_numpy(small).cuda()].cpu().numpy().view(np.uint16)
    pb_g = cv.as_records(res.pbest[torch.from_numpy(small).cuda()].reshape(-1, 12),
                         cv.PATTERN_PAIR_DTYPE).reshape(-1, 7)
    checked = 0
    for k in range(len(small)):
        if not ok[k]:
            continue
        seg = recs[offs[k]:offs[k + 1]]
        rays_o = np.zeros(grid[3], dtype=np.int64)
        np.maximum.at(rays_o, seg["j"].astype(np.int64), seg["i"].astype(np.int64) + 1)
        assert np.array_equal(rays_g[k].astype(np.int64), rays_o), k
        for p in range(1, 8):
            sp = seg[seg["pattern"] == p]
            g = pb_g[k, p - 1]
            if len(sp) == 0:
                assert g["flags"] == 0
                continue
            b = sp[np.lexsort((sp["j"], -sp["i"].astype(np.int64)))[0]]
            assert g["flags"] == 1 and (g["i"], g["j"]) == (b["i"], b["j"])
            if not b["flags"] & 1:
                assert np.array_equal(g["plus"], b["plus"]) and np.array_equal(g["minus"], b["minus"])
        checked += 1
    assert checked > 40
    print(f"frames: {n} distinct colours in {len(f)} frames of {npix_frame} pixels; "
          f"{int(has.sum())} pixels carry a pair")
