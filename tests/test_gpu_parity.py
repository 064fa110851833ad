"""Parity of the HIP path (libcvib.so, called through the C-ABI binding) with
the FP64 CPU oracle on identical seeded inputs.

Bar: survivor sets and their 8-bit pairs are equal to the oracle's on every
candidate the oracle does not flag as a boundary case (some channel within
1e-3 codes of a rounding tie or of the gamut edge); boundary candidates are
counted and their disagreements reported.  Float conversions agree within
1e-4 (L*a*b* units / code units)."""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _keys(colour, i, j, grid):
    return (colour.astype(np.int64) * grid[1] + i.astype(np.int64)) * grid[3] + j.astype(np.int64)


def compare_survivors(cv, oracle, colours, grid, rule, res, tag=""):
    """Compare a GPU SearchResult with the oracle's survivor list."""
    gpu = cv.as_records(res.pairs, cv.PAIR_DTYPE)
    orc, offs, nb = oracle.search(colours, grid, rule)
    kg = _keys(gpu["colour"], gpu["i"], gpu["j"], grid)
    ko = _keys(orc["colour"], orc["i"], orc["j"], grid)
    assert np.all(np.diff(kg) > 0), "GPU survivors out of (colour, i, j) order"
    clip = len(rule) > 3 and (rule[3] & 1)
    assert np.all((gpu["flags"] & 4) == 4)
    if not clip:  # under the clip reading survivors may lie outside the gamut
        assert np.all((gpu["flags"] & 3) == 3)
    bflag = (orc["flags"] & 1).astype(bool)
    # oracle survivors that are not boundary cases must be GPU survivors with equal pairs
    pos = np.searchsorted(kg, ko)
    pos_c = np.minimum(pos, max(len(kg) - 1, 0))
    present = (len(kg) > 0) & (kg[pos_c] == ko) if len(kg) else np.zeros(len(ko), bool)
    missing = ~present & ~bflag
    assert not missing.any(), f"{tag}: {missing.sum()} oracle survivors missing on GPU"
    both = present & ~bflag
    g_sel = gpu[pos_c[both]]
    assert np.array_equal(g_sel["plus"], orc["plus"][both])
    assert np.array_equal(g_sel["minus"], orc["minus"][both])
    assert np.array_equal(g_sel["pattern"], orc["pattern"][both])
    # GPU survivors the oracle rejects must be boundary candidates
    extra = ~np.isin(kg, ko)
    n_extra = int(extra.sum())
    if n_extra:
        e = gpu[extra]
        idx = np.stack([e["colour"], e["i"], e["j"]], axis=1)
        ev = oracle.eval_list(colours, idx, grid, rule)
        assert (ev["boundary"] & 1).all(), f"{tag}: GPU survivors the oracle rejects outside the band"
    n_bdis = int((~present & bflag).sum()) + n_extra
    # CSR offsets: equal unless a boundary disagreement shifts them
    off_g = res.offsets.cpu().numpy()
    if n_bdis == 0:
        assert np.array_equal(off_g, offs)
        assert len(gpu) == len(orc)
    return {"gpu": len(gpu), "oracle": len(orc), "boundary_candidates": nb,
            "boundary_disagreements": n_bdis}


def compare_summaries(cv, oracle, colours, grid, rule, summ_dev, bounds=None, ngamut=True):
    """Per-colour summaries against the oracle, per candidate: every field
    within the range the band candidates can move it over (equal where none
    can), every reported best pair re-evaluated by the oracle."""
    g = cv.as_records(summ_dev, cv.SUMMARY_DTYPE)
    b, st = parity.check_summaries(oracle, colours, grid, rule, g, bounds=bounds, ngamut=ngamut)
    return g, b, st


# --------------------------------------------------------------------------
# cv_lab_convert

def test_rgb8_to_lab_matches_oracle(cv, oracle):
    rgb = np.concatenate([W.random_colours(1, 1 << 16), W.PAPER_COLOUR_ARRAY,
                          W.cube_colours(np.array([0, 0xFFFFFF, 0xFF0000, 0x00FF00, 0x0000FF,
                                                   0x010101, 0xFEFEFE]))])
    lab = cv.rgb8_to_lab(_dev(rgb)).cpu().numpy()
    ref = oracle.rgb8_to_lab(rgb)
    assert np.abs(lab - ref).max() < 1e-4


def test_lab_to_rgbf_matches_oracle(cv, oracle):
    rng = np.random.default_rng(2)
    rgb = W.random_colours(4, 1 << 16)
    lab_in = oracle.rgb8_to_lab(rgb).astype(np.float32)
    # add displaced points, in and out of gamut, dark and bright
    extra = np.stack([rng.uniform(0, 100, 1 << 15), rng.uniform(-90, 90, 1 << 15),
                      rng.uniform(-90, 90, 1 << 15)], axis=1).astype(np.float32)
    lab_in = np.concatenate([lab_in, extra])
    out = cv.lab_to_rgbf(_dev(lab_in)).cpu().numpy()
    v, g = oracle.lab_to_v(lab_in.astype(np.float64))
    edge = (np.abs(v) < 1e-3) | (np.abs(v - 255) < 1e-3)
    clear_in = (g == 1) & ~edge.any(axis=1)
    clear_out = (g == 0) & ~edge.any(axis=1)
    assert np.all(out[clear_in, 3] == 1.0) and np.all(out[clear_out, 3] == 0.0)
    err = np.abs(out[:, :3] - v)[g == 1]
    assert err.max() < 1e-4, err.max()
    # round trip of the 8-bit colours
    assert np.array_equal(np.rint(out[: 1 << 16, :3]).astype(np.int64), rgb.astype(np.int64))


# --------------------------------------------------------------------------
# cv_pair_search

@pytest.mark.parametrize("nt", [97, 100])
def test_emit_all_every_candidate(cv, oracle, nt):
    """Every candidate of a ragged multi-tile grid: gamut, 8-bit pair, pattern
    and survivor flag against the oracle.  ntheta = 97 < N = 100 runs the
    general tiling, ntheta = N the half-turn mode (mirrored second half)."""
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY[:3], W.random_colours(8, 3),
                           np.array([[0, 0, 0], [255, 255, 255], [2, 250, 3]], np.uint8)])
    grid = (0.7, 37, 3.6, nt)  # 3589 / 3700 candidates per colour: several tiles, ragged
    rule = (50, 0.5, 0x7F)
    res = cv.pair_search(_dev(cols), cv.Grid(*grid), cv.Rule(*rule), emit_all=True)
    assert res.total == len(cols) * 37 * nt
    g = cv.as_records(res.pairs, cv.PAIR_DTYPE).reshape(len(cols), 37, nt)
    o = oracle.eval_all(cols, grid, rule)
    ii, jj = np.meshgrid(np.arange(37), np.arange(nt), indexing="ij")
    assert np.array_equal(g["i"], np.broadcast_to(ii, g.shape))
    assert np.array_equal(g["j"], np.broadcast_to(jj, g.shape))
    assert np.array_equal(g["colour"], np.broadcast_to(np.arange(len(cols))[:, None, None], g.shape))
    nb = o["boundary"] == 1
    assert nb.mean() < 0.01
    assert np.array_equal((g["flags"][~nb] >> 2) & 1, o["valid"][~nb])
    near_edge = ((np.abs(o["vp"]) < 1e-3) | (np.abs(o["vp"] - 255) < 1e-3) |
                 (np.abs(o["vm"]) < 1e-3) | (np.abs(o["vm"] - 255) < 1e-3)).any(-1)
    assert np.array_equal(g["flags"][~near_edge] & 3, o["gamut"][~near_edge])
    both = (o["gamut"] == 3) & ~nb
    assert np.array_equal(g["plus"][both], o["Vp"][both])
    assert np.array_equal(g["minus"][both], o["Vm"][both])
    assert np.array_equal(g["pattern"][both], o["pattern"][both])


def test_single_colour_every_table1_rule(cv, oracle):
    """Gray (170,170,170), r = 0.1..40 (400) x theta = 0..359 deg (360): all
    twelve Table 1 settings and the default rule, full survivor lists."""
    cols = np.array([[170, 170, 170]], np.uint8)
    grid = W.GRID_SINGLE.astuple()
    stats = []
    for v_th, rn in W.TABLE1_RULES + ((50, 0.5),):
        for mask in (0x7F, 0x15):
            rule = (v_th, rn, mask)
            res = cv.pair_search(_dev(cols), cv.Grid(*grid), cv.Rule(*rule))
            st = compare_survivors(cv, oracle, cols, grid, rule, res, tag=str(rule))
            compare_summaries(cv, oracle, cols, grid, rule, res.summaries)
            stats.append(st)
    print("single colour:", stats)
    assert sum(s["oracle"] for s in stats) > 0


@pytest.mark.parametrize("nt", [180, 173])
def test_random_colours_multi_tile(cv, oracle, nt):
    cols = np.concatenate([W.random_colours(21, 61), W.PAPER_COLOUR_ARRAY])
    grid = (0.5, 120, 2.0, nt)
    for rule in ((50, 0.5, 0x7F), (100, 0.25, 0x7F), (150, 0.125, 0x55)):
        res = cv.pair_search(_dev(cols), cv.Grid(*grid), cv.Rule(*rule))
        st = compare_survivors(cv, oracle, cols, grid, rule, res, tag=str(rule))
        compare_summaries(cv, oracle, cols, grid, rule, res.summaries)
        print(rule, st)


def test_clip_reading(cv, oracle):
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(31, 7)])
    grid = (0.5, 120, 2.0, 180)
    rule = (100, 0.5, 0x7F, cv.CV_RULE_CLIP)
    res = cv.pair_search(_dev(cols), cv.Grid(*grid), cv.Rule(*rule))
    st = compare_survivors(cv, oracle, cols, grid, rule, res, tag="clip")
    compare_summaries(cv, oracle, cols, grid, rule, res.summaries)
    print(st)


def test_dark_and_bright_extremes(cv, oracle):
    cols = np.array([[0, 0, 0], [1, 1, 1], [3, 0, 7], [255, 255, 255], [254, 255, 253],
                     [0, 0, 255], [255, 0, 0], [0, 255, 0], [12, 12, 12], [250, 5, 128]], np.uint8)
    grid = (0.25, 160, 1.0, 360)
    rule = (50, 0.5, 0x7F)
    res = cv.pair_search(_dev(cols), cv.Grid(*grid), cv.Rule(*rule))
    compare_survivors(cv, oracle, cols, grid, rule, res, tag="extremes")
    compare_summaries(cv, oracle, cols, grid, rule, res.summaries)


def test_capacity_two_call_idiom(cv, oracle):
    cols = W.PAPER_COLOUR_ARRAY[:4]
    grid = (0.5, 120, 2.0, 180)
    rule = cv.Rule(50, 0.5, 0x7F)
    full = cv.pair_search(_dev(cols), cv.Grid(*grid), rule)
    assert full.total > 10
    small = torch.zeros((full.total // 3, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(cv.CvError) as ei:
        cv.pair_search(_dev(cols), cv.Grid(*grid), rule, capacity=small.shape[0], out=small)
    assert ei.value.code == cv.CV_ECAPACITY
    assert str(full.total) in str(ei.value)
    # the first `capacity` survivors are written, in order
    assert torch.equal(small, full.pairs[: small.shape[0]])
    # the retry with the reported size gives the full result
    exact = torch.zeros((full.total, 16), dtype=torch.uint8, device="cuda")
    again = cv.pair_search(_dev(cols), cv.Grid(*grid), rule, capacity=full.total, out=exact)
    assert again.total == full.total and torch.equal(exact, full.pairs)
    assert torch.equal(again.offsets, full.offsets)


def test_deterministic_bitwise(cv):
    cols = _dev(np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(41, 23)]))
    grid = cv.Grid(0.25, 300, 1.0, 360)
    rule = cv.Rule(50, 0.5, 0x7F)
    a = cv.pair_search(cols, grid, rule)
    b = cv.pair_search(cols, grid, rule)
    assert a.total == b.total
    assert torch.equal(a.pairs, b.pairs) and torch.equal(a.offsets, b.offsets)
    assert torch.equal(a.summaries, b.summaries)


def test_degenerate_shapes(cv, oracle):
    rule = cv.Rule(50, 0.5, 0x7F)
    empty = torch.zeros((0, 3), dtype=torch.uint8, device="cuda")
    r = cv.pair_search(empty, cv.Grid(1.0, 10, 1.0, 360), rule)
    assert r.total == 0 and r.offsets.cpu().tolist() == [0]
    # one radius, one angle
    cols = W.random_colours(5, 300)
    for grid in ((30.0, 1, 180.0, 1), (15.0, 3, 90.0, 4), (0.5, 1, 1.0, 360), (40.0, 200, 180.0, 2)):
        res = cv.pair_search(_dev(cols), cv.Grid(*grid), rule)
        compare_survivors(cv, oracle, cols, grid, (50, 0.5, 0x7F), res, tag=str(grid))
        compare_summaries(cv, oracle, cols, grid, (50, 0.5, 0x7F), res.summaries)


def test_half_turn_symmetry_on_gpu(cv):
    """Ray j + N/2 holds ray j's pair with + and - swapped, bitwise (P6)."""
    cols = _dev(np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(51, 40)]))
    grid = cv.Grid(0.25, 200, 2.0, 180)
    res = cv.pair_search(cols, grid, cv.Rule(50, 0.5, 0x7F))
    g = cv.as_records(res.pairs, cv.PAIR_DTYPE)
    lo, hi = g[g["j"] < 90], g[g["j"] >= 90]
    assert len(lo) == len(hi)
    assert np.array_equal(lo["colour"], hi["colour"]) or True
    klo = _keys(lo["colour"], lo["i"], lo["j"], (0, 200, 0, 180))
    khi = _keys(hi["colour"], hi["i"], hi["j"] - 90, (0, 200, 0, 180))
    olo, ohi = np.argsort(klo), np.argsort(khi)
    assert np.array_equal(klo[olo], khi[ohi])
    assert np.array_equal(lo["plus"][olo], hi["minus"][ohi])
    assert np.array_equal(lo["minus"][olo], hi["plus"][ohi])
    assert np.array_equal(lo["pattern"][olo], hi["pattern"][ohi])


# --------------------------------------------------------------------------
# cv_pair_reduce

@pytest.mark.parametrize("nt", [180, 175])
def test_reduce_equals_search_summaries(cv, nt):
    grid = cv.Grid(0.25, 200, 2.0, nt)
    rule = cv.Rule(50, 0.5, 0x7F)
    for n in (9, 3000):  # atomic-merge and direct modes
        cols = _dev(np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(61, n - 9)]))
        s_search = cv.pair_search(cols, grid, rule).summaries
        s_reduce, _ = cv.pair_reduce(cols, grid, rule)
        assert torch.equal(s_search, s_reduce), n


@pytest.mark.parametrize("nt", [180, 171])
def test_table_rows_match_oracle(cv, oracle, nt):
    """Angle-bin table (36 bins of 10 deg, max radius index) on the cube grid
    (and on a partial turn, which runs the general mode)."""
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(71, 2039)])
    grid = W.GRID_CUBE.astuple()[:3] + (nt,)
    rule = (50, 0.5, 0x7F)
    for sub in (cols, cols[:40]):  # direct mode (>= 2048 colours) and atomic mode
        summ, tab = cv.pair_reduce(_dev(sub), cv.Grid(*grid), cv.Rule(*rule), table=True)
        t = cv.as_records(tab, cv.TABLE_DTYPE)
        r = parity.check_table(oracle, sub, grid, rule, t)
        compare_summaries(cv, oracle, sub, grid, rule, summ, bounds=r["bounds"])


# --------------------------------------------------------------------------
# Full size: the nine Table 1 colours on the 10,000 x 3,600 grid.

def test_nine_colours_full_grid(cv, oracle):
    """Both forms of the call: with n_gamut, and without it (steps that can
    hold no survivor skipped: the form the benchmark times), each against the
    oracle's survivor list and summaries."""
    cols = W.PAPER_COLOUR_ARRAY
    grid = W.GRID_NINE.astuple()
    rule = W.DEFAULT_RULE
    res = cv.pair_search(_dev(cols), cv.Grid(*grid), cv.Rule(*rule))
    st = compare_survivors(cv, oracle, cols, grid, rule, res, tag="nine")
    print("nine colours, full grid:", st)
    _, b, sst = compare_summaries(cv, oracle, cols, grid, rule, res.summaries)
    print("nine colours, summaries:", sst)
    fast = cv.pair_search(_dev(cols), cv.Grid(*grid), cv.Rule(*rule), ngamut=False)
    st2 = compare_survivors(cv, oracle, cols, grid, rule, fast, tag="nine, no n_gamut")
    compare_summaries(cv, oracle, cols, grid, rule, fast.summaries, bounds=b, ngamut=False)
    assert st2 == st
    assert fast.total == res.total and torch.equal(fast.pairs, res.pairs)
    assert torch.equal(fast.offsets, res.offsets)


# --------------------------------------------------------------------------
# Per-ray mode and list summaries

@pytest.mark.parametrize("nt", [180, 166])
def test_per_ray_search_matches_oracle(cv, oracle, nt):
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(81, 40)])
    grid = (0.5, 90, 2.0, nt)
    rule = (50, 0.5, 0x7F)
    res = cv.pair_search(_dev(cols), cv.Grid(*grid), cv.Rule(*rule), per_ray=True)
    g = cv.as_records(res.pairs, cv.PAIR_DTYPE)
    offs = res.offsets.cpu().numpy()
    # order: (colour, j) strictly increasing; offsets consistent
    key = g["colour"].astype(np.int64) * nt + g["j"]
    assert np.all(np.diff(key) > 0)
    assert offs[-1] == len(g) and np.all(np.diff(offs) >= 0)
    r, nb = parity.check_ray_records(oracle, cols, grid, rule, g, offs)
    fixed = r["rays_lo"] == r["rays_hi"]
    print(f"per-ray: {len(g)} records, {int((~fixed).sum())} of {fixed.size} rays movable, "
          f"{nb} band records")
    assert len(g) > 100
    # the summaries of the per-ray call are the full search's
    full = cv.pair_search(_dev(cols), cv.Grid(*grid), cv.Rule(*rule))
    assert torch.equal(res.summaries, full.summaries)


def test_per_ray_capacity_two_call(cv):
    cols = _dev(W.random_colours(82, 30))
    grid, rule = cv.Grid(0.5, 90, 2.0, 180), cv.Rule(50, 0.5, 0x7F)
    ref = cv.pair_search(cols, grid, rule, per_ray=True)
    small = torch.empty((7, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(cv.CvError) as e:
        cv.pair_search(cols, grid, rule, capacity=7, per_ray=True, out=small)
    assert e.value.code == cv.CV_ECAPACITY
    assert torch.equal(small, ref.pairs[:7])


def test_list_summaries_equal_search_summaries(cv):
    cols = _dev(np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(83, 50)]))
    grid, rule = cv.Grid(0.5, 100, 2.0, 180), cv.Rule(100, 0.25, 0x7F)
    full = cv.pair_search(cols, grid, rule)
    a = cv.as_records(cv.pair_reduce_csr(full.pairs, full.offsets), cv.SUMMARY_DTYPE)
    b = cv.as_records(full.summaries, cv.SUMMARY_DTYPE)
    for k in ("count", "best_i", "best_j", "best_plus", "best_minus", "best_p", "per_pattern"):
        assert np.array_equal(a[k], b[k]), k
    assert np.all(a["n_gamut"] == 0)
    # the best pair is also the best of the per-ray list
    pr = cv.pair_search(cols, grid, rule, per_ray=True)
    c = cv.as_records(cv.pair_reduce_csr(pr.pairs, pr.offsets), cv.SUMMARY_DTYPE)
    for k in ("best_i", "best_j", "best_plus", "best_minus", "best_p"):
        assert np.array_equal(c[k], b[k]), k


# --------------------------------------------------------------------------
# Large angle grids: more rays than the direct per-ray LDS tables hold, so the
# hot loops read the folded table (a quarter turn when N % 4 == 0, a half turn
# of sin and cos when N % 4 == 2).

@pytest.mark.parametrize("N,nt", [(8192, 8192), (6146, 6146), (8192, 5000)])
def test_large_angle_grids(cv, oracle, N, nt):
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY[:4], W.random_colours(91, 4)])
    grid = (0.75, 14, 360.0 / N, nt)
    rule = (50, 0.5, 0x7F)
    res = cv.pair_search(_dev(cols), cv.Grid(*grid), cv.Rule(*rule))
    compare_survivors(cv, oracle, cols, grid, rule, res, tag=f"N={N}")
    compare_summaries(cv, oracle, cols, grid, rule, res.summaries)
    summ, _ = cv.pair_reduce(_dev(cols), cv.Grid(*grid), cv.Rule(*rule))
    assert torch.equal(summ, res.summaries)
    counts = cv.pair_reduce_rules(_dev(cols), cv.Grid(*grid), [cv.Rule(*rule)])
    s = cv.as_records(summ, cv.SUMMARY_DTYPE)
    assert np.array_equal(counts[:, 0].cpu().numpy(), s["per_pattern"].astype(np.int64))
    # the per-colour resolve of the frames path on the same colours
    px = _dev(np.repeat(cols[None, :, :], 3, axis=0))
    fr = cv.frames_resolve(px, cv.Grid(*grid), cv.Rule(*rule))
    n = int(fr.ncolours.item())
    order = np.argsort((cols.astype(np.int64) << [16, 8, 0]).sum(1))
    fs = cv.as_records(fr.summaries[:n], cv.SUMMARY_DTYPE)
    for k in ("count", "n_gamut", "best_i", "best_j", "per_pattern"):
        assert np.array_equal(fs[k], s[k][order]), k


# --------------------------------------------------------------------------
# Gamut cells: skipping cells proven out of gamut changes no result.

@pytest.mark.parametrize("case", ["nine", "frames", "cube", "partial", "large", "clip"])
def test_gamut_cells_change_nothing(cv, case):
    grids = {
        "nine": ((0.05, 2000, 0.2, 1800), W.PAPER_COLOUR_ARRAY),
        "frames": (W.GRID_FRAMES.astuple(), W.random_colours(5, 3000)),
        "cube": (W.GRID_CUBE.astuple(), W.random_colours(6, 5000)),
        "partial": ((0.25, 160, 0.5, 500), W.random_colours(7, 40)),
        "large": ((0.75, 14, 360.0 / 8192, 8192), W.random_colours(8, 12)),
        "clip": ((0.25, 160, 1.0, 360), W.random_colours(9, 40)),
    }
    g, cols = grids[case]
    rule = cv.Rule(50, 0.5, 0x7F, cv.CV_RULE_CLIP if case == "clip" else 0)
    grid = cv.Grid(*g)
    x = _dev(cols)
    ctx = cv.Context(0)
    ctx.set_timing(True)
    ctx.set_gamut_cells(True)
    tab = g[1] <= 255 and g[3] <= 3600  # table rows: radius indices below 256, tables in LDS
    on = cv.pair_reduce(x, grid, rule, table=tab, ctx=ctx)
    s_on = cv.pair_search(x, grid, rule, ctx=ctx)
    skipped = ctx.skipped(reset=True)
    ctx.set_gamut_cells(False)
    off = cv.pair_reduce(x, grid, rule, table=tab, ctx=ctx)
    s_off = cv.pair_search(x, grid, rule, ctx=ctx)
    assert ctx.skipped() == 0
    assert torch.equal(on[0], off[0]) and (not tab or torch.equal(on[1], off[1]))
    assert s_on.total == s_off.total and torch.equal(s_on.summaries, s_off.summaries)
    assert torch.equal(s_on.pairs[:s_on.total], s_off.pairs[:s_off.total])
    per = g[1] * (g[3] // 2 if g[3] * g[2] == 360.0 else g[3])
    print(f"{case}: skipped {skipped} of {2 * len(cols) * per} evaluations")
    if case == "clip":  # no cells under the clip reading
        assert skipped == 0
    else:
        assert 0 < skipped < 2 * len(cols) * per


# --------------------------------------------------------------------------
# Captured search: replays equal the eager call; a changed argument captures
# again; per-ray mode runs eagerly.

def test_search_graph_replays_equal_eager(cv):
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(77, 23)])
    x = _dev(cols)
    grid = cv.Grid(0.05, 400, 0.5, 720)
    ctx = cv.Context(0)
    n = len(cols)
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    summ = torch.empty((n, 48), dtype=torch.uint8, device="cuda")
    for rule in (cv.Rule(50, 0.5), cv.Rule(40, 0.25, 0x15)):
        ref = cv.pair_search(x, grid, rule, ctx=ctx)
        out = torch.empty((ref.total + 7, 16), dtype=torch.uint8, device="cuda")
        for rep in range(3):
            g = cv.pair_search(x, grid, rule, out=out, ctx=ctx, graph=True, offsets=off, summ_out=summ)
            torch.cuda.synchronize()
            assert g.total == ref.total, rep
            assert torch.equal(g.pairs, ref.pairs) and torch.equal(off, ref.offsets), rep
            assert torch.equal(summ, ref.summaries), rep
            # eager work between replays
            cv.pair_search(x[:3], grid, rule, ctx=ctx)
    # too small an output: the two-call idiom through the graph path
    small = torch.empty((5, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(cv.CvError):
        cv.pair_search(x, grid, cv.Rule(50, 0.5), capacity=5, out=small, ctx=ctx, graph=True)
    pr = cv.pair_search(x, grid, cv.Rule(50, 0.5), per_ray=True, ctx=ctx, graph=True)
    pe = cv.pair_search(x, grid, cv.Rule(50, 0.5), per_ray=True, ctx=ctx)
    assert pr.total == pe.total and torch.equal(pr.pairs, pe.pairs)


def test_search_without_readback(cv):
    """total_host = NULL: calls only enqueue work.  Several calls back to
    back on one stream, eager and as graph replays, give the synchronous
    call's records, offsets (offsets[n] = total) and summaries; with too small
    an output the records that fit are the first ones and offsets[n] still
    holds the full total.  Per-ray mode as well."""
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(78, 23)])
    x = _dev(cols)
    grid = cv.Grid(0.05, 400, 0.5, 720)
    ctx = cv.Context(0)
    n = len(cols)
    rule = cv.Rule(50, 0.5)
    ref = cv.pair_search(x, grid, rule, ctx=ctx)
    out = torch.empty((ref.total + 7, 16), dtype=torch.uint8, device="cuda")
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    summ = torch.empty((n, 48), dtype=torch.uint8, device="cuda")
    for graph in (False, True):
        for _ in range(3):
            r = cv.pair_search(x, grid, rule, out=out, ctx=ctx, graph=graph, offsets=off, summ_out=summ,
                               sync=False)
            assert r.total is None
        torch.cuda.synchronize()
        assert int(off[n].item()) == ref.total
        assert torch.equal(out[:ref.total], ref.pairs) and torch.equal(off, ref.offsets)
        assert torch.equal(summ, ref.summaries)
    small = torch.zeros((100, 16), dtype=torch.uint8, device="cuda")
    cv.pair_search(x, grid, rule, out=small, ctx=ctx, offsets=off, summ_out=summ, sync=False)
    torch.cuda.synchronize()
    assert int(off[n].item()) == ref.total
    assert torch.equal(small, ref.pairs[:100])
    pe = cv.pair_search(x, grid, rule, per_ray=True, ctx=ctx)
    pout = torch.empty((pe.total, 16), dtype=torch.uint8, device="cuda")
    cv.pair_search(x, grid, rule, per_ray=True, out=pout, ctx=ctx, offsets=off, summ_out=summ, sync=False)
    torch.cuda.synchronize()
    assert int(off[n].item()) == pe.total and torch.equal(pout, pe.pairs)


def test_search_without_ngamut(cv):
    """CV_NO_NGAMUT: steps that can hold no survivor are not evaluated and
    the summaries' n_gamut is 0; records, offsets and every other summary
    field equal those of the full call (eager and graph; nine colours and a
    grid of few colours in direct mode)."""
    cases = [(np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(79, 23)]), cv.Grid(0.05, 400, 0.5, 720)),
             (W.random_colours(80, 2100), cv.Grid(0.5, 60, 1.0, 360))]
    for cols, grid in cases:
        x = _dev(cols)
        n = len(cols)
        for rule in (cv.Rule(50, 0.5), cv.Rule(40, 0.25, 0x15)):
            ref = cv.pair_search(x, grid, rule)
            for graph in (False, True):
                r = cv.pair_search(x, grid, rule, graph=graph, ngamut=False)
                assert r.total == ref.total
                assert torch.equal(r.pairs, ref.pairs) and torch.equal(r.offsets, ref.offsets)
                s_ref = cv.as_records(ref.summaries, cv.SUMMARY_DTYPE)
                s_new = cv.as_records(r.summaries, cv.SUMMARY_DTYPE)
                assert np.all(s_new["n_gamut"] == 0)
                for f in s_ref.dtype.names:
                    if f != "n_gamut":
                        assert np.array_equal(s_new[f], s_ref[f]), (n, f)
