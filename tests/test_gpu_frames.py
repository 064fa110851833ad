"""Batched frames on the GPU: de-duplication, per-colour resolve (summaries,
best pair per information pattern, per-ray maxima), rendering of the two
alternating frames, and hipGraph replays -- against the FP64 oracle and
plain host definitions."""
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


def _frames():
    # two small synthetic frames (gradients + Voronoi cells + noise) and a few
    # Table 1 colours painted in, so that colours repeat across frames
    f = W.frames([3, 4], height=72, width=128)
    f[0, :8, :9] = W.PAPER_COLOUR_ARRAY[None, :, :]
    f[1, -4:, :9] = W.PAPER_COLOUR_ARRAY[None, :, :]
    return f


@pytest.mark.parametrize("nt", [180, 172])
def test_frames_resolve_matches_oracle(cv, oracle, nt):
    f = _frames()
    npix = f.shape[0] * f.shape[1] * f.shape[2]
    rng = np.random.default_rng(0)
    info = rng.integers(0, 8, npix).astype(np.uint8)
    grid = (0.5, 70, 2.0, nt)
    rule = (50, 0.5, 0x7F)
    px = torch.from_numpy(f).cuda()
    res = cv.frames_resolve(px, cv.Grid(*grid), cv.Rule(*rule), info=torch.from_numpy(info).cuda(),
                            rays=True)
    torch.cuda.synchronize()
    ids = oracle.distinct_colours(f)
    n = int(res.ncolours.item())
    assert n == len(ids)
    cols = res.colours[:n].cpu().numpy()
    assert np.array_equal(cols, W.cube_colours(ids))
    pix = f.reshape(-1, 3)
    idx = res.pixel_index.cpu().numpy().astype(np.int64)
    assert np.array_equal(cols[idx], pix)
    # per-colour results on a sample of colours (the oracle is slow)
    sample = np.unique(np.concatenate([rng.choice(n, 60, replace=False),
                                       idx[:9]]))  # includes painted paper colours
    sc = cols[sample]
    s_g = cv.as_records(res.summaries, cv.SUMMARY_DTYPE)[sample]
    r = oracle.reduce_bounds(sc, grid, rule, rays=True)
    parity.check_summaries(oracle, sc, grid, rule, s_g, bounds=r["bounds"])
    pb = cv.as_records(res.pbest.reshape(-1, 12), cv.PATTERN_PAIR_DTYPE).reshape(-1, 7)[sample]
    parity.check_pattern_bests(oracle, sc, grid, rule, pb, bounds=r["bounds"])
    rays_g = res.rays.cpu().numpy().view(np.uint16)[sample]
    parity.check_rays(oracle, sc, grid, rule, rays_g, r)
    # rendering, against a host composition of the GPU's own per-colour pairs
    pball = cv.as_records(res.pbest.reshape(-1, 12), cv.PATTERN_PAIR_DTYPE).reshape(-1, 7)
    sall = cv.as_records(res.summaries, cv.SUMMARY_DTYPE)
    A = pix.copy()
    B = pix.copy()
    got = 0
    for p_ in range(npix):
        k, q = idx[p_], int(info[p_])
        if q:
            r = pball[k, q - 1]
            if r["flags"]:
                A[p_], B[p_] = r["plus"], r["minus"]
                got += 1
        elif sall["best_i"][k] != 0xFFFF:
            A[p_], B[p_] = sall["best_plus"][k], sall["best_minus"][k]
            got += 1
    assert np.array_equal(res.frame_a.cpu().numpy(), A)
    assert np.array_equal(res.frame_b.cpu().numpy(), B)
    assert int(res.resolved.item()) == got


def test_frames_graph_replay_matches_eager(cv):
    """The captured graph, replayed several times with eager work and
    synchronisations in between, reproduces the eager result each time."""
    f = torch.from_numpy(_frames()).cuda()
    grid = cv.Grid(0.5, 60, 2.0, 180)
    rule = cv.Rule(50, 0.5, 0x7F)
    eager = cv.frames_resolve(f, grid, rule, rays=True)
    torch.cuda.synchronize()
    ref = {k: getattr(eager, k).clone() for k in ("colours", "ncolours", "pixel_index", "summaries",
                                                    "pbest", "rays", "frame_a", "frame_b", "resolved")}
    out = cv.frames_resolve(f, grid, rule, rays=True, graph=True)
    for rep in range(4):
        # eager work in between replays
        other = cv.frames_resolve(f[:, :32], cv.Grid(0.5, 40, 2.0, 180), rule)
        torch.cuda.synchronize()
        for k in ref:
            getattr(out, k).zero_()
        torch.cuda.synchronize()
        cv.frames_resolve(f, grid, rule, rays=True, graph=True, out=out)
        torch.cuda.synchronize()
        n = int(ref["ncolours"].item())
        for k, v in ref.items():
            g = getattr(out, k)
            if k in ("colours", "summaries", "pbest", "rays"):
                assert torch.equal(g[:n], v[:n]), (rep, k)
            else:
                assert torch.equal(g, v), (rep, k)
        assert int(other.ncolours.item()) > 0


@pytest.mark.parametrize("nt", [180, 172])
def test_resolve_variants_and_autotune_agree(cv, nt):
    """Every per-colour resolve kernel (one colour per 4-wave block, one per
    wave with 4 or 8 waves per block) and the tuned choice give the same
    bytes."""
    f = torch.from_numpy(_frames()).cuda()
    grid = cv.Grid(0.5, 60, 2.0, nt)
    rule = cv.Rule(50, 0.5, 0x7F)
    info = torch.from_numpy(np.random.default_rng(2).integers(0, 8, f.numel() // 3).astype(np.uint8)).cuda()
    ctx = cv.Context(0)
    outs = []
    for v in (0, 1, 2):
        ctx.set_resolve_variant(v)
        assert ctx.resolve_variant(grid, rays=True) == (v, False)
        outs.append(cv.frames_resolve(f, grid, rule, info=info, rays=True, ctx=ctx))
    ctx.set_resolve_variant(-1)
    ctx.set_autotune(True)
    outs.append(cv.frames_resolve(f, grid, rule, info=info, rays=True, ctx=ctx))
    v, tuned = ctx.resolve_variant(grid, rays=True)
    assert tuned and v in (0, 1, 2)
    outs.append(cv.frames_resolve(f, grid, rule, info=info, rays=True, graph=True, ctx=ctx))
    torch.cuda.synchronize()
    n = int(outs[0].ncolours.item())
    for o in outs[1:]:
        for k in ("summaries", "pbest", "rays"):
            assert torch.equal(getattr(o, k)[:n], getattr(outs[0], k)[:n]), k
        for k in ("frame_a", "frame_b", "resolved", "pixel_index"):
            assert torch.equal(getattr(o, k), getattr(outs[0], k)), k
    print("tuned variant", v)


@pytest.mark.parametrize("nt", [360, 300])
def test_gamut_cells_change_no_frame_output(cv, nt):
    """Grids of at least 128 evaluated rays per row skip wave steps proven out
    of gamut in the per-colour resolve; every kernel variant, eager and
    captured, gives the bytes of the resolve without them."""
    f = torch.from_numpy(_frames()).cuda()
    grid = cv.Grid(0.25, 200, 1.0, nt)
    rule = cv.Rule(50, 0.5, 0x7F)
    info = torch.from_numpy(np.random.default_rng(3).integers(0, 8, f.numel() // 3).astype(np.uint8)).cuda()
    ctx = cv.Context(0)
    ctx.set_gamut_cells(False)
    ref = cv.frames_resolve(f, grid, rule, info=info, rays=True, ctx=ctx)
    outs = []
    ctx.set_gamut_cells(True)
    for v in (0, 1, 2):
        ctx.set_resolve_variant(v)
        outs.append(cv.frames_resolve(f, grid, rule, info=info, rays=True, ctx=ctx))
    outs.append(cv.frames_resolve(f, grid, rule, info=info, rays=True, graph=True, ctx=ctx))
    ctx.set_gamut_cells(False)  # a captured call of the other setting is not replayed
    outs.append(cv.frames_resolve(f, grid, rule, info=info, rays=True, graph=True, ctx=ctx))
    torch.cuda.synchronize()
    n = int(ref.ncolours.item())
    for o in outs:
        for k in ("summaries", "pbest", "rays"):
            assert torch.equal(getattr(o, k)[:n], getattr(ref, k)[:n]), k
        for k in ("frame_a", "frame_b", "resolved", "pixel_index"):
            assert torch.equal(getattr(o, k), getattr(ref, k)), k


@pytest.mark.parametrize("dth,nt", [(1.0, 360), (0.5, 720)])
def test_frames_without_ngamut(cv, dth, nt):
    """CV_NO_NGAMUT: steps without a high channel are skipped; every output
    but the summaries' n_gamut (0) equals the full resolve, for every kernel
    variant, eager and captured, and without summaries at all."""
    f = torch.from_numpy(_frames()).cuda()
    grid = cv.Grid(0.25, 200, dth, nt)
    rule = cv.Rule(50, 0.5, 0x7F)
    # patterns 1..7 only: pixels of map value 0 take the summaries' best pair,
    # which the call without summaries does not have
    info = torch.from_numpy(np.random.default_rng(4).integers(1, 8, f.numel() // 3).astype(np.uint8)).cuda()
    ctx = cv.Context(0)
    ref = cv.frames_resolve(f, grid, rule, info=info, rays=True, ctx=ctx)
    outs = []
    for v in (0, 1, 2):
        ctx.set_resolve_variant(v)
        outs.append(cv.frames_resolve(f, grid, rule, info=info, rays=True, ctx=ctx, ngamut=False))
    outs.append(cv.frames_resolve(f, grid, rule, info=info, rays=True, graph=True, ctx=ctx, ngamut=False))
    nosum = cv.frames_resolve(f, grid, rule, info=info, rays=True, summaries=False, ctx=ctx)
    torch.cuda.synchronize()
    n = int(ref.ncolours.item())
    s_ref = cv.as_records(ref.summaries[:n], cv.SUMMARY_DTYPE)
    for o in outs + [nosum]:
        for k in ("pbest", "rays"):
            assert torch.equal(getattr(o, k)[:n], getattr(ref, k)[:n]), k
        for k in ("frame_a", "frame_b", "resolved", "pixel_index"):
            assert torch.equal(getattr(o, k), getattr(ref, k)), k
    for o in outs:
        s = cv.as_records(o.summaries[:n], cv.SUMMARY_DTYPE)
        assert np.all(s["n_gamut"] == 0)
        for fld in s_ref.dtype.names:
            if fld != "n_gamut":
                assert np.array_equal(s[fld], s_ref[fld]), fld


def test_reused_buffers_are_checked(cv):
    """A result reused for a larger input, a wider grid or with a wrong dtype
    is refused on the host before any kernel runs."""
    small = torch.from_numpy(W.frames([6], height=16, width=16)).cuda()
    big = torch.from_numpy(W.frames([6], height=32, width=32)).cuda()
    grid, rule = cv.Grid(0.5, 20, 2.0, 180), cv.Rule(50, 0.5)
    res = cv.frames_resolve(small, grid, rule, rays=True)
    with pytest.raises(ValueError):
        cv.frames_resolve(big, grid, rule, rays=True, out=res)
    with pytest.raises(ValueError):
        cv.frames_resolve(small, cv.Grid(0.5, 20, 1.0, 360), rule, rays=True, out=res)
    again = cv.frames_resolve(small, grid, rule, rays=True, out=res)
    assert again is res
    cols = torch.from_numpy(W.random_colours(3, 5)).cuda()
    with pytest.raises(ValueError):
        cv.pair_search(cols, grid, rule, out=torch.empty((10, 12), dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError):
        cv.pair_search(cols, grid, rule, offsets=torch.empty(5, dtype=torch.int64, device="cuda"))
    with pytest.raises(ValueError):
        cv.pair_search(cols, grid, rule, summ_out=torch.empty((5, 48), dtype=torch.int8, device="cuda"))


def test_unaligned_and_ragged_pixel_arrays(cv):
    """The per-pixel kernels take four pixels (12 bytes) at a time as words
    from 4-byte aligned arrays, byte by byte from others, and the last
    npix % 4 pixels one by one: pixel and information arrays that start off a
    word, with pixel counts that are not multiples of 4, give the outputs of
    aligned copies (which the tests above hold to the oracle and to a host
    composition of the frames)."""
    f = _frames()
    base = torch.from_numpy(f.reshape(-1, 3)).cuda()
    grid, rule = cv.Grid(0.5, 70, 2.0, 180), cv.Rule(50, 0.5, 0x7F)
    g = torch.Generator(device="cuda").manual_seed(5)
    for start, npix in ((1, 1021), (0, 1023), (3, 4094), (2, 4097), (5, 3)):
        view = base[start:start + npix]          # starts 3 * start bytes in
        info_all = torch.randint(0, 8, (npix + 1,), dtype=torch.uint8, device="cuda", generator=g)
        a = cv.frames_resolve(view, grid, rule, info=info_all[1:])
        b = cv.frames_resolve(view.clone(), grid, rule, info=info_all[1:].clone())
        torch.cuda.synchronize()
        n = int(b.ncolours.item())
        assert int(a.ncolours.item()) == n, (start, npix)
        for x, y in ((a.colours[:n], b.colours[:n]), (a.pixel_index, b.pixel_index),
                     (a.frame_a, b.frame_a), (a.frame_b, b.frame_b), (a.resolved, b.resolved)):
            assert torch.equal(x, y), (start, npix)
        # the index points at each pixel's own colour, ragged tail included
        assert torch.equal(a.colours[a.pixel_index.long()], view)
