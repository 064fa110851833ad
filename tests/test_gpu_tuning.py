"""The autotuner's tiling choices for the chunked reduce (the count pass of
cv_pair_search and cv_pair_reduce with few colours) and its on-disk cache:
every tiling gives the same bytes, a tuned context gives what an untuned one
does, and a tuning file written on this GPU is read back by a new context."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

TARGETS = (1024, 2048, 4096, 8192, 16384)


@pytest.fixture(scope="module")
def cv():
    import paper_2507_22901_amd as cv
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cv.lib()
    return cv


def _colours():
    return torch.from_numpy(np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(40, 71)])).cuda()


def _search(cv, ctx, x, grid, rule):
    r = cv.pair_search(x, grid, rule, ctx=ctx)
    torch.cuda.synchronize()
    return r.pairs.cpu(), r.offsets.cpu(), r.summaries.cpu()


@pytest.mark.parametrize("grid", [(0.5, 200, 1.0, 360), (0.25, 150, 2.0, 131)])
def test_every_tiling_gives_the_same_bytes(cv, grid):
    x = _colours()
    g, r = cv.Grid(*grid), cv.Rule(50, 0.5)
    ctx = cv.Context(0)
    base = _search(cv, ctx, x, g, r)
    sbase, _ = cv.pair_reduce(x, g, r, ctx=ctx)
    for t in TARGETS + (64, 100000):
        ctx.set_tile_target(t)
        assert ctx.tile_target(x.shape[0], g) == (t, False)
        got = _search(cv, ctx, x, g, r)
        for a, b in zip(got, base):
            assert torch.equal(a, b), t
        s, _ = cv.pair_reduce(x, g, r, ctx=ctx)
        torch.cuda.synchronize()
        assert torch.equal(s.cpu(), sbase.cpu()), t


def test_autotune_and_tune_file(cv, tmp_path):
    x = _colours()
    n = x.shape[0]
    g, r = cv.Grid(0.5, 200, 1.0, 360), cv.Rule(50, 0.5)
    plain = cv.Context(0)
    want = _search(cv, plain, x, g, r)
    want_s, _ = cv.pair_reduce(x, g, r, ctx=plain)
    path = str(tmp_path / "tune.txt")
    ctx = cv.Context(0)
    ctx.set_tune_file(path)
    head = open(path).read().splitlines()
    assert len(head) == 1 and head[0].startswith("cvib-tune 1 ")
    ctx.set_autotune(True)
    assert ctx.tile_target(n, g) == (4096, False)
    got = _search(cv, ctx, x, g, r)
    for a, b in zip(got, want):
        assert torch.equal(a, b)
    t_search, tuned = ctx.tile_target(n, g)
    assert tuned and t_search in TARGETS
    s, _ = cv.pair_reduce(x, g, r, ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(s.cpu(), want_s.cpu())
    t_reduce, tuned = ctx.tile_target(n, g, search=False)
    assert tuned and t_reduce in TARGETS
    lines = open(path).read().splitlines()
    assert lines[0] == head[0] and sorted(ln.split()[0] for ln in lines[1:]) == ["tiles", "tiles"]
    # a new context reads the choices back and does not tune again
    ctx2 = cv.Context(0)
    ctx2.set_tune_file(path)
    assert ctx2.tile_target(n, g) == (t_search, True)
    assert ctx2.tile_target(n, g, search=False) == (t_reduce, True)
    got2 = _search(cv, ctx2, x, g, r)
    for a, b in zip(got2, want):
        assert torch.equal(a, b)
    # a forced tiling overrides the tuned one
    ctx2.set_tile_target(2048)
    assert ctx2.tile_target(n, g) == (2048, False)
    ctx2.set_tile_target(0)
    assert ctx2.tile_target(n, g) == (t_search, True)


def test_tune_file_of_another_gpu_or_not_a_tune_file(cv, tmp_path):
    g = cv.Grid(0.5, 200, 1.0, 360)
    other = tmp_path / "other.txt"
    other.write_text("cvib-tune 1 gfx000 1\ntiles 0123456789abcdef 2048\n")
    ctx = cv.Context(0)
    ctx.set_tune_file(str(other))
    assert ctx.tile_target(49, g) == (4096, False)
    assert not open(other).read().startswith("cvib-tune 1 gfx000")  # rewritten for this GPU
    bad = tmp_path / "bad.txt"
    bad.write_text("hello\n")
    with pytest.raises(cv.CvError):
        cv.Context(0).set_tune_file(str(bad))
    mine = open(other).read().splitlines()[0]
    bad.write_text(mine + "\ntiles 12 3000\n")  # not one of the tilings
    with pytest.raises(cv.CvError):
        cv.Context(0).set_tune_file(str(bad))
    with pytest.raises(cv.CvError):
        cv.Context(0).set_tune_file(str(tmp_path / "no_such_dir" / "t.txt"))
    ctx.set_tune_file(None)
