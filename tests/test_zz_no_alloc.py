"""The reduce entry point that allocates nothing (cv_pair_reduce_noalloc),
called through the C-ABI: byte-identical summaries and table rows to
cv_pair_reduce on two calls in a row, the second with fewer colours (and in
the other tiling mode), and a refusal, before any work, of a call whose
workspace exceeds the fixed scratch array."""
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


def _outputs(n):
    return (torch.full((n, 48), 0xA5, dtype=torch.uint8, device="cuda"),
            torch.full((n, 40), 0x5A, dtype=torch.uint8, device="cuda"))


def test_noalloc_reduce_equals_reduce(cv):
    grid = cv.Grid(*W.GRID_CUBE.astuple())
    rule = cv.Rule(*W.DEFAULT_RULE)
    cols = torch.from_numpy(np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(101, 4991)])).cuda()
    # 5000 colours: one tile per colour; then 700: tiles merged by atomics
    for n in (5000, 700):
        x = cols[:n].contiguous()
        ref_s, ref_t = cv.pair_reduce(x, grid, rule, table=True)
        s, t = _outputs(n)
        cv.pair_reduce_noalloc(x, grid, rule, s, t)
        torch.cuda.synchronize()
        assert torch.equal(s, ref_s), n
        assert torch.equal(t, ref_t), n
        print(f"noalloc reduce, {n} colours: equal")
    # summaries only on another grid (a partial turn), twice in a row
    g2 = cv.Grid(0.5, 60, 1.0, 300)
    for n in (2100, 37):
        x = cols[:n].contiguous()
        ref_s, _ = cv.pair_reduce(x, g2, rule)
        s, _ = _outputs(n)
        cv.pair_reduce_noalloc(x, g2, rule, s, None)
        torch.cuda.synchronize()
        assert torch.equal(s, ref_s), n


def test_noalloc_reduce_refuses_oversize(cv):
    grid = cv.Grid(*W.GRID_CUBE.astuple())
    rule = cv.Rule(*W.DEFAULT_RULE)
    n = 200_000  # 64 bytes each: beyond the 8 MiB array
    x = torch.zeros((n, 3), dtype=torch.uint8, device="cuda")
    s, _ = _outputs(n)
    with pytest.raises(cv.CvError) as e:
        cv.pair_reduce_noalloc(x, grid, rule, s, None)
    assert e.value.code == cv.CV_ECAPACITY
    assert "scratch" in str(e.value)
    assert int((s != 0xA5).sum()) == 0  # nothing was written
