"""Training checkpoint and resume on the GPU: a run stopped after k steps,
saved, loaded into a fresh network and continued ends with the parameters and
Adam moments of the uninterrupted run, bit for bit (mid-epoch and at an epoch
boundary); a checkpoint of another shape or a corrupted one is refused; the
cube-table cache is reused only for its own grid and rule."""
from __future__ import annotations

import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cv():
    import paper_2507_22901_amd as cv
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cv.lib()
    return cv


@pytest.fixture(scope="module")
def table():
    # a synthetic whole-cube table (the training loop gathers rows by colour id)
    g = torch.Generator(device="cuda").manual_seed(5)
    t = torch.randint(0, 201, (1 << 24, 40), dtype=torch.uint8, device="cuda", generator=g)
    t[:, :4] = 0
    t[:, 0] = (t[:, 4:].amax(1) > 0).to(torch.uint8)
    return t


def _net(cv):
    m = cv.surrogate_network(0)
    return m


@pytest.mark.parametrize("stop", [70, 49])
def test_resume_equals_uninterrupted(cv, table, tmp_path, stop):
    from paper_2507_22901_amd import surrogate as S
    ids = torch.randperm(1 << 24, device="cuda")[:50_000].to(torch.int32)
    kw = dict(epochs=2.5, batch=1024, log_every=0, seed=3)
    ref = _net(cv)
    S.train(ref, table, ids, 0.25, **kw)
    a = _net(cv)
    ck = str(tmp_path / "run.ckpt")
    S.train(a, table, ids, 0.25, stop=stop, checkpoint=ck, **kw)
    dims, step, key = cv.checkpoint_info(ck)
    assert dims == cv.SURROGATE_DIMS and step == stop and key == 3
    b = _net(cv)
    b.set_params(np.zeros(b.nparams, np.float32))
    st, k = b.load_checkpoint(ck)
    assert (st, k) == (stop, 3)
    S.train(b, table, ids, 0.25, start=st, **kw)
    torch.cuda.synchronize()
    assert torch.equal(b.params(), ref.params())
    # the moments as well: one more identical step on both keeps them equal
    fin_ref, fin_b = str(tmp_path / "ref.ckpt"), str(tmp_path / "b.ckpt")
    ref.save_checkpoint(fin_ref, 0)
    b.save_checkpoint(fin_b, 0)
    with open(fin_ref, "rb") as f1, open(fin_b, "rb") as f2:
        assert f1.read() == f2.read()


def test_foreign_and_corrupt_checkpoints_refused(cv, tmp_path):
    m = _net(cv)
    p = str(tmp_path / "m.ckpt")
    m.save_checkpoint(p, 5, 9)
    other = cv.MLP((3, 32, 37))
    with pytest.raises(cv.CvError) as e:
        other.load_checkpoint(p)
    assert e.value.code == cv.CV_EINVAL
    data = bytearray(open(p, "rb").read())
    data[len(data) // 3] ^= 1
    open(p, "wb").write(bytes(data))
    with pytest.raises(cv.CvError) as e:
        m.load_checkpoint(p)
    assert e.value.code == cv.CV_EINVAL


def test_table_cache(cv, tmp_path):
    from paper_2507_22901_amd import surrogate as S
    grid, rule = cv.Grid(0.25, 200, 2.0, 180), cv.Rule(50, 0.5)
    t = torch.randint(0, 255, (1 << 24, 40), dtype=torch.uint8, device="cuda")
    p = str(tmp_path / "cube.tab")
    S.save_table(p, t, grid, rule)
    back = S.load_table(p, grid, rule)
    assert back is not None and torch.equal(back, t)
    assert S.load_table(p, cv.Grid(0.25, 200, 2.0, 179), rule) is None
    assert S.load_table(p, grid, cv.Rule(100, 0.5)) is None
    with open(p, "r+b") as f:
        f.seek(os.path.getsize(p) - 5)
        f.write(b"\x01")
    assert S.load_table(p, grid, rule) is None
    assert S.load_table(str(tmp_path / "none.tab"), grid, rule) is None
