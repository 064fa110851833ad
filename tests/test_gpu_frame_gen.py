"""The device frame generator (cv_frames_generate) against its CPU twin in the
oracle, byte for byte: the same Philox4x64-10 words and the same integer
recipe give the same frames."""
from __future__ import annotations

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

SEEDS = [0, 1, (1 << 64) - 1]


@pytest.fixture(scope="module")
def cv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_22901_amd as cv
    return cv


@pytest.mark.parametrize("h,w,sites,noise", [(1, 1, 1, 0), (7, 13, 3, 4), (135, 240, 64, 4),
                                              (64, 96, 256, 255), (270, 480, 64, 0)])
def test_frames_equal_the_oracle(cv, h, w, sites, noise):
    got = cv.frames_generate(SEEDS, h, w, sites, noise).cpu().numpy()
    assert got.shape == (len(SEEDS), h, w, 3)
    for k, s in enumerate(SEEDS):
        np.testing.assert_array_equal(got[k], oracle.gen_frame(s, h, w, sites, noise), err_msg=f"seed {s}")


def test_4k_frame_equals_the_oracle(cv):
    """One frame of the benchmark's size and recipe (3840 x 2160, 64 sites,
    noise 4)."""
    got = cv.frames_generate([100], 2160, 3840).cpu().numpy()[0]
    np.testing.assert_array_equal(got, oracle.gen_frame(100, 2160, 3840))


def test_out_buffer_and_validation(cv):
    import torch
    out = torch.zeros((2, 16, 32, 3), dtype=torch.uint8, device="cuda")
    res = cv.frames_generate([4, 5], 16, 32, out=out)
    assert res.data_ptr() == out.data_ptr()
    np.testing.assert_array_equal(out[1].cpu().numpy(), oracle.gen_frame(5, 16, 32))
    with pytest.raises(ValueError):
        cv.frames_generate([4, 5], 16, 33, out=out)
    with pytest.raises(cv.CvError):
        cv.frames_generate([4], 16, 32, sites=0)
