"""The synthetic frame generator's CPU twin (oracle/frame_oracle.c): its
Philox4x64-10 pinned to numpy's Philox bit generator, and properties of the
frames it builds.  The device generator is compared with it byte for byte in
test_gpu_frame_gen.py."""
from __future__ import annotations

import numpy as np
import pytest

import oracle

MASK = (1 << 64) - 1
KEYS = [(0, 0), (123, 456), (MASK, (1 << 63) + 5), (0xDEADBEEF, 1)]
CTRS = [(0, 0, 0, 0), (7, 8, 9, 10), (MASK, 3, MASK, 0), (1, 1 << 40, 5, 0), (MASK - 1, 0, 0, 7)]


def _plus_one(ctr):
    """The 256-bit counter (word 0 least significant) plus one."""
    v = sum(int(w) << (64 * k) for k, w in enumerate(ctr)) + 1
    return [(v >> (64 * k)) & MASK for k in range(4)]


@pytest.mark.parametrize("key", KEYS)
@pytest.mark.parametrize("ctr", CTRS)
def test_philox_matches_numpy(key, ctr):
    """numpy's Philox is the same 4x64-10 function; it advances its counter
    before each block, so its first block is the function of counter + 1."""
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    want = [int(v) for v in bg.random_raw(8)]
    c1 = _plus_one(ctr)
    assert [int(v) for v in oracle.philox4x64(c1, key)] == want[:4]
    assert [int(v) for v in oracle.philox4x64(_plus_one(c1), key)] == want[4:]


def test_frames_are_deterministic_and_seeded():
    a = oracle.gen_frame(5, 48, 80)
    assert np.array_equal(a, oracle.gen_frame(5, 48, 80))
    assert not np.array_equal(a, oracle.gen_frame(6, 48, 80))
    assert a.dtype == np.uint8 and a.shape == (48, 80, 3)


@pytest.mark.parametrize("seed", [0, 11, 12345])
def test_one_site_without_noise_is_a_monotone_gradient(seed):
    """One region and no noise leave per channel an affine ramp (truncated and
    clamped), monotone along every row and every column."""
    f = oracle.gen_frame(seed, 80, 96, sites=1, noise=0).astype(np.int32)
    for c in range(3):
        dx = np.diff(f[:, :, c], axis=1)
        dy = np.diff(f[:, :, c], axis=0)
        assert (dx >= 0).all() or (dx <= 0).all(), c
        assert (dy >= 0).all() or (dy <= 0).all(), c
        # a slope of at most 64 codes over a side of at least 64 pixels
        assert np.abs(dx).max() <= 1 and np.abs(dy).max() <= 1


def test_noise_amplitude():
    """The noise is a sum of four uniform bytes, centred and scaled by
    noise / 128: standard deviation sqrt(4 (256^2 - 1) / 12) * 4 / 128 = 4.6
    codes for noise 4 (less where the clamp cuts it)."""
    a = oracle.gen_frame(3, 256, 256, sites=1, noise=4).astype(np.int32)
    b = oracle.gen_frame(3, 256, 256, sites=1, noise=0).astype(np.int32)
    inside = (b > 20) & (b < 235)
    d = (a - b)[inside]
    assert abs(d.mean()) < 0.1
    assert 4.2 < d.std() < 5.0
    assert np.abs(d).max() <= 510 * 4 // 128


def test_regions_are_the_nearest_sites():
    """Without noise and with gradients that cancel out of differences, two
    horizontally adjacent pixels differ by more than the ramp's one code only
    where the nearest site changes; many such edges exist with 64 sites."""
    f = oracle.gen_frame(8, 120, 200, sites=64, noise=0).astype(np.int32)
    jumps = (np.abs(np.diff(f, axis=1)) > 1).any(axis=2)
    assert 0 < jumps.mean() < 0.2


def test_bad_arguments():
    with pytest.raises(ValueError):
        oracle.gen_frame(1, 0, 10)
    with pytest.raises(ValueError):
        oracle.gen_frame(1, 10, 10, sites=257)
