"""Seeded synthetic workloads shared by the tests, the benchmark and the smoke check.

Holds input data and input generators only (no part of the search's
arithmetic): the paper's colours, information patterns and thresholds
(Table 1), the search grids of the benchmark configurations, seeded colour
samples, the synthetic 4K frame generator and per-pixel information maps.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Table 1: colours (RGB), in the column order of Table 2.
PAPER_COLOURS = {
    "Black": (100, 100, 100),
    "Gray": (170, 170, 170),
    "White": (240, 240, 240),
    "Red": (240, 100, 100),
    "Green": (100, 240, 100),
    "Blue": (100, 100, 240),
    "Yellow": (240, 240, 100),
    "Cyan": (100, 240, 240),
    "Magenta": (240, 100, 240),
}
PAPER_COLOUR_ARRAY = np.array(list(PAPER_COLOURS.values()), dtype=np.uint8)

# Table 1: information patterns (bits for R, G, B) and thresholds.
PATTERNS = ("100", "010", "001", "110", "101", "011", "111")
V_TH = (50, 100, 150, 200)
R_NOVIB = (0.5, 0.25, 0.125)
TABLE1_RULES = tuple((v, r) for v in V_TH for r in R_NOVIB)
DEFAULT_RULE = (50, 0.5, 0x7F)


@dataclass(frozen=True)
class GridSpec:
    dr: float
    nr: int
    dtheta_deg: float
    ntheta: int

    def astuple(self):
        return (self.dr, self.nr, self.dtheta_deg, self.ntheta)

    @property
    def per_colour(self) -> int:
        return self.nr * self.ntheta


# Search grids: r_i = (i+1) dr, theta_j = j dtheta.
GRID_SINGLE = GridSpec(0.1, 400, 1.0, 360)      # one colour, 144,000 pairs
GRID_NINE = GridSpec(0.01, 10000, 0.1, 3600)    # nine colours, 36 M pairs each
GRID_FRAMES = GridSpec(0.1, 500, 1.0, 360)      # distinct colours of 4K frames
GRID_CUBE = GridSpec(0.25, 200, 2.0, 180)       # all 2^24 colours


def random_colours(seed: int, n: int) -> np.ndarray:
    """n uniformly random sRGB8 colours, [n, 3] uint8."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    return rng.integers(0, 256, size=(n, 3), dtype=np.uint8)


def cube_colours(ids: np.ndarray) -> np.ndarray:
    """Colour ids R<<16 | G<<8 | B -> [n, 3] uint8."""
    ids = np.asarray(ids, dtype=np.uint32)
    return np.stack([(ids >> 16) & 255, (ids >> 8) & 255, ids & 255], axis=1).astype(np.uint8)


def frame(seed: int, height: int = 2160, width: int = 3840, sites: int = 64,
          noise_sigma: float = 4.0) -> np.ndarray:
    """Synthetic sRGB8 frame [height, width, 3]: smooth linear gradients +
    piecewise-constant Voronoi regions + Gaussian noise, clipped.

    I = clip(round(g0 + gx x/W + gy y/H + v[cell(x, y)] + n)) with
    g0 ~ U(64,192)^3, gx, gy ~ U(-64,64)^3, `sites` Voronoi sites uniform over
    the frame, per-cell offsets v ~ U(-48,48)^3 and n ~ N(0, sigma^2) per
    channel, drawn from a Philox stream keyed by `seed`."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    g0 = rng.uniform(64, 192, 3)
    gx = rng.uniform(-64, 64, 3)
    gy = rng.uniform(-64, 64, 3)
    sx = rng.uniform(0, width, sites).astype(np.float32)
    sy = rng.uniform(0, height, sites).astype(np.float32)
    v = rng.uniform(-48, 48, (sites, 3)).astype(np.float32)
    out = np.empty((height, width, 3), dtype=np.uint8)
    xs = np.arange(width, dtype=np.float32)
    base_x = (gx[None, :] * (xs[:, None] / width)).astype(np.float32)       # [W, 3]
    dx2 = (xs[:, None] - sx[None, :]) ** 2                                   # [W, S]
    rows = 32
    for y0 in range(0, height, rows):
        y1 = min(height, y0 + rows)
        ys = np.arange(y0, y1, dtype=np.float32)
        d2 = dx2[None, :, :] + ((ys[:, None] - sy[None, :]) ** 2)[:, None, :]  # [R, W, S]
        cell = np.argmin(d2, axis=2)                                            # [R, W]
        val = (g0[None, None, :] + base_x[None, :, :]
               + (gy[None, None, :] * (ys[:, None, None] / height)) + v[cell])
        val = val + rng.normal(0.0, noise_sigma, val.shape)
        out[y0:y1] = np.clip(np.rint(val), 0, 255).astype(np.uint8)
    return out


def frames(seeds, height: int = 2160, width: int = 3840, workers: int = 8) -> np.ndarray:
    """Stack of frames [len(seeds), height, width, 3] (each frame from its own
    seed, generated on a few host threads)."""
    from concurrent.futures import ThreadPoolExecutor
    seeds = list(seeds)
    with ThreadPoolExecutor(max_workers=max(1, min(workers, len(seeds)))) as ex:
        return np.stack(list(ex.map(lambda s: frame(s, height, width), seeds)))


def info_map(seed: int, height: int = 2160, width: int = 3840, block: int = 16) -> np.ndarray:
    """Per-pixel 3-bit information map [height, width] uint8: square blocks of
    `block` pixels, each carrying a pattern drawn uniformly from 1..7 (the
    seven patterns of Table 1), from a Philox stream keyed by `seed`."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    bh, bw = -(-height // block), -(-width // block)
    cells = rng.integers(1, 8, size=(bh, bw), dtype=np.uint8)
    return np.repeat(np.repeat(cells, block, axis=0), block, axis=1)[:height, :width].copy()


def cube_split(seed: int = 0, test_fraction: float = 0.1) -> np.ndarray:
    """Held-out mask over all 2^24 colour ids: colour id k is a test colour
    when the k-th uniform draw of a Philox stream keyed by `seed` is below
    `test_fraction` (about 10%, fixed per seed)."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    return rng.random(1 << 24) < test_fraction
