"""The gamut-cell proof, checked on the CPU against brute force.

The search kernels skip a block of candidates (rows i0..i1 by rays j0..j1)
when an interval bound shows that, for every candidate of the block, one
colour of the pair has a linear channel outside [0, 1] by more than 1e-6.
The bound is written out here once more in FP64 numpy, from its
mathematical statement:
- sin and cos over the rays lie between their end values, widened to +-1
  where the block passes 90, 180, 270 (or 360, 450) degrees;
- the displacements (i + 1) dr/500 sin and (i + 1) dr/200 cos are bilinear
  in the radius and the sine (cosine), so the four corners bound them;
- f^-1 is increasing, so it maps the intervals of f to intervals;
- a linear channel A f^-1(fx) + C f^-1(fz) + B is bounded term by term.
Three properties are checked on several hundred blocks of the shapes the
kernels use (one or two rows of 64 rays, the mirrored range of a half-turn
row crossing, 16 rows by 4 rays, several whole rows, up to 24 rows by 64
rays, and blocks of 256 rays, one row or a crossing):
- containment: every linear channel of both colours of every candidate
  (FP64 oracle) lies inside the block's intervals -- any narrowing fails it,
  whatever the gamut's shape;
- soundness: no block the bound rejects holds a candidate that the oracle
  finds in gamut;
- usefulness: the bound rejects most blocks that are wholly out of gamut.
A dropped term, a wrong sign, a missed widening or a transposed operand
breaks one of them.
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W

MARGIN = 1e-6
DELTA = 6.0 / 29.0


def _finv(u):
    return u ** 3 if u > DELTA else 3.0 * DELTA * DELTA * (u - 4.0 / 29.0)


class _Bound:
    def __init__(self, oracle, rgb, dr, dtheta):
        _, Minv, Wt = oracle.matrices()
        L, a, b = oracle.rgb8_to_lab(rgb)[0]
        fy = (L + 16.0) / 116.0
        self.fx0, self.fz0 = fy + a / 500.0, fy - b / 200.0
        Y = Wt[1] * _finv(fy)
        self.A = [Minv[k, 0] * Wt[0] for k in range(3)]
        self.C = [Minv[k, 2] * Wt[2] for k in range(3)]
        self.B = [Minv[k, 1] * Y for k in range(3)]
        self.ra, self.rb = dr / 500.0, dr / 200.0
        self.N = int(round(360.0 / dtheta))

    def _channels(self, xlo, xhi, zlo, zhi):
        gx = (_finv(xlo), _finv(xhi))
        gz = (_finv(zlo), _finv(zhi))
        res = []
        for k in range(3):
            ax = [self.A[k] * v for v in gx]
            cz = [self.C[k] * v for v in gz]
            lo = self.B[k] + min(ax) + min(cz)
            hi = self.B[k] + max(ax) + max(cz)
            res.append((lo, hi))
        return res

    def intervals(self, i0, i1, j0, j1):
        """[(lo, hi) of the three linear channels] of the + and - colours."""
        N = self.N
        th0, th1 = 2 * np.pi * j0 / N, 2 * np.pi * j1 / N
        s = (np.sin(th0), np.sin(th1))
        c = (np.cos(th0), np.cos(th1))
        slo, shi, clo, chi = min(s), max(s), min(c), max(c)
        J0, J1 = 4 * j0, 4 * j1
        if J0 <= N <= J1 or J0 <= 5 * N <= J1:
            shi = 1.0
        if J0 <= 2 * N <= J1:
            clo = -1.0
        if J0 <= 3 * N <= J1:
            slo = -1.0
        if J0 <= 4 * N <= J1:
            chi = 1.0
        r0, r1 = i0 + 1.0, i1 + 1.0
        dx = [r * self.ra * v for r in (r0, r1) for v in (slo, shi)]
        dz = [r * self.rb * v for r in (r0, r1) for v in (clo, chi)]
        dxlo, dxhi, dzlo, dzhi = min(dx), max(dx), min(dz), max(dz)
        return (self._channels(self.fx0 + dxlo, self.fx0 + dxhi, self.fz0 - dzhi, self.fz0 - dzlo),
                self._channels(self.fx0 - dxhi, self.fx0 - dxlo, self.fz0 + dzlo, self.fz0 + dzhi))

    def out(self, i0, i1, j0, j1):
        """True when no candidate of rows i0..i1 x rays j0..j1 (j1 < 2N) can
        have both colours in gamut."""
        return any(hi < -MARGIN or lo > 1.0 + MARGIN
                   for colour in self.intervals(i0, i1, j0, j1) for lo, hi in colour)


def _blocks(rng, nr, W_):
    """(kind, rows, ray ranges as the bound sees them, candidates (i, j))."""
    out = []
    for _ in range(60):
        i = int(rng.integers(0, nr)); j0 = int(rng.integers(0, W_ - 64))
        out.append(("row", (i, i, j0, j0 + 63), [(i, j) for j in range(j0, j0 + 64)]))
    for _ in range(30):
        i = int(rng.integers(0, nr - 1)); ja = int(rng.integers(W_ - 63, W_))
        jb = 63 - (W_ - ja)
        cand = [(i, j) for j in range(ja, W_)] + [(i + 1, j) for j in range(0, jb + 1)]
        out.append(("two rows", None, cand, (i, ja, jb)))
    for _ in range(30):
        i = int(rng.integers(0, nr - 1)); ja = int(rng.integers(W_ - 63, W_))
        jb = 63 - (W_ - ja)
        # half-turn crossing: rows i, i + 1 over rays ja .. W + jb; ray W + j
        # is ray j's pair with + and - swapped
        cand = [(r, j) for r in (i, i + 1) for j in list(range(ja, W_)) + list(range(0, jb + 1))]
        out.append(("mirrored", (i, i + 1, ja, W_ + jb), cand))
    for _ in range(40):
        b = int(rng.integers(0, nr // 16)); j0 = int(rng.integers(0, W_ - 4))
        out.append(("band", (16 * b, 16 * b + 15, j0, j0 + 3),
                    [(16 * b + q, j) for q in range(16) for j in range(j0, j0 + 4)]))
    for _ in range(30):
        # the count pass's coarse cells: the rows of a tile by 64 rays
        i0 = int(rng.integers(0, nr - 24)); i1 = i0 + int(rng.integers(1, 24))
        j0 = 64 * int(rng.integers(0, (W_ - 1) // 64 + 1)); j1 = min(j0 + 63, W_ - 1)
        out.append(("column", (i0, i1, j0, j1), [(i, j) for i in range(i0, i1 + 1) for j in range(j0, j1 + 1)]))
    if W_ > 256:
        # blocks of 256 evaluations: one row, or a half-turn crossing in
        # mirrored form
        for _ in range(20):
            i = int(rng.integers(0, nr)); j0 = int(rng.integers(0, W_ - 256))
            out.append(("row", (i, i, j0, j0 + 255), [(i, j) for j in range(j0, j0 + 256)]))
        for _ in range(20):
            i = int(rng.integers(0, nr - 1)); ja = int(rng.integers(W_ - 255, W_))
            jb = 255 - (W_ - ja)
            cand = [(r, j) for r in (i, i + 1) for j in list(range(ja, W_)) + list(range(0, jb + 1))]
            out.append(("mirrored", (i, i + 1, ja, W_ + jb), cand))
    return out


@pytest.mark.parametrize("dth,nt", [(1.0, 360), (0.5, 720)])
def test_gamut_cell_bound_is_sound_and_useful(oracle, dth, nt):
    rng = np.random.default_rng(11)
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(12, 15),
                           np.array([[255, 0, 0], [0, 0, 0], [250, 250, 5], [2, 3, 250]], np.uint8)])
    dr, nr = 0.25, 200   # rays of the half-turn: W = nt / 2
    W_ = nt // 2
    proven = wholly_out = 0
    for ci, rgb in enumerate(cols):
        bd = _Bound(oracle, rgb[None, :], dr, dth)
        for blk in _blocks(rng, nr, W_):
            kind, cand = blk[0], blk[2]
            if kind == "two rows":
                i, ja, jb = blk[3]
                rej = bd.out(i, i, ja, W_ - 1) and bd.out(i + 1, i + 1, 0, jb)
            else:
                rej = bd.out(*blk[1])
            idx = np.array([(0, i, j) for i, j in cand], np.int64)
            ev = oracle.eval_list(rgb[None, :], idx, (dr, nr, dth, nt))
            both = ev["gamut"] == 3
            if rej:
                assert not both.any(), (ci, kind, blk[1])
                proven += 1
            if not both.any():
                wholly_out += 1
    assert wholly_out > 100
    assert proven > 0.6 * wholly_out, (proven, wholly_out)


def test_gamut_cell_bound_whole_rows(oracle):
    """Blocks of several whole rows (a wave step when fewer than 64 rays make
    a row) and blocks that cross 360 degrees in the mirrored form."""
    rng = np.random.default_rng(12)
    dr, nr, dth, nt = 1.0, 60, 15.0, 24   # W = 12
    for rgb in W.random_colours(13, 12):
        bd = _Bound(oracle, rgb[None, :], dr, dth)
        for _ in range(20):
            i0 = int(rng.integers(0, nr - 6)); i1 = i0 + int(rng.integers(1, 6))
            cand = [(0, i, j) for i in range(i0, i1 + 1) for j in range(nt // 2)]
            ev = oracle.eval_list(rgb[None, :], np.array(cand, np.int64), (dr, nr, dth, nt))
            if bd.out(i0, i1, 0, nt // 2 - 1):
                assert not (ev["gamut"] == 3).any()
        for _ in range(20):  # rays 300 .. 420 degrees of one row: through 360
            i = int(rng.integers(0, nr))
            j0 = 20
            cand = [(0, i, j % nt) for j in range(j0, j0 + 9)]
            ev = oracle.eval_list(rgb[None, :], np.array(cand, np.int64), (dr, nr, dth, nt))
            if bd.out(i, i, j0, j0 + 8):
                assert not (ev["gamut"] == 3).any()


@pytest.mark.parametrize("dth,nt", [(1.0, 360), (0.5, 720)])
def test_gamut_cell_intervals_contain_every_candidate(oracle, dth, nt):
    """Containment: every linear channel of both colours of every candidate
    of a block (FP64 oracle) lies inside the block's intervals.  This holds
    for any colour and block, in or out of gamut, and fails for any bound
    that is too narrow somewhere."""
    rng = np.random.default_rng(14)
    dr, nr = 0.5, 100
    W_ = nt // 2
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY[:3], W.random_colours(15, 9)])
    for rgb in cols:
        bd = _Bound(oracle, rgb[None, :], dr, dth)
        for blk in _blocks(rng, nr, W_):
            kind, cand = blk[0], blk[2]
            if kind == "two rows":
                continue  # covered by its two one-row pieces in the other kinds
            iv = bd.intervals(*blk[1])
            idx = np.array([(0, i, j) for i, j in cand], np.int64)
            ev = oracle.eval_list(rgb[None, :], idx, (dr, nr, dth, nt))
            for q, (i, j) in enumerate(cand):
                # in the mirrored block, ray j < ja stands for ray W + j:
                # its + colour is the - colour of ray j
                swap = kind == "mirrored" and j < blk[1][2]
                lp, lm = (ev["linm"][q], ev["linp"][q]) if swap else (ev["linp"][q], ev["linm"][q])
                for colour, vals in ((0, lp), (1, lm)):
                    for k in range(3):
                        lo, hi = iv[colour][k]
                        assert lo - 1e-12 <= vals[k] <= hi + 1e-12, (kind, blk[1], i, j, colour, k)


def _encode255(l):
    """sRGB encode in 0..255 code units (IEC 61966-2-1), FP64."""
    l = np.asarray(l, np.float64)
    return np.where(l <= 0.0031308, 255.0 * 12.92 * l, 255.0 * (1.055 * np.power(np.maximum(l, 0.0), 1 / 2.4) - 0.055))


def _no_high(iv, v_th):
    """The kernels' second test of an open cell: with both colours' channel
    ranges cut to [0, 1] (after widening by the margin), whether every
    channel's code change stays at most v_th - 1.5 + 1 below a high one."""
    (p, m) = iv
    for k in range(3):
        pl = min(max(p[k][0] - MARGIN, 0.0), 1.0); ph = min(max(p[k][1] + MARGIN, 0.0), 1.0)
        ml = min(max(m[k][0] - MARGIN, 0.0), 1.0); mh = min(max(m[k][1] + MARGIN, 0.0), 1.0)
        d = max(_encode255(ph) - _encode255(ml), _encode255(mh) - _encode255(pl))
        if d > v_th - 1.5:
            return False
    return True


def test_high_channel_bound_is_sound_and_useful(oracle):
    """Cells where no channel can change by more than v_th codes: no pair of
    such a cell with both colours in gamut has a high channel (so none can
    carry an accepted pattern), while most small-radius cells are proven."""
    rng = np.random.default_rng(16)
    cols = np.concatenate([W.PAPER_COLOUR_ARRAY, W.random_colours(17, 9)])
    dr, nr, dth, nt = 0.25, 200, 1.0, 360
    W_ = nt // 2
    v_th = 50
    proven = small_open = 0
    for rgb in cols:
        bd = _Bound(oracle, rgb[None, :], dr, dth)
        for blk in _blocks(rng, nr, W_):
            kind, cand = blk[0], blk[2]
            if kind == "two rows" or bd.out(*blk[1]):
                continue
            idx = np.array([(0, i, j) for i, j in cand], np.int64)
            ev = oracle.eval_list(rgb[None, :], idx, (dr, nr, dth, nt), (v_th, 0.5, 0x7F))
            both = ev["gamut"] == 3
            d = np.abs(ev["Vp"].astype(int) - ev["Vm"].astype(int)).max(axis=1)
            small = blk[1][1] < 40
            small_open += small
            if _no_high(bd.intervals(*blk[1]), v_th):
                proven += small
                assert not (both & (d > v_th)).any(), (kind, blk[1])
                assert not (ev["valid"] != 0).any(), (kind, blk[1])
    assert small_open > 50
    assert proven > 0.5 * small_open, (proven, small_open)
