// Device helpers shared by the library's kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/cvib.h"
#include "cvib_device.h"

namespace cvib {

// ---------------------------------------------------------------------------
// Small wave-level helpers (wave64).

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// The lane index from an mbcnt the compiler can neither hoist nor merge:
// taken at the top of a persistent loop's body, the per-lane values derived
// from it (LDS addresses, lane tests) are recomputed every iteration instead
// of being kept live across the loop, where they would spill to scratch.
__device__ __forceinline__ uint32_t lane_id_fresh() {
    uint32_t l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
}

// A value known to be equal in every lane, moved to a scalar register.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// sRGB decode and L* companding in FP64 (per colour, not on the hot loop).

__device__ __forceinline__ double decode_srgb(double c) {
    return c <= 0.04045 ? c / 12.92 : pow((c + 0.055) / 1.055, 2.4);
}

__device__ __forceinline__ double lab_f(double t) {
    const double d3 = kDelta * kDelta * kDelta;
    return t > d3 ? cbrt(t) : t / kLinSlope + 4.0 / 29.0;
}

struct MatArgs {
    double M[9];    // linear RGB -> XYZ
    double Minv[9]; // XYZ -> linear RGB
    double W[3];    // white point
};

__device__ __forceinline__ void rgb8_lab(const MatArgs& m, const uint8_t* p, double lab[3]) {
    double lin[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) lin[k] = decode_srgb((double)p[k] / 255.0);
    double f[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double x = m.M[3 * r] * lin[0] + m.M[3 * r + 1] * lin[1] + m.M[3 * r + 2] * lin[2];
        f[r] = lab_f(x / m.W[r]);
    }
    lab[0] = 116.0 * f[1] - 16.0;
    lab[1] = 500.0 * (f[0] - f[1]);
    lab[2] = 200.0 * (f[1] - f[2]);
}

// ---------------------------------------------------------------------------
// Angle table.  theta_j = 360 j / N degrees.  sin(2 pi m / N) is evaluated
// after folding m with exact integer steps: the half-turn fold makes
// tab[j + N/2] = -tab[j] bitwise (so the + and - colours of ray j are the -
// and + colours of ray j + N/2), the pi - x fold keeps the argument within a
// quarter turn, and when 8 | N the octant fold keeps it within 45 degrees.

__device__ inline double sin_turn(int64_t m, int64_t N) {
    m %= N;
    if (m < 0) m += N;
    double sgn = 1.0;
    if (2 * m >= N) { m -= N / 2; sgn = -1.0; }
    if (4 * m > N) m = N / 2 - m;
    if (N % 8 == 0 && 8 * m > N) return sgn * cos((double)(N / 4 - m) * (2.0 * M_PI / (double)N));
    return sgn * sin((double)m * (2.0 * M_PI / (double)N));
}

__device__ inline double cos_turn(int64_t m, int64_t N) {
    m %= N;
    if (m < 0) m += N;
    double sgn = 1.0;
    if (2 * m >= N) { m -= N / 2; sgn = -sgn; }
    if (4 * m > N) { m = N / 2 - m; sgn = -sgn; }
    if (N % 8 == 0 && 8 * m > N) return sgn * sin((double)(N / 4 - m) * (2.0 * M_PI / (double)N));
    return sgn * cos((double)m * (2.0 * M_PI / (double)N));
}

// ---------------------------------------------------------------------------
// Shared pieces of the search kernels.

struct SumAcc {            // per-colour accumulators (zeroed before a launch)
    uint32_t count, n_gamut, best_key, _pad;
    uint32_t pat[7], _pad2;
    uint32_t bins[36];
};
static_assert(sizeof(SumAcc) == 192, "SumAcc layout");

struct TabArgs {
    const double* tab;
    int32_t tab_len;  // doubles in the table
    int32_t N;        // angles per full turn
    int32_t dW;       // rays 0..dW-1 get their own sin / cos entries in LDS (0 = none)
    int32_t _pad;
};

// Rays given their own LDS entries at most (16 bytes each).
constexpr int32_t kDirectRays = 3072;

// Direct rays for a kernel over rays j < (ntheta, or N/2 when theta spans the
// full turn) that keeps `extra` more bytes of dynamic LDS: all of them when
// the tables fit in 56 KiB together, else none.
inline int32_t direct_rays(int32_t ntheta, int32_t N, int32_t tab_len, size_t extra) {
    const int32_t W = ntheta == N ? N / 2 : ntheta;
    if (W > kDirectRays) return 0;
    if (8 * (size_t)tab_len + 16 * (size_t)W + extra > 56 * 1024) return 0;
    return W;
}

// Dynamic LDS of the angle tables: the folded table, then sin and cos of the
// direct rays.
__host__ __device__ inline size_t angle_lds_bytes(const TabArgs& t) {
    return 8 * (size_t)t.tab_len + 16 * (size_t)t.dW;
}

// sin and cos of theta_j = 2 pi j / N (0 <= j < N) from the folded table.
// The folds are exact integer steps, so ray j + N/2 reads the negated values
// of ray j bit for bit.
__device__ __forceinline__ void sincos_j(const double* tab, int32_t N, int32_t j, double& s,
                                         double& c) {
    const int32_t H = N >> 1;
    const bool back = j >= H;          // second half-turn: negate both
    const int32_t jj = back ? j - H : j;
    if ((N & 3) == 0) {
        const int32_t Q = N >> 2;
        const bool lo = jj <= Q;
        const double a = tab[lo ? jj : H - jj];  // sin(jj) = sin(pi - jj)
        const double b = tab[lo ? Q - jj : jj - Q];
        s = back ? -a : a;
        const double cc = lo ? b : -b;            // cos(jj) = -sin(jj - pi/2)
        c = back ? -cc : cc;
    } else {
        const double a = tab[jj], b = tab[H + 1 + jj];
        s = back ? -a : a;
        c = back ? -b : b;
    }
}

// Angle lookup for the hot loops: two LDS reads for a direct ray, else the
// folding of sincos_j.  Both give the same bits.
struct Angles {
    const double* fold;
    const double* sn;
    const double* cs;
    int32_t N;
    bool direct;
    __device__ __forceinline__ void get(int32_t j, double& s, double& c) const {
        if (direct) {
            s = sn[j];
            c = cs[j];
        } else {
            sincos_j(fold, N, j, s, c);
        }
    }
};

// Copy the folded table to LDS (s_dyn) and expand the direct rays from it.
// Every thread of the block must call it; it ends with a barrier.
__device__ inline Angles load_angles(const TabArgs& t, double* s_dyn) {
    const int nt = (int)blockDim.x;
    for (int k = (int)threadIdx.x; k < t.tab_len; k += nt) s_dyn[k] = t.tab[k];
    __syncthreads();
    Angles a;
    a.fold = s_dyn;
    a.sn = s_dyn + t.tab_len;
    a.cs = a.sn + t.dW;
    a.N = t.N;
    a.direct = t.dW > 0;
    if (a.direct) {
        for (int k = (int)threadIdx.x; k < t.dW; k += nt) {
            double sv, cv;
            sincos_j(s_dyn, t.N, k, sv, cv);
            s_dyn[t.tab_len + k] = sv;
            s_dyn[t.tab_len + t.dW + k] = cv;
        }
        __syncthreads();
    }
    return a;
}

// Gamut cells.  A cell is a block of candidates: rows i0..i1 by rays j0..j1
// (the reduce kernel makes one of each wave step's evaluations).
// cell_out_of_gamut proves, by interval arithmetic, that in every pair of the
// cell one colour has a linear channel outside [0, 1], so that no candidate
// of the cell is in gamut:
// - sin and cos of the cell's rays lie between their values at j0 and j1,
//   widened to +-1 where the rays pass 90, 180 or 270 degrees (between those
//   angles both are monotone);
// - the displacements (i + 1) ra sin and (i + 1) rb cos are bilinear in the
//   radius and the sine (cosine) with a positive radius, so their ranges are
//   spanned by the four corners;
// - finv is increasing, so f -> finv(f) maps the ranges of f to the ranges
//   of the companded values;
// - a linear channel A finv(fx) + C finv(fz) + B is bounded term by term.
// The verdict needs a channel beyond the unit interval by kCellMargin, far
// above the rounding of the bounds and of the kernels' own FP64 arithmetic,
// and the FP32 rounding of the channel cannot bring such a value back.
constexpr double kCellMargin = 1e-6;

// Cells are used only for grids of at least this many evaluated rays per row:
// a wave step of 64 rays that spans more than half of them rarely lies wholly
// out of gamut (measured: the 90-ray whole-cube table loses 6% with cells).
constexpr int32_t kCellMinRays = 128;
// Band-order steps (4 rays by 16 rows) need 16 W > 64 and pay from about 32
// rays per row.
constexpr int32_t kBandMinRays = 32;

// Ranges [lo[k], hi[k]] of the three linear channels of one colour over the
// f-space box [xlo, xhi] x [zlo, zhi].
__device__ inline void colour_bounds(const Geom& g, const ColorConst& cc, double xlo, double xhi, double zlo,
                                     double zhi, double lo[3], double hi[3]) {
    const double gx0 = finv(xlo), gx1 = finv(xhi), gz0 = finv(zlo), gz1 = finv(zhi);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double ax0 = g.A[k] * gx0, ax1 = g.A[k] * gx1, cz0 = g.C[k] * gz0, cz1 = g.C[k] * gz1;
        lo[k] = cc.B[k] + fmin(ax0, ax1) + fmin(cz0, cz1);
        hi[k] = cc.B[k] + fmax(ax0, ax1) + fmax(cz0, cz1);
    }
}

__device__ inline bool bounds_out(const double lo[3], const double hi[3]) {
    bool out = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) out = out || hi[k] < -kCellMargin || lo[k] > 1.0 + kCellMargin;
    return out;
}

__device__ inline bool colour_out(const Geom& g, const ColorConst& cc, double xlo, double xhi, double zlo,
                                  double zhi) {
    double lo[3], hi[3];
    colour_bounds(g, cc, xlo, xhi, zlo, zhi, lo, hi);
    return bounds_out(lo, hi);
}

// Whether a cell may hold a pair with some channel changing by more than
// v_th codes (a "high" channel, which every accepted pattern has), given the
// ranges of both colours' linear channels.  Only pairs with both colours in
// gamut can be accepted, so the ranges are cut to [0, 1] (widened by
// kCellMargin first); the 8-bit code rint(encode(l)) is increasing in l, so
// a channel's change is at most encode(hi of one colour) - encode(lo of the
// other) + 1.  The test asks for at most v_th - 1.5 before that + 1, which
// leaves half a code for the FP32 encode's own error.
__device__ inline void cut_unit(const double lo[3], const double hi[3], float l[3], float h[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        l[k] = (float)fmin(fmax(lo[k] - kCellMargin, 0.0), 1.0);
        h[k] = (float)fmin(fmax(hi[k] + kCellMargin, 0.0), 1.0);
    }
}

__device__ inline bool bounds_high(const float pl[3], const float ph[3], const float ml[3], const float mh[3],
                                   float v_th) {
    bool high = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float d = fmaxf(encode255(ph[k]) - encode255(ml[k]), encode255(mh[k]) - encode255(pl[k]));
        high = high || d > v_th - 1.5f;
    }
    return high;
}

// The gamut test of a cell with the end rays' sin and cos given (j0 <= j1 <
// 2N); with `high` given, it also receives bounds_high of the cell.
__device__ inline bool cell_out_of_gamut_ends(const ColorConst& cc, const Geom& g, int32_t N_, double ra,
                                              double rb, int32_t i0, int32_t i1, int32_t j0, int32_t j1,
                                              double s0, double c0, double s1, double c1,
                                              const RuleDev* rule = nullptr, bool* high = nullptr) {
    double slo = fmin(s0, s1), shi = fmax(s0, s1), clo = fmin(c0, c1), chi = fmax(c0, c1);
    const int64_t N = N_, J0 = 4 * (int64_t)j0, J1 = 4 * (int64_t)j1;
    if ((J0 <= N && N <= J1) || (J0 <= 5 * N && 5 * N <= J1)) shi = 1.0;   // 90, 450 deg
    if (J0 <= 2 * N && 2 * N <= J1) clo = -1.0;                               // 180 deg
    if (J0 <= 3 * N && 3 * N <= J1) slo = -1.0;                               // 270 deg
    if (J0 <= 4 * N && 4 * N <= J1) chi = 1.0;                                // 360 deg
    const double r0 = (double)(i0 + 1), r1 = (double)(i1 + 1);
    const double dxlo = fmin((r0 * ra) * slo, (r1 * ra) * slo), dxhi = fmax((r0 * ra) * shi, (r1 * ra) * shi);
    const double dzlo = fmin((r0 * rb) * clo, (r1 * rb) * clo), dzhi = fmax((r0 * rb) * chi, (r1 * rb) * chi);
    // + colour: (fx0 + dx, fz0 - dz); - colour: (fx0 - dx, fz0 + dz)
    double lo[3], hi[3];
    float pl[3], ph[3], ml[3], mh[3];
    colour_bounds(g, cc, cc.fx0 + dxlo, cc.fx0 + dxhi, cc.fz0 - dzhi, cc.fz0 - dzlo, lo, hi);
    bool out = bounds_out(lo, hi);
    cut_unit(lo, hi, pl, ph);
    colour_bounds(g, cc, cc.fx0 - dxhi, cc.fx0 - dxlo, cc.fz0 + dzlo, cc.fz0 + dzhi, lo, hi);
    out = out || bounds_out(lo, hi);
    cut_unit(lo, hi, ml, mh);
    if (high) *high = !out && bounds_high(pl, ph, ml, mh, rule->v_th);
    return out;
}

__device__ inline bool cell_out_of_gamut(const ColorConst& cc, const Geom& g, const Angles& ang, double ra,
                                         double rb, int32_t i0, int32_t i1, int32_t j0, int32_t j1,
                                         const RuleDev* rule = nullptr, bool* high = nullptr) {
    double s0, c0, s1, c1;
    ang.get(j0, s0, c0);
    ang.get(j1, s1, c1);
    return cell_out_of_gamut_ends(cc, g, ang.N, ra, rb, i0, i1, j0, j1, s0, c0, s1, c1, rule, high);
}

// Lane masks of the per-channel classification of a wave's candidates:
// H[k] = change above v_th (high), L[k] = change at most lo_max (low).  A
// lane carries pattern p = 4 R + 2 G + B exactly when, per channel, it is in
// H (bit set) or L (bit clear); high and low never overlap (lo_max < v_th).
struct PatMasks {
    uint64_t H[3], L[3];
};

__device__ __forceinline__ PatMasks pattern_masks(const float Vp[3], const float Vm[3],
                                                  const RuleDev& r) {
    PatMasks m;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float d = fabsf(Vp[k] - Vm[k]);
        m.H[k] = __ballot(d > r.v_th);
        m.L[k] = __ballot(d <= r.lo_max);
    }
    return m;
}

__device__ __forceinline__ uint64_t pattern_lanes(const PatMasks& m, uint32_t p) {
    return ((p & 4u) ? m.H[0] : m.L[0]) & ((p & 2u) ? m.H[1] : m.L[1]) & ((p & 1u) ? m.H[2] : m.L[2]);
}

// Lanes whose pattern the rule accepts.
// Every lane with a pattern (all channels high or low, one high at least);
// for a partial mask each lane looks its own pattern up in the mask, so that
// no per-pattern flag stays live across a loop.
__device__ __forceinline__ uint64_t accepted_lanes(const PatMasks& m, uint32_t mask) {
    const uint64_t any = (m.H[0] | m.L[0]) & (m.H[1] | m.L[1]) & (m.H[2] | m.L[2]) & (m.H[0] | m.H[1] | m.H[2]);
    if ((mask & 0x7Fu) == 0x7Fu) return any;
    const uint32_t lane = lane_id();
    const uint32_t p = (uint32_t)(((m.H[0] >> lane) & 1ull) << 2 | ((m.H[1] >> lane) & 1ull) << 1 |
                                  ((m.H[2] >> lane) & 1ull));
    return any & __ballot(((mask >> ((p - 1u) & 7u)) & 1u) != 0u);
}

// Lanes of each pattern among `lanes`, added to the wave's counts for every
// pattern whether the rule accepts it or not: a caller keeps the counts of the
// accepted patterns only (accepted_counts), outside its loop.
__device__ __forceinline__ void count_patterns(const PatMasks& m, uint64_t lanes, uint32_t pat[7]) {
#pragma unroll
    for (uint32_t p = 1; p <= 7; ++p) pat[p - 1] += (uint32_t)__builtin_popcountll(pattern_lanes(m, p) & lanes);
}

__device__ __forceinline__ uint32_t accepted_count(uint32_t mask, int q, uint32_t count) {
    return ((mask >> q) & 1u) ? count : 0u;
}

// Key of the maximum-amplitude pair: larger i wins, then smaller j.  0 = none.
__device__ __forceinline__ uint32_t best_key(int32_t i, int32_t j) {
    return ((uint32_t)i << 16) | (0xFFFFu - (uint32_t)j);
}

// Split x (< 2^24) by d using an FP32 reciprocal and one correction step.
__device__ __forceinline__ void divmod_small(int32_t x, int32_t d, float inv_d, int32_t& q,
                                             int32_t& r) {
    q = (int32_t)((float)x * inv_d);
    r = x - q * d;
    if (r < 0) { --q; r += d; }
    if (r >= d) { ++q; r -= d; }
}

// Whether a wave step may hold a pair with both colours in gamut.  The step
// covers evaluations e0..e1 (e1 - e0 < 64) counted in row-major order from
// ray jb0 of row row0 (jb0 + e1 < 2^24): one row, the end of one row and the
// start of the next, or (W < 64) every ray of several rows.  `any` says
// whether the step exists; e0 and e1 must be valid either way.  Every lane of
// the wave calls it (the test of a second row runs when any lane needs it).
// In half-turn mode (sym: W = N/2) ray j of a row is the mirror of ray j + W,
// so a step that runs into the next row covers, for both rows, the angles
// from ray ja up to ray W + jb: one test.
// With `high` given (and the rule), *high receives whether an open step may
// hold a pair with a high channel (bounds_high of its cells); a step that
// may not holds no survivor, and only its gamut count is needed.
__device__ inline bool step_open(const ColorConst& cc, const Geom& g, const Angles& ang, double ra, double rb,
                                 int32_t W, float inv_W, int32_t row0, int32_t jb0, int32_t e0, int32_t e1,
                                 bool any, bool sym = false, const RuleDev* rule = nullptr, bool* high = nullptr) {
    int32_t ia, ja, ib, jb;
    divmod_small(jb0 + e0, W, inv_W, ia, ja);
    divmod_small(jb0 + e1, W, inv_W, ib, jb);
    ia += row0;
    ib += row0;
    const bool two = ib == ia + 1, many = ib > ia + 1;
    if (sym && !many) {
        double s0, c0, s1, c1;
        ang.get(ja, s0, c0);
        ang.get(jb, s1, c1);
        if (two) {  // ray W + jb: the negated values of ray jb
            s1 = -s1;
            c1 = -c1;
        }
        return any && !cell_out_of_gamut_ends(cc, g, ang.N, ra, rb, ia, ib, ja, two ? W + jb : jb, s0, c0, s1, c1,
                                              rule, high);
    }
    bool h1 = true;
    bool open = !cell_out_of_gamut(cc, g, ang, ra, rb, ia, many ? ib : ia, many ? 0 : ja, ib > ia ? W - 1 : jb,
                                   rule, high ? &h1 : nullptr);
    bool hi = open && h1;
    if (__ballot(any && two) != 0ull) {
        bool h2 = true;
        const bool o2 = !cell_out_of_gamut(cc, g, ang, ra, rb, ib, ib, 0, jb, rule, high ? &h2 : nullptr);
        open = open || (two && o2);
        hi = hi || (two && o2 && h2);
    }
    if (high) *high = hi;
    return open && any;
}

// The same for a wave step of the band order: evaluations are numbered by
// bands of kBandRows rows, each band ray by ray and, within a ray, row by row
// (evaluation E is row kBandRows (E / (kBandRows W)) + E % kBandRows, ray
// (E % (kBandRows W)) / kBandRows), so that 64 consecutive evaluations cover
// 64 / kBandRows rays of kBandRows rows.  The step E0..E1 lies in one band or
// runs into the next one (kBandRows W > 64).  Rows past nr are bounded too
// (they are not live).
constexpr int32_t kBandRows = 16;

struct BandPos {
    int32_t i, j;
};

// Row and ray of band-order evaluation e (< 2^24); inv_WB = 1 / (kBandRows W).
__device__ __forceinline__ BandPos band_pos(int32_t e, int32_t W, float inv_WB) {
    int32_t band, q;
    divmod_small(e, kBandRows * W, inv_WB, band, q);
    return BandPos{kBandRows * band + (q & (kBandRows - 1)), q / kBandRows};
}

__device__ inline bool band_step_open(const ColorConst& cc, const Geom& g, const Angles& ang, double ra,
                                      double rb, int32_t W, float inv_WB, int32_t E0, int32_t E1, bool any,
                                      const RuleDev* rule = nullptr, bool* high = nullptr) {
    int32_t ba, qa, bb, qb;
    divmod_small(E0, kBandRows * W, inv_WB, ba, qa);
    divmod_small(E1, kBandRows * W, inv_WB, bb, qb);
    const bool two = bb != ba;
    const int32_t R = kBandRows;
    bool h1 = true;
    bool open = !cell_out_of_gamut(cc, g, ang, ra, rb, R * ba, R * ba + R - 1, qa / R, two ? W - 1 : qb / R, rule,
                                   high ? &h1 : nullptr);
    bool hi = open && h1;
    if (__ballot(any && two) != 0ull) {
        bool h2 = true;
        const bool o2 = !cell_out_of_gamut(cc, g, ang, ra, rb, R * bb, R * bb + R - 1, 0, qb / R, rule,
                                           high ? &h2 : nullptr);
        open = open || (two && o2);
        hi = hi || (two && o2 && h2);
    }
    if (high) *high = hi;
    return open && any;
}

__device__ __forceinline__ void write_summary(const ColorConst& cc, const Geom& g,
                                              const RuleDev& rule, const TabArgs& tab,
                                              double ra, double rb, uint32_t count, uint32_t ng,
                                              uint32_t key, const uint32_t pat[7],
                                              cv_color_summary* out) {
    cv_color_summary s;
    s.count = count;
    s.n_gamut = ng;
    s.best_i = 0xFFFF;
    s.best_j = 0;
    for (int k = 0; k < 3; ++k) s.best_plus[k] = s.best_minus[k] = 0;
    s.best_p = 0;
    s._pad = 0;
    for (int p = 0; p < 7; ++p) s.per_pattern[p] = pat[p];
    if (key) {
        const int32_t i = (int32_t)(key >> 16), j = (int32_t)(0xFFFFu - (key & 0xFFFFu));
        double sn, co;
        sincos_j(tab.tab, tab.N, j, sn, co);
        const double rr = (double)(i + 1);
        PairEval e;
        eval_pair(cc, g, (rr * ra) * sn, (rr * rb) * co, e);
        s.best_i = (uint16_t)i;
        s.best_j = (uint16_t)j;
        for (int k = 0; k < 3; ++k) {
            s.best_plus[k] = (uint8_t)e.Vp[k];
            s.best_minus[k] = (uint8_t)e.Vm[k];
        }
        s.best_p = (uint8_t)pattern_of(e.Vp, e.Vm, rule);
    }
    *out = s;
}

} // namespace cvib
