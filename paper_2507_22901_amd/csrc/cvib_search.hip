// Colour conversion, the fused generate -> convert -> predicate search with
// single-pass stream compaction, and the reduce-only search (gfx950).
//
// Paper map: Section 2 (target split into L*, a*, b*; displacement arrays
// D_a = r sin(theta), D_b = r cos(theta) added to and subtracted from a*, b*
// with L* fixed; the pairs meeting both conditions are picked out of the
// candidate array) and Section 3 / Table 1 (a channel bit is 1 when its
// change is above V_th and 0 when it is under V_th * R_novib).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "cvib_internal.h"
#include "cvib_kernels.h"

namespace cvib {

// CV_RGB8_TO_LAB
__global__ void k_rgb8_to_lab(const uint8_t* __restrict__ rgb, float* __restrict__ lab, int64_t n,
                              MatArgs m) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double L[3];
    rgb8_lab(m, rgb + 3 * k, L);
    lab[3 * k + 0] = (float)L[0];
    lab[3 * k + 1] = (float)L[1];
    lab[3 * k + 2] = (float)L[2];
}

// CV_LAB_TO_RGBF: the same geometry + transfer arithmetic as the search.
__global__ void k_lab_to_rgbf(const float* __restrict__ lab, float* __restrict__ out, int64_t n,
                              Geom g, MatArgs m) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double L = lab[3 * k], a = lab[3 * k + 1], b = lab[3 * k + 2];
    double fy = (L + 16.0) / 116.0;
    double Y = finv(fy) * m.W[1];
    double B[3] = {m.Minv[1] * Y, m.Minv[4] * Y, m.Minv[7] * Y};
    double lin[3];
    lab_f_to_linear(g, B, fy + a / 500.0, fy - b / 200.0, lin);
    bool in = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float l = (float)lin[c];
        in = in && (l >= 0.0f) && (l <= 1.0f);
        out[4 * k + c] = encode255(l);
    }
    out[4 * k + 3] = in ? 1.0f : 0.0f;
}

// Per-target prologue: RGB8 -> L*a*b* -> the constants of ColorConst.
__device__ __forceinline__ ColorConst color_const(const MatArgs& m, const uint8_t* rgb) {
    double lab[3];
    rgb8_lab(m, rgb, lab);
    double fy = (lab[0] + 16.0) / 116.0;
    double Y = finv(fy) * m.W[1];
    ColorConst c;
    c.fx0 = fy + lab[1] / 500.0;
    c.fz0 = fy - lab[2] / 200.0;
    c.B[0] = m.Minv[1] * Y;
    c.B[1] = m.Minv[4] * Y;
    c.B[2] = m.Minv[7] * Y;
    c.L = (float)lab[0];
    c.a = (float)lab[1];
    c.b = (float)lab[2];
    c._pad = 0;
    return c;
}

__global__ void k_color_prologue(const uint8_t* __restrict__ rgb, ColorConst* __restrict__ cc,
                                 int64_t n, MatArgs m) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    cc[k] = color_const(m, rgb + 3 * k);
}

// Table layout.  N % 4 == 0: tab[k] = sin(2 pi k / N) for 0 <= k <= N/4 (a
// quarter turn).  N % 4 == 2: tab[k] = sin, tab[H + 1 + k] = cos of
// 2 pi k / N for 0 <= k <= H = N/2 (a half turn).
__device__ __forceinline__ void angle_entry(double* __restrict__ tab, int32_t N, int64_t k) {
    if (N % 4 == 0) {
        if (k <= N / 4) tab[k] = sin_turn((int32_t)k, N);
    } else {
        const int32_t H = N / 2;
        if (k <= H) {
            tab[k] = sin_turn((int32_t)k, N);
            tab[H + 1 + k] = cos_turn((int32_t)k, N);
        }
    }
}

__global__ void k_angle_table(double* __restrict__ tab, int32_t N) {
    angle_entry(tab, N, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// The search's set-up in one launch: colour constants, the angle table, and
// zeroed words (the ticket and totals; the per-colour accumulators).
__global__ void k_search_prologue(const uint8_t* __restrict__ rgb, ColorConst* __restrict__ cc, int64_t n,
                                  MatArgs m, double* __restrict__ tab, int32_t N, uint64_t* __restrict__ za,
                                  int64_t na, uint64_t* __restrict__ zb, int64_t nb, uint64_t* __restrict__ zc,
                                  int64_t nc) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) cc[k] = color_const(m, rgb + 3 * k);
    angle_entry(tab, N, k);
    if (k < na) za[k] = 0;
    if (k < nb) zb[k] = 0;
    if (k < nc) zc[k] = 0;
}

struct SearchArgs {
    const ColorConst* cc;
    TabArgs tab;
    Geom g;
    RuleDev rule;
    double ra, rb;             // dr / 500, dr / 200
    int32_t nr, ntheta;
    int32_t W;                 // evaluations per row: ntheta, or N/2 in half-turn mode
    float inv_W;
    int32_t seg_len;           // evaluations per segment (one row in half-turn mode)
    int32_t segs_per_colour;
    int64_t n, nsegs;
    uint32_t* seg_cnt;         // output records per segment (count pass writes)
    const uint64_t* seg_prefix;// output offset per segment (write pass reads)
    uint4* out;                // survivor records (write pass)
    uint64_t capacity;         // records
    SumAcc* acc;               // nullable
    uint64_t* misc;            // [0] count-pass ticket, [2] survivor total
    int32_t cells, _pad;       // skip wave steps proven out of gamut (not with EMIT_ALL)
    const uint64_t* seg_mask;  // write pass: the passes of a segment holding survivors (nullable)
};

// Per-wave flush of a thread's running summary into the colour accumulator.
__device__ __forceinline__ void flush_summary(SumAcc* acc, int64_t col, uint32_t lane,
                                              uint32_t& cnt, uint32_t& ng, uint32_t& best,
                                              uint32_t pat[7]) {
    uint32_t s_cnt = wave_sum_u32(cnt), s_ng = wave_sum_u32(ng), s_best = wave_max_u32(best);
    uint32_t s_pat[7];
#pragma unroll
    for (int p = 0; p < 7; ++p) s_pat[p] = wave_sum_u32(pat[p]);
    if (lane == 0) {
        SumAcc* a = acc + col;
        if (s_cnt) atomicAdd(&a->count, s_cnt);
        if (s_ng) atomicAdd(&a->n_gamut, s_ng);
        if (s_best) atomicMax(&a->best_key, s_best);
#pragma unroll
        for (int p = 0; p < 7; ++p)
            if (s_pat[p]) atomicAdd(&a->pat[p], s_pat[p]);
    }
    cnt = ng = best = 0;
#pragma unroll
    for (int p = 0; p < 7; ++p) pat[p] = 0;
}

// One candidate of the hot loop: geometry in FP64, then (only if some lane of
// the wave has both colours in gamut, or every candidate is to be emitted)
// the FP32 transfer, rounding and the predicate.  Returns the packed record
// bytes and the decision.
// Threads per block of the search kernels: eight waves share one copy of the
// angle tables in LDS.
constexpr int kPassBlock = 512;

template <bool EMIT_ALL>
__device__ __forceinline__ void candidate(const ColorConst& cc, const SearchArgs& a, double s,
                                          double co, int32_t i, bool live, bool cube, uint32_t& lo,
                                          uint32_t& hi, bool& surv, bool& both, uint32_t& pat) {
    const double rr = (double)(i + 1);
    float fp[3], fm[3];
    pair_linear_w(cc, a.g, (rr * a.ra) * s, (rr * a.rb) * co, fp, fm, cube);
    const bool gp = in_unit_cube(fp), gm = in_unit_cube(fm);
    both = live && gp && gm;
    const bool need = a.rule.clip ? live : both;
    surv = false;
    pat = 0;
    lo = hi = 0;
    if (EMIT_ALL || __ballot(need) != 0ull) {
        // every emitted candidate carries its clamped codes: the full encode
        float Vp[3], Vm[3];
        codes_w(fp, fm, need, EMIT_ALL || a.rule.clip, Vp, Vm);
        const uint32_t p = pattern_of(Vp, Vm, a.rule);
        surv = need && accepts(a.rule, p);
        pat = (need || EMIT_ALL) && (a.rule.clip || (gp && gm)) ? p : 0u;
        const uint32_t flags = (gp ? 1u : 0u) | (gm ? 2u : 0u) | (surv ? 4u : 0u);
        pack_pair(Vp, Vm, pat, flags, lo, hi);
    } else if (EMIT_ALL) {
        hi = ((gp ? 1u : 0u) | (gm ? 2u : 0u)) << 24;
    }
}

// ---------------------------------------------------------------------------
// Fused search with compaction.
//
// General mode: a tile is TILE = BLOCK * K consecutive candidates of one
// colour in row-major (i, j) order; pass m of wave w covers evaluations
// [m*BLOCK + 64w, +64), so (m, w, lane) order is candidate order.
//
// Half-turn mode (the grid covers the full turn, ntheta = N): ray j + N/2
// carries ray j's pair with + and - swapped (the angle table is exactly
// antisymmetric), so only j < N/2 is evaluated and every survivor is written
// twice.  A tile is then a set of whole rows i; its output is, row by row, the
// survivors of the first half-row followed by their mirrors, which is again
// (colour, i, j) order.  Tiles follow each other in (colour, row) order, so
// the look-back prefix of a tile is its output offset.
// Fused search: count pass and write pass.
//
// The candidates of a colour are cut into segments of consecutive
// evaluations in row-major (i, j < W) order.  General mode: W = ntheta and a
// segment is seg_len = 512 evaluations.  Half-turn mode (the grid spans the
// full turn, ntheta = N): ray j + N/2 carries ray j's pair with + and -
// swapped (the angle table is exactly antisymmetric), so only j < W = N/2 is
// evaluated, a segment is one whole row, and the row's output is its half-row
// survivors followed by their mirrors -- (colour, i, j) order again.
//
// Each wave owns whole segments (statically strided over all waves of the
// grid), so no barrier, ticket or atomic is on the path:
//   count pass: survivors per segment (and the per-colour summaries);
//   scan:       segment counts -> output offsets, in segment order;
//   write pass: segments with survivors are evaluated again and each wave
//               writes its survivors at offset + (survivors before it in the
//               segment), found with a ballot and the lane rank.
template <bool EMIT_ALL, bool SUMM, bool SYM, bool WRITE>
__global__ __launch_bounds__(kPassBlock) void k_pair_pass(SearchArgs a) {
    constexpr int NW = kPassBlock / 64;
    extern __shared__ double s_tab[];
    const int tid = threadIdx.x;
    const uint32_t lane = (uint32_t)tid & 63u;
    const int w = tid >> 6;
    const Angles ang = load_angles(a.tab, s_tab);

    const uint32_t mult = SYM ? 2u : 1u;
    const int64_t per = (int64_t)a.nr * a.W;
    // Waves stride over the segments statically; most segments hold no
    // survivor and are skipped at the cost of one load.
    const int64_t GW = (int64_t)gridDim.x * NW;

    int64_t cur_c = -1;
    uint32_t acc_cnt = 0, acc_ng = 0, acc_best = 0, acc_pat[7] = {0, 0, 0, 0, 0, 0, 0};

    for (int64_t sg = (int64_t)blockIdx.x * NW + w; sg < a.nsegs; sg += GW) {
        const int64_t c = sg / a.segs_per_colour;
        const int32_t ls = (int32_t)(sg - c * a.segs_per_colour);
        uint64_t base = 0;
        uint32_t half = 0;
        if constexpr (WRITE) {
            const uint32_t cnt = a.seg_cnt[sg];
            if (cnt == 0) continue;
            base = a.seg_prefix[sg];
            half = SYM ? cnt / 2u : 0u;
        }
        if constexpr (SUMM && !WRITE) {
            if (c != cur_c) {
                if (cur_c >= 0) flush_summary(a.acc, cur_c, lane, acc_cnt, acc_ng, acc_best, acc_pat);
                cur_c = c;
            }
        }
        const ColorConst cc = a.cc[c];
        const int32_t base_e = ls * a.seg_len;
        const int32_t len = (int32_t)min((int64_t)a.seg_len, per - base_e);
        int32_t i, j;
        const bool cube = cube_branch_only(cc, (base_e + len - 1) / a.W, a.ra, a.rb);
        uint32_t wtop = 0;             // survivors of this segment before the current pass
        uint32_t cnt = 0, ng = 0, best = 0, steps = 0;
        uint64_t pk = 0;               // 8-bit pattern counters, flushed every 255 passes
        const int32_t iters = (len + 63) >> 6;  // at most 64: a segment is 512 evaluations or a row
        const int32_t i_seg = base_e / a.W, j_seg = base_e - i_seg * a.W;
        uint64_t open_m;
        if (WRITE && !EMIT_ALL && a.seg_mask) {
            open_m = uniform_u64(a.seg_mask[sg]);  // the passes holding survivors
        } else if (!EMIT_ALL && a.cells) {
            // lane l decides pass l; passes proven out of gamut hold no survivor
            const int32_t e0 = (int32_t)lane << 6;
            open_m = uniform_u64(__ballot(step_open(cc, a.g, ang, a.ra, a.rb, a.W, a.inv_W, i_seg, j_seg,
                                                    min(e0, len - 1), min(e0 + 63, len - 1),
                                                    (int32_t)lane < iters)));
        } else {
            open_m = iters >= 64 ? ~0ull : (1ull << iters) - 1ull;
        }
        while (open_m) {
            const int32_t it = (int32_t)__builtin_ctzll(open_m);
            open_m &= open_m - 1ull;
            const bool live = (it << 6) + (int32_t)lane < len;
            divmod_small(j_seg + min((it << 6) + (int32_t)lane, len - 1), a.W, a.inv_W, i, j);
            i += i_seg;
            double sn, co;
            ang.get(j, sn, co);
            uint32_t lo, hi, pat;
            bool surv, both;
            candidate<EMIT_ALL>(cc, a, sn, co, i, live, cube, lo, hi, surv, both, pat);
            const bool emit = EMIT_ALL ? live : surv;
            const uint64_t bal = __ballot(emit);
            if constexpr (WRITE) {
                if (emit) {
                    const uint64_t pos = base + wtop + rank_below(bal);
                    const uint32_t ij = (uint32_t)i | ((uint32_t)j << 16);
                    if (pos < a.capacity) a.out[pos] = make_uint4((uint32_t)c, ij, lo, hi);
                    if constexpr (SYM) {
                        if (pos + half < a.capacity) {
                            uint32_t mlo, mhi;
                            mirror_pair(lo, hi, mlo, mhi);
                            a.out[pos + half] =
                                make_uint4((uint32_t)c, ij + ((uint32_t)a.W << 16), mlo, mhi);
                        }
                    }
                }
            }
            wtop += (uint32_t)__builtin_popcountll(bal);
            if constexpr (SUMM && !WRITE) {
                cnt += surv ? 1u : 0u;
                pk += surv ? (1ull << (8u * ((pat - 1u) & 7u))) : 0ull;
                ng += both ? 1u : 0u;
                best = max(best, surv ? best_key(i, j) : 0u);
                if (++steps == 255) {
#pragma unroll
                    for (int q = 0; q < 7; ++q) acc_pat[q] += mult * ((uint32_t)(pk >> (8 * q)) & 0xFFu);
                    pk = 0;
                    steps = 0;
                }
            }
        }
        if constexpr (!WRITE) {
            if (lane == 0) a.seg_cnt[sg] = mult * wtop;
            if constexpr (SUMM) {
#pragma unroll
                for (int q = 0; q < 7; ++q) acc_pat[q] += mult * ((uint32_t)(pk >> (8 * q)) & 0xFFu);
                acc_cnt += mult * cnt;
                acc_ng += mult * ng;
                acc_best = max(acc_best, best);
            }
        }
    }
    if constexpr (SUMM && !WRITE) {
        if (cur_c >= 0) flush_summary(a.acc, cur_c, lane, acc_cnt, acc_ng, acc_best, acc_pat);
    }
}

// ---------------------------------------------------------------------------
// Per-ray survivors: for every ray of the grid the survivor of largest i, in
// (colour, j) order.  rays[c][jj] holds that i + 1 for the evaluated rays;
// ray j reads jj = j, or j - W (its mirror) in half-turn mode.

__global__ void k_ray_flags(const uint32_t* __restrict__ rays, int64_t n, int32_t W, int32_t ntheta,
                            uint32_t* __restrict__ flags) {
    const int64_t total = n * ntheta;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const int64_t c = t / ntheta;
        const int32_t j = (int32_t)(t - c * ntheta);
        const int32_t jj = j < W ? j : j - W;
        flags[t] = rays[c * W + jj] ? 1u : 0u;
    }
}

__global__ void k_ray_records(const uint32_t* __restrict__ rays, const uint64_t* __restrict__ prefix,
                              int64_t n, int32_t W, int32_t ntheta, const ColorConst* __restrict__ ccs,
                              Geom g, RuleDev rule, TabArgs tab, double ra, double rb,
                              uint4* __restrict__ out, uint64_t capacity) {
    const int64_t total = n * ntheta;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const int64_t c = t / ntheta;
        const int32_t j = (int32_t)(t - c * ntheta);
        const int32_t jj = j < W ? j : j - W;
        const uint32_t r = rays[c * W + jj];
        const uint64_t pos = prefix[t];
        if (!r || pos >= capacity) continue;
        const int32_t i = (int32_t)r - 1;
        double sn, co;
        sincos_j(tab.tab, tab.N, jj, sn, co);
        const double rr = (double)(i + 1);
        PairEval e;
        eval_pair(ccs[c], g, (rr * ra) * sn, (rr * rb) * co, e);
        const uint32_t p = pattern_of(e.Vp, e.Vm, rule);
        const uint32_t fl = (e.gp ? 1u : 0u) | (e.gm ? 2u : 0u) | 4u;
        uint32_t lo, hi;
        pack_pair(e.Vp, e.Vm, p, fl, lo, hi);
        if (j >= W) {  // the mirror: + and - swap
            uint32_t mlo, mhi;
            mirror_pair(lo, hi, mlo, mhi);
            lo = mlo;
            hi = mhi;
        }
        out[pos] = make_uint4((uint32_t)c, (uint32_t)i | ((uint32_t)j << 16), lo, hi);
    }
}

// Summaries of a survivor list: block per colour over its CSR range.  The
// list holds no gamut count (n_gamut = 0).
__global__ __launch_bounds__(256) void k_csr_summary(const uint4* __restrict__ recs,
                                                     const int64_t* __restrict__ offsets, int64_t n,
                                                     cv_color_summary* __restrict__ summ) {
    __shared__ uint32_t s_cnt[8];
    __shared__ uint32_t s_best;
    for (int64_t c = blockIdx.x; c < n; c += gridDim.x) {
        if (threadIdx.x < 8) s_cnt[threadIdx.x] = 0;
        if (threadIdx.x == 0) s_best = 0;
        __syncthreads();
        const int64_t b = offsets[c], e = offsets[c + 1];
        uint32_t best = 0, cnt = 0;
        for (int64_t k = b + threadIdx.x; k < e; k += blockDim.x) {
            const uint4 r = recs[k];
            const uint32_t i = r.y & 0xFFFFu, j = r.y >> 16, p = (r.w >> 16) & 0xFFu;
            best = max(best, (i << 16) | (0xFFFFu - j));
            ++cnt;
            if (p >= 1u && p <= 7u) atomicAdd(&s_cnt[p], 1u);
        }
        best = wave_max_u32(best);
        cnt = wave_sum_u32(cnt);
        if ((threadIdx.x & 63u) == 0) {
            atomicMax(&s_best, best);
            atomicAdd(&s_cnt[0], cnt);
        }
        __syncthreads();
        const uint32_t key = s_best;
        if (threadIdx.x == 0) {
            cv_color_summary o = {};
            o.count = s_cnt[0];
            o.n_gamut = 0;
            o.best_i = 0xFFFFu;
            for (int q = 0; q < 7; ++q) o.per_pattern[q] = s_cnt[q + 1];
            if (!key) summ[c] = o;
        }
        if (key) {
            for (int64_t k = b + threadIdx.x; k < e; k += blockDim.x) {
                const uint4 r = recs[k];
                const uint32_t i = r.y & 0xFFFFu, j = r.y >> 16;
                if (((i << 16) | (0xFFFFu - j)) != key) continue;
                cv_color_summary o = {};
                o.count = s_cnt[0];
                o.n_gamut = 0;
                o.best_i = (uint16_t)i;
                o.best_j = (uint16_t)j;
                const uint8_t* by = reinterpret_cast<const uint8_t*>(&r) + 8;  // plus[3], minus[3], p
                for (int q = 0; q < 3; ++q) {
                    o.best_plus[q] = by[q];
                    o.best_minus[q] = by[3 + q];
                }
                o.best_p = by[6];
                for (int q = 0; q < 7; ++q) o.per_pattern[q] = s_cnt[q + 1];
                summ[c] = o;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Segment record counts -> output offsets: an exclusive scan in segment
// order, which is (colour, i, j) order; also the per-colour CSR offsets.

constexpr int kScanBlock = 256;
constexpr int kScanPer = 16;                       // items per thread
constexpr int kScanChunk = kScanBlock * kScanPer;  // items per block

// Block-wide exclusive scan of one value per thread; `total` receives the sum.
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* s_w,
                                                         uint64_t& total) {
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    uint64_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t u = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o) incl += u;
    }
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    uint64_t before = 0;
    total = 0;
    for (uint32_t q = 0; q < blockDim.x / 64; ++q) {
        if (q < w) before += s_w[q];
        total += s_w[q];
    }
    __syncthreads();
    return before + incl - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(const uint32_t* __restrict__ cnt,
                                                          int64_t T, uint64_t* __restrict__ sums) {
    __shared__ uint64_t s_w[kScanBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    uint64_t v = 0;
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < T) v += cnt[base + k];
    uint64_t total;
    block_exclusive_scan(v, s_w, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the per-block sums by a single block.
__global__ __launch_bounds__(kScanBlock) void k_scan_top(uint64_t* __restrict__ sums, int64_t B,
                                                         uint64_t* __restrict__ total_out) {
    __shared__ uint64_t s_w[kScanBlock / 64];
    uint64_t carry = 0;
    for (int64_t b0 = 0; b0 < B; b0 += kScanBlock) {
        const int64_t b = b0 + threadIdx.x;
        const uint64_t v = b < B ? sums[b] : 0ull;
        uint64_t total;
        const uint64_t ex = block_exclusive_scan(v, s_w, total);
        if (b < B) sums[b] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const uint32_t* __restrict__ cnt,
                                                           int64_t T,
                                                           const uint64_t* __restrict__ sums,
                                                           uint64_t* __restrict__ prefix,
                                                           int64_t* __restrict__ offsets,
                                                           int32_t segs_per_colour, int64_t n,
                                                           const uint64_t* __restrict__ grand) {
    __shared__ uint64_t s_w[kScanBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    uint64_t v = 0;
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < T) v += cnt[base + k];
    uint64_t total;
    uint64_t run = sums[blockIdx.x] + block_exclusive_scan(v, s_w, total);
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t t = base + k;
        if (t >= T) break;
        prefix[t] = run;
        if (offsets && t % segs_per_colour == 0) offsets[t / segs_per_colour] = (int64_t)run;
        run += cnt[t];
    }
    if (offsets && blockIdx.x == 0 && threadIdx.x == 0) offsets[n] = (int64_t)*grand;
}

// ---------------------------------------------------------------------------
// Reduce-only search.  A tile is a chunk of one colour's candidates in
// row-major order (the whole colour when it fits, then results are written
// directly; otherwise per-colour accumulators are merged with atomics and a
// finalize kernel writes the outputs).  The per-ray maximum radius index is
// kept in LDS (one word per angle) when the angle-bin table is requested.

struct ReduceArgs {
    const ColorConst* cc;
    TabArgs tab;
    Geom g;
    RuleDev rule;
    double ra, rb;
    int32_t nr, ntheta;
    int32_t W;                // evaluations per row (ntheta, or N/2 in half-turn mode)
    float inv_W;
    int32_t si, sj;           // a step of one block = si rows + sj rays
    int32_t block;            // threads per block that si, sj were made for
    int32_t chunk;            // evaluations per tile (multiple of the block size)
    int32_t tiles_per_colour;
    int32_t bin_num, bin_den; // bin = (j * bin_num) / bin_den = floor(36 j / N)
    int64_t n, ntiles;
    SumAcc* acc;              // atomic mode
    cv_color_summary* summ;   // direct mode outputs (nullable)
    cv_table_row* table;      // direct mode outputs (nullable)
    uint64_t* misc;           // [0] ticket
    uint32_t* rays_out;       // TABLE: per-ray largest i + 1, [n][W], merged by atomicMax (nullable)
    uint32_t* seg_cnt;        // SEG: output records per segment of the search
    int32_t seg_len;          // SEG: evaluations per segment (chunk is a multiple)
    int32_t segs_per_colour;  // SEG
    // gamut cells: one per wave step, decided per tile into cell_words
    // 64-bit masks per wave (0 = off)
    int32_t cell_words;
    // 0: n_gamut is not asked for (left 0), so open steps proven to hold no
    // high channel are skipped rather than counted
    int32_t need_ng;
    uint64_t* stats;          // [0..7]: candidates skipped by the cells; [8..15]: in-gamut pairs of steps
                              // proven to hold no high channel (not encoded); summed (nullable)
    // SEG: per segment, bit k = survivors among its evaluations 64k..64k+63
    // (the write pass's k-th pass); mask_slots = segments per tile (nullable)
    uint64_t* seg_mask;
    int32_t mask_slots, _pad2;
    // SEG: per-block sums of the scan (kScanChunk segments each), added to
    // by every tile for its segments (zeroed beforehand; nullable)
    uint64_t* scan_sums;
};

// Reduce-only search.  A tile is a chunk of one colour's evaluations (i, j < W)
// in row-major order: the whole colour when it fits (results are then written
// directly), otherwise per-colour accumulators are merged with atomics and a
// finalize kernel writes the outputs.  With the angle-bin table, the largest
// surviving radius index of every evaluated ray is kept in LDS.  In half-turn
// mode (SYM) only rays j < N/2 are evaluated: counts double, and the bins of
// the second half-turn copy the first (bin(theta + 180 deg) = bin(theta) + 18).
// With gamut cells, each tile first decides, for every wave step, whether its
// 64 evaluations are proven out of gamut; such steps are not evaluated (their
// candidates could neither survive nor count as in gamut), and each wave walks
// only the open steps of its mask, deriving (i, j) from the step index.
// Large-chunk blocks of eight waves hold the register budget of six waves per
// SIMD, so that three blocks share a CU.
// Coarse cells of the count pass: at most this many 64-ray columns per row and
// this many listed steps per tile (else every step takes its own proof).
constexpr int32_t kMaxCols = 256;
constexpr int32_t kMaxListed = 2048;

template <int BLOCK, bool TABLE, bool DIRECT, bool SYM, bool SEG, bool CELLS>
__global__ __launch_bounds__(BLOCK, (DIRECT ? 1 : 6)) void k_pair_reduce(ReduceArgs a) {
    constexpr int NW = BLOCK / 64;
    constexpr int MAX_SEG = 2048;  // segments per tile (SEG)
    extern __shared__ double s_dyn[];
    __shared__ uint32_t s_red[NW][10];
    __shared__ uint32_t s_bins[36];
    __shared__ uint32_t s_seg[SEG ? MAX_SEG : 1];
    __shared__ int64_t s_tick;
    // coarse cells of the step proofs (CELLS kernels that deal out steps)
    constexpr bool LISTS = CELLS && !(DIRECT && !SEG);
    __shared__ uint8_t s_colv[LISTS ? kMaxCols : 1];
    __shared__ uint16_t s_list[LISTS ? kMaxListed : 1];
    __shared__ int32_t s_nlist;
    // with the coarse cells: the open steps, in proof order (bit 15: may hold
    // a high channel), dealt to the waves in turn, so that every wave of the
    // block gets as many as the others whatever rows they fall in
    __shared__ uint16_t s_olist[LISTS ? kMaxListed : 1];
    __shared__ int32_t s_nopen;

    const int w_s = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // the wave of the block
    const Angles ang = load_angles(a.tab, s_dyn);
    uint32_t* s_ray = reinterpret_cast<uint32_t*>(s_dyn + a.tab.tab_len + 2 * a.tab.dW);
    uint64_t* s_open =
        reinterpret_cast<uint64_t*>(s_dyn + a.tab.tab_len + 2 * a.tab.dW + (TABLE ? (a.W + 1) / 2 : 0));
    // steps that may hold a high channel (the rest are only counted for n_gamut)
    uint64_t* s_full = s_open + NW * a.cell_words;
    uint64_t* s_mask = s_full + NW * a.cell_words;  // SEG with seg_mask
    const uint32_t mult = SYM ? 2u : 1u;
    const bool clip = a.rule.clip != 0u;
    uint64_t skipped = 0;  // lane's share over the block's tiles
    uint64_t no_high = 0;  // in-gamut pairs of steps without a high channel (lane 0)

    for (;;) {
        // the thread's indices taken afresh every tile (nothing derived from
        // them stays live across the tiles); the wave index as a vector
        // value, as threadIdx.x >> 6 would give it, schedules the tile's
        // loops best
        const int tid = w_s * 64 + (int)lane_id_fresh();
        const uint32_t lane = (uint32_t)tid & 63u;
        const int w = tid >> 6;
        // the ticket, -1 once the tiles are dealt (tested by thread 0 alone,
        // so that the tile count is not held in every lane across the loop)
        if (tid == 0) {
            const int64_t tk = (int64_t)atomicAdd((unsigned long long*)&a.misc[0], 1ull);
            s_tick = tk < a.ntiles ? tk : -1;
        }
        if constexpr (TABLE) {
            for (int k = tid; k < a.W; k += BLOCK) s_ray[k] = 0;
        }
        if constexpr (SEG) {
            for (int k = tid; k < MAX_SEG; k += BLOCK) s_seg[k] = 0;
            if (a.seg_mask)
                for (int k = tid; k < a.mask_slots; k += BLOCK) s_mask[k] = 0;
        }
        if constexpr (CELLS && !(DIRECT && !SEG)) {
            for (int k = tid; k < 2 * NW * a.cell_words; k += BLOCK) s_open[k] = 0;
        }
        __syncthreads();
        const int64_t t = uniform_i64(s_tick);
        if (t < 0) break;
        // the divisor taken afresh every tile: its reciprocal is not hoisted
        // into a register held across the loop
        int32_t tpc = a.tiles_per_colour;
        asm volatile("" : "+s"(tpc));
        const int64_t c = t / tpc;
        const int32_t lt = (int32_t)(t - c * tpc);
        const ColorConst cc = a.cc[c];
        const int32_t begin = lt * a.chunk;
        const int32_t len = min(a.chunk, a.nr * a.W - begin);
        const int32_t seg0 = SEG ? begin / a.seg_len : 0;  // chunks start on segment bounds
        const int32_t row0 = begin / a.W;
        const int32_t jb0 = begin - row0 * a.W;  // ray of the tile's first evaluation
        const int32_t iters = (len + BLOCK - 1) / BLOCK;
        const int32_t nwords = (iters + 63) >> 6;
        bool coarse_tile = false;  // the open steps are in s_olist (else in the per-wave masks)
        if constexpr (CELLS && !(DIRECT && !SEG)) {
            // Which wave steps hold a candidate that may be in gamut.  Step s
            // = (it, wv) = it NW + wv covers evaluations 64 s .. 64 s + 63 of
            // the tile (one or two rows, several when W < 64); they form its
            // cell, and an open step sets its bit in wave wv's mask (zeroed
            // with the tile's other LDS).
            // Coarse level first: the tile's rows by 64 consecutive rays
            // (columns) are proven as a whole, one column per thread; a step
            // all of whose columns are proven out of gamut (or, without
            // n_gamut, unable to hold a high channel) needs no proof of its
            // own.  The other steps are listed and dealt out densely, one per
            // lane, so that no wave spends a round on closed steps.
            const int32_t nsteps = iters * NW;
            const int32_t ncol = (a.W + 63) >> 6;
            const bool coarse = ncol >= 2 && ncol <= kMaxCols && nsteps <= kMaxListed;
            coarse_tile = coarse;
            const bool need_ng = a.need_ng != 0;
            int32_t nlisted = nsteps;
            if (coarse) {
                const int32_t rlast = row0 + (jb0 + len - 1) / a.W;
                for (int32_t q = tid; q < ncol; q += BLOCK) {
                    bool high = true;
                    const bool out = cell_out_of_gamut(cc, a.g, ang, a.ra, a.rb, row0, rlast, 64 * q,
                                                       min(64 * q + 63, a.W - 1), &a.rule, &high);
                    s_colv[q] = out ? 1 : (high ? 0 : 2);  // 1: out of gamut, 2: no high channel
                }
                if (tid == 0) {
                    s_nlist = 0;
                    s_nopen = 0;
                }
                __syncthreads();
                for (int32_t sx = tid; sx < nsteps; sx += BLOCK) {
                    const int32_t e0 = 64 * sx;
                    if (e0 >= len) continue;
                    const int32_t e1 = min(e0 + 63, len - 1);
                    int32_t ia, ja, ib, jb;
                    divmod_small(jb0 + e0, a.W, a.inv_W, ia, ja);
                    divmod_small(jb0 + e1, a.W, a.inv_W, ib, jb);
                    // columns of the step's candidates: one row, or the end of
                    // one and the start of the next (64 rays never span more)
                    uint32_t all = 3u;  // bit 0: every column out; bit 1: every column out or no-high
                    const int32_t qa = ja >> 6, qb = (ib == ia ? jb : a.W - 1) >> 6;
                    for (int32_t q = qa; q <= qb; ++q) {
                        const uint32_t v = s_colv[q];
                        all &= (v == 1u ? 3u : (v == 2u ? 2u : 0u));
                    }
                    if (ib != ia)
                        for (int32_t q = 0; q <= (jb >> 6); ++q) {
                            const uint32_t v = s_colv[q];
                            all &= (v == 1u ? 3u : (v == 2u ? 2u : 0u));
                        }
                    if ((all & 1u) || ((all & 2u) && !need_ng)) {
                        skipped += (uint64_t)(e1 - e0 + 1);
                    } else {
                        s_list[atomicAdd(&s_nlist, 1)] = (uint16_t)sx;
                    }
                }
                __syncthreads();
                nlisted = s_nlist;
            }
            for (int32_t s0 = w * 64; s0 < nlisted; s0 += BLOCK) {
                const int32_t li = s0 + (int32_t)lane;
                const int32_t sidx = coarse ? (int32_t)s_list[min(li, nlisted - 1)] : li;
                const int32_t it = sidx / NW, wv = sidx - it * NW;
                const int32_t e0 = it * BLOCK + wv * 64;
                const bool any = li < nlisted && e0 < len;
                const int32_t e1 = min(e0 + 63, len - 1);
                bool high = true;
                const bool open = step_open(cc, a.g, ang, a.ra, a.rb, a.W, a.inv_W, row0, jb0, min(e0, len - 1),
                                            e1, any, SYM, &a.rule, &high);
                // without n_gamut, a step without a high channel needs nothing
                const bool take = open && (high || need_ng);
                if (any && !take) skipped += (uint64_t)(e1 - e0 + 1);
                if (coarse) {
                    const uint64_t tk = __ballot(take);
                    int32_t basew = 0;
                    if (lane == 0 && tk) basew = atomicAdd(&s_nopen, (int32_t)__builtin_popcountll(tk));
                    basew = __builtin_amdgcn_readlane(basew, 0);
                    if (take) s_olist[basew + (int32_t)rank_below(tk)] = (uint16_t)(sidx | ((open && high) ? 0x8000 : 0));
                } else {
                    if (take)
                        atomicOr((unsigned long long*)&s_open[wv * a.cell_words + (it >> 6)], 1ull << (it & 63));
                    if (open && high)
                        atomicOr((unsigned long long*)&s_full[wv * a.cell_words + (it >> 6)], 1ull << (it & 63));
                }
            }
            __syncthreads();
        }
        // wave totals (the same value in every lane) and the lane's best key
        uint32_t cnt = 0, ng = 0, best = 0;
        uint32_t pat[7] = {0, 0, 0, 0, 0, 0, 0};
        const bool cube = cube_branch_only(cc, (begin + len - 1) / a.W, a.ra, a.rb);
        // one wave step: evaluation e of the tile is candidate (i, j)
        auto step = [&](int32_t i, int32_t j, int32_t e, bool live) {
            double sn, co;
            ang.get(j, sn, co);
            const double rr = (double)(i + 1);
            float fp[3], fm[3];
            pair_linear_w(cc, a.g, (rr * a.ra) * sn, (rr * a.rb) * co, fp, fm, cube);
            const uint64_t live_m = __ballot(live);
            const uint64_t both_m = __ballot(in_unit_cube(fp) && in_unit_cube(fm)) & live_m;
            const uint64_t need_m = clip ? live_m : both_m;
            if (a.need_ng) ng += (uint32_t)__builtin_popcountll(both_m);
            uint64_t surv_m = 0;
            if (need_m != 0ull) {
                float Vp[3], Vm[3];
                codes_w(fp, fm, (need_m >> lane) & 1ull, clip, Vp, Vm);
                const PatMasks pm = pattern_masks(Vp, Vm, a.rule);
                surv_m = accepted_lanes(pm, a.rule.mask) & need_m;
                if (surv_m != 0ull) {
                    cnt += (uint32_t)__builtin_popcountll(surv_m);
                    count_patterns(pm, need_m, pat);
                    if ((surv_m >> lane) & 1ull) {
                        best = max(best, best_key(i, j));
                        if constexpr (TABLE) atomicMax(&s_ray[j], (uint32_t)(i + 1));
                    }
                }
            }
            if constexpr (SEG) {
                // survivors per search segment: split this pass's ballot by
                // segment (a pass of 64 evaluations touches few segments)
                if (surv_m != 0ull) {
                    const int32_t sa = SYM ? i : (begin + e) / a.seg_len;  // segment of the colour
                    const int32_t sl = sa - seg0;
                    // the write pass's pass of this evaluation within its segment
                    const int32_t kb = SYM ? (j >> 6) : ((begin + e - sa * a.seg_len) >> 6);
                    uint64_t rem = surv_m;
                    while (rem) {
                        const int32_t first = __builtin_ctzll(rem);
                        const int32_t sid = __builtin_amdgcn_readlane(sl, first);
                        const uint64_t m = __ballot(sl == sid) & rem;
                        if (a.seg_mask) {
                            // 64 consecutive evaluations meet at most two passes of a segment,
                            // and the lanes' passes rise with the lane
                            const int32_t k0 = __builtin_amdgcn_readlane(kb, first),
                                          k1 = __builtin_amdgcn_readlane(kb, 63 - __builtin_clzll(m));
                            if (lane == 0)
                                atomicOr((unsigned long long*)&s_mask[sid], (1ull << k0) | (1ull << k1));
                        }
                        if (lane == 0) atomicAdd(&s_seg[sid], (uint32_t)__builtin_popcountll(m));
                        rem &= ~m;
                    }
                }
            }
        };
        // a step proven to hold no high channel: only its in-gamut pairs are
        // counted (n_gamut); none can survive, so nothing is encoded
        [[maybe_unused]] auto gamut_step = [&](int32_t i, int32_t j, bool live) {
            double sn, co;
            ang.get(j, sn, co);
            const double rr = (double)(i + 1);
            float fp[3], fm[3];
            pair_linear_w(cc, a.g, (rr * a.ra) * sn, (rr * a.rb) * co, fp, fm, cube);
            const uint32_t nb =
                (uint32_t)__builtin_popcountll(__ballot(live && in_unit_cube(fp) && in_unit_cube(fm)));
            ng += nb;
            if (lane == 0) no_high += nb;
        };
        if constexpr (CELLS && DIRECT && !SEG) {
            // One whole colour, counts and maxima only: the band order (16
            // rows, ray by ray) gives steps of 4 rays by 16 rows, decided 64
            // at a time per wave, one per lane.  Skipped = the colour's
            // candidates less the evaluated ones (unsigned sums cancel).
            const int32_t per4 = ((a.nr + kBandRows - 1) / kBandRows) * kBandRows * a.W;  // whole bands
            const int32_t iters4 = (per4 + BLOCK - 1) / BLOCK;
            const float inv_W4 = a.inv_W / (float)kBandRows;  // exact: a power of two
            const int32_t wb = tid - (int32_t)lane;
            uint64_t evald = 0;
            // steps without a high channel hold no survivor: with summaries
            // they are counted for n_gamut, without them not evaluated at all
            const bool need_ng = a.summ != nullptr && a.need_ng != 0;
            for (int32_t word = 0; word < (iters4 + 63) >> 6; ++word) {
                const int32_t itl = word * 64 + (int32_t)lane, e0 = itl * BLOCK + wb;
                const bool any = itl < iters4 && e0 < per4;
                bool high = true;
                const bool open = band_step_open(cc, a.g, ang, a.ra, a.rb, a.W, inv_W4, min(e0, per4 - 1),
                                                 min(e0 + 63, per4 - 1), any, &a.rule, &high);
                const uint64_t full = uniform_u64(__ballot(open && high));
                uint64_t steps = need_ng ? uniform_u64(__ballot(open)) : full;
                while (steps) {
                    const int32_t bit = (int32_t)__builtin_ctzll(steps);
                    const int32_t e = (word * 64 + bit) * BLOCK + tid;
                    steps &= steps - 1ull;
                    const BandPos bp = band_pos(min(e, per4 - 1), a.W, inv_W4);
                    const int32_t i = bp.i;
                    const bool live = e < per4 && i < a.nr;
                    evald += (uint64_t)__builtin_popcountll(__ballot(live));
                    if ((full >> bit) & 1ull) step(min(i, a.nr - 1), bp.j, e, live);
                    else gamut_step(min(i, a.nr - 1), bp.j, live);
                }
            }
            if (lane == 0) skipped += (w == 0 ? (uint64_t)len : 0ull) - evald;
        } else if constexpr (CELLS) {
            const int32_t nopen = (LISTS && coarse_tile) ? s_nopen : 0;
            // the open steps dealt in turn (coarse cells), (i, j) from the step index
            for (int32_t q = w; q < nopen; q += NW) {
                const uint32_t ent = s_olist[q];
                const int32_t sidx = (int32_t)(ent & 0x7FFFu);
                const int32_t it = sidx / NW, wv = sidx - it * NW;
                const int32_t e = it * BLOCK + wv * 64 + (int32_t)lane;
                int32_t i, j;
                divmod_small(jb0 + min(e, len - 1), a.W, a.inv_W, i, j);
                if (ent & 0x8000u) step(i + row0, j, e, e < len);
                else gamut_step(i + row0, j, e < len);
            }
            // else the open steps of this wave, (i, j) from the step index
            for (int32_t word = 0; word < (coarse_tile ? 0 : nwords); ++word) {
                uint64_t steps = uniform_u64(s_open[w * a.cell_words + word]);
                const uint64_t full = uniform_u64(s_full[w * a.cell_words + word]);
                while (steps) {
                    const int32_t bit = (int32_t)__builtin_ctzll(steps);
                    const int32_t it = word * 64 + bit;
                    steps &= steps - 1ull;
                    const int32_t e = it * BLOCK + tid;
                    int32_t i, j;
                    divmod_small(jb0 + min(e, len - 1), a.W, a.inv_W, i, j);
                    if ((full >> bit) & 1ull) step(i + row0, j, e, e < len);
                    else gamut_step(i + row0, j, e < len);
                }
            }
        } else {
            // every step, (i, j) advanced by one block of evaluations per step
            int32_t i, j;
            divmod_small(jb0 + tid, a.W, a.inv_W, i, j);
            i += row0;
            for (int32_t it = 0; it < iters; ++it) {
                const int32_t e = it * BLOCK + tid;
                step(i, j, e, e < len);
                j += a.sj;
                i += a.si;
                if (j >= a.W) { j -= a.W; ++i; }
            }
        }

        // block reduction: count, n_gamut, best, 7 patterns (the accepted ones)
        uint32_t v[10] = {mult * cnt, mult * ng, wave_max_u32(best)};
#pragma unroll
        for (int q = 0; q < 7; ++q) v[3 + q] = mult * accepted_count(a.rule.mask, q, pat[q]);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 10; ++q) s_red[w][q] = v[q];
        }
        __syncthreads();
        if constexpr (TABLE) {
            if (a.rays_out) {
                uint32_t* dst = a.rays_out + c * (int64_t)a.W;
                for (int k = tid; k < a.W; k += BLOCK)
                    if (s_ray[k]) atomicMax(&dst[k], s_ray[k]);
            }
            if (tid < 36) s_bins[tid] = 0;
            __syncthreads();
            for (int k = tid; k < a.W; k += BLOCK) {
                const uint32_t r = s_ray[k];
                if (r) atomicMax(&s_bins[(k * a.bin_num) / a.bin_den], r);
            }
            __syncthreads();
            if (SYM && tid < 18) s_bins[tid + 18] = s_bins[tid];
            __syncthreads();
        }
        if (tid < 10) {
            uint32_t x = 0;
            for (int q = 0; q < NW; ++q) x = (tid == 2) ? max(x, s_red[q][tid]) : x + s_red[q][tid];
            s_red[0][tid] = x;  // column tid is touched by this thread only
        }
        __syncthreads();
        if constexpr (SEG) {
            const int32_t nseg = (len + a.seg_len - 1) / a.seg_len;
            uint32_t* dst = a.seg_cnt + c * (int64_t)a.segs_per_colour + seg0;
            for (int k = tid; k < nseg; k += BLOCK) dst[k] = mult * s_seg[k];
            if (a.seg_mask) {
                uint64_t* mdst = a.seg_mask + c * (int64_t)a.segs_per_colour + seg0;
                for (int k = tid; k < nseg; k += BLOCK) mdst[k] = s_mask[k];
            }
            if (a.scan_sums) {
                // the tile's segments meet at most two scan blocks (nseg <= 2048)
                const int64_t g0 = c * (int64_t)a.segs_per_colour + seg0;
                const int64_t q0 = g0 / kScanChunk;
                uint64_t s0 = 0, s1 = 0;
                for (int k = tid; k < nseg; k += BLOCK) {
                    const uint64_t v = (uint64_t)mult * s_seg[k];
                    if ((g0 + k) / kScanChunk == q0) s0 += v;
                    else s1 += v;
                }
                s0 = wave_sum_u64(s0);
                s1 = wave_sum_u64(s1);
                if (lane == 0) {
                    if (s0) atomicAdd((unsigned long long*)&a.scan_sums[q0], (unsigned long long)s0);
                    if (s1) atomicAdd((unsigned long long*)&a.scan_sums[q0 + 1], (unsigned long long)s1);
                }
            }
        }
        if constexpr (DIRECT) {
            if (tid == 0) {
                uint32_t pt[7];
                for (int q = 0; q < 7; ++q) pt[q] = s_red[0][3 + q];
                if (a.summ)
                    write_summary(cc, a.g, a.rule, a.tab, a.ra, a.rb, s_red[0][0], s_red[0][1],
                                  s_red[0][2], pt, a.summ + c);
                if constexpr (TABLE) {
                    if (a.table) a.table[c].count = s_red[0][0];
                }
            }
            if constexpr (TABLE) {
                if (tid < 36 && a.table) a.table[c].bin_ridx[tid] = (uint8_t)min(s_bins[tid], 255u);
            }
        } else {
            SumAcc* acc = a.acc + c;
            if (tid == 0 && s_red[0][0]) atomicAdd(&acc->count, s_red[0][0]);
            if (tid == 1 && s_red[0][1]) atomicAdd(&acc->n_gamut, s_red[0][1]);
            if (tid == 2 && s_red[0][2]) atomicMax(&acc->best_key, s_red[0][2]);
            if (tid >= 3 && tid < 10 && s_red[0][tid]) atomicAdd(&acc->pat[tid - 3], s_red[0][tid]);
            if constexpr (TABLE) {
                if (tid < 36 && s_bins[tid]) atomicMax(&acc->bins[tid], s_bins[tid]);
            }
        }
        __syncthreads();
    }
    // every thread left the loop at the same ticket, after a barrier
    if (a.stats) {
        const uint32_t lane = lane_id();
        const int w = w_s;
        const int tid = w * 64 + (int)lane;
        __shared__ uint64_t s_skip[NW], s_noh[NW];
        for (int o = 32; o > 0; o >>= 1) skipped += (uint64_t)__shfl_xor((unsigned long long)skipped, o, 64);
        if (lane == 0) {
            s_skip[w] = skipped;
            s_noh[w] = no_high;
        }
        __syncthreads();
        if (tid == 0) {
            uint64_t sum = 0, nh = 0;
            for (int q = 0; q < NW; ++q) {
                sum += s_skip[q];
                nh += s_noh[q];
            }
            if (sum) atomicAdd((unsigned long long*)&a.stats[blockIdx.x & 7u], (unsigned long long)sum);
            if (nh) atomicAdd((unsigned long long*)&a.stats[8 + (blockIdx.x & 7u)], (unsigned long long)nh);
        }
    }
}

// Accumulators -> summaries / table rows (atomic mode and the search kernel).
__global__ void k_finalize(const ColorConst* __restrict__ ccs, const SumAcc* __restrict__ acc,
                           int64_t n, Geom g, RuleDev rule, TabArgs tab, double ra, double rb,
                           cv_color_summary* summ, cv_table_row* table) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const SumAcc s = acc[c];
    if (summ) {
        const ColorConst cc = ccs[c];
        write_summary(cc, g, rule, tab, ra, rb, s.count, s.n_gamut, s.best_key, s.pat, summ + c);
    }
    if (table) {
        table[c].count = s.count;
        for (int k = 0; k < 36; ++k) table[c].bin_ridx[k] = (uint8_t)min(s.bins[k], 255u);
    }
}

// The scan's second half in one launch when the per-block sums fit one block
// (B <= kScanBlock): every block scans the sums itself and then writes the
// prefixes and offsets of its chunk as k_scan_apply does; block 0 writes the
// total; and, given acc and summ, the blocks share out the colours'
// summaries as k_finalize does.  Launched with B blocks.
__global__ __launch_bounds__(kScanBlock) void k_scan_finish(
    const uint32_t* __restrict__ cnt, int64_t T, const uint64_t* __restrict__ sums, int64_t B,
    uint64_t* __restrict__ prefix, int64_t* __restrict__ offsets, int32_t segs_per_colour, int64_t n,
    uint64_t* __restrict__ total_out, const ColorConst* __restrict__ ccs, const SumAcc* __restrict__ acc,
    Geom g, RuleDev rule, TabArgs tab, double ra, double rb, cv_color_summary* __restrict__ summ) {
    __shared__ uint64_t s_w[kScanBlock / 64];
    __shared__ uint64_t s_base;
    const uint64_t sv = (int64_t)threadIdx.x < B ? sums[threadIdx.x] : 0ull;
    uint64_t grand;
    const uint64_t sex = block_exclusive_scan(sv, s_w, grand);
    if (threadIdx.x == blockIdx.x) s_base = sex;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    uint64_t v = 0;
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < T) v += cnt[base + k];
    uint64_t total;
    uint64_t run = s_base + block_exclusive_scan(v, s_w, total);
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t t = base + k;
        if (t >= T) break;
        prefix[t] = run;
        if (offsets && t % segs_per_colour == 0) offsets[t / segs_per_colour] = (int64_t)run;
        run += cnt[t];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (offsets) offsets[n] = (int64_t)grand;
        *total_out = grand;
    }
    if (acc && summ) {
        for (int64_t c = (int64_t)blockIdx.x * kScanBlock + threadIdx.x; c < n; c += (int64_t)gridDim.x * kScanBlock) {
            const SumAcc sa = acc[c];
            write_summary(ccs[c], g, rule, tab, ra, rb, sa.count, sa.n_gamut, sa.best_key, sa.pat, summ + c);
        }
    }
}

__global__ void k_zero_u64(uint64_t* __restrict__ p, int64_t n) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; k < n; k += (int64_t)gridDim.x * blockDim.x) p[k] = 0;
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

} // namespace cvib

// ===========================================================================
// Host launchers.

namespace cvib {

namespace {

MatArgs mat_args() {
    const ColorSpace& cs = color_space();
    MatArgs m;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            m.M[3 * r + c] = cs.M[r][c];
            m.Minv[3 * r + c] = cs.Minv[r][c];
        }
    for (int k = 0; k < 3; ++k) m.W[k] = cs.W[k];
    return m;
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

int zero_u64(void* p, int64_t n, hipStream_t s) {
    if (n <= 0) return CV_OK;
    unsigned g = blocks_for(n, 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_zero_u64, dim3(g), dim3(256), 0, s, (uint64_t*)p, n);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

// Common set-up of a search: per-colour constants and the angle table.
template <typename Kern>
int persistent_grid(cv_context* ctx, Kern k, int block, size_t lds, int64_t ntiles, unsigned& grid) {
    // the angle tables (and per-ray maxima) of large grids may not fit
    hipFuncAttributes fa;
    CV_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k)));
    int lds_max = 0;
    CV_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    if (lds + fa.sharedSizeBytes > (size_t)lds_max)
        return fail(CV_EINVAL, "this grid needs " + std::to_string(lds + fa.sharedSizeBytes) +
                                   " bytes of LDS per block; the device has " + std::to_string(lds_max));
    int per_cu = 0;
    CV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, lds));
    if (per_cu < 1) per_cu = 1;
    int64_t g = (int64_t)per_cu * ctx->num_cu;
    if (g > ntiles) g = ntiles;
    grid = (unsigned)(g < 1 ? 1 : g);
    return CV_OK;
}

constexpr int kSearchBlock = kPassBlock;
constexpr int kSegLen = 512;

template <bool EMIT, bool SUMM, bool SYM, bool WRITE>
int launch_pass_t(cv_context* ctx, const SearchArgs& a, hipStream_t s) {
    auto k = k_pair_pass<EMIT, SUMM, SYM, WRITE>;
    const size_t lds = angle_lds_bytes(a.tab);
    unsigned grid;
    const int64_t blocks_needed = (a.nsegs + kPassBlock / 64 - 1) / (kPassBlock / 64);
    int rc = persistent_grid(ctx, k, kSearchBlock, lds, blocks_needed, grid);
    if (rc != CV_OK) return rc;
    hipLaunchKernelGGL(k, dim3(grid), dim3(kSearchBlock), lds, s, a);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

int launch_pass(cv_context* ctx, const SearchArgs& a, bool emit, bool summ, bool sym, bool write,
                hipStream_t s) {
    const int sel = (emit ? 8 : 0) | (summ && !write ? 4 : 0) | (sym ? 2 : 0) | (write ? 1 : 0);
    switch (sel) {
    case 0: return launch_pass_t<false, false, false, false>(ctx, a, s);
    case 1: return launch_pass_t<false, false, false, true>(ctx, a, s);
    case 2: return launch_pass_t<false, false, true, false>(ctx, a, s);
    case 3: return launch_pass_t<false, false, true, true>(ctx, a, s);
    case 4: return launch_pass_t<false, true, false, false>(ctx, a, s);
    case 6: return launch_pass_t<false, true, true, false>(ctx, a, s);
    case 8: return launch_pass_t<true, false, false, false>(ctx, a, s);
    case 9: return launch_pass_t<true, false, false, true>(ctx, a, s);
    case 10: return launch_pass_t<true, false, true, false>(ctx, a, s);
    case 11: return launch_pass_t<true, false, true, true>(ctx, a, s);
    case 12: return launch_pass_t<true, true, false, false>(ctx, a, s);
    default: return launch_pass_t<true, true, true, false>(ctx, a, s);
    }
}

// Threads per block of the reduce kernel: a tile that is one whole colour
// (direct mode, usually small) keeps 4 waves so that more tiles run per CU;
// large chunks take 8 waves to share one copy of the angle tables.
constexpr int kReduceBlock = 512;
constexpr int kReduceBlockDirect = 256;
// LDS bytes of a tile's open-step masks.
size_t cell_bytes(const ReduceArgs& a) { return 2 * (size_t)(a.block / 64) * a.cell_words * sizeof(uint64_t); }
constexpr int reduce_block(bool direct) { return direct ? kReduceBlockDirect : kReduceBlock; }

template <bool TABLE, bool DIRECT, bool SYM, bool SEG>
int launch_reduce_t(cv_context* ctx, const ReduceArgs& a_in, hipStream_t s) {
    constexpr int B = reduce_block(DIRECT);
    if (a_in.block != B) return fail(CV_ESTATE, "internal: reduce block size");
    ReduceArgs a = a_in;
    // one-colour tiles without segments take the band order, whose steps
    // cover 4 rays of 16 rows: worth cells from 32 rays per row
    if (DIRECT && !SEG && ctx->gamut_cells && !a.rule.clip && a.W >= kBandMinRays &&
        (int64_t)(a.nr + kBandRows - 1) * a.W < (1 << 24))
        a.cell_words = 1;
    auto k = a.cell_words > 0 ? k_pair_reduce<B, TABLE, DIRECT, SYM, SEG, true>
                              : k_pair_reduce<B, TABLE, DIRECT, SYM, SEG, false>;
    const size_t lds = angle_lds_bytes(a.tab) + (TABLE ? (size_t)(a.W + 1) / 2 * sizeof(double) : 0) + cell_bytes(a) +
                       (SEG && a.seg_mask ? (size_t)a.mask_slots * sizeof(uint64_t) : 0);
    unsigned grid;
    int rc = persistent_grid(ctx, k, B, lds, a.ntiles, grid);
    if (rc != CV_OK) return rc;
    hipLaunchKernelGGL(k, dim3(grid), dim3(B), lds, s, a);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

int launch_reduce(cv_context* ctx, const ReduceArgs& a, bool table, bool direct, bool sym,
                  bool seg, hipStream_t s) {
    if (seg) {  // count pass of the search (no table)
        const int sel = (direct ? 2 : 0) | (sym ? 1 : 0);
        switch (sel) {
        case 0: return launch_reduce_t<false, false, false, true>(ctx, a, s);
        case 1: return launch_reduce_t<false, false, true, true>(ctx, a, s);
        case 2: return launch_reduce_t<false, true, false, true>(ctx, a, s);
        default: return launch_reduce_t<false, true, true, true>(ctx, a, s);
        }
    }
    const int sel = (table ? 4 : 0) | (direct ? 2 : 0) | (sym ? 1 : 0);
    switch (sel) {
    case 0: return launch_reduce_t<false, false, false, false>(ctx, a, s);
    case 1: return launch_reduce_t<false, false, true, false>(ctx, a, s);
    case 2: return launch_reduce_t<false, true, false, false>(ctx, a, s);
    case 3: return launch_reduce_t<false, true, true, false>(ctx, a, s);
    case 4: return launch_reduce_t<true, false, false, false>(ctx, a, s);
    case 5: return launch_reduce_t<true, false, true, false>(ctx, a, s);
    case 6: return launch_reduce_t<true, true, false, false>(ctx, a, s);
    default: return launch_reduce_t<true, true, true, false>(ctx, a, s);
    }
}

// Tiling of the reduce-only kernel: one tile per colour when there are many
// colours of moderate size (direct mode), else chunks merged by atomics,
// about `target` tiles in all (at least 16 blocks of evaluations each; the
// autotuner's choice, kTilesDefault otherwise).  With seg_len > 0 the chunks
// start on multiples of seg_len and hold at most 2048 segments (count pass of
// the search).  Every tiling gives the same results: the merges are integer
// sums and maxima, and the survivors' order follows the segments.
struct ReducePlan {
    bool direct;
    int64_t chunk;
    int32_t tpc;
    int64_t ntiles;
};

ReducePlan plan_reduce(int64_t n, int64_t per, int32_t seg_len, int32_t target = kTilesDefault) {
    ReducePlan p;
    const int64_t max_chunk = seg_len > 0 ? (int64_t)2048 * seg_len : (int64_t)1 << 30;
    p.direct = n >= 2048 && per <= (1 << 20) && per <= max_chunk;
    if (p.direct) {
        p.chunk = per;
    } else {
        const int64_t want_tiles_per_colour = (target + n - 1) / n;
        int64_t chunk = (per + want_tiles_per_colour - 1) / want_tiles_per_colour;
        if (chunk < 16 * kReduceBlock) chunk = 16 * kReduceBlock;
        const int64_t unit = seg_len > 0 ? seg_len : kReduceBlock;
        chunk = (chunk + unit - 1) / unit * unit;
        if (chunk > max_chunk) chunk = max_chunk;
        p.chunk = chunk;
    }
    p.tpc = (int32_t)((per + p.chunk - 1) / p.chunk);
    p.ntiles = (int64_t)p.tpc * n;
    return p;
}

// Key of a call shape for the tiling tuner: count pass or reduce, colours,
// grid size (FNV-1a over the values).
uint64_t tiles_key_of(int search, int64_t n, const GridDev& gd) {
    const int64_t v[5] = {search, n, gd.nr, gd.ntheta, gd.N};
    uint64_t h = 1469598103934665603ull;
    for (int64_t x : v)
        for (int b = 0; b < 8; ++b) {
            h ^= (uint64_t)((x >> (8 * b)) & 0xFF);
            h *= 1099511628211ull;
        }
    return h;
}

int32_t tiles_target_of(cv_context* ctx, uint64_t key) {
    if (ctx->tiles_forced > 0) return ctx->tiles_forced;
    const auto it = ctx->tiles_tuned.find(key);
    return it == ctx->tiles_tuned.end() ? kTilesDefault : it->second;
}

// Time fn(target) for every tiling choice (one untimed run each first) and
// keep the fastest for `key`; the last run leaves the call's outputs in
// place (every tiling writes the same).  Timing events of the context are off
// meanwhile.
template <class F>
int tune_tiles(cv_context* ctx, uint64_t key, hipStream_t s, F fn) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CV_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    const bool timing = ctx->timing;
    ctx->timing = false;
    int rc = CV_OK;
    int32_t best = kTilesDefault;
    float best_ms = 0.0f;
    bool have = false;
    for (int32_t t : kTileTargets) {
        if ((rc = fn(t)) != CV_OK) break;
        float ms = 0.0f;
        if ((he = hipEventRecord(e0, s)) == hipSuccess && (rc = fn(t)) == CV_OK &&
            (he = hipEventRecord(e1, s)) == hipSuccess && (he = hipEventSynchronize(e1)) == hipSuccess)
            he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess && rc == CV_OK) rc = hip_fail(he, "timing a tiling");
        if (rc != CV_OK) break;
        if (!have || ms < best_ms) {
            best_ms = ms;
            best = t;
            have = true;
        }
    }
    ctx->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != CV_OK) return rc;
    ctx->tiles_tuned[key] = best;
    return ctx->save_tuning();
}

ReduceArgs reduce_args(cv_context* ctx, const TabArgs& tab, const GridDev& gd, const RuleDev& rd,
                       int32_t W, const ReducePlan& pl, int64_t n) {
    ReduceArgs a;
    a.cc = (const ColorConst*)ctx->colors.ptr;
    a.tab = tab;
    a.g = geom_constants();
    a.rule = rd;
    a.ra = gd.ra;
    a.rb = gd.rb;
    a.nr = gd.nr;
    a.ntheta = gd.ntheta;
    a.W = W;
    a.inv_W = 1.0f / (float)W;
    const int B = reduce_block(pl.direct);
    a.si = B / W;
    a.sj = B % W;
    a.block = B;
    a.chunk = (int32_t)pl.chunk;
    a.tiles_per_colour = pl.tpc;
    a.bin_num = 36;
    a.bin_den = gd.N;
    a.n = n;
    a.ntiles = pl.ntiles;
    a.acc = pl.direct ? nullptr : (SumAcc*)ctx->acc.ptr;
    a.summ = nullptr;
    a.table = nullptr;
    a.misc = (uint64_t*)ctx->misc.ptr;
    a.rays_out = nullptr;
    a.seg_cnt = nullptr;
    a.seg_len = 0;
    a.segs_per_colour = 0;
    // one open-step bit per wave step of a tile.  Under the clip reading every
    // candidate counts, so there are no cells; with fewer than 128 evaluated
    // rays per row a step spans more than half of them and the proof rarely
    // holds (measured: the 90-ray whole-cube table loses 6% with cells)
    a.cell_words = ctx->gamut_cells && !rd.clip && W >= kCellMinRays
                       ? (int32_t)(((pl.chunk + B - 1) / B + 63) / 64)
                       : 0;
    a.need_ng = 1;
    a.stats = ctx->timing ? (uint64_t*)ctx->stats.ptr : nullptr;
    a.seg_mask = nullptr;
    a.mask_slots = 0;
    a._pad2 = 0;
    a.scan_sums = nullptr;
    return a;
}

} // namespace

// Per-colour constants and the angle table of a call, written to the given
// device arrays (colors: ColorConst [n]; table: tab_len doubles).
static int prepare_colours_at(ColorConst* colors, double* table, const uint8_t* rgb, int64_t n,
                              const GridDev& gd, hipStream_t s, TabArgs& tab) {
    hipLaunchKernelGGL(k_angle_table, dim3(blocks_for(gd.N / 2 + 1, 256)), dim3(256), 0, s, table,
                       gd.N);
    CV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_color_prologue, dim3(blocks_for(n, 256)), dim3(256), 0, s, rgb, colors, n,
                       mat_args());
    CV_HIP(hipGetLastError());
    tab.tab = table;
    tab.tab_len = gd.tab_len;
    tab.N = gd.N;
    // room for the per-ray maxima of the angle-bin table as well
    tab.dW = direct_rays(gd.ntheta, gd.N, gd.tab_len, (size_t)gd.ntheta * 4);
    tab._pad = 0;
    return CV_OK;
}

// The same in the context's workspace (shared with the multi-rule pass).
int prepare_colours(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd, hipStream_t s,
            TabArgs& tab) {
    int rc;
    if ((rc = ctx->ensure(ctx->colors, (size_t)n * sizeof(ColorConst))) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->table, (size_t)gd.tab_len * sizeof(double))) != CV_OK) return rc;
    return prepare_colours_at((ColorConst*)ctx->colors.ptr, (double*)ctx->table.ptr, rgb, n, gd, s,
                              tab);
}

int launch_angle_table(double* tab, int32_t N, hipStream_t s) {
    hipLaunchKernelGGL(k_angle_table, dim3(blocks_for(N / 2 + 1, 256)), dim3(256), 0, s, tab, N);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

// Exclusive scan of per-unit counts into 64-bit offsets (unit order); the
// total goes to *total (device) and, if offsets is given, every spc-th unit's
// offset to offsets[unit / spc] and the total to offsets[n].
int run_scan_counts(cv_context* ctx, const uint32_t* cnt, int64_t T, uint64_t* prefix,
                    int64_t* offsets, int32_t spc, int64_t n, uint64_t* total, hipStream_t s) {
    const int64_t nsums = (T + kScanChunk - 1) / kScanChunk;
    int rc;
    if ((rc = ctx->ensure(ctx->scan, (size_t)(nsums > 0 ? nsums : 1) * 8)) != CV_OK) return rc;
    uint64_t* sums = (uint64_t*)ctx->scan.ptr;
    if (nsums > 0)
        hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nsums), dim3(kScanBlock), 0, s, cnt, T, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, s, sums, nsums, total);
    if (nsums > 0)
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nsums), dim3(kScanBlock), 0, s, cnt, T, sums,
                           prefix, offsets, spc, n, (const uint64_t*)total);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

int run_lab_convert(cv_context* ctx, const void* in, void* out, int64_t n, int dir,
                    hipStream_t s) {
    (void)ctx;
    if (n == 0) return CV_OK;
    if (dir == CV_RGB8_TO_LAB) {
        hipLaunchKernelGGL(k_rgb8_to_lab, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           (const uint8_t*)in, (float*)out, n, mat_args());
    } else {
        hipLaunchKernelGGL(k_lab_to_rgbf, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           (const float*)in, (float*)out, n, geom_constants(), mat_args());
    }
    CV_HIP(hipGetLastError());
    return CV_OK;
}

namespace {

// The search with CV_PER_RAY: per-ray maxima from the reduce kernel (its
// angle-bin path keeps them in LDS and merges them per colour), then flags in
// (colour, ray) order, a scan, and the records of the flagged rays evaluated
// again.
int run_pair_search_per_ray(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd,
                            const RuleDev& rd, cv_pair* out, int64_t capacity, int64_t* offsets,
                            cv_color_summary* summ, int64_t* total_host, hipStream_t s) {
    int rc;
    TabArgs tab;
    if ((rc = prepare_colours(ctx, rgb, n, gd, s, tab)) != CV_OK) return rc;
    const bool sym = gd.ntheta == gd.N;
    const int32_t W = sym ? gd.N / 2 : gd.ntheta;
    const int64_t per = (int64_t)gd.nr * W;
    const ReducePlan pl = plan_reduce(n, per, 0);
    const int64_t nrays = n * (int64_t)gd.ntheta;
    if ((rc = ctx->ensure(ctx->misc, 64)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->acc, (size_t)n * sizeof(SumAcc))) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->rays, (size_t)(n * W + 1) * 4)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->seg_cnt, (size_t)nrays * 4)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->seg_prefix, (size_t)nrays * 8)) != CV_OK) return rc;
    if ((rc = zero_u64(ctx->misc.ptr, 8, s)) != CV_OK) return rc;
    if ((rc = zero_u64(ctx->rays.ptr, (n * W + 1) / 2, s)) != CV_OK) return rc;
    if (!pl.direct && (rc = zero_u64(ctx->acc.ptr, n * (int64_t)(sizeof(SumAcc) / 8), s)) != CV_OK) return rc;
    ReduceArgs a = reduce_args(ctx, tab, gd, rd, W, pl, n);
    a.summ = summ;
    a.table = nullptr;
    a.rays_out = (uint32_t*)ctx->rays.ptr;
    if ((rc = ctx->mark(CV_TIME_CALL, 0, s)) != CV_OK) return rc;
    if ((rc = ctx->mark(CV_TIME_EVAL, 0, s)) != CV_OK) return rc;
    if ((rc = launch_reduce(ctx, a, true, pl.direct, sym, false, s)) != CV_OK) return rc;
    if ((rc = ctx->mark(CV_TIME_EVAL, 1, s)) != CV_OK) return rc;
    if (!pl.direct && summ) {
        hipLaunchKernelGGL(k_finalize, dim3(blocks_for(n, 128)), dim3(128), 0, s, a.cc,
                           (const SumAcc*)ctx->acc.ptr, n, a.g, rd, tab, gd.ra, gd.rb, summ,
                           (cv_table_row*)nullptr);
    }
    hipLaunchKernelGGL(k_ray_flags, dim3(blocks_for(nrays, 256)), dim3(256), 0, s,
                       (const uint32_t*)ctx->rays.ptr, n, W, gd.ntheta, (uint32_t*)ctx->seg_cnt.ptr);
    CV_HIP(hipGetLastError());
    uint64_t* misc = (uint64_t*)ctx->misc.ptr;
    if ((rc = run_scan_counts(ctx, (const uint32_t*)ctx->seg_cnt.ptr, nrays, (uint64_t*)ctx->seg_prefix.ptr,
                              offsets, gd.ntheta, n, misc + 2, s)) != CV_OK)
        return rc;
    if (out && capacity > 0) {
        hipLaunchKernelGGL(k_ray_records, dim3(blocks_for(nrays, 256)), dim3(256), 0, s,
                           (const uint32_t*)ctx->rays.ptr, (const uint64_t*)ctx->seg_prefix.ptr, n, W,
                           gd.ntheta, (const ColorConst*)ctx->colors.ptr, a.g, rd, tab, gd.ra, gd.rb,
                           (uint4*)out, (uint64_t)capacity);
        CV_HIP(hipGetLastError());
    }
    if ((rc = ctx->mark(CV_TIME_CALL, 1, s)) != CV_OK) return rc;
    if (!total_host) return ctx->collect();  // no readback: offsets[n] holds the total
    CV_HIP(hipMemcpyAsync(ctx->host_misc, ctx->misc.ptr, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    CV_HIP(hipStreamSynchronize(s));
    if ((rc = ctx->collect()) != CV_OK) return rc;
    *total_host = (int64_t)ctx->host_misc[2];
    if (*total_host > capacity)
        return fail(CV_ECAPACITY, "per-ray total " + std::to_string(*total_host) + " exceeds capacity " +
                                      std::to_string(capacity));
    return CV_OK;
}

} // namespace

int run_pair_csr_summary(cv_context* ctx, const cv_pair* recs, const int64_t* offsets, int64_t n,
                         cv_color_summary* summ, hipStream_t s) {
    (void)ctx;
    if (n == 0) return CV_OK;
    hipLaunchKernelGGL(k_csr_summary, dim3((unsigned)std::min<int64_t>(n, 65536)), dim3(256), 0, s,
                       (const uint4*)recs, offsets, n, summ);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

namespace {

// Segments of a search: one per row in half-turn mode, else 512 evaluations.
struct SearchShape {
    bool sym;
    int32_t W, seg_len, spc;
    int64_t per, nsegs;
};

SearchShape search_shape(int64_t n, const GridDev& gd) {
    SearchShape h;
    h.sym = gd.ntheta == gd.N;
    h.W = h.sym ? gd.N / 2 : gd.ntheta;
    h.seg_len = h.sym ? h.W : kSegLen;
    h.per = (int64_t)gd.nr * h.W;
    h.spc = (int32_t)((h.per + h.seg_len - 1) / h.seg_len);
    h.nsegs = (int64_t)h.spc * n;
    return h;
}

// Every workspace a search call uses, at its full size, before anything is
// enqueued (so that nothing allocates under graph capture).
int size_search(cv_context* ctx, int64_t n, const GridDev& gd) {
    const SearchShape h = search_shape(n, gd);
    const int64_t nsums = (h.nsegs + kScanChunk - 1) / kScanChunk;
    int rc;
    if ((rc = ctx->ensure(ctx->colors, (size_t)n * sizeof(ColorConst))) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->table, (size_t)gd.tab_len * sizeof(double))) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->seg_cnt, (size_t)h.nsegs * 4)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->seg_prefix, (size_t)h.nsegs * 8)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->seg_mask, (size_t)h.nsegs * 8)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->misc, 64)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->acc, (size_t)n * sizeof(SumAcc))) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->scan, (size_t)(nsums > 0 ? nsums : 1) * 8)) != CV_OK) return rc;
    return CV_OK;
}

// The kernels of a search call, in order, on stream s: colour constants and
// angle table, count pass, scan, write pass, summaries.  The survivor total
// ends in misc[2].
int enqueue_search(cv_context* ctx, const SearchCall& c, hipStream_t s) {
    const uint8_t* rgb = c.rgb;
    const int64_t n = c.n;
    const GridDev& gd = c.gd;
    const RuleDev& rd = c.rd;
    cv_pair* out = c.out;
    const int64_t capacity = c.capacity;
    int64_t* offsets = c.offsets;
    cv_color_summary* summ = c.summ;
    const uint32_t flags = c.flags;
    int rc;
    // half-turn mode when the grid spans the full turn: one row per segment
    const SearchShape h = search_shape(n, gd);
    const bool sym = h.sym;
    const int32_t W = h.W, seg_len = h.seg_len, spc = h.spc;
    const int64_t per = h.per, nsegs = h.nsegs;
    const bool emit = (flags & CV_EMIT_ALL) != 0;
    const ReducePlan pl = plan_reduce(n, per, seg_len, c.tiles);
    // colour constants, angle table, ticket and totals, accumulators: one launch
    TabArgs tab;
    tab.tab = (const double*)ctx->table.ptr;
    tab.tab_len = gd.tab_len;
    tab.N = gd.N;
    tab.dW = direct_rays(gd.ntheta, gd.N, gd.tab_len, (size_t)gd.ntheta * 4);
    tab._pad = 0;
    // with few scan blocks, the count pass adds up the scan's block sums and
    // one launch does the rest of the scan and the accumulators' summaries
    const int64_t nsums = (nsegs + kScanChunk - 1) / kScanChunk;
    const bool fin_acc = summ && !emit && !pl.direct;  // summaries from the accumulators
    const bool fused = !emit && nsums >= 1 && nsums <= kScanBlock && (!fin_acc || n <= ((int64_t)1 << 16));
    {
        const int64_t nacc = (emit || !pl.direct) ? n * (int64_t)(sizeof(SumAcc) / 8) : 0;
        const int64_t nz = fused ? nsums : 0;
        const int64_t threads =
            std::max<int64_t>(std::max<int64_t>(n, gd.N / 2 + 1), std::max<int64_t>(std::max<int64_t>(8, nacc), nz));
        hipLaunchKernelGGL(k_search_prologue, dim3(blocks_for(threads, 256)), dim3(256), 0, s, rgb,
                           (ColorConst*)ctx->colors.ptr, n, mat_args(), (double*)ctx->table.ptr, gd.N,
                           (uint64_t*)ctx->misc.ptr, (int64_t)8, (uint64_t*)ctx->acc.ptr, nacc,
                           (uint64_t*)ctx->scan.ptr, nz);
        CV_HIP(hipGetLastError());
    }

    SearchArgs a;
    a.cc = (const ColorConst*)ctx->colors.ptr;
    a.tab = tab;
    a.g = geom_constants();
    a.rule = rd;
    a.ra = gd.ra;
    a.rb = gd.rb;
    a.nr = gd.nr;
    a.ntheta = gd.ntheta;
    a.W = W;
    a.inv_W = 1.0f / (float)W;
    a.seg_len = seg_len;
    a.segs_per_colour = spc;
    a.n = n;
    a.nsegs = nsegs;
    a.seg_cnt = (uint32_t*)ctx->seg_cnt.ptr;
    a.seg_prefix = (const uint64_t*)ctx->seg_prefix.ptr;
    a.out = (uint4*)out;
    a.capacity = out ? (uint64_t)capacity : 0ull;
    a.acc = nullptr;
    a.misc = (uint64_t*)ctx->misc.ptr;
    a.cells = ctx->gamut_cells && !rd.clip && !emit ? 1 : 0;
    a._pad = 0;
    a.seg_mask = emit ? nullptr : (const uint64_t*)ctx->seg_mask.ptr;

    // Count pass: survivors per segment.  The reduce-only kernel does it
    // (with the summaries); in emit-all mode every candidate is a record and
    // the search kernel counts them itself.
    ReduceArgs ra = reduce_args(ctx, tab, gd, rd, W, pl, n);
    ra.summ = emit ? nullptr : summ;
    ra.need_ng = (flags & CV_NO_NGAMUT) ? 0 : 1;
    ra.seg_cnt = a.seg_cnt;
    ra.seg_len = seg_len;
    ra.segs_per_colour = spc;
    ra.seg_mask = (uint64_t*)ctx->seg_mask.ptr;
    ra.mask_slots = (int32_t)((pl.chunk + seg_len - 1) / seg_len);
    ra.scan_sums = fused ? (uint64_t*)ctx->scan.ptr : nullptr;
    if ((rc = ctx->mark(CV_TIME_CALL, 0, s)) != CV_OK) return rc;
    if ((rc = ctx->mark(CV_TIME_EVAL, 0, s)) != CV_OK) return rc;
    if (emit) {
        if ((rc = launch_pass(ctx, a, true, false, sym, false, s)) != CV_OK) return rc;
    } else {
        if ((rc = launch_reduce(ctx, ra, false, pl.direct, sym, true, s)) != CV_OK) return rc;
    }
    if ((rc = ctx->mark(CV_TIME_EVAL, 1, s)) != CV_OK) return rc;
    // segment counts -> output offsets
    uint64_t* misc = (uint64_t*)ctx->misc.ptr;
    if (fused) {
        uint64_t* sums = (uint64_t*)ctx->scan.ptr;
        hipLaunchKernelGGL(k_scan_finish, dim3((unsigned)nsums), dim3(kScanBlock), 0, s, a.seg_cnt, nsegs,
                           (const uint64_t*)sums, nsums, (uint64_t*)ctx->seg_prefix.ptr, offsets, spc, n, misc + 2,
                           a.cc, fin_acc ? (const SumAcc*)ctx->acc.ptr : (const SumAcc*)nullptr, a.g, rd, tab,
                           gd.ra, gd.rb, fin_acc ? summ : (cv_color_summary*)nullptr);
        CV_HIP(hipGetLastError());
    } else if ((rc = run_scan_counts(ctx, a.seg_cnt, nsegs, (uint64_t*)ctx->seg_prefix.ptr, offsets, spc,
                                     n, misc + 2, s)) != CV_OK) {
        return rc;
    }
    // write pass
    if (a.capacity > 0) {
        if ((rc = ctx->mark(CV_TIME_WRITE, 0, s)) != CV_OK) return rc;
        if ((rc = launch_pass(ctx, a, emit, false, sym, true, s)) != CV_OK) return rc;
        if ((rc = ctx->mark(CV_TIME_WRITE, 1, s)) != CV_OK) return rc;
    }
    if ((rc = ctx->mark(CV_TIME_CALL, 1, s)) != CV_OK) return rc;
    if (summ) {
        if (emit) {  // summaries of an emit-all call come from a reduce pass
            ReducePlan pa = plan_reduce(n, per, 0);
            pa.direct = false;
            ReduceArgs rb = reduce_args(ctx, tab, gd, rd, W, pa, n);
            rb.misc = misc + 4;  // a ticket of its own
            if ((rc = zero_u64(rb.misc, 1, s)) != CV_OK) return rc;
            if ((rc = launch_reduce(ctx, rb, false, false, sym, false, s)) != CV_OK) return rc;
        }
        if ((emit || !pl.direct) && !(fused && fin_acc)) {
            hipLaunchKernelGGL(k_finalize, dim3(blocks_for(n, 128)), dim3(128), 0, s, a.cc,
                               (const SumAcc*)ctx->acc.ptr, n, a.g, rd, tab, gd.ra, gd.rb, summ,
                               (cv_table_row*)nullptr);
            CV_HIP(hipGetLastError());
        }
    }
    return CV_OK;
}

} // namespace

bool SearchCall::same(const SearchCall& o) const { return std::memcmp(this, &o, sizeof(SearchCall)) == 0; }

int run_pair_search(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd,
                    const RuleDev& rd, cv_pair* out, int64_t capacity, int64_t* offsets,
                    cv_color_summary* summ, int64_t* total_host, uint32_t flags,
                    hipStream_t s) {
    int rc;
    if (n > 0 && (flags & CV_PER_RAY))
        return run_pair_search_per_ray(ctx, rgb, n, gd, rd, out, capacity, offsets, summ, total_host, s);
    if (n == 0) {
        if (offsets) hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, offsets, (int64_t)0);
        CV_HIP(hipGetLastError());
        if (total_host) *total_host = 0;
        return CV_OK;
    }
    if ((rc = size_search(ctx, n, gd)) != CV_OK) return rc;
    SearchCall call;
    std::memset(&call, 0, sizeof call);  // bytewise comparison for the graph cache
    call.rgb = rgb;
    call.n = n;
    call.gd = gd;
    call.rd = rd;
    call.out = out;
    call.capacity = capacity;
    call.offsets = offsets;
    call.summ = summ;
    const cvib::Buffer* ws[9] = {&ctx->colors, &ctx->table, &ctx->seg_cnt, &ctx->seg_prefix, &ctx->misc,
                                 &ctx->acc,    &ctx->scan,  &ctx->stats,   &ctx->seg_mask};
    for (int k = 0; k < 9; ++k) call.ws[k] = ws[k]->ptr;
    call.flags = flags & (uint32_t)(CV_EMIT_ALL | CV_NO_NGAMUT);
    call.cells = ctx->gamut_cells ? 1 : 0;
    // the count pass's tiling: tuned on the first eager call of a shape
    const uint64_t tkey = tiles_key_of(1, n, gd);
    {
        const SearchShape h = search_shape(n, gd);
        if (ctx->autotune && ctx->tiles_forced == 0 && !ctx->tiles_tuned.count(tkey) && !(flags & CV_GRAPH) &&
            !plan_reduce(n, h.per, h.seg_len).direct) {
            SearchCall tc = call;
            if ((rc = tune_tiles(ctx, tkey, s, [&](int32_t t) {
                     tc.tiles = t;
                     return enqueue_search(ctx, tc, s);
                 })) != CV_OK)
                return rc;
        }
    }
    call.tiles = tiles_target_of(ctx, tkey);
    if (!(flags & CV_GRAPH)) {
        if ((rc = enqueue_search(ctx, call, s)) != CV_OK) return rc;
    } else {
        if (!ctx->sgraph_exec || !ctx->sgraph_call.same(call)) {
            if (ctx->sgraph_exec) {
                CV_HIP(hipGraphExecDestroy(ctx->sgraph_exec));
                ctx->sgraph_exec = nullptr;
            }
            if (!ctx->cap_stream) CV_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
            const bool timing = ctx->timing;
            ctx->timing = false;  // no timing events inside a captured graph
            hipGraph_t g = nullptr;
            CV_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            rc = enqueue_search(ctx, call, ctx->cap_stream);
            hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
            ctx->timing = timing;
            if (rc != CV_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&ctx->sgraph_exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                ctx->sgraph_exec = nullptr;
                return hip_fail(e, "hipGraphInstantiate");
            }
            ctx->sgraph_call = call;
        }
        if ((rc = ctx->mark(CV_TIME_CALL, 0, s)) != CV_OK) return rc;
        CV_HIP(hipGraphLaunch(ctx->sgraph_exec, s));
        if ((rc = ctx->mark(CV_TIME_CALL, 1, s)) != CV_OK) return rc;
    }
    if (!total_host) return ctx->collect();  // no readback: offsets[n] holds the total
    CV_HIP(hipMemcpyAsync(ctx->host_misc, ctx->misc.ptr, 3 * sizeof(uint64_t),
                          hipMemcpyDeviceToHost, s));
    CV_HIP(hipStreamSynchronize(s));
    if ((rc = ctx->collect()) != CV_OK) return rc;
    *total_host = (int64_t)ctx->host_misc[2];
    if (*total_host > capacity)
        return fail(CV_ECAPACITY, "survivor total " + std::to_string(*total_host) +
                                      " exceeds capacity " + std::to_string(capacity));
    return CV_OK;
}

// Device arrays one reduce call works in.
struct ReduceWs {
    ColorConst* colors;  // [n]
    double* table;       // folded angle table
    uint64_t* misc;      // 8 words, zeroed by the call
    SumAcc* acc;         // [n] in atomic mode, zeroed by the call; unused in direct mode
};

static int reduce_in(cv_context* ctx, const ReduceWs& ws, bool timed, const uint8_t* rgb, int64_t n,
                     const GridDev& gd, const RuleDev& rd, cv_color_summary* summ,
                     cv_table_row* table, int32_t tiles, hipStream_t s) {
    int rc;
    TabArgs tab;
    if ((rc = prepare_colours_at(ws.colors, ws.table, rgb, n, gd, s, tab)) != CV_OK) return rc;
    const bool sym = gd.ntheta == gd.N;
    const int32_t W = sym ? gd.N / 2 : gd.ntheta;
    const int64_t per = (int64_t)gd.nr * W;  // evaluations per colour
    const ReducePlan pl = plan_reduce(n, per, 0, tiles);
    if ((rc = zero_u64(ws.misc, 8, s)) != CV_OK) return rc;
    if (!pl.direct && (rc = zero_u64(ws.acc, n * (int64_t)(sizeof(SumAcc) / 8), s)) != CV_OK)
        return rc;
    ReduceArgs a = reduce_args(ctx, tab, gd, rd, W, pl, n);
    a.cc = ws.colors;
    a.misc = ws.misc;
    a.acc = pl.direct ? nullptr : ws.acc;
    if (!timed) a.stats = nullptr;
    a.summ = summ;
    a.table = table;
    if (timed && (rc = ctx->mark(CV_TIME_CALL, 0, s)) != CV_OK) return rc;
    if (timed && (rc = ctx->mark(CV_TIME_EVAL, 0, s)) != CV_OK) return rc;
    if ((rc = launch_reduce(ctx, a, table != nullptr, pl.direct, sym, false, s)) != CV_OK) return rc;
    if (timed && (rc = ctx->mark(CV_TIME_EVAL, 1, s)) != CV_OK) return rc;
    if (!pl.direct) {
        hipLaunchKernelGGL(k_finalize, dim3(blocks_for(n, 128)), dim3(128), 0, s, a.cc,
                           (const SumAcc*)ws.acc, n, a.g, rd, tab, gd.ra, gd.rb, summ, table);
        CV_HIP(hipGetLastError());
    }
    if (timed && (rc = ctx->mark(CV_TIME_CALL, 1, s)) != CV_OK) return rc;
    if (timed && ctx->timing && (rc = ctx->collect()) != CV_OK) return rc;
    return CV_OK;
}

int run_pair_reduce(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd,
                    const RuleDev& rd, cv_color_summary* summ, cv_table_row* table,
                    hipStream_t s) {
    if (n == 0) return CV_OK;
    int rc;
    if ((rc = ctx->ensure(ctx->colors, (size_t)n * sizeof(ColorConst))) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->table, (size_t)gd.tab_len * sizeof(double))) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->misc, 64)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->acc, (size_t)n * sizeof(SumAcc))) != CV_OK) return rc;
    const ReduceWs ws{(ColorConst*)ctx->colors.ptr, (double*)ctx->table.ptr, (uint64_t*)ctx->misc.ptr,
                      (SumAcc*)ctx->acc.ptr};
    // chunked tilings are tuned on the first call of a shape
    const uint64_t tkey = tiles_key_of(0, n, gd);
    const int64_t per = (int64_t)gd.nr * (gd.ntheta == gd.N ? gd.N / 2 : gd.ntheta);
    if (ctx->autotune && ctx->tiles_forced == 0 && !ctx->tiles_tuned.count(tkey) && !plan_reduce(n, per, 0).direct &&
        (rc = tune_tiles(ctx, tkey, s, [&](int32_t t) {
             return reduce_in(ctx, ws, false, rgb, n, gd, rd, summ, table, t, s);
         })) != CV_OK)
        return rc;
    return reduce_in(ctx, ws, true, rgb, n, gd, rd, summ, table, tiles_target_of(ctx, tkey), s);
}

// ---------------------------------------------------------------------------
// The reduce without allocation: its workspace is this file-scope array, one
// copy per device, whose device address is looked up once per device when a
// context is created.  Host code uses only that address, never the array's
// name (in host code the name is a host-side stand-in).

__device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

int scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(CV_EINVAL, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return CV_OK;
    void* p = nullptr;
    CV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(CV_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch[device] = p;
    return CV_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t reduce_scratch_bytes(int64_t n, const GridDev& gd) {
    const bool sym = gd.ntheta == gd.N;
    const int64_t per = (int64_t)gd.nr * (sym ? gd.N / 2 : gd.ntheta);
    const ReducePlan pl = plan_reduce(n, per, 0);
    return align256(8 * sizeof(uint64_t)) + align256((size_t)gd.tab_len * sizeof(double)) +
           align256((size_t)n * sizeof(ColorConst)) + (pl.direct ? 0 : (size_t)n * sizeof(SumAcc));
}

int run_pair_reduce_noalloc(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd,
                            const RuleDev& rd, cv_color_summary* summ, cv_table_row* table,
                            hipStream_t s) {
    if (n == 0) return CV_OK;
    const size_t need = reduce_scratch_bytes(n, gd);
    if (need > kScratchBytes)
        return fail(CV_ECAPACITY, "this call needs " + std::to_string(need) +
                                      " bytes of scratch; the no-allocation reduce holds " +
                                      std::to_string(kScratchBytes));
    uint8_t* base;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = (uint8_t*)g_scratch[ctx->device];
    }
    if (!base) return fail(CV_ESTATE, "scratch address of this device not set up");
    size_t o = 0;
    ReduceWs ws;
    ws.misc = (uint64_t*)(base + o);
    o += align256(8 * sizeof(uint64_t));
    ws.table = (double*)(base + o);
    o += align256((size_t)gd.tab_len * sizeof(double));
    ws.colors = (ColorConst*)(base + o);
    o += align256((size_t)n * sizeof(ColorConst));
    ws.acc = (SumAcc*)(base + o);
    return reduce_in(ctx, ws, false, rgb, n, gd, rd, summ, table, tiles_target_of(ctx, tiles_key_of(0, n, gd)), s);
}

} // namespace cvib

namespace cvib {
uint64_t tiles_key(int search, int64_t n, const GridDev& gd) { return tiles_key_of(search, n, gd); }
int32_t tiles_target(cv_context* ctx, uint64_t key) { return tiles_target_of(ctx, key); }
} // namespace cvib
