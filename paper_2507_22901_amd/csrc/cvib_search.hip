// Colour conversion, the fused generate -> convert -> predicate search with
// single-pass stream compaction, and the reduce-only search (gfx950).
//
// Paper map: Section 2 (target split into L*, a*, b*; displacement arrays
// D_a = r sin(theta), D_b = r cos(theta) added to and subtracted from a*, b*
// with L* fixed; the pairs meeting both conditions are picked out of the
// candidate array) and Section 3 / Table 1 (a channel bit is 1 when its
// change is above V_th and 0 when it is under V_th * R_novib).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "cvib_internal.h"

namespace cvib {

// ---------------------------------------------------------------------------
// Small wave-level helpers (wave64).

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// A value known to be equal in every lane, moved to a scalar register.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
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
__global__ void k_color_prologue(const uint8_t* __restrict__ rgb, ColorConst* __restrict__ cc,
                                 int64_t n, MatArgs m) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double lab[3];
    rgb8_lab(m, rgb + 3 * k, lab);
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
    cc[k] = c;
}

// ---------------------------------------------------------------------------
// Angle table.  theta_j = 360 j / N degrees.  sin(2 pi m / N) is evaluated
// after folding m with exact integer steps: the half-turn fold makes
// tab[j + N/2] = -tab[j] bitwise (so the + and - colours of ray j are the -
// and + colours of ray j + N/2), the pi - x fold keeps the argument within a
// quarter turn, and when 8 | N the octant fold keeps it within 45 degrees.

__device__ double sin_turn(int64_t m, int64_t N) {
    m %= N;
    if (m < 0) m += N;
    double sgn = 1.0;
    if (2 * m >= N) { m -= N / 2; sgn = -1.0; }
    if (4 * m > N) m = N / 2 - m;
    if (N % 8 == 0 && 8 * m > N) return sgn * cos((double)(N / 4 - m) * (2.0 * M_PI / (double)N));
    return sgn * sin((double)m * (2.0 * M_PI / (double)N));
}

__device__ double cos_turn(int64_t m, int64_t N) {
    m %= N;
    if (m < 0) m += N;
    double sgn = 1.0;
    if (2 * m >= N) { m -= N / 2; sgn = -sgn; }
    if (4 * m > N) { m = N / 2 - m; sgn = -sgn; }
    if (N % 8 == 0 && 8 * m > N) return sgn * sin((double)(N / 4 - m) * (2.0 * M_PI / (double)N));
    return sgn * cos((double)m * (2.0 * M_PI / (double)N));
}

// tab[0, N) = sin; when 4 does not divide N, tab[N, 2N) = cos.  Otherwise
// cos(theta_j) is read as tab[(j + N/4) mod N].
__global__ void k_angle_table(double* __restrict__ tab, int32_t N, int32_t with_cos) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    tab[k] = sin_turn(k, N);
    if (with_cos) tab[N + k] = cos_turn(k, N);
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
    int32_t tab_len;       // doubles in the table
    int32_t qoff, wrap, N; // cos(theta_j) = tab[j + qoff - (j + qoff >= wrap ? N : 0)]
};

template <bool LDS>
__device__ __forceinline__ void sincos_j(const double* tab, const TabArgs& t, int32_t j, double& s,
                                         double& c) {
    int32_t jc = j + t.qoff;
    jc -= (jc >= t.wrap) ? t.N : 0;
    s = tab[j];
    c = tab[jc];
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

struct SearchArgs {
    const ColorConst* cc;
    TabArgs tab;
    Geom g;
    RuleDev rule;
    double ra, rb;        // dr / 500, dr / 200
    int32_t nr, ntheta;
    float inv_ntheta;
    int32_t si, sj;       // block stride = si * ntheta + sj candidates
    int32_t tiles_per_colour;
    int64_t n, ntiles;
    cv_pair* out;
    int64_t capacity;
    int64_t* offsets;     // nullable
    uint64_t* status;     // look-back words [ntiles]
    SumAcc* acc;          // nullable
    uint64_t* misc;       // [0] ticket, [1] total, [2] error bits
};

constexpr uint64_t kStAgg = 1ull << 62;
constexpr uint64_t kStIncl = 2ull << 62;
constexpr uint64_t kStVal = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 24;

__device__ __forceinline__ void st_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t st_load(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decoupled look-back (Merrill & Garland, "Single-pass Parallel Prefix Scan
// with Decoupled Look-back", 2016), run by one full wave.  Tiles are claimed
// through an in-order ticket, so every predecessor is resident or finished
// and publishes its aggregate without waiting: the wait always ends.  The
// spin count is still bounded; on overrun the error bit is set and the wave
// carries on with what it has (the host then reports CV_ESTATE).
__device__ uint64_t lookback(uint64_t* status, int64_t t, uint64_t tile_total, uint32_t lane,
                             uint64_t* err) {
    if (t == 0) {
        if (lane == 0) st_store(&status[0], kStIncl | tile_total);
        return 0;
    }
    if (lane == 0) st_store(&status[t], kStAgg | tile_total);
    uint64_t excl = 0;
    int64_t p = t - 1;
    uint32_t spins = 0;
    for (;;) {
        const int64_t q = p - (int64_t)lane;
        uint64_t s = q >= 0 ? st_load(&status[q]) : kStIncl;
        for (;;) {
            uint64_t pend = __ballot((s >> 62) == 0);
            if (pend == 0) break;
            if (++spins > kSpinLimit) {
                if (lane == 0) atomicOr((unsigned long long*)err, 1ull);
                if ((s >> 62) == 0) s = kStAgg;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            if ((s >> 62) == 0) s = st_load(&status[q]);
        }
        const uint64_t incl = __ballot((s >> 62) == 2);
        const uint32_t first = incl ? (uint32_t)__builtin_ctzll(incl) : 64u;
        excl += wave_sum_u64(lane <= first ? (s & kStVal) : 0ull);
        if (incl) break;
        p -= 64;
    }
    if (lane == 0) st_store(&status[t], kStIncl | (excl + tile_total));
    return excl;
}

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

// ---------------------------------------------------------------------------
// Fused search with compaction.  A tile is TILE = BLOCK * K consecutive
// candidates (i, j) of one colour in row-major order; tiles of a colour are
// contiguous and colours follow each other, so the output order of the tiles
// is the (colour, i, j) order.  Inside a tile, pass m of wave w covers
// candidates [m*BLOCK + 64w, m*BLOCK + 64w + 64), so (m, w, lane) order is
// candidate order as well.
template <int BLOCK, int K, bool EMIT_ALL, bool SUMM, bool TAB_LDS>
__global__ __launch_bounds__(BLOCK) void k_pair_search(SearchArgs a) {
    constexpr int NW = BLOCK / 64;
    constexpr int TILE = BLOCK * K;
    static_assert(K * NW <= 64, "tile scan runs in one wave");
    static_assert(K <= 15, "per-tile pattern nibbles");
    extern __shared__ double s_tab[];
    __shared__ uint32_t s_cnt[K * NW];
    __shared__ uint32_t s_pre[K * NW];
    __shared__ uint64_t s_base;
    __shared__ int64_t s_tick;

    const int tid = threadIdx.x;
    const uint32_t lane = (uint32_t)tid & 63u;
    const int w = tid >> 6;

    const double* tab = a.tab.tab;
    if constexpr (TAB_LDS) {
        for (int k = tid; k < a.tab.tab_len; k += BLOCK) s_tab[k] = a.tab.tab[k];
        tab = s_tab;
    }

    int64_t cur_c = -1;
    uint32_t acc_cnt = 0, acc_ng = 0, acc_best = 0, acc_pat[7] = {0, 0, 0, 0, 0, 0, 0};

    for (;;) {
        if (tid == 0) s_tick = (int64_t)atomicAdd((unsigned long long*)&a.misc[0], 1ull);
        __syncthreads();
        const int64_t t = uniform_i64(s_tick);
        if (t >= a.ntiles) break;
        const int64_t c = t / a.tiles_per_colour;
        const int32_t lt = (int32_t)(t - c * a.tiles_per_colour);
        if constexpr (SUMM) {
            if (c != cur_c) {
                if (cur_c >= 0) flush_summary(a.acc, cur_c, lane, acc_cnt, acc_ng, acc_best, acc_pat);
                cur_c = c;
            }
        }
        const ColorConst cc = a.cc[c];

        // (i, j) of this thread's first candidate
        const int32_t base_idx = lt * TILE;
        const int32_t ib = base_idx / a.ntheta;
        const int32_t jb = base_idx - ib * a.ntheta;
        int32_t di, j;
        divmod_small(jb + tid, a.ntheta, a.inv_ntheta, di, j);
        int32_t i = ib + di;

        uint32_t r_ij[K], r_lo[K], r_hi[K];
        uint64_t bal[K];
        uint32_t nib = 0, ng = 0, best = 0;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const bool live = i < a.nr;
            double s, co;
            sincos_j<TAB_LDS>(tab, a.tab, live ? j : 0, s, co);
            const double rr = (double)(i + 1);
            PairEval e;
            eval_pair(cc, a.g, (rr * a.ra) * s, (rr * a.rb) * co, e);
            float Vp[3], Vm[3];
            bool ing;
            uint32_t p = decide(e, a.rule, Vp, Vm, ing);
            const bool surv = live && ing && accepts(a.rule, p);
            const uint32_t flags = (e.gp ? 1u : 0u) | (e.gm ? 2u : 0u) | (surv ? 4u : 0u);
            pack_pair(Vp, Vm, ing ? p : 0u, flags, r_lo[m], r_hi[m]);
            r_ij[m] = (uint32_t)i | ((uint32_t)j << 16);
            const bool emit = EMIT_ALL ? live : surv;
            bal[m] = __ballot(emit);
            if (lane == 0) s_cnt[m * NW + w] = (uint32_t)__builtin_popcountll(bal[m]);
            if constexpr (SUMM) {
                nib += surv ? (1u << (4u * (p - 1u))) : 0u;
                ng += (live && e.gp && e.gm) ? 1u : 0u;
                best = max(best, surv ? best_key(i, j) : 0u);
            }
            j += a.sj;
            i += a.si;
            if (j >= a.ntheta) { j -= a.ntheta; ++i; }
        }
        if constexpr (SUMM) {
#pragma unroll
            for (int p = 0; p < 7; ++p) {
                acc_pat[p] += (nib >> (4 * p)) & 0xFu;
                acc_cnt += (nib >> (4 * p)) & 0xFu;
            }
            acc_ng += ng;
            acc_best = max(acc_best, best);
        }
        __syncthreads();
        if (w == 0) {
            const uint32_t v = lane < (uint32_t)(K * NW) ? s_cnt[lane] : 0u;
            uint32_t incl = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                uint32_t u = __shfl_up(incl, o, 64);
                if (lane >= (uint32_t)o) incl += u;
            }
            if (lane < (uint32_t)(K * NW)) s_pre[lane] = incl - v;
            const uint64_t tile_total = __shfl(incl, 63, 64);
            const uint64_t excl = lookback(a.status, t, tile_total, lane, &a.misc[2]);
            if (lane == 0) {
                s_base = excl;
                if (lt == 0 && a.offsets) a.offsets[c] = (int64_t)excl;
                if (t == a.ntiles - 1) {
                    a.misc[1] = excl + tile_total;
                    if (a.offsets) a.offsets[a.n] = (int64_t)(excl + tile_total);
                }
            }
        }
        __syncthreads();
        const uint64_t base = s_base;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            if ((bal[m] >> lane) & 1ull) {
                const uint64_t pos = base + s_pre[m * NW + w] + rank_below(bal[m]);
                if (pos < (uint64_t)a.capacity) {
                    uint4 rec = make_uint4((uint32_t)c, r_ij[m], r_lo[m], r_hi[m]);
                    *reinterpret_cast<uint4*>(a.out + pos) = rec;
                }
            }
        }
    }
    if constexpr (SUMM) {
        if (cur_c >= 0) flush_summary(a.acc, cur_c, lane, acc_cnt, acc_ng, acc_best, acc_pat);
    }
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
    float inv_ntheta;
    int32_t si, sj;
    int32_t chunk;            // candidates per tile (multiple of the block size)
    int32_t tiles_per_colour;
    int32_t bin_num, bin_den; // bin = (j * bin_num) / bin_den = floor(36 j / N)
    int64_t n, ntiles;
    SumAcc* acc;              // atomic mode
    cv_color_summary* summ;   // direct mode outputs (nullable)
    cv_table_row* table;      // direct mode outputs (nullable)
    uint64_t* misc;           // [0] ticket
};

__device__ __forceinline__ void write_summary(const ColorConst& cc, const Geom& g,
                                              const RuleDev& rule, const TabArgs& tab,
                                              const double* tabp, double ra, double rb,
                                              uint32_t count, uint32_t ng, uint32_t key,
                                              const uint32_t pat[7], cv_color_summary* out) {
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
        sincos_j<false>(tabp, tab, j, sn, co);
        const double rr = (double)(i + 1);
        PairEval e;
        eval_pair(cc, g, (rr * ra) * sn, (rr * rb) * co, e);
        float Vp[3], Vm[3];
        bool ing;
        const uint32_t p = decide(e, rule, Vp, Vm, ing);
        s.best_i = (uint16_t)i;
        s.best_j = (uint16_t)j;
        for (int k = 0; k < 3; ++k) {
            s.best_plus[k] = (uint8_t)Vp[k];
            s.best_minus[k] = (uint8_t)Vm[k];
        }
        s.best_p = (uint8_t)p;
    }
    *out = s;
}

template <int BLOCK, bool TABLE, bool DIRECT, bool TAB_LDS>
__global__ __launch_bounds__(BLOCK) void k_pair_reduce(ReduceArgs a) {
    constexpr int NW = BLOCK / 64;
    extern __shared__ double s_dyn[];
    __shared__ uint32_t s_red[NW][10];
    __shared__ uint32_t s_bins[36];
    __shared__ int64_t s_tick;

    const int tid = threadIdx.x;
    const uint32_t lane = (uint32_t)tid & 63u;
    const int w = tid >> 6;
    const double* tab = a.tab.tab;
    uint32_t* s_ray = nullptr;
    if constexpr (TAB_LDS) {
        for (int k = tid; k < a.tab.tab_len; k += BLOCK) s_dyn[k] = a.tab.tab[k];
        tab = s_dyn;
    }
    if constexpr (TABLE) s_ray = reinterpret_cast<uint32_t*>(s_dyn + (TAB_LDS ? a.tab.tab_len : 0));

    for (;;) {
        if (tid == 0) s_tick = (int64_t)atomicAdd((unsigned long long*)&a.misc[0], 1ull);
        if constexpr (TABLE) {
            for (int k = tid; k < a.ntheta; k += BLOCK) s_ray[k] = 0;
        }
        __syncthreads();
        const int64_t t = uniform_i64(s_tick);
        if (t >= a.ntiles) break;
        const int64_t c = t / a.tiles_per_colour;
        const int32_t lt = (int32_t)(t - c * a.tiles_per_colour);
        const ColorConst cc = a.cc[c];
        const int32_t begin = lt * a.chunk;
        const int64_t per = (int64_t)a.nr * a.ntheta;
        const int32_t len = (int32_t)min((int64_t)a.chunk, per - begin);
        const int32_t ib = begin / a.ntheta;
        const int32_t jb = begin - ib * a.ntheta;
        int32_t di, j;
        divmod_small(jb + tid, a.ntheta, a.inv_ntheta, di, j);
        int32_t i = ib + di;

        uint32_t cnt = 0, ng = 0, best = 0;
        uint64_t pk = 0;          // 8-bit pattern counters, flushed every 255 steps
        uint32_t pat[7] = {0, 0, 0, 0, 0, 0, 0};
        int32_t steps = 0;
        for (int32_t k = tid; k < len; k += BLOCK) {
            double s, co;
            sincos_j<TAB_LDS>(tab, a.tab, j, s, co);
            const double rr = (double)(i + 1);
            PairEval e;
            eval_pair(cc, a.g, (rr * a.ra) * s, (rr * a.rb) * co, e);
            float Vp[3], Vm[3];
            bool ing;
            const uint32_t p = decide(e, a.rule, Vp, Vm, ing);
            const bool surv = ing && accepts(a.rule, p);
            ng += (e.gp && e.gm) ? 1u : 0u;
            if (surv) {
                ++cnt;
                pk += 1ull << (8u * (p - 1u));
                best = max(best, best_key(i, j));
                if constexpr (TABLE) atomicMax(&s_ray[j], (uint32_t)(i + 1));
            }
            if (++steps == 255) {
#pragma unroll
                for (int q = 0; q < 7; ++q) pat[q] += (uint32_t)(pk >> (8 * q)) & 0xFFu;
                pk = 0;
                steps = 0;
            }
            j += a.sj;
            i += a.si;
            if (j >= a.ntheta) { j -= a.ntheta; ++i; }
        }
#pragma unroll
        for (int q = 0; q < 7; ++q) pat[q] += (uint32_t)(pk >> (8 * q)) & 0xFFu;

        // block reduction: count, n_gamut, best, 7 patterns
        uint32_t v[10] = {wave_sum_u32(cnt), wave_sum_u32(ng), wave_max_u32(best)};
#pragma unroll
        for (int q = 0; q < 7; ++q) v[3 + q] = wave_sum_u32(pat[q]);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 10; ++q) s_red[w][q] = v[q];
        }
        __syncthreads();
        if constexpr (TABLE) {
            if (tid < 36) s_bins[tid] = 0;
            __syncthreads();
            for (int k = tid; k < a.ntheta; k += BLOCK) {
                const uint32_t r = s_ray[k];
                if (r) atomicMax(&s_bins[(k * a.bin_num) / a.bin_den], r);
            }
            __syncthreads();
        }
        if (tid < 10) {
            uint32_t x = 0;
            for (int q = 0; q < NW; ++q) x = (tid == 2) ? max(x, s_red[q][tid]) : x + s_red[q][tid];
            s_red[0][tid] = x;  // only wave 0's row is overwritten; read after the sync below
        }
        __syncthreads();
        if constexpr (DIRECT) {
            if (tid == 0) {
                uint32_t pt[7];
                for (int q = 0; q < 7; ++q) pt[q] = s_red[0][3 + q];
                if (a.summ)
                    write_summary(cc, a.g, a.rule, a.tab, a.tab.tab, a.ra, a.rb, s_red[0][0],
                                  s_red[0][1], s_red[0][2], pt, a.summ + c);
                if constexpr (TABLE) a.table[c].count = s_red[0][0];
            }
            if constexpr (TABLE) {
                if (tid < 36) a.table[c].bin_ridx[tid] = (uint8_t)min(s_bins[tid], 255u);
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
        write_summary(cc, g, rule, tab, tab.tab, ra, rb, s.count, s.n_gamut, s.best_key, s.pat,
                      summ + c);
    }
    if (table) {
        table[c].count = s.count;
        for (int k = 0; k < 36; ++k) table[c].bin_ridx[k] = (uint8_t)min(s.bins[k], 255u);
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

constexpr int kTabLdsBytes = 32 * 1024;

// Common set-up of a search: per-colour constants and the angle table.
int prepare(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd, hipStream_t s,
            TabArgs& tab) {
    int rc;
    if ((rc = ctx->ensure(ctx->colors, (size_t)n * sizeof(ColorConst))) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->table, (size_t)gd.tab_len * sizeof(double))) != CV_OK) return rc;
    hipLaunchKernelGGL(k_angle_table, dim3(blocks_for(gd.N, 256)), dim3(256), 0, s,
                       (double*)ctx->table.ptr, gd.N, gd.tab_len > gd.N ? 1 : 0);
    CV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_color_prologue, dim3(blocks_for(n, 256)), dim3(256), 0, s, rgb,
                       (ColorConst*)ctx->colors.ptr, n, mat_args());
    CV_HIP(hipGetLastError());
    tab.tab = (const double*)ctx->table.ptr;
    tab.tab_len = gd.tab_len;
    tab.qoff = gd.qoff;
    tab.wrap = gd.wrap;
    tab.N = gd.N;
    return CV_OK;
}

template <typename Kern>
int persistent_grid(cv_context* ctx, Kern k, int block, size_t lds, int64_t ntiles, unsigned& grid) {
    int per_cu = 0;
    CV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, lds));
    if (per_cu < 1) per_cu = 1;
    int64_t g = (int64_t)per_cu * ctx->num_cu;
    if (g > ntiles) g = ntiles;
    grid = (unsigned)(g < 1 ? 1 : g);
    return CV_OK;
}

constexpr int kSearchBlock = 256;
constexpr int kSearchK = 8;
constexpr int kSearchTile = kSearchBlock * kSearchK;

template <bool EMIT, bool SUMM, bool LDS>
int launch_search_t(cv_context* ctx, const SearchArgs& a, hipStream_t s) {
    auto k = k_pair_search<kSearchBlock, kSearchK, EMIT, SUMM, LDS>;
    const size_t lds = LDS ? (size_t)a.tab.tab_len * sizeof(double) : 0;
    unsigned grid;
    int rc = persistent_grid(ctx, k, kSearchBlock, lds, a.ntiles, grid);
    if (rc != CV_OK) return rc;
    hipLaunchKernelGGL(k, dim3(grid), dim3(kSearchBlock), lds, s, a);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

int launch_search(cv_context* ctx, const SearchArgs& a, bool emit, bool summ, bool lds,
                  hipStream_t s) {
    const int sel = (emit ? 4 : 0) | (summ ? 2 : 0) | (lds ? 1 : 0);
    switch (sel) {
    case 0: return launch_search_t<false, false, false>(ctx, a, s);
    case 1: return launch_search_t<false, false, true>(ctx, a, s);
    case 2: return launch_search_t<false, true, false>(ctx, a, s);
    case 3: return launch_search_t<false, true, true>(ctx, a, s);
    case 4: return launch_search_t<true, false, false>(ctx, a, s);
    case 5: return launch_search_t<true, false, true>(ctx, a, s);
    case 6: return launch_search_t<true, true, false>(ctx, a, s);
    default: return launch_search_t<true, true, true>(ctx, a, s);
    }
}

constexpr int kReduceBlock = 256;

template <bool TABLE, bool DIRECT, bool LDS>
int launch_reduce_t(cv_context* ctx, const ReduceArgs& a, hipStream_t s) {
    auto k = k_pair_reduce<kReduceBlock, TABLE, DIRECT, LDS>;
    const size_t lds = (LDS ? (size_t)a.tab.tab_len * sizeof(double) : 0) +
                       (TABLE ? (size_t)a.ntheta * sizeof(uint32_t) : 0);
    unsigned grid;
    int rc = persistent_grid(ctx, k, kReduceBlock, lds, a.ntiles, grid);
    if (rc != CV_OK) return rc;
    hipLaunchKernelGGL(k, dim3(grid), dim3(kReduceBlock), lds, s, a);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

int launch_reduce(cv_context* ctx, const ReduceArgs& a, bool table, bool direct, bool lds,
                  hipStream_t s) {
    const int sel = (table ? 4 : 0) | (direct ? 2 : 0) | (lds ? 1 : 0);
    switch (sel) {
    case 0: return launch_reduce_t<false, false, false>(ctx, a, s);
    case 1: return launch_reduce_t<false, false, true>(ctx, a, s);
    case 2: return launch_reduce_t<false, true, false>(ctx, a, s);
    case 3: return launch_reduce_t<false, true, true>(ctx, a, s);
    case 4: return launch_reduce_t<true, false, false>(ctx, a, s);
    case 5: return launch_reduce_t<true, false, true>(ctx, a, s);
    case 6: return launch_reduce_t<true, true, false>(ctx, a, s);
    default: return launch_reduce_t<true, true, true>(ctx, a, s);
    }
}

} // namespace

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

int run_pair_search(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd,
                    const RuleDev& rd, cv_pair* out, int64_t capacity, int64_t* offsets,
                    cv_color_summary* summ, int64_t* total_host, uint32_t flags,
                    hipStream_t s) {
    int rc;
    if (n == 0) {
        if (offsets) hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, offsets, (int64_t)0);
        CV_HIP(hipGetLastError());
        *total_host = 0;
        return CV_OK;
    }
    TabArgs tab;
    if ((rc = prepare(ctx, rgb, n, gd, s, tab)) != CV_OK) return rc;
    const int32_t tpc = (int32_t)((gd.per_colour + kSearchTile - 1) / kSearchTile);
    const int64_t ntiles = (int64_t)tpc * n;
    if ((rc = ctx->ensure(ctx->status, (size_t)ntiles * 8)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->misc, 64)) != CV_OK) return rc;
    if (summ && (rc = ctx->ensure(ctx->acc, (size_t)n * sizeof(SumAcc))) != CV_OK) return rc;
    if ((rc = zero_u64(ctx->status.ptr, ntiles, s)) != CV_OK) return rc;
    if ((rc = zero_u64(ctx->misc.ptr, 8, s)) != CV_OK) return rc;
    if (summ && (rc = zero_u64(ctx->acc.ptr, n * (int64_t)(sizeof(SumAcc) / 8), s)) != CV_OK)
        return rc;

    SearchArgs a;
    a.cc = (const ColorConst*)ctx->colors.ptr;
    a.tab = tab;
    a.g = geom_constants();
    a.rule = rd;
    a.ra = gd.ra;
    a.rb = gd.rb;
    a.nr = gd.nr;
    a.ntheta = gd.ntheta;
    a.inv_ntheta = 1.0f / (float)gd.ntheta;
    a.si = kSearchBlock / gd.ntheta;
    a.sj = kSearchBlock % gd.ntheta;
    a.tiles_per_colour = tpc;
    a.n = n;
    a.ntiles = ntiles;
    a.out = out;
    a.capacity = out ? capacity : 0;
    a.offsets = offsets;
    a.status = (uint64_t*)ctx->status.ptr;
    a.acc = summ ? (SumAcc*)ctx->acc.ptr : nullptr;
    a.misc = (uint64_t*)ctx->misc.ptr;
    const bool lds = (size_t)gd.tab_len * sizeof(double) <= (size_t)kTabLdsBytes;
    if ((rc = ctx->time_begin(s)) != CV_OK) return rc;
    if ((rc = launch_search(ctx, a, (flags & CV_EMIT_ALL) != 0, summ != nullptr, lds, s)) != CV_OK)
        return rc;
    if ((rc = ctx->time_end(s, false)) != CV_OK) return rc;
    if (summ) {
        hipLaunchKernelGGL(k_finalize, dim3(blocks_for(n, 128)), dim3(128), 0, s, a.cc, a.acc, n,
                           a.g, rd, tab, gd.ra, gd.rb, summ, (cv_table_row*)nullptr);
        CV_HIP(hipGetLastError());
    }
    CV_HIP(hipMemcpyAsync(ctx->host_misc, ctx->misc.ptr, 3 * sizeof(uint64_t),
                          hipMemcpyDeviceToHost, s));
    CV_HIP(hipStreamSynchronize(s));
    if (ctx->timing) {
        float ms = 0.0f;
        CV_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        ctx->kernel_ms += ms;
        ctx->kernel_launches += 1;
    }
    if (ctx->host_misc[2] != 0) return fail(CV_ESTATE, "look-back wait exceeded its bound");
    *total_host = (int64_t)ctx->host_misc[1];
    if (*total_host > capacity)
        return fail(CV_ECAPACITY, "survivor total " + std::to_string(*total_host) +
                                      " exceeds capacity " + std::to_string(capacity));
    return CV_OK;
}

int run_pair_reduce(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd,
                    const RuleDev& rd, cv_color_summary* summ, cv_table_row* table,
                    hipStream_t s) {
    if (n == 0) return CV_OK;
    int rc;
    TabArgs tab;
    if ((rc = prepare(ctx, rgb, n, gd, s, tab)) != CV_OK) return rc;
    const int64_t per = gd.per_colour;
    const bool direct = n >= 2048 && per <= (1 << 20);
    int64_t chunk;
    if (direct) {
        chunk = per;
    } else {
        const int64_t want_tiles_per_colour = (8192 + n - 1) / n;
        chunk = (per + want_tiles_per_colour - 1) / want_tiles_per_colour;
        if (chunk < 16 * kReduceBlock) chunk = 16 * kReduceBlock;
        chunk = (chunk + kReduceBlock - 1) / kReduceBlock * kReduceBlock;
    }
    const int32_t tpc = (int32_t)((per + chunk - 1) / chunk);
    const int64_t ntiles = (int64_t)tpc * n;
    if ((rc = ctx->ensure(ctx->misc, 64)) != CV_OK) return rc;
    if ((rc = zero_u64(ctx->misc.ptr, 8, s)) != CV_OK) return rc;
    if (!direct) {
        if ((rc = ctx->ensure(ctx->acc, (size_t)n * sizeof(SumAcc))) != CV_OK) return rc;
        if ((rc = zero_u64(ctx->acc.ptr, n * (int64_t)(sizeof(SumAcc) / 8), s)) != CV_OK) return rc;
    }
    ReduceArgs a;
    a.cc = (const ColorConst*)ctx->colors.ptr;
    a.tab = tab;
    a.g = geom_constants();
    a.rule = rd;
    a.ra = gd.ra;
    a.rb = gd.rb;
    a.nr = gd.nr;
    a.ntheta = gd.ntheta;
    a.inv_ntheta = 1.0f / (float)gd.ntheta;
    a.si = kReduceBlock / gd.ntheta;
    a.sj = kReduceBlock % gd.ntheta;
    a.chunk = (int32_t)chunk;
    a.tiles_per_colour = tpc;
    a.bin_num = 36;
    a.bin_den = gd.N;
    a.n = n;
    a.ntiles = ntiles;
    a.acc = direct ? nullptr : (SumAcc*)ctx->acc.ptr;
    a.summ = summ;
    a.table = table;
    a.misc = (uint64_t*)ctx->misc.ptr;
    const bool lds = (size_t)gd.tab_len * sizeof(double) <= (size_t)kTabLdsBytes;
    if ((rc = ctx->time_begin(s)) != CV_OK) return rc;
    if ((rc = launch_reduce(ctx, a, table != nullptr, direct, lds, s)) != CV_OK) return rc;
    if ((rc = ctx->time_end(s, true)) != CV_OK) return rc;
    if (!direct) {
        hipLaunchKernelGGL(k_finalize, dim3(blocks_for(n, 128)), dim3(128), 0, s, a.cc, a.acc, n,
                           a.g, rd, tab, gd.ra, gd.rb, summ, table);
        CV_HIP(hipGetLastError());
    }
    return CV_OK;
}

} // namespace cvib
