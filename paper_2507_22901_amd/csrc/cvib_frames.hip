// Batched frames: de-duplicate the colours of many frames, search every
// distinct colour in one persistent launch (the colour count stays on the
// device), and render the two alternating frames that carry the per-pixel
// information (Fig. 1a of the paper: the display alternates the two colours
// of a pair; a device reads the per-channel change, people see the target).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <string>

#include "cvib_internal.h"
#include "cvib_kernels.h"

namespace cvib {

constexpr int64_t kCube = (int64_t)1 << 24;     // distinct 8-bit colours
constexpr int64_t kCubeWords = kCube / 32;      // bitmap words

// ---------------------------------------------------------------------------
// De-duplication through a 2^24-bit bitmap of colour ids R<<16 | G<<8 | B.

// Pixels are 3 bytes; the pixel index and the surrogate's renderer take them
// four at a time, 12 bytes as three aligned words when the arrays allow it
// (else byte by byte), and the last npix % 4 pixels one by one.  (The bitmap
// marking and the exact renderer, whose reads depend on atomics or branch per
// pixel, measured slower that way and keep one pixel per thread.)
struct Quad {
    uint32_t w[3];
};

__device__ __forceinline__ Quad load_quad(const uint8_t* __restrict__ px, int64_t q, bool aligned) {
    Quad r;
    if (aligned) {
        const uint32_t* p = reinterpret_cast<const uint32_t*>(px + 12 * q);
        r.w[0] = p[0];
        r.w[1] = p[1];
        r.w[2] = p[2];
    } else {
        const uint8_t* p = px + 12 * q;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            r.w[k] = (uint32_t)p[4 * k] | ((uint32_t)p[4 * k + 1] << 8) | ((uint32_t)p[4 * k + 2] << 16) |
                     ((uint32_t)p[4 * k + 3] << 24);
    }
    return r;
}

__device__ __forceinline__ void store_quad(uint8_t* __restrict__ out, int64_t q, const Quad& v, bool aligned) {
    if (aligned) {
        uint32_t* p = reinterpret_cast<uint32_t*>(out + 12 * q);
        p[0] = v.w[0];
        p[1] = v.w[1];
        p[2] = v.w[2];
    } else {
        uint8_t* p = out + 12 * q;
#pragma unroll
        for (int b = 0; b < 12; ++b) p[b] = (uint8_t)(v.w[b >> 2] >> (8 * (b & 3)));
    }
}

// Byte b of a quad, and colour k's id R<<16 | G<<8 | B.
__device__ __forceinline__ uint32_t quad_byte(const Quad& v, int b) { return (v.w[b >> 2] >> (8 * (b & 3))) & 255u; }
__device__ __forceinline__ uint32_t quad_id(const Quad& v, int k) {
    return (quad_byte(v, 3 * k) << 16) | (quad_byte(v, 3 * k + 1) << 8) | quad_byte(v, 3 * k + 2);
}
__device__ __forceinline__ void quad_set(Quad& v, int b, uint32_t x) {
    const int sh = 8 * (b & 3);
    v.w[b >> 2] = (v.w[b >> 2] & ~(255u << sh)) | ((x & 255u) << sh);
}
__device__ __forceinline__ uint32_t pixel_id(const uint8_t* __restrict__ px, int64_t p) {
    return ((uint32_t)px[3 * p] << 16) | ((uint32_t)px[3 * p + 1] << 8) | px[3 * p + 2];
}

__global__ void k_bitmap_mark(const uint8_t* __restrict__ px, int64_t npix,
                              uint32_t* __restrict__ bits) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
        const uint32_t id = ((uint32_t)px[3 * p] << 16) | ((uint32_t)px[3 * p + 1] << 8) | px[3 * p + 2];
        const uint32_t bit = 1u << (id & 31u);
        uint32_t* word = bits + (id >> 5);
        // most pixels repeat a colour already marked: read first (a cached
        // load; a stale zero only costs a redundant atomic, and a set bit is
        // final), then set
        if ((*word & bit) == 0u) atomicOr(word, bit);
    }
}

__global__ void k_bitmap_popc(const uint32_t* __restrict__ bits, uint32_t* __restrict__ cnt) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w < kCubeWords) cnt[w] = (uint32_t)__builtin_popcount(bits[w]);
}

// Sorted distinct colours: word w's colours start at prefix[w].
__global__ void k_bitmap_compact(const uint32_t* __restrict__ bits,
                                 const uint64_t* __restrict__ prefix,
                                 uint8_t* __restrict__ colours) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= kCubeWords) return;
    uint32_t m = bits[w];
    uint64_t k = prefix[w];
    while (m) {
        const uint32_t b = (uint32_t)__builtin_ctz(m);
        m &= m - 1u;
        const uint32_t id = ((uint32_t)w << 5) | b;
        colours[3 * k] = (uint8_t)(id >> 16);
        colours[3 * k + 1] = (uint8_t)(id >> 8);
        colours[3 * k + 2] = (uint8_t)id;
        ++k;
    }
}

// Index of each pixel's colour in the sorted list (idx16: the index array is
// 16-byte aligned, four indices written as one store).
__device__ __forceinline__ uint32_t colour_index(const uint32_t* __restrict__ bits, const uint64_t* __restrict__ prefix,
                                                 uint32_t id) {
    const uint32_t w = id >> 5, b = id & 31u;
    return (uint32_t)prefix[w] + (uint32_t)__builtin_popcount(bits[w] & ((1u << b) - 1u));
}

__global__ void k_pixel_index(const uint8_t* __restrict__ px, int64_t npix,
                              const uint32_t* __restrict__ bits,
                              const uint64_t* __restrict__ prefix, uint32_t* __restrict__ index, bool aligned,
                              bool idx16) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x, nq = npix >> 2;
    for (int64_t q = t; q < nq; q += stride) {
        const Quad v = load_quad(px, q, aligned);
        uint32_t r[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] = colour_index(bits, prefix, quad_id(v, k));
        if (idx16) {
            *reinterpret_cast<uint4*>(index + 4 * q) = make_uint4(r[0], r[1], r[2], r[3]);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) index[4 * q + k] = r[k];
        }
    }
    if (t < (npix & 3)) {
        const int64_t p = 4 * nq + t;
        index[p] = colour_index(bits, prefix, pixel_id(px, p));
    }
}

// Per-colour constants for a device-resident colour count.
__global__ void k_prologue_dev(const uint8_t* __restrict__ rgb, const uint64_t* __restrict__ n_dev,
                               ColorConst* __restrict__ cc, MatArgs m) {
    const int64_t n = (int64_t)*n_dev;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        double lab[3];
        rgb8_lab(m, rgb + 3 * k, lab);
        const double fy = (lab[0] + 16.0) / 116.0;
        const double Y = finv(fy) * m.W[1];
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
}

// ---------------------------------------------------------------------------
// Per-colour resolve: one block searches one colour completely (colours are
// strided over the persistent grid; the count is read from the device).  It
// produces the summary, the best pair of every information pattern and,
// optionally, the largest surviving radius of every ray.

struct ResolveArgs {
    const ColorConst* cc;
    const uint64_t* n_dev;
    TabArgs tab;
    Geom g;
    RuleDev rule;
    double ra, rb;
    int32_t nr, ntheta, W;
    float inv_W;
    int32_t si, sj;           // a step of 256 evaluations = si rows + sj rays
    int32_t si64, sj64;       // a step of 64 evaluations
    const uint32_t* list;     // nullable: the k-th colour searched is list[k]
    cv_color_summary* summ;   // nullable
    cv_pattern_pair* pbest;   // nullable, [n][7]
    uint16_t* rays;           // nullable, [n][ntheta]
    int32_t cells;            // skip wave steps proven out of gamut (CELLS kernels)
    // 0: n_gamut is not needed (no summaries, or CV_NO_NGAMUT), so steps
    // proven to hold no high channel are skipped rather than counted
    int32_t need_ng;
    uint64_t* stats;          // [0..7]: candidates skipped by the cells; [8..15]: in-gamut pairs of
                              // steps without a high channel (counted, not encoded); summed (nullable)
};

// Per-block sum of the lanes' skipped counts into stats (every thread calls
// it once, at the end; w = the wave of the block).
template <int NW>
__device__ __forceinline__ void add_skipped(uint64_t* stats, uint64_t skipped, uint64_t no_high, int w) {
    if (!stats) return;
    __shared__ uint64_t s_skip[NW], s_noh[NW];
    const uint32_t lane = lane_id_fresh();
    for (int o = 32; o > 0; o >>= 1) skipped += (uint64_t)__shfl_xor((unsigned long long)skipped, o, 64);
    if (lane == 0) {
        s_skip[w] = skipped;
        s_noh[w] = no_high;
    }
    __syncthreads();
    if (w == 0 && lane == 0) {
        uint64_t sum = 0, nh = 0;
        for (int q = 0; q < NW; ++q) {
            sum += s_skip[q];
            nh += s_noh[q];
        }
        if (sum) atomicAdd((unsigned long long*)&stats[blockIdx.x & 7u], (unsigned long long)sum);
        if (nh) atomicAdd((unsigned long long*)&stats[8 + (blockIdx.x & 7u)], (unsigned long long)nh);
    }
}

// All candidates of one colour, split over a group of g_size threads (a block
// or one wave): thread g_tid takes evaluations g_tid, g_tid + g_size, ... in
// row-major (i, j < W) order; a step of g_size evaluations is si rows + sj
// rays.  Wave totals accumulate in cnt, ng and pat (the same value in every
// lane), the lane's best key in best; survivors raise the pattern's best key
// in s_pb and, with RAYS, the ray's largest radius in s_ray.  With CELLS
// ((nr + kBandRows - 1) W < 2^24) the candidates are taken in the band order
// (bands of kBandRows rows, ray by ray; every result here is a count or a maximum, so the
// order is free) and each wave first decides 64 of its steps at a time, one
// per lane, evaluating only those that may hold a pair in gamut.
template <bool RAYS, bool CELLS>
__device__ __forceinline__ void resolve_colour(const ResolveArgs& a, const Angles& ang,
                                               const ColorConst& cc, int32_t g_tid, int32_t g_size,
                                               int32_t si, int32_t sj, uint32_t lane, uint32_t* s_pb,
                                               uint32_t* s_ray, uint32_t& cnt, uint32_t& ng,
                                               uint32_t& best, uint32_t pat[7], uint64_t& skipped,
                                               uint64_t& no_high) {
    const bool clip = a.rule.clip != 0u;
    const int32_t per = a.nr * a.W;
    const int32_t iters = (per + g_size - 1) / g_size;
    const bool cube = cube_branch_only(cc, a.nr - 1, a.ra, a.rb);
    auto step = [&](int32_t i, int32_t j, bool live) {
        double sn, co;
        ang.get(j, sn, co);
        const double rr = (double)(i + 1);
        float fp[3], fm[3];
        pair_linear_w(cc, a.g, (rr * a.ra) * sn, (rr * a.rb) * co, fp, fm, cube);
        const uint64_t live_m = __ballot(live);
        const uint64_t both_m = __ballot(in_unit_cube(fp) && in_unit_cube(fm)) & live_m;
        const uint64_t need_m = clip ? live_m : both_m;
        if (a.need_ng) ng += (uint32_t)__builtin_popcountll(both_m);
        if (need_m != 0ull) {
            float Vp[3], Vm[3];
            codes_w(fp, fm, (need_m >> lane) & 1ull, clip, Vp, Vm);
            const PatMasks pm = pattern_masks(Vp, Vm, a.rule);
            const uint64_t surv_m = accepted_lanes(pm, a.rule.mask) & need_m;
            if (surv_m != 0ull) {
                cnt += (uint32_t)__builtin_popcountll(surv_m);
                count_patterns(pm, need_m, pat);
                if ((surv_m >> lane) & 1ull) {
                    const uint32_t key = best_key(i, j);
                    best = max(best, key);
                    atomicMax(&s_pb[pattern_of(Vp, Vm, a.rule) - 1u], key);
                    if (RAYS) atomicMax(&s_ray[j], (uint32_t)(i + 1));
                }
            }
        }
    };
    if constexpr (CELLS) {
        // a step proven to hold no high channel holds no survivor: its
        // in-gamut pairs are counted when n_gamut is needed, else it is skipped
        auto gamut_step = [&](int32_t i, int32_t j, bool live) {
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
        const bool need_ng = a.need_ng != 0;
        const int32_t per4 = ((a.nr + kBandRows - 1) / kBandRows) * kBandRows * a.W;  // whole bands
        const int32_t iters4 = (per4 + g_size - 1) / g_size;
        const float inv_W4 = a.inv_W / (float)kBandRows;  // exact: a power of two
        const int32_t wb = g_tid - (int32_t)lane;  // the wave's first evaluation of a step
        uint64_t evald = 0;
        for (int32_t word = 0; word < (iters4 + 63) >> 6; ++word) {
            const int32_t itl = word * 64 + (int32_t)lane, e0 = itl * g_size + wb;
            const bool any = itl < iters4 && e0 < per4;
            bool high = true;
            const bool open = band_step_open(cc, a.g, ang, a.ra, a.rb, a.W, inv_W4, min(e0, per4 - 1),
                                             min(e0 + 63, per4 - 1), any, &a.rule, &high);
            const uint64_t full = uniform_u64(__ballot(open && high));
            uint64_t m = need_ng ? uniform_u64(__ballot(open)) : full;
            while (m) {
                const int32_t bit = (int32_t)__builtin_ctzll(m);
                const int32_t e = (word * 64 + bit) * g_size + g_tid;
                m &= m - 1ull;
                const BandPos bp = band_pos(min(e, per4 - 1), a.W, inv_W4);
                const int32_t i = bp.i;
                const bool live = e < per4 && i < a.nr;
                evald += (uint64_t)__builtin_popcountll(__ballot(live));
                if ((full >> bit) & 1ull) step(min(i, a.nr - 1), bp.j, live);
                else gamut_step(min(i, a.nr - 1), bp.j, live);
            }
        }
        // the colour's candidates less those evaluated (unsigned sums cancel)
        if (lane == 0) skipped += (wb == 0 ? (uint64_t)per : 0ull) - evald;
    } else {
        int32_t i, j;
        divmod_small(g_tid, a.W, a.inv_W, i, j);
        for (int32_t it = 0; it < iters; ++it) {
            step(i, j, it * g_size + g_tid < per);
            j += sj;
            i += si;
            if (j >= a.W) { j -= a.W; ++i; }
        }
    }
}

// The best pair of pattern q + 1 from its key (0 = none), codes evaluated again.
__device__ __forceinline__ cv_pattern_pair pattern_pair(const ResolveArgs& a, const Angles& ang,
                                                        const ColorConst& cc, uint32_t key, int q) {
    cv_pattern_pair r = {};
    if (key) {
        const int32_t bi = (int32_t)(key >> 16), bj = (int32_t)(0xFFFFu - (key & 0xFFFFu));
        double sn, co;
        ang.get(bj, sn, co);
        const double rr = (double)(bi + 1);
        PairEval e;
        eval_pair(cc, a.g, (rr * a.ra) * sn, (rr * a.rb) * co, e);
        r.i = (uint16_t)bi;
        r.j = (uint16_t)bj;
        for (int k = 0; k < 3; ++k) {
            r.plus[k] = (uint8_t)e.Vp[k];
            r.minus[k] = (uint8_t)e.Vm[k];
        }
        r.pattern = (uint8_t)(q + 1);
        r.flags = 1;
    }
    return r;
}

// One colour per block of four waves.
// Six waves per SIMD: the register budget of 80 keeps one more wave resident
// than the unbounded allocation (84) would.
template <bool SYM, bool RAYS, bool CELLS>
__global__ __launch_bounds__(256, 6) void k_colour_resolve(ResolveArgs a) {
    constexpr int BLOCK = 256, NW = BLOCK / 64;
    extern __shared__ double s_dyn[];
    __shared__ uint32_t s_red[NW][10];
    __shared__ uint32_t s_pb[7];
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // the wave of the block
    const Angles ang = load_angles(a.tab, s_dyn);
    uint32_t* s_ray = reinterpret_cast<uint32_t*>(s_dyn + a.tab.tab_len + 2 * a.tab.dW);
    const uint32_t mult = SYM ? 2u : 1u;
    const int64_t n = (int64_t)*a.n_dev;
    uint64_t skipped = 0, no_high = 0;

    for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
        // the thread's indices taken afresh every colour (nothing derived
        // from them stays live across the colours)
        const uint32_t lane = lane_id_fresh();
        const int tid = w * 64 + (int)lane;
        const int64_t c = a.list ? (int64_t)a.list[k] : k;
        if (RAYS)
            for (int q = tid; q < a.W; q += BLOCK) s_ray[q] = 0;
        if (tid < 7) s_pb[tid] = 0;
        __syncthreads();
        const ColorConst cc = a.cc[c];
        uint32_t cnt = 0, ng = 0, best = 0;
        uint32_t pat[7] = {0, 0, 0, 0, 0, 0, 0};
        resolve_colour<RAYS, CELLS>(a, ang, cc, tid, BLOCK, a.si, a.sj, lane, s_pb, s_ray, cnt, ng, best, pat,
                                    skipped, no_high);
        uint32_t v[10] = {mult * cnt, mult * ng, wave_max_u32(best)};
#pragma unroll
        for (int q = 0; q < 7; ++q) v[3 + q] = mult * accepted_count(a.rule.mask, q, pat[q]);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 10; ++q) s_red[w][q] = v[q];
        }
        __syncthreads();
        if (tid < 10) {
            uint32_t x = 0;
            for (int q = 0; q < NW; ++q) x = (tid == 2) ? max(x, s_red[q][tid]) : x + s_red[q][tid];
            s_red[0][tid] = x;  // column tid is touched by this thread only
        }
        __syncthreads();
        if (tid == 0 && a.summ) {
            uint32_t pt[7];
            for (int q = 0; q < 7; ++q) pt[q] = s_red[0][3 + q];
            write_summary(cc, a.g, a.rule, a.tab, a.ra, a.rb, s_red[0][0], s_red[0][1], s_red[0][2],
                          pt, a.summ + c);
        }
        if (tid < 7 && a.pbest) a.pbest[c * 7 + tid] = pattern_pair(a, ang, cc, s_pb[tid], tid);
        if (RAYS) {
            uint16_t* dst = a.rays + c * (int64_t)a.ntheta;
            for (int q = tid; q < a.W; q += BLOCK) {
                const uint16_t r = (uint16_t)s_ray[q];
                dst[q] = r;
                if (SYM) dst[q + a.W] = r;  // ray j + N/2 holds the same pairs
            }
        }
        __syncthreads();
    }
    add_skipped<NW>(a.stats, skipped, no_high, w);
}

// LDS written by some lanes of a wave visible to its other lanes: a wave's
// LDS operations complete in order; this keeps the compiler from moving
// accesses across the point and waits for the outstanding ones.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// One colour per wave, BLOCK / 64 colours per block: no block barrier after
// the start, each wave with its own pattern keys and per-ray maxima in LDS.
template <bool SYM, bool RAYS, int BLOCK, bool CELLS>
__global__ __launch_bounds__(BLOCK) void k_colour_resolve_w(ResolveArgs a) {
    constexpr int NW = BLOCK / 64;
    extern __shared__ double s_dyn[];
    __shared__ uint32_t s_pbw[NW][8];
    const int tid = threadIdx.x;
    const uint32_t lane = (uint32_t)tid & 63u;
    const int w = tid >> 6;
    const Angles ang = load_angles(a.tab, s_dyn);
    uint32_t* s_ray =
        reinterpret_cast<uint32_t*>(s_dyn + a.tab.tab_len + 2 * a.tab.dW) + (RAYS ? w * a.W : 0);
    uint32_t* s_pb = s_pbw[w];
    const uint32_t mult = SYM ? 2u : 1u;
    const int64_t n = (int64_t)*a.n_dev;
    uint64_t skipped = 0, no_high = 0;

    for (int64_t k = (int64_t)blockIdx.x * NW + w; k < n; k += (int64_t)gridDim.x * NW) {
        const int64_t c = a.list ? (int64_t)a.list[k] : k;
        if (RAYS)
            for (int q = (int)lane; q < a.W; q += 64) s_ray[q] = 0;
        if (lane < 7) s_pb[lane] = 0;
        wave_lds_sync();
        const ColorConst cc = a.cc[c];
        uint32_t cnt = 0, ng = 0, best = 0;
        uint32_t pat[7] = {0, 0, 0, 0, 0, 0, 0};
        resolve_colour<RAYS, CELLS>(a, ang, cc, (int32_t)lane, 64, a.si64, a.sj64, lane, s_pb, s_ray, cnt,
                                    ng, best, pat, skipped, no_high);
        best = wave_max_u32(best);
        wave_lds_sync();
        if (lane == 0 && a.summ) {
            uint32_t pt[7];
            for (int q = 0; q < 7; ++q) pt[q] = mult * accepted_count(a.rule.mask, q, pat[q]);
            write_summary(cc, a.g, a.rule, a.tab, a.ra, a.rb, mult * cnt, mult * ng, best, pt, a.summ + c);
        }
        if (lane < 7 && a.pbest) a.pbest[c * 7 + lane] = pattern_pair(a, ang, cc, s_pb[lane], (int)lane);
        if (RAYS) {
            uint16_t* dst = a.rays + c * (int64_t)a.ntheta;
            for (int q = (int)lane; q < a.W; q += 64) {
                const uint16_t r = (uint16_t)s_ray[q];
                dst[q] = r;
                if (SYM) dst[q + a.W] = r;
            }
        }
        wave_lds_sync();
    }
    add_skipped<NW>(a.stats, skipped, no_high, w);  // every wave reaches it once its colours are done
}

// ---------------------------------------------------------------------------
// Rendering: frame A shows the + colour and frame B the - colour of the pair
// chosen for each pixel (the best pair of the pixel's information pattern, or
// of any pattern when no map is given); pixels without a pair keep their
// colour in both frames.

__global__ void k_render(const uint8_t* __restrict__ px, int64_t npix,
                         const uint32_t* __restrict__ index, const uint8_t* __restrict__ info,
                         const cv_pattern_pair* __restrict__ pbest,
                         const cv_color_summary* __restrict__ summ, uint8_t* __restrict__ fa,
                         uint8_t* __restrict__ fb, unsigned long long* __restrict__ resolved) {
    uint32_t got = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
        const uint32_t k = index[p];
        const uint32_t q = info ? info[p] : 0u;
        uint8_t A[3] = {px[3 * p], px[3 * p + 1], px[3 * p + 2]};
        uint8_t B[3] = {A[0], A[1], A[2]};
        bool ok = false;
        if (q >= 1u && q <= 7u) {
            const cv_pattern_pair& r = pbest[(int64_t)k * 7 + (q - 1u)];
            if (r.flags & 1u) {
                for (int c = 0; c < 3; ++c) {
                    A[c] = r.plus[c];
                    B[c] = r.minus[c];
                }
                ok = true;
            }
        } else if (q == 0u && summ && summ[k].best_i != 0xFFFFu) {
            for (int c = 0; c < 3; ++c) {
                A[c] = summ[k].best_plus[c];
                B[c] = summ[k].best_minus[c];
            }
            ok = true;
        }
        for (int c = 0; c < 3; ++c) {
            fa[3 * p + c] = A[c];
            fb[3 * p + c] = B[c];
        }
        got += ok ? 1u : 0u;
    }
    const uint32_t s = wave_sum_u32(got);
    if ((threadIdx.x & 63u) == 0 && s && resolved) atomicAdd(resolved, (unsigned long long)s);
}

__global__ void k_zero_words(uint64_t* __restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = 0;
}

__global__ void k_copy_count(const uint64_t* __restrict__ src, int64_t* __restrict__ dst) {
    *dst = (int64_t)*src;
}

// ---------------------------------------------------------------------------
// Surrogate resolve.  The network's outputs for colour c are 36 predicted
// maximum radii (divided by 50) and a feasibility logit.  A colour whose
// logit reaches tau gets proposals: in each of its kbins bins of largest
// predicted radius r, every ray of the bin at the radii r + o for o on a
// fixed ladder (Delta E units: +1, 0, -1, -2.5, -5, -10), snapped to the grid.
// When theta spans the full turn, bin b + 18 holds the mirror images of bin
// b's pairs, so the 18 bins of the first half-turn are ranked by the mean of
// the two predictions and only they are proposed (the mirror image of a pair
// has the same validity and a larger j).  Each proposal runs through the
// exact predicate of the search (the same device functions and the same
// arithmetic), so a verified pair is a survivor of the exact search; the
// verified pair of largest i (then smallest j) is kept.  A local search then
// raises it:
// - climb: the radii of one ray from a start index upward, 64 at a time,
//   through the same predicate; the largest that passes is a candidate; the
//   climb stops at the first block of 64 with no survivor or after
//   kClimbBlocks blocks;
// - the kept pair's ray is climbed;
// - bin sweep: every ray of every proposed bin at the few radii above the
//   kept one (64 / rays of the bin, at least one); the survivor of largest
//   key replaces the kept pair and its ray is climbed; the sweep goes on down
//   the ranking through the bins whose predicted radius comes within
//   kSweepMargin of the kept pair's;
// - sweep: the 16 rays around the kept pair's ray (-8..+7) at the 4 radii
//   above it; a survivor replaces the kept pair and its ray is climbed;
//   repeated up to kSweeps times while it finds one.
// Colours with a low logit, without a verified proposal, or (with a fallback)
// whose verified radius lies more than kShortfall below the largest predicted
// bin radius go to the exact fallback.  One wave per colour.

constexpr int kBins = 36;
constexpr int kDeltas = 6;
constexpr int kClimbBlocks = 8;
constexpr int kSweeps = 4;
constexpr float kSweepMargin = 5.0f;  // Delta E
constexpr float kShortfall = 10.0f;   // Delta E
__constant__ float kLadder[kDeltas] = {1.0f, 0.0f, -1.0f, -2.5f, -5.0f, -10.0f};

// Largest value over the wave, returned in every lane; the whole wave must be
// active.  Within each row of 16 lanes by DPP (swap neighbours, swap pairs,
// mirror within 8, mirror within 16), then the four rows' maxima read as
// scalars: no LDS round trips, unlike a shuffle tree.
__device__ __forceinline__ uint32_t wave_max_full(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
    const uint32_t r3 = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    return max(max(r0, r1), max(r2, r3));
}

// A float of a lane given by a wave-uniform index, as a scalar.
__device__ __forceinline__ float lane_float(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Exact predicate of candidate (i, j) for one lane; false when not live.
__device__ __forceinline__ bool verify_candidate(const ColorConst& cc, const Angles& ang, const Geom& g,
                                                 const RuleDev& rule, double ra, double rb, int32_t i,
                                                 int32_t j, bool live, bool cube) {
    double sn, co;
    ang.get(j, sn, co);
    const double rr = (double)(i + 1);
    float fp[3], fm[3];
    pair_linear_w(cc, g, (rr * ra) * sn, (rr * rb) * co, fp, fm, cube);
    const bool both = live && in_unit_cube(fp) && in_unit_cube(fm);
    const bool need = rule.clip ? live : both;
    bool ok = false;
    if (__ballot(need) != 0ull) {
        float Vp[3], Vm[3];
        codes_w(fp, fm, need, rule.clip != 0u, Vp, Vm);
        ok = need && accepts(rule, pattern_of(Vp, Vm, rule));
    }
    return ok;
}

// Largest verified key on ray j over radii i_start, i_start + 1, ... (at most
// kClimbBlocks blocks of 64, stopping at an empty block), merged into best.
// Wave-uniform arguments and result.
__device__ __forceinline__ uint32_t climb_ray(const ColorConst& cc, const Angles& ang, const Geom& g,
                                              const RuleDev& rule, double ra, double rb, int32_t nr,
                                              int32_t j, int32_t i_start, uint32_t best, bool cube) {
    const int lane = threadIdx.x & 63;
    for (int32_t blk = 0, i0 = i_start; blk < kClimbBlocks && i0 < nr; ++blk, i0 += 64) {
        const int32_t i = i0 + lane;
        const bool ok = verify_candidate(cc, ang, g, rule, ra, rb, min(i, nr - 1), j, i < nr, cube);
        const uint32_t top = wave_max_full(ok ? best_key(i, j) : 0u);
        if (top == 0u) break;
        best = max(best, top);
    }
    return best;
}

struct ProposeArgs {
    const ColorConst* cc;
    const uint64_t* n_dev;
    const float* pred;         // [n][37]
    TabArgs tab;
    Geom g;
    RuleDev rule;
    double ra, rb;
    float dr;
    int32_t nr, ntheta;
    float tau;
    int32_t kbins;
    int32_t shortfall;         // 1: a verified radius far below the prediction goes to the fallback
    cv_pattern_pair* pairs;    // [n]
    uint8_t* status;           // [n]
    uint32_t* need;            // [n]: 1 = exact fallback
};

__global__ __launch_bounds__(256, 6) void k_propose_verify(ProposeArgs a) {
    extern __shared__ double s_tab[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const Angles ang = load_angles(a.tab, s_tab);
    const int64_t n = (int64_t)*a.n_dev;
    const int64_t GW = (int64_t)gridDim.x * 4;
    for (int64_t c = (int64_t)blockIdx.x * 4 + (tid >> 6); c < n; c += GW) {
        const float* p = a.pred + c * (kBins + 1);
        const bool half = a.ntheta == a.tab.N;  // rank the first half-turn only
        const int nb = half ? kBins / 2 : kBins;
        float rk = -INFINITY;
        if (lane < nb) rk = half ? 25.0f * (p[lane] + p[lane + kBins / 2]) : 50.0f * p[lane];
        const float logit = p[kBins];
        const ColorConst cc = a.cc[c];
        // the cube branch of the inverse companding holds over the whole grid
        const bool cube = cube_branch_only(cc, a.nr - 1, a.ra, a.rb);
        uint32_t best = 0;
        float top_pred = 0.0f;  // the largest predicted bin radius (Delta E)
        if (logit >= a.tau) {
            // rank of every bin by predicted radius (ties: lower bin first)
            int rank = 0;
            for (int q = 0; q < nb; ++q) {
                const float rq = lane_float(rk, q);
                rank += (rq > rk || (rq == rk && q < lane)) ? 1 : 0;
            }
            const int kb = min(a.kbins, nb);
            top_pred = lane_float(rk, (int)__builtin_ctzll(__ballot(lane < nb && rank == 0)));
            for (int b = 0; b < kb; ++b) {
                const uint64_t sel = __ballot(lane < nb && rank == b);
                const int bin = (int)__builtin_ctzll(sel);
                const float rh = lane_float(rk, bin);
                // rays of the bin: floor(36 j / N) = bin
                const int32_t j_lo = (bin * a.tab.N + kBins - 1) / kBins;
                const int32_t j_hi = min(((bin + 1) * a.tab.N + kBins - 1) / kBins, a.ntheta);
                const int32_t nrays = j_hi - j_lo;
                if (nrays <= 0) continue;
                const int32_t ncand = nrays * kDeltas;
                uint32_t bb = 0;
                for (int32_t u0 = 0; u0 < ncand; u0 += 64) {
                    const int32_t u = u0 + lane;
                    const int32_t t = min(u / nrays, kDeltas - 1), q = u - (u / nrays) * nrays;
                    // radius r_i = (i + 1) dr nearest to the ladder point
                    const float rr_t = fminf(fmaxf((rh + kLadder[t]) / a.dr, 0.0f), 65536.0f);
                    const int32_t i = (int32_t)rintf(rr_t) - 1;
                    const int32_t j = j_lo + (u < ncand ? q : 0);
                    const bool live = u < ncand && i >= 0 && i < a.nr;
                    const bool ok = verify_candidate(cc, ang, a.g, a.rule, a.ra, a.rb, i, j, live, cube);
                    bb = max(bb, wave_max_full(ok ? best_key(i, j) : 0u));
                }
                best = max(best, bb);
            }
            if (best) {
                best = climb_ray(cc, ang, a.g, a.rule, a.ra, a.rb, a.nr, (int32_t)(0xFFFFu - (best & 0xFFFFu)),
                                 (int32_t)(best >> 16) + 1, best, cube);
                for (int b = 0; b < nb; ++b) {
                    const uint64_t sel = __ballot(lane < nb && rank == b);
                    const int bin = (int)__builtin_ctzll(sel);
                    // past the proposed bins, only those whose predicted radius
                    // comes within kSweepMargin of the kept one (ranks fall)
                    if (b >= kb && lane_float(rk, bin) + kSweepMargin <= (float)((best >> 16) + 1) * a.dr) break;
                    const int32_t j_lo = (bin * a.tab.N + kBins - 1) / kBins;
                    const int32_t j_hi = min(((bin + 1) * a.tab.N + kBins - 1) / kBins, a.ntheta);
                    const int32_t nrays = j_hi - j_lo;
                    if (nrays <= 0) continue;
                    const int32_t per = max(1, 64 / nrays), span = min(nrays, 64);
                    for (int32_t q0 = 0; q0 < nrays; q0 += span) {
                        const int32_t bi = (int32_t)(best >> 16);
                        const int32_t q = q0 + lane % span, i = bi + 1 + lane / span;
                        const bool live = lane < span * per && q < nrays && i < a.nr;
                        const int32_t j = j_lo + min(q, nrays - 1);
                        const bool ok = verify_candidate(cc, ang, a.g, a.rule, a.ra, a.rb, min(i, a.nr - 1), j,
                                                         live, cube);
                        const uint32_t top = wave_max_full(ok ? best_key(i, j) : 0u);
                        if (top == 0u) continue;
                        best = climb_ray(cc, ang, a.g, a.rule, a.ra, a.rb, a.nr,
                                         (int32_t)(0xFFFFu - (top & 0xFFFFu)), (int32_t)(top >> 16) + 1,
                                         max(best, top), cube);
                    }
                }
                // mirrors of the second half-turn never win the tie on j
                const int32_t jend = half ? a.tab.N / 2 : a.ntheta;
                for (int sw = 0; sw < kSweeps; ++sw) {
                    const int32_t bi = (int32_t)(best >> 16), bj = (int32_t)(0xFFFFu - (best & 0xFFFFu));
                    const int32_t j = bj + (lane & 15) - 8, i = bi + 1 + (lane >> 4);
                    const bool live = j >= 0 && j < jend && j != bj && i < a.nr;
                    const bool ok = verify_candidate(cc, ang, a.g, a.rule, a.ra, a.rb, min(i, a.nr - 1),
                                                     live ? j : bj, live, cube);
                    const uint32_t top = wave_max_full(ok ? best_key(i, j) : 0u);
                    if (top == 0u) break;
                    best = climb_ray(cc, ang, a.g, a.rule, a.ra, a.rb, a.nr, (int32_t)(0xFFFFu - (top & 0xFFFFu)),
                                     (int32_t)(top >> 16) + 1, max(best, top), cube);
                }
            }
        }
        // low confidence: with the exact search to fall back on, a verified
        // radius more than kShortfall below the network's largest prediction
        // is left to it (the network saw a better bin that was not found)
        if (a.shortfall && best && (float)((best >> 16) + 1) * a.dr < top_pred - kShortfall) best = 0;
        if (lane == 0) {
            cv_pattern_pair r = {};
            if (best) {
                const int32_t bi = (int32_t)(best >> 16), bj = (int32_t)(0xFFFFu - (best & 0xFFFFu));
                double sn, co;
                ang.get(bj, sn, co);
                const double rr = (double)(bi + 1);
                PairEval e;
                eval_pair(cc, a.g, (rr * a.ra) * sn, (rr * a.rb) * co, e);
                r.i = (uint16_t)bi;
                r.j = (uint16_t)bj;
                for (int k = 0; k < 3; ++k) {
                    r.plus[k] = (uint8_t)e.Vp[k];
                    r.minus[k] = (uint8_t)e.Vm[k];
                }
                r.pattern = (uint8_t)pattern_of(e.Vp, e.Vm, a.rule);
                r.flags = CV_PAIR_FOUND | CV_PAIR_SURROGATE;
            }
            a.pairs[c] = r;
            a.status[c] = best ? (uint8_t)CV_RESOLVED_SURROGATE : (uint8_t)CV_RESOLVED_NONE;
            a.need[c] = best ? 0u : 1u;
        }
    }
}

// Fallback list: colours with need = 1, in colour order.
__global__ void k_make_list(const uint32_t* __restrict__ need, const uint64_t* __restrict__ prefix,
                            const uint64_t* __restrict__ n_dev, uint32_t* __restrict__ list) {
    const int64_t n = (int64_t)*n_dev;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride)
        if (need[c]) list[prefix[c]] = (uint32_t)c;
}

// Two frames from one pair per colour.
// Two frames from one pair per colour (the surrogate's): aligned and idx16 as
// in k_render.
__global__ void k_render_pairs(const uint8_t* __restrict__ px, int64_t npix,
                               const uint32_t* __restrict__ index,
                               const cv_pattern_pair* __restrict__ pairs, uint8_t* __restrict__ fa,
                               uint8_t* __restrict__ fb, unsigned long long* __restrict__ resolved, bool aligned,
                               bool idx16) {
    uint32_t got = 0;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x, nq = npix >> 2;
    for (int64_t qd = t; qd < nq; qd += stride) {
        const Quad v = load_quad(px, qd, aligned);
        Quad QA = v, QB = v;
        uint32_t ks[4];
        if (idx16) {
            const uint4 u = *reinterpret_cast<const uint4*>(index + 4 * qd);
            ks[0] = u.x;
            ks[1] = u.y;
            ks[2] = u.z;
            ks[3] = u.w;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) ks[k] = index[4 * qd + k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const cv_pattern_pair& r = pairs[ks[k]];
            if (r.flags & CV_PAIR_FOUND) {
                for (int c = 0; c < 3; ++c) {
                    quad_set(QA, 3 * k + c, r.plus[c]);
                    quad_set(QB, 3 * k + c, r.minus[c]);
                }
                ++got;
            }
        }
        store_quad(fa, qd, QA, aligned);
        store_quad(fb, qd, QB, aligned);
    }
    if (t < (npix & 3)) {
        const int64_t p = 4 * nq + t;
        const cv_pattern_pair& r = pairs[index[p]];
        const bool ok = (r.flags & CV_PAIR_FOUND) != 0;
        for (int c = 0; c < 3; ++c) {
            fa[3 * p + c] = ok ? r.plus[c] : px[3 * p + c];
            fb[3 * p + c] = ok ? r.minus[c] : px[3 * p + c];
        }
        got += ok ? 1u : 0u;
    }
    const uint32_t s = wave_sum_u32(got);
    if ((threadIdx.x & 63u) == 0 && s && resolved) atomicAdd(resolved, (unsigned long long)s);
}

__global__ void k_set_u64(uint64_t* __restrict__ p, uint64_t v) { *p = v; }

// ---------------------------------------------------------------------------
// Host side.

namespace {

MatArgs frame_mat_args() {
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

unsigned grid_for(int64_t items, int per_block, unsigned cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)(g > cap ? cap : g);
}

template <typename Kern>
int launch_resolve_k(cv_context* ctx, Kern k, int block, size_t lds, const ResolveArgs& a, hipStream_t s) {
    int lds_max = 0;
    CV_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    if (lds + 512 > (size_t)lds_max)
        return fail(CV_EINVAL, "angle table and per-ray maxima need " + std::to_string(lds) +
                                   " bytes of LDS; this device has " + std::to_string(lds_max));
    int per_cu = 0;
    CV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, lds));
    if (per_cu < 1) per_cu = 1;
    hipLaunchKernelGGL(k, dim3((unsigned)(per_cu * ctx->num_cu)), dim3(block), lds, s, a);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

// LDS of a resolve variant: the angle tables and, with per-ray maxima, one
// array of W words per colour in flight in the block.
size_t resolve_lds(const ResolveArgs& a, bool rays, int variant) {
    const size_t per_colour = rays ? (size_t)a.W * 4 : 0;
    const int colours = variant == 0 ? 1 : (variant == 1 ? 4 : 8);
    return angle_lds_bytes(a.tab) + per_colour * colours;
}

template <bool SYM, bool RAYS, bool CELLS>
int launch_resolve_c(cv_context* ctx, const ResolveArgs& a, int variant, hipStream_t s) {
    const size_t lds = resolve_lds(a, RAYS, variant);
    switch (variant) {
    case 1: return launch_resolve_k(ctx, k_colour_resolve_w<SYM, RAYS, 256, CELLS>, 256, lds, a, s);
    case 2: return launch_resolve_k(ctx, k_colour_resolve_w<SYM, RAYS, 512, CELLS>, 512, lds, a, s);
    default: return launch_resolve_k(ctx, k_colour_resolve<SYM, RAYS, CELLS>, 256, lds, a, s);
    }
}

template <bool SYM, bool RAYS>
int launch_resolve_t(cv_context* ctx, const ResolveArgs& a, int variant, hipStream_t s) {
    return a.cells ? launch_resolve_c<SYM, RAYS, true>(ctx, a, variant, s)
                   : launch_resolve_c<SYM, RAYS, false>(ctx, a, variant, s);
}

// De-duplication: sorted distinct colours, their number (device, also in
// ctx->fmisc[0]) and each pixel's index.
int enqueue_dedupe(cv_context* ctx, const uint8_t* pixels, int64_t npix, uint8_t* colours,
                   uint32_t* pixel_index, int64_t* ncolours, hipStream_t s) {
    int rc;
    uint32_t* bits = (uint32_t*)ctx->fbits.ptr;
    uint32_t* cnt = (uint32_t*)ctx->fcnt.ptr;
    uint64_t* prefix = (uint64_t*)ctx->fprefix.ptr;
    uint64_t* misc = (uint64_t*)ctx->fmisc.ptr;  // [0] colour count
    hipLaunchKernelGGL(k_zero_words, dim3(1024), dim3(256), 0, s, (uint64_t*)bits, kCubeWords / 2);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, misc, (int64_t)8);
    const bool px4 = ((uintptr_t)pixels & 3u) == 0, idx16 = ((uintptr_t)pixel_index & 15u) == 0;
    hipLaunchKernelGGL(k_bitmap_mark, dim3(grid_for(npix, 256, 8192)), dim3(256), 0, s, pixels,
                       npix, bits);
    hipLaunchKernelGGL(k_bitmap_popc, dim3((unsigned)(kCubeWords / 256)), dim3(256), 0, s, bits, cnt);
    CV_HIP(hipGetLastError());
    if ((rc = run_scan_counts(ctx, cnt, kCubeWords, prefix, nullptr, 1, 0, misc, s)) != CV_OK)
        return rc;
    hipLaunchKernelGGL(k_bitmap_compact, dim3((unsigned)(kCubeWords / 256)), dim3(256), 0, s, bits,
                       prefix, colours);
    hipLaunchKernelGGL(k_pixel_index, dim3(grid_for((npix + 3) / 4, 256, 8192)), dim3(256), 0, s, pixels, npix,
                       bits, prefix, pixel_index, px4, idx16);
    hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(1), 0, s, misc, ncolours);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

// Angle table and per-colour constants of n_dev colours (at most cap).
int enqueue_prologue(cv_context* ctx, const GridDev& gd, const uint8_t* colours, int64_t cap,
                     const uint64_t* n_dev, hipStream_t s) {
    int rc;
    if ((rc = launch_angle_table((double*)ctx->table.ptr, gd.N, s)) != CV_OK) return rc;
    hipLaunchKernelGGL(k_prologue_dev, dim3(grid_for(cap, 256, 8192)), dim3(256), 0, s, colours, n_dev,
                       (ColorConst*)ctx->colors.ptr, frame_mat_args());
    CV_HIP(hipGetLastError());
    return CV_OK;
}

ResolveArgs resolve_args(cv_context* ctx, const GridDev& gd, const RuleDev& rd, const uint64_t* n_dev) {
    ResolveArgs a;
    a.cc = (const ColorConst*)ctx->colors.ptr;
    a.n_dev = n_dev;
    a.tab.tab = (const double*)ctx->table.ptr;
    a.tab.tab_len = gd.tab_len;
    a.tab.N = gd.N;
    a.tab.dW = direct_rays(gd.ntheta, gd.N, gd.tab_len, (size_t)gd.ntheta * 4);
    a.tab._pad = 0;
    a.g = geom_constants();
    a.rule = rd;
    a.ra = gd.ra;
    a.rb = gd.rb;
    a.nr = gd.nr;
    a.ntheta = gd.ntheta;
    const bool sym = gd.ntheta == gd.N;
    a.W = sym ? gd.N / 2 : gd.ntheta;
    a.inv_W = 1.0f / (float)a.W;
    a.si = 256 / a.W;
    a.sj = 256 % a.W;
    a.si64 = 64 / a.W;
    a.sj64 = 64 % a.W;
    a.list = nullptr;
    a.summ = nullptr;
    a.pbest = nullptr;
    a.rays = nullptr;
    // gamut cells as in the reduce kernel, with exact FP32 index splits
    a.cells = ctx->gamut_cells && !rd.clip && a.W >= kCellMinRays && (int64_t)(a.nr + kBandRows - 1) * a.W < (1 << 24) ? 1 : 0;
    a.need_ng = 1;
    a.stats = ctx->timing ? (uint64_t*)ctx->stats.ptr : nullptr;
    return a;
}

int launch_resolve(cv_context* ctx, const ResolveArgs& a, bool sym, int variant, hipStream_t s) {
    if (sym)
        return a.rays ? launch_resolve_t<true, true>(ctx, a, variant, s)
                      : launch_resolve_t<true, false>(ctx, a, variant, s);
    return a.rays ? launch_resolve_t<false, true>(ctx, a, variant, s)
                  : launch_resolve_t<false, false>(ctx, a, variant, s);
}

} // namespace

// Everything the call enqueues, in order, on stream s (also used for capture).
int FramesCall::enqueue(cv_context* ctx, hipStream_t s) const {
    int rc;
    uint64_t* misc = (uint64_t*)ctx->fmisc.ptr;  // [0] colour count
    if ((rc = enqueue_dedupe(ctx, pixels, npix, colours, pixel_index, ncolours, s)) != CV_OK) return rc;
    // the search of every distinct colour
    if ((rc = enqueue_prologue(ctx, gd, colours, colour_cap, misc, s)) != CV_OK) return rc;
    ResolveArgs a = resolve_args(ctx, gd, rd, misc);
    const bool sym = gd.ntheta == gd.N;
    a.summ = summ;
    a.pbest = pbest;
    a.rays = rays;
    a.need_ng = summ && !no_ngamut ? 1 : 0;
    if ((rc = ctx->mark(CV_TIME_EVAL, 0, s)) != CV_OK) return rc;
    if ((rc = launch_resolve(ctx, a, sym, variant, s)) != CV_OK) return rc;
    if ((rc = ctx->mark(CV_TIME_EVAL, 1, s)) != CV_OK) return rc;
    if (frame_a) {
        if (resolved)
            hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, (uint64_t*)resolved, (int64_t)1);
        hipLaunchKernelGGL(k_render, dim3(grid_for(npix, 256, 8192)), dim3(256), 0, s, pixels, npix,
                           pixel_index, info, pbest, summ, frame_a, frame_b,
                           (unsigned long long*)resolved);
    }
    CV_HIP(hipGetLastError());
    return CV_OK;
}

bool FramesCall::same(const FramesCall& o) const {
    return std::memcmp(this, &o, sizeof(FramesCall)) == 0;
}

uint64_t resolve_key(const GridDev& gd, bool rays) {
    return (uint64_t)(uint32_t)gd.nr | ((uint64_t)(uint32_t)gd.ntheta << 16) | ((uint64_t)(uint32_t)gd.N << 32) |
           ((uint64_t)(rays ? 1 : 0) << 48);
}

int resolve_variant(cv_context* ctx, const GridDev& gd, bool rays) {
    if (ctx->resolve_forced >= 0) return ctx->resolve_forced;
    const auto it = ctx->resolve_tuned.find(resolve_key(gd, rays));
    return it == ctx->resolve_tuned.end() ? 0 : it->second;
}

namespace {

// Time every resolve variant that fits in LDS on up to kTuneColours of the
// call's colours (their constants are in place after an eager call) and keep
// the fastest for this grid shape.  The runs rewrite the first outputs with
// the same values.
constexpr int64_t kTuneColours = 8192;

int tune_resolve(cv_context* ctx, const FramesCall& call, hipStream_t s) {
    CV_HIP(hipMemcpyAsync(ctx->host_misc, ctx->fmisc.ptr, 8, hipMemcpyDeviceToHost, s));
    CV_HIP(hipStreamSynchronize(s));
    const int64_t n = (int64_t)ctx->host_misc[0];
    const bool rays = call.rays != nullptr;
    const uint64_t key = resolve_key(call.gd, rays);
    if (n < 1) return CV_OK;  // nothing to time: keep the default, tune on a later call
    uint64_t* cnt = (uint64_t*)ctx->fmisc.ptr + 1;
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, cnt, (uint64_t)std::min(n, kTuneColours));
    CV_HIP(hipGetLastError());
    ResolveArgs a = resolve_args(ctx, call.gd, call.rd, cnt);
    a.summ = call.summ;
    a.pbest = call.pbest;
    a.rays = call.rays;
    a.need_ng = call.summ && !call.no_ngamut ? 1 : 0;
    const bool sym = call.gd.ntheta == call.gd.N;
    int lds_max = 0;
    CV_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CV_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    int rc = CV_OK, best_v = 0;
    float best_ms = 0.0f;
    for (int v = 0; v < kResolveVariants && rc == CV_OK; ++v) {
        if (resolve_lds(a, rays, v) + 512 > (size_t)lds_max) continue;
        if ((rc = launch_resolve(ctx, a, sym, v, s)) != CV_OK) break;  // warm-up
        float ms = 0.0f;
        if ((he = hipEventRecord(e0, s)) == hipSuccess && (rc = launch_resolve(ctx, a, sym, v, s)) == CV_OK &&
            (he = hipEventRecord(e1, s)) == hipSuccess && (he = hipEventSynchronize(e1)) == hipSuccess)
            he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) rc = hip_fail(he, "timing a resolve variant");
        if (rc == CV_OK && (v == 0 || ms < best_ms)) {
            best_ms = ms;
            best_v = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == CV_OK) {
        ctx->resolve_tuned[key] = best_v;
        rc = ctx->save_tuning();
    }
    return rc;
}

} // namespace

int run_frames_resolve(cv_context* ctx, const FramesCall& call_in, bool graph, hipStream_t s) {
    int rc;
    FramesCall call = call_in;
    // every allocation happens before any capture
    if ((rc = ctx->ensure(ctx->fbits, (size_t)kCubeWords * 4)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->fcnt, (size_t)kCubeWords * 4)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->fprefix, (size_t)kCubeWords * 8)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->fmisc, 64)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->scan, (size_t)((kCubeWords + 4095) / 4096) * 8)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->colors, (size_t)call.colour_cap * sizeof(ColorConst))) != CV_OK)
        return rc;
    if ((rc = ctx->ensure(ctx->table, (size_t)call.gd.tab_len * 8)) != CV_OK) return rc;
    const cvib::Buffer* ws[7] = {&ctx->fbits, &ctx->fcnt, &ctx->fprefix, &ctx->fmisc,
                                 &ctx->scan,  &ctx->colors, &ctx->table};
    for (int k = 0; k < 7; ++k) call.ws[k] = ws[k]->ptr;
    const bool rays = call.rays != nullptr;
    if (ctx->autotune && ctx->resolve_forced < 0 && !ctx->resolve_tuned.count(resolve_key(call.gd, rays))) {
        // one eager call (its outputs stand), then the variants are timed on it
        const bool timing = ctx->timing;
        ctx->timing = false;
        call.variant = 0;
        rc = call.enqueue(ctx, s);
        if (rc == CV_OK) rc = tune_resolve(ctx, call, s);
        ctx->timing = timing;
        if (rc != CV_OK) return rc;
    }
    call.variant = resolve_variant(ctx, call.gd, rays);
    call.cells = ctx->gamut_cells ? 1 : 0;
    if (!graph) {
        if ((rc = ctx->mark(CV_TIME_CALL, 0, s)) != CV_OK) return rc;
        if ((rc = call.enqueue(ctx, s)) != CV_OK) return rc;
        if ((rc = ctx->mark(CV_TIME_CALL, 1, s)) != CV_OK) return rc;
        if (ctx->timing) {
            CV_HIP(hipStreamSynchronize(s));
            if ((rc = ctx->collect()) != CV_OK) return rc;
        }
        return CV_OK;
    }
    if (!ctx->fgraph_exec || !ctx->fgraph_call.same(call)) {
        if (ctx->fgraph_exec) {
            CV_HIP(hipGraphExecDestroy(ctx->fgraph_exec));
            ctx->fgraph_exec = nullptr;
        }
        if (!ctx->cap_stream) CV_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        const bool timing = ctx->timing;
        ctx->timing = false;  // no timing events inside a captured graph
        hipGraph_t g = nullptr;
        CV_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        rc = call.enqueue(ctx, ctx->cap_stream);
        hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
        ctx->timing = timing;
        if (rc != CV_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&ctx->fgraph_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            ctx->fgraph_exec = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        ctx->fgraph_call = call;
    }
    if ((rc = ctx->mark(CV_TIME_CALL, 0, s)) != CV_OK) return rc;
    CV_HIP(hipGraphLaunch(ctx->fgraph_exec, s));
    if ((rc = ctx->mark(CV_TIME_CALL, 1, s)) != CV_OK) return rc;
    if (ctx->timing) {
        CV_HIP(hipStreamSynchronize(s));
        if ((rc = ctx->collect()) != CV_OK) return rc;
    }
    return CV_OK;
}

// ---------------------------------------------------------------------------
// Surrogate resolve, host side.

namespace {

int ensure_surrogate(cv_context* ctx, const SurrogateCall& c, int64_t n) {
    int rc;
    const int64_t m = n > 0 ? n : 1;
    if ((rc = ctx->ensure(ctx->colors, (size_t)m * sizeof(ColorConst))) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->table, (size_t)c.gd.tab_len * 8)) != CV_OK) return rc;
    if (!c.pred && (rc = ctx->ensure(ctx->spred, (size_t)m * 37 * sizeof(float))) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->sneed, (size_t)m * 4)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->sprefix, (size_t)m * 8)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->slist, (size_t)m * 4)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->smisc, 64)) != CV_OK) return rc;
    return CV_OK;
}

// The surrogate resolve of n colours whose count is also at n_dev.
int enqueue_surrogate(cv_context* ctx, const SurrogateCall& c, const uint8_t* rgb, int64_t n,
                      const uint64_t* n_dev, hipStream_t s) {
    int rc;
    uint64_t* smisc = (uint64_t*)ctx->smisc.ptr;  // [1] fallback count
    float* pred = c.pred ? c.pred : (float*)ctx->spred.ptr;
    if ((rc = enqueue_prologue(ctx, c.gd, rgb, n, n_dev, s)) != CV_OK) return rc;
    if (!c.pred_given) {
        if ((rc = ctx->mark(CV_TIME_MLP, 0, s)) != CV_OK) return rc;
        if ((rc = mlp_forward_rgb8(c.mlp, rgb, n, pred, s)) != CV_OK) return rc;
        if ((rc = ctx->mark(CV_TIME_MLP, 1, s)) != CV_OK) return rc;
    }
    ProposeArgs p;
    p.cc = (const ColorConst*)ctx->colors.ptr;
    p.n_dev = n_dev;
    p.pred = pred;
    p.tab.tab = (const double*)ctx->table.ptr;
    p.tab.tab_len = c.gd.tab_len;
    p.tab.N = c.gd.N;
    p.tab.dW = direct_rays(c.gd.ntheta, c.gd.N, c.gd.tab_len, 0);
    p.tab._pad = 0;
    p.g = geom_constants();
    p.rule = c.rd;
    p.ra = c.gd.ra;
    p.rb = c.gd.rb;
    p.dr = (float)c.gd.dr;
    p.nr = c.gd.nr;
    p.ntheta = c.gd.ntheta;
    p.tau = c.tau;
    p.kbins = c.kbins;
    p.shortfall = c.fallback ? 1 : 0;
    p.pairs = c.pairs;
    p.status = c.status;
    p.need = (uint32_t*)ctx->sneed.ptr;
    if ((rc = ctx->mark(CV_TIME_VERIFY, 0, s)) != CV_OK) return rc;
    int lds_max = 0;
    CV_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    if (angle_lds_bytes(p.tab) > (size_t)lds_max) return fail(CV_EINVAL, "angle table exceeds LDS");
    hipLaunchKernelGGL(k_propose_verify, dim3(grid_for(n, 4, 65536)), dim3(256),
                       angle_lds_bytes(p.tab), s, p);
    CV_HIP(hipGetLastError());
    if ((rc = ctx->mark(CV_TIME_VERIFY, 1, s)) != CV_OK) return rc;
    // colours without a verified proposal, counted (and listed) in colour order
    uint64_t* prefix = (uint64_t*)ctx->sprefix.ptr;
    uint32_t* list = c.fallback_list ? c.fallback_list : (uint32_t*)ctx->slist.ptr;
    if ((rc = run_scan_counts(ctx, (const uint32_t*)ctx->sneed.ptr, n, prefix, nullptr, 1, 0, smisc + 1,
                              s)) != CV_OK)
        return rc;
    if (c.fallback || c.fallback_list) {
        hipLaunchKernelGGL(k_make_list, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s,
                           (const uint32_t*)ctx->sneed.ptr, prefix, n_dev, list);
        CV_HIP(hipGetLastError());
    }
    if (c.fallback) {
        // the exact maximum-amplitude pair of each listed colour: the one-pair
        // search with a global early exit (cvib_rays.hip)
        if ((rc = ctx->mark(CV_TIME_EVAL, 0, s)) != CV_OK) return rc;
        if ((rc = run_best_pair_list(ctx, c.gd, c.rd, list, smisc + 1, n, c.pairs, c.status, s)) != CV_OK) return rc;
        if ((rc = ctx->mark(CV_TIME_EVAL, 1, s)) != CV_OK) return rc;
    }
    if (c.nfallback) hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(1), 0, s, smisc + 1, c.nfallback);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

} // namespace

int run_surrogate(cv_context* ctx, const SurrogateCall& c, hipStream_t s) {
    int rc;
    if (c.n == 0) {
        if (c.nfallback) {
            if ((rc = ctx->ensure(ctx->smisc, 64)) != CV_OK) return rc;
            hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, (uint64_t*)c.nfallback, (int64_t)1);
            CV_HIP(hipGetLastError());
        }
        return CV_OK;
    }
    if ((rc = ensure_surrogate(ctx, c, c.n)) != CV_OK) return rc;
    uint64_t* smisc = (uint64_t*)ctx->smisc.ptr;
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, smisc, (uint64_t)c.n);
    CV_HIP(hipGetLastError());
    if ((rc = ctx->mark(CV_TIME_CALL, 0, s)) != CV_OK) return rc;
    if ((rc = enqueue_surrogate(ctx, c, c.rgb, c.n, smisc, s)) != CV_OK) return rc;
    if ((rc = ctx->mark(CV_TIME_CALL, 1, s)) != CV_OK) return rc;
    if (ctx->timing) {
        CV_HIP(hipStreamSynchronize(s));
        if ((rc = ctx->collect()) != CV_OK) return rc;
    }
    return CV_OK;
}

int run_frames_surrogate(cv_context* ctx, const SurrogateCall& c, const uint8_t* pixels, int64_t npix,
                         uint8_t* colours, int64_t colour_cap, int64_t* ncolours,
                         uint32_t* pixel_index, uint8_t* frame_a, uint8_t* frame_b,
                         int64_t* resolved, hipStream_t s) {
    int rc;
    if ((rc = ctx->ensure(ctx->fbits, (size_t)kCubeWords * 4)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->fcnt, (size_t)kCubeWords * 4)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->fprefix, (size_t)kCubeWords * 8)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->fmisc, 64)) != CV_OK) return rc;
    if ((rc = ctx->mark(CV_TIME_CALL, 0, s)) != CV_OK) return rc;
    if ((rc = enqueue_dedupe(ctx, pixels, npix, colours, pixel_index, ncolours, s)) != CV_OK) return rc;
    // the network runs on exactly the distinct colours: read their number
    CV_HIP(hipMemcpyAsync(ctx->host_misc, ctx->fmisc.ptr, 8, hipMemcpyDeviceToHost, s));
    CV_HIP(hipStreamSynchronize(s));
    const int64_t n = (int64_t)ctx->host_misc[0];
    if (n < 1 || n > colour_cap) return fail(CV_ESTATE, "internal: distinct colour count");
    if ((rc = ensure_surrogate(ctx, c, n)) != CV_OK) return rc;
    if ((rc = enqueue_surrogate(ctx, c, colours, n, (const uint64_t*)ctx->fmisc.ptr, s)) != CV_OK)
        return rc;
    if (frame_a) {
        if (resolved)
            hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, (uint64_t*)resolved, (int64_t)1);
        const bool al = (((uintptr_t)pixels | (uintptr_t)frame_a | (uintptr_t)frame_b) & 3u) == 0;
        hipLaunchKernelGGL(k_render_pairs, dim3(grid_for((npix + 3) / 4, 256, 8192)), dim3(256), 0, s, pixels,
                           npix, pixel_index, (const cv_pattern_pair*)c.pairs, frame_a, frame_b,
                           (unsigned long long*)resolved, al, ((uintptr_t)pixel_index & 15u) == 0);
        CV_HIP(hipGetLastError());
    }
    if ((rc = ctx->mark(CV_TIME_CALL, 1, s)) != CV_OK) return rc;
    if (ctx->timing) {
        CV_HIP(hipStreamSynchronize(s));
        if ((rc = ctx->collect()) != CV_OK) return rc;
    }
    return CV_OK;
}

} // namespace cvib
