// Several rules in one pass over the candidates (Table 1 lists twelve
// (V_th, R_novib) settings; Table 2 is the presence of each pattern under any
// of them).
//
// A rule classifies the change d of a channel (an integer 0..255) as high
// (d > v_th), low (d <= lo_max) or neither.  All rules' thresholds together
// cut 0..255 into at most 13 intervals in which every rule's class is
// constant, so a candidate is fully described, for every rule at once, by the
// interval index of its three channel changes.  The pass therefore builds,
// per colour, a histogram of in-gamut candidates over the (at most 13^3)
// interval triples, with one LDS table read per channel and one LDS atomic
// per candidate; a small finalize maps each triple to the pattern (or none)
// of every rule.  The counts are exact.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "cvib_internal.h"
#include "cvib_kernels.h"

namespace cvib {

int prepare_colours(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd, hipStream_t s,
                    TabArgs& tab);

namespace {

constexpr int kMaxRules = 16;
constexpr int kMaxBreaks = 12;         // distinct thresholds
constexpr int kMaxBins = 13 * 13 * 13;  // interval triples
constexpr int kRulesBlock = 512;
constexpr int64_t kMaxRuleColours = 65536;  // histogram of 13^3 words per colour

struct RulesArgs {
    const ColorConst* cc;
    TabArgs tab;
    Geom g;
    uint32_t clip;
    int32_t nint;              // intervals per channel
    double ra, rb;
    int32_t nr, W;
    float inv_W;
    int32_t si, sj;            // a step of one block = si rows + sj rays
    int32_t chunk;             // evaluations per tile
    int32_t tiles_per_colour;
    int64_t ntiles;
    uint64_t* ticket;
    const uint8_t* lut;        // [256]: interval of a change d
    uint32_t* hist;            // [n][nint^3]
    uint32_t mult;             // 2 when only half a turn is evaluated
    RuleDev low;               // v_th: the smallest threshold of the rules (for the high-channel cells)
};

// With CELLS each wave first decides 64 of its steps at a time (one per lane)
// and evaluates only those that may hold a pair in gamut with a channel
// changing by more than the smallest threshold of the rules: a pair without
// such a channel has no accepted pattern under any rule, so its bin adds to no
// count (the histogram itself is not an output).
template <bool SYM, bool CELLS>
__global__ __launch_bounds__(kRulesBlock) void k_rule_hist(RulesArgs a) {
    extern __shared__ double s_dyn[];
    __shared__ uint32_t s_hist[kMaxBins];
    __shared__ uint32_t s_lut[256];
    __shared__ int64_t s_tick;
    const int tid = threadIdx.x;
    const uint32_t lane = (uint32_t)tid & 63u;
    const Angles ang = load_angles(a.tab, s_dyn);
    for (int k = tid; k < 256; k += kRulesBlock) s_lut[k] = a.lut[k];
    const int32_t nbins = a.nint * a.nint * a.nint;
    const bool clip = a.clip != 0u;
    for (;;) {
        if (tid == 0) s_tick = (int64_t)atomicAdd((unsigned long long*)a.ticket, 1ull);
        for (int k = tid; k < nbins; k += kRulesBlock) s_hist[k] = 0;
        __syncthreads();
        const int64_t t = uniform_i64(s_tick);
        if (t >= a.ntiles) break;
        const int64_t c = t / a.tiles_per_colour;
        const int32_t lt = (int32_t)(t - c * a.tiles_per_colour);
        const ColorConst cc = a.cc[c];
        const int32_t begin = lt * a.chunk;
        const int32_t len = min(a.chunk, a.nr * a.W - begin);
        const int32_t row0 = begin / a.W, jb0 = begin - row0 * a.W;
        const int32_t iters = (len + kRulesBlock - 1) / kRulesBlock;
        auto step = [&](int32_t i, int32_t j, bool live) {
            double sn, co;
            ang.get(j, sn, co);
            const double rr = (double)(i + 1);
            float fp[3], fm[3];
            pair_linear_w(cc, a.g, (rr * a.ra) * sn, (rr * a.rb) * co, fp, fm);
            const bool need = clip ? live : (live && in_unit_cube(fp) && in_unit_cube(fm));
            if (__ballot(need) != 0ull) {
                float Vp[3], Vm[3];
                codes_w(fp, fm, need, clip, Vp, Vm);
                uint32_t bin = 0;
                if (need) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const uint32_t d = (uint32_t)fabsf(Vp[k] - Vm[k]);
                        bin = bin * (uint32_t)a.nint + s_lut[d];
                    }
                }
                // lanes of one bin add together: a wave holds few distinct bins
                uint64_t rem = __ballot(need);
                while (rem) {
                    const uint32_t b0 = (uint32_t)__shfl((int)bin, __builtin_ctzll(rem), 64);
                    const uint64_t same = __ballot(bin == b0) & rem;
                    if (lane == (uint32_t)__builtin_ctzll(rem))
                        atomicAdd(&s_hist[b0], (uint32_t)__builtin_popcountll(same));
                    rem &= ~same;
                }
            }
        };
        if constexpr (CELLS) {
            const int32_t wb = tid - (int32_t)lane;  // the wave's first evaluation of a step
            for (int32_t word = 0; word < (iters + 63) >> 6; ++word) {
                const int32_t itl = word * 64 + (int32_t)lane, e0 = itl * kRulesBlock + wb;
                const bool any = itl < iters && e0 < len;
                bool high = true;
                const bool open = step_open(cc, a.g, ang, a.ra, a.rb, a.W, a.inv_W, row0, jb0, min(e0, len - 1),
                                            min(e0 + 63, len - 1), any, false, &a.low, &high);
                uint64_t m = uniform_u64(__ballot(open && high));
                while (m) {
                    const int32_t e = (word * 64 + (int32_t)__builtin_ctzll(m)) * kRulesBlock + tid;
                    m &= m - 1ull;
                    int32_t i, j;
                    divmod_small(jb0 + min(e, len - 1), a.W, a.inv_W, i, j);
                    step(i + row0, j, e < len);
                }
            }
        } else {
            int32_t i, j;
            divmod_small(jb0 + tid, a.W, a.inv_W, i, j);
            i += row0;
            for (int32_t it = 0; it < iters; ++it) {
                step(i, j, it * kRulesBlock + tid < len);
                j += a.sj;
                i += a.si;
                if (j >= a.W) { j -= a.W; ++i; }
            }
        }
        __syncthreads();
        uint32_t* dst = a.hist + c * (int64_t)nbins;
        for (int k = tid; k < nbins; k += kRulesBlock)
            if (s_hist[k]) atomicAdd(&dst[k], a.mult * s_hist[k]);
        __syncthreads();
    }
}

// counts[c][r][p-1] from the histogram: block per colour, threads over bins.
// cls[r][t]: class of interval t under rule r (0 low, 1 high, 2 neither);
// masks[r]: the rule's accepted patterns.
__global__ __launch_bounds__(256) void k_rule_counts(const uint32_t* __restrict__ hist, int64_t n,
                                                     int32_t nint, int32_t nrules,
                                                     const uint8_t* __restrict__ cls,
                                                     const uint32_t* __restrict__ masks,
                                                     uint32_t* __restrict__ counts) {
    __shared__ uint32_t s_cnt[kMaxRules * 7];
    const int32_t nbins = nint * nint * nint;
    for (int64_t c = blockIdx.x; c < n; c += gridDim.x) {
        for (int k = threadIdx.x; k < kMaxRules * 7; k += blockDim.x) s_cnt[k] = 0;
        __syncthreads();
        const uint32_t* h = hist + c * (int64_t)nbins;
        for (int32_t b = threadIdx.x; b < nbins; b += blockDim.x) {
            const uint32_t v = h[b];
            if (!v) continue;
            const int32_t tR = b / (nint * nint), tG = (b / nint) % nint, tB = b % nint;
            for (int32_t r = 0; r < nrules; ++r) {
                const uint8_t* cr = cls + r * nint;
                const uint32_t cR = cr[tR], cG = cr[tG], cB = cr[tB];
                if (cR == 2u || cG == 2u || cB == 2u) continue;
                const uint32_t p = 4u * cR + 2u * cG + cB;
                if (p != 0u && ((masks[r] >> (p - 1u)) & 1u)) atomicAdd(&s_cnt[r * 7 + (int)p - 1], v);
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nrules * 7; k += blockDim.x) counts[c * nrules * 7 + k] = s_cnt[k];
        __syncthreads();
    }
}

__global__ void k_zero_u32(uint32_t* __restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = 0;
}

} // namespace

int run_pair_reduce_rules(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd,
                          const RuleDev* rules, int32_t nrules, uint32_t* counts, hipStream_t s) {
    if (n == 0) return CV_OK;
    if (n > kMaxRuleColours) return fail(CV_EINVAL, "at most 65536 colours per multi-rule call");
    if (nrules < 1 || nrules > kMaxRules) return fail(CV_EINVAL, "nrules must be in [1, 16]");
    for (int r = 1; r < nrules; ++r)
        if (rules[r].clip != rules[0].clip) return fail(CV_EINVAL, "all rules need the same gamut reading");
    // the intervals: 0..255 cut after every threshold (d <= lo_max, d <= v_th)
    std::vector<int> breaks;
    for (int r = 0; r < nrules; ++r) {
        breaks.push_back((int)rules[r].lo_max);
        breaks.push_back((int)rules[r].v_th);
    }
    std::sort(breaks.begin(), breaks.end());
    breaks.erase(std::unique(breaks.begin(), breaks.end()), breaks.end());
    breaks.erase(std::remove_if(breaks.begin(), breaks.end(), [](int b) { return b < 0 || b >= 255; }),
                 breaks.end());
    if ((int)breaks.size() > kMaxBreaks)
        return fail(CV_EINVAL, "the rules have more than 12 distinct thresholds");
    const int32_t nint = (int32_t)breaks.size() + 1;
    // host tables: interval of each d, class of each interval under each rule
    std::vector<uint8_t> host(256 + kMaxRules * 13 + 4 * kMaxRules, 0);
    for (int d = 0; d < 256; ++d) {
        int t = 0;
        while (t < (int)breaks.size() && d > breaks[t]) ++t;
        host[d] = (uint8_t)t;
    }
    for (int r = 0; r < nrules; ++r)
        for (int t = 0; t < nint; ++t) {
            const int d = t < (int)breaks.size() ? breaks[t] : 255;  // every d of interval t classes alike
            const uint8_t cl = (float)d > rules[r].v_th ? 1 : ((float)d <= rules[r].lo_max ? 0 : 2);
            host[256 + r * nint + t] = cl;
        }
    uint32_t* masks = reinterpret_cast<uint32_t*>(host.data() + 256 + kMaxRules * 13);
    for (int r = 0; r < nrules; ++r) masks[r] = rules[r].mask;
    int rc;
    TabArgs tab;
    if ((rc = prepare_colours(ctx, rgb, n, gd, s, tab)) != CV_OK) return rc;
    const bool sym = gd.ntheta == gd.N;
    const int32_t W = sym ? gd.N / 2 : gd.ntheta;
    const int64_t per = (int64_t)gd.nr * W;
    const int32_t nbins = nint * nint * nint;
    if ((rc = ctx->ensure(ctx->rtab, host.size())) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->rhist, (size_t)n * nbins * 4)) != CV_OK) return rc;
    if ((rc = ctx->ensure(ctx->misc, 64)) != CV_OK) return rc;
    CV_HIP(hipMemcpyAsync(ctx->rtab.ptr, host.data(), host.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_zero_u32, dim3(1024), dim3(256), 0, s, (uint32_t*)ctx->rhist.ptr, n * (int64_t)nbins);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, (uint32_t*)ctx->misc.ptr, (int64_t)16);
    CV_HIP(hipGetLastError());
    // tiles: about 8 per CU in flight, at least 16 block steps each
    int64_t want = std::max<int64_t>(1, (int64_t)ctx->num_cu * 8 / n);
    int64_t chunk = (per + want - 1) / want;
    chunk = std::max<int64_t>(chunk, 16 * kRulesBlock);
    chunk = (chunk + kRulesBlock - 1) / kRulesBlock * kRulesBlock;
    chunk = std::min<int64_t>(chunk, per);
    RulesArgs a;
    a.cc = (const ColorConst*)ctx->colors.ptr;
    a.tab = tab;
    a.g = geom_constants();
    a.clip = rules[0].clip;
    a.nint = nint;
    a.ra = gd.ra;
    a.rb = gd.rb;
    a.nr = gd.nr;
    a.W = W;
    a.inv_W = 1.0f / (float)W;
    a.si = kRulesBlock / W;
    a.sj = kRulesBlock % W;
    a.chunk = (int32_t)chunk;
    a.tiles_per_colour = (int32_t)((per + chunk - 1) / chunk);
    a.ntiles = (int64_t)a.tiles_per_colour * n;
    a.ticket = (uint64_t*)ctx->misc.ptr;
    a.lut = (const uint8_t*)ctx->rtab.ptr;
    a.hist = (uint32_t*)ctx->rhist.ptr;
    a.mult = sym ? 2u : 1u;
    a.low = rules[0];
    for (int32_t r = 1; r < nrules; ++r) a.low.v_th = std::min(a.low.v_th, rules[r].v_th);
    const bool cells = ctx->gamut_cells && !a.clip && W >= kCellMinRays;
    auto k = sym ? (cells ? k_rule_hist<true, true> : k_rule_hist<true, false>)
                 : (cells ? k_rule_hist<false, true> : k_rule_hist<false, false>);
    const size_t lds = angle_lds_bytes(tab);
    hipFuncAttributes fa;
    CV_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k)));
    int lds_max = 0;
    CV_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    if (lds + fa.sharedSizeBytes > (size_t)lds_max)
        return fail(CV_EINVAL, "this grid needs " + std::to_string(lds + fa.sharedSizeBytes) +
                                   " bytes of LDS per block; the device has " + std::to_string(lds_max));
    int per_cu = 0;
    CV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kRulesBlock, lds));
    if (per_cu < 1) per_cu = 1;
    const int64_t grid = std::min<int64_t>((int64_t)per_cu * ctx->num_cu, a.ntiles);
    if ((rc = ctx->mark(CV_TIME_EVAL, 0, s)) != CV_OK) return rc;
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kRulesBlock), lds, s, a);
    CV_HIP(hipGetLastError());
    if ((rc = ctx->mark(CV_TIME_EVAL, 1, s)) != CV_OK) return rc;
    const uint8_t* dev = (const uint8_t*)ctx->rtab.ptr;
    hipLaunchKernelGGL(k_rule_counts, dim3((unsigned)std::min<int64_t>(n, 65536)), dim3(256), 0, s,
                       (const uint32_t*)ctx->rhist.ptr, n, nint, nrules, dev + 256,
                       (const uint32_t*)(dev + 256 + kMaxRules * 13), counts);
    CV_HIP(hipGetLastError());
    if (ctx->timing) {
        CV_HIP(hipStreamSynchronize(s));
        if ((rc = ctx->collect()) != CV_OK) return rc;
    }
    return CV_OK;
}

} // namespace cvib
