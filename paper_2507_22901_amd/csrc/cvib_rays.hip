// Adaptive per-ray search (gfx950): for every colour and every ray j, the
// largest radius index i whose pair passes Section 3's predicate, without
// evaluating the whole ray.
//
// The paper notes how large the search space is (Section 1) and evaluates
// every displaced pair of Section 2's arrays.  Along one ray the pair moves
// continuously with the radius, so a block of consecutive radii can often be
// settled as a whole: interval bounds on its linear channels show either that
// one colour leaves the gamut throughout the block, or that no channel can
// change by more than V_th there (so no pattern can be encoded).  A ray is
// taken from its outermost radius inward in blocks of 64: a coarse pass proves
// blocks empty, and only the blocks it cannot close are refined, by evaluating
// all their candidates with the exact predicate; the first survivor found is
// the ray's maximum and ends the ray.  The maximum is therefore the one the
// exhaustive search finds, bit for bit (same arithmetic on every candidate
// that is evaluated), while most candidates are never evaluated.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>

#include "cvib_internal.h"
#include "cvib_kernels.h"

namespace cvib {

// Per-colour constants and the angle table of a call (cvib_search.hip).
int prepare_colours(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd, hipStream_t s,
                    TabArgs& tab);

namespace {

constexpr int kRayBlock = 256;   // threads per block: 4 waves, one task each at a time
constexpr int kRowsPerBlock = 64;  // radii per row block (one lane each when refined)

struct RayArgs {
    const ColorConst* cc;
    TabArgs tab;
    Geom g;
    RuleDev rule;
    double ra, rb;
    int32_t nr, ntheta;
    int32_t W;                // rays evaluated per colour (N / 2 in half-turn mode)
    int32_t nb;               // row blocks per ray, numbered from the outermost
    int32_t rays_per_task;    // rays one wave takes at once: 64 / nb, at least 1
    int32_t tasks_per_colour;
    int32_t sym;              // ray j + W is ray j with + and - swapped
    int32_t proofs;           // interval proofs on (not under the clip reading)
    int64_t ntasks;
    uint16_t* rays;           // [n][ntheta]: largest valid i + 1, 0 = none
    cv_pair* recs;            // nullable [n][ntheta]: the pair at that radius, zero where none
    unsigned long long* counts;  // nullable [3]: candidates evaluated, blocks tested, blocks closed
    uint32_t* best;           // nullable [n]: the colour's largest key (i << 16 | 0xFFFF - j), zeroed before
    cv_pair* pairs;           // k_best_pair, nullable [n]: the pair of that key (flags 0 where none)
    int64_t n;                // k_best_pair: colours (with n_dev: an upper bound of *n_dev)
    // k_best_pair over a list (the surrogate's exact fallback): colour list[k]
    // for k < *n_dev, its pair to ppairs[colour] and status[colour]
    const uint32_t* list;
    const uint64_t* n_dev;
    cv_pattern_pair* ppairs;
    uint8_t* status;
};

__device__ __forceinline__ void store_ray(const RayArgs& a, int64_t c, int32_t j, uint32_t best,
                                          uint32_t lo, uint32_t hi) {
    const int64_t o = c * a.ntheta + j;
    a.rays[o] = (uint16_t)best;
    if (a.sym) a.rays[o + a.W] = (uint16_t)best;
    if (a.recs) {
        uint32_t* r = reinterpret_cast<uint32_t*>(a.recs + o);
        const uint32_t w0 = (uint32_t)c, w1 = best ? ((best - 1u) | ((uint32_t)j << 16)) : 0u;
        r[0] = w0;
        r[1] = w1;
        r[2] = best ? lo : 0u;
        r[3] = best ? hi : 0u;
        if (a.sym) {
            uint32_t mlo = 0, mhi = 0;
            if (best) mirror_pair(lo, hi, mlo, mhi);
            uint32_t* m = reinterpret_cast<uint32_t*>(a.recs + o + a.W);
            m[0] = w0;
            m[1] = best ? ((best - 1u) | ((uint32_t)(j + a.W) << 16)) : 0u;
            m[2] = mlo;
            m[3] = mhi;
        }
    }
}

__global__ __launch_bounds__(kRayBlock) void k_ray_search(RayArgs a) {
    extern __shared__ double s_dyn[];
    const Angles ang = load_angles(a.tab, s_dyn);
    const uint32_t lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * kRayBlock + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * kRayBlock) >> 6;
    const bool clip = a.rule.clip != 0u;
    const int32_t nbs = a.nb < 64 ? a.nb : 64;          // blocks of one ray per sweep
    const int32_t sweeps = (a.nb + 63) / 64;
    const uint64_t ray_bits = nbs == 64 ? ~0ull : ((1ull << nbs) - 1ull);
    uint64_t evald = 0, tested = 0, closed = 0;

    for (int64_t t = wave; t < a.ntasks; t += nwaves) {
        const int64_t c = t / a.tasks_per_colour;
        const int32_t j0 = (int32_t)(t - c * a.tasks_per_colour) * a.rays_per_task;
        const int32_t R = min(a.rays_per_task, a.W - j0);
        const ColorConst cc = a.cc[c];
        const bool cube = cube_branch_only(cc, a.nr - 1, a.ra, a.rb);
        uint64_t done = 0;  // rays of the task already settled (bit r)
        for (int32_t sw = 0; sw < sweeps; ++sw) {
            // coarse pass: lane -> (ray r, block b), one interval proof each
            const int32_t r = (int32_t)lane / nbs, b = sw * 64 + (int32_t)lane % nbs;
            const bool live = r < R && b < a.nb && !((done >> r) & 1ull);
            bool open = live;
            if (a.proofs) {
                const int32_t rr = live ? r : 0, bb = live ? b : 0;
                const int32_t hi_i = a.nr - 1 - kRowsPerBlock * bb;
                const int32_t lo_i = max(hi_i - (kRowsPerBlock - 1), 0);
                double s, co;
                ang.get(j0 + rr, s, co);
                bool high = true;
                const int32_t j = j0 + rr;
                const bool out = cell_out_of_gamut_ends(cc, a.g, ang.N, a.ra, a.rb, lo_i, hi_i, j, j, s, co, s,
                                                        co, &a.rule, &high);
                open = live && !out && high;
            }
            const uint64_t lm = __ballot(live), om = uniform_u64(__ballot(open));
            tested += (uint64_t)__builtin_popcountll(lm);
            closed += (uint64_t)__builtin_popcountll(lm & ~om);
            // refinement: each ray's open blocks from the outermost inward
            for (int32_t q = 0; q < R; ++q) {
                if ((done >> q) & 1ull) continue;
                uint64_t m = (om >> (q * nbs)) & ray_bits;
                const int32_t j = j0 + q;
                double s, co;
                ang.get(j, s, co);
                while (m) {
                    const int32_t bb = sw * 64 + (int32_t)__builtin_ctzll(m);
                    m &= m - 1ull;
                    const int32_t i = a.nr - 1 - kRowsPerBlock * bb - (int32_t)lane;  // lane 0 outermost
                    const bool lv = i >= 0;
                    const double rad = (double)(lv ? i + 1 : 1);
                    float fp[3], fm[3];
                    pair_linear_w(cc, a.g, (rad * a.ra) * s, (rad * a.rb) * co, fp, fm, cube);
                    const uint64_t live_m = __ballot(lv);
                    evald += (uint64_t)__builtin_popcountll(live_m);
                    const bool gp = in_unit_cube(fp), gm = in_unit_cube(fm);
                    const uint64_t need_m = clip ? live_m : (__ballot(gp && gm) & live_m);
                    if (need_m == 0ull) continue;
                    float Vp[3], Vm[3];
                    codes_w(fp, fm, (need_m >> lane) & 1ull, clip, Vp, Vm);
                    const PatMasks pm = pattern_masks(Vp, Vm, a.rule);
                    const uint64_t surv = uniform_u64(accepted_lanes(pm, a.rule.mask) & need_m);
                    if (surv == 0ull) continue;
                    const uint32_t first = (uint32_t)__builtin_ctzll(surv);  // largest i
                    if (lane == first) {
                        uint32_t lo, hi;
                        const uint32_t flags = 4u | (gp ? 1u : 0u) | (gm ? 2u : 0u);
                        pack_pair(Vp, Vm, pattern_of(Vp, Vm, a.rule), flags, lo, hi);
                        store_ray(a, c, j, (uint32_t)(i + 1), lo, hi);
                        // the mirrored ray j + W has the same i and a larger j: never the better key
                        if (a.best) atomicMax(&a.best[c], best_key(i, j));
                    }
                    done |= 1ull << q;
                    break;
                }
            }
        }
        // rays with no survivor
        if ((int32_t)lane < R && !((done >> lane) & 1ull)) store_ray(a, c, j0 + (int32_t)lane, 0u, 0u, 0u);
    }
    if (a.counts && lane == 0) {
        if (evald) atomicAdd(&a.counts[0], (unsigned long long)evald);
        if (tested) atomicAdd(&a.counts[1], (unsigned long long)tested);
        if (closed) atomicAdd(&a.counts[2], (unsigned long long)closed);
    }
}

// Exact one-pair resolve with a global early exit: the maximum-amplitude pair
// (largest i, then smallest j) of every colour.  One wave per colour takes the
// levels of 64 radii from the outermost inward; eight levels by eight angular
// sectors are first proven as coarse cells, then at each level every ray of
// an open sector has its block proven empty where the interval bound can
// (lane -> ray), and the open ones are evaluated with the search's arithmetic
// (lane -> radius, lane 0 outermost), each only above the largest i found so
// far at that level.  The
// first level with a survivor holds the colour's largest i, so the walk stops
// there; the key is then the exhaustive search's best, bit for bit.  The
// mirrored rays of the half-turn hold the same radii at larger j: never better.
// Six waves per SIMD (80 registers; a 20-byte spill reloaded per colour) run
// faster than the five that its unbounded allocation (91) would allow.
__global__ __launch_bounds__(kRayBlock, 6) void k_best_pair(RayArgs a) {
    extern __shared__ double s_dyn[];
    const Angles ang = load_angles(a.tab, s_dyn);
    const int64_t wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * kRayBlock + threadIdx.x) >> 6));
    const int64_t nwaves = ((int64_t)gridDim.x * kRayBlock) >> 6;
    const bool clip = a.rule.clip != 0u;
    uint64_t evald = 0, tested = 0, closed = 0;
    const int64_t n = a.n_dev ? (int64_t)*a.n_dev : a.n;
    for (int64_t k = wave; k < n; k += nwaves) {
        const uint32_t lane = lane_id_fresh();  // taken afresh per colour (nothing derived from it held across)
        const int64_t c = a.list ? (int64_t)a.list[k] : k;
        const ColorConst cc = a.cc[c];
        const bool cube = cube_branch_only(cc, a.nr - 1, a.ra, a.rb);
        uint32_t best = 0, blo = 0, bhi = 0;  // the same in every lane
        uint64_t cells = ~0ull;               // coarse cells of the current eight levels (bit 8 level + sector)
        for (int32_t bb = 0; bb < a.nb && best == 0u; ++bb) {
            const int32_t hi_i = a.nr - 1 - kRowsPerBlock * bb;
            const int32_t lo_i = max(hi_i - (kRowsPerBlock - 1), 0);
            if (a.proofs && (bb & 7) == 0) {
                // Coarse cells of levels bb .. bb + 7: lane -> (level bb + lane / 8,
                // sector lane % 8 of the rays, those j with 8 j / W = sector),
                // one interval proof each; a level whose sectors are all proven
                // is skipped, and a step of 64 rays that all lie in proven
                // sectors takes no per-ray proof.
                const int32_t lv = bb + ((int32_t)lane >> 3), sec = (int32_t)lane & 7;
                const int32_t js0 = (sec * a.W + 7) >> 3, js1 = ((sec + 1) * a.W + 7) / 8 - 1;
                const int32_t chi = a.nr - 1 - kRowsPerBlock * lv, clo = max(chi - (kRowsPerBlock - 1), 0);
                const bool any = lv < a.nb && js0 <= js1;
                double s0, c0, s1, c1;
                ang.get(any ? js0 : 0, s0, c0);
                ang.get(any ? js1 : 0, s1, c1);
                bool high = true;
                const bool out = cell_out_of_gamut_ends(cc, a.g, ang.N, a.ra, a.rb, any ? clo : 0,
                                                        any ? chi : 0, any ? js0 : 0, any ? js1 : 0, s0, c0, s1,
                                                        c1, &a.rule, &high);
                cells = uniform_u64(__ballot(any && !out && high));
            }
            const uint32_t lvcells = a.proofs ? (uint32_t)(cells >> (8 * (bb & 7))) & 0xFFu : 0xFFu;
            if (lvcells == 0u) {
                // every sector of the level proven: no survivor at this level
                tested += (uint64_t)a.W;
                closed += (uint64_t)a.W;
                continue;
            }
            int32_t floor_i = -1;  // radii at or below this cannot beat the level's best so far
            for (int32_t j0 = 0; j0 < a.W && floor_i < hi_i; j0 += 64) {
                const int32_t jl = j0 + (int32_t)lane;
                const bool live = jl < a.W;
                const bool in_open = live && ((lvcells >> ((8 * jl) / a.W)) & 1u);
                bool open = in_open;
                if (a.proofs && __ballot(in_open) != 0ull) {
                    const int32_t jj = live ? jl : 0;
                    double s, co;
                    ang.get(jj, s, co);
                    bool high = true;
                    const bool out = cell_out_of_gamut_ends(cc, a.g, ang.N, a.ra, a.rb, lo_i, hi_i, jj, jj, s, co, s,
                                                            co, &a.rule, &high);
                    open = in_open && !out && high;
                }
                const uint64_t lm = __ballot(live);
                uint64_t om = uniform_u64(__ballot(open));
                tested += (uint64_t)__builtin_popcountll(lm);
                closed += (uint64_t)__builtin_popcountll(lm & ~om);
                while (om && floor_i < hi_i) {
                    // Past the level's first survivor, the open rays left only
                    // need the radii above it: when those rows are fewer than
                    // the rays, take them row by row (lane -> ray, the chunk's
                    // rays together) and stop at the first row with a
                    // survivor (its smallest j); else ray by ray.
                    if (floor_i >= 0 && hi_i - floor_i < __builtin_popcountll(om)) {
                        const bool mine = (om >> lane) & 1ull;
                        double s, co;
                        ang.get(mine ? jl : j0 + (int32_t)__builtin_ctzll(om), s, co);
                        for (int32_t i = hi_i; i > floor_i; --i) {
                            const double rad = (double)(i + 1);
                            float fp[3], fm[3];
                            pair_linear_w(cc, a.g, (rad * a.ra) * s, (rad * a.rb) * co, fp, fm, cube);
                            const uint64_t live_m = __ballot(mine);
                            evald += (uint64_t)__builtin_popcountll(live_m);
                            const bool gp = in_unit_cube(fp), gm = in_unit_cube(fm);
                            const uint64_t need_m = clip ? live_m : (__ballot(gp && gm) & live_m);
                            if (need_m == 0ull) continue;
                            float Vp[3], Vm[3];
                            codes_w(fp, fm, (need_m >> lane) & 1ull, clip, Vp, Vm);
                            const PatMasks pm = pattern_masks(Vp, Vm, a.rule);
                            const uint64_t surv = uniform_u64(accepted_lanes(pm, a.rule.mask) & need_m);
                            if (surv == 0ull) continue;
                            const int32_t first = (int32_t)__builtin_ctzll(surv);  // smallest j of the row
                            uint32_t lo, hi;
                            const uint32_t flags = 4u | (gp ? 1u : 0u) | (gm ? 2u : 0u);
                            pack_pair(Vp, Vm, pattern_of(Vp, Vm, a.rule), flags, lo, hi);
                            floor_i = i;
                            best = best_key(i, j0 + first);
                            blo = (uint32_t)__shfl((int)lo, first, 64);
                            bhi = (uint32_t)__shfl((int)hi, first, 64);
                            break;
                        }
                        om = 0ull;
                        break;
                    }
                    const int32_t j = j0 + (int32_t)__builtin_ctzll(om);
                    om &= om - 1ull;
                    double s, co;
                    ang.get(j, s, co);
                    const int32_t i = hi_i - (int32_t)lane;
                    const bool lv = i >= lo_i && i > floor_i;
                    const double rad = (double)(lv ? i + 1 : 1);
                    float fp[3], fm[3];
                    pair_linear_w(cc, a.g, (rad * a.ra) * s, (rad * a.rb) * co, fp, fm, cube);
                    const uint64_t live_m = __ballot(lv);
                    evald += (uint64_t)__builtin_popcountll(live_m);
                    const bool gp = in_unit_cube(fp), gm = in_unit_cube(fm);
                    const uint64_t need_m = clip ? live_m : (__ballot(gp && gm) & live_m);
                    if (need_m == 0ull) continue;
                    float Vp[3], Vm[3];
                    codes_w(fp, fm, (need_m >> lane) & 1ull, clip, Vp, Vm);
                    const PatMasks pm = pattern_masks(Vp, Vm, a.rule);
                    const uint64_t surv = uniform_u64(accepted_lanes(pm, a.rule.mask) & need_m);
                    if (surv == 0ull) continue;
                    const int32_t first = (int32_t)__builtin_ctzll(surv);  // largest i of this ray
                    uint32_t lo, hi;
                    const uint32_t flags = 4u | (gp ? 1u : 0u) | (gm ? 2u : 0u);
                    pack_pair(Vp, Vm, pattern_of(Vp, Vm, a.rule), flags, lo, hi);
                    // a larger i than the level's best so far (rays come in increasing j)
                    floor_i = hi_i - first;
                    best = best_key(floor_i, j);
                    blo = (uint32_t)__shfl((int)lo, first, 64);
                    bhi = (uint32_t)__shfl((int)hi, first, 64);
                }
            }
        }
        if (lane == 0) {
            if (a.ppairs) {
                // cv_pattern_pair: i, j, then the record's codes and pattern (bytes 8..14 of cv_pair)
                cv_pattern_pair r = {};
                if (best) {
                    r.i = (uint16_t)(best >> 16);
                    r.j = (uint16_t)(0xFFFFu - (best & 0xFFFFu));
                    r.plus[0] = (uint8_t)blo;
                    r.plus[1] = (uint8_t)(blo >> 8);
                    r.plus[2] = (uint8_t)(blo >> 16);
                    r.minus[0] = (uint8_t)(blo >> 24);
                    r.minus[1] = (uint8_t)bhi;
                    r.minus[2] = (uint8_t)(bhi >> 8);
                    r.pattern = (uint8_t)(bhi >> 16);
                    r.flags = CV_PAIR_FOUND | CV_PAIR_FALLBACK;
                }
                a.ppairs[c] = r;
                a.status[c] = best ? (uint8_t)CV_RESOLVED_EXACT : (uint8_t)CV_RESOLVED_NONE;
            }
            if (a.best) a.best[c] = best;
            if (a.pairs) {
                uint32_t* r = reinterpret_cast<uint32_t*>(a.pairs + c);
                const uint32_t bi = best >> 16, bj = 0xFFFFu - (best & 0xFFFFu);
                r[0] = (uint32_t)c;
                r[1] = best ? (bi | (bj << 16)) : 0u;
                r[2] = best ? blo : 0u;
                r[3] = best ? bhi : 0u;
            }
        }
    }
    const uint32_t lane = lane_id_fresh();
    if (a.counts && lane == 0) {
        if (evald) atomicAdd(&a.counts[0], (unsigned long long)evald);
        if (tested) atomicAdd(&a.counts[1], (unsigned long long)tested);
        if (closed) atomicAdd(&a.counts[2], (unsigned long long)closed);
    }
}

__global__ void k_zero_counts(unsigned long long* p) {
    if (threadIdx.x < 3) p[threadIdx.x] = 0ull;
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = 0u;
}

inline unsigned ray_blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int run_ray_search(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd, const RuleDev& rd,
                   uint16_t* rays, cv_pair* recs, uint32_t* best, uint64_t* counts, hipStream_t s) {
    if (counts) {
        hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(64), 0, s, (unsigned long long*)counts);
        CV_HIP(hipGetLastError());
    }
    if (n == 0) return CV_OK;
    if (best) {
        hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s,
                           best, n);
        CV_HIP(hipGetLastError());
    }
    int rc;
    TabArgs tab;
    if ((rc = prepare_colours(ctx, rgb, n, gd, s, tab)) != CV_OK) return rc;
    RayArgs a;
    a.cc = (const ColorConst*)ctx->colors.ptr;
    a.tab = tab;
    a.g = geom_constants();
    a.rule = rd;
    a.ra = gd.ra;
    a.rb = gd.rb;
    a.nr = gd.nr;
    a.ntheta = gd.ntheta;
    a.sym = gd.ntheta == gd.N ? 1 : 0;
    a.W = a.sym ? gd.N / 2 : gd.ntheta;
    a.nb = (gd.nr + kRowsPerBlock - 1) / kRowsPerBlock;
    a.rays_per_task = a.nb >= 64 ? 1 : 64 / a.nb;
    if (a.rays_per_task > a.W) a.rays_per_task = a.W;
    a.tasks_per_colour = (a.W + a.rays_per_task - 1) / a.rays_per_task;
    a.proofs = rd.clip ? 0 : 1;
    a.ntasks = n * (int64_t)a.tasks_per_colour;
    a.rays = rays;
    a.recs = recs;
    a.counts = (unsigned long long*)counts;
    a.best = best;
    const size_t lds = angle_lds_bytes(tab);
    int lds_max = 0;
    CV_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    hipFuncAttributes fa;
    CV_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k_ray_search)));
    if (lds + fa.sharedSizeBytes > (size_t)lds_max)
        return fail(CV_EINVAL, "this grid needs " + std::to_string(lds + fa.sharedSizeBytes) +
                                   " bytes of LDS per block; the device has " + std::to_string(lds_max));
    int per_cu = 0;
    CV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ray_search, kRayBlock, lds));
    if (per_cu < 1) per_cu = 1;
    int64_t grid = (int64_t)per_cu * ctx->num_cu;
    const int64_t need = (int64_t)ray_blocks_for(a.ntasks, kRayBlock / 64);
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    if ((rc = ctx->mark(CV_TIME_CALL, 0, s)) != CV_OK) return rc;
    if ((rc = ctx->mark(CV_TIME_EVAL, 0, s)) != CV_OK) return rc;
    hipLaunchKernelGGL(k_ray_search, dim3((unsigned)grid), dim3(kRayBlock), lds, s, a);
    CV_HIP(hipGetLastError());
    if ((rc = ctx->mark(CV_TIME_EVAL, 1, s)) != CV_OK) return rc;
    if ((rc = ctx->mark(CV_TIME_CALL, 1, s)) != CV_OK) return rc;
    if (ctx->timing && (rc = ctx->collect()) != CV_OK) return rc;
    return CV_OK;
}

namespace {

// Launch k_best_pair on the colour constants and angle table of the context
// (already prepared for the call's colours).
int launch_best_pair(cv_context* ctx, RayArgs& a, const GridDev& gd, const RuleDev& rd, int64_t n_max,
                     hipStream_t s) {
    a.g = geom_constants();
    a.rule = rd;
    a.ra = gd.ra;
    a.rb = gd.rb;
    a.nr = gd.nr;
    a.ntheta = gd.ntheta;
    a.sym = gd.ntheta == gd.N ? 1 : 0;
    a.W = a.sym ? gd.N / 2 : gd.ntheta;
    a.nb = (gd.nr + kRowsPerBlock - 1) / kRowsPerBlock;
    a.proofs = rd.clip ? 0 : 1;
    const size_t lds = angle_lds_bytes(a.tab);
    int lds_max = 0;
    CV_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    hipFuncAttributes fa;
    CV_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k_best_pair)));
    if (lds + fa.sharedSizeBytes > (size_t)lds_max)
        return fail(CV_EINVAL, "this grid needs " + std::to_string(lds + fa.sharedSizeBytes) +
                                   " bytes of LDS per block; the device has " + std::to_string(lds_max));
    int per_cu = 0;
    CV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_best_pair, kRayBlock, lds));
    if (per_cu < 1) per_cu = 1;
    int64_t grid = (int64_t)per_cu * ctx->num_cu;
    const int64_t need = (int64_t)ray_blocks_for(n_max, kRayBlock / 64);
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_best_pair, dim3((unsigned)grid), dim3(kRayBlock), lds, s, a);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

}  // namespace

int run_best_pair_list(cv_context* ctx, const GridDev& gd, const RuleDev& rd, const uint32_t* list,
                       const uint64_t* n_dev, int64_t n_max, cv_pattern_pair* pairs, uint8_t* status, hipStream_t s) {
    if (n_max == 0) return CV_OK;
    RayArgs a = {};
    a.cc = (const ColorConst*)ctx->colors.ptr;
    a.tab.tab = (const double*)ctx->table.ptr;
    a.tab.tab_len = gd.tab_len;
    a.tab.N = gd.N;
    a.tab.dW = direct_rays(gd.ntheta, gd.N, gd.tab_len, 0);
    a.tab._pad = 0;
    a.list = list;
    a.n_dev = n_dev;
    a.n = n_max;
    a.ppairs = pairs;
    a.status = status;
    return launch_best_pair(ctx, a, gd, rd, n_max, s);
}

int run_best_pair(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd, const RuleDev& rd,
                  uint32_t* best, cv_pair* pairs, uint64_t* counts, hipStream_t s) {
    if (counts) {
        hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(64), 0, s, (unsigned long long*)counts);
        CV_HIP(hipGetLastError());
    }
    if (n == 0) return CV_OK;
    int rc;
    TabArgs tab;
    if ((rc = prepare_colours(ctx, rgb, n, gd, s, tab)) != CV_OK) return rc;
    RayArgs a = {};
    a.cc = (const ColorConst*)ctx->colors.ptr;
    a.tab = tab;
    a.counts = (unsigned long long*)counts;
    a.best = best;
    a.pairs = pairs;
    a.n = n;
    if ((rc = ctx->mark(CV_TIME_CALL, 0, s)) != CV_OK) return rc;
    if ((rc = ctx->mark(CV_TIME_EVAL, 0, s)) != CV_OK) return rc;
    if ((rc = launch_best_pair(ctx, a, gd, rd, n, s)) != CV_OK) return rc;
    if ((rc = ctx->mark(CV_TIME_EVAL, 1, s)) != CV_OK) return rc;
    if ((rc = ctx->mark(CV_TIME_CALL, 1, s)) != CV_OK) return rc;
    if (ctx->timing && (rc = ctx->collect()) != CV_OK) return rc;
    return CV_OK;
}

}  // namespace cvib
