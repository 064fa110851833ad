// Host-side internals shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <exception>
#include <map>
#include <string>

#include "../../include/cvib.h"
#include "cvib_device.h"

namespace cvib {

// Colour-space constants derived in FP64 from the sRGB primaries and the D65
// white (IEC 61966-2-1): M maps linear RGB to XYZ (Y of white = 1).
struct ColorSpace {
    double M[3][3];
    double Minv[3][3];
    double W[3]; // Xn, Yn = 1, Zn
};
const ColorSpace& color_space();
Geom geom_constants();

// Error reporting (thread-local message behind cv_last_error).
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
#define CV_HIP(call)                                        \
    do {                                                    \
        hipError_t _e = (call);                             \
        if (_e != hipSuccess) return ::cvib::hip_fail(_e, #call); \
    } while (0)

// Every C entry point runs inside this guard: no exception crosses the ABI.
#define CV_GUARD_BEGIN try {
#define CV_GUARD_END                                                                 \
    }                                                                                \
    catch (const std::exception& ex) {                                               \
        return ::cvib::fail(CV_ESTATE, std::string("internal error: ") + ex.what()); \
    }                                                                                \
    catch (...) {                                                                    \
        return ::cvib::fail(CV_ESTATE, "internal error");                            \
    }

// Make a device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Validated, device-ready form of a grid.
struct GridDev {
    double dr;       // radius step
    double ra, rb;   // dr / 500, dr / 200: radius step in f(X), f(Z) units
    int32_t nr, ntheta;
    int32_t N;       // 360 / dtheta: angles per full turn
    int32_t tab_len; // folded angle table length in doubles
    int64_t per_colour;
};
int make_grid(const cv_grid* g, GridDev* out);
int make_rule(const cv_rule* r, RuleDev* out);

// Device workspace owned by a context, grown on demand.
struct Buffer {
    void* ptr = nullptr;
    size_t bytes = 0;
};

int run_lab_convert(cv_context* ctx, const void* in, void* out, int64_t n, int dir,
                    hipStream_t s);
int run_pair_search(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd,
                    const RuleDev& rd, cv_pair* out, int64_t capacity, int64_t* offsets,
                    cv_color_summary* summ, int64_t* total_host, uint32_t flags, hipStream_t s);
// Scratch array of the no-allocation reduce (one per device, kept until the
// process ends) and its set-up, once per device with the device current.
constexpr size_t kScratchBytes = (size_t)8 << 20;
int scratch_init(int device);
size_t reduce_scratch_bytes(int64_t n, const GridDev& gd);
int run_pair_reduce_noalloc(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd,
                            const RuleDev& rd, cv_color_summary* summ, cv_table_row* table,
                            hipStream_t s);
int run_ray_search(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd, const RuleDev& rd,
                   uint16_t* rays, cv_pair* recs, uint32_t* best, uint64_t* counts, hipStream_t s);
int run_best_pair(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd, const RuleDev& rd,
                  uint32_t* best, cv_pair* pairs, uint64_t* counts, hipStream_t s);
// The exact search's maximum-amplitude pair of the colours list[k], k < *n_dev
// (n_max bounds it), on the colour constants and angle table the context
// holds for the call, into pairs[colour] (flags CV_PAIR_FOUND |
// CV_PAIR_FALLBACK) and status[colour].
int run_best_pair_list(cv_context* ctx, const GridDev& gd, const RuleDev& rd, const uint32_t* list,
                       const uint64_t* n_dev, int64_t n_max, cv_pattern_pair* pairs, uint8_t* status, hipStream_t s);
int run_pair_csr_summary(cv_context* ctx, const cv_pair* recs, const int64_t* offsets, int64_t n,
                         cv_color_summary* summ, hipStream_t s);
int run_pair_reduce(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd,
                    const RuleDev& rd, cv_color_summary* summ, cv_table_row* table,
                    hipStream_t s);
int run_scan_counts(cv_context* ctx, const uint32_t* cnt, int64_t T, uint64_t* prefix,
                    int64_t* offsets, int32_t spc, int64_t n, uint64_t* total, hipStream_t s);
Geom geom_constants();
int launch_angle_table(double* tab, int32_t N, hipStream_t s);

// One cv_frames_resolve call (compared bytewise to reuse a captured graph).
struct FramesCall {
    const uint8_t* pixels;
    int64_t npix;
    const uint8_t* info;
    GridDev gd;
    RuleDev rd;
    uint8_t* colours;
    int64_t colour_cap;
    int64_t* ncolours;
    uint32_t* pixel_index;
    cv_color_summary* summ;
    cv_pattern_pair* pbest;
    uint16_t* rays;
    uint8_t* frame_a;
    uint8_t* frame_b;
    int64_t* resolved;
    const void* ws[7];  // context workspaces the call uses (a regrown one voids a cached graph)
    int32_t variant;    // per-colour resolve kernel (see resolve_variant)
    int32_t cells;      // gamut cells on in the context when captured
    int32_t no_ngamut;  // CV_NO_NGAMUT: summaries without n_gamut
    int32_t _pad;
    int enqueue(cv_context* ctx, hipStream_t s) const;
    bool same(const FramesCall& o) const;
};
int run_frames_resolve(cv_context* ctx, const FramesCall& call, bool graph, hipStream_t s);

// Everything a cv_pair_search call (not per-ray) depends on: compared
// bytewise to reuse a captured graph.
struct SearchCall {
    const uint8_t* rgb;
    int64_t n;
    GridDev gd;
    RuleDev rd;
    cv_pair* out;
    int64_t capacity;
    int64_t* offsets;
    cv_color_summary* summ;
    const void* ws[9];  // context workspaces the call uses
    uint32_t flags;
    int32_t cells;
    int32_t tiles;      // tiles per call of the count pass (plan_reduce's target)
    int32_t _pad;
    bool same(const SearchCall& o) const;
};

// Tiles per call of the chunked reduce kernels (the count pass of
// cv_pair_search, and cv_pair_reduce when colours are few): the default and
// the choices the autotuner times.
constexpr int32_t kTilesDefault = 4096;
constexpr int32_t kTileTargets[5] = {1024, 2048, 4096, 8192, 16384};
uint64_t tiles_key(int search, int64_t n, const GridDev& gd);
int32_t tiles_target(cv_context* ctx, uint64_t key);

int run_pair_reduce_rules(cv_context* ctx, const uint8_t* rgb, int64_t n, const GridDev& gd,
                          const RuleDev* rules, int32_t nrules, uint32_t* counts, hipStream_t s);

// Per-colour resolve kernels: 0 = one colour per block of 4 waves, 1 = one
// colour per wave with 4 waves per block, 2 = the same with 8 waves per block.
constexpr int kResolveVariants = 3;
uint64_t resolve_key(const GridDev& gd, bool rays);
int resolve_variant(cv_context* ctx, const GridDev& gd, bool rays);

// Surrogate resolve of n colours (n_dev: the same count on the device).
struct SurrogateCall {
    cv_mlp* mlp;
    const uint8_t* rgb;
    int64_t n;
    GridDev gd;
    RuleDev rd;
    float tau;
    int32_t kbins;
    bool fallback;
    float* pred;              // nullable: a context workspace is used
    cv_pattern_pair* pairs;
    uint8_t* status;
    int64_t* nfallback;       // nullable
    uint32_t* fallback_list;  // nullable [n]: colour indices sent to the exact search, in order
    bool pred_given;          // pred is the caller's input; the network does not run
};
int run_surrogate(cv_context* ctx, const SurrogateCall& call, hipStream_t s);
int run_frames_surrogate(cv_context* ctx, const SurrogateCall& call, const uint8_t* pixels,
                         int64_t npix, uint8_t* colours, int64_t colour_cap, int64_t* ncolours,
                         uint32_t* pixel_index, uint8_t* frame_a, uint8_t* frame_b,
                         int64_t* resolved, hipStream_t s);

// Network pieces used by the surrogate resolve (defined with the network).
int mlp_forward_rgb8(cv_mlp* m, const uint8_t* rgb, int64_t n, float* out, hipStream_t s);
int mlp_out_width(const cv_mlp* m);
int mlp_in_width(const cv_mlp* m);
int mlp_device(const cv_mlp* m);

} // namespace cvib

struct cv_context {
    int device = 0;
    int num_cu = 0;
    cvib::Buffer colors;  // ColorConst [n]
    cvib::Buffer table;   // angle table
    cvib::Buffer seg_cnt;     // records per search segment
    cvib::Buffer seg_prefix;  // output offset per search segment
    cvib::Buffer seg_mask;    // passes holding survivors per search segment
    cvib::Buffer scan;        // per-block partial sums of the segment scan
    cvib::Buffer acc;         // per-colour accumulators
    cvib::Buffer misc;        // ticket, -, survivor total
    cvib::Buffer fbits;       // frames: 2^24-bit colour bitmap
    cvib::Buffer fcnt;        // frames: colours per bitmap word
    cvib::Buffer fprefix;     // frames: first colour index per bitmap word
    cvib::Buffer fmisc;       // frames: [0] colour count
    cvib::Buffer spred;       // surrogate: network outputs [n][37]
    cvib::Buffer sneed;       // surrogate: 1 = exact fallback, per colour
    cvib::Buffer sprefix;     // surrogate: fallback list positions
    cvib::Buffer slist;       // surrogate: fallback colour indices
    cvib::Buffer smisc;       // surrogate: [0] colour count, [1] fallback count
    cvib::Buffer rays;        // per-ray search: largest i + 1 per evaluated ray
    cvib::Buffer rtab;        // multi-rule: interval table, classes, masks
    cvib::Buffer rhist;       // multi-rule: interval-triple histogram per colour
    // gamut cells in the reduce kernels (cv_context_set_gamut_cells), and the
    // device counter of the candidates they skipped (counted while timing)
    bool gamut_cells = true;
    cvib::Buffer stats;
    uint64_t stats_base = 0;
    uint64_t no_high_base = 0;
    // per-colour resolve kernel choice: forced (-1 = none), or tuned per grid shape
    bool autotune = false;
    // tiles per call of the chunked reduce: forced (0 = none), or tuned per
    // call shape (count pass or reduce, colours, grid)
    int32_t tiles_forced = 0;
    std::map<uint64_t, int32_t> tiles_tuned;
    // on-disk cache of the tuned choices (cv_context_set_tune_file; empty = none)
    std::string tune_file;
    int save_tuning();  // rewrite tune_file with every tuned choice (nothing without one)
    int resolve_forced = -1;
    std::map<uint64_t, int> resolve_tuned;
    hipStream_t cap_stream = nullptr;        // stream used for graph capture
    hipGraphExec_t fgraph_exec = nullptr;    // captured cv_frames_resolve
    hipGraphExec_t sgraph_exec = nullptr;    // captured cv_pair_search
    cvib::SearchCall sgraph_call{};          // the call it was captured for
    cvib::FramesCall fgraph_call{};          // the call it was captured for
    uint64_t* host_misc = nullptr; // pinned mirror of misc for the total
    // kernel timing (cv_context_set_timing): event pairs and totals per phase
    bool timing = false;
    static constexpr int kPhases = 5;
    hipEvent_t ev[kPhases][2] = {};
    bool armed[kPhases] = {};
    double kernel_ms[kPhases] = {};
    int64_t kernel_calls[kPhases] = {};
    int ensure(cvib::Buffer& b, size_t bytes);
    int mark(int phase, int end, hipStream_t s);  // record a phase's start / end event
    int collect();                                // after a sync: add armed phases
};
