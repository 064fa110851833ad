// C-ABI entry points of libcvib: argument validation, error reporting, the
// context and its workspace, and the colour-space constants.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <cstdio>
#include <cstring>
#include <exception>
#include <string>

#include "cvib_internal.h"

namespace cvib {

namespace {
thread_local std::string g_last_error;

// det / inverse of a 3x3 matrix by the adjugate (FP64).
double det3(const double m[3][3]) {
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
           m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
           m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

void invert3(const double m[3][3], double out[3][3]) {
    const double d = det3(m);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            // cofactor of element (c, r), transposed into (r, c)
            const int r0 = (c + 1) % 3, r1 = (c + 2) % 3, c0 = (r + 1) % 3, c1 = (r + 2) % 3;
            out[r][c] = (m[r0][c0] * m[r1][c1] - m[r0][c1] * m[r1][c0]) / d;
        }
}

ColorSpace build_color_space() {
    // CIE xy of the sRGB primaries and of D65 (IEC 61966-2-1).
    const double xy[4][2] = {{0.64, 0.33}, {0.30, 0.60}, {0.15, 0.06}, {0.3127, 0.3290}};
    ColorSpace cs;
    double P[3][3]; // columns: XYZ of each primary with Y = 1
    for (int k = 0; k < 3; ++k) {
        const double x = xy[k][0], y = xy[k][1];
        P[0][k] = x / y;
        P[1][k] = 1.0;
        P[2][k] = (1.0 - x - y) / y;
    }
    const double wx = xy[3][0], wy = xy[3][1];
    cs.W[0] = wx / wy;
    cs.W[1] = 1.0;
    cs.W[2] = (1.0 - wx - wy) / wy;
    // scale each primary so that R = G = B = 1 reproduces the white point
    double Pinv[3][3];
    invert3(P, Pinv);
    double S[3];
    for (int k = 0; k < 3; ++k) S[k] = Pinv[k][0] * cs.W[0] + Pinv[k][1] * cs.W[1] + Pinv[k][2] * cs.W[2];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) cs.M[r][c] = P[r][c] * S[c];
    invert3(cs.M, cs.Minv);
    return cs;
}
} // namespace

const ColorSpace& color_space() {
    static const ColorSpace cs = build_color_space();
    return cs;
}

Geom geom_constants() {
    const ColorSpace& cs = color_space();
    Geom g;
    for (int k = 0; k < 3; ++k) {
        g.A[k] = cs.Minv[k][0] * cs.W[0];
        g.C[k] = cs.Minv[k][2] * cs.W[2];
    }
    return g;
}

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? CV_ENOMEM : CV_EHIP;
}

int make_grid(const cv_grid* g, GridDev* out) {
    if (!g) return fail(CV_EINVAL, "grid is NULL");
    if (!(g->dr > 0.0) || !isfinite(g->dr)) return fail(CV_EINVAL, "grid.dr must be > 0");
    if (g->nr < 1 || g->nr > 65535) return fail(CV_EINVAL, "grid.nr must be in [1, 65535]");
    if (g->ntheta < 1 || g->ntheta > 65535)
        return fail(CV_EINVAL, "grid.ntheta must be in [1, 65535]");
    if ((int64_t)g->nr * g->ntheta >= (int64_t)1 << 31)
        return fail(CV_EINVAL, "grid.nr * grid.ntheta must be < 2^31");
    if (!(g->dtheta_deg > 0.0) || !isfinite(g->dtheta_deg))
        return fail(CV_EINVAL, "grid.dtheta_deg must be > 0");
    const double q = 360.0 / g->dtheta_deg;
    const double Nr = nearbyint(q);
    if (fabs(q - Nr) > 1e-9 * Nr || Nr < 2 || Nr > 8192 || fmod(Nr, 2.0) != 0.0)
        return fail(CV_EINVAL, "360 / grid.dtheta_deg must be an even integer <= 8192");
    const int32_t N = (int32_t)Nr;
    if (g->ntheta > N) return fail(CV_EINVAL, "grid.ntheta exceeds one full turn");
    out->dr = g->dr;
    out->ra = g->dr / 500.0;
    out->rb = g->dr / 200.0;
    out->nr = g->nr;
    out->ntheta = g->ntheta;
    out->N = N;
    // folded angle table: a quarter turn of sin, or a half turn of sin and cos
    out->tab_len = (N % 4 == 0) ? N / 4 + 1 : 2 * (N / 2 + 1);
    out->per_colour = (int64_t)g->nr * g->ntheta;
    return CV_OK;
}

int make_rule(const cv_rule* r, RuleDev* out) {
    if (!r) return fail(CV_EINVAL, "rule is NULL");
    if (r->v_th <= 0 || r->v_th > 255) return fail(CV_EINVAL, "rule.v_th must be in [1, 255]");
    if (!(r->r_novib > 0.0 && r->r_novib < 1.0))
        return fail(CV_EINVAL, "rule.r_novib must be in (0, 1)");
    if ((r->pattern_mask & 0x7Fu) == 0) return fail(CV_EINVAL, "rule.pattern_mask is empty");
    if (r->flags & ~(uint32_t)CV_RULE_CLIP) return fail(CV_EINVAL, "unknown rule flags");
    // d < v_th * r_novib  <=>  d <= ceil(v_th * r_novib) - 1 for integer d
    const double lo = (double)r->v_th * r->r_novib;
    out->v_th = (float)r->v_th;
    out->lo_max = (float)(ceil(lo) - 1.0);
    out->mask = r->pattern_mask & 0x7Fu;
    out->clip = (r->flags & CV_RULE_CLIP) ? 1u : 0u;
    return CV_OK;
}

} // namespace cvib

namespace {

// First line of a tuning file: format tag, GPU architecture and compute-unit
// count (choices made on one GPU model are not reused on another).
std::string tune_header(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "";
    std::string arch(prop.gcnArchName);
    for (char& ch : arch)
        if (ch == ' ') ch = '_';
    return "cvib-tune 1 " + arch + " " + std::to_string(prop.multiProcessorCount);
}

bool tile_choice(int32_t v) {
    for (int32_t t : cvib::kTileTargets)
        if (t == v) return true;
    return false;
}

} // namespace

int cv_context::save_tuning() {
    if (tune_file.empty()) return CV_OK;
    const std::string head = tune_header(device);
    if (head.empty()) return cvib::fail(CV_EHIP, "hipGetDeviceProperties");
    const std::string tmp = tune_file + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return cvib::fail(CV_EINVAL, "cannot write the tuning file " + tmp);
    bool ok = fprintf(f, "%s\n", head.c_str()) > 0;
    for (const auto& kv : resolve_tuned)
        ok = ok && fprintf(f, "resolve %016llx %d\n", (unsigned long long)kv.first, kv.second) > 0;
    for (const auto& kv : tiles_tuned)
        ok = ok && fprintf(f, "tiles %016llx %d\n", (unsigned long long)kv.first, (int)kv.second) > 0;
    ok = (fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), tune_file.c_str()) != 0) {
        std::remove(tmp.c_str());
        return cvib::fail(CV_EINVAL, "cannot write the tuning file " + tune_file);
    }
    return CV_OK;
}

int cv_context::ensure(cvib::Buffer& b, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return CV_OK;
    if (b.ptr) {
        CV_HIP(hipFree(b.ptr)); // synchronises: earlier work on the old buffer is done
        b.ptr = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes + bytes / 4; // grow with headroom
    hipError_t e = hipMalloc(&b.ptr, want);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        return cvib::hip_fail(e, "hipMalloc(workspace)");
    }
    b.bytes = want;
    return CV_OK;
}

int cv_context::mark(int phase, int end, hipStream_t s) {
    if (!timing) return CV_OK;
    CV_HIP(hipEventRecord(ev[phase][end], s));
    if (end) armed[phase] = true;
    return CV_OK;
}

int cv_context::collect() {
    for (int p = 0; p < kPhases; ++p) {
        if (!armed[p]) continue;
        float ms = 0.0f;
        CV_HIP(hipEventSynchronize(ev[p][1]));
        CV_HIP(hipEventElapsedTime(&ms, ev[p][0], ev[p][1]));
        kernel_ms[p] += ms;
        kernel_calls[p] += 1;
        armed[p] = false;
    }
    return CV_OK;
}

using cvib::fail;

using cvib::DeviceGuard;

extern "C" {

const char* cv_last_error(void) { return cvib::g_last_error.c_str(); }

int cv_context_create(int device, cv_context** out) {
    CV_GUARD_BEGIN
    if (!out) return fail(CV_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    CV_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(CV_EINVAL, "no such device");
    DeviceGuard dg(device);
    if (!dg.ok) return fail(CV_EHIP, "hipSetDevice failed");
    cv_context* c = new cv_context();
    c->device = device;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete c;
        return cvib::hip_fail(e, "hipGetDeviceProperties");
    }
    c->num_cu = prop.multiProcessorCount;
    e = hipHostMalloc((void**)&c->host_misc, 64, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete c;
        return cvib::hip_fail(e, "hipHostMalloc");
    }
    // device address of the no-allocation reduce's scratch array on this device
    int rc = cvib::scratch_init(device);
    if (rc != CV_OK) {
        (void)hipHostFree(c->host_misc);
        delete c;
        return rc;
    }
    *out = c;
    return CV_OK;
    CV_GUARD_END
}

int cv_context_destroy(cv_context* ctx) {
    CV_GUARD_BEGIN
    if (!ctx) return CV_OK;
    DeviceGuard dg(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->fgraph_exec) (void)hipGraphExecDestroy(ctx->fgraph_exec);
    if (ctx->sgraph_exec) (void)hipGraphExecDestroy(ctx->sgraph_exec);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    cvib::Buffer* bufs[] = {&ctx->colors, &ctx->table, &ctx->seg_cnt, &ctx->seg_prefix,
                            &ctx->scan,   &ctx->acc,   &ctx->misc,    &ctx->fbits,
                            &ctx->fcnt,   &ctx->fprefix, &ctx->fmisc, &ctx->spred,
                            &ctx->sneed,  &ctx->sprefix, &ctx->slist, &ctx->smisc,
                            &ctx->rtab,   &ctx->rhist,   &ctx->rays,    &ctx->stats,
                            &ctx->seg_mask};
    for (cvib::Buffer* b : bufs)
        if (b->ptr) (void)hipFree(b->ptr);
    if (ctx->host_misc) (void)hipHostFree(ctx->host_misc);
    for (auto& pr : ctx->ev)
        for (hipEvent_t e : pr)
            if (e) (void)hipEventDestroy(e);
    delete ctx;
    return CV_OK;
    CV_GUARD_END
}

int cv_lab_convert(cv_context* ctx, const void* in, void* out, int64_t n, int dir, void* stream) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (n < 0) return fail(CV_EINVAL, "n < 0");
    if (dir != CV_RGB8_TO_LAB && dir != CV_LAB_TO_RGBF) return fail(CV_EINVAL, "unknown dir");
    if (n > 0 && (!in || !out)) return fail(CV_EINVAL, "null array");
    DeviceGuard dg(ctx->device);
    return cvib::run_lab_convert(ctx, in, out, n, dir, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_pair_search(cv_context* ctx, const uint8_t* rgb, int64_t n, const cv_grid* grid,
                   const cv_rule* rule, cv_pair* out, int64_t capacity, int64_t* offsets,
                   cv_color_summary* summ, int64_t* total_host, uint32_t flags, void* stream) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (!total_host && !offsets) return fail(CV_EINVAL, "total_host and offsets are both NULL");
    if (n < 0 || n > 0xFFFFFFFFll) return fail(CV_EINVAL, "n out of range");
    if (capacity < 0) return fail(CV_EINVAL, "capacity < 0");
    if (capacity > 0 && !out) return fail(CV_EINVAL, "out is NULL with capacity > 0");
    if (n > 0 && !rgb) return fail(CV_EINVAL, "rgb is NULL");
    if (flags & ~(uint32_t)(CV_EMIT_ALL | CV_PER_RAY | CV_GRAPH | CV_NO_NGAMUT)) return fail(CV_EINVAL, "unknown flags");
    if ((flags & CV_EMIT_ALL) && (flags & CV_PER_RAY))
        return fail(CV_EINVAL, "CV_EMIT_ALL and CV_PER_RAY exclude each other");
    cvib::GridDev gd;
    cvib::RuleDev rd;
    int rc;
    if ((rc = cvib::make_grid(grid, &gd)) != CV_OK) return rc;
    if ((rc = cvib::make_rule(rule, &rd)) != CV_OK) return rc;
    DeviceGuard dg(ctx->device);
    return cvib::run_pair_search(ctx, rgb, n, gd, rd, out, capacity, offsets, summ, total_host,
                                 flags, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_pair_reduce(cv_context* ctx, const uint8_t* rgb, int64_t n, const cv_grid* grid,
                   const cv_rule* rule, cv_color_summary* summ, cv_table_row* table,
                   void* stream) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (n < 0 || n > 0xFFFFFFFFll) return fail(CV_EINVAL, "n out of range");
    if (n > 0 && !rgb) return fail(CV_EINVAL, "rgb is NULL");
    if (!summ && !table) return fail(CV_EINVAL, "summ and table are both NULL");
    cvib::GridDev gd;
    cvib::RuleDev rd;
    int rc;
    if ((rc = cvib::make_grid(grid, &gd)) != CV_OK) return rc;
    if ((rc = cvib::make_rule(rule, &rd)) != CV_OK) return rc;
    if (table && gd.nr > 255) return fail(CV_EINVAL, "table rows need grid.nr <= 255");
    if (table && (size_t)gd.tab_len * 8 + (size_t)gd.ntheta * 4 > 48 * 1024)
        return fail(CV_EINVAL, "table rows need 8 * table + 4 * ntheta <= 48 KiB of LDS");
    DeviceGuard dg(ctx->device);
    return cvib::run_pair_reduce(ctx, rgb, n, gd, rd, summ, table, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_pair_reduce_noalloc(cv_context* ctx, const uint8_t* rgb, int64_t n, const cv_grid* grid,
                           const cv_rule* rule, cv_color_summary* summ, cv_table_row* table,
                           void* stream) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (n < 0 || n > 0xFFFFFFFFll) return fail(CV_EINVAL, "n out of range");
    if (n > 0 && !rgb) return fail(CV_EINVAL, "rgb is NULL");
    if (!summ && !table) return fail(CV_EINVAL, "summ and table are both NULL");
    cvib::GridDev gd;
    cvib::RuleDev rd;
    int rc;
    if ((rc = cvib::make_grid(grid, &gd)) != CV_OK) return rc;
    if ((rc = cvib::make_rule(rule, &rd)) != CV_OK) return rc;
    if (table && gd.nr > 255) return fail(CV_EINVAL, "table rows need grid.nr <= 255");
    if (table && (size_t)gd.tab_len * 8 + (size_t)gd.ntheta * 4 > 48 * 1024)
        return fail(CV_EINVAL, "table rows need 8 * table + 4 * ntheta <= 48 KiB of LDS");
    DeviceGuard dg(ctx->device);
    return cvib::run_pair_reduce_noalloc(ctx, rgb, n, gd, rd, summ, table, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_ray_search(cv_context* ctx, const uint8_t* rgb, int64_t n, const cv_grid* grid, const cv_rule* rule,
                  uint16_t* rays, cv_pair* recs, uint32_t* best, uint64_t* counts, void* stream) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (n < 0 || n > 0xFFFFFFFFll) return fail(CV_EINVAL, "n out of range");
    if (n > 0 && (!rgb || !rays)) return fail(CV_EINVAL, "rgb or rays is NULL");
    cvib::GridDev gd;
    cvib::RuleDev rd;
    int rc;
    if ((rc = cvib::make_grid(grid, &gd)) != CV_OK) return rc;
    if ((rc = cvib::make_rule(rule, &rd)) != CV_OK) return rc;
    DeviceGuard dg(ctx->device);
    return cvib::run_ray_search(ctx, rgb, n, gd, rd, rays, recs, best, counts, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_best_pair_search(cv_context* ctx, const uint8_t* rgb, int64_t n, const cv_grid* grid, const cv_rule* rule,
                        uint32_t* best, cv_pair* pairs, uint64_t* counts, void* stream) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (n < 0 || n > 0xFFFFFFFFll) return fail(CV_EINVAL, "n out of range");
    if (!best && !pairs) return fail(CV_EINVAL, "best and pairs are both NULL");
    if (n > 0 && !rgb) return fail(CV_EINVAL, "rgb is NULL");
    cvib::GridDev gd;
    cvib::RuleDev rd;
    int rc;
    if ((rc = cvib::make_grid(grid, &gd)) != CV_OK) return rc;
    if ((rc = cvib::make_rule(rule, &rd)) != CV_OK) return rc;
    DeviceGuard dg(ctx->device);
    return cvib::run_best_pair(ctx, rgb, n, gd, rd, best, pairs, counts, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_frames_resolve(cv_context* ctx, const uint8_t* pixels, int64_t npix, const uint8_t* info,
                      const cv_grid* grid, const cv_rule* rule, uint8_t* colours,
                      int64_t colour_cap, int64_t* ncolours, uint32_t* pixel_index,
                      cv_color_summary* summ, cv_pattern_pair* pbest, uint16_t* rays,
                      uint8_t* frame_a, uint8_t* frame_b, int64_t* resolved, uint32_t flags,
                      void* stream) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (npix < 1) return fail(CV_EINVAL, "npix must be >= 1");
    if (!pixels || !colours || !ncolours || !pixel_index || !pbest)
        return fail(CV_EINVAL, "null array");
    if ((frame_a == nullptr) != (frame_b == nullptr))
        return fail(CV_EINVAL, "frame_a and frame_b go together");
    if (resolved && !frame_a) return fail(CV_EINVAL, "resolved needs the frames");
    const int64_t need = npix < ((int64_t)1 << 24) ? npix : ((int64_t)1 << 24);
    if (colour_cap < need) return fail(CV_EINVAL, "colour_cap < min(npix, 2^24)");
    if (flags & ~(uint32_t)(CV_GRAPH | CV_NO_NGAMUT)) return fail(CV_EINVAL, "unknown flags");
    cvib::FramesCall call;
    std::memset(&call, 0, sizeof call);  // bytewise comparison for the graph cache
    call.no_ngamut = (flags & CV_NO_NGAMUT) ? 1 : 0;
    int rc;
    if ((rc = cvib::make_grid(grid, &call.gd)) != CV_OK) return rc;
    if ((rc = cvib::make_rule(rule, &call.rd)) != CV_OK) return rc;
    call.pixels = pixels;
    call.npix = npix;
    call.info = info;
    call.colours = colours;
    call.colour_cap = colour_cap;
    call.ncolours = ncolours;
    call.pixel_index = pixel_index;
    call.summ = summ;
    call.pbest = pbest;
    call.rays = rays;
    call.frame_a = frame_a;
    call.frame_b = frame_b;
    call.resolved = resolved;
    DeviceGuard dg(ctx->device);
    return cvib::run_frames_resolve(ctx, call, (flags & CV_GRAPH) != 0, (hipStream_t)stream);
    CV_GUARD_END
}

namespace {
int surrogate_call(cv_context* ctx, cv_mlp* mlp, const cv_grid* grid, const cv_rule* rule, float tau,
                   int32_t kbins, uint32_t flags, cvib::SurrogateCall* c) {
    const bool given = (flags & CV_PRED_GIVEN) != 0;
    if (!ctx || (!mlp && !given)) return fail(CV_EINVAL, "ctx or network is NULL");
    if (mlp && (cvib::mlp_in_width(mlp) != 3 || cvib::mlp_out_width(mlp) != 37))
        return fail(CV_EINVAL, "the surrogate network must map 3 inputs to 37 outputs");
    if (mlp && cvib::mlp_device(mlp) != ctx->device)
        return fail(CV_EINVAL, "network and context on different devices");
    if (kbins < 1 || kbins > 36) return fail(CV_EINVAL, "kbins must be in [1, 36]");
    if (!(tau == tau)) return fail(CV_EINVAL, "tau is NaN");
    if (flags & ~(uint32_t)(CV_NO_FALLBACK | CV_PRED_GIVEN)) return fail(CV_EINVAL, "unknown flags");
    std::memset(c, 0, sizeof *c);
    c->pred_given = given;
    int rc;
    if ((rc = cvib::make_grid(grid, &c->gd)) != CV_OK) return rc;
    if ((rc = cvib::make_rule(rule, &c->rd)) != CV_OK) return rc;
    c->mlp = mlp;
    c->tau = tau;
    c->kbins = kbins;
    c->fallback = (flags & CV_NO_FALLBACK) == 0;
    return CV_OK;
}
} // namespace

int cv_surrogate_infer(cv_context* ctx, cv_mlp* mlp, const uint8_t* rgb, int64_t n,
                       const cv_grid* grid, const cv_rule* rule, float tau, int32_t kbins,
                       float* pred, cv_pattern_pair* pairs, uint8_t* status, uint32_t* fallback,
                       int64_t* nfallback, uint32_t flags, void* stream) {
    CV_GUARD_BEGIN
    cvib::SurrogateCall c;
    int rc;
    if ((rc = surrogate_call(ctx, mlp, grid, rule, tau, kbins, flags, &c)) != CV_OK) return rc;
    if (n < 0 || n > ((int64_t)1 << 30)) return fail(CV_EINVAL, "n must be in [0, 2^30]");
    if (n > 0 && (!rgb || !pairs || !status)) return fail(CV_EINVAL, "null array");
    if (n > 0 && c.pred_given && !pred) return fail(CV_EINVAL, "CV_PRED_GIVEN needs pred");
    c.rgb = rgb;
    c.n = n;
    c.pred = pred;
    c.pairs = pairs;
    c.status = status;
    c.nfallback = nfallback;
    c.fallback_list = fallback;
    DeviceGuard dg(ctx->device);
    return cvib::run_surrogate(ctx, c, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_frames_surrogate(cv_context* ctx, cv_mlp* mlp, const uint8_t* pixels, int64_t npix,
                        const cv_grid* grid, const cv_rule* rule, float tau, int32_t kbins,
                        uint8_t* colours, int64_t colour_cap, int64_t* ncolours,
                        uint32_t* pixel_index, cv_pattern_pair* pairs, uint8_t* status,
                        uint8_t* frame_a, uint8_t* frame_b, int64_t* resolved, int64_t* nfallback,
                        uint32_t flags, void* stream) {
    CV_GUARD_BEGIN
    cvib::SurrogateCall c;
    int rc;
    if ((rc = surrogate_call(ctx, mlp, grid, rule, tau, kbins, flags, &c)) != CV_OK) return rc;
    if (npix < 1) return fail(CV_EINVAL, "npix must be >= 1");
    if (!pixels || !colours || !ncolours || !pixel_index || !pairs || !status)
        return fail(CV_EINVAL, "null array");
    if ((frame_a == nullptr) != (frame_b == nullptr))
        return fail(CV_EINVAL, "frame_a and frame_b go together");
    if (resolved && !frame_a) return fail(CV_EINVAL, "resolved needs the frames");
    const int64_t need = npix < ((int64_t)1 << 24) ? npix : ((int64_t)1 << 24);
    if (colour_cap < need) return fail(CV_EINVAL, "colour_cap < min(npix, 2^24)");
    c.pairs = pairs;
    c.status = status;
    c.nfallback = nfallback;
    c.fallback_list = nullptr;
    if (c.pred_given) return fail(CV_EINVAL, "CV_PRED_GIVEN is for cv_surrogate_infer");
    DeviceGuard dg(ctx->device);
    return cvib::run_frames_surrogate(ctx, c, pixels, npix, colours, colour_cap, ncolours, pixel_index,
                                      frame_a, frame_b, resolved, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_pair_reduce_csr(cv_context* ctx, const cv_pair* recs, const int64_t* offsets, int64_t n,
                       cv_color_summary* summ, void* stream) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (n < 0) return fail(CV_EINVAL, "n < 0");
    if (n > 0 && (!offsets || !summ)) return fail(CV_EINVAL, "null array");
    DeviceGuard dg(ctx->device);
    return cvib::run_pair_csr_summary(ctx, recs, offsets, n, summ, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_pair_reduce_rules(cv_context* ctx, const uint8_t* rgb, int64_t n, const cv_grid* grid,
                         const cv_rule* rules, int32_t nrules, uint32_t* counts, void* stream) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (n < 0) return fail(CV_EINVAL, "n < 0");
    if (!rules || nrules < 1 || nrules > 16) return fail(CV_EINVAL, "rules: 1..16 of them");
    if (n > 0 && (!rgb || !counts)) return fail(CV_EINVAL, "null array");
    cvib::GridDev gd;
    int rc;
    if ((rc = cvib::make_grid(grid, &gd)) != CV_OK) return rc;
    cvib::RuleDev rd[16];
    for (int r = 0; r < nrules; ++r)
        if ((rc = cvib::make_rule(&rules[r], &rd[r])) != CV_OK) return rc;
    DeviceGuard dg(ctx->device);
    return cvib::run_pair_reduce_rules(ctx, rgb, n, gd, rd, nrules, counts, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_context_set_autotune(cv_context* ctx, int on) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    ctx->autotune = on != 0;
    return CV_OK;
    CV_GUARD_END
}

int cv_context_set_tile_target(cv_context* ctx, int32_t tiles) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (tiles != 0 && (tiles < 64 || tiles > (1 << 20))) return fail(CV_EINVAL, "tiles must be 0 or in [64, 2^20]");
    ctx->tiles_forced = tiles;
    return CV_OK;
    CV_GUARD_END
}

int cv_context_tile_target(cv_context* ctx, int64_t n, const cv_grid* grid, int search, int32_t* tiles_host,
                           int* tuned_host) {
    CV_GUARD_BEGIN
    if (!ctx || !tiles_host) return fail(CV_EINVAL, "null argument");
    if (n < 0) return fail(CV_EINVAL, "n < 0");
    cvib::GridDev gd;
    int rc;
    if ((rc = cvib::make_grid(grid, &gd)) != CV_OK) return rc;
    const uint64_t key = cvib::tiles_key(search ? 1 : 0, n, gd);
    *tiles_host = cvib::tiles_target(ctx, key);
    if (tuned_host) *tuned_host = ctx->tiles_forced == 0 && ctx->tiles_tuned.count(key) ? 1 : 0;
    return CV_OK;
    CV_GUARD_END
}

int cv_context_set_tune_file(cv_context* ctx, const char* path) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (!path || !*path) {
        ctx->tune_file.clear();
        return CV_OK;
    }
    const std::string head = tune_header(ctx->device);
    if (head.empty()) return fail(CV_EHIP, "hipGetDeviceProperties");
    std::map<uint64_t, int> res;
    std::map<uint64_t, int32_t> til;
    FILE* f = fopen(path, "r");
    if (f) {
        char line[512];
        bool first = true, mine = false, bad = false;
        while (fgets(line, sizeof line, f)) {
            std::string t(line);
            while (!t.empty() && (t.back() == '\n' || t.back() == '\r')) t.pop_back();
            if (first) {
                first = false;
                if (t.rfind("cvib-tune ", 0) != 0) {
                    bad = true;
                    break;
                }
                mine = t == head;  // another GPU's choices are left unread
                if (!mine) break;
                continue;
            }
            if (t.empty()) continue;
            char kind[16];
            unsigned long long key = 0;
            int v = 0;
            char extra = 0;
            if (sscanf(t.c_str(), "%15s %llx %d %c", kind, &key, &v, &extra) != 3) {
                bad = true;
                break;
            }
            if (std::strcmp(kind, "resolve") == 0 && v >= 0 && v < cvib::kResolveVariants) {
                res[(uint64_t)key] = v;
            } else if (std::strcmp(kind, "tiles") == 0 && tile_choice(v)) {
                til[(uint64_t)key] = v;
            } else {
                bad = true;
                break;
            }
        }
        fclose(f);
        if (bad) return fail(CV_EINVAL, std::string("not a tuning file: ") + path);
    }
    ctx->tune_file = path;
    const int rc = ctx->save_tuning();  // creates the file, or checks that it can be written
    if (rc != CV_OK) {
        ctx->tune_file.clear();
        return rc;
    }
    for (const auto& kv : res) ctx->resolve_tuned[kv.first] = kv.second;
    for (const auto& kv : til) ctx->tiles_tuned[kv.first] = kv.second;
    return ctx->save_tuning();
    CV_GUARD_END
}

int cv_context_set_resolve_variant(cv_context* ctx, int variant) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (variant < -1 || variant >= cvib::kResolveVariants) return fail(CV_EINVAL, "unknown resolve variant");
    ctx->resolve_forced = variant;
    return CV_OK;
    CV_GUARD_END
}

int cv_context_resolve_variant(cv_context* ctx, const cv_grid* grid, int rays, int* variant_host,
                               int* tuned_host) {
    CV_GUARD_BEGIN
    if (!ctx || !variant_host) return fail(CV_EINVAL, "null argument");
    cvib::GridDev gd;
    int rc;
    if ((rc = cvib::make_grid(grid, &gd)) != CV_OK) return rc;
    *variant_host = cvib::resolve_variant(ctx, gd, rays != 0);
    if (tuned_host)
        *tuned_host = ctx->resolve_forced < 0 && ctx->resolve_tuned.count(cvib::resolve_key(gd, rays != 0)) ? 1 : 0;
    return CV_OK;
    CV_GUARD_END
}

int cv_context_set_timing(cv_context* ctx, int on) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    if (on && !ctx->ev[0][0]) {
        for (auto& pr : ctx->ev)
            for (hipEvent_t& e : pr) CV_HIP(hipEventCreate(&e));
    }
    if (on && !ctx->stats.ptr) {
        int rc = ctx->ensure(ctx->stats, 128);
        if (rc != CV_OK) return rc;
        CV_HIP(hipMemset(ctx->stats.ptr, 0, 128));
        ctx->stats_base = 0;
        ctx->no_high_base = 0;
    }
    ctx->timing = on != 0;
    return CV_OK;
    CV_GUARD_END
}

int cv_context_set_gamut_cells(cv_context* ctx, int on) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    ctx->gamut_cells = on != 0;
    return CV_OK;
    CV_GUARD_END
}

int cv_context_skipped(cv_context* ctx, int64_t* skipped_host, int reset) {
    CV_GUARD_BEGIN
    if (!ctx || !skipped_host) return fail(CV_EINVAL, "null argument");
    DeviceGuard dg(ctx->device);
    uint64_t v = 0;
    if (ctx->stats.ptr) {
        uint64_t w[8];
        CV_HIP(hipDeviceSynchronize());
        CV_HIP(hipMemcpy(w, ctx->stats.ptr, sizeof(w), hipMemcpyDeviceToHost));
        for (uint64_t x : w) v += x;
    }
    *skipped_host = (int64_t)(v - ctx->stats_base);
    if (reset) ctx->stats_base = v;
    return CV_OK;
    CV_GUARD_END
}

int cv_context_no_high(cv_context* ctx, int64_t* in_gamut_host, int reset) {
    CV_GUARD_BEGIN
    if (!ctx || !in_gamut_host) return fail(CV_EINVAL, "null argument");
    DeviceGuard dg(ctx->device);
    uint64_t v = 0;
    if (ctx->stats.ptr) {
        uint64_t w[16];
        CV_HIP(hipDeviceSynchronize());
        CV_HIP(hipMemcpy(w, ctx->stats.ptr, sizeof(w), hipMemcpyDeviceToHost));
        for (int k = 8; k < 16; ++k) v += w[k];
    }
    *in_gamut_host = (int64_t)(v - ctx->no_high_base);
    if (reset) ctx->no_high_base = v;
    return CV_OK;
    CV_GUARD_END
}

int cv_context_kernel_time(cv_context* ctx, int phase, double* ms_host, int64_t* calls_host,
                           int reset) {
    CV_GUARD_BEGIN
    if (!ctx || !ms_host || !calls_host) return fail(CV_EINVAL, "null argument");
    if (phase < 0 || phase >= cv_context::kPhases) return fail(CV_EINVAL, "unknown timing phase");
    *ms_host = ctx->kernel_ms[phase];
    *calls_host = ctx->kernel_calls[phase];
    if (reset) {
        ctx->kernel_ms[phase] = 0.0;
        ctx->kernel_calls[phase] = 0;
    }
    return CV_OK;
    CV_GUARD_END
}

} // extern "C"
