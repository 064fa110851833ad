/*
 * cvib — colour-vibration pair search on AMD Instinct MI355X (gfx950).
 *
 * C-ABI of libcvib.so.  The operations follow Hattori & Hiraki, "Accelerated
 * and Optimized Search of Imperceptible Color Vibration for Embedding
 * Information into LCD images" (SIGGRAPH Asia 2022 Posters):
 *   - Section 2: the target colour is split into L*, a*, b*; displacement arrays
 *     D_a[i][j] = r_i sin(theta_j) and D_b[i][j] = r_i cos(theta_j) are added to
 *     a* and b* for one colour of the pair and subtracted for the other, L* is
 *     kept; both colours are turned back into RGB and the per-channel RGB
 *     difference decides whether the pair carries information (Fig. 1b).
 *   - Section 3: a channel bit is high (1) when its change exceeds V_th and low
 *     (0) when it is below V_th * R_novib; Table 1 lists the colours, the seven
 *     information patterns and the V_th / R_novib values.
 *
 * Conventions shared by every entry point
 *   - Every call returns an int status (CV_OK = 0 or a negative CV_E* code).
 *     No C++ exception crosses this boundary.  cv_last_error() returns a
 *     message for the calling thread's most recent failure.
 *   - Array pointers are DEVICE pointers owned by the caller unless the name
 *     ends in _host.  The library allocates device memory only inside a
 *     cv_context (workspace, tables), never in the caller's arrays.
 *   - Work is enqueued on the given stream (a hipStream_t passed as void*;
 *     NULL = the null stream) and is asynchronous, except where a *_host
 *     output forces a synchronisation (stated per call).
 *   - Calls on one context must not overlap in time (the workspace is
 *     shared); use one context per host thread / stream for concurrency.
 *   - Results are bitwise deterministic for a given input.
 *
 * Colour space (the paper names only "L*a*b*"): CIE 1976 L*a*b* with the D65
 * white and IEC 61966-2-1 sRGB primaries and transfer function.  A pair is in
 * gamut when every linear channel of both colours lies in [0, 1]; 8-bit values
 * use round-half-to-even; the channel change is |V+ - V-|; "exceeds" and
 * "below" are strict; pattern p = 4*bit_R + 2*bit_G + bit_B and p = 0 is never
 * a survivor.
 */
#ifndef CVIB_H
#define CVIB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define CV_OK 0
#define CV_EINVAL (-1)    /* bad argument (null pointer, bad grid or rule)  */
#define CV_ECAPACITY (-2) /* output too small; required size reported      */
#define CV_EHIP (-3)      /* a HIP runtime call failed                     */
#define CV_ENOMEM (-4)    /* device allocation failed                      */
#define CV_ESTATE (-5)    /* internal consistency check failed on device   */

/* ---- cv_lab_convert directions ---------------------------------------- */
#define CV_RGB8_TO_LAB 0  /* uint8 [n][3] sRGB -> float [n][3] L*, a*, b*   */
#define CV_LAB_TO_RGBF 1  /* float [n][3] L*a*b* -> float [n][4]:           */
                          /*   v_R, v_G, v_B = 255 * encode(linear), not     */
                          /*   rounded; [3] = 1.0 if in gamut else 0.0       */

/* ---- cv_pair_search flags --------------------------------------------- */
#define CV_EMIT_ALL 0x1u  /* testing: emit every candidate; cv_pair.flags   */
                          /* then tells gamut / validity                     */
#define CV_PER_RAY 0x8u   /* only the survivor of largest i of every ray    */
                          /* (colour, j), in (colour, j) order               */
#define CV_NO_NGAMUT 0x10u /* summaries without n_gamut (left 0): steps    */
                          /* that can hold no survivor are not evaluated    */

/* ---- rule flags -------------------------------------------------------- */
#define CV_RULE_CLIP 0x1u /* alternative gamut reading: clamp each encoded  */
                          /* value to [0, 255] instead of rejecting the pair */

/*
 * Search grid.  r_i = (i + 1) * dr for 0 <= i < nr; theta_j = j * dtheta_deg
 * degrees for 0 <= j < ntheta, measured from +b* towards +a* (D_a = r sin,
 * D_b = r cos, Section 2).  Requirements: dr > 0; 1 <= nr, ntheta <= 65535;
 * nr * ntheta < 2^31; 360 / dtheta_deg is an even integer N <= 8192 (the
 * angle table lives in LDS); ntheta <= N.
 */
typedef struct {
    double dr;
    int32_t nr;
    int32_t _pad0;
    double dtheta_deg;
    int32_t ntheta;
    int32_t _pad1;
} cv_grid;

/*
 * Predicate (Section 3, Table 1).  d_k = |V+_k - V-_k| for k in R, G, B.
 * high_k = d_k > v_th; low_k = d_k < v_th * r_novib.  A candidate survives when
 * both colours are in gamut, every channel is high or low, p != 0 and bit
 * (p - 1) of pattern_mask is set (0x7F accepts any pattern).
 * Requirements: 0 < v_th <= 255; 0 < r_novib < 1; pattern_mask & 0x7F != 0.
 */
typedef struct {
    int32_t v_th;
    int32_t _pad0;
    double r_novib;
    uint32_t pattern_mask;
    uint32_t flags; /* CV_RULE_* */
} cv_rule;

/* One surviving pair, 16 bytes, written in (colour, i, j) order. */
typedef struct {
    uint32_t colour;   /* index into the caller's colour array */
    uint16_t i, j;     /* radius and angle index                */
    uint8_t plus[3];   /* 8-bit RGB of (L, a + D_a, b + D_b)    */
    uint8_t minus[3];  /* 8-bit RGB of (L, a - D_a, b - D_b)    */
    uint8_t pattern;   /* p in 1..7 (0 in CV_EMIT_ALL rows that encode none) */
    uint8_t flags;     /* bit0 + in gamut, bit1 - in gamut, bit2 survivor   */
} cv_pair;

/*
 * Per-colour summary, 48 bytes.  best_* is the maximum-amplitude survivor:
 * largest radius index i, ties broken by the smallest j (best_i = 0xFFFF and
 * the rest zero when there is no survivor).
 */
typedef struct {
    uint32_t count;          /* survivors                                   */
    uint32_t n_gamut;        /* candidates with both colours in gamut (0    */
                             /* with CV_NO_NGAMUT)                          */
    uint16_t best_i, best_j;
    uint8_t best_plus[3], best_minus[3], best_p, _pad;
    uint32_t per_pattern[7]; /* survivors with pattern p at index p - 1     */
} cv_color_summary;

/*
 * Angle-bin table row, 40 bytes: the valid count and, for each of 36 bins of
 * 10 degrees (bin = floor(theta_j / 10 deg)), the largest radius index i + 1
 * that has a survivor in that bin (0 = none).  Requires nr <= 255 and, for
 * the per-angle maxima kept in LDS, N <= 4096 with ntheta <= 4096.
 */
typedef struct {
    uint32_t count;
    uint8_t bin_ridx[36];
} cv_table_row;

/*
 * Best pair of one information pattern for one colour, 12 bytes: the
 * maximum-amplitude survivor (largest i, then smallest j) whose pattern is
 * p.  flags bit0 = a pair exists (all other fields zero otherwise).
 */
typedef struct {
    uint16_t i, j;
    uint8_t plus[3], minus[3];
    uint8_t pattern;
    uint8_t flags;
} cv_pattern_pair;

/* ---- cv_frames_resolve and cv_pair_search flags ----------------------- */
#define CV_GRAPH 0x2u     /* capture the whole call once as a hipGraph (on a */
                          /* stream of the context) and replay it; the graph */
                          /* is rebuilt when any argument changes            */

typedef struct cv_context cv_context;

/* Create a context on HIP device `device`.  *out receives the handle.
 * Errors: CV_EINVAL (out NULL / bad device), CV_EHIP. */
int cv_context_create(int device, cv_context** out);

/* Destroy a context and free its device memory (synchronises the device).
 * NULL is accepted and ignored. */
int cv_context_destroy(cv_context* ctx);

/* Message of the calling thread's most recent failed call ("" if none).
 * The pointer stays valid until the thread's next cvib call. */
const char* cv_last_error(void);

/*
 * Colour conversion (Section 2 and Fig. 2: the target colour is split into its
 * L*, a*, b* components; the inverse turns a displaced candidate back into
 * RGB).  `in` and `out` are device arrays of n items in the layouts of
 * CV_RGB8_TO_LAB / CV_LAB_TO_RGBF above.  n == 0 is a no-op.
 * Errors: CV_EINVAL (null pointer with n > 0, n < 0, unknown dir), CV_EHIP.
 */
int cv_lab_convert(cv_context* ctx, const void* in, void* out, int64_t n, int dir,
                   void* stream);

/*
 * Full search with stream compaction (Sections 1-2: the candidate pairs are
 * generated as arrays and the ones meeting both conditions are picked out).
 * rgb: uint8 [n][3] device array of target colours.  Survivors are written to
 * out[0 .. total) in (colour, i, j) order; offsets (int64 [n + 1], nullable)
 * receives per-colour CSR offsets; summ (cv_color_summary [n], nullable)
 * receives per-colour summaries.  *total_host receives the survivor total
 * (this synchronises the stream).  If total > capacity the call returns
 * CV_ECAPACITY and *total_host still holds the required total; offsets and
 * summ are complete and out holds the first `capacity` survivors (two-call
 * idiom: call again with capacity >= total).  capacity = 0 with out = NULL
 * is a pure count.  total_host may be NULL when offsets is not: the call
 * then returns once its work is enqueued, without reading anything back
 * (calls can follow each other on the stream with no host round trip);
 * offsets[n] holds the total on the device, survivors past `capacity` are
 * not written, and no CV_ECAPACITY is raised (compare offsets[n] with
 * capacity once the stream has reached the call).  The context's workspace grows with the number of
 * segments (one per row of radius when theta covers the full turn, else one
 * per 512 candidates): 12 bytes each.
 * With CV_GRAPH everything the call enqueues before the total is read back
 * is captured once as a hipGraph (on a stream of the context) and replayed by
 * later calls with the same arguments (pointers, sizes, grid, rule, flags)
 * and the same context workspaces; anything else captures again.  Results
 * are those of the eager call; no timing events are recorded inside the
 * graph.  CV_GRAPH is ignored with CV_PER_RAY.
 * With CV_NO_NGAMUT (not with CV_EMIT_ALL or CV_PER_RAY, where it is
 * ignored) the summaries' n_gamut is left 0, and the count pass does not
 * evaluate steps that its bounds show can hold no survivor; every other
 * output is unchanged.
 * With CV_PER_RAY (not with CV_EMIT_ALL) the records are, for every colour
 * and every ray j < ntheta that has a survivor, the survivor of largest
 * radius index i, in (colour, j) order; offsets and the two-call idiom work
 * as above, and the workspace holds 16 bytes per ray of every colour.
 * Errors: CV_EINVAL, CV_ECAPACITY, CV_EHIP, CV_ENOMEM, CV_ESTATE.
 */
int cv_pair_search(cv_context* ctx, const uint8_t* rgb, int64_t n, const cv_grid* grid,
                   const cv_rule* rule, cv_pair* out, int64_t capacity, int64_t* offsets,
                   cv_color_summary* summ, int64_t* total_host, uint32_t flags, void* stream);

/*
 * Search without materialising survivors (paper Section 2: the displaced
 * pairs of every (radius, angle) of the target's a*-b* plane, converted back
 * to RGB; Section 3 / Table 1: the high / low channel conditions that pick
 * the pairs out), reduced per colour: the survivor count, the per-pattern
 * counts, the in-gamut count and the maximum-amplitude pair (largest radius
 * index, then smallest angle index) -- and, if table is non-NULL, the largest
 * valid radius index of each 10-degree angle bin.  Fully asynchronous.
 * rgb: uint8 [n][3] device array, n on the host (a colour count that lives on
 * the device is served by cv_frames_resolve, which de-duplicates pixels and
 * searches the distinct colours without reading their number back).
 * summ: cv_color_summary [n] (nullable when table is given).  table:
 * cv_table_row [n] (nullable; requires nr <= 255).  The context's workspace
 * holds 64 bytes per colour (and 192 more per colour below 2048 colours).
 * Errors: CV_EINVAL, CV_EHIP, CV_ENOMEM.
 */
int cv_pair_reduce(cv_context* ctx, const uint8_t* rgb, int64_t n, const cv_grid* grid,
                   const cv_rule* rule, cv_color_summary* summ, cv_table_row* table,
                   void* stream);

/*
 * cv_pair_reduce without any allocation, for callers that cannot allocate
 * device memory during the call (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, outputs and
 * results as cv_pair_reduce, byte for byte.  The workspace is a fixed
 * 8 MiB device array per GPU (reserved when the library's code object loads,
 * kept until the process ends, its address looked up once per device by
 * cv_context_create); a call whose workspace would exceed it returns
 * CV_ECAPACITY, naming the bytes it would need, without enqueuing anything.
 * The workspace is 64 bytes per colour plus the angle table, and 192 more
 * per colour below 2048 colours: e.g. up to ~130,000 colours on the 2-degree
 * cube grid.  Every call on one GPU shares that array, so calls
 * that overlap on one GPU (two streams, two threads, two contexts) race and
 * must be serialised by the caller; each call clears what it needs zeroed.
 * Kernel timing (cv_context_set_timing) records nothing for these calls.
 * Errors: CV_EINVAL, CV_ECAPACITY, CV_EHIP, CV_ESTATE.
 */
int cv_pair_reduce_noalloc(cv_context* ctx, const uint8_t* rgb, int64_t n, const cv_grid* grid,
                           const cv_rule* rule, cv_color_summary* summ, cv_table_row* table,
                           void* stream);

/*
 * Summaries of a survivor list (the output of cv_pair_search, either mode):
 * recs (cv_pair, device) with CSR offsets (int64 [n + 1], device) -> summ
 * (cv_color_summary [n], device): count, per-pattern counts and the
 * maximum-amplitude record of each colour's range.  A list carries no gamut
 * count: n_gamut is 0.  Asynchronous.  Errors: CV_EINVAL, CV_EHIP.
 */
int cv_pair_reduce_csr(cv_context* ctx, const cv_pair* recs, const int64_t* offsets, int64_t n,
                       cv_color_summary* summ, void* stream);

/*
 * Adaptive per-ray search (the search space of Section 1 cut down without
 * changing what is found): for every colour and every ray j < ntheta, the
 * largest radius index i at which the pair of Section 2 passes Section 3's
 * predicate under `rule` -- the maximum of the ray's survivors, as
 * CV_PER_RAY finds it.  Each ray is taken from its outermost radius inward in
 * blocks of 64 radii: an interval bound first closes the blocks in which one
 * colour is out of gamut throughout or no channel can change by more than
 * v_th; the first block it cannot close is evaluated candidate by candidate,
 * and so on inward until a survivor is found.  The result equals the
 * exhaustive search's bit for bit (same arithmetic on every evaluated
 * candidate).  Under CV_RULE_CLIP no block is closed.
 * rgb: uint8 [n][3] device.  rays: uint16 [n][ntheta] device: i + 1 of the
 * ray's largest survivor, 0 for a ray without one.  recs: nullable cv_pair
 * [n][ntheta] device: that survivor's record (flags bit 2 set), all zero
 * except the colour index for a ray without one.  best: nullable uint32 [n]
 * device: the colour's maximum-amplitude pair as a key i << 16 | (65535 - j)
 * (largest i, then smallest j; 0 = no survivor) -- the exact one-pair resolve
 * of a colour, found from the outermost radius inward.  counts: nullable
 * uint64 [3] device, overwritten: candidates evaluated, row blocks tested, row
 * blocks closed by the bound.  Asynchronous.  Errors: CV_EINVAL, CV_EHIP,
 * CV_ENOMEM.
 */
int cv_ray_search(cv_context* ctx, const uint8_t* rgb, int64_t n, const cv_grid* grid, const cv_rule* rule,
                  uint16_t* rays, cv_pair* recs, uint32_t* best, uint64_t* counts, void* stream);

/*
 * Exact one-pair resolve (the maximum-amplitude survivor of Sections 2-3 for
 * each colour, as the exhaustive search defines it: largest i, then smallest
 * j), with a global early exit: the radii are taken in levels of 64 from the
 * outermost inward; at each level every ray's block is closed by the interval
 * bound of cv_ray_search where it can, the others are evaluated with the
 * search's arithmetic, and the walk stops at the first level holding a
 * survivor.  Under CV_RULE_CLIP no block is closed.
 * rgb: uint8 [n][3] device.  best: nullable uint32 [n] device, the key
 * i << 16 | (65535 - j) (0 = no survivor).  pairs: nullable cv_pair [n]
 * device, that survivor's record (flags bit 2 set; all zero except the colour
 * index for a colour without one).  At least one of best and pairs.  counts:
 * nullable uint64 [3] device, overwritten: candidates evaluated, (ray, level)
 * blocks tested, blocks closed by the bound.  Asynchronous.
 * Errors: CV_EINVAL, CV_EHIP, CV_ENOMEM.
 */
int cv_best_pair_search(cv_context* ctx, const uint8_t* rgb, int64_t n, const cv_grid* grid, const cv_rule* rule,
                        uint32_t* best, cv_pair* pairs, uint64_t* counts, void* stream);

/*
 * Several rules in one pass (Table 1's twelve settings give Table 2): for
 * each colour and rule, the survivors of each pattern.  rules: host array of
 * nrules (1..16) cv_rule with the same flags (one gamut reading); together
 * their thresholds (v_th and ceil(v_th * r_novib) - 1 of each) may take at
 * most 12 distinct values.  rgb: uint8 [n][3] device (n <= 65536).  counts:
 * uint32 [n][nrules][7] device; [c][r][p-1] counts colour c's survivors of
 * pattern p under rule r (0 where the rule's mask leaves p out).
 * Asynchronous.  Errors: CV_EINVAL, CV_EHIP, CV_ENOMEM.
 */
int cv_pair_reduce_rules(cv_context* ctx, const uint8_t* rgb, int64_t n, const cv_grid* grid,
                         const cv_rule* rules, int32_t nrules, uint32_t* counts, void* stream);

/*
 * Batched frames (all device arrays).  The colours of npix pixels (uint8
 * [npix][3], e.g. several frames back to back) are de-duplicated: `colours`
 * receives the distinct colours in ascending R<<16|G<<8|B order (uint8
 * [colour_cap][3]), *ncolours (a DEVICE int64) their number and pixel_index
 * (uint32 [npix]) each pixel's position in that list.  Every distinct colour
 * is then searched on `grid` under `rule` in one persistent launch whose
 * colour count stays on the device: summ (cv_color_summary [colour_cap],
 * nullable), pbest (cv_pattern_pair [colour_cap][7]: the best pair of every
 * information pattern) and rays (uint16 [colour_cap][ntheta], nullable: per
 * ray the largest surviving radius index + 1, 0 = none).  If frame_a and
 * frame_b are given (uint8 [npix][3] each), they receive the two colours
 * that alternate on the display (Fig. 1a): for pixel k the pair of pattern
 * info[k] (1..7) of its colour, or, with info NULL or info[k] = 0, the
 * colour's maximum-amplitude pair (info[k] > 7 selects none); a pixel
 * without such a pair keeps its colour in both frames.  *resolved (DEVICE
 * int64, nullable; needs the frames) counts the pixels that received a pair.
 * Nothing is copied to the host: the call is asynchronous, and with CV_GRAPH
 * it is one graph launch (captured again when an argument changes or a
 * context workspace had to grow).  With CV_NO_NGAMUT the summaries' n_gamut
 * is left 0 and steps that can hold no survivor are not evaluated (every
 * other output is unchanged; without summ this is always so).  The caller
 * owns every array; the context owns a 2^24-bit colour bitmap and its scan
 * (about 8 MiB).
 * Requirements: colour_cap >= min(npix, 2^24); the angle table (8 * (N/4 + 1)
 * bytes when N % 4 == 0, else 16 * (N/2 + 1)) plus, with rays, 4 bytes per
 * evaluated ray (ntheta, or N/2 when theta spans the full turn) must fit in
 * one block's LDS.
 * Errors: CV_EINVAL, CV_EHIP, CV_ENOMEM.
 */
int cv_frames_resolve(cv_context* ctx, const uint8_t* pixels, int64_t npix, const uint8_t* info,
                      const cv_grid* grid, const cv_rule* rule, uint8_t* colours,
                      int64_t colour_cap, int64_t* ncolours, uint32_t* pixel_index,
                      cv_color_summary* summ, cv_pattern_pair* pbest, uint16_t* rays,
                      uint8_t* frame_a, uint8_t* frame_b, int64_t* resolved, uint32_t flags,
                      void* stream);

/*
 * Synthetic frames for the batched calls (the paper's display frames are not
 * given; these stand in for them): n frames of height x width sRGB8 pixels,
 * frame f from seeds[f] (host array), written back to back to out (DEVICE
 * uint8 [n][height][width][3], owned by the caller).  Each frame is smooth
 * per-channel gradients, plus a constant offset per region of the nearest of
 * `sites` random sites, plus a rounded noise of amplitude `noise`.  All its
 * arithmetic is integer and every random word is Philox4x64-10 (Salmon et
 * al., SC'11) of a fixed counter under the key (seeds[f], 0), so that the
 * bytes are the same on any implementation of that definition:
 *   words(0, 0, 0, 0): per channel c from byte c of words 0, 1, 2:
 *     g0 = 64 + b % 129, gx = b % 129 - 64, gy = b % 129 - 64;
 *   words(1, s, 0, 0), site s: x = word0 % width, y = word1 % height,
 *     v_c = (byte c of word2) % 97 - 48;
 *   words(2, y, x, 0), pixel (x, y): n_c = (sum of bytes 4c..4c+3 of words
 *     0 and 1 as 16 little-endian bytes - 510) * noise / 128;
 *   channel c = clamp(g0 + gx x / width + gy y / height + v_c(nearest site)
 *     + n_c, 0, 255), the nearest site by squared distance with ties to the
 *     lowest index, every division truncating toward zero.
 * height and width in [1, 16384], sites in [1, 256], noise in [0, 255].
 * Asynchronous (one launch per frame).  Errors: CV_EINVAL, CV_EHIP.
 */
int cv_frames_generate(cv_context* ctx, const uint64_t* seeds, int64_t n, int32_t height, int32_t width,
                       int32_t sites, int32_t noise, uint8_t* out, void* stream);

/*
 * Kernel timing for measurement.  When enabled, the library brackets its
 * kernels with HIP events on the caller's stream and accumulates the elapsed
 * time per phase:
 *   CV_TIME_EVAL  - the evaluation kernel over every candidate (the reduce-only
 *                   kernel; in cv_pair_search its count pass),
 *   CV_TIME_WRITE - the write pass of cv_pair_search,
 *   CV_TIME_CALL  - everything a cv_pair_search / cv_pair_reduce call enqueues
 *                   after its set-up (evaluation, scan, write).
 * In cv_frames_resolve, CV_TIME_EVAL is the per-colour resolve kernel; in the
 * surrogate calls it is the exact fallback, CV_TIME_MLP the network and
 * CV_TIME_VERIFY the proposal check.
 * While timing is on, cv_pair_reduce synchronises its stream.
 * cv_context_kernel_time returns the accumulated milliseconds and the number
 * of timed calls for one phase (host pointers) and clears that phase when
 * reset != 0.  Errors: CV_EINVAL (null ctx / outputs, bad phase), CV_EHIP.
 */
/*
 * Gamut cells.  Before evaluating, the search kernels prove by interval
 * arithmetic (FP64, with a margin of 1e-6 on the linear channels) which wave
 * steps of 64 candidates hold no pair with both colours in gamut, and skip
 * them: the reduce-only kernel (cv_pair_reduce, the count pass of
 * cv_pair_search), the write pass of cv_pair_search (not with CV_EMIT_ALL),
 * the multi-rule pass (cv_pair_reduce_rules) and the per-colour resolve (cv_frames_resolve, the exact fallback of the
 * surrogate calls), which takes its candidates in bands of 16 rows so that
 * a step covers 4 rays.  Cells are used when the rule requires the gamut
 * (not CV_RULE_CLIP) and a row holds at least 128 evaluated rays.  Results
 * are identical with the cells on (the default) or off.
 * cv_context_set_gamut_cells turns them on or off for later calls.
 * cv_context_skipped returns (host pointer) the number of candidates the
 * cells skipped in the reduce-only kernel (the count pass) in the calls made
 * while timing was on, since context creation
 * or the last reset (reset != 0 clears it after reading); it synchronises the
 * device.  Errors: CV_EINVAL (null ctx / output), CV_EHIP.
 * With the cells on, the reduce-only kernel over chunks of rows (the count
 * pass of cv_pair_search among them) also bounds the 8-bit codes of each
 * open step: an accepted pattern needs a channel that changes by more than
 * v_th codes, and where the bound shows that no channel can, the step's
 * pairs are only counted for n_gamut, without the encode (Section 3's
 * predicate cannot hold there).  cv_context_no_high returns, like
 * cv_context_skipped, the number of in-gamut pairs counted that way.
 */
int cv_context_set_gamut_cells(cv_context* ctx, int on);
int cv_context_skipped(cv_context* ctx, int64_t* skipped_host, int reset);
int cv_context_no_high(cv_context* ctx, int64_t* in_gamut_host, int reset);

/*
 * Kernel choice for the per-colour resolve (cv_frames_resolve and the exact
 * fallback of the surrogate calls; the project's autotuner, which also picks
 * the tiling of the chunked reduce below): variant 0 gives one colour to a block of
 * four waves, 1 one colour to each wave with four waves per block, 2 the
 * same with eight waves per block.  All give identical results.  With
 * autotuning on, the first cv_frames_resolve call of a grid shape (nr,
 * ntheta, N, per-ray output or not) runs once eagerly, then times every
 * variant that fits in LDS on up to 8192 of its colours and keeps the
 * fastest for that shape in the context.  A forced variant (0..2) overrides
 * the tuning; -1 returns to it.  cv_context_resolve_variant reports the
 * variant a call of that shape would use and (tuned_host, nullable) whether it
 * came from tuning.  Errors: CV_EINVAL.
 */
int cv_context_set_autotune(cv_context* ctx, int on);
int cv_context_set_resolve_variant(cv_context* ctx, int variant);
int cv_context_resolve_variant(cv_context* ctx, const cv_grid* grid, int rays, int* variant_host,
                               int* tuned_host);

/*
 * Tiling of the chunked reduce (the count pass of cv_pair_search, and
 * cv_pair_reduce when the colours are too few for one block each): about
 * `tiles` tiles per call, each a run of one colour's (i, j) grid.  Every
 * tiling gives identical results.  With autotuning on, the first eager call
 * of a shape (count pass or reduce, colour count, nr, ntheta, N) times the
 * tilings 1024, 2048, 4096, 8192 and 16384 (two runs each; the last leaves
 * the call's outputs) and keeps the fastest in the context; a captured
 * (CV_GRAPH) call uses the choice made so far.  cv_context_set_tile_target
 * forces a tiling (64 .. 2^20) or returns to the tuned one (0; 4096 untuned).
 * cv_context_tile_target reports the tiling a call of that shape would use
 * (search != 0: the count pass) and (tuned_host, nullable) whether it came
 * from tuning.  Errors: CV_EINVAL.
 */
int cv_context_set_tile_target(cv_context* ctx, int32_t tiles);
int cv_context_tile_target(cv_context* ctx, int64_t n, const cv_grid* grid, int search, int32_t* tiles_host,
                           int* tuned_host);

/*
 * On-disk cache of the tuned choices (resolve variants and tilings): a text
 * file whose first line names the format, the GPU architecture and its
 * compute-unit count, then one line per choice ("resolve <key> <variant>" or
 * "tiles <key> <tiles>", keys in hex).  Setting a path loads the choices of a
 * file written for this GPU model (a file of another model is left unread and
 * is rewritten at the next tuning), creates the file if it is missing, and
 * has every later tuning rewrite it (through a temporary file and a rename).
 * NULL or "" detaches the file.  Errors: CV_EINVAL (a file that is not a
 * tuning file, or a path that cannot be written), CV_EHIP.
 */
int cv_context_set_tune_file(cv_context* ctx, const char* path);

#define CV_TIME_EVAL 0
#define CV_TIME_WRITE 1
#define CV_TIME_CALL 2
#define CV_TIME_MLP 3     /* surrogate: the network's forward pass            */
#define CV_TIME_VERIFY 4  /* surrogate: proposals through the exact predicate */
int cv_context_set_timing(cv_context* ctx, int on);
int cv_context_kernel_time(cv_context* ctx, int phase, double* ms_host, int64_t* calls_host,
                           int reset);

/* ---- Surrogate network ------------------------------------------------
 *
 * A multilayer perceptron dims[0] -> dims[1] -> ... -> dims[nlayers] with
 * ReLU after every layer but the last; the first hidden layer may instead be
 * sinusoidal, sin(omega0 z) (cv_mlp_set_first_sine).  The surrogate of the
 * exact search is 3 -> 256 -> 256 -> 256 -> 37 with a sinusoidal first layer
 * (omega0 = 20): input RGB / 255 - 1/2, outputs the largest
 * valid radius of each of the 36 angle bins divided by 50 (the table of
 * cv_pair_reduce) and a feasibility logit.  The paper describes no learned
 * part; the network only proposes pairs that the exact predicate re-checks
 * (cv_surrogate_infer), and its targets come from the exact search.
 *
 * Arithmetic: the input layer in FP32; every other layer multiplies BF16
 * activations by BF16 copies of the weights with FP32 accumulation, adds the
 * FP32 bias, and rounds hidden activations to BF16 after the activation.  The
 * backward pass of a sinusoidal first layer recomputes z in FP32 from x.  The
 * network owns FP32 master weights, their gradients and the Adam moments.
 * Parameters are one flat FP32 array, layer by layer: W_l row-major
 * [dims[l+1]][dims[l]], then b_l [dims[l+1]].  All array arguments are
 * device pointers owned by the caller unless noted.
 * Limits: 2 <= nlayers <= 8, dims[0] = 3, hidden widths multiples of 32 in
 * [32, 1024], output width in [2, 256].
 */
typedef struct cv_mlp cv_mlp;

#define CV_MLP_KEEP 0x1u  /* keep the activations for cv_mlp_backward        */
#define CV_MLP_RGB8 0x2u  /* x is uint8 RGB [B][3] instead of float [B][3]   */

/* Create / destroy.  Weights start at zero: set them with cv_mlp_set_params
 * or cv_mlp_load.  Errors: CV_EINVAL, CV_EHIP. */
int cv_mlp_create(cv_context* ctx, const int32_t* dims_host, int32_t nlayers, cv_mlp** out);
int cv_mlp_destroy(cv_mlp* m);
int cv_mlp_num_params(const cv_mlp* m, int64_t* n_host);

/* First hidden layer h1 = sin(omega0 (W_0 x + b_0)) for omega0 > 0, ReLU for
 * omega0 = 0 (the default).  Applies to every later forward and backward
 * pass; the training step does not change it.  Errors: CV_EINVAL for a
 * negative or non-finite omega0. */
int cv_mlp_set_first_sine(cv_mlp* m, float omega0);
int cv_mlp_first_sine(const cv_mlp* m, float* omega0_host);

/* Copy the flat FP32 parameters in (this also clears the Adam moments) or
 * out, and the gradients of the last cv_mlp_backward out (either output may
 * be NULL, not both).  Asynchronous on `stream`. */
int cv_mlp_set_params(cv_mlp* m, const float* params, void* stream);
int cv_mlp_get_params(const cv_mlp* m, float* params, float* grads, void* stream);

/* Forward pass of B rows: x float [B][3] (or uint8 [B][3] with CV_MLP_RGB8)
 * -> out float [B][dims[nlayers]].  With CV_MLP_KEEP (B <= 2^24) the hidden
 * activations stay in the network for the next cv_mlp_backward; without it
 * rows go through in chunks of 2^20 (B <= 2^30). */
int cv_mlp_forward(cv_mlp* m, const void* x, int64_t B, float* out, uint32_t flags, void* stream);

/* The BF16 activations of hidden layer `layer` (1 .. nlayers - 1) kept by the
 * last forward pass with CV_MLP_KEEP, widened to FP32: out [B][dims[layer]]
 * device, for the first B rows of that batch (CV_ESTATE without such a pass).
 * These are the values the next layer's matrix product and the backward pass
 * read.  Asynchronous.  Errors: CV_EINVAL, CV_ESTATE, CV_EHIP. */
int cv_mlp_hidden(const cv_mlp* m, int32_t layer, float* out, int64_t B, void* stream);

/* Training loss of B rows and its gradient with respect to the outputs.
 * out [B][D] (D = dims[nlayers]); t_r [B][D-1] radius targets (a bin with
 * t_r <= 0 carries no radius loss); t_f [B] feasibility targets in {0, 1}.
 *   loss = (1/B) sum_s [ (1/(D-1)) sum_k [t_r > 0] huber_delta(out_k - t_r,k)
 *                        + log(1 + e^z) - z t_f ],   z = out_{D-1}
 * *loss: device float [1].  gout [B][D] (nullable) receives dloss/dout. */
int cv_mlp_loss(cv_mlp* m, const float* out, const float* t_r, const float* t_f, int64_t B,
                float huber_delta, float* loss, float* gout, void* stream);

/* Gradients of sum(gout * out) with respect to all parameters, for the batch
 * of the last kept forward pass (same x and B; CV_ESTATE otherwise).  The
 * gradients stay in the network (cv_mlp_get_params reads them). */
int cv_mlp_backward(cv_mlp* m, const float* x, const float* gout, int64_t B, void* stream);

/* One Adam step (Kingma & Ba 2015) with bias correction for step t >= 1 on
 * the gradients of the last backward pass. */
int cv_adam_step(cv_mlp* m, float lr, float beta1, float beta2, float eps, int64_t t, void* stream);

/* A run of training steps in one call: rows ids[0..n) (colour ids, already
 * shuffled; device int32) are taken batch by batch from the whole-cube table
 * (as cv_mlp_table_batch), and each batch does forward, loss (huber_delta),
 * backward and an Adam step (beta 0.9, 0.999; eps 1e-8) whose learning rate
 * decays by a cosine from lr_max at step 0 to lr_min at step total_steps - 1
 * (steps counted from step0 across calls; Adam's t = step + 1).  The last
 * batch may be short.  loss_log (device float [ceil(n / batch)], nullable)
 * receives each step's loss.  The call leaves no kept forward pass
 * (cv_mlp_hidden and cv_mlp_backward return CV_ESTATE until the next forward
 * with CV_MLP_KEEP).  Asynchronous. */
int cv_mlp_train_steps(cv_mlp* m, const int32_t* ids, int64_t n, const cv_table_row* table, double dr,
                       int64_t batch, float huber_delta, float lr_max, float lr_min, int64_t step0,
                       int64_t total_steps, float* loss_log, void* stream);

/* Training rows from a whole-cube table (cv_table_row [2^24], indexed by
 * colour id R<<16 | G<<8 | B, made on a grid of radius step dr): for each of
 * the B colour ids, x = RGB / 255 - 1/2, t_r[k] = bin_ridx[k] * dr / 50,
 * t_f = (count > 0).  Needs a 3 -> ... -> 37 network. */
int cv_mlp_table_batch(cv_mlp* m, const int32_t* ids, const cv_table_row* table, int64_t B,
                       double dr, float* x, float* t_r, float* t_f, void* stream);

/* Training order: out[i] = in[pi(i)] for a keyed pseudorandom permutation pi
 * of [0, n) (a four-round Feistel network on the smallest even bit width
 * that holds n, cycle-walked into [0, n); Black and Rogaway 2002).  The same
 * key gives the same order on every device.  in and out are device int32
 * arrays of n entries that must not overlap; n <= 2^31.  Asynchronous.
 * Errors: CV_EINVAL. */
int cv_permute_ids(cv_context* ctx, const int32_t* in, int64_t n, uint64_t key, int32_t* out, void* stream);

/* Parameters to / from a file (host path): magic "CVMLP02", int32 nlayers,
 * int32 dims[nlayers+1], int64 count, float omega0, float params[count],
 * little-endian.  Loading requires the same shape, takes omega0 from the file
 * (a "CVMLP01" file has no omega0 field and loads as omega0 = 0) and clears
 * the Adam moments.  Both synchronise the device. */
int cv_mlp_save(const cv_mlp* m, const char* path);
int cv_mlp_load(cv_mlp* m, const char* path);

/* Training checkpoint (host path), to stop training and resume it later with
 * results identical to an uninterrupted run: magic "CVCKP01", int32 nlayers,
 * int32 dims[nlayers+1], int64 count, float omega0, int64 step (training
 * steps done, the next Adam step is step + 1), uint64 key (the caller's
 * training-order key), float params[count], float adam_m[count], float
 * adam_v[count], then uint64 FNV-1a-64 of every preceding byte;
 * little-endian.  Loading checks the magic, the field sizes against the file
 * length, the hash (a corrupt or truncated file is CV_EINVAL) and the shape
 * (another network's checkpoint is CV_EINVAL), then restores parameters,
 * moments and omega0, and returns step and key (either may be NULL).  Save
 * and load synchronise the device.  cv_mlp_checkpoint_info reads and checks a
 * file without any device: nlayers, dims (int32 [nlayers + 1], room for 9),
 * step, key (each nullable). */
int cv_mlp_save_checkpoint(const cv_mlp* m, const char* path, int64_t step, uint64_t key);
int cv_mlp_load_checkpoint(cv_mlp* m, const char* path, int64_t* step, uint64_t* key);
int cv_mlp_checkpoint_info(const char* path, int32_t* nlayers, int32_t* dims, int64_t* step, uint64_t* key);

/* ---- Surrogate resolve -------------------------------------------------
 *
 * One verified pair per target colour, proposed by a 3 -> ... -> 37 network
 * (radii of the 36 angle bins / 50 and a feasibility logit, as trained on
 * the table of cv_pair_reduce) and checked by the exact predicate.
 *
 * For a colour whose logit is >= tau, the network's kbins bins of largest
 * predicted radius r (1 <= kbins <= 36) each propose every ray j of the bin
 * (floor(36 j / N) = bin, j < ntheta) at the grid radii nearest to r + o,
 * o in {+1, 0, -1, -2.5, -5, -10} (Delta E 1976 units).  When theta spans
 * the full turn only the 18 bins of the first half-turn are ranked (by the
 * mean prediction of bin b and its mirror b + 18) and proposed.  Every
 * proposal runs through the same arithmetic as the exact search, so a
 * verified pair is one of its survivors; the verified proposal of largest i
 * (then smallest j) is kept.  A local search through the same predicate then
 * raises it: its ray is climbed (the radii above it, 64 at a time, up to 512,
 * stopping at a block of 64 with no survivor), every ray of every proposed
 * bin is tried at the few radii above the kept one (64 / rays of the bin),
 * and the 16 rays around the kept ray (-8..+7) at the 4 radii above it, up
 * to 4 times; a survivor of larger i replaces the kept pair and its ray is
 * climbed.  The bin sweep continues down the ranking through the bins whose
 * predicted radius comes within 5 Delta E of the kept one.  The result is
 * never above the exact search's best pair.  Low confidence: unless
 * CV_NO_FALLBACK is set, a colour whose verified radius is more than 10
 * Delta E below the largest predicted bin radius goes to the exact search.
 * Colours with a lower logit or with no verified proposal go to the exact
 * search (its maximum-amplitude pair), unless CV_NO_FALLBACK is set.
 */
#define CV_NO_FALLBACK 0x4u
/* cv_surrogate_infer only: `pred` is an input -- proposals from the caller in
 * the network's output layout (36 bin radii / 50, then a feasibility logit),
 * e.g. a lookup in a table or a constant prior -- and no network runs (mlp
 * may be NULL).  Everything after the network is the same: proposals are
 * verified by the exact predicate and the rest falls back. */
#define CV_PRED_GIVEN 0x20u

/* cv_pattern_pair.flags of a resolved pair */
#define CV_PAIR_FOUND 0x1u      /* the pair exists                          */
#define CV_PAIR_SURROGATE 0x2u  /* proposed by the network and verified     */
#define CV_PAIR_FALLBACK 0x4u   /* found by the exact search                */

/* per-colour status */
#define CV_RESOLVED_SURROGATE 0  /* verified proposal                       */
#define CV_RESOLVED_EXACT 1      /* exact fallback found a pair             */
#define CV_RESOLVED_NONE 2       /* no pair (infeasible, or no fallback)    */

/* A list of n colours (uint8 [n][3], the same colour layout as every other
 * call).  pairs: cv_pattern_pair [n]; status: uint8 [n]; pred: float [n][37]
 * (nullable) receives the network outputs (the 36 bin radii / 50, then the
 * feasibility logit); fallback (uint32 [n], nullable) receives the indices of
 * the colours that need the exact search (low logit, no verified proposal, or
 * low confidence), in increasing order -- sent to it unless CV_NO_FALLBACK is
 * set; *nfallback (DEVICE int64, nullable) their number.  All device arrays.  Asynchronous.
 * Errors: CV_EINVAL, CV_EHIP, CV_ENOMEM. */
int cv_surrogate_infer(cv_context* ctx, cv_mlp* mlp, const uint8_t* rgb, int64_t n,
                       const cv_grid* grid, const cv_rule* rule, float tau, int32_t kbins,
                       float* pred, cv_pattern_pair* pairs, uint8_t* status, uint32_t* fallback,
                       int64_t* nfallback, uint32_t flags, void* stream);

/* Batched frames through the surrogate: the de-duplication of
 * cv_frames_resolve (colours, *ncolours, pixel_index as there), one
 * surrogate-resolved pair per distinct colour (pairs, status [colour_cap]),
 * and frames A / B (uint8 [npix][3] each, nullable together) showing the +
 * and - colour of the pixel's pair (a pixel without one keeps its colour);
 * *resolved (DEVICE int64, nullable) counts pixels with a pair and
 * *nfallback (DEVICE int64, nullable) the colours sent to the exact search.
 * Reads the colour count back to the host once (the network runs on exactly
 * that many rows), so the call synchronises its stream.
 * Errors: CV_EINVAL, CV_EHIP, CV_ENOMEM. */
int cv_frames_surrogate(cv_context* ctx, cv_mlp* mlp, const uint8_t* pixels, int64_t npix,
                        const cv_grid* grid, const cv_rule* rule, float tau, int32_t kbins,
                        uint8_t* colours, int64_t colour_cap, int64_t* ncolours,
                        uint32_t* pixel_index, cv_pattern_pair* pairs, uint8_t* status,
                        uint8_t* frame_a, uint8_t* frame_b, int64_t* resolved, int64_t* nfallback,
                        uint32_t flags, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CVIB_H */
