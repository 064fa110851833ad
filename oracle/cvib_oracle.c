/*
 * FP64 CPU oracle for the imperceptible colour-vibration pair search
 * (Hattori & Hiraki, "Accelerated and Optimized Search of Imperceptible Color
 * Vibration for Embedding Information into LCD images", SIGGRAPH Asia 2022
 * Posters).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow definition that the
 * GPU library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant generator with the HIP library: every constant below is
 * derived here from the published standards (IEC 61966-2-1 sRGB, CIE 1976
 * L*a*b*, D65 white).
 *
 * What the paper fixes and what is a reading:
 *  - Section 2: a pair is two colours point-symmetric about the target in
 *    L*a*b* with L* held fixed.  The target is split into L*, a*, b*; the
 *    displacement arrays D_a[i][j] = i sin j and D_b[i][j] = i cos j are added
 *    to a* and b* for one colour of the pair and subtracted for the other.
 *  - Section 2 / Fig. 1b: the RGB difference between the two colours decides
 *    whether the pair vibrates.
 *  - Section 3: a channel bit is high when its change exceeds V_th and low when
 *    its change is below V_th * R_novib (Table 1 gives the values).
 *  - Readings where the paper is silent (all listed in the design notes):
 *    CIE 1976 L*a*b* with D65/2deg and sRGB primaries; the IEC piecewise
 *    transfer; r_i = (i+1)*dr and theta_j = j*dtheta degrees; a pair is in
 *    gamut only if every linear channel of both colours lies in [0,1]; 8-bit
 *    values use round-half-to-even; "change" is the peak-to-peak |V+ - V-| of
 *    the 8-bit pair; "exceeds"/"below" are strict; a channel between the two
 *    thresholds encodes nothing; pattern p = 4*R + 2*G + B, p = 0 is never a
 *    survivor; amplitude order = larger i first, then smaller j.
 *
 * Boundary candidates: a candidate is flagged when an FP32 evaluation could
 * plausibly decide it differently: some channel of an in-gamut-or-nearly pair
 * lies within 1e-3 (in 0..255 units) of a rounding tie (k + 0.5) or of the
 * gamut edges 0 / 255.  Survivor parity is exact on every other candidate.
 *
 * Function "parity pins" (the checks that tie this code to something other
 * than itself) live in the test suite: round trip of all 2^24 colours, the
 * r = 0 and point-symmetry invariants, fixed-Y (fixed L*) closed form, neutral
 * axis a* = b* = 0, a 50-digit brute force of a hand grid, Table 2's presence
 * bits, and finite differences for the MLP gradients.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Types shared with the Python side through ctypes (layouts mirrored there). */

typedef struct {
    double dr;          /* radius step; r_i = (i+1) * dr                      */
    int32_t nr;         /* number of radii                                    */
    int32_t _pad0;
    double dtheta_deg;  /* angle step in degrees; theta_j = j * dtheta_deg     */
    int32_t ntheta;     /* number of angles                                   */
    int32_t _pad1;
} orc_grid;

typedef struct {
    int32_t v_th;       /* V_th of Table 1                                    */
    int32_t _pad0;
    double r_novib;     /* R_novib of Table 1                                 */
    uint32_t mask;      /* bit (p-1) set => pattern p accepted (0x7F = any)   */
    uint32_t flags;     /* bit0: clip reading (clamp codes to [0,255] instead  */
                        /*       of rejecting out-of-gamut pairs)              */
} orc_rule;

/* One evaluated candidate: everything the tests compare. */
typedef struct {
    double vp[3];       /* 255 * encode(linear) for the + colour, unrounded   */
    double vm[3];       /* same for the - colour                              */
    double linp[3];     /* linear RGB of the + colour                         */
    double linm[3];
    uint8_t Vp[3];      /* rounded 8-bit values (valid when in gamut)         */
    uint8_t Vm[3];
    uint8_t gamut;      /* bit0: + in gamut, bit1: - in gamut                 */
    uint8_t pattern;    /* 4*hiR + 2*hiG + hiB when every channel is hi or lo */
    uint8_t valid;      /* survivor under the rule                            */
    uint8_t boundary;   /* bit0: some channel within the 1e-3 band; bit1: a    */
                        /* value inside the band changes the decision         */
    uint8_t dset;       /* decisions reachable inside the band: bit 0 = not a  */
                        /* survivor, bit p = survivor of pattern p (0 without */
                        /* a rule)                                            */
    uint8_t _pad[3];
} orc_cand;

/* Survivor record, 16 bytes, emitted in (colour, i, j) order. */
typedef struct {
    uint32_t colour;
    uint16_t i, j;
    uint8_t plus[3], minus[3];
    uint8_t pattern;
    uint8_t flags;      /* bit0: boundary candidate */
} orc_rec;

/* Per-colour summary. */
typedef struct {
    uint32_t count;          /* survivors                                    */
    uint32_t n_gamut;        /* candidates with both colours in gamut        */
    uint32_t n_boundary;     /* boundary candidates (bit0)                   */
    uint32_t n_ambiguous;    /* candidates whose decision the band can flip  */
    uint16_t best_i, best_j; /* max-amplitude survivor (0xFFFF if none)      */
    uint8_t best_plus[3], best_minus[3], best_p, _pad;
    uint32_t per_pattern[7]; /* survivors with pattern p at index p-1        */
} orc_summary;

/* ------------------------------------------------------------------------- */
/* Colour science (IEC 61966-2-1 sRGB, CIE 1976 L*a*b*).                      */

static const double DELTA = 6.0 / 29.0;

/* sRGB primaries and the D65 white point, CIE xy chromaticities. */
static const double XR = 0.64, YR = 0.33;
static const double XG = 0.30, YG = 0.60;
static const double XB = 0.15, YB = 0.06;
static const double XW = 0.3127, YW = 0.3290;

static void inv3(const double a[9], double out[9]) {
    double c00 = a[4] * a[8] - a[5] * a[7];
    double c01 = a[5] * a[6] - a[3] * a[8];
    double c02 = a[3] * a[7] - a[4] * a[6];
    double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    out[0] = c00 / det;
    out[1] = (a[2] * a[7] - a[1] * a[8]) / det;
    out[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    out[3] = c01 / det;
    out[4] = (a[0] * a[8] - a[2] * a[6]) / det;
    out[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    out[6] = c02 / det;
    out[7] = (a[1] * a[6] - a[0] * a[7]) / det;
    out[8] = (a[0] * a[4] - a[1] * a[3]) / det;
}

/* M maps linear sRGB to XYZ: columns are the primaries' XYZ scaled so that
 * RGB = (1,1,1) lands on the white point W (with Y_W = 1). */
void orc_matrices(double M[9], double Minv[9], double W[3]) {
    double P[9] = {
        XR / YR, XG / YG, XB / YB,
        1.0, 1.0, 1.0,
        (1.0 - XR - YR) / YR, (1.0 - XG - YG) / YG, (1.0 - XB - YB) / YB,
    };
    double w[3] = {XW / YW, 1.0, (1.0 - XW - YW) / YW};
    double Pinv[9], S[3];
    inv3(P, Pinv);
    for (int r = 0; r < 3; ++r)
        S[r] = Pinv[3 * r] * w[0] + Pinv[3 * r + 1] * w[1] + Pinv[3 * r + 2] * w[2];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] = P[3 * r + c] * S[c];
    inv3(M, Minv);
    if (W) { W[0] = w[0]; W[1] = w[1]; W[2] = w[2]; }
}

/* sRGB transfer: non-linear c in [0,1] -> linear. */
double orc_decode(double c) {
    return c <= 0.04045 ? c / 12.92 : pow((c + 0.055) / 1.055, 2.4);
}

/* sRGB transfer: linear -> non-linear.  Extended to all reals by its own
 * branches (the linear branch for l <= 0.0031308, the power branch above), so
 * that out-of-gamut values keep a finite, monotone code value. */
double orc_encode(double l) {
    return l <= 0.0031308 ? 12.92 * l : 1.055 * pow(l, 1.0 / 2.4) - 0.055;
}

static double lab_f(double t) {
    return t > DELTA * DELTA * DELTA ? cbrt(t) : t / (3.0 * DELTA * DELTA) + 4.0 / 29.0;
}

static double lab_finv(double u) {
    return u > DELTA ? u * u * u : 3.0 * DELTA * DELTA * (u - 4.0 / 29.0);
}

void orc_rgb8_to_lab(const uint8_t* rgb, int64_t n, double* lab) {
    double M[9], Minv[9], W[3];
    orc_matrices(M, Minv, W);
    for (int64_t k = 0; k < n; ++k) {
        double lin[3], xyz[3];
        for (int c = 0; c < 3; ++c) lin[c] = orc_decode(rgb[3 * k + c] / 255.0);
        for (int r = 0; r < 3; ++r)
            xyz[r] = M[3 * r] * lin[0] + M[3 * r + 1] * lin[1] + M[3 * r + 2] * lin[2];
        double fx = lab_f(xyz[0] / W[0]);
        double fy = lab_f(xyz[1] / W[1]);
        double fz = lab_f(xyz[2] / W[2]);
        lab[3 * k + 0] = 116.0 * fy - 16.0;
        lab[3 * k + 1] = 500.0 * (fx - fy);
        lab[3 * k + 2] = 200.0 * (fy - fz);
    }
}

/* L*a*b* -> linear sRGB (not clipped). */
static void lab_to_linear1(const double M_inv[9], const double W[3], const double lab[3], double lin[3]) {
    double fy = (lab[0] + 16.0) / 116.0;
    double fx = fy + lab[1] / 500.0;
    double fz = fy - lab[2] / 200.0;
    double xyz[3] = {W[0] * lab_finv(fx), W[1] * lab_finv(fy), W[2] * lab_finv(fz)};
    for (int r = 0; r < 3; ++r)
        lin[r] = M_inv[3 * r] * xyz[0] + M_inv[3 * r + 1] * xyz[1] + M_inv[3 * r + 2] * xyz[2];
}

void orc_lab_to_linear(const double* lab, int64_t n, double* lin) {
    double M[9], Minv[9], W[3];
    orc_matrices(M, Minv, W);
    for (int64_t k = 0; k < n; ++k) lab_to_linear1(Minv, W, lab + 3 * k, lin + 3 * k);
}

/* L*a*b* -> v = 255 * encode(linear), unrounded, plus a gamut flag
 * (1 when all three linear channels lie in [0,1]). */
void orc_lab_to_v(const double* lab, int64_t n, double* v, uint8_t* gamut) {
    double M[9], Minv[9], W[3];
    orc_matrices(M, Minv, W);
    for (int64_t k = 0; k < n; ++k) {
        double lin[3];
        lab_to_linear1(Minv, W, lab + 3 * k, lin);
        int g = 1;
        for (int c = 0; c < 3; ++c) {
            v[3 * k + c] = 255.0 * orc_encode(lin[c]);
            if (!(lin[c] >= 0.0 && lin[c] <= 1.0)) g = 0;
        }
        if (gamut) gamut[k] = (uint8_t)g;
    }
}

/* ------------------------------------------------------------------------- */
/* The search.                                                                */

static const double BAND = 1e-3;
static const double PI = 3.14159265358979323846;

/* Angle theta_j = j * dtheta degrees; returned as radians after reducing the
 * degree value into [0, 360). */
static double theta_rad(const orc_grid* g, int32_t j) {
    double deg = fmod((double)j * g->dtheta_deg, 360.0);
    return deg * (PI / 180.0);
}

static int near_tie(double v) {
    double t = floor(v) + 0.5;
    return fabs(v - t) < BAND;
}

static int clearly_out(double v) { return v < -BAND || v > 255.0 + BAND; }
static int near_edge(double v) { return fabs(v) < BAND || fabs(v - 255.0) < BAND; }

typedef struct {
    double Minv[9], W[3];
    double L, a, b;
} orc_target;

static void target_init(orc_target* t, const uint8_t rgb[3]) {
    double M[9];
    orc_matrices(M, t->Minv, t->W);
    double lab[3];
    orc_rgb8_to_lab(rgb, 1, lab);
    t->L = lab[0]; t->a = lab[1]; t->b = lab[2];
}

/* Decision of a candidate from its gamut flags and 8-bit values under rule
 * ru: returns 0 when not a survivor, else 8 + pattern. */
static int decide_codes(const orc_rule* ru, int clip, int gp, int gm, const int Vp[3],
                        const int Vm[3]) {
    if (!(clip || (gp && gm))) return 0;
    double lo = (double)ru->v_th * ru->r_novib;
    int p = 0, ok = 1;
    for (int k = 0; k < 3; ++k) {
        int d = abs(Vp[k] - Vm[k]);
        int hi = d > ru->v_th;
        int low = (double)d < lo;
        if (!(hi || low)) ok = 0;
        p = 2 * p + hi;
    }
    return (ok && p != 0 && ((ru->mask >> (p - 1)) & 1u)) ? 8 + p : 0;
}

/* The decisions (bit 0: not a survivor; bit p: a survivor of pattern p) that
 * moving channels by less than the band can reach: rounding a channel to the
 * other side of a nearby tie, or taking a colour across a nearby gamut edge.
 * Every combination of such moves is tried.  More than one bit set means the
 * candidate is decision-ambiguous. */
static int dec_bit(int d) { return d ? 1 << (d - 8) : 1; }

static int decision_set(const orc_rule* ru, int clip, const double vp[3], const double vm[3],
                        int gp, int gm) {
    const double v[6] = {vp[0], vp[1], vp[2], vm[0], vm[1], vm[2]};
    int nom[6], alt[6];
    int edge_p = 0, edge_m = 0, out_p = 0, out_m = 0;
    for (int k = 0; k < 6; ++k) {
        double a = v[k];
        if (clip) a = a < 0.0 ? 0.0 : (a > 255.0 ? 255.0 : a);
        nom[k] = (int)nearbyint(a);
        alt[k] = nom[k];
        if (near_tie(a)) {
            const int f = (int)floor(a);
            alt[k] = (nom[k] == f) ? f + 1 : f;
        }
        if (!clip) {
            const int e = near_edge(v[k]), o = clearly_out(v[k]);
            if (k < 3) { edge_p |= e; out_p |= o; } else { edge_m |= e; out_m |= o; }
        }
    }
    const int gp_alt = (edge_p && !out_p) ? !gp : gp;
    const int gm_alt = (edge_m && !out_m) ? !gm : gm;
    int set = dec_bit(decide_codes(ru, clip, gp, gm, nom, nom + 3));
    for (int mask = 1; mask < 256; ++mask) {
        int code[6];
        for (int k = 0; k < 6; ++k) code[k] = ((mask >> k) & 1) ? alt[k] : nom[k];
        const int g1 = ((mask >> 6) & 1) ? gp_alt : gp;
        const int g2 = ((mask >> 7) & 1) ? gm_alt : gm;
        set |= dec_bit(decide_codes(ru, clip, g1, g2, code, code + 3));
    }
    return set;
}

/* Evaluate candidate (i, j) of target t under rule ru (ru may be NULL: then
 * only the pair itself and its gamut/boundary state are filled in). */
static void eval_cand(const orc_target* t, const orc_grid* g, const orc_rule* ru,
                      int32_t i, int32_t j, int r_zero, orc_cand* c) {
    double r = r_zero ? 0.0 : (double)(i + 1) * g->dr;
    double th = theta_rad(g, j);
    double Da = r * sin(th);   /* movement along a* */
    double Db = r * cos(th);   /* movement along b* */
    double labp[3] = {t->L, t->a + Da, t->b + Db};
    double labm[3] = {t->L, t->a - Da, t->b - Db};
    lab_to_linear1(t->Minv, t->W, labp, c->linp);
    lab_to_linear1(t->Minv, t->W, labm, c->linm);
    const int clip = ru && (ru->flags & 1u);
    int gp = 1, gm = 1, any_out = 0, edge = 0, tie = 0;
    for (int k = 0; k < 3; ++k) {
        c->vp[k] = 255.0 * orc_encode(c->linp[k]);
        c->vm[k] = 255.0 * orc_encode(c->linm[k]);
        if (!(c->linp[k] >= 0.0 && c->linp[k] <= 1.0)) gp = 0;
        if (!(c->linm[k] >= 0.0 && c->linm[k] <= 1.0)) gm = 0;
        any_out |= clearly_out(c->vp[k]) | clearly_out(c->vm[k]);
        edge |= near_edge(c->vp[k]) | near_edge(c->vm[k]);
    }
    /* 8-bit values, round half to even (the default rounding mode); under the
     * clip reading the code value is first clamped to [0, 255] */
    for (int k = 0; k < 3; ++k) {
        double a = c->vp[k], b = c->vm[k];
        if (clip) {
            a = a < 0.0 ? 0.0 : (a > 255.0 ? 255.0 : a);
            b = b < 0.0 ? 0.0 : (b > 255.0 ? 255.0 : b);
        }
        tie |= near_tie(a) | near_tie(b);
        c->Vp[k] = (uint8_t)((gp || clip) ? nearbyint(a) : 0);
        c->Vm[k] = (uint8_t)((gm || clip) ? nearbyint(b) : 0);
    }
    c->gamut = (uint8_t)(gp | (gm << 1));
    /* A clearly out-of-gamut channel decides "invalid" on its own; under the
     * clip reading only rounding ties can flip a decision. */
    c->boundary = (uint8_t)(clip ? tie : (!any_out && (edge || tie)));
    c->pattern = 0;
    c->valid = 0;
    c->dset = 0;
    memset(c->_pad, 0, sizeof c->_pad);
    if (!ru) return;
    if ((clip || (gp && gm))) {
        double lo = (double)ru->v_th * ru->r_novib;
        int p = 0, ok = 1;
        for (int k = 0; k < 3; ++k) {
            int d = abs((int)c->Vp[k] - (int)c->Vm[k]);
            int hi = d > ru->v_th;
            int low = (double)d < lo;
            if (!(hi || low)) ok = 0;
            p = 2 * p + hi;
        }
        if (ok) c->pattern = (uint8_t)p;
        c->valid = (uint8_t)(ok && p != 0 && ((ru->mask >> (p - 1)) & 1u));
    }
    c->dset = (uint8_t)(c->valid ? 1 << c->pattern : 1);
    if (c->boundary) {
        c->dset = (uint8_t)decision_set(ru, clip, c->vp, c->vm, gp, gm);
        if (c->dset & (c->dset - 1)) c->boundary |= 2;
    }
}

/* Single candidate evaluation, exposed for the tests.  r_zero forces r = 0. */
void orc_eval(const uint8_t rgb[3], const orc_grid* g, const orc_rule* ru,
              int32_t i, int32_t j, int32_t r_zero, orc_cand* out) {
    orc_target t;
    target_init(&t, rgb);
    eval_cand(&t, g, ru, i, j, r_zero, out);
}

/* Every candidate of every colour, in (colour, i, j) order (small grids). */
void orc_eval_all(const uint8_t* rgb, int64_t n, const orc_grid* g, const orc_rule* ru,
                  orc_cand* out, int32_t nthreads) {
    const int64_t per = (int64_t)g->nr * g->ntheta;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t row = 0; row < n * g->nr; ++row) {
        int64_t col = row / g->nr;
        int32_t i = (int32_t)(row % g->nr);
        orc_target t;
        target_init(&t, rgb + 3 * col);
        for (int32_t j = 0; j < g->ntheta; ++j)
            eval_cand(&t, g, ru, i, j, 0, out + col * per + (int64_t)i * g->ntheta + j);
    }
}

/* Selected candidates: (colour index, i, j) triples -> evaluations. */
void orc_eval_list(const uint8_t* rgb, const int64_t* idx, int64_t m, const orc_grid* g,
                   const orc_rule* ru, orc_cand* out, int32_t nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t k = 0; k < m; ++k) {
        orc_target t;
        target_init(&t, rgb + 3 * idx[3 * k]);
        eval_cand(&t, g, ru, (int32_t)idx[3 * k + 1], (int32_t)idx[3 * k + 2], 0, out + k);
    }
}

/* Survivors of all colours in (colour, i, j) order.  Writes up to cap records;
 * returns the total number of survivors.  offsets[n+1] (nullable) receives the
 * per-colour CSR offsets; *nboundary (nullable) the boundary-candidate count
 * over all candidates (survivor or not).  Rows (colour, i) are independent:
 * the first pass counts each row's survivors, a prefix sum places the rows,
 * the second pass writes them (both passes parallel over rows). */
int64_t orc_search(const uint8_t* rgb, int64_t n, const orc_grid* g, const orc_rule* ru,
                   orc_rec* out, int64_t cap, int64_t* offsets, int64_t* nboundary,
                   int32_t nthreads) {
    const int64_t rows = n * g->nr;
    int64_t* cnt = (int64_t*)calloc((size_t)rows + 1, sizeof(int64_t));
    int64_t* bnd = (int64_t*)calloc((size_t)rows + 1, sizeof(int64_t));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t row = 0; row < rows; ++row) {
        orc_target t;
        target_init(&t, rgb + 3 * (row / g->nr));
        const int32_t i = (int32_t)(row % g->nr);
        for (int32_t j = 0; j < g->ntheta; ++j) {
            orc_cand c;
            eval_cand(&t, g, ru, i, j, 0, &c);
            bnd[row] += c.boundary & 1;
            cnt[row] += c.valid;
        }
    }
    int64_t total = 0, nb = 0;
    for (int64_t row = 0; row < rows; ++row) {
        int64_t k = cnt[row];
        cnt[row] = total; /* now the row's start */
        total += k;
        nb += bnd[row];
    }
    cnt[rows] = total;
    if (offsets) {
        for (int64_t col = 0; col < n; ++col) offsets[col] = cnt[col * g->nr];
        offsets[n] = total;
    }
    if (out && cap > 0) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
        for (int64_t row = 0; row < rows; ++row) {
            if (cnt[row] >= cap) continue;
            orc_target t;
            const int64_t col = row / g->nr;
            target_init(&t, rgb + 3 * col);
            const int32_t i = (int32_t)(row % g->nr);
            int64_t pos = cnt[row];
            for (int32_t j = 0; j < g->ntheta && pos < cap; ++j) {
                orc_cand c;
                eval_cand(&t, g, ru, i, j, 0, &c);
                if (!c.valid) continue;
                orc_rec* o = out + pos++;
                o->colour = (uint32_t)col;
                o->i = (uint16_t)i;
                o->j = (uint16_t)j;
                memcpy(o->plus, c.Vp, 3);
                memcpy(o->minus, c.Vm, 3);
                o->pattern = c.pattern;
                o->flags = c.boundary;
            }
        }
    }
    if (nboundary) *nboundary = nb;
    free(cnt);
    free(bnd);
    return total;
}

/* Per-colour summaries and (optionally) the angle-bin table: for each of 36
 * bins of 10 degrees, the largest radius index i+1 with a survivor (0: none).
 * Parallel over colours; every colour is summed by one thread in (i, j) order. */
void orc_reduce(const uint8_t* rgb, int64_t n, const orc_grid* g, const orc_rule* ru,
                orc_summary* summ, uint32_t* table_count, uint8_t* table_bins,
                int32_t nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t col = 0; col < n; ++col) {
        orc_target t;
        target_init(&t, rgb + 3 * col);
        orc_summary s;
        memset(&s, 0, sizeof s);
        s.best_i = 0xFFFF;
        s.best_j = 0xFFFF;
        uint8_t bins[36];
        memset(bins, 0, sizeof bins);
        const int64_t turn = llround(360.0 / g->dtheta_deg);
        for (int32_t i = 0; i < g->nr; ++i) {
            for (int32_t j = 0; j < g->ntheta; ++j) {
                orc_cand c;
                eval_cand(&t, g, ru, i, j, 0, &c);
                s.n_boundary += c.boundary & 1;
                s.n_ambiguous += (c.boundary >> 1) & 1;
                if (c.gamut == 3) s.n_gamut++;
                if (!c.valid) continue;
                s.count++;
                s.per_pattern[c.pattern - 1]++;
                /* larger i wins; for equal i the first (smallest) j is kept */
                if (s.best_i == 0xFFFF || i > s.best_i) {
                    s.best_i = (uint16_t)i;
                    s.best_j = (uint16_t)j;
                    memcpy(s.best_plus, c.Vp, 3);
                    memcpy(s.best_minus, c.Vm, 3);
                    s.best_p = c.pattern;
                }
                /* bin = floor(theta_j / 10 deg) with theta_j = 360 j / N degrees,
                 * N = 360 / dtheta (exact integer form) */
                int bin = (int)(((int64_t)j * 36) / turn);
                int ridx = i + 1 > 255 ? 255 : i + 1;
                if (ridx > bins[bin]) bins[bin] = (uint8_t)ridx;
            }
        }
        if (summ) summ[col] = s;
        if (table_count) table_count[col] = s.count;
        if (table_bins) memcpy(table_bins + 36 * col, bins, 36);
    }
}

/* What an evaluation that agrees with this one outside the band may report
 * for each colour: every output of the reduce as the range it can take when
 * each decision-ambiguous candidate may end either way (any decision in its
 * dset).  A candidate that must survive (dset = {p}) counts in both ends; one
 * that may survive counts in the upper end only.  Keys order the survivors
 * as the maximum-amplitude rule does: key = i << 16 | (0xFFFF - j), 0 = none. */
typedef struct {
    uint32_t count_lo, count_hi;
    uint32_t pat_lo[7], pat_hi[7];   /* survivors of pattern p at p - 1          */
    uint32_t key_lo, key_hi;         /* best key over must / may survivors        */
    uint32_t pkey_lo[7], pkey_hi[7]; /* best key of each pattern                  */
    uint32_t n_gamut, n_boundary, n_ambiguous;
    uint8_t best_band;               /* the must-survivor of key_lo is in the band */
    uint8_t pbest_band[7];           /* (its codes may differ by a rounding)       */
    uint32_t _pad;
} orc_bounds;

static uint32_t cand_key(int32_t i, int32_t j) { return ((uint32_t)i << 16) | (0xFFFFu - (uint32_t)j); }

/* Per colour: bounds (nullable); bins_lo / bins_hi [n][36] (nullable) the
 * per-bin largest i + 1 over must / may survivors (capped at 255);
 * rays_lo / rays_hi [n][ntheta] (nullable) the same per ray, uncapped. */
void orc_reduce_bounds(const uint8_t* rgb, int64_t n, const orc_grid* g, const orc_rule* ru,
                       orc_bounds* bounds, uint8_t* bins_lo, uint8_t* bins_hi, uint16_t* rays_lo,
                       uint16_t* rays_hi, int32_t nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t col = 0; col < n; ++col) {
        orc_target t;
        target_init(&t, rgb + 3 * col);
        orc_bounds b;
        memset(&b, 0, sizeof b);
        uint8_t blo[36], bhi[36];
        memset(blo, 0, sizeof blo);
        memset(bhi, 0, sizeof bhi);
        uint16_t* rlo = rays_lo ? rays_lo + col * g->ntheta : NULL;
        uint16_t* rhi = rays_hi ? rays_hi + col * g->ntheta : NULL;
        if (rlo) memset(rlo, 0, sizeof(uint16_t) * (size_t)g->ntheta);
        if (rhi) memset(rhi, 0, sizeof(uint16_t) * (size_t)g->ntheta);
        const int64_t turn = llround(360.0 / g->dtheta_deg);
        for (int32_t i = 0; i < g->nr; ++i) {
            for (int32_t j = 0; j < g->ntheta; ++j) {
                orc_cand c;
                eval_cand(&t, g, ru, i, j, 0, &c);
                b.n_boundary += c.boundary & 1;
                b.n_ambiguous += (c.boundary >> 1) & 1;
                if (c.gamut == 3) b.n_gamut++;
                const int may = (c.dset & 0xFE) != 0, must = !(c.dset & 1);
                if (!may) continue;
                const uint32_t key = cand_key(i, j);
                const int bin = (int)(((int64_t)j * 36) / turn);
                const int ridx = i + 1 > 255 ? 255 : i + 1;
                b.count_hi++;
                if (ridx > bhi[bin]) bhi[bin] = (uint8_t)ridx;
                if (rhi && i + 1 > rhi[j]) rhi[j] = (uint16_t)(i + 1);
                if (key > b.key_hi) b.key_hi = key;
                if (must) {
                    b.count_lo++;
                    if (ridx > blo[bin]) blo[bin] = (uint8_t)ridx;
                    if (rlo && i + 1 > rlo[j]) rlo[j] = (uint16_t)(i + 1);
                    if (key > b.key_lo) {
                        b.key_lo = key;
                        b.best_band = c.boundary & 1;
                    }
                }
                for (int p = 1; p <= 7; ++p) {
                    if (!((c.dset >> p) & 1)) continue;
                    b.pat_hi[p - 1]++;
                    if (key > b.pkey_hi[p - 1]) b.pkey_hi[p - 1] = key;
                    if (c.dset == (1 << p)) {
                        b.pat_lo[p - 1]++;
                        if (key > b.pkey_lo[p - 1]) {
                            b.pkey_lo[p - 1] = key;
                            b.pbest_band[p - 1] = c.boundary & 1;
                        }
                    }
                }
            }
        }
        if (bounds) bounds[col] = b;
        if (bins_lo) memcpy(bins_lo + 36 * col, blo, 36);
        if (bins_hi) memcpy(bins_hi + 36 * col, bhi, 36);
    }
}

/* Largest radius index (i+1) at which both colours of some pair are in gamut,
 * per colour (0 if none): shows whether a grid's radius range is exhaustive. */
void orc_max_gamut_radius(const uint8_t* rgb, int64_t n, const orc_grid* g,
                          int32_t* out, int32_t nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t col = 0; col < n; ++col) {
        orc_target t;
        target_init(&t, rgb + 3 * col);
        int32_t best = 0;
        for (int32_t i = g->nr - 1; i >= 0 && best == 0; --i)
            for (int32_t j = 0; j < g->ntheta; ++j) {
                orc_cand c;
                eval_cand(&t, g, NULL, i, j, 0, &c);
                if (c.gamut == 3) { best = i + 1; break; }
            }
        out[col] = best;
    }
}

int32_t orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
