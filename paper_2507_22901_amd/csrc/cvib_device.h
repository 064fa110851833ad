// Device-side building blocks of the colour-vibration pair search (gfx950).
//
// Arithmetic split (chosen for MI355X):
//   * geometry in FP64 -- the displaced f(X/Xn), f(Z/Zn) of both colours, the
//     inverse L* companding (cube / linear branch) and the 3x3 XYZ -> linear
//     RGB product.  The dark end of the sRGB curve magnifies an error in f by
//     roughly 1.6e4 codes per unit, so FP32's 24-bit mantissa alone would put
//     ~1e-3-code errors on dark channels; gfx950 issues FP64 FMA/ADD/MUL at the
//     same per-lane rate as non-packed FP32, so this costs registers, not
//     issue slots.
//   * transfer in FP32 -- the sRGB encode (linear segment or
//     1.055 * l^(1/2.4) - 0.055) on the hardware log2/exp2 units, the x255
//     scale and round-half-to-even; error <= ~3e-5 codes against FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cvib {

// Per-target constants (Section 2: the target split into L*, a*, b*).  Holding
// L* fixed fixes f(Y) and Y, so the Y column of the XYZ -> RGB product is a
// per-colour constant B_k.
struct alignas(16) ColorConst {
    double fx0;    // f(X/Xn) of the target = (L+16)/116 + a/500
    double fz0;    // f(Z/Zn) of the target = (L+16)/116 - b/200
    double B[3];   // Minv[k][1] * Y of the target
    float L, a, b; // target L*a*b* (FP32 copy, reporting only)
    uint32_t _pad;
};
static_assert(sizeof(ColorConst) == 64, "ColorConst layout");

// Per-launch constants: the X and Z columns of the XYZ -> linear RGB matrix
// with the white point folded in.
struct Geom {
    double A[3]; // Minv[k][0] * Xn
    double C[3]; // Minv[k][2] * Zn
};

constexpr double kDelta = 6.0 / 29.0;
constexpr double kLinSlope = 3.0 * kDelta * kDelta;            // 3 delta^2
constexpr double kLinOffset = -3.0 * kDelta * kDelta * 4.0 / 29.0;

// Inverse of the L* companding function f (CIE 1976).
__device__ __forceinline__ double finv(double u) {
    double cube = u * u * u;
    double lin = __builtin_fma(kLinSlope, u, kLinOffset);
    return u > kDelta ? cube : lin;
}

constexpr float kEncodeKnee = 0.0031308f;  // linear segment at or below

// Power segment of the sRGB encode in code units: 255 (1.055 l^(1/2.4) - 0.055).
__device__ __forceinline__ float encode255_pow(float l) {
    float lg = __builtin_amdgcn_logf(l);                 // log2 (v_log_f32)
    float p = __builtin_amdgcn_exp2f(lg * (1.0f / 2.4f)); // 2^(log2(l)/2.4)
    return __builtin_fmaf(255.0f * 1.055f, p, -255.0f * 0.055f);
}

// sRGB encode of an FP32 linear value, in 0..255 code units (unrounded).
// Outside [0,1] the two branches extend the curve monotonically.
__device__ __forceinline__ float encode255(float l) {
    float g = encode255_pow(l);
    float s = l * (255.0f * 12.92f);
    return l <= kEncodeKnee ? s : g;
}

// One colour of a candidate pair: displaced (fx, fz) -> linear RGB (FP64).
__device__ __forceinline__ void lab_f_to_linear(const Geom& g, const double B[3], double fx,
                                                double fz, double lin[3]) {
    double gx = finv(fx);
    double gz = finv(fz);
#pragma unroll
    for (int k = 0; k < 3; ++k) lin[k] = __builtin_fma(g.A[k], gx, __builtin_fma(g.C[k], gz, B[k]));
}

// Linear RGB of both colours of the pair at displacement (dx, dz) =
// (r sin / 500, r cos / 200): (L, a +- D_a, b +- D_b) is (fx0 +- dx, fz0 -+ dz)
// in f-space (Section 2).  Rounded to FP32 once the FP64 product is done.
__device__ __forceinline__ void pair_linear(const ColorConst& cc, const Geom& g, double dx,
                                           double dz, float fp[3], float fm[3]) {
    double lp[3], lm[3];
    lab_f_to_linear(g, cc.B, cc.fx0 + dx, cc.fz0 - dz, lp);
    lab_f_to_linear(g, cc.B, cc.fx0 - dx, cc.fz0 + dz, lm);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        fp[k] = (float)lp[k];
        fm[k] = (float)lm[k];
    }
}

// pair_linear for a whole wave, with the cube branch of finv taken without a
// select when no lane of the wave needs the linear branch (same results).
// cube_known: the caller has shown that every f of the call exceeds delta.
__device__ __forceinline__ void pair_linear_w(const ColorConst& cc, const Geom& g, double dx,
                                             double dz, float fp[3], float fm[3],
                                             bool cube_known = false) {
    const double xp = cc.fx0 + dx, zp = cc.fz0 - dz, xm = cc.fx0 - dx, zm = cc.fz0 + dz;
    double gxp, gzp, gxm, gzm;
    if (cube_known || __ballot(fmin(fmin(xp, zp), fmin(xm, zm)) <= kDelta) == 0ull) {
        gxp = xp * xp * xp;
        gzp = zp * zp * zp;
        gxm = xm * xm * xm;
        gzm = zm * zm * zm;
    } else {
        gxp = finv(xp);
        gzp = finv(zp);
        gxm = finv(xm);
        gzm = finv(zm);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        fp[k] = (float)__builtin_fma(g.A[k], gxp, __builtin_fma(g.C[k], gzp, cc.B[k]));
        fm[k] = (float)__builtin_fma(g.A[k], gxm, __builtin_fma(g.C[k], gzm, cc.B[k]));
    }
}

// Whether every f = f0 +- r sin / 500 (X) and f0 -+ r cos / 200 (Z) of radii
// up to (imax + 1) dr lies above delta, so that finv takes its cube branch:
// |sin|, |cos| <= 1, with a margin far above the rounding of the products.
__device__ __forceinline__ bool cube_branch_only(const ColorConst& cc, int32_t imax, double ra,
                                                 double rb) {
    const double r = (double)(imax + 1);
    return cc.fx0 - r * ra > kDelta + 1e-9 && cc.fz0 - r * rb > kDelta + 1e-9;
}

// All three linear channels in [0, 1]: the IEEE bit patterns of non-negative
// floats order like the values, and every negative float (sign bit set)
// compares above 1.0f's pattern as an unsigned integer.
__device__ __forceinline__ bool in_unit_cube(const float l[3]) {
    const uint32_t a = __float_as_uint(l[0]), b = __float_as_uint(l[1]), c = __float_as_uint(l[2]);
    return max(max(a, b), c) <= 0x3F800000u;
}

// 8-bit code of a linear value: sRGB encode, clamp to [0, 255], round half to
// even.  For values inside the gamut the clamp changes nothing; under the clip
// reading it is the reading itself.
__device__ __forceinline__ float code8(float l) {
    return __builtin_rintf(__builtin_amdgcn_fmed3f(encode255(l), 0.0f, 255.0f));
}

// 8-bit codes of both colours of a wave's candidates; lanes with need = false
// get unspecified codes.  Without the clip reading every needed lane is in
// gamut, so its codes lie in [0, 255] and the clamp is idle; when no needed
// lane has a channel on the linear segment either, the power segment alone
// gives the same codes as code8.
__device__ __forceinline__ void codes_w(const float fp[3], const float fm[3], bool need, bool clip,
                                        float Vp[3], float Vm[3]) {
    const float lo = fminf(fminf(fminf(fp[0], fp[1]), fp[2]), fminf(fminf(fm[0], fm[1]), fm[2]));
    if (!clip && __ballot(need && lo <= kEncodeKnee) == 0ull) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Vp[k] = __builtin_rintf(encode255_pow(fp[k]));
            Vm[k] = __builtin_rintf(encode255_pow(fm[k]));
        }
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Vp[k] = code8(fp[k]);
            Vm[k] = code8(fm[k]);
        }
    }
}

// Integer form of a rule (Section 3): high = d > v_th, low = d <= lo_max where
// lo_max = ceil(v_th * r_novib) - 1 is the largest integer change below
// v_th * r_novib.
struct RuleDev {
    float v_th;
    float lo_max;
    uint32_t mask;  // bit (p-1) accepts pattern p
    uint32_t clip;  // CV_RULE_CLIP reading
};

// Pattern p = 4 hi_R + 2 hi_G + hi_B when every channel is high or low, else 0.
__device__ __forceinline__ uint32_t pattern_of(const float Vp[3], const float Vm[3],
                                               const RuleDev& r) {
    uint32_t p = 0;
    bool every = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float d = fabsf(Vp[k] - Vm[k]);
        const bool hi = d > r.v_th;
        every = every && (hi || d <= r.lo_max);
        p = 2u * p + (hi ? 1u : 0u);
    }
    return every ? p : 0u;
}

__device__ __forceinline__ bool accepts(const RuleDev& r, uint32_t p) {
    return p != 0u && ((r.mask >> (p - 1u)) & 1u);
}

// Bytes of a pair record's last 8 bytes: lo = R+ | G+<<8 | B+<<16 | R-<<24,
// hi = G- | B-<<8 | p<<16 | flags<<24 (codes are already integral in [0,255]).
__device__ __forceinline__ void pack_pair(const float Vp[3], const float Vm[3], uint32_t p,
                                          uint32_t flags, uint32_t& lo, uint32_t& hi) {
    lo = __builtin_amdgcn_cvt_pk_u8_f32(Vp[0], 0, 0u);
    lo = __builtin_amdgcn_cvt_pk_u8_f32(Vp[1], 1, lo);
    lo = __builtin_amdgcn_cvt_pk_u8_f32(Vp[2], 2, lo);
    lo = __builtin_amdgcn_cvt_pk_u8_f32(Vm[0], 3, lo);
    hi = (p << 16) | (flags << 24);
    hi = __builtin_amdgcn_cvt_pk_u8_f32(Vm[1], 0, hi);
    hi = __builtin_amdgcn_cvt_pk_u8_f32(Vm[2], 1, hi);
}

// The same pair seen from the opposite ray (theta + 180 deg): + and - swap.
// Gamut bits 0 and 1 of the flags swap as well.
__device__ __forceinline__ void mirror_pair(uint32_t lo, uint32_t hi, uint32_t& mlo,
                                            uint32_t& mhi) {
    mlo = __builtin_amdgcn_perm(hi, lo, 0x00050403u); // R-, G-, B-, R+
    const uint32_t fl = hi >> 24;
    const uint32_t mfl = (fl & 4u) | ((fl & 1u) << 1) | ((fl >> 1) & 1u);
    mhi = (__builtin_amdgcn_perm(hi, lo, 0x07060201u) & 0x00FFFFFFu) | (mfl << 24); // G+, B+, p
}

// Full evaluation of one candidate (used outside the hot loop).
struct PairEval {
    float Vp[3], Vm[3];
    bool gp, gm;
};

__device__ __forceinline__ void eval_pair(const ColorConst& cc, const Geom& g, double dx,
                                          double dz, PairEval& e) {
    float fp[3], fm[3];
    pair_linear(cc, g, dx, dz, fp, fm);
    e.gp = in_unit_cube(fp);
    e.gm = in_unit_cube(fm);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        e.Vp[k] = code8(fp[k]);
        e.Vm[k] = code8(fm[k]);
    }
}

} // namespace cvib
