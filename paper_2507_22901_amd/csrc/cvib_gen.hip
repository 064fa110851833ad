// Synthetic 4K frames generated on the device (the batched workloads' input):
// a counter-based recipe in integer arithmetic only, so that any
// implementation of the same definition writes the same bytes.
//
// Random words come from Philox4x64-10 (Salmon, Moraes, Dror and Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4 x 64-bit counter
// and a 2 x 64-bit key, ten rounds of two 64 x 64 -> 128-bit products each,
// the key bumped by the Weyl constants between rounds.  Frame f uses key
// (seed_f, 0) and three counter families:
//   (0, 0, 0, 0)  frame parameters: per channel c, from byte c of words 0, 1, 2:
//                 base g0 = 64 + b % 129, x slope gx = b % 129 - 64,
//                 y slope gy = b % 129 - 64;
//   (1, s, 0, 0)  site s < sites: x = word0 % width, y = word1 % height,
//                 offset v_c = (byte c of word2) % 97 - 48;
//   (2, y, x, 0)  pixel (x, y): noise n_c = (sum of bytes 4c .. 4c + 3 of
//                 words 0, 1 as 16 little-endian bytes - 510) * noise / 128.
// Pixel channel c = clamp(g0 + gx x / width + gy y / height + v_c(cell) + n_c,
// 0, 255): smooth gradients, the piecewise-constant regions of the nearest
// site (squared distance; ties to the lowest site) and a rounded Irwin-Hall
// noise.  Every division truncates toward zero.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "cvib_internal.h"

namespace cvib {
namespace {

// Philox4x64 round constants (SC'11): the multipliers and the Weyl sequence
// increments of the key.
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull, kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull, kPhiloxW1 = 0xBB67AE8584CAA73Bull;
constexpr int kGenBlock = 256;
constexpr int kGenMaxSites = 256;

struct Words {
    uint64_t w[4];
};

__device__ __forceinline__ Words philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                            uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
        const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return Words{{c0, c1, c2, c3}};
}

__device__ __forceinline__ int32_t byte_of(uint64_t w, int b) { return (int32_t)((w >> (8 * b)) & 255u); }

// One frame: the sites and parameters in LDS (every block derives them), then
// a grid-stride loop over the pixels, one thread per pixel.
__global__ __launch_bounds__(kGenBlock) void k_gen_frame(uint64_t seed, int32_t H, int32_t W, int32_t S,
                                                         int32_t noise, uint8_t* __restrict__ out) {
    __shared__ int32_t s_sx[kGenMaxSites], s_sy[kGenMaxSites], s_v[kGenMaxSites * 3];
    __shared__ int32_t s_par[9];
    for (int s = threadIdx.x; s < S; s += kGenBlock) {
        const Words r = philox4x64(1, (uint64_t)s, 0, 0, seed, 0);
        s_sx[s] = (int32_t)(r.w[0] % (uint64_t)W);
        s_sy[s] = (int32_t)(r.w[1] % (uint64_t)H);
#pragma unroll
        for (int c = 0; c < 3; ++c) s_v[s * 3 + c] = byte_of(r.w[2], c) % 97 - 48;
    }
    if (threadIdx.x == 0) {
        const Words r = philox4x64(0, 0, 0, 0, seed, 0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            s_par[c] = 64 + byte_of(r.w[0], c) % 129;
            s_par[3 + c] = byte_of(r.w[1], c) % 129 - 64;
            s_par[6 + c] = byte_of(r.w[2], c) % 129 - 64;
        }
    }
    __syncthreads();
    const int64_t npix = (int64_t)H * W;
    for (int64_t p = (int64_t)blockIdx.x * kGenBlock + threadIdx.x; p < npix; p += (int64_t)gridDim.x * kGenBlock) {
        const int32_t y = (int32_t)(p / W), x = (int32_t)(p - (int64_t)y * W);
        int32_t best = 0x7FFFFFFF, cell = 0;
        for (int s = 0; s < S; ++s) {
            const int32_t dx = x - s_sx[s], dy = y - s_sy[s];
            const int32_t d2 = dx * dx + dy * dy;
            if (d2 < best) {
                best = d2;
                cell = s;
            }
        }
        const Words r = philox4x64(2, (uint64_t)y, (uint64_t)x, 0, seed, 0);
        uint8_t* o = out + p * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const uint64_t wq = c < 2 ? r.w[0] : r.w[1];
            const int b0 = c == 1 ? 4 : 0;
            const int32_t sum = byte_of(wq, b0) + byte_of(wq, b0 + 1) + byte_of(wq, b0 + 2) + byte_of(wq, b0 + 3);
            const int32_t nz = (sum - 510) * noise / 128;
            const int32_t v = s_par[c] + s_par[3 + c] * x / W + s_par[6 + c] * y / H + s_v[cell * 3 + c] + nz;
            o[c] = (uint8_t)std::min(255, std::max(0, v));
        }
    }
}

}  // namespace
}  // namespace cvib

int cv_frames_generate(cv_context* ctx, const uint64_t* seeds, int64_t n, int32_t height, int32_t width,
                       int32_t sites, int32_t noise, uint8_t* out, void* stream) {
    CV_GUARD_BEGIN
    using namespace cvib;
    if (!ctx) return fail(CV_EINVAL, "ctx is NULL");
    if (n < 0) return fail(CV_EINVAL, "n < 0");
    if (n > 0 && (!seeds || !out)) return fail(CV_EINVAL, "null array");
    if (height < 1 || width < 1 || height > 16384 || width > 16384)
        return fail(CV_EINVAL, "frame size out of [1, 16384]");
    if (sites < 1 || sites > kGenMaxSites) return fail(CV_EINVAL, "sites out of [1, 256]");
    if (noise < 0 || noise > 255) return fail(CV_EINVAL, "noise out of [0, 255]");
    DeviceGuard dg(ctx->device);
    const int64_t npix = (int64_t)height * width;
    const unsigned blocks = (unsigned)std::min<int64_t>((npix + kGenBlock - 1) / kGenBlock, 8192);
    for (int64_t f = 0; f < n; ++f) {
        hipLaunchKernelGGL(k_gen_frame, dim3(blocks), dim3(kGenBlock), 0, (hipStream_t)stream, seeds[f], height,
                           width, sites, noise, out + f * npix * 3);
        CV_HIP(hipGetLastError());
    }
    return CV_OK;
    CV_GUARD_END
}
