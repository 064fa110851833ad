/*
 * CPU twin of the library's synthetic frame generator (cv_frames_generate).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of this folder: it shares no code
 * with the HIP library and exists to check, byte for byte, that the device
 * generator follows the definition below.  The random words are Philox4x64
 * with 10 rounds (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11), written here from that paper's definition: per
 * round, the products of the multipliers with counter words 0 and 2 (128 bits
 * each), the new words (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1,
 * lo(M0 x0)), and the key bumped by the Weyl increments.  The test suite pins
 * it to numpy's Philox bit generator (the same 4x64-10 function).
 *
 * The frame recipe (integer arithmetic only, every division truncating toward
 * zero), key (seed, 0):
 *   words(0,0,0,0): channel c: g0 = 64 + b0 % 129, gx = b1 % 129 - 64,
 *                   gy = b2 % 129 - 64, bk = byte c of word k;
 *   words(1,s,0,0): site s: sx = word0 % width, sy = word1 % height,
 *                   v_c = (byte c of word2) % 97 - 48;
 *   words(2,y,x,0): pixel noise n_c = (bytes 4c..4c+3 of words 0,1 taken as
 *                   16 little-endian bytes, summed, - 510) * noise / 128;
 *   value_c = clamp(g0 + gx*x/width + gy*y/height + v_c[nearest] + n_c, 0, 255),
 *   nearest = the site of least (x-sx)^2 + (y-sy)^2, the lowest index on ties.
 */
#include <stdint.h>

static const uint64_t PH_M0 = 0xD2E7470EE14C6C93ull, PH_M1 = 0xCA5A826395121157ull;
static const uint64_t PH_W0 = 0x9E3779B97F4A7C15ull, PH_W1 = 0xBB67AE8584CAA73Bull;

/* out = Philox4x64-10(ctr, key). */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        const unsigned __int128 p0 = (unsigned __int128)PH_M0 * x0;
        const unsigned __int128 p1 = (unsigned __int128)PH_M1 * x2;
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
        k0 += PH_W0;
        k1 += PH_W1;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

static int32_t byte_at(uint64_t w, int b) { return (int32_t)((w >> (8 * b)) & 255u); }

static void words(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t seed, uint64_t out[4]) {
    const uint64_t ctr[4] = {c0, c1, c2, 0};
    const uint64_t key[2] = {seed, 0};
    orc_philox4x64(ctr, key, out);
}

/* One frame, out = uint8 [height][width][3].  Returns 0, or -1 on bad sizes. */
int orc_gen_frame(uint64_t seed, int32_t height, int32_t width, int32_t sites, int32_t noise, uint8_t* out) {
    if (height < 1 || width < 1 || sites < 1 || sites > 256 || noise < 0) return -1;
    int32_t g0[3], gx[3], gy[3];
    int32_t sx[256], sy[256], v[256][3];
    uint64_t r[4];
    words(0, 0, 0, seed, r);
    for (int c = 0; c < 3; ++c) {
        g0[c] = 64 + byte_at(r[0], c) % 129;
        gx[c] = byte_at(r[1], c) % 129 - 64;
        gy[c] = byte_at(r[2], c) % 129 - 64;
    }
    for (int s = 0; s < sites; ++s) {
        words(1, (uint64_t)s, 0, seed, r);
        sx[s] = (int32_t)(r[0] % (uint64_t)width);
        sy[s] = (int32_t)(r[1] % (uint64_t)height);
        for (int c = 0; c < 3; ++c) v[s][c] = byte_at(r[2], c) % 97 - 48;
    }
    for (int32_t y = 0; y < height; ++y) {
        for (int32_t x = 0; x < width; ++x) {
            int64_t best = -1;
            int nearest = 0;
            for (int s = 0; s < sites; ++s) {
                const int64_t dx = x - sx[s], dy = y - sy[s];
                const int64_t d2 = dx * dx + dy * dy;
                if (best < 0 || d2 < best) {
                    best = d2;
                    nearest = s;
                }
            }
            words(2, (uint64_t)y, (uint64_t)x, seed, r);
            uint8_t bytes[16];
            for (int k = 0; k < 16; ++k) bytes[k] = (uint8_t)byte_at(r[k / 8], k % 8);
            uint8_t* px = out + ((int64_t)y * width + x) * 3;
            for (int c = 0; c < 3; ++c) {
                const int32_t sum = bytes[4 * c] + bytes[4 * c + 1] + bytes[4 * c + 2] + bytes[4 * c + 3];
                const int32_t n = (sum - 510) * noise / 128;
                int32_t val = g0[c] + gx[c] * x / width + gy[c] * y / height + v[nearest][c] + n;
                if (val < 0) val = 0;
                if (val > 255) val = 255;
                px[c] = (uint8_t)val;
            }
        }
    }
    return 0;
}
