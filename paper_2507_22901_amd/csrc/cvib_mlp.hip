// Surrogate network: a multilayer perceptron (ReLU hidden layers, linear
// output) that maps a target colour to the largest valid radius of each
// angle bin plus a feasibility logit.  It is trained and evaluated by the
// kernels in this file:
//   - the input layer (3 inputs) is a per-element FP32 kernel on the vector
//     ALUs: a 3-long reduction has nothing to give to a matrix core;
//   - every other layer is a BF16 matrix product on the matrix cores
//     (v_mfma_f32_16x16x32_bf16, FP32 accumulation) with the bias, ReLU or
//     ReLU-derivative mask fused into the epilogue;
//   - weight gradients reduce over the batch with a fixed split and a
//     fixed-order sum of the partials, so training is bitwise repeatable;
//   - FP32 master weights with Adam; BF16 copies feed the matrix cores.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "cvib_internal.h"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace cvib {
namespace {

constexpr int kMaxLayers = 8;
constexpr int kMaxIn = 4;          // input width handled by the vector-ALU layer
constexpr int kMaxHidden = 1024;
constexpr int kMaxOut = 256;
constexpr int32_t kSplitRows = 512;   // batch rows per split of a weight-gradient reduction
constexpr int64_t kInferChunk = 1 << 20;  // rows per forward chunk when nothing is kept

int32_t pad32(int32_t d) { return (d + 31) / 32 * 32; }

// ---------------------------------------------------------------------------
// Matrix-core product.  C[M][N] = sum_k A(m, k) B(n, k) over one split of k.
// A_KC: A is stored [m][k] (k contiguous), else [k][m].  B_KC: B is stored
// [n][k], else [k][n].  Tiles of 64 x 64 outputs, 32-deep k steps, 4 waves of
// 32 x 32 (2 x 2 MFMA tiles of 16 x 16).  LDS keeps both tiles k-contiguous
// (row pitch 40 elements = 80 bytes) so that each lane's fragment (8
// consecutive k) is one 16-byte LDS read.
//
// MFMA 16x16x32 BF16 operand layout (lane l = 0..63): A row l % 16, k
// 8 (l / 16) .. + 7; B column l % 16, same k; result rows 4 (l / 16) .. + 3,
// column l % 16.
enum { EPI_RELU_BF16 = 0, EPI_BIAS_F32 = 1, EPI_MASK_BF16 = 2, EPI_PARTIAL_F32 = 3, EPI_SINE_BF16 = 4 };

struct GemmArgs {
    const bf16* A;
    int64_t lda;
    const bf16* B;
    int64_t ldb;
    int32_t M, N, K, kchunk;   // kchunk: reduction length per blockIdx.z (multiple of 32)
    const float* bias;         // [N]
    bf16* cb;                  // bf16 result
    float* cf;                 // fp32 result / partials
    int64_t ldc;
    int64_t zstride;           // partials: elements between splits
    const bf16* mask;          // ReLU-derivative mask source (post-ReLU activations)
    int64_t ldm;
    int32_t nstore;            // result columns written (<= N)
    // EPI_SINE_BF16: the derivative omega0 cos(omega0 z) of a sinusoidal first
    // layer, stored by the forward pass [M][ldd] (dsin), or else recomputed
    // from z = b0 + W0 x and the FP32 inputs x [M][d0]
    const float* dsin;
    int64_t ldd;
    const float* x0;
    const float* w0;
    const float* b0;
    int32_t d0;
    float omega0;
    // bf16 epilogues: the result also transposed, [N][ldct] (nullable), for
    // the weight-gradient products, whose operands must be k-contiguous
    bf16* cbt;
    int64_t ldct;
    // EPI_PARTIAL_F32 with A k-contiguous: blocks of the first column tile
    // also write the row sums of A over their k range (bias gradients),
    // [blockIdx.z][M] (nullable)
    float* bpart;
};

constexpr int kDepth = 32;

// Network input of an 8-bit code: v * fl(1/255) - 1/2, the product and the
// difference each rounded to FP32 (never contracted into one FMA), the same
// in every kernel that converts colours.
__device__ __forceinline__ float rgb_input(uint32_t v) {
#pragma clang fp contract(off)
    return (float)v * (1.0f / 255.0f) - 0.5f;
}

// Sine and cosine of x (radians) on the hardware's sine and cosine units,
// whose argument is in turns: x / 2 pi reduced to [-1/2, 1/2] by taking off
// the nearest integer.  For |x| <= 2^10 the error stays below 1e-5 (the
// reduction's FP32 rounding, about 2^-24 |x| / 2 pi turns, and the units'
// own), far below the BF16 rounding that the activation gets next; a full
// range reduction would cost the input layer several times its arithmetic.
__device__ __forceinline__ float to_turns(float x) {
    const float t = x * 0.159154943f;  // 1 / 2 pi
    return t - rintf(t);
}
__device__ __forceinline__ float sin_hw(float x) { return __builtin_amdgcn_sinf(to_turns(x)); }
__device__ __forceinline__ float cos_hw(float x) { return __builtin_amdgcn_cosf(to_turns(x)); }

// Activation of the first hidden layer: ReLU, or sin(omega0 z) when omega0 > 0
// (a sinusoidal layer, which lets the network follow finer detail of its
// three inputs).  Every later hidden layer is ReLU.  Every kernel takes the
// activation and its derivative omega0 cos(omega0 z) from these functions.
__device__ __forceinline__ float first_act(float z, float omega0) {
    return omega0 > 0.0f ? sin_hw(omega0 * z) : fmaxf(z, 0.0f);
}
__device__ __forceinline__ float first_deriv_sine(float z, float omega0) { return omega0 * cos_hw(omega0 * z); }

// A tile of R rows x KD k of one operand, global -> registers: PER 8-element
// chunks per thread (R * KD / 8 / 256 of them).  KC: stored [row][k] (a chunk
// that runs past ke is loaded element by element, so k need not be a multiple
// of 8); else [k][row].
template <bool KC, int R, int KD>
struct TileLoad {
    static constexpr int PER = R * KD / 8 / 256;
    static constexpr int CPR = KD / 8;  // chunks per row (KC)
    bf16x8 v[PER];
    __device__ __forceinline__ void load(const bf16* __restrict__ P, int64_t ld, int32_t r0, int32_t rows,
                                         int32_t k0, int32_t ke, int tid) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int u = tid + 256 * q;
            v[q] = bf16x8{};
            if constexpr (KC) {
                const int r = u / CPR, c = (u % CPR) * 8;
                if (r0 + r < rows && k0 + c < ke) {
                    const bf16* src = P + (int64_t)(r0 + r) * ld + k0 + c;
                    if (k0 + c + 8 <= ke) {
                        v[q] = *reinterpret_cast<const bf16x8*>(src);
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            if (k0 + c + e < ke) v[q][e] = src[e];
                    }
                }
            } else {
                const int kr = u / (R / 8), c = (u % (R / 8)) * 8;
                if (k0 + kr < ke && r0 + c < rows)
                    v[q] = *reinterpret_cast<const bf16x8*>(P + (int64_t)(k0 + kr) * ld + r0 + c);
            }
        }
    }
    // registers -> LDS tile [row][k] (k contiguous, pitch KD + 8)
    __device__ __forceinline__ void store(bf16* s, int tid) const {
        constexpr int pitch = KD + 8;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int u = tid + 256 * q;
            if constexpr (KC) {
                const int r = u / CPR, c = (u % CPR) * 8;
                *reinterpret_cast<bf16x8*>(s + r * pitch + c) = v[q];
            } else {
                const int kr = u / (R / 8), c = (u % (R / 8)) * 8;
#pragma unroll
                for (int e = 0; e < 8; ++e) s[(c + e) * pitch + kr] = v[q][e];
            }
        }
    }
};

// BM x BN outputs per block of 4 waves (2 x 2), each wave (BM/2) x (BN/2) as
// MFMA tiles of 16 x 16; KD-deep k steps (one barrier pair each, KD / 32 MFMA
// passes), the next step of both operands fetched into registers while the
// current one is multiplied from LDS.  The k order (32-deep slices in
// ascending order, each one MFMA) does not depend on KD.
// Tile (bx, by) of split bz.
template <bool A_KC, bool B_KC, int EPI, int BM, int BN, int KD>
__device__ __forceinline__ void gemm_tile(const GemmArgs& a, int32_t bx, int32_t by, int32_t bz) {
    constexpr int TM = BM / 32, TN = BN / 32;  // MFMA tiles per wave
    constexpr int pitch = KD + 8;
    __shared__ __attribute__((aligned(16))) bf16 sA[BM * pitch];
    __shared__ __attribute__((aligned(16))) bf16 sB[BN * pitch];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int32_t m0 = bx * BM, n0 = by * BN;
    const int32_t kb = bz * a.kchunk;
    const int32_t ke = min(a.K, kb + a.kchunk);
    // bias-gradient row sums of A (first column tile only): thread -> row
    // tid / 4 (BM = 64), a quarter of each k step
    constexpr bool ROWSUM = EPI == EPI_PARTIAL_F32 && A_KC && BM == 64;
    const bool rowsum = ROWSUM && a.bpart != nullptr && by == 0;
    float rsum = 0.0f;
    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    TileLoad<A_KC, BM, KD> la;
    TileLoad<B_KC, BN, KD> lb;
    la.load(a.A, a.lda, m0, a.M, kb, ke, tid);
    lb.load(a.B, a.ldb, n0, a.N, kb, ke, tid);
    for (int32_t k0 = kb; k0 < ke; k0 += KD) {
        la.store(sA, tid);
        lb.store(sB, tid);
        __syncthreads();
        if (k0 + KD < ke) {  // next step in flight during the products
            la.load(a.A, a.lda, m0, a.M, k0 + KD, ke, tid);
            lb.load(a.B, a.ldb, n0, a.N, k0 + KD, ke, tid);
        }
        if constexpr (ROWSUM) {
            if (rowsum) {
                const bf16* row = sA + (tid >> 2) * pitch + (tid & 3) * (KD / 4);
#pragma unroll
                for (int e = 0; e < KD / 4; ++e) rsum += (float)row[e];
            }
        }
#pragma unroll
        for (int kk = 0; kk < KD; kk += kDepth) {
            bf16x8 fa[TM], fb[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                fa[i] = *reinterpret_cast<const bf16x8*>(sA + ((BM / 2) * wm + 16 * i + fr) * pitch + kk + fk);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                fb[j] = *reinterpret_cast<const bf16x8*>(sB + ((BN / 2) * wn + 16 * j + fr) * pitch + kk + fk);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    if constexpr (ROWSUM) {
        if (rowsum) {
            rsum += __shfl_xor(rsum, 1, 64);
            rsum += __shfl_xor(rsum, 2, 64);
            const int32_t m = m0 + (tid >> 2);
            if ((tid & 3) == 0 && m < a.M) a.bpart[(int64_t)bz * a.M + m] = rsum;
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int32_t mb = m0 + (BM / 2) * wm + 16 * i + (lane >> 4) * 4;  // 4 consecutive rows
            const int32_t n = n0 + (BN / 2) * wn + 16 * j + fr;
            if (n >= a.nstore) continue;
            bf16 r[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int32_t m = mb + e;
                const float v = acc[i][j][e];
                r[e] = (bf16)0.0f;
                if (m >= a.M) continue;
                if constexpr (EPI == EPI_RELU_BF16) {
                    r[e] = (bf16)fmaxf(v + a.bias[n], 0.0f);
                    a.cb[(int64_t)m * a.ldc + n] = r[e];
                } else if constexpr (EPI == EPI_BIAS_F32) {
                    a.cf[(int64_t)m * a.ldc + n] = v + a.bias[n];
                } else if constexpr (EPI == EPI_MASK_BF16) {
                    const float h = (float)a.mask[(int64_t)m * a.ldm + n];
                    r[e] = (bf16)(h > 0.0f ? v : 0.0f);
                    a.cb[(int64_t)m * a.ldc + n] = r[e];
                } else if constexpr (EPI == EPI_SINE_BF16) {
                    float d;
                    if (a.dsin) {
                        d = a.dsin[(int64_t)m * a.ldd + n];
                    } else {
                        float z = a.b0[n];
                        for (int32_t c = 0; c < a.d0; ++c) z = fmaf(a.w0[n * a.d0 + c], a.x0[(int64_t)m * a.d0 + c], z);
                        d = first_deriv_sine(z, a.omega0);
                    }
                    r[e] = (bf16)(v * d);
                    a.cb[(int64_t)m * a.ldc + n] = r[e];
                } else {
                    a.cf[(int64_t)bz * a.zstride + (int64_t)m * a.ldc + n] = v;
                }
            }
            if constexpr (EPI == EPI_RELU_BF16 || EPI == EPI_MASK_BF16 || EPI == EPI_SINE_BF16) {
                if (a.cbt) {
                    bf16* dst = a.cbt + (int64_t)n * a.ldct + mb;
                    if (mb + 3 < a.M) {
                                                *reinterpret_cast<bf16x4*>(dst) = bf16x4{r[0], r[1], r[2], r[3]};
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (mb + e < a.M) dst[e] = r[e];
                    }
                }
            }
        }
}

template <bool A_KC, bool B_KC, int EPI, int BM, int BN, int KD>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs a) {
    gemm_tile<A_KC, B_KC, EPI, BM, BN, KD>(a, (int32_t)blockIdx.x, (int32_t)blockIdx.y, (int32_t)blockIdx.z);
}

struct SumAdamArgs {
    float* p; float* g; float* m; float* v;
    float lr, b1, b2, eps, c1, c2;
    int64_t woff[4], boff[4];
    int32_t din[4], dout[4], dpad[4];   // per layer l: inputs, outputs, padded outputs
    const float* wpart[4];     // l = 1..3: [wsplits][dpad][din]
    int32_t wsplits;
    const float* bpart[4];     // l = 1..3: [nblk][bw[l]] (bias of layer l)
    int32_t bw[4];
    const float* p0;           // [nblk][256][4]
    int32_t nblk;
    int32_t nlong;             // parameters summed over the row blocks
    bf16* wb[4]; bf16* wpf[4]; bf16* wpb[4];
    const float* lpart; float* loss; int64_t B;
};

// The input layer's weights and every bias: gradients summed over the row
// blocks, and their Adam step (block blk of ceil(nlong / 4); defined below).
__device__ void sum_adam_long(const SumAdamArgs& a, int32_t blk);

// Up to three products of one kind in one launch: blockIdx.z = problem *
// splits + split; blocks beyond a problem's row tiles return at once.
struct GemmBatch {
    GemmArgs g[3];
    int32_t lblocks;           // k_wgrad: leading blocks that run sum_adam_long (a multiple of 8)
    int32_t splits;
    int32_t mtiles[3];
    int32_t ntiles[3];
    int32_t toff[4];           // first tile of each problem within a split; toff[3] = tiles per split
};

// Rows from which the larger tiles pay (enough blocks to fill the chip;
// measured: at 8192 rows the 64 x 64 tiles are faster).
constexpr int32_t kBigTileRows = 32768;

template <bool A_KC, bool B_KC, int EPI>
int gemm(const GemmArgs& a, int32_t splits, hipStream_t s) {
    // vector loads need 8-element alignment along every contiguous dimension
    // (a k-contiguous operand may end in a partial chunk); transposed results
    // are stored 4 rows at a time
    const bool ok = (a.lda % 8 == 0) && (a.ldb % 8 == 0) && (A_KC || a.M % 8 == 0) &&
                    (B_KC || a.N % 8 == 0) && a.kchunk % kDepth == 0 && a.M > 0 && a.N > 0 && a.K > 0 &&
                    splits >= 1 && (int64_t)splits * a.kchunk >= a.K && (!a.cbt || a.ldct % 4 == 0) &&
                    (!a.bpart || A_KC);
    if (!ok) return fail(CV_ESTATE, "internal: matrix product shape");
    const bool deep = a.kchunk % 64 == 0;
    if (a.M >= kBigTileRows && splits == 1 && !a.bpart) {
        const dim3 grid((unsigned)((a.M + 127) / 128), (unsigned)((a.N + 63) / 64), 1);
        if (deep) hipLaunchKernelGGL((k_gemm<A_KC, B_KC, EPI, 128, 64, 64>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_gemm<A_KC, B_KC, EPI, 128, 64, 32>), grid, dim3(256), 0, s, a);
    } else {
        const dim3 grid((unsigned)((a.M + 63) / 64), (unsigned)((a.N + 63) / 64), (unsigned)splits);
        if (deep) hipLaunchKernelGGL((k_gemm<A_KC, B_KC, EPI, 64, 64, 64>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_gemm<A_KC, B_KC, EPI, 64, 64, 32>), grid, dim3(256), 0, s, a);
    }
    CV_HIP(hipGetLastError());
    return CV_OK;
}

// The three weight-gradient products of a fused training step in one launch
// (k_wgrad): k (the batch) split every kSplitRows rows, as in the unfused
// backward pass, so that both give the same sums.
constexpr int kWgBM = 64, kWgBN = 64;

// One block: a 64 x 64 tile of one product over one split (k_gemm's tile,
// EPI_PARTIAL_F32, both operands k-contiguous, one stage of 64 k ahead), on a
// one-dimensional grid mapped to the chip's eight XCDs: workgroups go to the
// XCDs in turn (workgroup L to XCD L % 8), so workgroup L takes split
// L % 8 + 8 q with q = (L / 8) / tiles, tile (L / 8) % tiles.  Every tile of
// a split then runs on one XCD and the split's operands come into that XCD's
// L2 once.  (Issuing all of a split's loads at once, held in registers, was
// slower: 13.7 against 12.8 us for the surrogate's 8192-row step.)  The
// first b.lblocks blocks instead sum the gradients of the input layer and the
// biases over the training step's row blocks and take their Adam step
// (sum_adam_long), which needs only the step's own partials: that work runs
// beside the products rather than in a launch of its own.  lblocks is a
// multiple of 8, so the XCD of every product block stays L % 8.
__global__ __launch_bounds__(256) void k_wgrad(GemmBatch b, SumAdamArgs sa) {
    if ((int32_t)blockIdx.x < b.lblocks) {
        sum_adam_long(sa, (int32_t)blockIdx.x);
        return;
    }
    const int32_t L = (int32_t)blockIdx.x - b.lblocks, xcd = L & 7, j = L >> 3;
    const int32_t z = xcd + 8 * (j / b.toff[3]), t = j % b.toff[3];
    if (z >= b.splits) return;
    const int32_t p = t < b.toff[1] ? 0 : t < b.toff[2] ? 1 : 2;
    const GemmArgs& a = p == 0 ? b.g[0] : p == 1 ? b.g[1] : b.g[2];
    const int32_t tl = t - b.toff[p], bx = tl / b.ntiles[p], by = tl - bx * b.ntiles[p];
    gemm_tile<true, true, EPI_PARTIAL_F32, 64, 64, 64>(a, bx, by, z);
}

int gemm_wgrad3(const GemmArgs (&g)[3], int32_t splits, const SumAdamArgs& sa, int32_t lblocks, hipStream_t s) {
    if (lblocks < 0 || lblocks % 8 != 0) return fail(CV_ESTATE, "internal: leading blocks of the weight gradients");
    GemmBatch b = {};
    b.lblocks = lblocks;
    for (int p = 0; p < 3; ++p) {
        const GemmArgs& a = g[p];
        const bool ok = a.lda % 8 == 0 && a.ldb % 8 == 0 && a.kchunk % 64 == 0 && a.M > 0 && a.N > 0 &&
                        a.K > 0 && (int64_t)splits * a.kchunk >= a.K && !a.bpart;
        if (!ok) return fail(CV_ESTATE, "internal: weight-gradient product shape");
        b.g[p] = a;
        b.mtiles[p] = (a.M + kWgBM - 1) / kWgBM;
        b.ntiles[p] = (a.N + kWgBN - 1) / kWgBN;
        b.toff[p + 1] = b.toff[p] + b.mtiles[p] * b.ntiles[p];
    }
    b.splits = splits;
    const int64_t nblocks = lblocks + (int64_t)8 * ((splits + 7) / 8) * b.toff[3];
    hipLaunchKernelGGL(k_wgrad, dim3((unsigned)nblocks), dim3(256), 0, s, b, sa);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

// ---------------------------------------------------------------------------
// Input layer on the vector ALUs: H1[s][o] = act(b0[o] + sum_c W0[o][c] x_c)
// with act = first_act (ReLU or the sinusoid) and x either FP32 [B][d0] or
// 8-bit RGB (x = v / 255 - 1/2).  d1 / 8 threads per row, each 8 consecutive
// outputs written as one 16-byte store; the weights sit in LDS.  d1 must be a
// multiple of 32 and at most 1024.
template <bool RGB8>
__global__ __launch_bounds__(256) void k_input_layer(const void* __restrict__ xin, int64_t B, int32_t d0,
                                                     int32_t d1, const float* __restrict__ W0,
                                                     const float* __restrict__ b0, float omega0,
                                                     bf16* __restrict__ H1, float* __restrict__ dsin) {
    __shared__ float s_w[kMaxHidden * (kMaxIn + 1)];
    for (int k = threadIdx.x; k < d1 * d0; k += 256) s_w[k] = W0[k];
    for (int k = threadIdx.x; k < d1; k += 256) s_w[d1 * d0 + k] = b0[k];
    __syncthreads();
    const int32_t groups = d1 / 8;                       // threads per row
    const int64_t total = B * groups;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += stride) {
        const int64_t s = t / groups;
        const int32_t o0 = (int32_t)(t - s * groups) * 8;
        float x[kMaxIn] = {0.f, 0.f, 0.f, 0.f};
        for (int32_t c = 0; c < d0; ++c) {
            if constexpr (RGB8) x[c] = rgb_input(static_cast<const uint8_t*>(xin)[s * 3 + c]);
            else x[c] = static_cast<const float*>(xin)[s * d0 + c];
        }
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int32_t o = o0 + e;
            float acc = s_w[d1 * d0 + o];
            for (int32_t c = 0; c < d0; ++c) acc = fmaf(s_w[o * d0 + c], x[c], acc);
            v[e] = (bf16)first_act(acc, omega0);
            // kept for the backward pass: the sine's derivative, as the
            // backward epilogue would recompute it
            if (dsin && omega0 > 0.0f) dsin[s * d1 + o] = first_deriv_sine(acc, omega0);
        }
        *reinterpret_cast<bf16x8*>(H1 + s * d1 + o0) = v;
    }
}

// Offset of element (n, k) of an [N][32 KS] matrix-core operand in the
// fragment-packed layout of the fused training step: per 16-row tile and
// 32-deep k step, the 64 lanes' 8-element fragments (lane n % 16 +
// 16 ((k % 32) / 8)) back to back, so that a wave's fragment load is 1 KB
// contiguous (twice as fast as 16 row pieces of 64 bytes).  N a multiple of
// 16.
__device__ __forceinline__ int64_t frag_off(int32_t n, int32_t k, int32_t KS) {
    return ((int64_t)((n >> 4) * KS + (k >> 5)) * 64 + (n & 15) + 16 * ((k & 31) >> 3)) * 8 + (k & 7);
}

// The 8-element fragment of lane (n % 16, k step ks) of a packed operand:
// fragments of one 16-row tile and k step are 1 KB contiguous over the wave.
__device__ __forceinline__ bf16x8 packed_frag(const bf16* __restrict__ Wp, int32_t KS, int32_t n, int32_t ks, int fk) {
    return *reinterpret_cast<const bf16x8*>(Wp + ((int64_t)((n >> 4) * KS + ks) * 64 + (n & 15) + 2 * fk) * 8);
}

// ---------------------------------------------------------------------------
// Fused inference of the surrogate's shape (inputs <= 4, three hidden layers
// of 256, outputs <= 64) from 8-bit colours: a block of eight waves takes
// kFusedRows rows through every layer with the activations in LDS, so
// nothing but the colours and the outputs touches HBM (the weights stay in
// L2).
//   - input layer: per element on the vector ALUs, as k_input_layer<true>
//     (ReLU or the sinusoid), thread t -> column t % 256, half the rows;
//   - hidden layers: wave w computes columns 64 (w % 4) .. + 63 of rows
//     64 (w / 4) .. + 63 (4 x 4 MFMA tiles), the weights (packed, frag_off)
//     as the A operand so that a lane's results are four consecutive
//     columns of one row (one 8-byte LDS store); the two waves of a column
//     group read the same fragments, the second from L1, and two blocks
//     share a CU so that one's loads and barriers overlap the other's
//     products.  Then a barrier, and the bias + ReLU results overwrite the
//     activations in LDS;
//   - output layer: wave w computes columns 16 (w % 4) .. + 15 of rows
//     64 (w / 4) .. + 63.
// Same instruction, fragment layout, k order and epilogue arithmetic as
// k_gemm, so the results equal the unfused pass bit for bit.
constexpr int kFusedRows = 128, kFusedWidth = 256, kFusedPitch = kFusedWidth + 8;

__global__ __launch_bounds__(512, 4) void k_mlp_infer_fused(const uint8_t* __restrict__ rgb, int64_t B, int32_t d0,
                                                            int32_t dout, const float* __restrict__ W0,
                                                            const float* __restrict__ b0, float omega0,
                                                            const bf16* __restrict__ W1, const float* __restrict__ b1,
                                                            const bf16* __restrict__ W2, const float* __restrict__ b2,
                                                            const bf16* __restrict__ W3, const float* __restrict__ b3,
                                                            float* __restrict__ out) {
    constexpr int TM = 4, KS = kFusedWidth / kDepth;  // row tiles per wave, k steps
    __shared__ __attribute__((aligned(16))) bf16 sH[kFusedRows * kFusedPitch];
    __shared__ float s_x[kFusedRows * kMaxIn];
    __shared__ __attribute__((aligned(16))) float s_bias[2 * kFusedWidth];  // hidden layers 2 and 3
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    const int rg = 64 * (w >> 2), cg = w & 3;  // the wave's first row, column group
    s_bias[tid] = tid < kFusedWidth ? b1[tid] : b2[tid - kFusedWidth];
    const int64_t r0 = (int64_t)blockIdx.x * kFusedRows;
    const int32_t rows = (int32_t)min((int64_t)kFusedRows, B - r0);
    for (int k = tid; k < kFusedRows * kMaxIn; k += 512) {
        const int r = k / kMaxIn, c = k - r * kMaxIn;
        s_x[k] = (r < rows && c < d0) ? rgb_input(rgb[(r0 + r) * 3 + c]) : 0.0f;
    }
    // input layer: thread t -> columns 2 (t % 128) and the next of rows
    // 32 (t / 128) .. + 31, their weights in registers
    {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        const int o = 2 * (tid & 127), rb = 32 * (tid >> 7);
        float wa[kMaxIn], wb[kMaxIn];
#pragma unroll
        for (int c = 0; c < kMaxIn; ++c) {
            wa[c] = c < d0 ? W0[o * d0 + c] : 0.0f;
            wb[c] = c < d0 ? W0[(o + 1) * d0 + c] : 0.0f;
        }
        const float ba = b0[o], bb = b0[o + 1];
        __syncthreads();
        if (d0 == 3) {
            for (int r = rb; r < rb + 32; ++r) {
                const float x0 = s_x[r * kMaxIn + 0], x1 = s_x[r * kMaxIn + 1], x2 = s_x[r * kMaxIn + 2];
                float za = ba, zb = bb;
                za = fmaf(wa[0], x0, za);
                zb = fmaf(wb[0], x0, zb);
                za = fmaf(wa[1], x1, za);
                zb = fmaf(wb[1], x1, zb);
                za = fmaf(wa[2], x2, za);
                zb = fmaf(wb[2], x2, zb);
                *reinterpret_cast<bf16x2*>(sH + r * kFusedPitch + o) =
                    bf16x2{(bf16)first_act(za, omega0), (bf16)first_act(zb, omega0)};
            }
        } else {
            for (int r = rb; r < rb + 32; ++r) {
                float za = ba, zb = bb;
                for (int32_t c = 0; c < d0; ++c) {
                    za = fmaf(wa[c < kMaxIn ? c : 0], s_x[r * kMaxIn + c], za);
                    zb = fmaf(wb[c < kMaxIn ? c : 0], s_x[r * kMaxIn + c], zb);
                }
                *reinterpret_cast<bf16x2*>(sH + r * kFusedPitch + o) =
                    bf16x2{(bf16)first_act(za, omega0), (bf16)first_act(zb, omega0)};
            }
        }
    }
    __syncthreads();
    // hidden layers
    for (int layer = 0; layer < 2; ++layer) {
        const bf16* Wl = layer == 0 ? W1 : W2;
        const float* bl = s_bias + layer * kFusedWidth;
        f32x4 acc[TM][4];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        // two blocks share a CU: the other hides this one's fragment loads
#pragma unroll 2
        for (int ks = 0; ks < KS; ++ks) {
            bf16x8 fb[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) fb[j] = packed_frag(Wl, KS, 64 * cg + 16 * j + fr, ks, fk);
            // weights as the A operand: a lane's results are four consecutive
            // columns of one row, stored with one 8-byte LDS write
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const bf16x8 fa =
                    *reinterpret_cast<const bf16x8*>(sH + (rg + 16 * i + fr) * kFusedPitch + kDepth * ks + fk);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[j], fa, acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();  // every wave has read the layer's input
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = 64 * cg + 16 * j + (lane >> 4) * 4;
            const float4 bias = *reinterpret_cast<const float4*>(bl + n);
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int m = rg + 16 * i + fr;
                const bf16x4 v = {(bf16)fmaxf(acc[i][j][0] + bias.x, 0.0f), (bf16)fmaxf(acc[i][j][1] + bias.y, 0.0f),
                                  (bf16)fmaxf(acc[i][j][2] + bias.z, 0.0f), (bf16)fmaxf(acc[i][j][3] + bias.w, 0.0f)};
                *reinterpret_cast<bf16x4*>(sH + m * kFusedPitch + n) = v;
            }
        }
        __syncthreads();
    }
    // output layer: 64 columns (dout <= 64, rows of W3 padded with zeros)
    {
        const int n = 16 * cg + fr;
        f32x4 acc[TM];
#pragma unroll
        for (int i = 0; i < TM; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
        bf16x8 fb = packed_frag(W3, KS, n, 0, fk), fbn = fb;
        for (int ks = 0; ks < KS; ++ks) {
            if (ks + 1 < KS) fbn = packed_frag(W3, KS, n, ks + 1, fk);
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const bf16x8 fa =
                    *reinterpret_cast<const bf16x8*>(sH + (rg + 16 * i + fr) * kFusedPitch + kDepth * ks + fk);
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[i], 0, 0, 0);
            }
            fb = fbn;
        }
        const float bias = n < dout ? b3[n] : 0.0f;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = rg + 16 * i + (lane >> 4) * 4 + e;
                if (m < rows && n < dout) out[(r0 + m) * dout + n] = acc[i][e] + bias;
            }
    }
}

// Column reductions for the bias gradients and the input layer's weight
// gradients.  Block (x, y) covers columns 64x .. 64x+63 and rows
// kColRows y .. + kColRows-1.  Thread (q, r) reads eight columns
// 64x + 8q .. + 7 as one 16-byte load from rows r, r + 32, ... of the tile
// and sums them in that order; the 32 row groups are then added in LDS in
// their fixed order, and part[y][o][k] receives, for column o,
// sum_s G[s][o] x[s][k] (k < d0) and sum_s G[s][o] (k = d0).  With d0 = 0
// only the column sums are formed.  ldg must be a multiple of 8.
constexpr int kColRows = 256, kColGroups = 32;

__global__ __launch_bounds__(256) void k_colgrad(const bf16* __restrict__ G, int64_t ldg,
                                                 const float* __restrict__ x, int32_t d0, int64_t B,
                                                 int32_t ncols, float* __restrict__ part) {
    __shared__ float s_acc[kColGroups][64][kMaxIn + 1];
    const int q = threadIdx.x & 7, r = threadIdx.x >> 3;
    const int32_t o0 = (int32_t)blockIdx.x * 64 + 8 * q;
    const int64_t s0 = (int64_t)blockIdx.y * kColRows, s1 = min(B, s0 + kColRows);
    float acc[8][kMaxIn + 1];
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int k = 0; k <= kMaxIn; ++k) acc[e][k] = 0.0f;
    if (o0 + 8 <= ldg) {
        for (int64_t sr = s0 + r; sr < s1; sr += kColGroups) {
            const bf16x8 v = *reinterpret_cast<const bf16x8*>(G + sr * ldg + o0);
            float xs[kMaxIn];
#pragma unroll
            for (int k = 0; k < kMaxIn; ++k) xs[k] = k < d0 ? x[sr * d0 + k] : 0.0f;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float ve = (float)v[e];
#pragma unroll
                for (int k = 0; k < kMaxIn; ++k)
                    if (k < d0) acc[e][k] = fmaf(ve, xs[k], acc[e][k]);
                acc[e][kMaxIn] += ve;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int k = 0; k <= kMaxIn; ++k) s_acc[r][8 * q + e][k] = acc[e][k];
    __syncthreads();
    for (int t = threadIdx.x; t < 64 * (kMaxIn + 1); t += 256) {
        const int c = t / (kMaxIn + 1), k = t - c * (kMaxIn + 1);
        const int32_t o = (int32_t)blockIdx.x * 64 + c;
        if (o >= ncols || (k < kMaxIn && k >= d0)) continue;
        float sum = 0.0f;
        for (int g = 0; g < kColGroups; ++g) sum += s_acc[g][c][k];
        part[((int64_t)blockIdx.y * ncols + o) * (d0 + 1) + (k == kMaxIn ? d0 : k)] = sum;
    }
}

__global__ void k_input_grad_sum(const float* __restrict__ part, int32_t splits, int32_t d0,
                                 int32_t d1, float* __restrict__ gW0, float* __restrict__ gb0) {
    const int32_t t = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    const int32_t per = d0 + 1;
    if (t >= d1 * per) return;
    float acc = 0.0f;
#pragma unroll 8
    for (int32_t z = 0; z < splits; ++z) acc += part[(int64_t)z * d1 * per + t];
    const int32_t o = t / per, c = t - o * per;
    if (c < d0) gW0[o * d0 + c] = acc;
    else gb0[o] = acc;
}

// One launch for a layer's two fixed-order sums: the weight gradient from
// its split partials pw [z][rows][ldp] (threads t < rows * cols), then the
// bias gradient from the column partials pb [z][rows] (the next rows threads).
__global__ void k_sum_grads(const float* __restrict__ pw, int32_t wsplits, int64_t zstride, int32_t rows,
                            int32_t cols, int64_t ldp, float* __restrict__ gw, const float* __restrict__ pb,
                            int32_t bsplits, int64_t ldpb, float* __restrict__ gb) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nw = (int64_t)rows * cols;
    if (t < nw) {
        const int32_t r = (int32_t)(t / cols), c = (int32_t)(t - (int64_t)r * cols);
        float acc = 0.0f;
#pragma unroll 8
        for (int32_t z = 0; z < wsplits; ++z) acc += pw[z * zstride + (int64_t)r * ldp + c];
        gw[t] = acc;
    } else if (t < nw + rows) {
        const int32_t o = (int32_t)(t - nw);
        float acc = 0.0f;
#pragma unroll 8
        for (int32_t z = 0; z < bsplits; ++z) acc += pb[(int64_t)z * ldpb + o];
        gb[o] = acc;
    }
}

// FP32 output gradient -> BF16, zero-padded to the padded output width.
__global__ void k_grad_to_bf16(const float* __restrict__ g, int64_t B, int32_t d, int32_t dp,
                               bf16* __restrict__ G) {
    const int64_t total = B * dp;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const int64_t s = t / dp;
        const int32_t c = (int32_t)(t - s * dp);
        G[t] = (bf16)(c < d ? g[s * d + c] : 0.0f);
    }
}

// FP32 master weights -> BF16 copy [dp][din], rows d..dp-1 zero.
__global__ void k_weights_bf16(const float* __restrict__ W, int32_t d, int32_t dp, int32_t din,
                               bf16* __restrict__ Wb) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)dp * din) return;
    const int32_t o = (int32_t)(t / din);
    Wb[t] = (bf16)(o < d ? W[t] : 0.0f);
}

// FP32 master weights W [d][din] -> the packed BF16 operands of the fused
// training step: Wf (forward, n = output padded to dp, k = input) and Wb
// (backward, n = input, k = output padded to dp); padding zero.  din a
// multiple of 32.
__global__ void k_weights_packed(const float* __restrict__ W, int32_t d, int32_t dp, int32_t din,
                                 bf16* __restrict__ Wf, bf16* __restrict__ Wb) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)dp * din) return;
    const int32_t o = (int32_t)(t / din), c = (int32_t)(t - (int64_t)o * din);
    const bf16 v = (bf16)(o < d ? W[t] : 0.0f);
    Wf[frag_off(o, c, din / 32)] = v;
    Wb[frag_off(c, o, dp / 32)] = v;
}

// Loss of a batch and its gradient with respect to the outputs.  Per sample s
// with outputs z[0..D-1] (D-1 radii and the feasibility logit):
//   l_s = (1/(D-1)) sum_k [t_k > 0] huber(z_k - t_k) + softplus(z) - z f
// gradient dl/dz / B, written as FP32 [B][D] (gout) and / or rounded to BF16
// with zero padding [B][ldgb] (gb, ldgb >= D: the first operand of the
// backward pass).  Block x takes rows 16x .. 16x+15, one wave per row and one
// lane per output; its loss terms are summed by a fixed tree into part[x].
constexpr int kLossRows = 16;

__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ out, const float* __restrict__ tr,
                                              const float* __restrict__ tf, int64_t B, int32_t D,
                                              float delta, float* __restrict__ gout, bf16* __restrict__ gb,
                                              int32_t ldgb, float* __restrict__ part) {
    __shared__ float s_sum[256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t R = D - 1;
    const int32_t width = gb ? max(D, ldgb) : D;
    const float invR = 1.0f / (float)R, invB = 1.0f / (float)B;
    float ls = 0.0f;
    const int64_t s0 = (int64_t)blockIdx.x * kLossRows;
#pragma unroll
    for (int rr = w; rr < kLossRows; rr += 4) {
        const int64_t s = s0 + rr;
        if (s >= B) continue;
        for (int32_t c = lane; c < width; c += 64) {
            float g = 0.0f;
            if (c < R) {
                const float t = tr[s * R + c];
                if (t > 0.0f) {
                    const float e = out[s * D + c] - t, ae = fabsf(e);
                    ls += (ae <= delta ? 0.5f * e * e : delta * (ae - 0.5f * delta)) * invR;
                    g = (ae <= delta ? e : copysignf(delta, e)) * invR;
                }
            } else if (c == R) {
                const float z = out[s * D + R], f = tf[s];
                ls += fmaxf(z, 0.0f) - z * f + log1pf(expf(-fabsf(z)));
                g = 1.0f / (1.0f + expf(-z)) - f;
            }
            g *= invB;
            if (gout && c < D) gout[s * D + c] = g;
            if (gb) gb[s * ldgb + c] = (bf16)g;
        }
    }
    s_sum[threadIdx.x] = ls;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s_sum[threadIdx.x] += s_sum[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s_sum[0];
}

// Total of the per-block loss partials in FP64: thread t sums partials
// t, t + 256, ... in order, then a fixed tree.
__global__ __launch_bounds__(256) void k_loss_total(const float* __restrict__ part, int32_t nparts, int64_t B,
                                                    float* __restrict__ loss) {
    __shared__ double s_sum[256];
    double acc = 0.0;
    for (int32_t k = (int32_t)threadIdx.x; k < nparts; k += 256) acc += part[k];
    s_sum[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s_sum[threadIdx.x] += s_sum[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(s_sum[0] / (double)B);
}

// Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr (m c1) / (sqrt(v c2) + eps) with c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
// The new value of every matrix-core weight also goes to its BF16 copy
// (the rows of W_l [d][din] are the first d rows of the copy [dpad][din]).
struct BF16Copies {
    int32_t n = 0;
    int64_t off[kMaxLayers] = {};
    int64_t cnt[kMaxLayers] = {};
    bf16* dst[kMaxLayers] = {};
    // packed copies (frag_off; nullable): forward [dp][din], backward [din][dp]
    bf16* pf[kMaxLayers] = {};
    bf16* pb[kMaxLayers] = {};
    int32_t din[kMaxLayers] = {};
    int32_t dp[kMaxLayers] = {};
};

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, BF16Copies cp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    for (int32_t l = 0; l < cp.n; ++l)
        if (i >= cp.off[l] && i < cp.off[l] + cp.cnt[l]) {
            const int64_t k = i - cp.off[l];
            cp.dst[l][k] = (bf16)pi;
            if (cp.pf[l]) {
                const int32_t o = (int32_t)(k / cp.din[l]), c = (int32_t)(k - (int64_t)o * cp.din[l]);
                cp.pf[l][frag_off(o, c, cp.din[l] / 32)] = (bf16)pi;
                cp.pb[l][frag_off(c, o, cp.dp[l] / 32)] = (bf16)pi;
            }
        }
}

// ---------------------------------------------------------------------------
// Fused training step of the surrogate's shape (3 inputs, three hidden layers
// of 256, 37 outputs padded to 64): three launches per step instead of about
// twenty.
//  1. k_train_step: per block of kTrainRows rows, the training rows from the
//     cube table (k_table_batch's arithmetic), the input layer and the three
//     matrix-core layers (the arithmetic of k_mlp_infer_fused), the loss and
//     its gradient in the output layer's epilogue (the arithmetic of k_loss),
//     then the gradient back through the three layers (the arithmetic of the
//     unfused backward pass; the sine's derivative recomputed from the
//     inputs, bit for bit the forward's).  Activations and gradients stay in
//     LDS, each layer's in a buffer of its own (a gradient overwrites the
//     activation whose ReLU mask it consumed, element by element).  It
//     writes the activations and the gradients transposed (the weight
//     gradients' k-contiguous operands) and the block's sums for the loss,
//     the bias gradients and the input layer's gradient.
//  2. the three weight-gradient products in one launch (k_wgrad, split over
//     the batch);
//  3. k_sum_adam: every parameter's gradient summed from its partials in a
//     fixed order, the Adam step, and the weights' BF16 copies.
// A block has 16 waves: wave w owns the 16 columns 16 w .. 16 w + 15 of every
// hidden layer for the block's 32 rows (two MFMA row tiles) and holds all
// eight 32-deep weight fragments of its columns in registers, fetched while
// the previous layer's epilogue runs, so a layer waits for one round of
// loads.  A batch of 8192 rows gives one block per CU; the waves per block
// are what hide the latencies.
constexpr int kTrainRows = 32, kTW = 256, kTPitch = kTW + 8, kTThreads = 1024, kTWaves = kTThreads / 64;
constexpr int kTK = kTW / kDepth;  // 32-deep k steps of a hidden layer
constexpr int kGP = 72;            // LDS pitch of the output gradient [32][64]

struct TrainArgs {
    const int32_t* ids;          // [B] colour ids (low 24 bits)
    const cv_table_row* table;   // [2^24]
    float rscale;                // radius target per index step (dr / 50)
    int64_t B;
    float omega0;                // > 0: sinusoidal first layer
    float delta;                 // Huber threshold
    const float* W0;             // [256][3] FP32
    const float* b0;
    const bf16* W1;              // forward operands, packed (frag_off): [256][256]
    const float* b1;
    const bf16* W2;
    const float* b2;
    const bf16* W3;              // [64][256], rows 37..63 zero
    const float* b3;
    const bf16* W3t;             // backward operands, packed: W3 transposed [256][64]
    const bf16* W2t;             // [256][256]
    const bf16* W1t;
    int64_t ldt;
    bf16* h1t; bf16* h2t; bf16* h3t;   // activations transposed [256][ldt]
    bf16* goutt;                 // output gradient transposed [64][ldt]
    bf16* g3t; bf16* g2t;        // gradients of layers 3 and 2's pre-activations, transposed [256][ldt]
    float* lpart;                // [nblk]: the block's loss sum
    float* pb3;                  // [nblk][64]: sums of the output gradient (output bias)
    float* pb2;                  // [nblk][256]
    float* pb1;                  // [nblk][256]
    float* p0;                   // [nblk][256][4]: sum G1 x_c (c < 3), sum G1
};

// The KS fragments (kDepth deep each) of row n of a packed operand (see
// frag_off): the B operands of one 16-column MFMA tile over k < 32 KS.
template <int KS>
__device__ __forceinline__ void load_frags(bf16x8 (&fb)[KS], const bf16* __restrict__ Wp, int n, int fk) {
#pragma unroll
    for (int k = 0; k < KS; ++k)
        fb[k] = *reinterpret_cast<const bf16x8*>(Wp + ((int64_t)((n >> 4) * KS + k) * 64 + (n & 15) + 2 * fk) * 8);
}

// acc[i] = rows 16 (i0 + i) .. + 15 of sA (LDS, pitch lda) times the
// fragments, k ascending (k_gemm's order).
template <int TM, int KS>
__device__ __forceinline__ void tile_products(f32x4 (&acc)[TM], const bf16* sA, int lda, int i0,
                                              const bf16x8 (&fb)[KS], int fr, int fk) {
#pragma unroll
    for (int i = 0; i < TM; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < KS; ++k)
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const bf16x8 fa = *reinterpret_cast<const bf16x8*>(sA + (16 * (i0 + i) + fr) * lda + kDepth * k + fk);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb[k], acc[i], 0, 0, 0);
        }
}

// Rows mb .. mb + 3 of one column of a transposed operand (dst = its row
// at mb), written whole: the operands' rows are padded to whole blocks of
// kTrainRows, and what lands past the batch is never read.  The kernel's
// global stores have no branch around them, so that the compiler knows how
// many memory operations follow each load and never waits for a store when
// it waits for a load (the counters count both).
__device__ __forceinline__ void store_col4(bf16* __restrict__ dst, const bf16 (&r)[4]) {
    *reinterpret_cast<bf16x4*>(dst) = bf16x4{r[0], r[1], r[2], r[3]};
}

// Epilogue of one backward layer for column n: the products times the
// activation derivative (sine: the factor; else the ReLU mask), rounded to
// BF16.  Not FIRST: to sOut (LDS) and transposed to gt, the column's sums
// over the block's rows to pb.  FIRST (the first hidden layer): with x (sx)
// the input layer's sums to p0.  Every lane stores the column's sums (the
// four lanes of a column hold the same values), so no branch holds a store.
template <bool FIRST>
__device__ __forceinline__ void back_epilogue(const f32x4 (&acc)[kTrainRows / 16], const float (&d)[kTrainRows / 16][4],
                                              bool sine, bf16* sOut, bf16* __restrict__ gt, int64_t ldt,
                                              float* __restrict__ pb, const float* sx, float* __restrict__ p0,
                                              int64_t r0, int32_t rows, int n, int lane) {
    float cs = 0.0f, cx[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < kTrainRows / 16; ++i) {
        const int mb = 16 * i + (lane >> 4) * 4;
        bf16 r[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int mm = mb + e;
            r[e] = (bf16)0.0f;
            if (mm < rows) {
                const float v = acc[i][e];
                r[e] = sine ? (bf16)(v * d[i][e]) : (bf16)(d[i][e] > 0.0f ? v : 0.0f);
            }
            const float rv = (float)r[e];
            cs += rv;
            if constexpr (FIRST) {
#pragma unroll
                for (int c = 0; c < 3; ++c) cx[c] = fmaf(rv, sx[mm * 4 + c], cx[c]);
            } else {
                sOut[mm * kTPitch + n] = r[e];
            }
        }
        if constexpr (!FIRST) store_col4(gt + (int64_t)n * ldt + r0 + mb, r);
    }
    // the four lane groups hold the other rows of column n (each lane adds
    // the same pairs: the same value on all four)
    cs += __shfl_xor(cs, 16, 64);
    cs += __shfl_xor(cs, 32, 64);
    if constexpr (FIRST) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx[c] += __shfl_xor(cx[c], 16, 64);
            cx[c] += __shfl_xor(cx[c], 32, 64);
        }
    }
    if constexpr (FIRST) {
        p0[(int64_t)n * 4 + 0] = cx[0];
        p0[(int64_t)n * 4 + 1] = cx[1];
        p0[(int64_t)n * 4 + 2] = cx[2];
        p0[(int64_t)n * 4 + 3] = cs;
    } else {
        pb[n] = cs;
    }
}

// The ReLU masks of a lane's results (rows 16 i + 4 (lane / 16) + e of
// column n) from a layer's activations in LDS.
__device__ __forceinline__ void lds_mask(float (&d)[kTrainRows / 16][4], const bf16* sH, int n, int lane) {
#pragma unroll
    for (int i = 0; i < kTrainRows / 16; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) d[i][e] = (float)sH[(16 * i + (lane >> 4) * 4 + e) * kTPitch + n];
}

// The same masks from bits kept by the forward pass (bit b0 + 4 i + e set
// where that activation is positive): the lane's forward results are the
// same rows of the same column.
__device__ __forceinline__ void bit_mask(float (&d)[kTrainRows / 16][4], uint32_t bits, int b0) {
#pragma unroll
    for (int i = 0; i < kTrainRows / 16; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) d[i][e] = (bits >> (b0 + 4 * i + e)) & 1u ? 1.0f : 0.0f;
}

__global__ __launch_bounds__(kTThreads) void k_train_step(TrainArgs a) {
    constexpr int TM = kTrainRows / 16;  // MFMA row tiles per wave
    __shared__ __attribute__((aligned(16))) bf16 sH1[kTrainRows * kTPitch];
    __shared__ __attribute__((aligned(16))) bf16 sH2[kTrainRows * kTPitch];
    __shared__ __attribute__((aligned(16))) bf16 sH3[kTrainRows * kTPitch];
    __shared__ __attribute__((aligned(16))) bf16 sG[kTrainRows * kGP];
    __shared__ float s_w0[kTW * 4];
    __shared__ __attribute__((aligned(16))) float s_x[kTrainRows * 4];
    __shared__ uint32_t s_row[kTrainRows * 10];  // the rows' table entries (cv_table_row, 40 bytes)
    __shared__ float s_red[kTWaves];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    const int n = 16 * w + fr;  // this lane's column of the hidden layers
    const int64_t r0 = (int64_t)blockIdx.x * kTrainRows;
    const int32_t rows = (int32_t)min((int64_t)kTrainRows, a.B - r0);
    const int64_t blk = blockIdx.x;
    // Loads in the order they are waited for (the counters are in order): the
    // input layer's weights and the ids, then the W1 fragments, then the
    // rows' table entries (thread -> 4 bytes of row tid / 10), which only the
    // loss needs and which reach LDS just before it.  Every thread loads (an
    // id of the block's last row, the first word of entry 0 past the rows):
    // no branch holds a load, so none is waited for before its use.
    const float w0v = tid < kTW * 3 ? a.W0[tid] : a.b0[tid - kTW * 3];
    const int rr = tid / 10;
    const uint32_t idw = (uint32_t)a.ids[r0 + min(rr, rows - 1)];
    __builtin_amdgcn_sched_barrier(0);  // these two first: the first barrier waits for them alone
    bf16x8 fb[kTK];
    load_frags(fb, a.W1, n, fk);
    const int no = 16 * (w & 3) + fr;  // the output column of waves 0..7
    const float bias1 = a.b1[n], bias2 = a.b2[n], bias3 = a.b3[no < 37 ? no : 0];
    const bool rowthread = tid < kTrainRows * 10;
    const uint32_t rid = rowthread && rr < rows ? idw & 0xFFFFFFu : 0u;
    const uint32_t tword = reinterpret_cast<const uint32_t*>(a.table + rid)[rowthread ? tid - 10 * rr : 0];
    s_w0[tid] = w0v;
    // the block's training rows (k_table_batch's arithmetic)
    if (rowthread && tid == 10 * rr) {
        s_x[rr * 4 + 0] = rgb_input(rid >> 16);
        s_x[rr * 4 + 1] = rgb_input((rid >> 8) & 255u);
        s_x[rr * 4 + 2] = rgb_input(rid & 255u);
        s_x[rr * 4 + 3] = 0.0f;
    }
    __syncthreads();
    // input layer (k_input_layer's arithmetic): thread -> column tid % 256,
    // 8 rows (consecutive columns over the lanes: no LDS bank conflicts),
    // stored transposed as one 16-byte chunk
    static_assert(kTW * (kTrainRows / 8) == kTThreads, "input layer: one thread per column and 8 rows");
    {
        const int o = tid & (kTW - 1), rg = (tid / kTW) * 8;
        const float w00 = s_w0[o * 3 + 0], w01 = s_w0[o * 3 + 1], w02 = s_w0[o * 3 + 2], bo = s_w0[kTW * 3 + o];
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float4 x = *reinterpret_cast<const float4*>(s_x + (rg + e) * 4);
            float acc = bo;
            acc = fmaf(w00, x.x, acc);
            acc = fmaf(w01, x.y, acc);
            acc = fmaf(w02, x.z, acc);
            v[e] = (bf16)first_act(acc, a.omega0);
            sH1[(rg + e) * kTPitch + o] = v[e];
        }
        *reinterpret_cast<bf16x8*>(a.h1t + (int64_t)o * a.ldt + r0 + rg) = v;
    }
    __syncthreads();
    f32x4 acc[TM];
    uint32_t mbits = 0;  // ReLU masks of the lane's results in hidden layers 2 (bits 0..7) and 3 (8..15)
    // hidden layer 2 (sH1 -> sH2), then 3 (sH2 -> sH3)
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const bf16* sIn = layer == 0 ? sH1 : sH2;
        bf16* sOut = layer == 0 ? sH2 : sH3;
        tile_products<TM, kTK>(acc, sIn, kTPitch, 0, fb, fr, fk);
        // the next layer's fragments in flight during the epilogue
        if (layer == 0) load_frags(fb, a.W2, n, fk);
        else if (w < 8) load_frags(fb, a.W3, no, fk);
        const float bias = layer == 0 ? bias1 : bias2;
        bf16* ht = (layer == 0 ? a.h2t : a.h3t) + (int64_t)n * a.ldt + r0;
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int mb = 16 * i + (lane >> 4) * 4;
            bf16 r[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                r[e] = (bf16)fmaxf(acc[i][e] + bias, 0.0f);
                sOut[(mb + e) * kTPitch + n] = r[e];
                if ((float)r[e] > 0.0f) mbits |= 1u << (8 * layer + 4 * i + e);
            }
            store_col4(ht + mb, r);
        }
        if (layer == 1 && tid < kTrainRows * 10) s_row[tid] = tword;
        __syncthreads();
    }
    // output layer: waves 0..7, wave w -> row tile w / 4, columns 16 (w % 4) ..;
    // the loss and its gradient (k_loss's arithmetic) in the epilogue, the
    // gradient to sG (zero beyond the batch and in the padding columns)
    bf16x8 f3[64 / kDepth], f2[kTK];
    load_frags(f3, a.W3t, n, fk);
    float ls = 0.0f;
    if (w < 8) {
        const int i = w >> 2;
        f32x4 ao[1];
        tile_products<1, kTK>(ao, sH3, kTPitch, i, fb, fr, fk);
        const int32_t R = 36;
        const float invR = 1.0f / (float)R, invB = 1.0f / (float)a.B;
        const float bias = bias3;
        const int mb = 16 * i + (lane >> 4) * 4;
        bf16 gv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int mm = mb + e;
            float g = 0.0f;
            if (mm < rows) {
                const float z = ao[0][e] + bias;
                const cv_table_row* trow = reinterpret_cast<const cv_table_row*>(s_row + 10 * mm);
                if (no < R) {
                    const float t = (float)trow->bin_ridx[no] * a.rscale;
                    if (t > 0.0f) {
                        const float er = z - t, ae = fabsf(er);
                        ls += (ae <= a.delta ? 0.5f * er * er : a.delta * (ae - 0.5f * a.delta)) * invR;
                        g = (ae <= a.delta ? er : copysignf(a.delta, er)) * invR;
                    }
                } else if (no == R) {
                    const float f = trow->count > 0 ? 1.0f : 0.0f;
                    ls += fmaxf(z, 0.0f) - z * f + log1pf(expf(-fabsf(z)));
                    g = 1.0f / (1.0f + expf(-z)) - f;
                }
                g *= invB;
            }
            gv[e] = (bf16)g;
            sG[mm * kGP + no] = gv[e];
        }
        store_col4(a.goutt + (int64_t)no * a.ldt + r0 + mb, gv);
    }
    load_frags(f2, a.W2t, n, fk);
    // the block's loss: each wave's sum, then the waves in order
    for (int off = 32; off > 0; off >>= 1) ls += __shfl_xor(ls, off, 64);
    if (lane == 0) s_red[w] = ls;
    float d[TM][4];
    bit_mask(d, mbits, 8);
    __syncthreads();
    if (tid == 0) {
        float t = 0.0f;
        for (int q = 0; q < kTWaves; ++q) t += s_red[q];
        a.lpart[blk] = t;
    }
    // output bias: column sums of the output gradient
    if (tid >= 64 && tid < 128) {
        const int c = tid - 64;
        float cs = 0.0f;
        for (int r = 0; r < kTrainRows; ++r) cs += (float)sG[r * kGP + c];
        a.pb3[blk * 64 + c] = cs;
    }
    // backward layer 3: G3 = (Gout W3) . [H3 > 0] -> sH3 (over H3), G3^T; bias of the third hidden layer
    tile_products<TM, 64 / kDepth>(acc, sG, kGP, 0, f3, fr, fk);
    bf16x8 f1[kTK];
    load_frags(f1, a.W1t, n, fk);
    back_epilogue<false>(acc, d, false, sH3, a.g3t, a.ldt, a.pb2 + blk * kTW, nullptr, nullptr, r0, rows, n, lane);
    bit_mask(d, mbits, 0);
    __syncthreads();
    // backward layer 2: G2 = (G3 W2) . [H2 > 0] -> sH2 (over H2), G2^T
    tile_products<TM, kTK>(acc, sH3, kTPitch, 0, f2, fr, fk);
    back_epilogue<false>(acc, d, false, sH2, a.g2t, a.ldt, a.pb1 + blk * kTW, nullptr, nullptr, r0, rows, n, lane);
    const bool sine = a.omega0 > 0.0f;
    if (sine) {
        // omega0 cos(omega0 z), z = b0 + W0 x: the forward's operations in its order
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int mm = 16 * i + (lane >> 4) * 4 + e;
                float z = s_w0[kTW * 3 + n];
                z = fmaf(s_w0[n * 3 + 0], s_x[mm * 4 + 0], z);
                z = fmaf(s_w0[n * 3 + 1], s_x[mm * 4 + 1], z);
                z = fmaf(s_w0[n * 3 + 2], s_x[mm * 4 + 2], z);
                d[i][e] = mm < rows ? first_deriv_sine(z, a.omega0) : 0.0f;
            }
    } else {
        lds_mask(d, sH1, n, lane);
    }
    __syncthreads();
    // backward layer 1: G1 = (G2 W1) . act'(z1); the input layer's sums
    tile_products<TM, kTK>(acc, sH2, kTPitch, 0, f1, fr, fk);
    back_epilogue<true>(acc, d, sine, nullptr, nullptr, a.ldt, nullptr, s_x, a.p0 + blk * kTW * 4, r0, rows, n, lane);
}


// One Adam step: new moments mi, vi and value pi from gradient gi and the
// old moments and value m0, v0, p0.
__device__ __forceinline__ void adam_math(const SumAdamArgs& a, float gi, float m0, float v0, float p0, float& mi,
                                          float& vi, float& pi) {
    mi = a.b1 * m0 + (1.0f - a.b1) * gi;
    vi = a.b2 * v0 + (1.0f - a.b2) * gi * gi;
    pi = p0 - a.lr * (mi * a.c1) / (sqrtf(vi * a.c2) + a.eps);
}

// Adam on parameter i with gradient gi and its moments and value m0, v0, p0
// (loaded before the gradient's sum, so that their latency overlaps it).
__device__ __forceinline__ void adam_one(const SumAdamArgs& a, int64_t i, float gi, float m0, float v0, float p0) {
    float mi, vi, pi;
    adam_math(a, gi, m0, v0, p0, mi, vi, pi);
    a.g[i] = gi;
    a.m[i] = mi;
    a.v[i] = vi;
    a.p[i] = pi;
}

// Adam on parameters i .. i + 3, weights k .. k + 3 of matrix-core layer l
// (k a multiple of 4, so the four share a row of W_l and sit together in
// its row-major and forward packed copies), with their BF16 copies.
__device__ __forceinline__ void adam_four(const SumAdamArgs& a, int64_t i, const float4& g4, int l, int64_t k,
                                          const float4& m4, const float4& v4, const float4& p4) {
    const float gs[4] = {g4.x, g4.y, g4.z, g4.w}, ms[4] = {m4.x, m4.y, m4.z, m4.w},
                vs[4] = {v4.x, v4.y, v4.z, v4.w}, ps[4] = {p4.x, p4.y, p4.z, p4.w};
    float mi[4], vi[4], pi[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) adam_math(a, gs[e], ms[e], vs[e], ps[e], mi[e], vi[e], pi[e]);
    *reinterpret_cast<float4*>(a.g + i) = g4;
    *reinterpret_cast<float4*>(a.m + i) = make_float4(mi[0], mi[1], mi[2], mi[3]);
    *reinterpret_cast<float4*>(a.v + i) = make_float4(vi[0], vi[1], vi[2], vi[3]);
    *reinterpret_cast<float4*>(a.p + i) = make_float4(pi[0], pi[1], pi[2], pi[3]);
    const int32_t o = (int32_t)(k / a.din[l]), c = (int32_t)(k - (int64_t)o * a.din[l]);
    const bf16x4 h = {(bf16)pi[0], (bf16)pi[1], (bf16)pi[2], (bf16)pi[3]};
    *reinterpret_cast<bf16x4*>(a.wb[l] + k) = h;
    *reinterpret_cast<bf16x4*>(a.wpf[l] + frag_off(o, c, a.din[l] / 32)) = h;
#pragma unroll
    for (int e = 0; e < 4; ++e) a.wpb[l][frag_off(c + e, o, a.dpad[l] / 32)] = h[e];
}

// Wave -> one parameter whose gradient sums one partial per row block (the
// input layer's weights and every bias): lane j adds the partials j, j + 64,
// .. in order, then the lanes in a fixed tree (lane 0's result).  Block 0
// also sums the loss partials (k_loss_total's way).
__device__ void sum_adam_long(const SumAdamArgs& a, int32_t blk) {
    if (blk == 0 && a.loss) {
        __shared__ double s_sum[256];
        double acc = 0.0;
        for (int32_t k = (int32_t)threadIdx.x; k < a.nblk; k += 256) acc += a.lpart[k];
        s_sum[threadIdx.x] = acc;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) s_sum[threadIdx.x] += s_sum[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) *a.loss = (float)(s_sum[0] / (double)a.B);
    }
    const int lane = threadIdx.x & 63;
    int32_t q = blk * 4 + (int32_t)(threadIdx.x >> 6);
    if (q >= a.nlong) return;
    // parameter q: W0 [dout0][din0], b0, then b1, b2, b3
    const float* src;
    int64_t stride, i;
    const int32_t nw0 = a.dout[0] * a.din[0];
    if (q < nw0) {
        const int32_t o = q / a.din[0], c = q - o * a.din[0];
        src = a.p0 + (int64_t)o * 4 + c;
        stride = 256 * 4;
        i = a.woff[0] + q;
    } else if (q < nw0 + a.dout[0]) {
        const int32_t o = q - nw0;
        src = a.p0 + (int64_t)o * 4 + 3;
        stride = 256 * 4;
        i = a.boff[0] + o;
    } else {
        q -= nw0 + a.dout[0];
        int l = 1;
        while (l < 3 && q >= a.dout[l]) q -= a.dout[l++];
        src = a.bpart[l] + q;
        stride = a.bw[l];
        i = a.boff[l] + q;
    }
    const float m0 = a.m[i], v0 = a.v[i], p0 = a.p[i];
    float gi = 0.0f;
    for (int32_t b = lane; b < a.nblk; b += 64) gi += src[(int64_t)b * stride];
    for (int off = 32; off > 0; off >>= 1) gi += __shfl_xor(gi, off, 64);
    if (lane == 0) adam_one(a, i, gi, m0, v0, p0);
}

// Thread -> four consecutive weights of the matrix-core layers, each gradient
// the sum of wsplits partials in split order (16-byte loads, coalesced over
// the threads), then their Adam step.  The biases between the layers' weights
// are left to sum_adam_long.
__global__ __launch_bounds__(256) void k_sum_adam(SumAdamArgs a) {
    const int64_t i = a.woff[1] + ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (i >= a.boff[3]) return;
    const int l = i < a.woff[2] ? 1 : i < a.woff[3] ? 2 : 3;
    if (i >= a.boff[l]) return;  // a bias
    const int64_t k = i - a.woff[l];
    const int64_t zs = (int64_t)a.dpad[l] * a.din[l];
    const float4 m0 = *reinterpret_cast<const float4*>(a.m + i), v0 = *reinterpret_cast<const float4*>(a.v + i),
                 p0 = *reinterpret_cast<const float4*>(a.p + i);
    const float* src = a.wpart[l] + k;
    float4 gi = make_float4(0.f, 0.f, 0.f, 0.f);
    int32_t z = 0;
    for (; z + 8 <= a.wsplits; z += 8) {  // 8 loads in flight, added in order
        float4 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = *reinterpret_cast<const float4*>(src + (int64_t)(z + q) * zs);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            gi.x += v[q].x;
            gi.y += v[q].y;
            gi.z += v[q].z;
            gi.w += v[q].w;
        }
    }
    for (; z < a.wsplits; ++z) {
        const float4 v = *reinterpret_cast<const float4*>(src + (int64_t)z * zs);
        gi.x += v.x;
        gi.y += v.y;
        gi.z += v.z;
        gi.w += v.w;
    }
    adam_four(a, i, gi, l, k, m0, v0, p0);
}

// Training rows from a table of the whole cube: x = RGB / 255 - 1/2 of colour
// id, radius targets ridx * dr / 50 per bin (0 = no valid radius), feasibility
// = count > 0.
__global__ void k_table_batch(const int32_t* __restrict__ ids, const cv_table_row* __restrict__ table,
                              int64_t B, float rscale, float* __restrict__ x, float* __restrict__ tr,
                              float* __restrict__ tf) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const uint32_t id = (uint32_t)ids[s] & 0xFFFFFFu;
    x[s * 3 + 0] = rgb_input(id >> 16);
    x[s * 3 + 1] = rgb_input((id >> 8) & 255u);
    x[s * 3 + 2] = rgb_input(id & 255u);
    const cv_table_row& r = table[id];
    for (int k = 0; k < 36; ++k) tr[s * 36 + k] = (float)r.bin_ridx[k] * rscale;
    tf[s] = r.count > 0 ? 1.0f : 0.0f;
}

// A keyed pseudorandom permutation of [0, n): a balanced Feistel network of
// four rounds on 2h-bit values (2^2h >= n, at most 4n), with cycle walking
// back into [0, n) (Black and Rogaway 2002, "Ciphers with arbitrary finite
// domains").  A Feistel network is a bijection whatever its round function,
// so cycle walking ends at the latest when it comes back round to the start;
// the expected number of steps is below 4.  Round r: (L, R) -> (R, L xor
// (mix64(R + k_r) mod 2^h)), mix64 the SplitMix64 finaliser, k_r =
// mix64(key + (r + 1) 0x9E3779B97F4A7C15).
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct FeistelKey {
    uint64_t k[4];
    uint32_t h;  // bits per half
};

__device__ __forceinline__ uint64_t feistel(uint64_t v, const FeistelKey& fk) {
    const uint64_t mask = (1ull << fk.h) - 1ull;
    uint64_t L = v >> fk.h, R = v & mask;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint64_t t = L ^ (mix64(R + fk.k[r]) & mask);
        L = R;
        R = t;
    }
    return (L << fk.h) | R;
}

__global__ void k_permute_ids(const int32_t* __restrict__ in, int64_t n, FeistelKey fk,
                              int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t v = feistel((uint64_t)i, fk);
    while (v >= (uint64_t)n) v = feistel(v, fk);
    out[i] = in[v];
}

unsigned blocks(int64_t n, int per) {
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > (1 << 20)) b = 1 << 20;
    return (unsigned)b;
}

} // namespace
} // namespace cvib


// ---------------------------------------------------------------------------
// The network object.

struct cv_mlp {
    cv_context* ctx = nullptr;
    int device = 0;
    int32_t L = 0;                      // layers
    int32_t dims[cvib::kMaxLayers + 1] = {};
    int32_t dpad[cvib::kMaxLayers + 1] = {};  // d_l rounded up to 32 (l >= 1)
    float omega0 = 0.0f;                // > 0: first hidden layer sin(omega0 z), else ReLU
    int64_t woff[cvib::kMaxLayers] = {}, boff[cvib::kMaxLayers] = {};
    int64_t nparam = 0;
    float* params = nullptr;  // FP32 master weights, per layer W_l [d_{l+1}][d_l] then b_l
    float* grads = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    bf16* wb[cvib::kMaxLayers] = {};    // BF16 W_l, l >= 1, [dpad_{l+1}][d_l]
    bf16* wpf[cvib::kMaxLayers] = {};   // W_l packed for the fused training step (frag_off), l >= 1, when d_l % 32 == 0:
    bf16* wpb[cvib::kMaxLayers] = {};   //   forward [dpad_{l+1}][d_l] and backward (transposed) [d_l][dpad_{l+1}]
    int64_t bcap = 0;                   // rows of the activation buffers
    bf16* h[cvib::kMaxLayers] = {};     // post-ReLU H_l, l = 1..L-1, [bcap][d_l]
    bf16* g[2] = {nullptr, nullptr};    // back-propagated gradients [bcap][gw]
    int32_t gw = 0;                     // widest padded layer
    // k-contiguous copies for the weight-gradient products, rows of length ldt
    // (the kept batch rounded up to 8; allocated for the batch rounded up to a whole block of the fused step): H_l transposed [d_l][ldt] and the
    // back-propagated gradients transposed [gw][ldt]
    bf16* ht[cvib::kMaxLayers] = {};
    bf16* gt[3] = {nullptr, nullptr, nullptr};
    int64_t ldt = 0;
    float* dsin = nullptr;              // sinusoidal first layer: omega0 cos(omega0 z) [bcap][d1]
    float* part = nullptr;              // split partials
    size_t part_bytes = 0;
    float* lpart = nullptr;             // loss partials
    int64_t lpart_n = 0;
    int64_t fwd_rows = -1;              // batch of the last kept forward
    // training-step buffers (cv_mlp_train_steps)
    int64_t tcap = 0;
    float* tx = nullptr;    // [tcap][3]
    float* ttr = nullptr;   // [tcap][36]
    float* ttf = nullptr;   // [tcap]
    float* tout = nullptr;  // [tcap][37]
    float* tloss = nullptr; // [1]: loss of a step that is not logged
    float* fpart = nullptr;  // fused training step: per-block bias, input-layer and loss partials
    size_t fpart_bytes = 0;
};

namespace cvib {
namespace {

int grow(void** p, size_t* have, size_t want) {
    if (*have >= want) return CV_OK;
    if (*p) CV_HIP(hipFree(*p));
    *p = nullptr;
    *have = 0;
    hipError_t e = hipMalloc(p, want);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(e, "hipMalloc(network workspace)");
    }
    *have = want;
    return CV_OK;
}

// Activation and gradient buffers for `rows` rows.
int ensure_rows(cv_mlp* m, int64_t rows) {
    if (rows <= m->bcap) return CV_OK;
    CV_HIP(hipDeviceSynchronize());
    for (int l = 1; l < m->L; ++l) {
        if (m->h[l]) CV_HIP(hipFree(m->h[l]));
        m->h[l] = nullptr;
    }
    for (bf16*& q : m->g) {
        if (q) CV_HIP(hipFree(q));
        q = nullptr;
    }
    for (int l = 1; l < m->L; ++l) {
        if (m->ht[l]) CV_HIP(hipFree(m->ht[l]));
        m->ht[l] = nullptr;
    }
    for (bf16*& q : m->gt) {
        if (q) CV_HIP(hipFree(q));
        q = nullptr;
    }
    if (m->dsin) CV_HIP(hipFree(m->dsin));
    m->dsin = nullptr;
    m->bcap = 0;
    // transposed rows: the batch rounded up to whole blocks of the fused step
    const size_t rt = (size_t)((rows + kTrainRows - 1) / kTrainRows * kTrainRows);
    for (int l = 1; l < m->L; ++l) {
        CV_HIP(hipMalloc((void**)&m->h[l], (size_t)rows * m->dims[l] * sizeof(bf16)));
        CV_HIP(hipMalloc((void**)&m->ht[l], rt * m->dims[l] * sizeof(bf16)));
    }
    for (bf16*& q : m->g) CV_HIP(hipMalloc((void**)&q, (size_t)rows * m->gw * sizeof(bf16)));
    for (bf16*& q : m->gt) CV_HIP(hipMalloc((void**)&q, rt * m->gw * sizeof(bf16)));
    CV_HIP(hipMalloc((void**)&m->dsin, (size_t)rows * m->dims[1] * sizeof(float)));
    m->bcap = rows;
    return CV_OK;
}

int ensure_part(cv_mlp* m, size_t bytes) {
    return grow((void**)&m->part, &m->part_bytes, bytes);
}

// dst [cols][ldd] = src [rows][lds] transposed, through 64 x 64 LDS tiles:
// rows read and written 16 bytes per thread (lds, ldd and cols multiples of 8).
__global__ __launch_bounds__(256) void k_transpose_bf16(const bf16* __restrict__ src, int64_t rows, int32_t cols,
                                                        int64_t lds, bf16* __restrict__ dst, int64_t ldd) {
    __shared__ bf16 t[64][72];
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int32_t c0 = (int32_t)blockIdx.y * 64;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int u = threadIdx.x + 256 * q, r = u >> 3, c = (u & 7) * 8;
        bf16x8 v = bf16x8{};
        if (r0 + r < rows && c0 + c < cols) v = *reinterpret_cast<const bf16x8*>(src + (r0 + r) * lds + c0 + c);
        *reinterpret_cast<bf16x8*>(&t[r][c]) = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int u = threadIdx.x + 256 * q, c = u >> 3, r = (u & 7) * 8;  // dst row c, columns r .. r + 7
        if (c0 + c >= cols || r0 + r >= rows) continue;
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = t[r + e][c];
        bf16* d = dst + (int64_t)(c0 + c) * ldd + r0 + r;
        if (r0 + r + 8 <= rows) {
            *reinterpret_cast<bf16x8*>(d) = v;
        } else {
            for (int e = 0; e < 8 && r0 + r + e < rows; ++e) d[e] = v[e];
        }
    }
}

int transpose_bf16(const bf16* src, int64_t rows, int32_t cols, int64_t lds, bf16* dst, int64_t ldd,
                   hipStream_t s) {
    if (rows == 0) return CV_OK;
    if (lds % 8 || ldd % 8 || cols % 8) return fail(CV_ESTATE, "internal: transpose alignment");
    hipLaunchKernelGGL(k_transpose_bf16, dim3((unsigned)((rows + 63) / 64), (unsigned)((cols + 63) / 64)),
                       dim3(256), 0, s, src, rows, cols, lds, dst, ldd);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

int refresh_bf16(cv_mlp* m, hipStream_t s) {
    for (int l = 1; l < m->L; ++l) {
        const int64_t n = (int64_t)m->dpad[l + 1] * m->dims[l];
        hipLaunchKernelGGL(k_weights_bf16, dim3(blocks(n, 256)), dim3(256), 0, s,
                           m->params + m->woff[l], m->dims[l + 1], m->dpad[l + 1], m->dims[l], m->wb[l]);
        if (m->dims[l] % 32 == 0)
            hipLaunchKernelGGL(k_weights_packed, dim3(blocks(n, 256)), dim3(256), 0, s, m->params + m->woff[l],
                               m->dims[l + 1], m->dpad[l + 1], m->dims[l], m->wpf[l], m->wpb[l]);
    }
    CV_HIP(hipGetLastError());
    return CV_OK;
}

// Hidden layers and the output layer for rows already in H_1.
int forward_tail(cv_mlp* m, bf16* const* H, bf16* const* Ht, int64_t ldt, int64_t rows, float* out,
                 hipStream_t s) {
    int rc;
    for (int l = 1; l < m->L; ++l) {
        GemmArgs a = {};
        a.A = H[l];
        a.lda = m->dims[l];
        a.B = m->wb[l];
        a.ldb = m->dims[l];
        a.M = (int32_t)rows;
        a.N = m->dpad[l + 1];
        a.K = m->dims[l];
        a.kchunk = pad32(a.K);
        a.bias = m->params + m->boff[l];
        a.nstore = m->dims[l + 1];
        if (l + 1 < m->L) {
            a.cb = H[l + 1];
            a.ldc = m->dims[l + 1];
            a.cbt = Ht ? Ht[l + 1] : nullptr;
            a.ldct = ldt;
            rc = gemm<true, true, EPI_RELU_BF16>(a, 1, s);
        } else {
            a.cf = out;
            a.ldc = m->dims[m->L];
            rc = gemm<true, true, EPI_BIAS_F32>(a, 1, s);
        }
        if (rc != CV_OK) return rc;
    }
    return CV_OK;
}

// Whether the fused inference kernel takes this network.
bool fused_shape(const cv_mlp* m) {
    return m->L == 4 && m->dims[0] <= kMaxIn && m->dims[1] == kFusedWidth && m->dims[2] == kFusedWidth &&
           m->dims[3] == kFusedWidth && m->dpad[4] == 64;  // 33 to 64 outputs
}

// Forward pass.  keep: the activations of all rows stay for a backward pass;
// otherwise rows go through in chunks that reuse the buffers (or, for 8-bit
// colours and the surrogate's shape, through the fused kernel).
int run_forward(cv_mlp* m, const void* x, bool rgb8, int64_t rows, float* out, bool keep,
                hipStream_t s) {
    int rc;
    if (rgb8 && !keep && fused_shape(m)) {
        if (rows == 0) return CV_OK;
        const bf16* W3 = m->wpf[3];  // 64 rows, zero beyond dims[4]
        hipLaunchKernelGGL(k_mlp_infer_fused, dim3((unsigned)((rows + kFusedRows - 1) / kFusedRows)), dim3(512),
                           0, s, (const uint8_t*)x, rows, m->dims[0], m->dims[4], m->params + m->woff[0],
                           m->params + m->boff[0], m->omega0, m->wpf[1], m->params + m->boff[1], m->wpf[2],
                           m->params + m->boff[2], W3, m->params + m->boff[3], out);
        CV_HIP(hipGetLastError());
        m->fwd_rows = -1;
        return CV_OK;
    }
    const int64_t chunk = keep ? rows : std::min(rows, kInferChunk);
    if ((rc = ensure_rows(m, chunk)) != CV_OK) return rc;
    for (int64_t r0 = 0; r0 < rows; r0 += chunk) {
        const int64_t nr = std::min(chunk, rows - r0);
        const void* xs = rgb8 ? (const void*)((const uint8_t*)x + r0 * 3)
                              : (const void*)((const float*)x + r0 * m->dims[0]);
        const unsigned ib = blocks(nr * (m->dims[1] / 8), 256);
        // a kept pass also writes what the weight-gradient products read:
        // the activations transposed and the sine's derivative
        float* ds = keep ? m->dsin : nullptr;
        const int64_t ldt = (nr + 7) / 8 * 8;
        if (rgb8)
            hipLaunchKernelGGL(k_input_layer<true>, dim3(ib), dim3(256), 0, s, xs, nr, m->dims[0],
                               m->dims[1], m->params + m->woff[0], m->params + m->boff[0], m->omega0, m->h[1],
                               ds);
        else
            hipLaunchKernelGGL(k_input_layer<false>, dim3(ib), dim3(256), 0, s, xs, nr, m->dims[0],
                               m->dims[1], m->params + m->woff[0], m->params + m->boff[0], m->omega0, m->h[1],
                               ds);
        CV_HIP(hipGetLastError());
        if (keep && (rc = transpose_bf16(m->h[1], nr, m->dims[1], m->dims[1], m->ht[1], ldt, s)) != CV_OK)
            return rc;
        if ((rc = forward_tail(m, m->h, keep ? m->ht : nullptr, ldt, nr, out + r0 * m->dims[m->L], s)) != CV_OK)
            return rc;
    }
    m->fwd_rows = keep ? rows : -1;
    m->ldt = keep ? (rows + 7) / 8 * 8 : 0;
    return CV_OK;
}

// gout: FP32 [B][dims_L]; or nullptr when run_loss has already put the BF16
// gradient in g[0].  The weight gradients take k-contiguous operands: the
// kept activations transposed (forward pass) and the back-propagated
// gradients transposed (each layer's epilogue writes both layouts); the
// blocks of a weight-gradient product's first column tile also sum the
// gradient over their rows, which gives the bias gradient's split partials.
int run_backward(cv_mlp* m, const float* x, const float* gout, int64_t B, hipStream_t s) {
    int rc;
    const int32_t L = m->L;
    const int64_t ldt = m->ldt;
    if (ldt < B) return fail(CV_ESTATE, "internal: no transposed activations for this batch");
    const int32_t splits = (int32_t)((B + kSplitRows - 1) / kSplitRows);
    const int32_t csplits = (int32_t)((B + kColRows - 1) / kColRows);  // input layer column reductions
    // partials: a layer's weight partials followed by its bias partials
    size_t need = (size_t)csplits * m->dpad[1] * (m->dims[0] + 1);
    for (int l = 1; l < L; ++l)
        need = std::max(need, (size_t)splits * m->dpad[l + 1] * (m->dims[l] + 1));
    if ((rc = ensure_part(m, need * sizeof(float))) != CV_OK) return rc;
    bf16* Gc = m->g[0];  // gradient w.r.t. the pre-activations of layer l's output
    bf16* Gn = m->g[1];
    bf16* Gct = m->gt[0];  // the same, transposed [dpad][ldt]
    bf16* Gnt = m->gt[1];
    if (gout) {
        hipLaunchKernelGGL(k_grad_to_bf16, dim3(blocks(B * m->dpad[L], 256)), dim3(256), 0, s, gout, B,
                           m->dims[L], m->dpad[L], Gc);
        CV_HIP(hipGetLastError());
    }
    if ((rc = transpose_bf16(Gc, B, m->dpad[L], m->dpad[L], Gct, ldt, s)) != CV_OK) return rc;
    int32_t ldg = m->dpad[L];
    for (int l = L - 1; l >= 1; --l) {
        const int32_t dout = m->dims[l + 1], dop = m->dpad[l + 1], din = m->dims[l];
        // weight gradient: dW_l[o][i] = sum_s G[s][o] H_l[s][i], from G^T and H_l^T
        float* pb = m->part + (size_t)splits * dop * din;
        GemmArgs a = {};
        a.A = Gct;
        a.lda = ldt;
        a.B = m->ht[l];
        a.ldb = ldt;
        a.M = dop;
        a.N = din;
        a.K = (int32_t)B;
        a.kchunk = (int32_t)kSplitRows;
        a.cf = m->part;
        a.ldc = din;
        a.zstride = (int64_t)dop * din;
        a.nstore = din;
        a.bpart = pb;
        if ((rc = gemm<true, true, EPI_PARTIAL_F32>(a, splits, s)) != CV_OK) return rc;
        hipLaunchKernelGGL(k_sum_grads, dim3(blocks((int64_t)dout * din + dout, 256)), dim3(256), 0, s,
                           m->part, splits, (int64_t)dop * din, dout, din, (int64_t)din, m->grads + m->woff[l],
                           pb, splits, (int64_t)dop, m->grads + m->boff[l]);
        CV_HIP(hipGetLastError());
        // input gradient through W_l and the ReLU of H_l (or the sine's derivative)
        GemmArgs d = {};
        d.A = Gc;
        d.lda = ldg;
        d.B = m->wb[l];
        d.ldb = din;
        d.M = (int32_t)B;
        d.N = din;
        d.K = dop;
        d.kchunk = dop;
        d.cb = Gn;
        d.ldc = din;
        d.cbt = l > 1 ? Gnt : nullptr;  // the input layer's gradient is reduced on the vector ALUs
        d.ldct = ldt;
        d.mask = m->h[l];
        d.ldm = din;
        d.nstore = din;
        if (l == 1 && m->omega0 > 0.0f) {
            d.dsin = m->dsin;
            d.ldd = din;
            d.omega0 = m->omega0;
            rc = gemm<true, false, EPI_SINE_BF16>(d, 1, s);
        } else {
            rc = gemm<true, false, EPI_MASK_BF16>(d, 1, s);
        }
        if (rc != CV_OK) return rc;
        std::swap(Gc, Gn);
        std::swap(Gct, Gnt);
        ldg = din;
    }
    // input layer
    const int32_t d0 = m->dims[0], d1 = m->dims[1];
    hipLaunchKernelGGL(k_colgrad, dim3((unsigned)((d1 + 63) / 64), (unsigned)csplits), dim3(256), 0, s,
                       Gc, (int64_t)ldg, x, d0, B, d1, m->part);
    hipLaunchKernelGGL(k_input_grad_sum, dim3(blocks((int64_t)d1 * (d0 + 1), 256)), dim3(256), 0, s,
                       m->part, csplits, d0, d1, m->grads + m->woff[0], m->grads + m->boff[0]);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

// gb (nullable): the BF16 output gradient [B][dpad_L] for run_backward's
// first operand, written in the same pass.
int run_loss(cv_mlp* m, const float* out, const float* tr, const float* tf, int64_t B, float delta,
             float* loss, float* gout, bf16* gb, hipStream_t s) {
    const int64_t nb = (B + kLossRows - 1) / kLossRows;
    int rc;
    size_t have = (size_t)m->lpart_n * sizeof(float);
    if ((rc = grow((void**)&m->lpart, &have, (size_t)nb * sizeof(float))) != CV_OK) return rc;
    m->lpart_n = (int64_t)(have / sizeof(float));
    hipLaunchKernelGGL(k_loss, dim3((unsigned)nb), dim3(256), 0, s, out, tr, tf, B, m->dims[m->L], delta,
                       gout, gb, m->dpad[m->L], m->lpart);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, s, m->lpart, (int32_t)nb, B, loss);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

int run_adam(cv_mlp* m, float lr, float b1, float b2, float eps, int64_t t, hipStream_t s) {
    const float c1 = (float)(1.0 / (1.0 - pow((double)b1, (double)t)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)b2, (double)t)));
    BF16Copies cp;
    for (int l = 1; l < m->L; ++l) {
        cp.off[cp.n] = m->woff[l];
        cp.cnt[cp.n] = (int64_t)m->dims[l + 1] * m->dims[l];
        cp.dst[cp.n] = m->wb[l];
        if (m->dims[l] % 32 == 0) {
            cp.pf[cp.n] = m->wpf[l];
            cp.pb[cp.n] = m->wpb[l];
            cp.din[cp.n] = m->dims[l];
            cp.dp[cp.n] = m->dpad[l + 1];
        }
        ++cp.n;
    }
    hipLaunchKernelGGL(k_adam, dim3(blocks(m->nparam, 256)), dim3(256), 0, s, m->params, m->grads,
                       m->adam_m, m->adam_v, m->nparam, lr, b1, b2, eps, c1, c2, cp);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

int ensure_train(cv_mlp* m, int64_t B) {
    if (B <= m->tcap) return CV_OK;
    CV_HIP(hipDeviceSynchronize());
    float** bufs[] = {&m->tx, &m->ttr, &m->ttf, &m->tout};
    for (float** b : bufs) {
        if (*b) CV_HIP(hipFree(*b));
        *b = nullptr;
    }
    m->tcap = 0;
    CV_HIP(hipMalloc((void**)&m->tx, (size_t)B * 3 * sizeof(float)));
    CV_HIP(hipMalloc((void**)&m->ttr, (size_t)B * 36 * sizeof(float)));
    CV_HIP(hipMalloc((void**)&m->ttf, (size_t)B * sizeof(float)));
    CV_HIP(hipMalloc((void**)&m->tout, (size_t)B * 37 * sizeof(float)));
    if (!m->tloss) CV_HIP(hipMalloc((void**)&m->tloss, sizeof(float)));
    m->tcap = B;
    return CV_OK;
}

// One training step of the surrogate's shape through the fused kernels (see
// k_train_forward): nb rows of colour ids, loss of the step to *loss.
int train_step_fused(cv_mlp* m, const int32_t* ids, int64_t nb, const cv_table_row* table, double dr,
                     float delta, float lr, int64_t t, float* loss, hipStream_t s) {
    int rc;
    // transposed rows padded to whole blocks (k_train_step writes every row of a block)
    const int64_t ldt = (nb + kTrainRows - 1) / kTrainRows * kTrainRows;
    if (nb > m->bcap) return fail(CV_ESTATE, "internal: training buffers smaller than the batch");
    const int32_t nblk = (int32_t)((nb + kTrainRows - 1) / kTrainRows);
    const int32_t splits = (int32_t)((nb + kSplitRows - 1) / kSplitRows);
    // weight partials of the three matrix-core layers side by side
    const int64_t zw3 = (int64_t)m->dpad[4] * m->dims[3], zw2 = (int64_t)m->dpad[3] * m->dims[2],
                  zw1 = (int64_t)m->dpad[2] * m->dims[1];
    if ((rc = ensure_part(m, (size_t)splits * (zw3 + zw2 + zw1) * sizeof(float))) != CV_OK) return rc;
    const size_t per_blk = 64 + 256 + 256 + 256 * 4 + 1;
    if ((rc = grow((void**)&m->fpart, &m->fpart_bytes, (size_t)nblk * per_blk * sizeof(float))) != CV_OK) return rc;
    float* pw3 = m->part;
    float* pw2 = pw3 + (size_t)splits * zw3;
    float* pw1 = pw2 + (size_t)splits * zw2;
    float* pb3 = m->fpart;
    float* pb2 = pb3 + (size_t)nblk * 64;
    float* pb1 = pb2 + (size_t)nblk * 256;
    float* p0 = pb1 + (size_t)nblk * 256;
    float* lp = p0 + (size_t)nblk * 256 * 4;
    TrainArgs f;
    f.ids = ids;
    f.table = table;
    f.rscale = (float)(dr / 50.0);
    f.B = nb;
    f.omega0 = m->omega0;
    f.delta = delta;
    f.W0 = m->params + m->woff[0];
    f.b0 = m->params + m->boff[0];
    f.W1 = m->wpf[1];
    f.b1 = m->params + m->boff[1];
    f.W2 = m->wpf[2];
    f.b2 = m->params + m->boff[2];
    f.W3 = m->wpf[3];
    f.b3 = m->params + m->boff[3];
    f.W3t = m->wpb[3];
    f.W2t = m->wpb[2];
    f.W1t = m->wpb[1];
    f.ldt = ldt;
    f.h1t = m->ht[1];
    f.h2t = m->ht[2];
    f.h3t = m->ht[3];
    f.goutt = m->gt[0];
    f.g3t = m->gt[1];
    f.g2t = m->gt[2];
    f.lpart = lp;
    f.pb3 = pb3;
    f.pb2 = pb2;
    f.pb1 = pb1;
    f.p0 = p0;
    hipLaunchKernelGGL(k_train_step, dim3((unsigned)nblk), dim3(kTThreads), 0, s, f);
    CV_HIP(hipGetLastError());
    // weight gradients dW_l[o][i] = sum_s G[s][o] H_l[s][i] from the transposed operands
    const bf16* As[4] = {nullptr, m->gt[2], m->gt[1], m->gt[0]};
    float* Ps[4] = {nullptr, pw1, pw2, pw3};
    GemmArgs wg[3] = {};
    for (int l = 1; l <= 3; ++l) {
        GemmArgs& a = wg[l - 1];
        a.A = As[l];
        a.lda = ldt;
        a.B = m->ht[l];
        a.ldb = ldt;
        a.M = m->dpad[l + 1];
        a.N = m->dims[l];
        a.K = (int32_t)nb;
        a.kchunk = kSplitRows;
        a.cf = Ps[l];
        a.ldc = m->dims[l];
        a.zstride = (int64_t)m->dpad[l + 1] * m->dims[l];
        a.nstore = m->dims[l];
    }
    SumAdamArgs d;
    d.p = m->params;
    d.g = m->grads;
    d.m = m->adam_m;
    d.v = m->adam_v;
    d.lr = lr;
    d.b1 = 0.9f;
    d.b2 = 0.999f;
    d.eps = 1e-8f;
    d.c1 = (float)(1.0 / (1.0 - pow(0.9, (double)t)));
    d.c2 = (float)(1.0 / (1.0 - pow(0.999, (double)t)));
    for (int l = 0; l < 4; ++l) {
        d.woff[l] = m->woff[l];
        d.boff[l] = m->boff[l];
        d.din[l] = m->dims[l];
        d.dout[l] = m->dims[l + 1];
        d.dpad[l] = m->dpad[l + 1];
        d.wpart[l] = Ps[l];
        d.wb[l] = m->wb[l];
        d.wpf[l] = m->wpf[l];
        d.wpb[l] = m->wpb[l];
    }
    d.wsplits = splits;
    d.bpart[0] = nullptr;
    d.bpart[1] = pb1;
    d.bpart[2] = pb2;
    d.bpart[3] = pb3;
    d.bw[0] = 0;
    d.bw[1] = 256;
    d.bw[2] = 256;
    d.bw[3] = 64;
    d.p0 = p0;
    d.nblk = nblk;
    d.nlong = m->dims[1] * m->dims[0] + m->dims[1] + m->dims[2] + m->dims[3] + m->dims[4];
    d.lpart = lp;
    d.loss = loss;
    d.B = nb;
    // four weights per thread: every layer's weights start and end on a multiple of 4
    for (int l = 1; l <= 3; ++l)
        if (m->woff[l] % 4 != 0 || (m->boff[l] - m->woff[l]) % 4 != 0 || m->dims[l] % 4 != 0)
            return fail(CV_ESTATE, "internal: weight blocks not in fours");
    if ((rc = gemm_wgrad3(wg, splits, d, (d.nlong + 31) / 32 * 8, s)) != CV_OK) return rc;
    hipLaunchKernelGGL(k_sum_adam, dim3((unsigned)blocks((m->boff[3] - m->woff[1] + 3) / 4, 256)), dim3(256), 0, s,
                       d);
    CV_HIP(hipGetLastError());
    return CV_OK;
}

void free_mlp(cv_mlp* m) {
    void* ps[] = {m->params, m->grads, m->adam_m, m->adam_v, m->g[0], m->g[1], m->part, m->lpart,
                  m->tx, m->ttr, m->ttf, m->tout, m->tloss, m->fpart};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    for (int l = 0; l < kMaxLayers; ++l) {
        if (m->wb[l]) (void)hipFree(m->wb[l]);
        if (m->wpf[l]) (void)hipFree(m->wpf[l]);
        if (m->wpb[l]) (void)hipFree(m->wpb[l]);
        if (m->h[l]) (void)hipFree(m->h[l]);
        if (m->ht[l]) (void)hipFree(m->ht[l]);
    }
    for (bf16* q : m->gt)
        if (q) (void)hipFree(q);
    if (m->dsin) (void)hipFree(m->dsin);
    delete m;
}

// File tags: version 02 adds the first layer's omega0 (a float after the
// parameter count); a version 01 file is a ReLU network (omega0 = 0).
const char kMagic[8] = {'C', 'V', 'M', 'L', 'P', '0', '2', '\0'};
const char kMagic01[8] = {'C', 'V', 'M', 'L', 'P', '0', '1', '\0'};
// Training checkpoint: parameters, both Adam moments, the step count and the
// caller's training-order key, followed by a 64-bit FNV-1a hash of every byte
// before it.
const char kMagicCkpt[8] = {'C', 'V', 'C', 'K', 'P', '0', '1', '\0'};

uint64_t fnv1a64(const void* p, size_t n, uint64_t h = 0xCBF29CE484222325ull) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t k = 0; k < n; ++k) {
        h ^= c[k];
        h *= 0x100000001B3ull;
    }
    return h;
}

// A checkpoint file read into host memory and checked: magic, shape fields
// consistent with the byte count, finite omega0 and the content hash.
struct Checkpoint {
    int32_t L = 0;
    int32_t dims[kMaxLayers + 1] = {};
    int64_t n = 0;
    float omega0 = 0.0f;
    int64_t step = 0;
    uint64_t key = 0;
    std::string params, mom1, mom2;  // n floats each
};

int read_checkpoint(const char* path, Checkpoint& ck) {
    FILE* f = fopen(path, "rb");
    if (!f) return fail(CV_EINVAL, std::string("cannot open ") + path);
    std::string all;
    char chunk[1 << 16];
    size_t got;
    while ((got = fread(chunk, 1, sizeof chunk, f)) > 0) all.append(chunk, got);
    fclose(f);
    const std::string bad = std::string("not a valid network checkpoint: ") + path;
    size_t o = 0;
    auto take = [&](void* dst, size_t b) {
        if (o + b > all.size()) return false;
        std::memcpy(dst, all.data() + o, b);
        o += b;
        return true;
    };
    char magic[8];
    if (!take(magic, 8) || std::memcmp(magic, kMagicCkpt, 8) != 0) return fail(CV_EINVAL, bad + " (magic)");
    if (!take(&ck.L, 4) || ck.L < 1 || ck.L > kMaxLayers) return fail(CV_EINVAL, bad + " (layers)");
    if (!take(ck.dims, 4 * ((size_t)ck.L + 1))) return fail(CV_EINVAL, bad + " (dims)");
    int64_t want = 0;
    for (int l = 0; l < ck.L; ++l) {
        if (ck.dims[l] < 1 || ck.dims[l + 1] < 1 || ck.dims[l] > 4096 || ck.dims[l + 1] > 4096)
            return fail(CV_EINVAL, bad + " (dims)");
        want += (int64_t)ck.dims[l] * ck.dims[l + 1] + ck.dims[l + 1];
    }
    if (!take(&ck.n, 8) || ck.n != want) return fail(CV_EINVAL, bad + " (parameter count)");
    if (!take(&ck.omega0, 4) || !std::isfinite(ck.omega0) || ck.omega0 < 0.0f)
        return fail(CV_EINVAL, bad + " (omega0)");
    if (!take(&ck.step, 8) || ck.step < 0) return fail(CV_EINVAL, bad + " (step)");
    if (!take(&ck.key, 8)) return fail(CV_EINVAL, bad + " (key)");
    const size_t pb = (size_t)ck.n * sizeof(float);
    if (all.size() != o + 3 * pb + 8) return fail(CV_EINVAL, bad + " (length)");
    uint64_t h = 0;
    std::memcpy(&h, all.data() + o + 3 * pb, 8);
    if (h != fnv1a64(all.data(), o + 3 * pb)) return fail(CV_EINVAL, bad + " (content hash)");
    ck.params.assign(all.data() + o, pb);
    ck.mom1.assign(all.data() + o + pb, pb);
    ck.mom2.assign(all.data() + o + 2 * pb, pb);
    return CV_OK;
}

} // namespace

// BF16 activations widened to FP32 (cv_mlp_hidden).
__global__ void k_bf16_to_f32(const bf16* __restrict__ in, float* __restrict__ out, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = (float)in[k];
}

int mlp_forward_rgb8(cv_mlp* m, const uint8_t* rgb, int64_t n, float* out, hipStream_t s) {
    return run_forward(m, rgb, true, n, out, false, s);
}
int mlp_out_width(const cv_mlp* m) { return m->dims[m->L]; }
int mlp_in_width(const cv_mlp* m) { return m->dims[0]; }
int mlp_device(const cv_mlp* m) { return m->device; }

} // namespace cvib

using cvib::DeviceGuard;
using cvib::fail;

extern "C" {

int cv_mlp_create(cv_context* ctx, const int32_t* dims, int32_t nlayers, cv_mlp** out) {
    CV_GUARD_BEGIN
    if (!ctx || !dims || !out) return fail(CV_EINVAL, "null argument");
    *out = nullptr;
    if (nlayers < 2 || nlayers > cvib::kMaxLayers)
        return fail(CV_EINVAL, "nlayers must be in [2, " + std::to_string(cvib::kMaxLayers) + "]");
    if (dims[0] < 1 || dims[0] > cvib::kMaxIn) return fail(CV_EINVAL, "dims[0] must be in [1, 4]");
    if (dims[0] != 3) return fail(CV_EINVAL, "dims[0] must be 3 (an RGB colour)");
    for (int l = 1; l < nlayers; ++l)
        if (dims[l] < 32 || dims[l] > cvib::kMaxHidden || dims[l] % 32 != 0)
            return fail(CV_EINVAL, "hidden widths must be multiples of 32 in [32, 1024]");
    if (dims[nlayers] < 2 || dims[nlayers] > cvib::kMaxOut)
        return fail(CV_EINVAL, "output width must be in [2, 256]");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(CV_EHIP, "hipSetDevice failed");
    cv_mlp* m = new cv_mlp();
    m->ctx = ctx;
    m->device = ctx->device;
    m->L = nlayers;
    int64_t off = 0;
    for (int l = 0; l <= nlayers; ++l) {
        m->dims[l] = dims[l];
        m->dpad[l] = l == 0 ? dims[0] : cvib::pad32(dims[l]);
        m->gw = std::max(m->gw, m->dpad[l]);
    }
    for (int l = 0; l < nlayers; ++l) {
        m->woff[l] = off;
        off += (int64_t)dims[l + 1] * dims[l];
        m->boff[l] = off;
        off += dims[l + 1];
    }
    m->nparam = off;
    const size_t pb = (size_t)off * sizeof(float);
    hipError_t e = hipSuccess;
    float** arrs[] = {&m->params, &m->grads, &m->adam_m, &m->adam_v};
    for (float** a : arrs)
        if (e == hipSuccess) e = hipMalloc((void**)a, pb);
    for (int l = 1; l < nlayers && e == hipSuccess; ++l) {
        e = hipMalloc((void**)&m->wb[l], (size_t)m->dpad[l + 1] * dims[l] * sizeof(bf16));
        if (e == hipSuccess) e = hipMalloc((void**)&m->wpf[l], (size_t)m->dpad[l + 1] * dims[l] * sizeof(bf16));
        if (e == hipSuccess) e = hipMalloc((void**)&m->wpb[l], (size_t)m->dpad[l + 1] * dims[l] * sizeof(bf16));
    }
    for (float** a : arrs)
        if (e == hipSuccess) e = hipMemset(*a, 0, pb);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        cvib::free_mlp(m);
        return cvib::hip_fail(e, "network allocation");
    }
    int rc = cvib::refresh_bf16(m, nullptr);
    if (rc == CV_OK) rc = (hipDeviceSynchronize() == hipSuccess) ? CV_OK : fail(CV_EHIP, "sync");
    if (rc != CV_OK) {
        cvib::free_mlp(m);
        return rc;
    }
    *out = m;
    return CV_OK;
    CV_GUARD_END
}

int cv_mlp_destroy(cv_mlp* m) {
    CV_GUARD_BEGIN
    if (!m) return CV_OK;
    DeviceGuard dg(m->device);
    (void)hipDeviceSynchronize();
    cvib::free_mlp(m);
    return CV_OK;
    CV_GUARD_END
}

int cv_mlp_set_first_sine(cv_mlp* m, float omega0) {
    CV_GUARD_BEGIN
    if (!m) return fail(CV_EINVAL, "null network");
    if (!std::isfinite(omega0) || omega0 < 0.0f) return fail(CV_EINVAL, "omega0 must be finite and >= 0");
    m->omega0 = omega0;
    return CV_OK;
    CV_GUARD_END
}

int cv_mlp_first_sine(const cv_mlp* m, float* omega0_host) {
    CV_GUARD_BEGIN
    if (!m || !omega0_host) return fail(CV_EINVAL, "null argument");
    *omega0_host = m->omega0;
    return CV_OK;
    CV_GUARD_END
}

int cv_mlp_num_params(const cv_mlp* m, int64_t* n_host) {
    CV_GUARD_BEGIN
    if (!m || !n_host) return fail(CV_EINVAL, "null argument");
    *n_host = m->nparam;
    return CV_OK;
    CV_GUARD_END
}

int cv_mlp_set_params(cv_mlp* m, const float* params, void* stream) {
    CV_GUARD_BEGIN
    if (!m || !params) return fail(CV_EINVAL, "null argument");
    DeviceGuard dg(m->device);
    hipStream_t s = (hipStream_t)stream;
    const size_t pb = (size_t)m->nparam * sizeof(float);
    CV_HIP(hipMemcpyAsync(m->params, params, pb, hipMemcpyDeviceToDevice, s));
    CV_HIP(hipMemsetAsync(m->adam_m, 0, pb, s));
    CV_HIP(hipMemsetAsync(m->adam_v, 0, pb, s));
    return cvib::refresh_bf16(m, s);
    CV_GUARD_END
}

int cv_mlp_get_params(const cv_mlp* m, float* params, float* grads, void* stream) {
    CV_GUARD_BEGIN
    if (!m || (!params && !grads)) return fail(CV_EINVAL, "null argument");
    DeviceGuard dg(m->device);
    hipStream_t s = (hipStream_t)stream;
    const size_t pb = (size_t)m->nparam * sizeof(float);
    if (params) CV_HIP(hipMemcpyAsync(params, m->params, pb, hipMemcpyDeviceToDevice, s));
    if (grads) CV_HIP(hipMemcpyAsync(grads, m->grads, pb, hipMemcpyDeviceToDevice, s));
    return CV_OK;
    CV_GUARD_END
}

int cv_mlp_forward(cv_mlp* m, const void* x, int64_t B, float* out, uint32_t flags, void* stream) {
    CV_GUARD_BEGIN
    if (!m) return fail(CV_EINVAL, "network is NULL");
    if (B < 0) return fail(CV_EINVAL, "B < 0");
    if (flags & ~(uint32_t)(CV_MLP_KEEP | CV_MLP_RGB8)) return fail(CV_EINVAL, "unknown flags");
    if (B == 0) return CV_OK;
    if (!x || !out) return fail(CV_EINVAL, "null array");
    if (B > ((int64_t)1 << 30)) return fail(CV_EINVAL, "B > 2^30");
    if ((flags & CV_MLP_KEEP) && B > ((int64_t)1 << 24)) return fail(CV_EINVAL, "kept batch > 2^24 rows");
    DeviceGuard dg(m->device);
    return cvib::run_forward(m, x, (flags & CV_MLP_RGB8) != 0, B, out, (flags & CV_MLP_KEEP) != 0,
                             (hipStream_t)stream);
    CV_GUARD_END
}

int cv_mlp_hidden(const cv_mlp* m, int32_t layer, float* out, int64_t B, void* stream) {
    CV_GUARD_BEGIN
    if (!m) return fail(CV_EINVAL, "network is NULL");
    if (layer < 1 || layer >= m->L) return fail(CV_EINVAL, "layer must be a hidden layer (1 .. nlayers - 1)");
    if (B < 1 || B > m->fwd_rows) return fail(CV_ESTATE, "no kept forward pass of that many rows");
    if (!out) return fail(CV_EINVAL, "out is NULL");
    DeviceGuard dg(m->device);
    const int64_t nv = B * m->dims[layer];
    hipLaunchKernelGGL(cvib::k_bf16_to_f32, dim3((unsigned)std::min<int64_t>((nv + 255) / 256, 65535)), dim3(256),
                       0, (hipStream_t)stream, (const bf16*)m->h[layer], out, nv);
    CV_HIP(hipGetLastError());
    return CV_OK;
    CV_GUARD_END
}

int cv_mlp_loss(cv_mlp* m, const float* out, const float* t_r, const float* t_f, int64_t B,
                float huber_delta, float* loss, float* gout, void* stream) {
    CV_GUARD_BEGIN
    if (!m) return fail(CV_EINVAL, "network is NULL");
    if (B < 1) return fail(CV_EINVAL, "B < 1");
    if (!out || !t_r || !t_f || !loss) return fail(CV_EINVAL, "null array");
    if (!(huber_delta > 0.0f)) return fail(CV_EINVAL, "huber_delta must be > 0");
    DeviceGuard dg(m->device);
    return cvib::run_loss(m, out, t_r, t_f, B, huber_delta, loss, gout, nullptr, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_mlp_backward(cv_mlp* m, const float* x, const float* gout, int64_t B, void* stream) {
    CV_GUARD_BEGIN
    if (!m) return fail(CV_EINVAL, "network is NULL");
    if (!x || !gout) return fail(CV_EINVAL, "null array");
    if (B < 1 || B != m->fwd_rows)
        return fail(CV_ESTATE, "backward needs a kept forward pass of the same batch");
    DeviceGuard dg(m->device);
    return cvib::run_backward(m, x, gout, B, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_adam_step(cv_mlp* m, float lr, float beta1, float beta2, float eps, int64_t t, void* stream) {
    CV_GUARD_BEGIN
    if (!m) return fail(CV_EINVAL, "network is NULL");
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f) || t < 1)
        return fail(CV_EINVAL, "Adam needs lr >= 0, betas in [0, 1), eps > 0, step >= 1");
    DeviceGuard dg(m->device);
    return cvib::run_adam(m, lr, beta1, beta2, eps, t, (hipStream_t)stream);
    CV_GUARD_END
}

int cv_mlp_train_steps(cv_mlp* m, const int32_t* ids, int64_t n, const cv_table_row* table, double dr,
                       int64_t batch, float huber_delta, float lr_max, float lr_min, int64_t step0,
                       int64_t total_steps, float* loss_log, void* stream) {
    CV_GUARD_BEGIN
    if (!m) return fail(CV_EINVAL, "network is NULL");
    if (n < 1 || !ids || !table) return fail(CV_EINVAL, "no training rows");
    if (batch < 1 || batch > ((int64_t)1 << 20)) return fail(CV_EINVAL, "batch must be in [1, 2^20]");
    if (!(dr > 0.0) || !(huber_delta > 0.0f)) return fail(CV_EINVAL, "dr and huber_delta must be > 0");
    if (!(lr_max >= 0.0f) || !(lr_min >= 0.0f)) return fail(CV_EINVAL, "learning rates must be >= 0");
    if (step0 < 0 || total_steps < 1) return fail(CV_EINVAL, "step0 >= 0 and total_steps >= 1");
    if (m->dims[0] != 3 || m->dims[m->L] != 37) return fail(CV_EINVAL, "network is not 3 -> ... -> 37");
    DeviceGuard dg(m->device);
    hipStream_t s = (hipStream_t)stream;
    const int64_t B = std::min(batch, n);
    int rc;
    if ((rc = cvib::ensure_train(m, B)) != CV_OK) return rc;
    if ((rc = cvib::ensure_rows(m, B)) != CV_OK) return rc;
    const int64_t steps = (n + batch - 1) / batch;
    const bool fused = cvib::fused_shape(m) && m->dims[4] == 37;
    if (fused && (rc = cvib::refresh_bf16(m, s)) != CV_OK) return rc;  // the packed copies follow the parameters
    for (int64_t k = 0; k < steps; ++k) {
        const int64_t r0 = k * batch, nb = std::min(batch, n - r0);
        if (fused) {
            const int64_t t = step0 + k;
            const double frac =
                total_steps > 1 ? (double)std::min(t, total_steps - 1) / (double)(total_steps - 1) : 0.0;
            const float lr = (float)(lr_min + 0.5 * (lr_max - lr_min) * (1.0 + cos(M_PI * frac)));
            float* lp = loss_log ? loss_log + k : m->tloss;
            m->fwd_rows = -1;
            if ((rc = cvib::train_step_fused(m, ids + r0, nb, table, dr, huber_delta, lr, t + 1, lp, s)) != CV_OK)
                return rc;
            continue;
        }
        hipLaunchKernelGGL(cvib::k_table_batch, dim3(cvib::blocks(nb, 256)), dim3(256), 0, s, ids + r0,
                           table, nb, (float)(dr / 50.0), m->tx, m->ttr, m->ttf);
        CV_HIP(hipGetLastError());
        if ((rc = cvib::run_forward(m, m->tx, false, nb, m->tout, true, s)) != CV_OK) return rc;
        float* lp = loss_log ? loss_log + k : m->tloss;
        // the loss writes the BF16 output gradient straight into the backward pass's first operand
        if ((rc = cvib::run_loss(m, m->tout, m->ttr, m->ttf, nb, huber_delta, lp, nullptr, m->g[0], s)) != CV_OK)
            return rc;
        if ((rc = cvib::run_backward(m, m->tx, nullptr, nb, s)) != CV_OK) return rc;
        // cosine decay from lr_max to lr_min over total_steps
        const int64_t t = step0 + k;
        const double frac = total_steps > 1 ? (double)std::min(t, total_steps - 1) / (double)(total_steps - 1) : 0.0;
        const float lr = (float)(lr_min + 0.5 * (lr_max - lr_min) * (1.0 + cos(M_PI * frac)));
        if ((rc = cvib::run_adam(m, lr, 0.9f, 0.999f, 1e-8f, t + 1, s)) != CV_OK) return rc;
    }
    m->fwd_rows = -1;  // the activation buffers now hold a training step's state, not a kept forward
    return CV_OK;
    CV_GUARD_END
}

int cv_mlp_table_batch(cv_mlp* m, const int32_t* ids, const cv_table_row* table, int64_t B,
                       double dr, float* x, float* t_r, float* t_f, void* stream) {
    CV_GUARD_BEGIN
    if (!m) return fail(CV_EINVAL, "network is NULL");
    if (B < 0) return fail(CV_EINVAL, "B < 0");
    if (B == 0) return CV_OK;
    if (!ids || !table || !x || !t_r || !t_f) return fail(CV_EINVAL, "null array");
    if (!(dr > 0.0)) return fail(CV_EINVAL, "dr must be > 0");
    if (m->dims[0] != 3 || m->dims[m->L] != 37) return fail(CV_EINVAL, "network is not 3 -> ... -> 37");
    DeviceGuard dg(m->device);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(cvib::k_table_batch, dim3(cvib::blocks(B, 256)), dim3(256), 0, s, ids, table, B,
                       (float)(dr / 50.0), x, t_r, t_f);
    CV_HIP(hipGetLastError());
    return CV_OK;
    CV_GUARD_END
}

int cv_permute_ids(cv_context* ctx, const int32_t* in, int64_t n, uint64_t key, int32_t* out, void* stream) {
    CV_GUARD_BEGIN
    if (!ctx) return fail(CV_EINVAL, "context is NULL");
    if (n < 0 || n > ((int64_t)1 << 31)) return fail(CV_EINVAL, "n must be in [0, 2^31]");
    if (n == 0) return CV_OK;
    if (!in || !out) return fail(CV_EINVAL, "null array");
    if (in == out) return fail(CV_EINVAL, "in and out must not overlap");
    cvib::FeistelKey fk;
    fk.h = 1;
    while ((int64_t)1 << (2 * fk.h) < n) ++fk.h;
    for (int r = 0; r < 4; ++r) fk.k[r] = cvib::mix64(key + (uint64_t)(r + 1) * 0x9E3779B97F4A7C15ull);
    DeviceGuard dg(ctx->device);
    hipLaunchKernelGGL(cvib::k_permute_ids, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       in, n, fk, out);
    CV_HIP(hipGetLastError());
    return CV_OK;
    CV_GUARD_END
}

int cv_mlp_save(const cv_mlp* m, const char* path) {
    CV_GUARD_BEGIN
    if (!m || !path) return fail(CV_EINVAL, "null argument");
    DeviceGuard dg(m->device);
    std::string buf((size_t)m->nparam * sizeof(float), '\0');
    CV_HIP(hipDeviceSynchronize());
    CV_HIP(hipMemcpy(&buf[0], m->params, buf.size(), hipMemcpyDeviceToHost));
    FILE* f = fopen(path, "wb");
    if (!f) return fail(CV_EINVAL, std::string("cannot open ") + path);
    const int32_t L = m->L;
    const int64_t n = m->nparam;
    bool ok = fwrite(cvib::kMagic, 1, 8, f) == 8 && fwrite(&L, 4, 1, f) == 1 &&
              fwrite(m->dims, 4, (size_t)L + 1, f) == (size_t)L + 1 && fwrite(&n, 8, 1, f) == 1 &&
              fwrite(&m->omega0, 4, 1, f) == 1 && fwrite(buf.data(), 1, buf.size(), f) == buf.size();
    ok = (fclose(f) == 0) && ok;
    return ok ? CV_OK : fail(CV_EINVAL, std::string("write failed: ") + path);
    CV_GUARD_END
}

int cv_mlp_save_checkpoint(const cv_mlp* m, const char* path, int64_t step, uint64_t key) {
    CV_GUARD_BEGIN
    if (!m || !path) return fail(CV_EINVAL, "null argument");
    if (step < 0) return fail(CV_EINVAL, "step < 0");
    DeviceGuard dg(m->device);
    const size_t pb = (size_t)m->nparam * sizeof(float);
    std::string body;
    body.append(cvib::kMagicCkpt, 8);
    const int32_t L = m->L;
    body.append((const char*)&L, 4);
    body.append((const char*)m->dims, 4 * ((size_t)L + 1));
    body.append((const char*)&m->nparam, 8);
    body.append((const char*)&m->omega0, 4);
    body.append((const char*)&step, 8);
    body.append((const char*)&key, 8);
    const size_t o = body.size();
    body.resize(o + 3 * pb);
    CV_HIP(hipDeviceSynchronize());
    CV_HIP(hipMemcpy(&body[o], m->params, pb, hipMemcpyDeviceToHost));
    CV_HIP(hipMemcpy(&body[o + pb], m->adam_m, pb, hipMemcpyDeviceToHost));
    CV_HIP(hipMemcpy(&body[o + 2 * pb], m->adam_v, pb, hipMemcpyDeviceToHost));
    const uint64_t h = cvib::fnv1a64(body.data(), body.size());
    body.append((const char*)&h, 8);
    FILE* f = fopen(path, "wb");
    if (!f) return fail(CV_EINVAL, std::string("cannot open ") + path);
    bool ok = fwrite(body.data(), 1, body.size(), f) == body.size();
    ok = (fclose(f) == 0) && ok;
    return ok ? CV_OK : fail(CV_EINVAL, std::string("write failed: ") + path);
    CV_GUARD_END
}

int cv_mlp_checkpoint_info(const char* path, int32_t* nlayers, int32_t* dims, int64_t* step, uint64_t* key) {
    CV_GUARD_BEGIN
    if (!path) return fail(CV_EINVAL, "null path");
    cvib::Checkpoint ck;
    int rc = cvib::read_checkpoint(path, ck);
    if (rc != CV_OK) return rc;
    if (nlayers) *nlayers = ck.L;
    if (dims) std::memcpy(dims, ck.dims, 4 * ((size_t)ck.L + 1));
    if (step) *step = ck.step;
    if (key) *key = ck.key;
    return CV_OK;
    CV_GUARD_END
}

int cv_mlp_load_checkpoint(cv_mlp* m, const char* path, int64_t* step, uint64_t* key) {
    CV_GUARD_BEGIN
    if (!m || !path) return fail(CV_EINVAL, "null argument");
    cvib::Checkpoint ck;
    int rc = cvib::read_checkpoint(path, ck);
    if (rc != CV_OK) return rc;
    if (ck.L != m->L || std::memcmp(ck.dims, m->dims, 4 * ((size_t)m->L + 1)) != 0)
        return fail(CV_EINVAL, std::string("checkpoint of another network shape: ") + path);
    DeviceGuard dg(m->device);
    const size_t pb = (size_t)m->nparam * sizeof(float);
    CV_HIP(hipDeviceSynchronize());
    CV_HIP(hipMemcpy(m->params, ck.params.data(), pb, hipMemcpyHostToDevice));
    CV_HIP(hipMemcpy(m->adam_m, ck.mom1.data(), pb, hipMemcpyHostToDevice));
    CV_HIP(hipMemcpy(m->adam_v, ck.mom2.data(), pb, hipMemcpyHostToDevice));
    m->omega0 = ck.omega0;
    rc = cvib::refresh_bf16(m, nullptr);
    if (rc != CV_OK) return rc;
    CV_HIP(hipDeviceSynchronize());
    if (step) *step = ck.step;
    if (key) *key = ck.key;
    return CV_OK;
    CV_GUARD_END
}

int cv_mlp_load(cv_mlp* m, const char* path) {
    CV_GUARD_BEGIN
    if (!m || !path) return fail(CV_EINVAL, "null argument");
    FILE* f = fopen(path, "rb");
    if (!f) return fail(CV_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    int32_t L = 0, dims[cvib::kMaxLayers + 1];
    int64_t n = 0;
    float omega0 = 0.0f;
    bool ok = fread(magic, 1, 8, f) == 8;
    const bool v02 = ok && std::memcmp(magic, cvib::kMagic, 8) == 0;
    ok = ok && (v02 || std::memcmp(magic, cvib::kMagic01, 8) == 0) && fread(&L, 4, 1, f) == 1 &&
         L == m->L && fread(dims, 4, (size_t)L + 1, f) == (size_t)L + 1 &&
         std::memcmp(dims, m->dims, sizeof(int32_t) * ((size_t)L + 1)) == 0 && fread(&n, 8, 1, f) == 1 &&
         n == m->nparam && (!v02 || fread(&omega0, 4, 1, f) == 1) && std::isfinite(omega0) && omega0 >= 0.0f;
    std::string buf;
    if (ok) {
        buf.resize((size_t)n * sizeof(float));
        ok = fread(&buf[0], 1, buf.size(), f) == buf.size();
    }
    fclose(f);
    if (!ok) return fail(CV_EINVAL, std::string("not a network file of this shape: ") + path);
    DeviceGuard dg(m->device);
    CV_HIP(hipDeviceSynchronize());
    CV_HIP(hipMemcpy(m->params, buf.data(), buf.size(), hipMemcpyHostToDevice));
    CV_HIP(hipMemset(m->adam_m, 0, buf.size()));
    CV_HIP(hipMemset(m->adam_v, 0, buf.size()));
    m->omega0 = omega0;
    int rc = cvib::refresh_bf16(m, nullptr);
    if (rc != CV_OK) return rc;
    CV_HIP(hipDeviceSynchronize());
    return CV_OK;
    CV_GUARD_END
}

} // extern "C"
