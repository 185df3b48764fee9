// Learned move scorer: per-move features and an MLP 16 -> 64 -> 64 -> 1 (ReLU) evaluated by one wavefront
// for 64 moves at a time on the matrix cores (bfloat16 inputs, float32 accumulation).
//
// Features of a move at period t of a product (float32, in this order):
//   0-3 one-hot type (flip zM, flip zR, swap zM, swap zR); 4,5 zM(t), zR(t) of the current pattern;
//   6,7 D(t)/200, R(t)/200; 8,9 D(t-1)/200, D(t+1)/200 (0 outside the horizon); 10-13 kM/2000, kR/2000,
//   hM/8, hR/8; 14 (t - p)/T with p the last setup period <= t (1 if none); 15 (n - t)/T with n the first
//   setup period > t (T if none).
// Parameters (float32 master copy, 5313 values): W1 [16][64] row-major, b1 [64], W2 [64][64], b2 [64],
// W3 [64], b3.  The forward pass rounds weights and every layer's input to bfloat16 (nearest even); the
// products are accumulated in float32 by v_mfma_f32_16x16x32_bf16 (all three layers; the training pass
// takes layer 3 as float32 dot products).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vns_device.hpp"

namespace vns {
namespace mlp {

constexpr int kF = 16;
constexpr int kH = 64;
constexpr int kParams = 5313;
constexpr int oW1 = 0, oB1 = 1024, oW2 = 1088, oB2 = 5184, oW3 = 5248, oB3 = 5312;
constexpr int kWaveLdsBytes = 64 * kF * 2;   // feature tile of 64 moves, bfloat16
constexpr int kGradWaves = 1024;             // a gradient is the fixed-order sum of at most this many partials

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef short s2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ReLU of two float32 values rounded to bfloat16 (nearest even), packed: one v_cvt_pk_bf16_f32 and one
// v_pk_max_i16 (a negative bfloat16, -0 included, is a negative int16; rounding keeps the sign, so the
// order of rounding and ReLU does not matter).  The pair is converted as one 2-vector: converting the two
// values one by one costs two conversions and a permute.
__device__ __forceinline__ bf2 relu_pack(float a, float b) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = {a, b};
    const bf2 p = __builtin_convertvector(v, bf2);
    const s2 zero = {0, 0};
    return __builtin_bit_cast(bf2, __builtin_elementwise_max(__builtin_bit_cast(s2, p), zero));
}

// The network is evaluated transposed, H^T = W^T X^T, on v_mfma_f32_16x16x32_bf16 (lane l = 16 g + c holds
// A[c][8g..8g+7], B[8g..8g+7][c] and D[4g..4g+3][c]): with hidden units as the M dimension and moves as N,
// the D fragment of layer 1 is, unchanged, the B fragment of layer 2 once layer 2's input units are taken
// in the order pi(kt, 8g + e) = 32 kt + 16 (e / 4) + 4 g + e % 4 (D of hidden tiles 2kt and 2kt+1), so no
// activation leaves the registers.  Biases initialise the accumulators.
struct Frags {
    bf8 w1t[4];       // [hidden tile]: W1^T rows 16mt + c, features 8g..8g+7 (features >= 16 are zero)
    bf8 w2t[4][2];    // [output tile][k-slice]: W2^T rows 16mo + c, inputs pi(kt, 8g..8g+7)
    f4 b1[4];         // [hidden tile]: b1[16mt + 4g + e]
    f4 b2[4];         // [output tile]: b2[16mo + 4g + e]
    bf2 w3[4][2];     // [output tile][pair]: W3[16mo + 4g + 2pair + (0, 1)] in bfloat16
    bf8 w3a[2];       // [k-slice]: every row of layer 3's A operand is W3, inputs pi(kt, 8g..8g+7)
    float b3;
};

__device__ __forceinline__ void load_frags(const float *__restrict__ P, Frags &fr) {
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 8 * g + e;
            fr.w1t[mt][e] = k < kF ? (__bf16)P[oW1 + k * kH + 16 * mt + c] : (__bf16)0.f;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            fr.b1[mt][e] = P[oB1 + 16 * mt + 4 * g + e];
            fr.b2[mt][e] = P[oB2 + 16 * mt + 4 * g + e];
            fr.w3[mt][e >> 1][e & 1] = (__bf16)P[oW3 + 16 * mt + 4 * g + e];
        }
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int in = 32 * kt + 16 * (e >> 2) + 4 * g + (e & 3);
                fr.w2t[mt][kt][e] = (__bf16)P[oW2 + in * kH + 16 * mt + c];
            }
    }
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int e = 0; e < 8; ++e) fr.w3a[kt][e] = (__bf16)P[oW3 + 32 * kt + 16 * (e >> 2) + 4 * g + (e & 3)];
    fr.b3 = P[oB3];
}

// Scores of 64 rows whose features sit in sx ([64][16] bfloat16).  Every lane of the wavefront must call it;
// lane l receives the score of row l.  When z1 / z2 are given, the pre-activations of the two hidden layers
// (float32, [64][64] row-major) are stored there as well.  UNROLL groups of 16 rows are interleaved (more
// independent matrix-core work in flight, more registers); the fused search kernels use 1.
template <int UNROLL = 1>
__device__ __forceinline__ float forward64(const __bf16 *sx, const Frags &fr, float *z1 = nullptr,
                                           float *z2 = nullptr) {
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
    const bf8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
    float mine = 0.f;
#pragma unroll UNROLL
    for (int nt = 0; nt < 4; ++nt) {       // 16 moves at a time
        const int row = 16 * nt + c;
        const bf8 x = g < 2 ? *reinterpret_cast<const bf8 *>(sx + row * kF + 8 * g) : zero8;
        f4 d1[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) d1[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.w1t[mt], x, fr.b1[mt], 0, 0, 0);
        if (z1) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) *reinterpret_cast<f4 *>(z1 + row * kH + 16 * mt + 4 * g) = d1[mt];
        }
        bf8 h[2];
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int e = 0; e < 4; e += 2) {
                const bf2 lo = relu_pack(d1[2 * kt][e], d1[2 * kt][e + 1]);
                const bf2 hi = relu_pack(d1[2 * kt + 1][e], d1[2 * kt + 1][e + 1]);
                h[kt][e] = lo[0];
                h[kt][e + 1] = lo[1];
                h[kt][4 + e] = hi[0];
                h[kt][4 + e + 1] = hi[1];
            }
        f4 d2[4];
#pragma unroll
        for (int mo = 0; mo < 4; ++mo) {
            d2[mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.w2t[mo][0], h[0], fr.b2[mo], 0, 0, 0);
            d2[mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.w2t[mo][1], h[1], d2[mo], 0, 0, 0);
            if (z2) *reinterpret_cast<f4 *>(z2 + row * kH + 16 * mo + 4 * g) = d2[mo];
        }
        // layer 3 on the matrix cores as well: layer 2's D fragments are its B fragments (order pi, as layer 2
        // takes layer 1's), and every row of A is W3, so every row of D is the 16 moves' scores and lane
        // 16 g + c holds move c's in each element
        bf8 h2[2];
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int e = 0; e < 4; e += 2) {
                const bf2 lo = relu_pack(d2[2 * kt][e], d2[2 * kt][e + 1]);
                const bf2 hi = relu_pack(d2[2 * kt + 1][e], d2[2 * kt + 1][e + 1]);
                h2[kt][e] = lo[0];
                h2[kt][e + 1] = lo[1];
                h2[kt][4 + e] = hi[0];
                h2[kt][4 + e + 1] = hi[1];
            }
        const f4 zero4 = {0.f, 0.f, 0.f, 0.f};
        f4 d3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.w3a[0], h2[0], zero4, 0, 0, 0);
        d3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.w3a[1], h2[1], d3, 0, 0, 0);
        mine = nt == g ? d3[0] : mine;   // lane 16 nt + c keeps move c's score
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return fr.b3 + mine;
}

// Last setup period <= t and first setup period > t of the pattern s (either type); -1 / T when none.
__device__ __forceinline__ void setup_neighbours(const uint32_t (&s)[kWords], int t, int T, int &prev, int &next) {
    prev = -1;
    next = T;
#pragma unroll
    for (int j = 0; j < kWords; ++j) {
        const int lo = 32 * j;
        // bits of word j at positions <= t
        const uint32_t le = t >= lo + 31 ? ~0u : (t < lo ? 0u : (0xFFFFFFFFu >> (31 - (t - lo))));
        const uint32_t wle = s[j] & le;
        if (wle) prev = lo + 31 - __clz(wle);
        // bits of word j at positions > t (scan from the highest word down so the lowest one wins)
    }
#pragma unroll
    for (int j = kWords - 1; j >= 0; --j) {
        const int lo = 32 * j;
        const uint32_t gt = t >= lo + 31 ? 0u : (t < lo ? ~0u : (0xFFFFFFFFu << (t - lo + 1)));
        const uint32_t wgt = s[j] & gt;
        if (wgt) next = lo + __ffs(wgt) - 1;
    }
    if (next > T) next = T;
}

// Features of local slot l of a product with current pattern b, rows (D, PR), horizon T.
template <class RowPtr>
__device__ __forceinline__ void move_features(const Bits &b, RowPtr row, int T, const ProdParams &pp, int l,
                                              float (&f)[kF]) {
    const int ty = (l >= T) + (l >= 2 * T) + (l >= 3 * T);
    const int t = l - ty * T;
#pragma unroll
    for (int i = 0; i < 4; ++i) f[i] = ty == i ? 1.f : 0.f;
    f[4] = test_bit(b.m, t) ? 1.f : 0.f;
    f[5] = test_bit(b.r, t) ? 1.f : 0.f;
    const int2 cur = row[t];
    const int Rt = cur.y - (t > 0 ? row[t - 1].y : 0);
    f[6] = (float)cur.x / 200.f;
    f[7] = (float)Rt / 200.f;
    f[8] = t > 0 ? (float)row[t - 1].x / 200.f : 0.f;
    f[9] = t + 1 < T ? (float)row[t + 1].x / 200.f : 0.f;
    f[10] = (float)pp.kM / 2000.f;
    f[11] = (float)pp.kR / 2000.f;
    f[12] = (float)pp.hM / 8.f;
    f[13] = (float)pp.hR / 8.f;
    uint32_t s[kWords];
#pragma unroll
    for (int j = 0; j < kWords; ++j) s[j] = b.m[j] | b.r[j];
    int prev, next;
    setup_neighbours(s, t, T, prev, next);
    f[14] = prev >= 0 ? (float)(t - prev) / (float)T : 1.f;
    f[15] = (float)(next - t) / (float)T;
}

// Order-preserving map of a float score to an unsigned key (lower score -> lower key).
__device__ __forceinline__ uint32_t sortable(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

}  // namespace mlp
}  // namespace vns
