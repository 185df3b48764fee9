// Device building blocks of the lot-sizing VNS for gfx950 (64-lane wavefronts).
//
// The hot loop is decode_cost(): the exact cost of one product's setup pattern, evaluated by one lane in
// one forward pass over the T periods.  It is the same cost the look-ahead decode defines (Section 2
// quantities: lots x_M, x_R and inventories y_M, y_R; setup plus holding cost), rewritten so that no
// period needs to look ahead to the next setup:
//   * a unit of demand consumed at tau and produced at p spends tau - p periods in serviceable stock;
//   * a unit remanufactured at s leaves recoverable stock for the T - s remaining periods;
//   * demand is served from the capacity fixed at the last remanufacturing setup lsR (all returns so far
//     minus those used, PR(lsR) - XR) first, the rest by the last manufacturing setup lastM (in its own
//     interval, or carried back to it from a remanufacture-only interval);
//   * a manufacturing setup closes the remanufacturing capacity (its interval makes everything new).
// With A1 = sum u*lsR (u = units remanufactured) and A2 = sum r*lastM (r = units manufactured):
//   cost = kM*nM + kR*nR + hM*(sum t*D - A1 - A2) + hR*(sum PR - T*XR + A1).
// Every period-step is 14 int32 operations; masks come from sign-extended bit extracts so that all the
// setup-dependent updates are bitwise selects, and the two products use the full-rate 24-bit multiply.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vns_types.hpp"

namespace vns {

__device__ __forceinline__ int32_t sel(int32_t mask, int32_t a, int32_t b) { return (mask & a) | (~mask & b); }

__device__ __forceinline__ uint32_t word_bit(int pos, int j) {
    return ((pos >> 5) == j) ? (1u << (pos & 31)) : 0u;
}

__device__ __forceinline__ bool test_bit(const uint32_t (&w)[kWords], int pos) {
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < kWords; ++j) v |= w[j] & word_bit(pos, j);
    return v != 0u;
}

__device__ __forceinline__ void flip_bit(uint32_t (&w)[kWords], int pos) {
#pragma unroll
    for (int j = 0; j < kWords; ++j) w[j] ^= word_bit(pos, j);
}

// Apply local slot l of a product with T periods to b.  Slots: [0,T) flip zM(t); [T,2T) flip zR(t);
// [2T,3T-1) swap zM(t),zM(t+1); [3T,4T-1) swap zR(t),zR(t+1); 3T-1 and 4T-1 are pads.  Returns false,
// leaving b unchanged, for a pad or a swap of two equal bits.
__device__ __forceinline__ bool apply_move(Bits &b, int l, int T) {
    const int blk = (l >= T) + (l >= 2 * T) + (l >= 3 * T);
    const int t = l - blk * T;
    if (blk == 0) { flip_bit(b.m, t); return true; }
    if (blk == 1) { flip_bit(b.r, t); return true; }
    if (t >= T - 1) return false;
    uint32_t (&z)[kWords] = (blk == 2) ? b.m : b.r;
    if (test_bit(z, t) == test_bit(z, t + 1)) return false;
    flip_bit(z, t);
    flip_bit(z, t + 1);
    return true;
}

// Readings of the decode (a bit set of a context's VNS_OPT_DECODE, a template argument of the kernels):
//   kModelStrict   a period whose latest setup is remanufacturing only and lacks returns makes the pattern
//                  infeasible, instead of the shortfall being made by the last manufacturing lot;
//   kModelDispose  returns no lot needs are disposed of, and recoverable holding is charged on the kept stock.
constexpr int kModelStrict = 1;
constexpr int kModelDispose = 2;
constexpr int kModels = 4;

// State of the forward decode of one pattern (one lane).
struct DecodeState {
    int32_t lim = 0, XR = 0, lsR = 0, lastM = 0, A1 = 0, A2 = 0;
    int32_t nolast = -1, bad = 0;
};

// acc += a * b with a, b < 2^24 (the host rejects larger demands and returns), as one v_mad_u32_u24: the
// compiler would otherwise regroup consecutive periods' products into mul + add3 trees (three instructions
// per two periods instead of two).
__device__ __forceinline__ void mad_u24(int32_t &acc, int32_t a, int32_t b) {
    asm("v_mad_u32_u24 %0, %1, %2, %0" : "+v"(acc) : "v"(a), "v"(b));
}

// acc |= a & b as one v_and_or_b32.
__device__ __forceinline__ void and_or(int32_t &acc, int32_t a, int32_t b) {
    asm("v_and_or_b32 %0, %1, %2, %0" : "+v"(acc) : "v"(a), "v"(b));
}

// One period-step: sm, sr are the setup bits of period tau as 0 / -1 masks, dp = (D(tau), PR(tau)).
template <int MODEL = 0>
__device__ __forceinline__ void decode_step(DecodeState &s, int32_t sm, int32_t sr, int32_t tau, int2 dp) {
    s.lim = sel(sm, s.XR, s.lim);         // a manufacturing setup closes the remanufacturing capacity
    s.lastM = sel(sm, tau, s.lastM);
    if constexpr ((MODEL & kModelStrict) != 0)
        s.nolast = ~sm & (s.nolast | sr);   // no manufacturing allowed since the latest setup (R-only, or none)
    else
        s.nolast &= ~sm;                    // no manufacturing setup yet
    s.lim = sel(sr, dp.y, s.lim);         // a remanufacturing setup may use every return so far
    s.lsR = sel(sr, tau, s.lsR);
    const int32_t xn = min(s.XR + dp.x, s.lim);
    const int32_t u = xn - s.XR;          // units remanufactured at lsR for period tau
    s.XR = xn;
    mad_u24(s.A1, u, s.lsR);
    const int32_t rr = dp.x - u;          // units manufactured at lastM for period tau
    mad_u24(s.A2, rr, s.lastM);
    and_or(s.bad, rr, s.nolast);          // demand manufactured where no manufacturing lot may make it
}

// Disposal (kModelDispose): sum over t of m(t) = min_{s >= t} yR(s), the recoverable stock without disposal
// that no later lot uses, from a backward pass.  yR(t) = PR(t) - c, with c the units remanufactured by the end
// of t's setup interval (XR after the forward pass for the last one); going back over a remanufacturing setup,
// c drops by the interval's demand (a lot that left stock covered all of it; one that used every return left
// yR = 0 there, so every earlier m is 0 whatever c is, and m is clamped at 0).  Only the first NW setup words
// of b are read.
template <int NW, class RowPtr>
__device__ __forceinline__ int32_t dispose_credit(const Bits &b, RowPtr row, int T, int32_t XR) {
    int32_t c = XR, dint = 0, m = INT32_MAX, acc = 0;
#pragma unroll
    for (int j = NW - 1; j >= 0; --j) {
        if (32 * j >= T) continue;
        const int32_t wr = (int32_t)b.r[j], ws = (int32_t)(b.m[j] | b.r[j]);
        for (int t = min(32 * j + 31, T - 1); t >= 32 * j; --t) {
            const int2 dp = row[t];
            dint += dp.x;
            m = max(min(m, dp.y - c), 0);   // min(m, yR(t)), never below 0 (one v_med3_i32)
            acc += m;
            c -= dint & __builtin_amdgcn_sbfe(wr, t & 31, 1);   // a remanufacturing lot covered the interval
            dint &= ~__builtin_amdgcn_sbfe(ws, t & 31, 1);      // a setup starts the interval
        }
    }
    return acc;
}

// Cost from the final decode state; only the first NW setup words of b are read (the others are zero when
// T <= 32 NW).  credit: the disposal reading's sum of never-needed recoverable stock (0 otherwise).
template <int NW = kWords>
__device__ __forceinline__ int64_t decode_finish(const DecodeState &s, const Bits &b, int T, const ProdParams &pp,
                                                 int32_t credit = 0) {
    if (s.bad) return kInf;
    int32_t nM = 0, nR = 0;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
        nM += __popc(b.m[j]);
        nR += __popc(b.r[j]);
    }
    // kM nM + kR nR + hM (S_tD - A1 - A2) + hR (S_PR - T XR + A1) + pM (SD - XR) + pR XR, the constant and
    // the XR terms folded into C and cXR (every demanded item is made once, XR of them remanufactured)
    return (int64_t)pp.kM * nM + (int64_t)pp.kR * nR - (int64_t)pp.hM * ((int64_t)s.A1 + (int64_t)s.A2) +
           (int64_t)pp.hR * ((int64_t)s.A1 - credit) + pp.cXR * s.XR + pp.C;
}

template <class RowPtr>
__device__ __forceinline__ void load_chunk(RowPtr row, int at, int2 (&c)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = row[at + i];
}

// Four period-steps from period tau (a multiple of four) of the setup words m, r that hold it.
template <int MODEL = 0>
__device__ __forceinline__ void decode_chunk(DecodeState &s, int32_t m, int32_t r, int tau, const int2 (&c)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
        decode_step<MODEL>(s, __builtin_amdgcn_sbfe(m, (tau + i) & 31, 1), __builtin_amdgcn_sbfe(r, (tau + i) & 31, 1),
                           tau + i, c[i]);
}

// Exact cost of one product's pattern (kInf when infeasible), any T <= kTMax.  row points at the product's
// (D, PR) pairs; it may be an LDS or a global pointer (after inlining the address space is known).  T must
// be the same in every active lane.  The periods are walked in chunks of four; the rows of the next chunk
// are read while the current one is decoded, alternating between two register sets so that nothing is
// copied, and never past period T - 1.
template <int NW = kWords, int MODEL = 0, class RowPtr>
__device__ __forceinline__ int64_t decode_cost(const Bits &b, RowPtr row, int T, const ProdParams &pp) {
    static_assert(NW >= 1 && NW <= kWords, "setup words");
    T = __builtin_amdgcn_readfirstlane(T);
    DecodeState s;
    const int Tc = T - 4;   // start of the last whole chunk
    int2 ca[4], cb[4];
    if (Tc >= 0) load_chunk(row, 0, ca);
    int tau = 0;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
        if (32 * j >= T) break;
        const int32_t m = (int32_t)b.m[j], r = (int32_t)b.r[j];
        const int wend = min(32 * j + 32, T);
        for (; tau + 8 <= wend; tau += 8) {
            load_chunk(row, min(tau + 4, Tc), cb);
            decode_chunk<MODEL>(s, m, r, tau, ca);
            load_chunk(row, min(tau + 8, Tc), ca);
            decode_chunk<MODEL>(s, m, r, tau + 4, cb);
        }
        if (tau + 4 <= wend) {
            load_chunk(row, min(tau + 4, Tc), cb);
            decode_chunk<MODEL>(s, m, r, tau, ca);
#pragma unroll
            for (int i = 0; i < 4; ++i) ca[i] = cb[i];
            tau += 4;
        }
        for (; tau < wend; ++tau)   // the last one to three periods
            decode_step<MODEL>(s, __builtin_amdgcn_sbfe(m, tau & 31, 1), __builtin_amdgcn_sbfe(r, tau & 31, 1), tau,
                               row[tau]);
    }
    int32_t credit = 0;
    if constexpr ((MODEL & kModelDispose) != 0) credit = dispose_credit<NW>(b, row, T, s.XR);
    return decode_finish<NW>(s, b, T, pp, credit);
}

// Apply a move given as (block, t) to the first NW setup words of b: block 0 flips zM(t), 1 flips zR(t),
// 2 swaps zM(t), zM(t+1), 3 swaps zR(t), zR(t+1) (a valid swap: the two bits differ, so the swap flips
// both).  The change is one XOR mask over the 32 NW bits of the pattern.
template <int NW>
__device__ __forceinline__ void xor_move(Bits &b, int blk, int t) {
    static_assert(NW == 2 || NW == 4, "setup words");
    const uint64_t w = blk >= 2 ? 3ull : 1ull;
    const bool on_r = blk & 1;
    uint64_t lo, hi = 0;
    if constexpr (NW == 2) {
        lo = w << t;
    } else {
        const uint64_t sh = w << (t & 63);
        lo = t < 64 ? sh : 0ull;
        hi = t >= 64 ? sh : (t == 63 ? (w >> 1) : 0ull);   // a swap at 63 reaches bit 64
    }
    const uint64_t xm0 = on_r ? 0ull : lo, xr0 = on_r ? lo : 0ull;
    b.m[0] ^= (uint32_t)xm0;
    b.m[1] ^= (uint32_t)(xm0 >> 32);
    b.r[0] ^= (uint32_t)xr0;
    b.r[1] ^= (uint32_t)(xr0 >> 32);
    if constexpr (NW == 4) {
        const uint64_t xm1 = on_r ? 0ull : hi, xr1 = on_r ? hi : 0ull;
        b.m[2] ^= (uint32_t)xm1;
        b.m[3] ^= (uint32_t)(xm1 >> 32);
        b.r[2] ^= (uint32_t)xr1;
        b.r[3] ^= (uint32_t)(xr1 >> 32);
    }
}

// Feasibility of a pattern under the carry-back reading: only the periods before the first manufacturing
// setup can fail (afterwards every shortfall is made by a manufacturing lot).  Uniform use by a whole wave.
template <class RowPtr>
__device__ __forceinline__ bool feasible(const Bits &b, RowPtr row, int T) {
    int32_t lim = 0, XR = 0;
    for (int tau = 0; tau < T; ++tau) {
        const int j = tau >> 5, q = tau & 31;
        uint32_t m = 0, r = 0;
#pragma unroll
        for (int w = 0; w < kWords; ++w) {
            m = (w == j) ? b.m[w] : m;
            r = (w == j) ? b.r[w] : r;
        }
        if ((m >> q) & 1u) return true;
        const int2 dp = row[tau];
        if ((r >> q) & 1u) lim = dp.y;
        const int32_t xn = min(XR + dp.x, lim);
        if (dp.x - (xn - XR) > 0) return false;
        XR = xn;
    }
    return true;
}

// Whether a shaken product's pattern is feasible under the reading MODEL: with the carry-back reading a
// manufacturing setup in period 0 is enough, else the prefix check; with the strict reading the full decode.
template <int MODEL, class RowPtr>
__device__ __forceinline__ bool shake_feasible(const Bits &b, RowPtr row, int T, const ProdParams &pp) {
    if constexpr ((MODEL & kModelStrict) != 0) {
        return decode_cost<kWords, MODEL & kModelStrict>(b, row, T, pp) != kInf;
    } else {
        return (b.m[0] & 1u) != 0u || feasible(b, row, T);
    }
}

// ---------------------------------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds, each two 64x64 -> 128-bit products with
// the published multipliers, the key advanced by the published Weyl increments.  Returns word 0.
// ---------------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t philox_word0(uint64_t key0, uint64_t key1, uint64_t c0, uint64_t c1,
                                                 uint64_t c2, uint64_t c3) {
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull, kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull, kWeylB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t hiA = __umul64hi(kMulA, c0), loA = kMulA * c0;
        const uint64_t hiB = __umul64hi(kMulB, c2), loB = kMulB * c2;
        const uint64_t n0 = hiB ^ c1 ^ key0;
        const uint64_t n2 = hiA ^ c3 ^ key1;
        c0 = n0;
        c1 = loB;
        c2 = n2;
        c3 = loA;
        key0 += kWeylA;
        key1 += kWeylB;
    }
    return c0;
}

// Index in [0, n) of draw j of iteration it of random stream `stream` for the chain keyed (seed, chain):
// multiply-shift of the high 32 bits of Philox word 0, counter (it, j, stream, 0).  Stream 0 is the chain's
// own shake; the best-of-G search shakes with streams 0 .. G-1.
__device__ __forceinline__ uint32_t shake_draw(uint64_t seed, uint64_t chain, uint64_t it, uint64_t j, uint64_t n,
                                               uint64_t stream = 0) {
    const uint64_t w = philox_word0(seed, chain, it, j, stream, 0);
    return (uint32_t)(((w >> 32) * n) >> 32);
}

// ---------------------------------------------------------------------------------------------------
// Wave reductions (64 lanes).
// ---------------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace vns
