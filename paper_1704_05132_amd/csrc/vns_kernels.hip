// Kernels of the lot-sizing VNS for gfx950.
//
//   k_init_costs    exact cost of every (chain, product) of the current solutions; F per chain
//   k_eval          one workgroup per (product, group of chains of its instance): exact price of every move
//                   of the selected neighbourhoods, one lane per move (Section 3: the new objective value of
//                   each product is computed independently of the others).  Moves are compacted (pads and
//                   swaps of equal bits never take a lane) and the chains of the group share one LDS copy of
//                   the product's row, so a wavefront is full whatever T is
//   k_chain_best    per chain: lexicographic (price, slot) minimum over its products
//   k_run           one workgroup per chain running whole GVNS iterations (Algorithm 2): Philox shake,
//                   VND (Algorithm 1) with one wavefront per product that needs it, acceptance
//   k_run_spec      the same with the neighbourhoods of a product's VND priced side by side
//   k_run_learned   the same with the learned scorer choosing which moves are priced exactly
#include <hip/hip_runtime.h>

#include <algorithm>

#include "vns_device.hpp"
#include "vns_launch.hpp"
#include "vns_search.hpp"

namespace vns {


// ---------------------------------------------------------------------------------------------------
// k_init_costs: one workgroup per chain.  Costs of the current solution, copy to the working solution,
// F, best, shake size 1.
// ---------------------------------------------------------------------------------------------------
template <int MODEL>
__global__ __launch_bounds__(256) void k_init_costs(InitArgs a) {
    const int g = a.chain0 + blockIdx.x;
    const ChainInfo ci = a.chains[g];
    int64_t sum = 0;
    int inf = 0;
    for (int p = threadIdx.x; p < ci.K; p += blockDim.x) {
        const ProdParams pp = a.prod[ci.prod0 + p];
        const int64_t cp = ci.cp0 + p;
        const Bits b = a.cur[cp];
        const int64_t c = decode_cost<kWords, MODEL>(b, a.rows + pp.row, ci.T, pp);
        a.cur_cost[cp] = c;
        a.work[cp] = b;
        a.work_cost[cp] = c;
        a.best[cp] = b;
        if (c == kInf) inf = 1; else sum += c;
    }
    __shared__ int64_t s_sum[4];
    __shared__ int s_inf[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    sum = wave_sum_i64(sum);
    const int any_inf = __any(inf);
    if (lane == 0) { s_sum[wave] = sum; s_inf[wave] = any_inf; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t F = 0;
        int bad = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { F += s_sum[w]; bad |= s_inf[w]; }
        ChainState cs;
        cs.F = bad ? kInf : F;
        cs.F_best = cs.F;
        cs.evals = 0;
        cs.k = 1;
        cs.lopt = 0;
        cs.err = 0;
        cs.bsync = 1;
        cs.nb_evals = 0;
        cs.fallbacks = 0;
        cs.discarded = 0;
        a.cstate[g] = cs;
    }
}

// ---------------------------------------------------------------------------------------------------
// k_eval
// ---------------------------------------------------------------------------------------------------
namespace {

struct EvalShared {
    int2 row[kTMax];              // the rows of the workgroup's products, one after the other (np T <= kTMax)
    ProdParams pp[kEvalProds];    // their parameters (more than one product)
    Bits bits[kEvalPairs];        // per (chain, product) pair j = product index * chains + chain index
    unsigned long long key[kEvalPairs];
    int64_t F[kEvalPairs];
    int64_t cost[kEvalPairs];
    int64_t out_off[kEvalPairs];
    int32_t off[kEvalPairs + 1];
    uint8_t pidx[kEvalPairs];     // product index of each pair within the workgroup's products
    // the workgroup's moves, pair by pair (flips, then zM swaps, then zR swaps): pair << 9 | block << 7 | t
    uint16_t item[kEvalItems];
    int32_t tcount[kTMax];        // incremental pricing: moves per period, then their offsets
    int32_t decoded;              //   and the period-steps its batches ran, per lane
};
static_assert(kEvalPairs <= 128 && kTMax <= 128, "item packing");
static_assert(kEvalPairs <= 64, "one wavefront scans the pairs' move counts");
static_assert(kEvalGroup * 4 * kTMax <= kEvalItems, "one product of a full group of chains fits the item table");

__device__ __forceinline__ uint16_t pack_item(int j, int blk, int t) { return (uint16_t)((j << 9) | (blk << 7) | t); }

// One lane per item: apply the move to the pair's pattern, decode, fold (cost, slot) into the pair's key.
// One product (np = 1): its row and parameters are the same for every lane; several (short horizons): each
// lane reads those of its pair's product.
template <int NW, int MODEL>
__device__ __forceinline__ void eval_items(const EvalArgs &a, EvalShared &sh, int N, int T, const ProdParams &pp,
                                           int np) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int basei = wave * 64; basei < N; basei += blockDim.x) {
        const int idx = basei + lane;
        const bool in = idx < N;
        const int e = sh.item[in ? idx : basei];
        const int j = e >> 9, blk = (e >> 7) & 3, t = e & 127;
        const int slot = blk * T + t;
        Bits mb = sh.bits[j];
        xor_move<NW>(mb, blk, t);
        int64_t c;
        if (np == 1) {
            c = decode_cost<NW, MODEL>(mb, sh.row, T, pp);
        } else {
            const int pi = sh.pidx[j];
            c = decode_cost<NW, MODEL>(mb, sh.row + pi * T, T, sh.pp[pi]);
        }
        if (in) {
            if (c != kInf) atomicMin(&sh.key[j], ((unsigned long long)c << kSlotBits) | (unsigned long long)slot);
            if (a.slot_price) a.slot_price[sh.out_off[j] + slot] = c == kInf ? kInf : sh.F[j] - sh.cost[j] + c;
        }
    }
}

// Incremental exact pricing.  A move changes the pattern only from its first changed period t on, so its
// decode starts from the base pattern's state before t (snapshot, per chain and period: A = (lim, XR, lsR,
// last manufacturing setup or -1 before the first one), B = (A1, A2)).  Once every changed period is
// decoded and the moved pattern's state A equals the base's before some period, every later step adds the
// same amounts to both, so the cost is the base cost plus the setup-count change, -hM (dA1 + dA2) and hR dA1
// (the forward decode's cost is linear in A1, A2 and the final XR).  A decode that turns infeasible stops
// there (kInf).
__device__ __forceinline__ int32_t enc_last(const DecodeState &s) { return s.nolast ? -1 : s.lastM; }

// The base pattern b of one chain, decoded by one lane: its state before every period 0..T.
template <int NW>
__device__ __forceinline__ void base_snapshot(const Bits &b, const int2 *row, int T, int4 *sa, int2 *sb) {
    DecodeState s;
    for (int tau = 0; tau < T; ++tau) {
        sa[tau] = make_int4(s.lim, s.XR, s.lsR, enc_last(s));
        sb[tau] = make_int2(s.A1, s.A2);
        const int w = tau >> 5;
        uint32_t m = b.m[0], r = b.r[0];
#pragma unroll
        for (int q = 1; q < NW; ++q) {
            m = w == q ? b.m[q] : m;
            r = w == q ? b.r[q] : r;
        }
        decode_step(s, __builtin_amdgcn_sbfe((int32_t)m, tau & 31, 1), __builtin_amdgcn_sbfe((int32_t)r, tau & 31, 1),
                    tau, row[tau]);
    }
    sa[T] = make_int4(s.lim, s.XR, s.lsR, enc_last(s));
    sb[T] = make_int2(s.A1, s.A2);
}

// Moves sorted by first changed period, 64 at a time: every lane of a batch starts from the base's state
// before the batch's first period t0 (a move changes nothing before its own first period, so its decode
// there equals the base's) and the lanes step through the same periods, reading rows and setup bits at a
// uniform position as the full decode does: single periods up to a multiple of 8, then blocks of 8 in the
// full decode's form (two chunks of four, the setup words chosen once per block), then single periods to the
// horizon.  Before each block every lane checks whether it has rejoined the base (or turned infeasible); the
// batch ends when all have, or at the horizon.
template <int NW>
__device__ __forceinline__ void eval_items_inc(const EvalArgs &a, EvalShared &sh, const int4 *snapA, const int2 *snapB,
                                               int N, int T, const ProdParams &pp) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int decoded = 0;
    for (int basei = wave * 64; basei < N; basei += blockDim.x) {
        const int idx = basei + lane;
        const bool in = idx < N;
        const int e = sh.item[in ? idx : basei];
        const int j = e >> 9, blk = (e >> 7) & 3, t = e & 127;
        const int slot = blk * T + t;
        const int t0 = __builtin_amdgcn_readfirstlane(sh.item[basei] & 127);   // sorted: the batch's first period
        Bits mb = sh.bits[j];
        const int dnM = blk == 0 ? (test_bit(mb.m, t) ? -1 : 1) : 0;   // a swap keeps the number of setups
        const int dnR = blk == 1 ? (test_bit(mb.r, t) ? -1 : 1) : 0;
        xor_move<NW>(mb, blk, t);
        const int t1 = blk >= 2 ? t + 1 : t;                             // last changed period
        DecodeState s;
        {
            const int4 sa = snapA[j * (T + 1) + t0];
            const int2 sb = snapB[j * (T + 1) + t0];
            s.lim = sa.x;
            s.XR = sa.y;
            s.lsR = sa.z;
            s.lastM = sa.w < 0 ? 0 : sa.w;
            s.nolast = sa.w < 0 ? -1 : 0;
            s.A1 = sb.x;
            s.A2 = sb.y;
        }
        bool done = !in;
        int64_t c = kInf;
        // the lane's setup word w (w wave-uniform)
        auto word = [&](const uint32_t (&v)[kWords], int w) {
            uint32_t x = v[0];
#pragma unroll
            for (int q = 1; q < NW; ++q) x = w == q ? v[q] : x;
            return (int32_t)x;
        };
        // before period tau: has this lane rejoined the base (its cost is then known) or turned infeasible?
        // True when every lane of the batch is done.
        auto check = [&](int tau) -> bool {
            if (!done) {
                if (s.bad) {   // infeasible: kInf
                    done = true;
                } else if (tau > t1) {
                    const int4 sa = snapA[j * (T + 1) + tau];
                    if (sa.x == s.lim && sa.y == s.XR && sa.z == s.lsR && sa.w == enc_last(s)) {   // rejoined
                        const int2 sb = snapB[j * (T + 1) + tau];
                        const int64_t dA1 = (int64_t)s.A1 - sb.x, dA2 = (int64_t)s.A2 - sb.y;
                        c = sh.cost[j] + (int64_t)pp.kM * dnM + (int64_t)pp.kR * dnR - (int64_t)pp.hM * (dA1 + dA2) +
                            (int64_t)pp.hR * dA1;
                        done = true;
                    }
                }
            }
            return !__any(!done);
        };
        auto single = [&](int tau) {
            const int w = tau >> 5;
            decode_step(s, __builtin_amdgcn_sbfe(word(mb.m, w), tau & 31, 1),
                        __builtin_amdgcn_sbfe(word(mb.r, w), tau & 31, 1), tau, sh.row[tau]);
        };
        int tau = t0;
        bool all = false;
        for (; tau < T && (tau & 7) != 0; ++tau) single(tau);
        int2 ca[4], cb[4];
        for (; tau + 8 <= T; tau += 8) {
            if (tau > t0 && check(tau)) {
                all = true;
                break;
            }
            load_chunk(sh.row, tau, ca);
            load_chunk(sh.row, tau + 4, cb);
            const int w = tau >> 5;   // a block of 8 never crosses a setup word
            const int32_t m = word(mb.m, w), r = word(mb.r, w);
            decode_chunk(s, m, r, tau, ca);
            decode_chunk(s, m, r, tau + 4, cb);
        }
        if (!all && tau < T && tau > t0 && (tau & 7) == 0) all = check(tau);
        for (; !all && tau < T; ++tau) single(tau);
        if (!done) c = decode_finish<NW>(s, mb, T, pp);   // decoded to the horizon (kInf when infeasible)
        if (in) {
            decoded += tau - t0;                           // period-steps this lane's batch ran
            if (c != kInf) atomicMin(&sh.key[j], ((unsigned long long)c << kSlotBits) | (unsigned long long)slot);
            if (a.slot_price) a.slot_price[sh.out_off[j] + slot] = c == kInf ? kInf : sh.F[j] - sh.cost[j] + c;
        }
    }
    atomicAdd(&sh.decoded, decoded);
}

// Pair j of a pricing workgroup: its product index pi within the workgroup's products and its chain index ci
// (from g0), in the rectangular form (j = pi * nc + ci) or the range form.
__device__ __forceinline__ void eval_pair(const EvalWg &d, int j, int &pi, int &ci) {
    if (d.G > 0) {
        const int q = d.q0 + j;
        pi = q / d.G - d.p;
        ci = q - (q / d.G) * d.G;
    } else {
        pi = j / d.n;
        ci = j - pi * d.n;
    }
}

template <bool INC, int MODEL = 0>
__device__ __forceinline__ void eval_body(const EvalArgs &a, const EvalWg *__restrict__ wg, EvalShared &sh,
                                          int4 *s_snap) {
    const EvalWg d = wg[blockIdx.x];
    if (d.n == 0) return;   // an empty entry (uniform for the workgroup)
    const int g0 = d.g0, K = d.K, T = d.T, p = d.p;
    const int np = INC ? 1 : max(d.np, 1);
    const int n = d.G > 0 ? d.n : d.n * np;   // pairs
    const ProdParams pp = a.prod[d.prod];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int t = threadIdx.x; t < np * T; t += blockDim.x) sh.row[t] = a.rows[d.row + t];
    if (np > 1)
        for (int q = threadIdx.x; q < np; q += blockDim.x) sh.pp[q] = a.prod[d.prod + q];
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        int pi, ci;
        eval_pair(d, j, pi, ci);
        const int64_t cp = d.cp + (int64_t)ci * K + pi;
        sh.pidx[j] = (uint8_t)pi;
        sh.bits[j] = a.cur[cp];
        sh.cost[j] = a.cur_cost[cp];
        sh.F[j] = a.cstate[g0 + ci].F;
        sh.key[j] = kInfKey;
        sh.out_off[j] = a.slot_price ? a.price_off[g0 + ci] + (int64_t)(p + pi) * 4 * T : 0;
    }
    __syncthreads();

    const bool fm = a.nb_mask & 1u, fr = a.nb_mask & 2u, shift = a.nb_mask & 4u;
    const int nflip = (fm ? T : 0) + (fr ? T : 0);
    // the pairs' move counts (one lane per pair, n <= 64) and their exclusive prefix, by wavefront 0
    if (wave == 0) {
        int cnt = 0;
        if (lane < n) {
            cnt = nflip;
            if (shift) {
                uint32_t vm[kWords], vr[kWords];
                swap_valid(sh.bits[lane].m, T, vm);
                swap_valid(sh.bits[lane].r, T, vr);
                cnt += popc_words(vm) + popc_words(vr);
            }
        }
        int inc = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int up = __shfl_up(inc, d, 64);
            inc += lane >= d ? up : 0;
        }
        if (lane < n) sh.off[lane] = inc - cnt;
        if (lane == 63) sh.off[n] = inc;
    }
    if (a.slot_price) {  // every slot of the group starts as "not a priced move"
        for (int j = 0; j < n; ++j)
            for (int l = threadIdx.x; l < 4 * T; l += blockDim.x) a.slot_price[sh.out_off[j] + l] = kInf;
    }
    __syncthreads();
    // the item table: flips (zM then zR), then each chain's valid swaps in period order; for incremental
    // pricing sorted by period instead (period t: every chain's flips and valid swaps at t)
    const int fblk0 = fm ? 0 : 1;
    if constexpr (INC) {
        for (int t = threadIdx.x; t < T; t += blockDim.x) {
            int cnt = 0;
            for (int j = 0; j < n; ++j) {
                const Bits &b = sh.bits[j];
                cnt += (fm ? 1 : 0) + (fr ? 1 : 0);
                if (shift && t + 1 < T) {
                    cnt += test_bit(b.m, t) != test_bit(b.m, t + 1);
                    cnt += test_bit(b.r, t) != test_bit(b.r, t + 1);
                }
            }
            sh.tcount[t] = cnt;
        }
        __syncthreads();
        if (wave == 0) {   // exclusive prefix over the periods (T <= 128: two per lane)
            const int c0 = 2 * lane < T ? sh.tcount[2 * lane] : 0;
            const int c1 = 2 * lane + 1 < T ? sh.tcount[2 * lane + 1] : 0;
            int inc = c0 + c1;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int up = __shfl_up(inc, d, 64);
                inc += lane >= d ? up : 0;
            }
            const int ex = inc - c0 - c1;
            if (2 * lane < T) sh.tcount[2 * lane] = ex;
            if (2 * lane + 1 < T) sh.tcount[2 * lane + 1] = ex + c0;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < T; t += blockDim.x) {
            int o = sh.tcount[t];
            for (int j = 0; j < n; ++j) {
                const Bits &b = sh.bits[j];
                if (fm) sh.item[o++] = pack_item(j, 0, t);
                if (fr) sh.item[o++] = pack_item(j, 1, t);
                if (shift && t + 1 < T) {
                    if (test_bit(b.m, t) != test_bit(b.m, t + 1)) sh.item[o++] = pack_item(j, 2, t);
                    if (test_bit(b.r, t) != test_bit(b.r, t + 1)) sh.item[o++] = pack_item(j, 3, t);
                }
            }
        }
    }
    for (int j = wave; j < n && !INC; j += nw) {
        uint16_t *it = sh.item + sh.off[j];
        for (int i = lane; i < nflip; i += 64) {
            const int blk = fblk0 + (i >= T ? 1 : 0);
            it[i] = pack_item(j, blk, i - (i >= T ? T : 0));
        }
        if (shift)   // each chain's valid swaps in period order, the zM swaps first
            compact_swaps(sh.bits[j], T, it + nflip, [j](int z, int t) { return pack_item(j, 2 + z, t); });
    }
    __syncthreads();

    const int N = sh.off[n];
    if constexpr (INC) {
        int4 *snapA = s_snap;                                              // [n][T+1]
        int2 *snapB = reinterpret_cast<int2 *>(s_snap + (size_t)n * (T + 1));   // [n][T+1]
        if (threadIdx.x < n) {
            const int j = threadIdx.x;
            if (T <= 64)
                base_snapshot<2>(sh.bits[j], sh.row, T, snapA + j * (T + 1), snapB + j * (T + 1));
            else
                base_snapshot<4>(sh.bits[j], sh.row, T, snapA + j * (T + 1), snapB + j * (T + 1));
        }
        if (threadIdx.x == 0) sh.decoded = 0;
        __syncthreads();
        if (T <= 64)
            eval_items_inc<2>(a, sh, snapA, snapB, N, T, pp);
        else
            eval_items_inc<4>(a, sh, snapA, snapB, N, T, pp);
    } else {
        if (T <= 64)
            eval_items<2, MODEL>(a, sh, N, T, pp, np);
        else
            eval_items<4, MODEL>(a, sh, N, T, pp, np);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        int pi, ci;
        eval_pair(d, j, pi, ci);
        a.prod_key[d.cp + (int64_t)ci * K + pi] = sh.key[j];
    }
    if (threadIdx.x == 0) {
        unsigned long long *ctr = a.evals + (size_t)(blockIdx.x & (kCounterSlots - 1)) * kCounterStride;
        atomicAdd(ctr, (unsigned long long)N);
        atomicAdd(ctr + 1, (unsigned long long)N * (unsigned long long)T);
        // period-steps decoded: the base snapshots and the moves' incremental decodes, or every move in full
        atomicAdd(ctr + 2, INC ? (unsigned long long)sh.decoded + (unsigned long long)n * T
                               : (unsigned long long)N * (unsigned long long)T);
    }
}

}  // namespace

template <int MODEL>
__global__ __launch_bounds__(256) void k_eval(EvalArgs a, const EvalWg *__restrict__ wg) {
    __shared__ EvalShared sh;
    eval_body<false, MODEL>(a, wg, sh, nullptr);
}

// The same with 512-1024-thread workgroups (the range form spread over the compute units).
template <int MODEL>
__global__ __launch_bounds__(1024) void k_eval_wide(EvalArgs a, const EvalWg *__restrict__ wg) {
    __shared__ EvalShared sh;
    eval_body<false, MODEL>(a, wg, sh, nullptr);
}

// The same sweep priced incrementally; dynamic LDS holds the base snapshots (24 bytes per chain and period).
__global__ __launch_bounds__(256) void k_eval_inc(EvalArgs a, const EvalWg *__restrict__ wg) {
    __shared__ EvalShared sh;
    extern __shared__ __attribute__((aligned(16))) int4 s_snap[];
    eval_body<true>(a, wg, sh, s_snap);
}

// The pricing table for chains g0 .. g0+ng-1 and zeroed counters, on the device (see EvalPrepArgs).
__global__ __launch_bounds__(256) void k_eval_prep(EvalPrepArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = tid; i < a.n_cp; i += stride) {
        const int64_t cp = a.cp_begin + i;
        const int g = a.cp_chain[cp];
        const ChainInfo ci = a.chains[g];
        const int first = max(a.g0, ci.inst * a.chains_per_inst);            // the instance's first chain in range
        const int end = min(a.g0 + a.ng, (ci.inst + 1) * a.chains_per_inst);  // and one past its last
        EvalWg w{};
        if ((g - first) % a.group == 0) {
            const int p = (int)(cp - ci.cp0);
            w.cp = cp;
            w.g0 = g;
            w.n = min(a.group, end - g);
            w.K = ci.K;
            w.T = ci.T;
            w.p = p;
            w.prod = ci.prod0 + p;
            w.row = a.prod[ci.prod0 + p].row;
            w.np = 1;
        }
        a.table[i] = w;
    }
    for (int64_t j = tid; j < counter_words(); j += stride) a.counters[j] = 0ull;
}

// ---------------------------------------------------------------------------------------------------
// k_chain_best: one workgroup per chain; per-product (price, slot) and the chain's lexicographic minimum.
// ---------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chain_best(ChainBestArgs a) {
    const int g = a.chain0 + blockIdx.x;
    const ChainInfo ci = a.chains[g];
    const int64_t F = a.cstate[g].F;
    int64_t bp = kInf;
    int64_t bs = -1;
    for (int p = threadIdx.x; p < ci.K; p += blockDim.x) {
        const int64_t cp = ci.cp0 + p;
        const uint64_t key = a.prod_key[cp];
        int64_t price = kInf;
        int32_t slot = -1;
        if (key != kInfKey) {
            price = F - a.cur_cost[cp] + (int64_t)(key >> kSlotBits);
            slot = (int32_t)(key & ((1u << kSlotBits) - 1));
        }
        a.prod_price[cp] = price;
        a.prod_slot[cp] = slot;
        const int64_t gs = slot < 0 ? -1 : (int64_t)p * 4 * ci.T + slot;
        if (slot >= 0 && (price < bp || (price == bp && gs < bs))) { bp = price; bs = gs; }
    }
    // lexicographic (price, slot) minimum over the workgroup
    for (int off = 32; off >= 1; off >>= 1) {
        const int64_t op = __shfl_xor(bp, off, 64);
        const int64_t os = __shfl_xor(bs, off, 64);
        if (os >= 0 && (bs < 0 || op < bp || (op == bp && os < bs))) { bp = op; bs = os; }
    }
    __shared__ int64_t s_p[4], s_s[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { s_p[wave] = bp; s_s[wave] = bs; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            if (s_s[w] >= 0 && (bs < 0 || s_p[w] < bp || (s_p[w] == bp && s_s[w] < bs))) { bp = s_p[w]; bs = s_s[w]; }
        }
        a.best[blockIdx.x] = bs < 0 ? kInf : bp;
        a.best_slot[blockIdx.x] = (int32_t)bs;
    }
}

// ---------------------------------------------------------------------------------------------------
// k_run: persistent GVNS.  One workgroup per chain, W wavefronts.  Invariant at every iteration start:
// work == cur for every product of the chain.  The instance's rows sit in LDS when they fit
// (K*T <= a.lds_rows), otherwise each wavefront stages the row of the product it works on.  The first
// iteration index comes from device memory so that a captured launch can be replayed unchanged.
// ---------------------------------------------------------------------------------------------------
namespace {

struct RunShared {
    uint16_t list[kMaxWaves][2 * kTMax];   // compacted swap moves of each wavefront's product
    Bits db[kShakeMax];                    // shaken products (dirty list): bits after the shake
    int32_t dp[kShakeMax];                 //   and product index
    int64_t part[kMaxWaves];
    int64_t shk[kMaxWaves];
    int64_t ev[kMaxWaves];
    int64_t fb[kMaxWaves];
    int32_t verr[kMaxWaves];
    int32_t nd;
    // speculative iterations: the chain's state at a round start (read by one thread, so that the whole
    // workgroup decides alike), the round's accepted slot (-1: none) and abort flag
    ChainState coop_cs;
    int64_t coop_done_it;
    int32_t coop_round;   // the round this workgroup computes
    int32_t next_prod;    // VND: the next product index to hand to a wavefront that has finished its own
    int32_t coop_stop;
    int32_t coop_acc;
    int32_t coop_abort;
    int32_t coop_bmode;   // the round's update of the best solution: 0 none, 1 the accepted products, 2 all of x
    int64_t nbr[kMaxWaves];   // a round's learned counters per wavefront
    int64_t fbr[kMaxWaves];
};

// The next VND product index of a wavefront: one LDS add by lane 0, the value in lane 0.
__device__ __forceinline__ int next_index(int32_t &counter, int lane) {
    int v = 0;
    if (lane == 0) v = atomicAdd(&counter, 1);
    return __shfl(v, 0, 64);
}


// Speculative VND (plain search): each product in work is handled by a group of n_nb wavefronts, one per
// neighbourhood of the list.  In every round the neighbourhoods not yet settled in the current pass are
// priced in parallel on the group's current pattern; the group's leader then walks them in list order and
// applies the first strictly improving best move; results priced after an applied move are stale and are
// priced again in the next round on the new pattern.  The moves applied, and so the result, are those of
// the sequential pass of Algorithm 1; only the consumed evaluations are counted.
struct SpecGroup {
    Bits b;               // current pattern of the group's product
    int64_t cost;         // its exact cost (kInf until the unchanged pattern of a shaken product is priced)
    int64_t c_cur;        // cost of the product in x (before the shake)
    uint64_t res[4];      // best-move key of each neighbourhood priced this round
    uint64_t ck[4];       // contrast keys for the move log
    int64_t idc;          // cost of the unchanged pattern (first round of a shaken product)
    int32_t cnt[4];       // moves priced per neighbourhood this round
    int32_t p, q, improved, active, need_ident, passes;
};

struct SpecShared {
    SpecGroup grp[kMaxWaves];
    int32_t next;         // next product index to hand out
};

template <bool SPEC, bool LEARNED, bool COOP = false, int MODEL = 0, bool PACK = false, bool MULTI = false>
__device__ __forceinline__ void run_chain(const RunArgs &a, RunShared &sh, SpecShared &sp, int2 *s_rows) {
    static_assert(!PACK || LEARNED, "the packed form is the learned VND's");
    static_assert(!(SPEC && LEARNED), "the speculative VND prices whole neighbourhoods");
    static_assert(!(COOP && SPEC), "speculative iterations run the sequential VND");
    int g = blockIdx.x, slot = 0;   // chain, and (speculative iterations) the iteration of a round it computes
    if constexpr (COOP) {
        const int m = a.coop_m;
        if (a.coop_xcd) {   // consecutive workgroups go to consecutive XCDs: keep a chain's m on one
            const int xcd = blockIdx.x & 7, w = blockIdx.x >> 3;
            g = (w / m) * 8 + xcd;
            slot = w % m;
        } else {
            g = blockIdx.x / m;
            slot = blockIdx.x % m;
        }
    }
    if constexpr (COOP) {
        // Issue priority by slot: a round always needs slot 0 and needs slot j only if iterations 0..j-1 are
        // all rejected, so on a shared SIMD the earlier slots go first and the later ones take what is left.
        // (The best-of-G form needs every slot; its streams are alike.)
        if (!a.best_of) {
            if (slot == 0)
                __builtin_amdgcn_s_setprio(3);
            else if (slot < 4)
                __builtin_amdgcn_s_setprio(2);
            else if (slot < 8)
                __builtin_amdgcn_s_setprio(1);
        }
    }
    const ChainInfo ci = a.chains[g];
    const int K = ci.K, T = ci.T;
    const int64_t cp0 = ci.cp0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int W = blockDim.x >> 6;
    const int2 *inst_rows = a.rows + a.prod[ci.prod0].row;   // an instance's rows are contiguous
    const bool rows_in_lds = K * T <= a.lds_rows;
    const int64_t it_first = *a.it0;

    if (rows_in_lds) {
        for (int i = threadIdx.x; i < K * T; i += blockDim.x) s_rows[i] = inst_rows[i];
        __syncthreads();
    }
    // the chain's solution state, indexed by product: in LDS for the whole launch when it fits (copied in
    // here and back at the end), else in device memory
    Bits *s_cur, *s_work;
    int64_t *s_cur_cost, *s_work_cost;
    if (COOP) {   // x in device memory, shared by the chain's workgroups; each iteration's VND into its slot
        const int64_t sb = ((int64_t)g * a.coop_m + slot) * a.coop_kmax;
        s_cur = a.cur + cp0;
        s_cur_cost = a.cur_cost + cp0;
        s_work = a.coop_res + sb;   // (a split round uses slot 0's region)
        s_work_cost = a.coop_res_cost + sb;
    } else if (a.state_off >= 0) {
        char *base = reinterpret_cast<char *>(s_rows) + a.state_off;
        s_cur = reinterpret_cast<Bits *>(base);
        s_work = s_cur + K;
        s_cur_cost = reinterpret_cast<int64_t *>(s_work + K);
        s_work_cost = s_cur_cost + K;
        for (int i = threadIdx.x; i < K; i += blockDim.x) {
            s_cur[i] = a.cur[cp0 + i];
            s_work[i] = a.work[cp0 + i];
            s_cur_cost[i] = a.cur_cost[cp0 + i];
            s_work_cost[i] = a.work_cost[cp0 + i];
        }
        __syncthreads();
    } else {
        s_cur = a.cur + cp0;
        s_work = a.work + cp0;
        s_cur_cost = a.cur_cost + cp0;
        s_work_cost = a.work_cost + cp0;
    }

    ChainState cs = a.cstate[g];
    int64_t evals = 0;   // per wavefront (uniform)
    int vnd_err = 0;     // per wavefront (uniform)
    int64_t nb_evals = 0, fallbacks = 0;   // learned mode, per wavefront
    // learned search: this wavefront's tiles after the rows region (kept 16-byte aligned), and the scorer's
    // weight fragments
    const int rows_entries = run_rows_entries(a.lds_rows, W);
    // (the packed form: one region for the workgroup)
    char *lbase = reinterpret_cast<char *>(s_rows + rows_entries) + (PACK ? 0 : wave * kLearnedWaveBytes);
    LearnedLds L{reinterpret_cast<__bf16 *>(lbase), reinterpret_cast<uint16_t *>(lbase + 64 * 16 * 2)};
    mlp::Frags fr;
    if constexpr (LEARNED) mlp::load_frags(a.mlp, fr);
    const uint64_t nflip_all = 2ull * (uint64_t)K * (uint64_t)T;

    int32_t coop_round = 0;   // speculative iterations: the round this workgroup computes
    int32_t coop_known = -1;  //   thread 0: the round counter as last acquired (-1: not yet)
    int64_t done_it = 0;      //   and the iterations resolved before it
    int64_t executed = 0;     //   move-evaluations this workgroup computed (thread 0)
    for (int i = 0; COOP || i < a.iters; ++i) {
        int64_t it = it_first + i;
        int kshake = cs.k;
        bool go = true;           // this workgroup has an iteration to compute in this round
        int active = 1;           // iterations computed in this round
        bool split = false;       // one iteration whose products are shared out over the chain's workgroups
        int vfirst = wave, vstep = W;   // this wavefront's products in the VND loop
        bool may_abandon = false;       // the iteration is dropped once the leader resolves the round without it
        const int64_t ev_round = evals, nb_round = nb_evals, fb_round = fallbacks;
        if constexpr (COOP) {
            // the chain's state as the leader left it.  The round counter comes first: a workgroup that
            // computed an abandoned iteration may join a round the leader has already moved past, and
            // then reads a newer state than that round's; its summary carries the older round and is
            // never used.
            if (threadIdx.x == 0) {
                sh.coop_round = coop_known >= 0 ? coop_known
                                                : __hip_atomic_load(&a.coop_ctl[g].round, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                sh.coop_cs = a.cstate[g];
                sh.coop_done_it = a.coop_ctl[g].iters_done;
                sh.coop_stop = sh.coop_done_it >= a.iters ||
                               __hip_atomic_load(&a.coop_ctl[g].abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
            cs = sh.coop_cs;
            done_it = sh.coop_done_it;
            coop_round = sh.coop_round;
            if (sh.coop_stop) break;
            // Until x is known to be a local optimum an iteration runs the VND of every product (the first
            // iteration from the initial solution is most of a short run's time): then the m workgroups
            // share that one iteration's products, which are independent (Section 3), each shaking alike
            // and writing its products' results into slot 0's region.  Otherwise each workgroup computes
            // its own iteration of the round.
            // Best-of-G: every workgroup runs the same iteration from x, shaking with its own stream (slot).
            split = !cs.lopt && !a.best_of;
            active = (split || a.best_of) ? 1 : (int)min<int64_t>(a.coop_m, a.iters - done_it);
            go = split || a.best_of || slot < active;
            it = it_first + done_it + ((split || a.best_of) ? 0 : slot);
            may_abandon = !split && !a.best_of && slot > 0;
            kshake = cs.k;   // the shake size after this workgroup's slot rejections
            for (int q = 0; q < slot && !split && !a.best_of; ++q) kshake = kshake >= a.kmax ? 1 : kshake + 1;
            const int64_t sb = ((int64_t)g * a.coop_m + (split ? 0 : slot)) * a.coop_kmax;
            s_work = a.coop_res + sb;
            s_work_cost = a.coop_res_cost + sb;
            if (split) {
                vfirst = slot * W + wave;
                vstep = a.coop_m * W;
            }
        }
        int nd = 0;
        int64_t part = 0, shk = 0;
        if (go) {

        // ---- Shake(x, k): wavefront 0 draws k flips and keeps the feasible ones in the dirty list ----
        if (wave == 0) {
            const bool draw = lane < kshake;
            const uint32_t my = draw ? shake_draw(a.seed, (uint64_t)g, (uint64_t)it, (uint64_t)lane, nflip_all,
                                                  COOP && a.best_of ? (uint64_t)slot : 0u) : 0u;
            const int pd = (int)(my / (uint32_t)(2 * T));          // lane j: product and flip slot of draw j
            const int ld = (int)(my - (uint32_t)pd * (uint32_t)(2 * T));
            bool dup = false;                                        // an earlier draw hit the same product
            for (int j = 0; j < kshake; ++j) {
                const int pj = __shfl(pd, j, 64);
                dup |= draw && j < lane && pj == pd;
            }
            int nd = 0;
            if (!__any(dup)) {
                // distinct products: the draws are independent, so each lane resolves its own and the
                // feasible ones are compacted in draw order
                bool ok = false;
                Bits b = s_cur[draw ? pd : 0];
                if (draw) {
                    apply_move(b, ld, T);
                    const ProdParams pp = a.prod[ci.prod0 + pd];
                    ok = rows_in_lds ? shake_feasible<MODEL>(b, s_rows + pd * T, T, pp)
                                     : shake_feasible<MODEL>(b, inst_rows + pd * T, T, pp);
                }
                const unsigned long long okm = __ballot(ok);
                if (ok) {
                    const int e = __popcll(okm & ((1ull << lane) - 1ull));
                    sh.dp[e] = pd;
                    sh.db[e] = b;
                }
                nd = __popcll(okm);
            } else {
                for (int j = 0; j < kshake; ++j) {
                    const uint32_t f = (uint32_t)__shfl((int)my, j, 64);
                    const int p = (int)(f / (uint32_t)(2 * T));
                    const int l = (int)(f - (uint32_t)p * (uint32_t)(2 * T));
                    int e = -1;
                    for (int q = 0; q < nd; ++q) e = (e < 0 && sh.dp[q] == p) ? q : e;
                    Bits b = e >= 0 ? sh.db[e] : s_cur[p];
                    apply_move(b, l, T);
                    const ProdParams pp = a.prod[ci.prod0 + p];
                    const bool ok = rows_in_lds ? shake_feasible<MODEL>(b, s_rows + p * T, T, pp)
                                                : shake_feasible<MODEL>(b, inst_rows + p * T, T, pp);
                    if (ok) {
                        if (e < 0) {
                            e = nd++;
                            if (lane == 0) sh.dp[e] = p;
                        }
                        if (lane == 0) sh.db[e] = b;
                    }
                    wave_sync_lds();
                }
            }
            if (lane == 0) {
                sh.nd = nd;
                sh.next_prod = W;   // wavefront w starts with product index w
            }
        }
        __syncthreads();
        nd = sh.nd;

        // ---- speculative VND: groups of n_nb wavefronts, one neighbourhood each ----
        if constexpr (SPEC) {
            const int nprod = cs.lopt ? nd : K;
            const int gsz = a.n_nb, G = W / gsz;
            const int gid = wave / gsz, role = wave - gid * gsz;
            int staged = -1;   // product whose row this wavefront holds in its LDS slice (uniform)
            // hands the group its next product (one lane)
            auto take = [&](SpecGroup &gr) {
                const int idx = atomicAdd(&sp.next, 1);
                if (idx >= nprod) {
                    gr.active = 0;
                    return;
                }
                int p, e = -1;
                if (cs.lopt) {
                    p = sh.dp[idx];
                    e = idx;
                } else {
                    p = idx;
                    for (int q = 0; q < nd; ++q) e = (e < 0 && sh.dp[q] == p) ? q : e;
                }
                gr.p = p;
                gr.b = e >= 0 ? sh.db[e] : s_cur[p];
                gr.c_cur = s_cur_cost[p];
                gr.cost = e >= 0 ? kInf : gr.c_cur;
                gr.need_ident = e >= 0;
                gr.q = 0;
                gr.improved = 0;
                gr.passes = 0;
                gr.active = 1;
            };
            if (threadIdx.x == 0) sp.next = 0;
            __syncthreads();
            if (gid < G && role == 0 && lane == 0) take(sp.grp[gid]);
            __syncthreads();
            for (;;) {
                bool any = false;
                for (int gg = 0; gg < G; ++gg) any |= sp.grp[gg].active != 0;
                if (!any) break;
                // pricing: every neighbourhood not settled in this pass, on the group's current pattern
                if (gid < G && sp.grp[gid].active && role >= sp.grp[gid].q) {
                    SpecGroup &gr = sp.grp[gid];
                    const int p = gr.p;
                    const ProdParams pp = a.prod[ci.prod0 + p];
                    const int2 *row;
                    if (rows_in_lds) {
                        row = s_rows + p * T;
                    } else {
                        int2 *slice = s_rows + wave * kTMax;
                        if (staged != p) {
                            for (int t = lane; t < T; t += 64) slice[t] = inst_rows[p * T + t];
                            wave_sync_lds();
                            staged = p;
                        }
                        row = slice;
                    }
                    const uint32_t nb = (a.nb_list >> (4 * role)) & 0xFu;
                    const bool id = gr.need_ident && role == gr.q;
                    const int chash = a.log_x ? (int)(((uint32_t)it * 2654435761u + (uint32_t)p * 40503u +
                                                       (uint32_t)(role + 4 * gr.passes) * 97u) & 0x7FFFFFFFu) : -1;
                    int64_t idc = 0, dummy = 0;
                    uint64_t ckey = kInfKey;
                    int nitems = 0;
                    const Bits b = gr.b;
                    const uint64_t key = wave_best_move(b, row, T, pp, nb, sh.list[wave], id, &idc, dummy, chash, &ckey,
                                                        &nitems);
                    if (lane == 0) {
                        gr.res[role] = key;
                        gr.ck[role] = ckey;
                        gr.cnt[role] = nitems;
                        if (id) gr.idc = idc;
                    }
                }
                __syncthreads();
                // resolution in list order by the group's leader lane
                if (gid < G && role == 0 && lane == 0 && sp.grp[gid].active) {
                    SpecGroup &gr = sp.grp[gid];
                    if (gr.need_ident) {
                        gr.cost = gr.idc;
                        shk += gr.idc - gr.c_cur;
                        gr.need_ident = 0;
                    }
                    bool applied = false;
                    for (int j = gr.q; j < gsz; ++j) {
                        evals += gr.cnt[j];
                        const uint64_t key = gr.res[j];
                        if (key != kInfKey && (int64_t)(key >> kSlotBits) < gr.cost) {
                            const int slot = (int)(key & ((1u << kSlotBits) - 1));
                            const int64_t c = (int64_t)(key >> kSlotBits);
                            if (a.log_x) {
                                const ProdParams pp = a.prod[ci.prod0 + gr.p];
                                const uint64_t ck = gr.ck[j];
                                const bool has_c = ck != kInfKey && ck != key;
                                const int2 *row = rows_in_lds ? s_rows + gr.p * T : inst_rows + gr.p * T;
                                log_moves(gr.b, row, T, pp, slot, c - gr.cost, has_c ? (int)(ck & 0xFFFFu) : -1,
                                          has_c ? (int64_t)(ck >> kSlotBits) - gr.cost : 0, a.log_x, a.log_y, a.log_n,
                                          a.log_cap);
                            }
                            apply_move(gr.b, slot, T);
                            gr.cost = c;
                            gr.improved = 1;
                            gr.q = j + 1;
                            applied = true;
                            break;
                        }
                    }
                    if (!applied || gr.q == gsz) {   // the pass is over
                        if (gr.improved && ++gr.passes <= kMaxPasses) {
                            gr.q = 0;
                            gr.improved = 0;
                        } else {
                            if (gr.improved) vnd_err = 1;
                            s_work[gr.p] = gr.b;
                            s_work_cost[gr.p] = gr.cost;
                            part += gr.cost - gr.c_cur;
                            take(gr);
                        }
                    }
                }
                __syncthreads();
            }
        } else {
            // ---- VND (Algorithm 1) per product: the shaken products, or every product until x is known to
            //      be a local optimum ----
            const int nprod = cs.lopt ? nd : K;
            bool stale = false;   // the round moved on without this iteration (uniform)
            // Products go to wavefronts as they finish (a product's VND length varies, and a shake of more
            // products than wavefronts would otherwise put two on one wavefront however short the others
            // are); the products of a split round are shared out over the chain's workgroups in fixed order.
            const bool dyn = vstep == W;
            if constexpr (PACK) {
                // the packed learned VND: batches of up to P products, each searched by the whole workgroup
                // (a split round's batches shared out over the chain's workgroups in fixed order)
                const int P = a.learned_pack;
                const PackLds PL = pack_lds(lbase, W, P);
                auto round_now = [&]() -> int32_t {
                    if constexpr (COOP) {
                        if (may_abandon)
                            return __hip_atomic_load(&a.coop_ctl[g].round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    return coop_round;
                };
                const int bfirst = dyn ? 0 : vfirst / W, bstep = dyn ? 1 : vstep / W;   // in batches
                for (int base = bfirst * P; base < nprod && !stale; base += bstep * P) {
                    const int cnt = min(P, nprod - base);
                    if (threadIdx.x == 0) {
                        for (int i = 0; i < cnt; ++i) {
                            const int idx = base + i;
                            int p, e = -1;
                            if (cs.lopt) {
                                p = sh.dp[idx];
                                e = idx;
                            } else {
                                p = idx;
                                for (int q = 0; q < nd; ++q) e = (e < 0 && sh.dp[q] == p) ? q : e;
                            }
                            PackProd &pr = PL.pk[i];
                            pr.p = p;
                            pr.b = e >= 0 ? sh.db[e] : s_cur[p];
                            pr.c_cur = s_cur_cost[p];
                            pr.cost = e >= 0 ? kInf : pr.c_cur;   // a shaken product is priced with its first list
                            pr.need_ident = e >= 0 ? 1 : 0;
                        }
                    }
                    __syncthreads();
                    if (!learned_vnd_packed(PL, cnt, rows_in_lds ? s_rows : nullptr, inst_rows, a.prod + ci.prod0, T,
                                            a.nb_list, a.n_nb, a.memo, fr, a.permille, evals, nb_evals, fallbacks,
                                            coop_round, round_now)) {
                        stale = true;
                        break;
                    }
                    for (int i = 0; i < cnt; ++i) {
                        const PackProd &pr = PL.pk[i];
                        if (threadIdx.x == 0) {
                            s_work[pr.p] = pr.b;
                            s_work_cost[pr.p] = pr.cost;
                        }
                        if (wave == 0) {   // the per-wavefront sums, once
                            part += pr.cost - pr.c_cur;
                            shk += pr.shk;
                            vnd_err |= pr.err;
                        }
                    }
                    __syncthreads();
                }
            } else {
            for (int idx = vfirst; idx < nprod && !stale;
                 idx = dyn ? __builtin_amdgcn_readfirstlane(next_index(sh.next_prod, lane)) : idx + vstep) {
                int p, e = -1;
                if (cs.lopt) {
                    p = sh.dp[idx];
                    e = idx;
                } else {
                    p = idx;
                    for (int q = 0; q < nd; ++q) e = (e < 0 && sh.dp[q] == p) ? q : e;
                }
                const ProdParams pp = a.prod[ci.prod0 + p];
                const int2 *row;
                if (rows_in_lds) {
                    row = s_rows + p * T;
                } else {
                    int2 *slice = s_rows + wave * kTMax;
                    for (int t = lane; t < T; t += 64) slice[t] = inst_rows[p * T + t];
                    wave_sync_lds();
                    row = slice;
                }
                Bits b = e >= 0 ? sh.db[e] : s_cur[p];
                const int64_t c_cur = s_cur_cost[p];
                int64_t cost = e >= 0 ? kInf : c_cur;   // a shaken product is priced with its first move list
                bool need_ident = e >= 0;
                bool improved = true;
                int passes = 0;
                uint32_t clean = 0;   // neighbourhoods priced without improvement since the last applied move
                // short horizons: consecutive neighbourhoods priced side by side in one pass when they fit 64 lanes
                // (a kernel of its own, so that the others keep their registers)
                const bool multi = MULTI && !a.log_x && !a.memo && T <= kMultiMaxT;
                while (improved && !stale) {
                    if (++passes > kMaxPasses) {
                        vnd_err = 1;
                        break;
                    }
                    improved = false;
                    for (int q = 0; q < a.n_nb;) {
                        if (multi) {
                            int32_t rnow = coop_round;
                            if constexpr (COOP) {
                                if (may_abandon)
                                    rnow = __hip_atomic_load(&a.coop_ctl[g].round, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                            }
                            int used = 1;
                            const bool id = need_ident;
                            const uint64_t key = wave_best_move_multi<2, MODEL>(b, row, T, pp, a.nb_list, q, a.n_nb,
                                                                                sh.list[wave], id, cost, evals, used);
                            if (id) {
                                shk += cost - c_cur;
                                need_ident = false;
                            }
                            if (key != kInfKey) {   // improving by construction
                                apply_move(b, (int)(key & ((1u << kSlotBits) - 1)), T);
                                cost = (int64_t)(key >> kSlotBits);
                                improved = true;
                            }
                            q += used;
                            wave_sync_lds();
                            if (__builtin_amdgcn_readfirstlane(rnow) != coop_round) {
                                stale = true;
                                break;
                            }
                            continue;
                        }
                        if (a.memo && ((clean >> q) & 1u)) {   // same pattern: nothing to find
                            ++q;
                            continue;
                        }
                        // the round counter, read before the evaluation and looked at after it, so that the
                        // load's latency is hidden behind the pricing
                        int32_t rnow = coop_round;
                        if constexpr (COOP) {
                            if (may_abandon)
                                rnow = __hip_atomic_load(&a.coop_ctl[g].round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                        bool applied = false;
                        const uint32_t nb = (a.nb_list >> (4 * q)) & 0xFu;
                        uint64_t key, ckey = kInfKey;
                        int nitems = 0;
                        // contrast move for the log: a fixed pseudo-random item of this evaluation
                        const int chash = a.log_x ? (int)(((uint32_t)it * 2654435761u + (uint32_t)p * 40503u +
                                                           (uint32_t)(q + 4 * passes) * 97u) & 0x7FFFFFFFu) : -1;
                        if constexpr (LEARNED) {
                            int fb = 0;
                            const bool id = need_ident;
                            key = learned_best_move(b, row, T, pp, nb, sh.list[wave], L, fr, a.permille, id, cost,
                                                    evals, fb);
                            ++nb_evals;
                            fallbacks += fb;
                            if (id) {
                                shk += cost - c_cur;
                                need_ident = false;
                            }
                        } else {
                            int64_t idc = 0;
                            key = wave_best_move<MODEL>(b, row, T, pp, nb, sh.list[wave], need_ident, &idc, evals, chash,
                                                        &ckey,
                                                 &nitems);
                            if (need_ident) {
                                cost = idc;
                                shk += idc - c_cur;
                                need_ident = false;
                            }
                        }
                        if (key != kInfKey) {
                            const int64_t c = (int64_t)(key >> kSlotBits);
                            if (c < cost) {
                                const int slot = (int)(key & ((1u << kSlotBits) - 1));
                                if (!LEARNED && a.log_x) {
                                    const bool has_c = ckey != kInfKey && ckey != key;
                                    log_moves(b, row, T, pp, slot, c - cost, has_c ? (int)(ckey & 0xFFFFu) : -1,
                                              has_c ? (int64_t)(ckey >> kSlotBits) - cost : 0, a.log_x, a.log_y, a.log_n,
                                              a.log_cap);
                                }
                                apply_move(b, slot, T);
                                cost = c;
                                improved = true;
                                applied = true;
                            }
                        }
                        // a move changes the pattern: every earlier pricing is stale
                        clean = applied ? 0u : (clean | (1u << q));
                        ++q;
                        wave_sync_lds();
                        if (__builtin_amdgcn_readfirstlane(rnow) != coop_round) {
                            stale = true;
                            break;
                        }
                    }
                }
                if (stale) break;
                if (lane == 0) {
                    s_work[p] = b;
                    s_work_cost[p] = cost;
                }
                part += cost - c_cur;
            }
            }
        }
        }   // go
        if (lane == 0) {
            sh.part[wave] = part;
            sh.shk[wave] = shk;
            if constexpr (COOP) {
                sh.ev[wave] = evals - ev_round;
                sh.verr[wave] = vnd_err;
                sh.nbr[wave] = nb_evals - nb_round;
                sh.fbr[wave] = fallbacks - fb_round;
            }
        }
        __syncthreads();

        if constexpr (COOP) {
            CoopCtl *ctl = a.coop_ctl + g;
            CoopSlot *mine = a.coop_slot + (int64_t)g * a.coop_m + slot;
            if (go && threadIdx.x == 0) {   // this iteration's summary
                int64_t delta = 0, dshake = 0, ev = 0, nbe = 0, fbe = 0;
                int err = 0;
                for (int w = 0; w < W; ++w) {
                    delta += sh.part[w];
                    dshake += sh.shk[w];
                    ev += sh.ev[w];
                    err |= sh.verr[w];
                    nbe += sh.nbr[w];
                    fbe += sh.fbr[w];
                }
                executed += ev;
                mine->F_local = cs.F + delta;
                mine->F_shaken = cs.F + dshake;
                mine->evals = ev;
                mine->nb_evals = nbe;
                mine->fallbacks = fbe;
                mine->err = err;
                mine->n_touch = cs.lopt ? nd : -1;   // -1: every product
                for (int q = 0; q < nd; ++q) mine->dp[q] = sh.dp[q];
            }
            // the VND results (written by every wavefront) and the summary, before the stamp: each wavefront's
            // stores completed, then one agent-scope release (it writes back the XCD's L2, whoever stored)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __syncthreads();
            if (go && threadIdx.x == 0)
                __hip_atomic_store(&mine->stamp, coop_round + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (slot == 0) {
                // the leader resolves the round in iteration order: the first accepted iteration ends it, so
                // it waits only for the slots up to that one (a split or best-of round needs all of them).
                // Wavefront 0 polls the m stamps side by side (lane j: slot j), loads each summary once its
                // slot and every earlier one have reported, and resolves them with wave-uniform arithmetic;
                // lane 0 writes.
                if (wave == 0) {
                    const int need = (split || a.best_of) ? a.coop_m : active;   // slots holding this round
                    const CoopSlot *sj = a.coop_slot + (int64_t)g * a.coop_m + min(lane, a.coop_m - 1);
                    int64_t dl = 0, ds = 0, le = 0;   // lane j: slot j's F_local - F, F_shaken - F, evaluations
                    int64_t lnb = 0, lfb = 0;          //   and its learned counters
                    int lerr = 0;
                    int have = 0;                      // leading slots whose summaries are loaded (uniform)
                    bool ok = true;
                    const int64_t t0 = wall_clock64();
                    for (uint32_t n = 0;; ++n) {
                        const int32_t st =
                            lane < need ? __hip_atomic_load(&sj->stamp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
                        const unsigned long long rdy = __ballot(lane < need && st == coop_round + 1);
                        const int r = (int)__builtin_ctzll(~rdy);   // need <= 16, so ~rdy has a zero bit
                        if (r > have) {
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the summaries behind the stamps
                            if (lane >= have && lane < r) {
                                dl = sj->F_local - cs.F;
                                ds = sj->F_shaken - cs.F;
                                le = sj->evals;
                                lerr = sj->err;
                                lnb = sj->nb_evals;
                                lfb = sj->fallbacks;
                            }
                            have = r;
                        }
                        if (have >= need) break;
                        // no earlier iteration of the round is accepted, so iteration j is accepted when its
                        // local cost is below F
                        if (!(split || a.best_of) && __ballot(lane < have && dl < 0)) break;
                        if (n >= kCoopSpinLimit || wall_clock64() - t0 > a.coop_wait_ticks) {
                            ok = false;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                    if (split) {   // the one iteration is the sum of every slot's share
                        dl = wave_sum_i64(dl);
                        ds = wave_sum_i64(ds);
                        le = wave_sum_i64(le);
                        lnb = wave_sum_i64(lnb);
                        lfb = wave_sum_i64(lfb);
                        lerr = __any(lerr != 0) ? 1 : 0;
                    }
                    int sel = 0;   // best-of-G: the stream whose result is kept
                    if (a.best_of) {
                        // the minimum local cost over the G streams, the lowest stream among equal values; every
                        // stream's evaluations count
                        const bool mine = ok && lane < a.coop_m;
                        const uint64_t myF = mine ? (uint64_t)(cs.F + dl) : ~0ull;
                        const uint64_t minF = wave_min_u64(myF);
                        const unsigned long long at = __ballot(mine && myF == minF);
                        sel = at ? (int)__builtin_ctzll(at) : 0;
                        dl = __shfl(dl, sel, 64);
                        ds = __shfl(ds, sel, 64);
                        le = wave_sum_i64(le);
                        lnb = wave_sum_i64(lnb);
                        lfb = wave_sum_i64(lfb);
                        lerr = __any(lerr != 0) ? 1 : 0;
                    }
                    const bool literal = a.best_of && a.best_literal;   // k fixed, the minimum always kept
                    int acc = -1, consumed = active, k = cs.k, err = ok ? 0 : 2;
                    int64_t F = cs.F, Fb = cs.F_best, ev = 0, nbe = 0, fbe = 0;
                    for (int j = 0; j < active && ok; ++j) {
                        const int64_t Fl = cs.F + __shfl(dl, j, 64), Fs = cs.F + __shfl(ds, j, 64);
                        ev += __shfl(le, j, 64);
                        nbe += __shfl(lnb, j, 64);
                        fbe += __shfl(lfb, j, 64);
                        err |= __shfl(lerr, j, 64);
                        const int accepted = literal ? 1 : Fl < F;
                        if (a.trace && lane == 0) {
                            Record r;
                            r.iter = (int32_t)(it_first + done_it + j);
                            r.k = k;
                            r.accepted = accepted;
                            r.winner = sel;
                            r.F_shaken = Fs;
                            r.F_local = Fl;
                            r.F_best = (accepted && Fl < Fb) ? Fl : Fb;
                            a.trace[(int64_t)g * a.iters + done_it + j] = r;
                        }
                        if (accepted) {
                            acc = a.best_of ? sel : j;   // the slot whose VND results x takes
                            consumed = j + 1;
                            F = Fl;
                            Fb = Fl < Fb ? Fl : Fb;
                            k = literal ? k : 1;
                            break;
                        }
                        k = k >= a.kmax ? 1 : k + 1;
                    }
                    // the best solution follows x when x becomes the cheapest so far: the accepted products
                    // when it held x before, all of x otherwise (x had moved to a worse solution)
                    const int bmode = (ok && acc >= 0 && F < cs.F_best) ? (cs.bsync ? 1 : 2) : 0;
                    if (lane == 0) {
                        sh.coop_acc = ok ? acc : -1;
                        sh.coop_abort = !ok;
                        sh.coop_bmode = bmode;
                        if (ok) {
                            cs.F = F;
                            cs.F_best = Fb;
                            cs.k = k;
                            cs.bsync = bmode ? 1 : (acc >= 0 ? 0 : cs.bsync);
                            if (acc >= 0) cs.lopt = 1;
                            ctl->iters_done = done_it + consumed;
                            ctl->evals += ev;
                            ctl->nb_evals += nbe;
                            ctl->fallbacks += fbe;
                        }
                        if (err) atomicOr(&ctl->err, err);
                    }
                }
                // (wavefront 0's acquires after the stamps invalidated the caches the compute unit reads
                // through; the barrier orders every thread's reads of the results after them)
                __syncthreads();
                const int acc = sh.coop_acc, bmode = sh.coop_bmode;
                if (acc >= 0) {   // x takes the accepted iteration's VND results
                    const CoopSlot *sj = a.coop_slot + (int64_t)g * a.coop_m + acc;
                    const int64_t sb = ((int64_t)g * a.coop_m + acc) * a.coop_kmax;
                    const int n = sj->n_touch < 0 ? K : sj->n_touch;
                    for (int q = threadIdx.x; q < n; q += blockDim.x) {
                        const int p = sj->n_touch < 0 ? q : sj->dp[q];
                        const Bits b = a.coop_res[sb + p];
                        a.cur[cp0 + p] = b;
                        a.cur_cost[cp0 + p] = a.coop_res_cost[sb + p];
                        if (bmode == 1) a.best[cp0 + p] = b;
                    }
                }
                if (bmode == 2) {
                    __syncthreads();
                    for (int q = threadIdx.x; q < K; q += blockDim.x) a.best[cp0 + q] = a.cur[cp0 + q];
                }
                // every wavefront's stores to x completed, then one agent-scope release with the round count
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __syncthreads();
                if (threadIdx.x == 0) {
                    a.cstate[g] = cs;
                    if (sh.coop_abort) ctl->abort = 1;
                    __hip_atomic_fetch_add(&ctl->round, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    coop_known = coop_round + 1;
                }
            } else if (threadIdx.x == 0) {
                // (the wait's acquire invalidates the caches the whole compute unit reads through; the barrier
                // then orders the workgroup's later reads of x after it)
                if (!coop_wait_ge(&ctl->round, coop_round + 1, a.coop_wait_ticks, &coop_known)) {
                    __hip_atomic_store(&ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    atomicOr(&ctl->err, 2);
                    coop_known = -1;
                }
            }
            __syncthreads();
            continue;
        }

        // ---- acceptance ----
        int64_t delta = 0, dshake = 0;
        for (int w = 0; w < W; ++w) {
            delta += sh.part[w];
            dshake += sh.shk[w];
        }
        const int64_t F_local = cs.F + delta;
        const int accepted = F_local < cs.F;
        // the best solution follows x when x becomes the cheapest so far: the touched products when it held
        // x before, all of x otherwise
        const int bmode = (accepted && F_local < cs.F_best) ? (cs.bsync ? 1 : 2) : 0;
        const int ntouch = cs.lopt ? nd : K;
        for (int idx = threadIdx.x; idx < ntouch; idx += blockDim.x) {
            const int p = cs.lopt ? sh.dp[idx] : idx;
            if (accepted) {
                s_cur[p] = s_work[p];
                s_cur_cost[p] = s_work_cost[p];
                if (bmode == 1) a.best[cp0 + p] = s_work[p];
            } else {
                s_work[p] = s_cur[p];
                s_work_cost[p] = s_cur_cost[p];
            }
        }
        if (a.trace && threadIdx.x == 0) {
            Record r;
            r.iter = (int32_t)it;
            r.k = kshake;
            r.accepted = accepted;
            r.winner = 0;
            r.F_shaken = cs.F + dshake;
            r.F_local = F_local;
            r.F_best = (accepted && F_local < cs.F_best) ? F_local : cs.F_best;
            a.trace[(int64_t)g * a.iters + i] = r;
        }
        if (bmode == 2) {
            __syncthreads();
            for (int q = threadIdx.x; q < K; q += blockDim.x) a.best[cp0 + q] = s_cur[q];
        }
        if (accepted) {
            cs.F = F_local;
            cs.k = 1;
            cs.lopt = 1;
            cs.bsync = bmode ? 1 : 0;
        } else {
            cs.k = cs.k >= a.kmax ? 1 : cs.k + 1;
        }
        cs.F_best = cs.F < cs.F_best ? cs.F : cs.F_best;
        __syncthreads();
    }

    if constexpr (COOP) {
        CoopCtl *ctl = a.coop_ctl + g;
        if (slot == 0) {   // the leader: this launch's counters, and work == cur for the other search kernels
            __syncthreads();
            for (int q = threadIdx.x; q < K; q += blockDim.x) {
                a.work[cp0 + q] = a.cur[cp0 + q];
                a.work_cost[cp0 + q] = a.cur_cost[cp0 + q];
            }
            if (threadIdx.x == 0) {
                cs.evals = ctl->evals;
                cs.discarded = 0;
                cs.err |= ctl->err;
                cs.nb_evals = ctl->nb_evals;
                cs.fallbacks = ctl->fallbacks;
                a.cstate[g] = cs;
            }
        }
        // the last workgroup of the chain to leave records the move-evaluations computed and not consumed
        // (the iterations after an accepted one, finished or abandoned), and any error a slot raised
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(&ctl->executed, executed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int32_t n = __hip_atomic_fetch_add(&ctl->exited, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (n == a.coop_m - 1) {
                const int64_t ex = __hip_atomic_load(&ctl->executed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                a.cstate[g].discarded = ex - ctl->evals;
                a.cstate[g].err |= __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        return;
    }
    if (a.state_off >= 0) {   // every iteration ended with a barrier
        for (int i = threadIdx.x; i < K; i += blockDim.x) {
            a.cur[cp0 + i] = s_cur[i];
            a.work[cp0 + i] = s_work[i];
            a.cur_cost[cp0 + i] = s_cur_cost[i];
            a.work_cost[cp0 + i] = s_work_cost[i];
        }
    }
    if (lane == 0) {
        sh.ev[wave] = evals;
        sh.part[wave] = vnd_err;
        sh.shk[wave] = nb_evals;
        sh.fb[wave] = fallbacks;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t e = 0, ne = 0, nf = 0;
        int32_t err = 0;
        for (int w = 0; w < W; ++w) {
            e += sh.ev[w];
            err |= (int32_t)sh.part[w];
            ne += sh.shk[w];
            nf += sh.fb[w];
        }
        cs.evals = e;
        cs.err |= err;
        cs.nb_evals = ne;
        cs.fallbacks = nf;
        cs.discarded = 0;
        a.cstate[g] = cs;
    }
}

}  // namespace

template <int MODEL>
__global__ __launch_bounds__(512) void k_run(RunArgs a) {
    __shared__ RunShared sh;
    __shared__ SpecShared sp;
    extern __shared__ __attribute__((aligned(16))) int2 s_rows[];
    run_chain<false, false, false, MODEL>(a, sh, sp, s_rows);
}

// The same for batches with short horizons (up to kMultiMaxT): consecutive neighbourhoods priced side by side.
// Bounded to 128 registers: four wavefronts per SIMD for every decode reading.
template <int MODEL>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_run_short(RunArgs a) {
    __shared__ RunShared sh;
    __shared__ SpecShared sp;
    extern __shared__ __attribute__((aligned(16))) int2 s_rows[];
    run_chain<false, false, false, MODEL, false, true>(a, sh, sp, s_rows);
}

__global__ __launch_bounds__(1024) void k_run_spec(RunArgs a) {
    __shared__ RunShared sh;
    __shared__ SpecShared sp;
    extern __shared__ __attribute__((aligned(16))) int2 s_rows[];
    run_chain<true, false>(a, sh, sp, s_rows);
}

// speculative iterations: m workgroups per chain compute the next m iterations side by side (cooperative
// launch: every workgroup of a chain is resident while it waits for the others)
template <int MODEL>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3))) void k_run_coop(RunArgs a) {
    __shared__ RunShared sh;
    __shared__ SpecShared sp;
    extern __shared__ __attribute__((aligned(16))) int2 s_rows[];
    run_chain<false, false, true, MODEL>(a, sh, sp, s_rows);
}

// learned VND: the scorer's weight fragments stay in registers for the whole launch
// speculative iterations of the learned search
__global__ __launch_bounds__(512) void k_run_learned_coop(RunArgs a) {
    __shared__ RunShared sh;
    __shared__ SpecShared sp;
    extern __shared__ __attribute__((aligned(16))) int2 s_rows[];
    run_chain<false, true, true>(a, sh, sp, s_rows);
}

__global__ __launch_bounds__(512) void k_run_learned(RunArgs a) {
    __shared__ RunShared sh;
    __shared__ SpecShared sp;
    extern __shared__ __attribute__((aligned(16))) int2 s_rows[];
    run_chain<false, true>(a, sh, sp, s_rows);
}

// the packed learned VND (batches of products per wavefront), alone and with speculative iterations
__global__ __launch_bounds__(512) void k_run_learned_packed(RunArgs a) {
    __shared__ RunShared sh;
    __shared__ SpecShared sp;
    extern __shared__ __attribute__((aligned(16))) int2 s_rows[];
    run_chain<false, true, false, 0, true>(a, sh, sp, s_rows);
}

__global__ __launch_bounds__(512) void k_run_learned_coop_packed(RunArgs a) {
    __shared__ RunShared sh;
    __shared__ SpecShared sp;
    extern __shared__ __attribute__((aligned(16))) int2 s_rows[];
    run_chain<false, true, true, 0, true>(a, sh, sp, s_rows);
}

// ---------------------------------------------------------------------------------------------------
// k_eval_learned: one wavefront per (chain, product) of a chain range: the learned choice of one
// neighbourhood's move for the current solution, with the scores and the selection of every move.
// ---------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_eval_learned(EvalLearnedArgs a, int64_t cp_begin) {
    __shared__ int2 s_row[kTMax];
    __shared__ uint16_t s_list[2 * kTMax];
    __shared__ uint16_t s_sel[2 * kTMax];
    __shared__ __attribute__((aligned(16))) __bf16 s_x[64 * 16];   // read as 16-byte vectors
    const int64_t cp = cp_begin + blockIdx.x;
    const int g = a.cp_chain[cp];
    const ChainInfo ci = a.chains[g];
    const int T = ci.T;
    const int p = (int)(cp - ci.cp0);
    const ProdParams pp = a.prod[ci.prod0 + p];
    for (int t = threadIdx.x; t < T; t += 64) s_row[t] = a.rows[pp.row + t];
    wave_sync_lds();
    mlp::Frags fr;
    mlp::load_frags(a.mlp, fr);
    const Bits b = a.cur[cp];
    int64_t cost = a.cur_cost[cp], evals = 0;
    int fb = 0;
    const int64_t off = a.slot_off[g] + (int64_t)p * 4 * T;
    LearnedLds L{s_x, s_sel};
    const uint64_t key = learned_best_move(b, s_row, T, pp, a.nb, s_list, L, fr, a.permille, false, cost, evals,
                                           fb, a.scores ? a.scores + off : nullptr, a.selected ? a.selected + off : nullptr);
    if (threadIdx.x == 0) {
        const int64_t F = a.cstate[g].F;
        a.prod_price[cp] = key == kInfKey ? kInf : F - cost + (int64_t)(key >> kSlotBits);
        a.prod_slot[cp] = key == kInfKey ? -1 : (int32_t)(key & 0xFFFFu);
        a.fallback[cp] = (uint8_t)fb;
        atomicAdd(a.evals + (size_t)(blockIdx.x & (kCounterSlots - 1)) * kCounterStride, (unsigned long long)evals);
    }
}

// k_advance: the iteration counter moves on once every chain of the launch has read it.
__global__ void k_advance(int64_t *it, int32_t iters) { *it += iters; }

// ---------------------------------------------------------------------------------------------------
// Host-side launchers (called by the runtime).
// ---------------------------------------------------------------------------------------------------
// One instantiation per decode reading (kModelStrict | kModelDispose).
template <template <int> class Pick>
static const void *by_model(int model) {
    switch (model) {
        case 1: return Pick<1>::fn();
        case 2: return Pick<2>::fn();
        case 3: return Pick<3>::fn();
        default: return Pick<0>::fn();
    }
}
template <int M> struct PickInit { static const void *fn() { return reinterpret_cast<const void *>(&k_init_costs<M>); } };
template <int M> struct PickEval { static const void *fn() { return reinterpret_cast<const void *>(&k_eval<M>); } };
template <int M> struct PickEvalWide {
    static const void *fn() { return reinterpret_cast<const void *>(&k_eval_wide<M>); }
};
template <int M> struct PickRun { static const void *fn() { return reinterpret_cast<const void *>(&k_run<M>); } };
template <int M> struct PickRunShort {
    static const void *fn() { return reinterpret_cast<const void *>(&k_run_short<M>); }
};
template <int M> struct PickCoop { static const void *fn() { return reinterpret_cast<const void *>(&k_run_coop<M>); } };

hipError_t launch_init(const InitArgs &a, int n_chains, hipStream_t s, int model) {
    if (n_chains <= 0) return hipSuccess;
    InitArgs args = a;
    void *params[] = {&args};
    return hipLaunchKernel(by_model<PickInit>(model), dim3(n_chains), dim3(256), params, 0, s);
}

hipError_t launch_eval(const EvalArgs &a, const EvalWg *wg, int64_t n_wg, hipStream_t s, int model, int waves) {
    if (n_wg <= 0) return hipSuccess;
    if (waves != 4 && waves != 8 && waves != 12 && waves != 16) return hipErrorInvalidValue;
    EvalArgs args = a;
    const EvalWg *w = wg;
    void *params[] = {&args, &w};
    const void *fn = waves == 4 ? by_model<PickEval>(model) : by_model<PickEvalWide>(model);
    return hipLaunchKernel(fn, dim3((unsigned)n_wg), dim3(64 * waves), params, 0, s);
}

hipError_t launch_eval_prep(const EvalPrepArgs &a, hipStream_t s) {
    const int64_t n = std::max<int64_t>(a.n_cp, counter_words());
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_eval_prep, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_eval_inc(const EvalArgs &a, const EvalWg *wg, int64_t n_wg, size_t lds_bytes, hipStream_t s) {
    if (n_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eval_inc, dim3((unsigned)n_wg), dim3(256), lds_bytes, s, a, wg);
    return hipGetLastError();
}

hipError_t launch_chain_best(const ChainBestArgs &a, int n_chains, hipStream_t s) {
    if (n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chain_best, dim3(n_chains), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_eval_learned(const EvalLearnedArgs &a, int64_t cp_begin, int64_t n_cp, hipStream_t s) {
    if (n_cp <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eval_learned, dim3((unsigned)n_cp), dim3(64), 0, s, a, cp_begin);
    return hipGetLastError();
}

static const void *run_kernel(RunKind kind, int model) {
    switch (kind) {
        case RunKind::kSpec: return reinterpret_cast<const void *>(&k_run_spec);
        case RunKind::kLearned: return reinterpret_cast<const void *>(&k_run_learned);
        case RunKind::kLearnedPacked: return reinterpret_cast<const void *>(&k_run_learned_packed);
        case RunKind::kPlainShort: return by_model<PickRunShort>(model);
        default: return by_model<PickRun>(model);
    }
}

hipError_t run_kernel_lds(RunKind kind, size_t *static_bytes, size_t dynamic_bytes, int model) {
    const void *fn = run_kernel(kind, model);
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    *static_bytes = fa.sharedSizeBytes;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dynamic_bytes);
}

static const void *coop_kernel(RunKind kind, int model) {
    if (kind == RunKind::kLearned) return reinterpret_cast<const void *>(&k_run_learned_coop);
    if (kind == RunKind::kLearnedPacked) return reinterpret_cast<const void *>(&k_run_learned_coop_packed);
    return by_model<PickCoop>(model);
}

hipError_t coop_fits(int waves, size_t lds_bytes, int64_t blocks, bool *fits, RunKind kind, int model) {
    *fits = false;
    const void *fn = coop_kernel(kind, model);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    int per_cu = 0, dev = 0, cus = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * waves, lds_bytes);
    if (e != hipSuccess) return e;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    *fits = (int64_t)per_cu * cus >= blocks;
    return hipSuccess;
}

hipError_t launch_run_coop(const RunArgs &a, int n_chains, int waves, size_t lds_bytes, int64_t *it_counter,
                           hipStream_t s, RunKind kind, int model) {
    if (n_chains <= 0 || a.iters <= 0) return hipSuccess;
    RunArgs args = a;
    void *params[] = {&args};
    hipError_t e = hipLaunchCooperativeKernel(coop_kernel(kind, model),
                                              dim3((unsigned)(n_chains * a.coop_m)), dim3(64 * waves), params,
                                              (unsigned)lds_bytes, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, it_counter, a.iters);
    return hipGetLastError();
}

hipError_t launch_run(const RunArgs &a, RunKind kind, int n_chains, int waves, size_t lds_bytes, int64_t *it_counter,
                      hipStream_t s, int model) {
    if (n_chains <= 0 || a.iters <= 0) return hipSuccess;
    RunArgs args = a;
    void *params[] = {&args};
    hipError_t e = hipLaunchKernel(run_kernel(kind, model), dim3(n_chains), dim3(64 * waves), params, lds_bytes, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, it_counter, a.iters);
    return hipGetLastError();
}

}  // namespace vns
