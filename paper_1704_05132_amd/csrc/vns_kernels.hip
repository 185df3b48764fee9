// Kernels of the lot-sizing VNS for gfx950.
//
//   k_init_costs    exact cost of every (chain, product) of the current solutions; F per chain
//   k_eval          one workgroup per (chain, product), one lane per move: exact price of every move of the
//                   selected neighbourhoods and the product's best move (Section 3: the new objective value
//                   of each product is computed independently of the others)
//   k_chain_best    per chain: lexicographic (price, slot) minimum over its products
//   k_run           one workgroup per chain running whole GVNS iterations (Algorithm 2): Philox shake,
//                   VND (Algorithm 1) with one wavefront per product that needs it, acceptance
#include <hip/hip_runtime.h>

#include "vns_device.hpp"
#include "vns_launch.hpp"

namespace vns {

namespace {

// Neighbourhood mask -> ordered list of slot blocks (0 flip zM, 1 flip zR, 2 swap zM, 3 swap zR), packed
// 8 bits per entry so that it stays in a scalar register.  Returns the number of blocks.
__device__ __forceinline__ int blocks_of(uint32_t nb, uint32_t &packed) {
    int n = 0;
    packed = 0;
    if (nb & 1u) { packed |= 0u << (8 * n); ++n; }
    if (nb & 2u) { packed |= 1u << (8 * n); ++n; }
    if (nb & 4u) { packed |= 2u << (8 * n); ++n; packed |= 3u << (8 * n); ++n; }
    return n;
}

// Local slot of flat index idx over the selected blocks.
__device__ __forceinline__ int flat_to_slot(int idx, int T, uint32_t packed) {
    const int bi = (idx >= T) + (idx >= 2 * T) + (idx >= 3 * T);
    const int b = (int)((packed >> (8 * bi)) & 0xFFu);
    return b * T + (idx - bi * T);
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace

// ---------------------------------------------------------------------------------------------------
// k_init_costs: one workgroup per chain.  Costs of the current solution, copy to the working solution,
// F, best, shake size 1.
// ---------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init_costs(InitArgs a) {
    const int g = a.chain0 + blockIdx.x;
    const ChainInfo ci = a.chains[g];
    int64_t sum = 0;
    int inf = 0;
    for (int p = threadIdx.x; p < ci.K; p += blockDim.x) {
        const ProdParams pp = a.prod[ci.prod0 + p];
        const int64_t cp = ci.cp0 + p;
        const Bits b = a.cur[cp];
        const int64_t c = decode_cost(b, a.rows + pp.row, ci.T, pp);
        a.cur_cost[cp] = c;
        a.work[cp] = b;
        a.work_cost[cp] = c;
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
        cs.pad = 0;
        a.cstate[g] = cs;
    }
}

// ---------------------------------------------------------------------------------------------------
// k_eval: workgroup = (chain, product) with 4 wavefronts; lanes take the selected slots in order.
// ---------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_eval(EvalArgs a, int64_t cp_begin, const int32_t *__restrict__ cp_chain) {
    __shared__ int2 s_row[kTMax];
    __shared__ uint64_t s_key[4];
    __shared__ unsigned s_cnt[4];
    const int64_t cp = cp_begin + blockIdx.x;
    const int g = cp_chain[cp];
    const ChainInfo ci = a.chains[g];
    const int p = (int)(cp - ci.cp0);
    const int T = ci.T;
    const ProdParams pp = a.prod[ci.prod0 + p];
    for (int t = threadIdx.x; t < T; t += blockDim.x) s_row[t] = a.rows[pp.row + t];
    const Bits base = a.cur[cp];
    const int64_t base_cost = a.cur_cost[cp];
    const int64_t F = a.cstate[g].F;
    __syncthreads();

    uint32_t blk;
    const int nsel = blocks_of(a.nb_mask, blk);
    const int nslots = nsel * T;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t *out = a.slot_price ? a.slot_price + a.price_off[g] + (int64_t)p * 4 * T : nullptr;

    uint64_t best = kInfKey;
    unsigned cnt = 0;
    for (int basei = wave * 64; basei < nslots; basei += blockDim.x) {
        const int idx = basei + lane;
        const bool in = idx < nslots;
        const int l = in ? flat_to_slot(idx, T, blk) : 0;
        Bits mb = base;
        const bool valid = in && apply_move(mb, l, T);
        const int64_t c = decode_cost(mb, s_row, T, pp);
        const bool ok = valid && c != kInf;
        if (out && in) out[l] = ok ? F - base_cost + c : kInf;
        const uint64_t key = ok ? (((uint64_t)c << kSlotBits) | (uint64_t)l) : kInfKey;
        best = key < best ? key : best;
        cnt += (unsigned)__popcll(__ballot(valid));
    }
    if (out) {  // slots of unselected neighbourhoods
        for (int l = threadIdx.x; l < 4 * T; l += blockDim.x) {
            const int b = (l >= T) + (l >= 2 * T) + (l >= 3 * T);
            const uint32_t nb = b == 0 ? 1u : b == 1 ? 2u : 4u;
            if (!(a.nb_mask & nb)) out[l] = kInf;
        }
    }
    best = wave_min_u64(best);
    if (lane == 0) { s_key[wave] = best; s_cnt[wave] = cnt; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t k = s_key[0];
        unsigned n = s_cnt[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            k = s_key[w] < k ? s_key[w] : k;
            n += s_cnt[w];
        }
        a.prod_key[cp] = k;
        atomicAdd(a.evals, (unsigned long long)n);
    }
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
// work == cur for every product of the chain.
// ---------------------------------------------------------------------------------------------------
namespace {

// Best move of one neighbourhood for a product, computed by one wavefront: key = cost << 16 | slot.
__device__ __forceinline__ uint64_t wave_best_move(const Bits &b, const int2 *row, int T, const ProdParams &pp,
                                                   uint32_t nb, int64_t &evals) {
    uint32_t blk;
    const int nsel = blocks_of(nb, blk);
    const int nslots = nsel * T;
    const int lane = threadIdx.x & 63;
    uint64_t best = kInfKey;
    for (int basei = 0; basei < nslots; basei += 64) {
        const int idx = basei + lane;
        const bool in = idx < nslots;
        const int l = in ? flat_to_slot(idx, T, blk) : 0;
        Bits mb = b;
        const bool valid = in && apply_move(mb, l, T);
        const int64_t c = decode_cost(mb, row, T, pp);
        const uint64_t key = (valid && c != kInf) ? (((uint64_t)c << kSlotBits) | (uint64_t)l) : kInfKey;
        best = key < best ? key : best;
        evals += __popcll(__ballot(valid));
    }
    return wave_min_u64(best);
}

}  // namespace

__global__ __launch_bounds__(1024) void k_run(RunArgs a) {
    __shared__ int2 s_row[kMaxWaves][kTMax];
    __shared__ Bits s_db[kShakeMax];
    __shared__ int32_t s_dp[kShakeMax];
    __shared__ int64_t s_part[kMaxWaves];
    __shared__ int64_t s_ev[kMaxWaves];
    __shared__ int64_t s_shake;
    __shared__ int32_t s_nd;

    const int g = blockIdx.x;
    const ChainInfo ci = a.chains[g];
    const int K = ci.K, T = ci.T;
    const int64_t cp0 = ci.cp0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int W = blockDim.x >> 6;

    ChainState cs = a.cstate[g];
    int64_t evals = 0;  // per wave (uniform)
    int vnd_err = 0;    // per wave (uniform)
    const uint64_t nflip = 2ull * (uint64_t)K * (uint64_t)T;

    for (int i = 0; i < a.iters; ++i) {
        const int64_t it = a.it0 + i;
        const int kshake = cs.k;

        // ---- Shake(x, k): wavefront 0 draws k flips and keeps the feasible ones in a dirty list ----
        if (wave == 0) {
            const uint32_t my = lane < kshake ? shake_draw(a.seed, (uint64_t)g, (uint64_t)it, (uint64_t)lane, nflip) : 0u;
            int nd = 0;
            for (int j = 0; j < kshake; ++j) {
                const uint32_t f = (uint32_t)__shfl((int)my, j, 64);
                const int p = (int)(f / (uint32_t)(2 * T));
                const int l = (int)(f - (uint32_t)p * (uint32_t)(2 * T));
                int e = -1;
                for (int q = 0; q < nd; ++q) e = (e < 0 && s_dp[q] == p) ? q : e;
                Bits b = e >= 0 ? s_db[e] : a.work[cp0 + p];
                apply_move(b, l, T);
                const ProdParams pp = a.prod[ci.prod0 + p];
                if (feasible(b, a.rows + pp.row, T)) {
                    if (e < 0) {
                        e = nd++;
                        if (lane == 0) s_dp[e] = p;
                    }
                    if (lane == 0) s_db[e] = b;
                }
                wave_sync_lds();
            }
            if (lane == 0) s_nd = nd;
        }
        __syncthreads();
        const int nd = s_nd;

        // costs of the shaken products; x' = work
        {
            int64_t d = 0;
            if ((int)threadIdx.x < nd) {
                const int p = s_dp[threadIdx.x];
                const ProdParams pp = a.prod[ci.prod0 + p];
                const Bits b = s_db[threadIdx.x];
                const int64_t c = decode_cost(b, a.rows + pp.row, T, pp);
                a.work[cp0 + p] = b;
                a.work_cost[cp0 + p] = c;
                d = c - a.cur_cost[cp0 + p];
            }
            if (wave == 0) {
                d = wave_sum_i64(d);
                if (lane == 0) s_shake = d;
            }
        }
        __syncthreads();
        const int64_t F_shaken = cs.F + s_shake;

        // ---- VND (Algorithm 1) per product: the shaken products, or every product until x is known to
        //      be a local optimum ----
        const int nprod = cs.lopt ? nd : K;
        int64_t part = 0;
        for (int idx = wave; idx < nprod; idx += W) {
            const int p = cs.lopt ? s_dp[idx] : idx;
            const int64_t cp = cp0 + p;
            const ProdParams pp = a.prod[ci.prod0 + p];
            for (int t = lane; t < T; t += 64) s_row[wave][t] = a.rows[pp.row + t];
            wave_sync_lds();
            Bits b = a.work[cp];
            int64_t cost = a.work_cost[cp];
            bool improved = true;
            int passes = 0;
            while (improved) {
                if (++passes > kMaxPasses) {
                    vnd_err = 1;
                    break;
                }
                improved = false;
                for (int q = 0; q < a.n_nb; ++q) {
                    const uint32_t nb = (a.nb_list >> (4 * q)) & 0xFu;
                    const uint64_t key = wave_best_move(b, s_row[wave], T, pp, nb, evals);
                    if (key != kInfKey) {
                        const int64_t c = (int64_t)(key >> kSlotBits);
                        if (c < cost) {
                            apply_move(b, (int)(key & ((1u << kSlotBits) - 1)), T);
                            cost = c;
                            improved = true;
                        }
                    }
                }
            }
            if (lane == 0) {
                a.work[cp] = b;
                a.work_cost[cp] = cost;
            }
            part += cost - a.cur_cost[cp];
            wave_sync_lds();
        }
        if (lane == 0) s_part[wave] = part;
        __syncthreads();

        // ---- acceptance ----
        int64_t delta = 0;
        for (int w = 0; w < W; ++w) delta += s_part[w];
        const int64_t F_local = cs.F + delta;
        const int accepted = F_local < cs.F;
        const int ntouch = cs.lopt ? nd : K;
        for (int idx = threadIdx.x; idx < ntouch; idx += blockDim.x) {
            const int p = cs.lopt ? s_dp[idx] : idx;
            const int64_t cp = cp0 + p;
            if (accepted) {
                a.cur[cp] = a.work[cp];
                a.cur_cost[cp] = a.work_cost[cp];
            } else {
                a.work[cp] = a.cur[cp];
                a.work_cost[cp] = a.cur_cost[cp];
            }
        }
        if (accepted) {
            cs.F = F_local;
            cs.k = 1;
            cs.lopt = 1;
        } else {
            cs.k = cs.k >= a.kmax ? 1 : cs.k + 1;
        }
        cs.F_best = cs.F < cs.F_best ? cs.F : cs.F_best;
        if (a.trace && threadIdx.x == 0) {
            Record r;
            r.iter = (int32_t)it;
            r.k = kshake;
            r.accepted = accepted;
            r.pad = 0;
            r.F_shaken = F_shaken;
            r.F_local = F_local;
            r.F_best = cs.F_best;
            a.trace[(int64_t)g * a.iters + i] = r;
        }
        __syncthreads();
    }

    if (lane == 0) {
        s_ev[wave] = evals;
        s_part[wave] = vnd_err;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t e = 0;
        int32_t err = 0;
        for (int w = 0; w < W; ++w) {
            e += s_ev[w];
            err |= (int32_t)s_part[w];
        }
        cs.evals = e;
        cs.err |= err;
        a.cstate[g] = cs;
    }
}

// ---------------------------------------------------------------------------------------------------
// Host-side launchers (called by the runtime).
// ---------------------------------------------------------------------------------------------------
hipError_t launch_init(const InitArgs &a, int n_chains, hipStream_t s) {
    if (n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_costs, dim3(n_chains), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_eval(const EvalArgs &a, int64_t cp_begin, int64_t n_cp, const int32_t *cp_chain, hipStream_t s) {
    if (n_cp <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eval, dim3((unsigned)n_cp), dim3(256), 0, s, a, cp_begin, cp_chain);
    return hipGetLastError();
}

hipError_t launch_chain_best(const ChainBestArgs &a, int n_chains, hipStream_t s) {
    if (n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chain_best, dim3(n_chains), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_run(const RunArgs &a, int n_chains, int waves, hipStream_t s) {
    if (n_chains <= 0 || a.iters <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_run, dim3(n_chains), dim3(64 * waves), 0, s, a);
    return hipGetLastError();
}

}  // namespace vns
