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
#include <hip/hip_runtime.h>

#include "vns_device.hpp"
#include "vns_launch.hpp"

namespace vns {

namespace {

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bit t of v set iff swapping bits t and t+1 of z is a move (t < T-1 and the bits differ).
__device__ __forceinline__ void swap_valid(const uint32_t (&z)[kWords], int T, uint32_t (&v)[kWords]) {
#pragma unroll
    for (int j = 0; j < kWords; ++j) {
        const uint32_t next = (j + 1 < kWords) ? z[j + 1] : 0u;
        const uint32_t d = z[j] ^ ((z[j] >> 1) | (next << 31));
        const int lim = T - 1 - 32 * j;  // valid positions q < lim in this word
        const uint32_t keep = lim >= 32 ? ~0u : (lim <= 0 ? 0u : ((1u << lim) - 1u));
        v[j] = d & keep;
    }
}

__device__ __forceinline__ int popc_words(const uint32_t (&v)[kWords]) {
    int n = 0;
#pragma unroll
    for (int j = 0; j < kWords; ++j) n += __popc(v[j]);
    return n;
}

// Rank of bit t among the set bits of v, and whether it is set.
__device__ __forceinline__ int rank_bit(const uint32_t (&v)[kWords], int t, bool &set) {
    const int jt = t >> 5;
    const uint32_t below = (1u << (t & 31)) - 1u;
    int r = 0;
    set = false;
#pragma unroll
    for (int j = 0; j < kWords; ++j) {
        r += (j < jt) ? __popc(v[j]) : (j == jt ? __popc(v[j] & below) : 0);
        set |= (j == jt) && ((v[j] >> (t & 31)) & 1u);
    }
    return r;
}

// One wavefront writes the local slots of the valid swaps of b (zM swaps, then zR swaps) to list and
// returns how many there are.  The caller synchronises the wavefront before reading the list.
__device__ __forceinline__ int build_swap_list(const Bits &b, int T, uint16_t *list, int lane) {
    uint32_t vm[kWords], vr[kWords];
    swap_valid(b.m, T, vm);
    swap_valid(b.r, T, vr);
    const int nm = popc_words(vm);
    for (int t = lane; t < T - 1; t += 64) {
        bool sm, sr;
        const int pm = rank_bit(vm, t, sm);
        const int pr = rank_bit(vr, t, sr);
        if (sm) list[pm] = (uint16_t)(2 * T + t);
        if (sr) list[nm + pr] = (uint16_t)(3 * T + t);
    }
    return nm + popc_words(vr);
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
// k_eval
// ---------------------------------------------------------------------------------------------------
namespace {

struct EvalShared {
    int2 row[kTMax];
    Bits bits[kEvalGroup];
    unsigned long long key[kEvalGroup];
    int64_t F[kEvalGroup];
    int64_t cost[kEvalGroup];
    int64_t out_off[kEvalGroup];
    int32_t off[kEvalGroup + 1];
    int32_t nswap[kEvalGroup];
    uint16_t swap[kEvalGroup][2 * kTMax];
};

__device__ __forceinline__ void eval_items(const EvalArgs &a, EvalShared &sh, int n, int nflip, bool fm, int T,
                                           const ProdParams &pp) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int N = sh.off[n];
    for (int basei = wave * 64; basei < N; basei += blockDim.x) {
        const int idx = basei + lane;
        const bool in = idx < N;
        int j = 0;
        for (int q = 1; q < n; ++q) j += (idx >= sh.off[q]) ? 1 : 0;
        const int i = idx - sh.off[j];
        int slot = 0;
        if (in) slot = i < nflip ? (fm ? i : T + i) : (int)sh.swap[j][i - nflip];
        Bits mb = sh.bits[j];
        apply_move(mb, slot, T);
        const int64_t c = decode_cost(mb, sh.row, T, pp);
        if (in) {
            if (c != kInf) atomicMin(&sh.key[j], ((unsigned long long)c << kSlotBits) | (unsigned long long)slot);
            if (a.slot_price) a.slot_price[sh.out_off[j] + slot] = c == kInf ? kInf : sh.F[j] - sh.cost[j] + c;
        }
    }
}

}  // namespace

__global__ __launch_bounds__(256) void k_eval(EvalArgs a, const EvalWg *__restrict__ wg) {
    __shared__ EvalShared sh;
    const EvalWg d = wg[blockIdx.x];
    const int g0 = a.cp_chain[d.cp];
    const ChainInfo ci = a.chains[g0];
    const int K = ci.K, T = ci.T;
    const int p = (int)(d.cp - ci.cp0);
    const int n = d.n;
    const ProdParams pp = a.prod[ci.prod0 + p];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int t = threadIdx.x; t < T; t += blockDim.x) sh.row[t] = a.rows[pp.row + t];
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int64_t cp = d.cp + (int64_t)j * K;
        sh.bits[j] = a.cur[cp];
        sh.cost[j] = a.cur_cost[cp];
        sh.F[j] = a.cstate[g0 + j].F;
        sh.key[j] = kInfKey;
        sh.out_off[j] = a.slot_price ? a.price_off[g0 + j] + (int64_t)p * 4 * T : 0;
    }
    __syncthreads();

    const bool fm = a.nb_mask & 1u, fr = a.nb_mask & 2u, shift = a.nb_mask & 4u;
    const int nflip = (fm ? T : 0) + (fr ? T : 0);
    for (int j = wave; j < n; j += nw) {
        int ns = 0;
        if (shift) ns = build_swap_list(sh.bits[j], T, sh.swap[j], lane);
        if (lane == 0) sh.nswap[j] = ns;
    }
    if (a.slot_price) {  // every slot of the group starts as "not a priced move"
        for (int j = 0; j < n; ++j)
            for (int l = threadIdx.x; l < 4 * T; l += blockDim.x) a.slot_price[sh.out_off[j] + l] = kInf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int o = 0;
        for (int j = 0; j < n; ++j) {
            sh.off[j] = o;
            o += nflip + sh.nswap[j];
        }
        sh.off[n] = o;
    }
    __syncthreads();

    eval_items(a, sh, n, nflip, fm, T, pp);
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) a.prod_key[d.cp + (int64_t)j * K] = sh.key[j];
    if (threadIdx.x == 0) atomicAdd(a.evals, (unsigned long long)sh.off[n]);
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
// (a.rows_in_lds), otherwise each wavefront stages the row of the product it works on.
// ---------------------------------------------------------------------------------------------------
namespace {

struct RunShared {
    uint16_t list[kMaxWaves][2 * kTMax];   // compacted swap moves of each wavefront's product
    Bits db[kShakeMax];                    // shaken products (dirty list): bits after the shake
    int32_t dp[kShakeMax];                 //   and product index
    int64_t part[kMaxWaves];
    int64_t shk[kMaxWaves];
    int64_t ev[kMaxWaves];
    int32_t nd;
};

// Best move of one neighbourhood for a product, computed by one wavefront: key = cost << 16 | slot.
// With `ident`, one more item prices the unchanged pattern and its cost is returned in *ident_cost.
__device__ __forceinline__ uint64_t wave_best_move(const Bits &b, const int2 *row, int T, const ProdParams &pp,
                                                   uint32_t nb, uint16_t *list, bool ident, int64_t *ident_cost,
                                                   int64_t &evals) {
    const int lane = threadIdx.x & 63;
    const bool fm = nb & 1u;
    const int nflip = (nb & 3u) ? T : 0;   // the list holds one neighbourhood: flip zM, flip zR or shift
    int nswap = 0;
    if (nb & 4u) {
        nswap = build_swap_list(b, T, list, lane);
        wave_sync_lds();
    }
    const int nitems = nflip + nswap;
    const int total = nitems + (ident ? 1 : 0);
    evals += nitems;
    uint64_t best = kInfKey;
    int64_t idc = 0;
    for (int basei = 0; basei < total; basei += 64) {
        const int idx = basei + lane;
        int slot = -1;
        if (idx < nitems) slot = idx < nflip ? (fm ? idx : T + idx) : (int)list[idx - nflip];
        Bits mb = b;
        if (slot >= 0) apply_move(mb, slot, T);
        const int64_t c = decode_cost(mb, row, T, pp);
        if (idx == nitems) idc = c;
        const uint64_t key = (slot >= 0 && c != kInf) ? (((uint64_t)c << kSlotBits) | (uint64_t)slot) : kInfKey;
        best = key < best ? key : best;
    }
    if (ident) *ident_cost = __shfl(idc, nitems & 63, 64);
    return wave_min_u64(best);
}

__device__ __forceinline__ void run_chain(const RunArgs &a, RunShared &sh, int2 *s_rows) {
    const int g = blockIdx.x;
    const ChainInfo ci = a.chains[g];
    const int K = ci.K, T = ci.T;
    const int64_t cp0 = ci.cp0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int W = blockDim.x >> 6;
    const int2 *inst_rows = a.rows + a.prod[ci.prod0].row;   // an instance's rows are contiguous

    if (a.rows_in_lds) {
        for (int i = threadIdx.x; i < K * T; i += blockDim.x) s_rows[i] = inst_rows[i];
        __syncthreads();
    }

    ChainState cs = a.cstate[g];
    int64_t evals = 0;   // per wavefront (uniform)
    int vnd_err = 0;     // per wavefront (uniform)
    const uint64_t nflip_all = 2ull * (uint64_t)K * (uint64_t)T;

    for (int i = 0; i < a.iters; ++i) {
        const int64_t it = a.it0 + i;
        const int kshake = cs.k;

        // ---- Shake(x, k): wavefront 0 draws k flips and keeps the feasible ones in the dirty list ----
        if (wave == 0) {
            const uint32_t my = lane < kshake ? shake_draw(a.seed, (uint64_t)g, (uint64_t)it, (uint64_t)lane, nflip_all) : 0u;
            int nd = 0;
            for (int j = 0; j < kshake; ++j) {
                const uint32_t f = (uint32_t)__shfl((int)my, j, 64);
                const int p = (int)(f / (uint32_t)(2 * T));
                const int l = (int)(f - (uint32_t)p * (uint32_t)(2 * T));
                int e = -1;
                for (int q = 0; q < nd; ++q) e = (e < 0 && sh.dp[q] == p) ? q : e;
                Bits b = e >= 0 ? sh.db[e] : a.work[cp0 + p];
                apply_move(b, l, T);
                // a manufacturing setup in period 0 makes any pattern feasible; otherwise check the prefix
                bool ok = (b.m[0] & 1u) != 0u;
                if (!ok) ok = a.rows_in_lds ? feasible(b, s_rows + p * T, T) : feasible(b, inst_rows + p * T, T);
                if (ok) {
                    if (e < 0) {
                        e = nd++;
                        if (lane == 0) sh.dp[e] = p;
                    }
                    if (lane == 0) sh.db[e] = b;
                }
                wave_sync_lds();
            }
            if (lane == 0) sh.nd = nd;
        }
        __syncthreads();
        const int nd = sh.nd;

        // ---- VND (Algorithm 1) per product: the shaken products, or every product until x is known to
        //      be a local optimum ----
        const int nprod = cs.lopt ? nd : K;
        int64_t part = 0, shk = 0;
        for (int idx = wave; idx < nprod; idx += W) {
            int p, e = -1;
            if (cs.lopt) {
                p = sh.dp[idx];
                e = idx;
            } else {
                p = idx;
                for (int q = 0; q < nd; ++q) e = (e < 0 && sh.dp[q] == p) ? q : e;
            }
            const int64_t cp = cp0 + p;
            const ProdParams pp = a.prod[ci.prod0 + p];
            const int2 *row;
            if (a.rows_in_lds) {
                row = s_rows + p * T;
            } else {
                int2 *slice = s_rows + wave * kTMax;
                for (int t = lane; t < T; t += 64) slice[t] = inst_rows[p * T + t];
                wave_sync_lds();
                row = slice;
            }
            Bits b = e >= 0 ? sh.db[e] : a.work[cp];
            const int64_t c_cur = a.cur_cost[cp];
            int64_t cost = e >= 0 ? kInf : a.work_cost[cp];   // a shaken product is priced with its first move list
            bool need_ident = e >= 0;
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
                    int64_t idc = 0;
                    const uint64_t key = wave_best_move(b, row, T, pp, nb, sh.list[wave], need_ident, &idc, evals);
                    if (need_ident) {
                        cost = idc;
                        shk += idc - c_cur;
                        need_ident = false;
                    }
                    if (key != kInfKey) {
                        const int64_t c = (int64_t)(key >> kSlotBits);
                        if (c < cost) {
                            apply_move(b, (int)(key & ((1u << kSlotBits) - 1)), T);
                            cost = c;
                            improved = true;
                        }
                    }
                    wave_sync_lds();
                }
            }
            if (lane == 0) {
                a.work[cp] = b;
                a.work_cost[cp] = cost;
            }
            part += cost - c_cur;
        }
        if (lane == 0) {
            sh.part[wave] = part;
            sh.shk[wave] = shk;
        }
        __syncthreads();

        // ---- acceptance ----
        int64_t delta = 0, dshake = 0;
        for (int w = 0; w < W; ++w) {
            delta += sh.part[w];
            dshake += sh.shk[w];
        }
        const int64_t F_local = cs.F + delta;
        const int accepted = F_local < cs.F;
        const int ntouch = cs.lopt ? nd : K;
        for (int idx = threadIdx.x; idx < ntouch; idx += blockDim.x) {
            const int p = cs.lopt ? sh.dp[idx] : idx;
            const int64_t cp = cp0 + p;
            if (accepted) {
                a.cur[cp] = a.work[cp];
                a.cur_cost[cp] = a.work_cost[cp];
            } else {
                a.work[cp] = a.cur[cp];
                a.work_cost[cp] = a.cur_cost[cp];
            }
        }
        if (a.trace && threadIdx.x == 0) {
            Record r;
            r.iter = (int32_t)it;
            r.k = kshake;
            r.accepted = accepted;
            r.pad = 0;
            r.F_shaken = cs.F + dshake;
            r.F_local = F_local;
            r.F_best = (accepted && F_local < cs.F_best) ? F_local : cs.F_best;
            a.trace[(int64_t)g * a.iters + i] = r;
        }
        if (accepted) {
            cs.F = F_local;
            cs.k = 1;
            cs.lopt = 1;
        } else {
            cs.k = cs.k >= a.kmax ? 1 : cs.k + 1;
        }
        cs.F_best = cs.F < cs.F_best ? cs.F : cs.F_best;
        __syncthreads();
    }

    if (lane == 0) {
        sh.ev[wave] = evals;
        sh.part[wave] = vnd_err;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t e = 0;
        int32_t err = 0;
        for (int w = 0; w < W; ++w) {
            e += sh.ev[w];
            err |= (int32_t)sh.part[w];
        }
        cs.evals = e;
        cs.err |= err;
        a.cstate[g] = cs;
    }
}

}  // namespace

__global__ __launch_bounds__(512) void k_run(RunArgs a) {
    __shared__ RunShared sh;
    extern __shared__ int2 s_rows[];
    run_chain(a, sh, s_rows);
}

// ---------------------------------------------------------------------------------------------------
// Host-side launchers (called by the runtime).
// ---------------------------------------------------------------------------------------------------
hipError_t launch_init(const InitArgs &a, int n_chains, hipStream_t s) {
    if (n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_costs, dim3(n_chains), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_eval(const EvalArgs &a, const EvalWg *wg, int64_t n_wg, hipStream_t s) {
    if (n_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eval, dim3((unsigned)n_wg), dim3(256), 0, s, a, wg);
    return hipGetLastError();
}

hipError_t launch_chain_best(const ChainBestArgs &a, int n_chains, hipStream_t s) {
    if (n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chain_best, dim3(n_chains), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_run(const RunArgs &a, int n_chains, int waves, size_t lds_bytes, hipStream_t s) {
    if (n_chains <= 0 || a.iters <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_run, dim3(n_chains), dim3(64 * waves), lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace vns
