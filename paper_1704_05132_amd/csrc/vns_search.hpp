// Per-wavefront move search used by the search kernel and the learned pricing kernel: the move list of a
// neighbourhood (all flips, or the compacted list of swaps of differing bits), the exact best move of a
// neighbourhood (one lane per move), its learned variant (the scorer ranks the moves, the best-ranked are
// priced exactly, the whole neighbourhood is priced if none of them improves) and the move log.
#pragma once
#include <hip/hip_runtime.h>

#include "vns_device.hpp"
#include "vns_mlp.hpp"

namespace vns {

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bounded wait until *p >= v, false if the wait ran out (after `ticks` of the steady clock, or
// kCoopSpinLimit polls).  The polls are relaxed (an acquire per poll would invalidate the caches the other
// workgroups of the XCD are working from); one acquire follows success.  *seen: the value observed.
__device__ __forceinline__ bool coop_wait_ge(int32_t *p, int32_t v, int64_t ticks, int32_t *seen = nullptr) {
    const int64_t t0 = wall_clock64();
    for (uint32_t n = 0; n < kCoopSpinLimit; ++n) {
        const int32_t now = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (now >= v) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (seen) *seen = now;
            return true;
        }
        if (wall_clock64() - t0 > ticks) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    return false;
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

// One wavefront lists the valid swaps of b in period order, the zM swaps first, compacted by ballots:
// out[i] = item(z, t) for the i-th swap (z = 0 for zM, 1 for zR, t its first period).  Returns how many there
// are (wave-uniform).  The caller synchronises the wavefront before reading out.  (The swap masks stay in
// this function: passed by reference into another, the compiler kept them as per-thread arrays and moved
// them to LDS, 32 bytes per thread.)
template <class Item>
__device__ __forceinline__ int compact_swaps(const Bits &b, int T, uint16_t *out, Item item) {
    uint32_t vm[kWords], vr[kWords];
    swap_valid(b.m, T, vm);
    swap_valid(b.r, T, vr);
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    int o = 0;
#pragma unroll
    for (int z = 0; z < 2; ++z) {
        for (int t0 = 0; t0 < T - 1; t0 += 64) {
            const int t = t0 + lane, w = t >> 5;
            uint32_t word = z ? vr[0] : vm[0];
#pragma unroll
            for (int q = 1; q < kWords; ++q) word = w == q ? (z ? vr[q] : vm[q]) : word;
            const bool v = w < kWords && ((word >> (t & 31)) & 1u);   // bits past T - 2 are clear
            const uint64_t bal = __ballot(v);
            if (v) out[o + __popcll(bal & below)] = item(z, t);
            o += __popcll(bal);
        }
    }
    return o;
}

// One wavefront writes the local slots of the valid swaps of b (zM swaps, then zR swaps) to list and
// returns how many there are.  The caller synchronises the wavefront before reading the list.
__device__ __forceinline__ int build_swap_list(const Bits &b, int T, uint16_t *list) {
    return compact_swaps(b, T, list, [T](int z, int t) { return (uint16_t)((2 + z) * T + t); });
}


// Slot of item idx of a neighbourhood's move list: flips first (zM or zR), then the compacted swaps.
__device__ __forceinline__ int item_slot(int idx, int nflip, bool fm, int T, const uint16_t *list) {
    return idx < nflip ? (fm ? idx : T + idx) : (int)list[idx - nflip];
}

// Builds the move list of one neighbourhood (nb: 1 flip zM, 2 flip zR, 4 shift) for the pattern b;
// returns the number of moves, sets nflip / fm.  Synchronises the wavefront when it writes the list.
__device__ __forceinline__ int move_list(const Bits &b, int T, uint32_t nb, uint16_t *list, int &nflip, bool &fm) {
    const int lane = threadIdx.x & 63;
    fm = nb & 1u;
    nflip = (nb & 3u) ? T : 0;
    int nswap = 0;
    if (nb & 4u) {
        nswap = build_swap_list(b, T, list);
        wave_sync_lds();
    }
    return nflip + nswap;
}

// One lane per item of a neighbourhood's move list (plus, at index nitems, the unchanged pattern when
// total > nitems): exact costs folded into the lane's best key; the contrast item's key and the unchanged
// pattern's cost are kept by the lanes that priced them.  NW setup words (2 when T <= 64).
template <int NW, int MODEL = 0>
__device__ __forceinline__ void price_items(const Bits &b, const int2 *row, int T, const ProdParams &pp,
                                            const uint16_t *list, int nitems, int nflip, bool fm, int total,
                                            int citem, uint64_t &best, uint64_t &ck, int64_t &idc) {
    const int lane = threadIdx.x & 63;
    for (int basei = 0; basei < total; basei += 64) {
        const int idx = basei + lane;
        const int slot = idx < nitems ? item_slot(idx, nflip, fm, T, list) : -1;
        Bits mb = b;
        if (slot >= 0) {
            const int blk = (slot >= T) + (slot >= 2 * T) + (slot >= 3 * T);
            xor_move<NW>(mb, blk, slot - blk * T);
        }
        const int64_t c = decode_cost<NW, MODEL>(mb, row, T, pp);
        if (idx == nitems) idc = c;
        const uint64_t key = (slot >= 0 && c != kInf) ? (((uint64_t)c << kSlotBits) | (uint64_t)slot) : kInfKey;
        if (idx == citem) ck = key;
        best = key < best ? key : best;
    }
}

// Exact best move of one neighbourhood for one product, computed by one wavefront: key = cost << 16 | slot.
// With `ident`, one more item prices the unchanged pattern and its cost is returned in *ident_cost.  With
// contrast >= 0 (any non-negative hash), *contrast_key receives the key of item contrast mod the number of
// moves (kInfKey when infeasible or when there is no move).
template <int MODEL = 0>
__device__ __forceinline__ uint64_t wave_best_move(const Bits &b, const int2 *row, int T, const ProdParams &pp,
                                                   uint32_t nb, uint16_t *list, bool ident, int64_t *ident_cost,
                                                   int64_t &evals, int contrast = -1, uint64_t *contrast_key = nullptr,
                                                   int *n_items = nullptr) {
    int nflip;
    bool fm;
    const int nitems = move_list(b, T, nb, list, nflip, fm);
    if (n_items) *n_items = nitems;
    const int total = nitems + (ident ? 1 : 0);
    evals += nitems;
    uint64_t best = kInfKey, ck = kInfKey;
    int64_t idc = 0;
    const int citem = (contrast >= 0 && nitems > 0) ? contrast % nitems : -1;
    if (T <= 64)
        price_items<2, MODEL>(b, row, T, pp, list, nitems, nflip, fm, total, citem, best, ck, idc);
    else
        price_items<4, MODEL>(b, row, T, pp, list, nitems, nflip, fm, total, citem, best, ck, idc);
    if (ident) *ident_cost = __shfl(idc, nitems & 63, 64);
    if (contrast_key) *contrast_key = citem >= 0 ? __shfl(ck, citem & 63, 64) : kInfKey;
    return wave_min_u64(best);
}

// Several consecutive neighbourhoods q0, q0 + 1, ... (at most three, of the n_nb in nb_list) of one pattern
// priced side by side in one wavefront pass, for horizons short enough that their moves, and the unchanged
// pattern with `ident`, fit 64 lanes (at most one of them may hold swaps: one list).  In Algorithm 1's order
// the first neighbourhood whose best move beats `cost` is the one the VND takes; those after it were priced on
// the pattern before that move, so they are dropped.  Returns that best key (kInfKey when none improves), sets
// *used to the neighbourhoods consumed and counts evaluations for those only, so the moves and counts equal
// one neighbourhood at a time.  With `ident`, cost is set to the unchanged pattern's price first.
template <int NW, int MODEL = 0>
__device__ __forceinline__ uint64_t wave_best_move_multi(const Bits &b, const int2 *row, int T, const ProdParams &pp,
                                                         uint32_t nb_list, int q0, int n_nb, uint16_t *list,
                                                         bool ident, int64_t &cost, int64_t &evals, int &used) {
    const int lane = threadIdx.x & 63;
    // the segments: neighbourhood k's moves at lanes [o_k, o_k + n_k)
    int n0 = 0, n1 = 0, n2 = 0, f0 = 0, f1 = 0, f2 = 0, r = 0, sk = -1;
    bool m0 = false, m1 = false, m2 = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (q0 + k >= n_nb) break;
        const uint32_t nb = (nb_list >> (4 * (q0 + k))) & 0xFu;
        const int nflip = (nb & 3u) ? T : 0;
        int nsw = 0;
        if (nb & 4u) {
            if (sk >= 0) break;   // one swap list per pass
            uint32_t vm[kWords], vr[kWords];
            swap_valid(b.m, T, vm);
            swap_valid(b.r, T, vr);
            nsw = popc_words(vm) + popc_words(vr);
        }
        const int n = nflip + nsw;
        if (k > 0 && n0 + n1 + n + (ident ? 1 : 0) > 64) break;
        if (nb & 4u) sk = k;
        if (k == 0) { n0 = n; f0 = nflip; m0 = nb & 1u; }
        if (k == 1) { n1 = n; f1 = nflip; m1 = nb & 1u; }
        if (k == 2) { n2 = n; f2 = nflip; m2 = nb & 1u; }
        r = k + 1;
    }
    if (sk >= 0) {
        build_swap_list(b, T, list);
        wave_sync_lds();
    }
    const int o1 = n0, o2 = n0 + n1, total = n0 + n1 + n2;
    const int seg = (lane >= o1) + (lane >= o2);
    const int local = lane - (seg == 0 ? 0 : seg == 1 ? o1 : o2);
    const int nflip = seg == 0 ? f0 : seg == 1 ? f1 : f2;
    const bool fm = seg == 0 ? m0 : seg == 1 ? m1 : m2;
    const int slot = lane < total ? (local < nflip ? (fm ? local : T + local) : (int)list[local - nflip]) : -1;
    Bits mb = b;
    if (slot >= 0) {
        const int blk = (slot >= T) + (slot >= 2 * T) + (slot >= 3 * T);
        xor_move<NW>(mb, blk, slot - blk * T);
    }
    const int64_t c = decode_cost<NW, MODEL>(mb, row, T, pp);
    if (ident) cost = __shfl(c, total & 63, 64);
    const uint64_t key = (slot >= 0 && c != kInf) ? (((uint64_t)c << kSlotBits) | (uint64_t)slot) : kInfKey;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k >= r) break;
        const uint64_t best = wave_min_u64(seg == k && lane < total ? key : kInfKey);
        evals += k == 0 ? n0 : k == 1 ? n1 : n2;
        if (best != kInfKey && (int64_t)(best >> kSlotBits) < cost) {
            used = k + 1;
            return best;
        }
    }
    used = r;
    return kInfKey;
}

// Per-wavefront LDS of the learned search: the scorer's feature tile and the selected moves.
struct LearnedLds {
    __bf16 *sx;        // [64][16]
    uint16_t *sel;     // [2 * kTMax]
};

// Steps 1 and 2 of a learned neighbourhood evaluation by one wavefront, for a neighbourhood of nitems >= 1
// moves (list, nflip, fm from move_list): every move is scored, and the best-ranked
// ceil(permille * nitems / 1000) (at least one; lowest score first, ties to the lower slot) are written to
// sel in rank order.  Returns their number.  score_out / sel_out (by slot, may be null) receive the scores and
// the selection.
__device__ __forceinline__ int learned_select(const Bits &b, const int2 *row, int T, const ProdParams &pp, int nitems,
                                              int nflip, bool fm, const uint16_t *list, __bf16 *sx, uint16_t *sel,
                                              const mlp::Frags &fr, int permille, float *score_out, uint8_t *sel_out) {
    const int lane = threadIdx.x & 63;
    // 1. scores of every move, kept as (sortable score << 32 | slot) keys, up to four per lane
    uint64_t sk[4] = {kInfKey, kInfKey, kInfKey, kInfKey};
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        if (ch * 64 >= nitems) break;
        const int idx = ch * 64 + lane;
        const int slot = idx < nitems ? item_slot(idx, nflip, fm, T, list) : 0;
        float f[mlp::kF];
        if (idx < nitems) {
            mlp::move_features(b, row, T, pp, slot, f);
        } else {
#pragma unroll
            for (int i = 0; i < mlp::kF; ++i) f[i] = 0.f;
        }
#pragma unroll
        for (int i = 0; i < mlp::kF; ++i) sx[lane * mlp::kF + i] = (__bf16)f[i];
        wave_sync_lds();
        const float s = mlp::forward64(sx, fr);
        if (idx < nitems) {
            sk[ch] = ((uint64_t)mlp::sortable(s) << 32) | (uint64_t)slot;
            if (score_out) score_out[slot] = s;
        }
    }
    // 2. the best-ranked moves, by repeated wavefront minima
    int n_sel = (permille * nitems + 999) / 1000;   // nitems >= 1 here
    n_sel = n_sel < 1 ? 1 : (n_sel > nitems ? nitems : n_sel);
    for (int r = 0; r < n_sel; ++r) {
        uint64_t my = sk[0];
#pragma unroll
        for (int ch = 1; ch < 4; ++ch) my = sk[ch] < my ? sk[ch] : my;
        const uint64_t m = wave_min_u64(my);
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) sk[ch] = sk[ch] == m ? kInfKey : sk[ch];
        if (lane == 0) sel[r] = (uint16_t)(m & 0xFFFFu);
        if (sel_out && lane == 0 && m != kInfKey) sel_out[m & 0xFFFFu] = 1;
    }
    wave_sync_lds();
    return n_sel;
}

// Learned best move of one neighbourhood (one wavefront).  The scorer ranks the moves (lowest score first,
// ties to the lower slot), the best-ranked ceil(permille * n / 1000) (at least one) are priced exactly and
// the best of them is returned if it is cheaper than `cost`; otherwise the whole neighbourhood is priced
// exactly (fallback) and its best move is returned.  A neighbourhood without moves returns kInfKey with no
// evaluation and no fallback.  With `ident` the unchanged pattern is priced with the
// selected moves and *cost is set to it first.  score_out / sel_out (indexed by slot, may be null) receive
// the scores and the selection.
__device__ __forceinline__ uint64_t learned_best_move(const Bits &b, const int2 *row, int T, const ProdParams &pp,
                                                      uint32_t nb, uint16_t *list, const LearnedLds &L,
                                                      const mlp::Frags &fr, int permille,
                                                      bool ident, int64_t &cost, int64_t &evals, int &fallback,
                                                      float *score_out = nullptr, uint8_t *sel_out = nullptr) {
    const int lane = threadIdx.x & 63;
    int nflip;
    bool fm;
    const int nitems = move_list(b, T, nb, list, nflip, fm);
    fallback = 0;
    if (nitems == 0) {
        // an empty neighbourhood (every adjacent pair equal in a shift, or T = 1): nothing is scored,
        // selected or priced; with `ident` the unchanged pattern is still priced, by every lane alike
        if (ident) cost = decode_cost(b, row, T, pp);
        return kInfKey;
    }
    // 1-2. scores of every move and the best-ranked ones
    const int n_sel = learned_select(b, row, T, pp, nitems, nflip, fm, list, L.sx, L.sel, fr, permille, score_out, sel_out);
    evals += n_sel;
    if (nitems + (ident ? 1 : 0) <= 128) {
        // 3-4 together: when the whole neighbourhood (and the unchanged pattern) takes at most two wavefront
        // passes, every move is priced at once, since pricing only the selection costs one pass of the same
        // latency and most evaluations fall back (about three in four here); the selection's best and,
        // should it not improve, the whole neighbourhood's best come from the same exact prices, as the two
        // steps below would give them
        uint64_t best_sel = kInfKey, best_all = kInfKey;
        int64_t idc = 0;
        const int total = nitems + (ident ? 1 : 0);
        for (int basei = 0; basei < total; basei += 64) {
            const int idx = basei + lane;
            const int slot = idx < nitems ? item_slot(idx, nflip, fm, T, list) : -1;
            bool selected = false;
            for (int r = 0; r < n_sel; ++r) selected |= slot >= 0 && slot == (int)L.sel[r];
            Bits mb = b;
            if (slot >= 0) apply_move(mb, slot, T);
            const int64_t c = decode_cost(mb, row, T, pp);
            if (idx == nitems) idc = c;
            const uint64_t key = (slot >= 0 && c != kInf) ? (((uint64_t)c << kSlotBits) | (uint64_t)slot) : kInfKey;
            best_all = key < best_all ? key : best_all;
            best_sel = (selected && key < best_sel) ? key : best_sel;
        }
        if (ident) cost = __shfl(idc, nitems & 63, 64);
        best_sel = wave_min_u64(best_sel);
        if (best_sel != kInfKey && (int64_t)(best_sel >> kSlotBits) < cost) {
            fallback = 0;
            return best_sel;
        }
        fallback = 1;   // the whole neighbourhood, exactly (already priced)
        evals += nitems;
        return wave_min_u64(best_all);
    }
    // 3. exact prices of the selection (and of the unchanged pattern)
    const int total = n_sel + (ident ? 1 : 0);
    uint64_t best = kInfKey;
    int64_t idc = 0;
    for (int basei = 0; basei < total; basei += 64) {
        const int idx = basei + lane;
        const int slot = idx < n_sel ? (int)L.sel[idx] : -1;
        Bits mb = b;
        if (slot >= 0) apply_move(mb, slot, T);
        const int64_t c = decode_cost(mb, row, T, pp);
        if (idx == n_sel) idc = c;
        const uint64_t key = (slot >= 0 && c != kInf) ? (((uint64_t)c << kSlotBits) | (uint64_t)slot) : kInfKey;
        best = key < best ? key : best;
    }
    if (ident) cost = __shfl(idc, n_sel & 63, 64);
    best = wave_min_u64(best);
    if (best != kInfKey && (int64_t)(best >> kSlotBits) < cost) {
        fallback = 0;
        return best;
    }
    // 4. fallback: the whole neighbourhood, exactly
    fallback = 1;
    return wave_best_move(b, row, T, pp, nb, list, false, nullptr, evals);
}

// ---------------------------------------------------------------------------------------------------
// The learned VND of several products at once, by the workgroup's wavefronts together (packed form).  The
// products of a batch step through Algorithm 1 in lockstep: per step every product still searching takes its
// next neighbourhood (in list order, skipping one already priced without improvement on the current pattern
// when the memo is on); the wavefronts share the products out, each building the move lists, scores and
// selections of its own (learned_select); then the selections of all of them, with the unchanged shaken
// patterns still to price, are priced exactly in one packed list over every lane of the workgroup; the
// products whose selection holds no improving move get their whole neighbourhood priced, all of them in one
// packed list again; and each applies its move.  Per product the selections, prices, fallbacks, moves and
// counted evaluations are those of learned_best_move in the one-product VND: only the packing of lanes
// differs, so a selection of a few moves no longer takes a whole T-period pass of its own.
// ---------------------------------------------------------------------------------------------------
struct PackProd {
    Bits b;                    // the product's current pattern
    int64_t cost;              // its exact cost (kInf until the unchanged shaken pattern is priced)
    int64_t c_cur;             // its cost in x
    int64_t shk;               // cost after the shake minus cost in x (shaken products)
    int64_t idc;               // this step's price of the unchanged pattern
    unsigned long long best;   // this step's best key (the selection's, then the fallback's)
    int32_t p, q, passes, clean, improved, need_ident, active, err;
    int32_t nb, nitems, nflip, fm, nsel, fb;
};
static_assert(sizeof(PackProd) == kPackProdBytes, "the packed region's layout");

// The workgroup's LDS for the packed form: a feature tile per wavefront, a small control block, then per
// product its record, move list, selection and (when the instance's rows are not resident) staged row.
struct PackLds {
    __bf16 *sx;      // [W][64][16]
    int32_t *ctl;    // [4]: the round count read at a step's start
    PackProd *pk;    // [P]
    uint16_t *list;  // [P][2 kTMax]
    uint16_t *sel;   // [P][2 kTMax]
    int2 *rows;      // [P][kTMax]
};

// The region of pack_region_bytes(W, P) bytes at base.
__device__ __forceinline__ PackLds pack_lds(char *base, int W, int P) {
    PackLds L;
    L.sx = reinterpret_cast<__bf16 *>(base);
    base += W * 64 * 16 * 2;
    L.ctl = reinterpret_cast<int32_t *>(base);
    base += 16;
    L.pk = reinterpret_cast<PackProd *>(base);
    base += P * sizeof(PackProd);
    L.list = reinterpret_cast<uint16_t *>(base);
    base += P * 2 * kTMax * 2;
    L.sel = reinterpret_cast<uint16_t *>(base);
    base += P * 2 * kTMax * 2;
    L.rows = reinterpret_cast<int2 *>(base);
    return L;
}

// Item idx of a step's packed list: the product i with off[i] <= idx < off[i + 1] (n products).
__device__ __forceinline__ int pack_owner(const int (&off)[kPackMax + 1], int n, int idx) {
    int i = 0;
#pragma unroll
    for (int j = 1; j < kPackMax; ++j) i += (j < n && idx >= off[j]) ? 1 : 0;
    return i;
}

// Runs the batch L.pk[0 .. n-1] (p, b, cost, c_cur, need_ident set by the caller before a barrier) to its
// local optima; every thread of the workgroup calls it.  rows: the instance's rows when resident in LDS, else
// null (inst_rows in device memory are staged per product).  prod: the instance's product parameters.
// round_now() is read (by thread 0) at each step's start and compared with `round` at its end: false means
// the round moved on and the batch was abandoned.  The evaluation counters are advanced in wavefront 0 only.
template <class RoundNow>
__device__ __forceinline__ bool learned_vnd_packed(const PackLds &L, int n, const int2 *rows, const int2 *inst_rows,
                                                   const ProdParams *prod, int T, uint32_t nb_list, int n_nb, int memo,
                                                   const mlp::Frags &fr, int permille, int64_t &evals,
                                                   int64_t &nb_evals, int64_t &fallbacks, int32_t round,
                                                   RoundNow round_now) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6, nthr = blockDim.x;
    const bool counter = wave == 0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < n; ++i) {
            PackProd &s = L.pk[i];
            s.q = 0;
            s.passes = 1;
            s.clean = 0;
            s.improved = 0;
            s.active = 1;
            s.err = 0;
            s.shk = 0;
        }
    }
    if (!rows) {
        for (int i = 0; i < n; ++i) {
            const int p = L.pk[i].p;
            for (int t = threadIdx.x; t < T; t += nthr) L.rows[i * kTMax + t] = inst_rows[p * T + t];
        }
    }
    __syncthreads();
    auto row_of = [&](int i, int p) -> const int2 * { return rows ? rows + p * T : L.rows + i * kTMax; };
    __bf16 *sx = L.sx + wave * 64 * mlp::kF;
    for (;;) {
        // 1. each product's next neighbourhood (thread 0 advances the states)
        if (threadIdx.x == 0) {
            for (int i = 0; i < n; ++i) {
                PackProd &s = L.pk[i];
                s.nb = -1;
                while (s.active) {
                    while (s.q < n_nb && memo && ((s.clean >> s.q) & 1)) ++s.q;
                    if (s.q < n_nb) {
                        s.nb = (int32_t)((nb_list >> (4 * s.q)) & 0xFu);
                        break;
                    }
                    if (s.improved && s.passes < kMaxPasses) {   // another pass
                        ++s.passes;
                        s.improved = 0;
                        s.q = 0;
                    } else {
                        s.err |= s.improved;   // the pass guard (cannot happen with a consistent decode)
                        s.active = 0;
                    }
                }
            }
            L.ctl[0] = round_now();
        }
        __syncthreads();
        int stepping = 0;
        for (int i = 0; i < n; ++i) stepping += L.pk[i].nb >= 0 ? 1 : 0;
        if (stepping == 0) return true;
        // 2. move lists, scores and selections: the stepping products shared out over the wavefronts
        for (int i = 0, r = 0; i < n; ++i) {
            const int nb = L.pk[i].nb;
            if (nb < 0) continue;
            if ((r++ % W) != wave) continue;
            const Bits b = L.pk[i].b;
            const int p = L.pk[i].p;
            const ProdParams pp = prod[p];
            uint16_t *list = L.list + i * 2 * kTMax;
            int nflip;
            bool fm;
            const int nitems = move_list(b, T, (uint32_t)nb, list, nflip, fm);
            const int nsel = nitems > 0 ? learned_select(b, row_of(i, p), T, pp, nitems, nflip, fm, list, sx,
                                                         L.sel + i * 2 * kTMax, fr, permille, nullptr, nullptr)
                                        : 0;
            if (lane == 0) {
                PackProd &s = L.pk[i];
                s.nitems = nitems;
                s.nflip = nflip;
                s.fm = fm ? 1 : 0;
                s.nsel = nsel;
                s.best = kInfKey;
                s.fb = 0;
            }
        }
        __syncthreads();
        // 3. every selection, and every unchanged pattern still to price, in one packed list
        int off[kPackMax + 1];
        off[0] = 0;
#pragma unroll
        for (int i = 0; i < kPackMax; ++i)
            off[i + 1] = off[i] + ((i < n && L.pk[i].nb >= 0) ? L.pk[i].nsel + L.pk[i].need_ident : 0);
        const int total = off[kPackMax];
        for (int basei = 0; basei < total; basei += nthr) {
            const int idx = basei + (int)threadIdx.x;
            if (idx < total) {
                const int i = pack_owner(off, n, idx), k = idx - off[i];
                const int p = L.pk[i].p;
                const int slot = k < L.pk[i].nsel ? (int)L.sel[i * 2 * kTMax + k] : -1;
                Bits mb = L.pk[i].b;
                if (slot >= 0) apply_move(mb, slot, T);
                const int64_t c = decode_cost(mb, row_of(i, p), T, prod[p]);
                if (slot < 0)
                    L.pk[i].idc = c;
                else if (c != kInf)
                    atomicMin(&L.pk[i].best, ((unsigned long long)c << kSlotBits) | (unsigned long long)slot);
            }
        }
        if (counter)
            for (int i = 0; i < n; ++i) evals += L.pk[i].nb >= 0 ? L.pk[i].nsel : 0;
        __syncthreads();
        // 4. the unchanged patterns' prices, and which selections hold no improving move
        if (threadIdx.x == 0) {
            for (int i = 0; i < n; ++i) {
                PackProd &s = L.pk[i];
                if (s.nb < 0) continue;
                if (s.need_ident) {
                    s.cost = s.idc;
                    s.shk = s.idc - s.c_cur;
                    s.need_ident = 0;
                }
                const bool better = s.best != kInfKey && (int64_t)(s.best >> kSlotBits) < s.cost;
                s.fb = (s.nitems > 0 && !better) ? 1 : 0;
                if (s.fb) s.best = kInfKey;
            }
        }
        __syncthreads();
        // 5. fallback: the whole neighbourhoods of those products, in one packed list
#pragma unroll
        for (int i = 0; i < kPackMax; ++i) off[i + 1] = off[i] + ((i < n && L.pk[i].nb >= 0 && L.pk[i].fb) ? L.pk[i].nitems : 0);
        const int ftotal = off[kPackMax];
        for (int basei = 0; basei < ftotal; basei += nthr) {
            const int idx = basei + (int)threadIdx.x;
            if (idx < ftotal) {
                const int i = pack_owner(off, n, idx), k = idx - off[i];
                const int p = L.pk[i].p;
                const int slot = item_slot(k, L.pk[i].nflip, L.pk[i].fm != 0, T, L.list + i * 2 * kTMax);
                Bits mb = L.pk[i].b;
                apply_move(mb, slot, T);
                const int64_t c = decode_cost(mb, row_of(i, p), T, prod[p]);
                if (c != kInf) atomicMin(&L.pk[i].best, ((unsigned long long)c << kSlotBits) | (unsigned long long)slot);
            }
        }
        if (counter) {
            for (int i = 0; i < n; ++i) {
                if (L.pk[i].nb < 0) continue;
                evals += L.pk[i].fb ? L.pk[i].nitems : 0;
                nb_evals += 1;
                fallbacks += L.pk[i].fb;
            }
        }
        __syncthreads();
        // 6. each product's move, when it improves
        if (threadIdx.x == 0) {
            for (int i = 0; i < n; ++i) {
                PackProd &s = L.pk[i];
                if (s.nb < 0) continue;
                const unsigned long long key = s.best;
                const bool applied = key != kInfKey && (int64_t)(key >> kSlotBits) < s.cost;
                if (applied) {
                    apply_move(s.b, (int)(key & ((1u << kSlotBits) - 1)), T);
                    s.cost = (int64_t)(key >> kSlotBits);
                    s.improved = 1;
                }
                s.clean = applied ? 0 : (s.clean | (1 << s.q));
                ++s.q;
            }
        }
        __syncthreads();
        if (L.ctl[0] != round) return false;
    }
}

// Appends the records of an applied move and of a contrast move of the same neighbourhood to the move log:
// 16 features each (w.r.t. the pattern b before the move) and the cost change / 1000.  One lane writes.
template <class RowPtr>
__device__ __forceinline__ void log_moves(const Bits &b, RowPtr row, int T, const ProdParams &pp, int slot_a, int64_t dc_a,
                                          int slot_b, int64_t dc_b, float *log_x, float *log_y,
                                          unsigned long long *log_n, int64_t cap) {
    if ((threadIdx.x & 63) != 0 || cap <= 0) return;
    const unsigned long long pos = atomicAdd(log_n, slot_b >= 0 ? 2ull : 1ull);
    float f[mlp::kF];
    if ((int64_t)pos < cap) {
        mlp::move_features(b, row, T, pp, slot_a, f);
        for (int i = 0; i < mlp::kF; ++i) log_x[pos * mlp::kF + i] = f[i];
        log_y[pos] = (float)dc_a / 1000.f;
    }
    if (slot_b >= 0 && (int64_t)pos + 1 < cap) {
        mlp::move_features(b, row, T, pp, slot_b, f);
        for (int i = 0; i < mlp::kF; ++i) log_x[(pos + 1) * mlp::kF + i] = f[i];
        log_y[pos + 1] = (float)dc_b / 1000.f;
    }
}

}  // namespace vns
