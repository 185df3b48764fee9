// Data layout shared by the host runtime and the kernels of the lot-sizing VNS.
//
// Everything lives in HBM for the whole life of a context (the paper's Section 3 notes that keeping the
// data on the device, instead of copying it per VND call, is what made the GPU version pay off).
//
//   rows      int2 [sum over products of T]   (D(t), PR(t)) per period, PR = returns up to and including t
//   prod      ProdParams [P]                  per product of every instance (costs, row offset, sums)
//   chains    ChainInfo [G]                   per chain: its instance and where its products start
//   cur/work  Bits [sum over chains of K]     32-byte setup record per (chain, product): the current
//                                             solution x and the working copy x' / x'' of the search
//   cur_cost/work_cost int64 [same]           exact cost of each (chain, product)
//   cstate    ChainState [G]                  objective, best, shake size, counters
#pragma once
#include <stdint.h>

namespace vns {

constexpr int kWords = 4;          // 32-bit words per setup row: T <= 128
constexpr int kTMax = 32 * kWords;
constexpr int kShakeMax = 64;
constexpr int kMaxWaves = 16;     // wavefronts per search workgroup (8 for the sequential VND, 16 speculative)
constexpr int kEvalGroup = 16;
constexpr int kEvalPairs = 64;    // (chain, product) pairs one pricing workgroup may price
constexpr int kEvalProds = 8;     //   of at most this many products (short horizons: their rows share LDS)
constexpr int kEvalItems = 8192;  //   and at most this many moves
constexpr int kMultiMaxT = 31;          // search: neighbourhoods priced side by side when 2T + 1 lanes fit a wavefront
constexpr int kEvalTargetMoves = 1024;  // moves a pricing workgroup should get (4 passes of its 256 lanes)
constexpr int kEvalShortT = 32;         //   by pricing several products when T is at most this
constexpr int kSnapBytes = 24;          // incremental pricing: base state per chain and period (int4 + int2)
constexpr int kSnapLdsMax = 40 * 1024;  //   and the dynamic LDS a pricing workgroup may use for them
// Workgroup counters are spread over kCounterSlots slots, kCounterStride words apart (one 64-byte line
// each): every workgroup adding to one device-scope address serialises the launch on that address.
constexpr int kCounterSlots = 256;
constexpr int kCounterStride = 8;
__host__ __device__ constexpr int counter_words() { return kCounterSlots * kCounterStride; }
constexpr int64_t kRunLdsMax = 128 * 1024;  // dynamic LDS the search kernel may request for instance rows
constexpr int kMaxPasses = 1 << 16;  // VND passes per product and iteration: a guard, not a limit of the method
constexpr int64_t kInf = INT64_MAX;
constexpr uint64_t kInfKey = ~0ull;
constexpr int kSlotBits = 16;      // argmin key = cost << 16 | local slot; cost < 2^47 is checked at create

struct Bits {
    uint32_t m[kWords];   // zM, bit t of word t/32
    uint32_t r[kWords];   // zR
};

struct ProdParams {
    int32_t kM, kR, hM, hR;
    // the cost's constant part and the coefficient of the remanufactured total XR (the decode reads these):
    //   C = hM * S_tD + hR * S_PR + pM * SD,  cXR = pR - pM - hR * T
    int64_t C;
    int64_t cXR;
    int32_t T;
    int32_t row;    // offset of the product's first period in rows
    int64_t S_tD;   // sum_t t * D(t)
    int64_t S_PR;   // sum_t PR(t)
    int64_t SD;     // sum_t D(t): the items made, sum x_M + sum x_R
    int32_t pM, pR; // unit costs of a manufactured and a remanufactured item (0 unless set)
};
// The two derived fields of a product.
inline void set_cost_terms(ProdParams &pp) {
    pp.C = (int64_t)pp.hM * pp.S_tD + (int64_t)pp.hR * pp.S_PR + (int64_t)pp.pM * pp.SD;
    pp.cXR = (int64_t)pp.pR - pp.pM - (int64_t)pp.hR * pp.T;
}

struct ChainInfo {
    int32_t inst;
    int32_t K;
    int32_t T;
    int32_t prod0;  // global index of product 0 of the chain's instance
    int64_t cp0;    // index of the chain's product 0 in the cur/work arrays
};

struct ChainState {
    int64_t F;
    int64_t F_best;
    int64_t evals;  // move-evaluations of this chain during the last run
    int32_t k;      // shake size for the next iteration
    int32_t lopt;   // 1 when every product of x is known to be a VND local optimum
    int32_t err;    // nonzero if a VND exceeded kMaxPasses (cannot happen with a consistent decode)
    int32_t bsync;  // 1 when the chain's best-solution rows hold x itself (so a cheaper x updates them
                    // product by product); 0 after x moved to a worse solution (best-of-G as printed)
    int64_t nb_evals;   // learned mode: neighbourhood evaluations during the last run
    int64_t fallbacks;  //   and how many of them priced the whole neighbourhood
    int64_t discarded;  // speculative iterations: move-evaluations of iterations computed and thrown away
};

struct Record {    // identical layout to vns_record
    int32_t iter, k, accepted, winner;
    int64_t F_shaken, F_local, F_best;
};

struct RunArgs {
    const ChainInfo *chains;
    const ProdParams *prod;
    const int2 *rows;
    Bits *cur;
    int64_t *cur_cost;
    Bits *work;
    int64_t *work_cost;
    ChainState *cstate;
    Bits *best;             // [sum over chains of K] the chain's best solution so far (objective F_best)
    Record *trace;          // [G][iters] or nullptr
    const int64_t *it0;     // device iteration counter: the first iteration of this launch
    uint64_t seed;
    int32_t iters;
    int32_t kmax;
    uint32_t nb_list;       // one neighbourhood id per nibble
    int32_t n_nb;
    int32_t lds_rows;       // int2 entries of dynamic LDS for an instance's rows: a chain whose instance has
                            // at most that many periods in total keeps them all in LDS for the whole launch
    int32_t permille;       // learned scorer: price the best-ranked permille/1000 of each neighbourhood; 0 = off
    int32_t learned_pack;   // learned VND: > 1 = products per workgroup batch (packed form), else one at a time
    const float *mlp;       // scorer parameters (5313 float32)
    float *log_x;           // move log: [log_cap][16] features, [log_cap] targets, count (null = off)
    float *log_y;
    unsigned long long *log_n;
    int64_t log_cap;
    int32_t state_off;      // byte offset in dynamic LDS of the chain's solution state (cur, work, their
                            // costs: 80 bytes per product, 16-byte aligned); -1 = kept in device memory
    int32_t memo;           // 1 = skip a neighbourhood priced without improvement on the current pattern
    // speculative iterations (cooperative launch): m workgroups per chain, see CoopCtl
    int32_t coop_m;             // iterations speculated per round
    int32_t coop_xcd;           // 1 = a chain's m workgroups are placed on one XCD (chains % 8 == 0)
    int32_t coop_kmax;          // products per chain slot in coop_res (the largest K)
    struct CoopCtl *coop_ctl;   // [chains]
    struct CoopSlot *coop_slot; // [chains][m]
    Bits *coop_res;             // [chains][m][coop_kmax] VND results of a slot
    int64_t *coop_res_cost;     // [chains][m][coop_kmax]
    int64_t coop_wait_ticks;    // ticks of the device's steady clock a wait for the chain may last
    int32_t best_of;            // 1: best-of-G search (Algorithm 2): the coop_m workgroups of a chain shake the
                                //    same x with streams 0 .. coop_m-1 and the minimum is kept
    int32_t best_literal;       // best-of-G as printed: k fixed, the minimum always replaces x
};

// Speculative iterations.  A rejected GVNS iteration leaves x unchanged, and its shake depends only on
// (seed, chain, iteration, k), so the m iterations that follow a state are computed side by side, each by
// its own workgroup, as if the earlier ones were rejected; they are then resolved in order and everything
// after the first accepted one is discarded.  Records, moves and counted evaluations are those of the
// sequential search.  The leader resolves a round as soon as the slots up to its first accepted iteration
// have reported; the workgroups still computing later iterations see the round counter move and abandon
// them.  Per chain, in device memory (set up by the host before each launch):
struct alignas(128) CoopCtl {   // one cache line per chain
    int32_t round;        // rounds completed (the leader increments it to start the next round)
    int32_t exited;       // workgroups of the chain that have left the launch
    int64_t iters_done;   // iterations of this launch resolved so far
    int64_t evals;        // move-evaluations of the resolved iterations
    int64_t executed;     // move-evaluations every workgroup of the chain computed, abandoned ones included
    int64_t nb_evals;     // learned search: neighbourhood evaluations of the resolved iterations
    int64_t fallbacks;    //   and how many of them priced the whole neighbourhood
    int32_t abort;        // a bounded wait ran out: every workgroup of the chain leaves
    int32_t err;
};
struct CoopSlot {
    int64_t F_local, F_shaken, evals;
    int64_t nb_evals, fallbacks;   // learned search: the iteration's neighbourhood evaluations and fallbacks
    int32_t n_touch;      // products in dp (K = every product: the VND of a state not yet a local optimum)
    int32_t err;
    int32_t stamp;        // 1 + the round this summary belongs to (0: none in this launch)
    int32_t dp[kShakeMax];
};
constexpr double kCoopWaitSeconds = 20.0;       // a wait for the other workgroups of a chain gives up after this
constexpr uint32_t kCoopSpinLimit = 1u << 28;   // and after this many polls (at least ~14 s), should the clock stall

// Dynamic LDS of the search kernel: the rows region (int2 entries, an even number so that what follows is
// 16-byte aligned), then per wavefront the learned-search tiles, then (optionally) the chain's solution
// state.
constexpr int kLearnedWaveBytes = 64 * 16 * 2 + 2 * kTMax * 2;
static_assert(kLearnedWaveBytes % 16 == 0, "learned tiles stay 16-byte aligned");
// The packed learned VND (VNS_OPT_LEARNED_PACK): batches of up to P <= kPackMax products per workgroup.  Its
// region: a feature tile per wavefront, a 16-byte control block, then per product its record
// (kPackProdBytes), move list, selection and staged row.
constexpr int kPackMax = 8;
constexpr int kPackProdBytes = 128;
constexpr int kPackPerProduct = kPackProdBytes + 2 * (2 * kTMax * 2) + kTMax * 8;
__host__ __device__ inline int pack_region_bytes(int W, int P) { return W * 64 * 16 * 2 + 16 + P * kPackPerProduct; }
static_assert(kPackPerProduct % 16 == 0, "packed regions stay 16-byte aligned");
__host__ __device__ inline int run_rows_entries(int lds_rows, int waves) {
    const int e = lds_rows > waves * kTMax ? lds_rows : waves * kTMax;
    return (e + 1) & ~1;
}

// One pricing workgroup: products p .. p+np-1 of chains g0 .. g0+n-1 of one instance (chains of an instance
// are consecutive, their products K apart; its products' rows are consecutive).  n = 0: an empty entry.
// Range form (G > 0): the n (chain, product) pairs q0 .. q0+n-1 of the instance's G chains g0 .. g0+G-1,
// numbered product-major (pair q: product q / G, chain g0 + q % G); p = q0 / G is the first product and np
// the products the range spans.  Everything the workgroup needs to start is here, so its first loads do
// not wait on one another.
struct EvalWg {
    int64_t cp;      // (chain g0, product p) index into the solution arrays
    int32_t g0, n;   // first chain, number of chains (range form: number of pairs)
    int32_t K, T;    // the instance's products and periods
    int32_t p;       // first product index within the instance
    int32_t prod;    // its global product index (ProdParams)
    int32_t row;     // offset of its row
    int32_t np;      // products (1, or more for short horizons)
    int32_t q0, G;   // range form: first pair and the instance's chains; G = 0 otherwise
};
static_assert(sizeof(EvalWg) == 48, "the allocation-free pricing call documents 48 + 8 bytes per pair");

// The pricing workgroup table built on the device, for the allocation-free pricing call: entry i is the
// (chain, product) cp_begin + i; a chain leads a group when it is the first of its instance in the range or
// `group` chains after the previous leader, and a non-leader's entry is empty (n = 0: its workgroup exits).
struct EvalPrepArgs {
    const ChainInfo *chains;
    const ProdParams *prod;
    const int32_t *cp_chain;
    int64_t cp_begin, n_cp;
    int32_t g0, ng, group, chains_per_inst;
    EvalWg *table;                // [n_cp]
    unsigned long long *counters; // counter_words() words, set to zero
};

struct EvalArgs {
    const int32_t *cp_chain;     // [sum over chains of K] chain of each (chain, product)
    const ChainInfo *chains;
    const ProdParams *prod;
    const int2 *rows;
    const Bits *cur;
    const int64_t *cur_cost;
    const ChainState *cstate;
    int64_t *slot_price;         // optional [sum over chains of 4*K*T]
    const int64_t *price_off;    // [G] offset of each chain's slot block in slot_price
    uint64_t *prod_key;          // [sum over chains of K]: cost << 16 | slot of each product's best move
    unsigned long long *evals;   // device counters, kCounterSlots slots: [0] move-evaluations, [1] their period-steps,
                                 // [2] period-steps decoded
    uint32_t nb_mask;
};

}  // namespace vns
