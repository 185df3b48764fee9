// Kernel argument blocks and host-side launchers of the lot-sizing VNS kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vns_types.hpp"

namespace vns {

struct InitArgs {
    const ChainInfo *chains;
    const ProdParams *prod;
    const int2 *rows;
    const Bits *cur;
    int64_t *cur_cost;
    Bits *work;
    int64_t *work_cost;
    ChainState *cstate;
    Bits *best;          // the best solution starts as the current one
    int32_t chain0;
};

struct ChainBestArgs {
    const ChainInfo *chains;
    const ChainState *cstate;
    const int64_t *cur_cost;
    const uint64_t *prod_key;
    int64_t *prod_price;   // [cp] price of each product's best move
    int32_t *prod_slot;    // [cp] its local slot
    int64_t *best;         // [chains of the launch]
    int32_t *best_slot;
    int32_t chain0;
};

// Variants of the search kernel: sequential VND, speculative VND, learned VND.
// kPlainShort: the plain search kernel with consecutive neighbourhoods priced side by side in one pass at
// horizons up to kMultiMaxT (launched when an instance has one; the same moves and counts as kPlain).
enum class RunKind { kPlain = 0, kSpec = 1, kLearned = 2, kLearnedPacked = 3, kPlainShort = 4 };

// Static LDS bytes of a search kernel variant, and permission for it to request dynamic_bytes more.
// model: the decode reading (kModelStrict | kModelDispose; the plain sequential VND only).
hipError_t run_kernel_lds(RunKind kind, size_t *static_bytes, size_t dynamic_bytes, int model);
// Learned scorer (vns_mlp.hip).  P: 5313 float32 parameters.  Scores of n feature rows [n][16].
hipError_t launch_mlp_score(const float *P, const float *X, int64_t n, float *out, hipStream_t s);
// Gradient (and loss in grad_out[5313]) of the mean squared error over rows idx[0..n) (all rows when idx is
// null): forward and backward on the matrix cores, one partial per wavefront in part
// [mlp_grad_partials(n)][5314], then their fixed-order sum.
hipError_t launch_mlp_grad(const float *P, const float *X, const float *y, const int64_t *idx, int64_t n, float *part,
                           float *grad_out, hipStream_t s);
int64_t mlp_grad_partials(int64_t n);
// Training rows of a minibatch: row r of it is (mul (start + r) + add) mod n of the training set.
struct RowPerm {
    uint64_t mul, add;
    int64_t start, n;
};
// One training step (Adam step number `step`): the gradient of the minibatch's cnt rows (partials in part,
// sized for mlp_grad_partials(cnt)), then in one kernel their fixed-order sum into grad_out (loss at
// [5313]) and the Adam update of P, m, v.
hipError_t launch_mlp_train_step(float *P, float *m, float *v, const float *X, const float *y, const RowPerm &perm,
                                 int64_t cnt, float *part, float *grad_out, float lr, int64_t step, hipStream_t s);
struct EvalLearnedArgs {
    const int32_t *cp_chain;
    const ChainInfo *chains;
    const ProdParams *prod;
    const int2 *rows;
    const Bits *cur;
    const int64_t *cur_cost;
    const ChainState *cstate;
    const float *mlp;
    const int64_t *slot_off;   // [G] first slot of each chain in scores / selected
    float *scores;             // optional: score of every move, by slot
    uint8_t *selected;         // optional: 1 for the moves priced exactly before any fallback
    int64_t *prod_price;       // [cp]
    int32_t *prod_slot;        // [cp]
    uint8_t *fallback;         // [cp]
    unsigned long long *evals; // kCounterSlots slots of kCounterStride words: [0] move-evaluations
    uint32_t nb;
    int32_t permille;
};

hipError_t launch_init(const InitArgs &a, int n_chains, hipStream_t s, int model);
hipError_t launch_eval_learned(const EvalLearnedArgs &a, int64_t cp_begin, int64_t n_cp, hipStream_t s);
// waves: 4 (k_eval) or 8, 12, 16 (k_eval_wide) wavefronts per workgroup.
hipError_t launch_eval(const EvalArgs &a, const EvalWg *wg, int64_t n_wg, hipStream_t s, int model, int waves = 4);
// The pricing table of a chain range and zeroed counters, built on the device (no host staging).
hipError_t launch_eval_prep(const EvalPrepArgs &a, hipStream_t s);
// Incremental pricing of the same sweep; lds_bytes of dynamic LDS hold each workgroup's base snapshots
// (kSnapBytes per chain and period 0..T).
hipError_t launch_eval_inc(const EvalArgs &a, const EvalWg *wg, int64_t n_wg, size_t lds_bytes, hipStream_t s);
hipError_t launch_chain_best(const ChainBestArgs &a, int n_chains, hipStream_t s);
// Speculative iterations (a.coop_m workgroups per chain, cooperative launch): whether blocks workgroups of
// `waves` wavefronts and lds_bytes of dynamic LDS are all resident at once, and the launch itself (then the
// device iteration counter advances by a.iters).  kind: kPlain (any decode reading `model`), kLearned or
// kLearnedPacked.
hipError_t coop_fits(int waves, size_t lds_bytes, int64_t blocks, bool *fits, RunKind kind, int model);
hipError_t launch_run_coop(const RunArgs &a, int n_chains, int waves, size_t lds_bytes, int64_t *it_counter,
                           hipStream_t s, RunKind kind, int model);
// The search kernel variant `kind` over n_chains workgroups, then the device iteration counter advances by a.iters (two kernels on s;
// both can be captured in a graph).
hipError_t launch_run(const RunArgs &a, RunKind kind, int n_chains, int waves, size_t lds_bytes, int64_t *it_counter,
                      hipStream_t s, int model);

}  // namespace vns
