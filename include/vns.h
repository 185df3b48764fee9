/*
 * vns.h — C ABI of the MI355X (gfx950) variable neighbourhood search for the uncapacitated multi-item
 * economic lot-sizing problem with remanufacturing (Antoniadis & Sifaleras 2017).
 *
 * Problem (Section 2 of the paper): K products, T periods; per product k and period t a demand D(k,t) and
 * a quantity of returns R(k,t) that can be remanufactured and sold as new; per product the setup costs
 * kM(k) (manufacturing) and kR(k) (remanufacturing) and the unit holding costs hM(k) (serviceable stock)
 * and hR(k) (recoverable stock).  A solution is a pair of setup bit rows zM(k,t), zR(k,t); its lots and
 * inventories follow from the decode (a setup covers demand until the next setup of either type, returns
 * are used first, a remanufacture-only shortfall is made by the last manufacturing lot) and its cost is
 * setups plus holding, an exact int64.
 *
 * The search (Section 3): VND (Algorithm 1) applies, per product and per neighbourhood, the best move when
 * it strictly improves, until a pass changes nothing; GVNS (Algorithm 2, with the accept-if-better rule of
 * Section 1) shakes k random setup flips, runs the VND and accepts the result if it is cheaper.
 *
 * Moves: product k owns 4T slots — [0,T) flip zM(t); [T,2T) flip zR(t); [2T,3T-1) move a manufacturing
 * setup one period (swap zM(t), zM(t+1), a move only if they differ); 3T-1 pad; [3T,4T-1) the same for zR;
 * 4T-1 pad.  The global slot of local slot l of product k is 4T*k + l.
 *
 * Conventions for every call:
 *   - Input arrays are host pointers, read during the call and copied: the caller keeps ownership.
 *   - Output arrays are host pointers allocated by the caller, written only when the call returns VNS_OK.
 *   - Work runs on the context's stream (its own, or the one given to vns_bind_stream); every call that
 *     returns results waits for them before returning.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - After a VNS_EDEVICE error only vns_destroy and vns_last_error are valid (others return VNS_ESTATE).
 */
#ifndef VNS_H
#define VNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vns_ctx vns_ctx;

typedef enum vns_status {
    VNS_OK = 0,
    VNS_EINVAL = -1,   /* bad argument: NULL required pointer, size out of range, negative input */
    VNS_ENOMEM = -2,   /* device or host allocation failed                                       */
    VNS_EDEVICE = -3,  /* a HIP call failed (message in vns_last_error); the context is dead    */
    VNS_ERANGE = -4,   /* the exact-cost bounds cannot be guaranteed, or an infeasible solution  */
    VNS_ESTATE = -5    /* call not valid in the context's state                                  */
} vns_status;

/* Neighbourhood ids (bit masks). */
enum { VNS_NB_FLIP_M = 1, VNS_NB_FLIP_R = 2, VNS_NB_SHIFT = 4 };

#define VNS_T_MAX 128          /* periods per instance                                  */
#define VNS_K_MAX 1048576      /* products per instance                                 */
#define VNS_KSHAKE_MAX 64      /* largest shake size k_max                              */
#define VNS_ALL_CHAINS (-1)    /* chain argument of vns_eval_neighbourhood: every chain  */
#define VNS_PRICE_INF INT64_MAX
#define VNS_MLP_PARAMS 5313    /* float32 parameters of the learned move scorer                  */
#define VNS_MLP_FEATURES 16    /* features per move                                             */

/* Options (vns_set_option / vns_get_option). */
enum vns_option {
    VNS_OPT_CHAINS = 1,   /* chains per instance, 1..65536 (default 1); setting it resets every chain    */
    VNS_OPT_KMAX = 2,     /* largest shake size k_max, 1..VNS_KSHAKE_MAX (default 5)                    */
    VNS_OPT_NB_LIST = 3,  /* VND neighbourhood order, one id per 4-bit nibble, lowest nibble first,
                             up to 4 entries (default 0x421 = flip zM, flip zR, shift)                   */
    VNS_OPT_TRACE = 4,    /* 1 = vns_run keeps one record per chain and iteration (default 1)           */
    VNS_OPT_RUN_WAVES = 5, /* wavefronts per workgroup of the search kernel, 1..8 (default 8)           */
    VNS_OPT_EVAL_GROUP = 6, /* chains of one instance priced together by one pricing workgroup, 1..16
                              (default 4); a tuning knob, results do not depend on it                   */
    VNS_OPT_RUN_LDS = 7,   /* bytes of LDS the search kernel may use to keep an instance's rows resident,
                              0..131072 (default 65536); a tuning knob, results do not depend on it     */
    VNS_OPT_GRAPH = 8,     /* 1 = vns_run captures its launch (search kernel + iteration-counter advance)
                              in a HIP graph once per (iters, layout) and replays it (default 0); needs a
                              stream other than the legacy default stream                               */
    VNS_OPT_LEARNED = 9,   /* 0 = plain VND; p in 1..1000 = learned VND: in every neighbourhood evaluation
                              the scorer ranks the moves, the best-ranked ceil(p*n/1000) are priced
                              exactly and the best of them is applied if it improves, otherwise the whole
                              neighbourhood is priced exactly and its best move applied if it improves   */
    VNS_OPT_LOG = 10,      /* move-log capacity in records (0 = off, default); a plain vns_run appends, for
                              every applied move, its features and cost change and those of one other
                              priced move of the same evaluation                                       */
    VNS_OPT_SPECULATE = 11, /* plain search only: 1 = each product's VND runs on a group of wavefronts,
                              one per neighbourhood of the list, pricing the neighbourhoods not yet
                              settled in the current pass side by side and applying, in list order, the
                              first improving one (the others are priced again); the moves applied are
                              those of the sequential pass and only consumed evaluations are counted.
                              0 (default) = one wavefront per product, neighbourhoods in turn           */
    VNS_OPT_SPEC_WAVES = 12, /* wavefronts per workgroup of the speculative search, 1..16 (default 16)  */
    VNS_OPT_STATE_LDS = 13, /* 1 (default) = the search kernel keeps each chain's current and working
                              solutions and costs (80 bytes per product) in LDS for the whole launch
                              when they fit beside the per-wavefront row slices; 0 = in device memory.
                              Results do not depend on it                                             */
    VNS_OPT_VND_MEMO = 14,  /* 1 = a VND pass skips a neighbourhood already priced without improvement
                              since the product's last applied move (its pattern has not changed, so it
                              would find nothing again): the same moves are applied and the records are
                              the same, with fewer move-evaluations.  0 (default) = every neighbourhood
                              is priced in every pass, as Algorithm 1 states.  Not used by the
                              speculative search                                                      */
    VNS_OPT_SPEC_ITERS = 15, /* m in 1..16 (default 1 = off): a rejected iteration leaves x unchanged and
                              the shake of an iteration depends only on (seed, chain, iteration, k), so
                              m workgroups per chain compute the next m iterations side by side as if
                              the earlier ones were rejected; they are resolved in order and what
                              follows the first accepted one is discarded.  Records, solutions and
                              counted move-evaluations equal those of the one-workgroup search.  A round
                              is resolved once the iterations up to its first accepted one are done; the
                              workgroups computing later ones abandon them.  Used for the plain and the
                              learned search when every workgroup of the launch can be resident
                              at once, the move log is off and the run is not captured in a graph;
                              otherwise the run falls back to one workgroup per chain
                              (vns_stats.last_run_spec_iters = 1).  A chain's workgroups wait for each
                              other with bounded spins: if one runs out, vns_run returns VNS_EDEVICE */
    VNS_OPT_BEST_OF = 16,  /* G in 0..16 (default 0 = off; 1 = the plain chain): the search of Algorithm 2,
                              whose GPUs shake the same solution and keep the minimum (Section 3).  Every
                              iteration shakes x G times with the same k, with random streams 0..G-1 (the
                              third Philox counter word; stream 0 is the plain chain's shake), runs the VND
                              on each, and selects the lowest objective (lowest stream among equals;
                              vns_record.winner).  It moves to it iff strictly better, with the usual k
                              schedule.  Runs as G workgroups per chain in one cooperative launch: vns_run
                              returns VNS_EINVAL if they cannot all be resident, or with the learned
                              scorer, speculative VND, speculative iterations, move log or graph
                              capture.  Every stream's move-evaluations count                        */
    VNS_OPT_BEST_OF_LITERAL = 17, /* 0/1 (default 0): best-of-G as Algorithm 2 prints it: k never changes and
                              the selected result always replaces x (accepted = 1 in every record);
                              with VNS_OPT_BEST_OF = 0 or 1 it runs one stream                       */
    VNS_OPT_EVAL_INCREMENTAL = 18, /* 0/1 (default 0): vns_eval_neighbourhood prices every move exactly but
                              decodes it only from its first changed period, starting from the current
                              pattern's state there, until its state equals the current pattern's again
                              (the rest of the cost then differs by known amounts) or it turns
                              infeasible.  Same prices, argmins and counted evaluations;
                              vns_stats.last_eval_decoded_steps reports the period-steps decoded      */
    VNS_OPT_DECODE = 19,   /* decode reading, a bit set (default 0); the paper leaves both points open
                              (Section 2 names returns and recoverable stock without the rules):
                              bit 1 (strict): a period whose latest setup is remanufacturing only must be
                              covered by the returns there; a shortfall makes the pattern infeasible
                              instead of being made and held by the last manufacturing lot;
                              bit 2 (disposal): returns no lot needs are disposed of at no cost, and
                              recoverable holding is charged on the stock later lots still need, per
                              period yR(t) - min over s >= t of yR(s).  Setting it restarts every chain
                              from the initial solution.  The learned search, the speculative VND,
                              incremental pricing and vns_eval_learned take only 0 (VNS_EINVAL)       */
    VNS_OPT_LEARNED_PACK = 20, /* learned VND only: P in 2..8 = a workgroup's wavefronts run the VNDs of up to
                              P products in lockstep together (packed form), pricing their selections
                              in shared passes and their fallbacks in shared passes; 0 or 1 (default 0)
                              = one product per wavefront at a time.  Moves, prices, records and counted
                              evaluations are the same.  The workgroup then needs 2 KB of LDS per
                              wavefront and 2.1 KB per product                                       */
    VNS_OPT_EVAL_SPREAD = 21 /* vns_eval_neighbourhood's launch shape: W in {4, 8, 12, 16} = the (chain,
                              product) pairs of each instance, product by product, are split into
                              near-equal ranges, 24 / W workgroups of W wavefronts per compute unit
                              (one for W = 16), each pricing every move of its range (a range spans a
                              few products when their rows fit its LDS); 0 (default) = one workgroup
                              per product and group of VNS_OPT_EVAL_GROUP chains.  Same prices and
                              argmins.  Not used with incremental pricing                             */
};

/* One GVNS iteration of one chain. */
typedef struct vns_record {
    int32_t iter;      /* absolute iteration index (continues across vns_run calls)                     */
    int32_t k;         /* shake size used                                                               */
    int32_t accepted;  /* 1 if the VND result replaced the current solution                             */
    int32_t winner;    /* best-of-G search: the random stream whose result was selected; otherwise 0      */
    int64_t F_shaken;  /* objective after the shake (of the winner)                                     */
    int64_t F_local;   /* objective after the VND (of the winner)                                       */
    int64_t F_best;    /* best objective of the chain so far                                            */
} vns_record;

typedef struct vns_stats {
    int64_t iterations;      /* GVNS iterations run per chain since creation or the last reset            */
    int64_t move_evals;      /* exactly priced moves (valid slots) in all chains since creation            */
    int64_t last_run_evals;  /* move-evaluations of the last vns_run call                                 */
    double last_run_ms;      /* device time of the last vns_run call (HIP events on the context stream)  */
    int64_t last_eval_evals; /* move-evaluations of the last vns_eval_neighbourhood call                  */
    double last_eval_ms;     /* device time of the pricing kernel of that call                           */
    int64_t last_run_period_steps;   /* sum over the last run's move-evaluations of their instance's T   */
    int64_t last_eval_period_steps;  /* the same for the last vns_eval_neighbourhood call                */
    int64_t last_run_learned_evals;  /* learned VND: neighbourhood evaluations of the last run           */
    int64_t last_run_fallbacks;      /*   and how many of them priced the whole neighbourhood            */
    double last_mlp_ms;              /* device time of the kernels of the last vns_mlp_score / _grad / _train */
    int64_t last_mlp_rows;           /*   and the feature rows they processed (rows x epochs for training)   */
    int64_t last_run_spec_iters;     /* iterations computed side by side per chain by the last vns_run (1 or
                                        VNS_OPT_SPEC_ITERS)                                               */
    int64_t last_run_discarded_evals;/*   and the move-evaluations of its iterations that followed an accepted
                                        one in their round, computed and thrown away (not in
                                        last_run_evals); abandoned iterations count what they computed
                                        before they stopped, so this figure varies from run to run        */
    int64_t last_eval_decoded_steps; /* period-steps the last vns_eval_neighbourhood decoded (equal to the
                                        evaluations' period-steps unless VNS_OPT_EVAL_INCREMENTAL)          */
} vns_stats;

/*
 * vns_create — one instance (Section 2 data).
 *   K in [1, VNS_K_MAX], T in [1, VNS_T_MAX].
 *   D, R: [K*T] int32, row-major [k][t], all >= 0 and < 2^24.
 *   kM, kR, hM, hR: [K] int32, all >= 0.
 *   seed: Philox key word 0 for every chain (word 1 is the chain index).
 * The context starts with 1 chain whose solution is zM = 1, zR = 0 (every period manufactures its own
 * demand), shake size 1, iteration 0.  Returns VNS_ERANGE if a product's cost or the int32 accumulators of
 * the decode could overflow (per product: sum(D)*T and sum(R)*T must stay below 2^31, the worst-case cost
 * below 2^47).  *out receives the context (NULL on error).
 */
vns_status vns_create(int32_t K, int32_t T, const int32_t *D, const int32_t *R, const int32_t *kM,
                      const int32_t *kR, const int32_t *hM, const int32_t *hR, uint64_t seed, vns_ctx **out);

/*
 * vns_create_batch — n_inst independent instances in one context (same rules as vns_create for each).
 *   K, T: [n_inst] sizes.  D, R: concatenation of the instances' [K_i*T_i] rows.  kM, kR, hM, hR:
 *   concatenation of the [K_i] vectors.  Chain c of instance i has the global chain index
 *   i*n_chains + c, which is also its Philox key word 1.
 */
vns_status vns_create_batch(int32_t n_inst, const int32_t *K, const int32_t *T, const int32_t *D,
                            const int32_t *R, const int32_t *kM, const int32_t *kR, const int32_t *hM,
                            const int32_t *hR, uint64_t seed, vns_ctx **out);

/* vns_destroy — frees every device and host resource of the context; NULL is accepted. */
void vns_destroy(vns_ctx *ctx);

/*
 * vns_set_unit_costs — unit costs of a manufactured item (pM) and of a remanufactured item (pR) per product,
 * the p_M, p_R of Algorithm 1's signature: the objective adds pM * sum x_M + pR * sum x_R (every demanded item
 * is made once, so this is pM * (sum D - X) + pR * X with X the remanufactured total).  pM, pR: [sum of K over
 * the instances] int32 in [0, 2^16), products in instance order, host memory, copied.  Zero at creation.
 * Every chain keeps its solution; its costs are recomputed and its search state restarts as at creation
 * (F = best = the new objective, k = 1).  VNS_ERANGE if a product's worst-case cost would reach 2^47.
 */
vns_status vns_set_unit_costs(vns_ctx *ctx, const int32_t *pM, const int32_t *pR);

/* vns_set_option / vns_get_option — see enum vns_option.  VNS_EINVAL for an unknown key or a value out of
 * range. */
vns_status vns_set_option(vns_ctx *ctx, int32_t key, int64_t value);
vns_status vns_get_option(const vns_ctx *ctx, int32_t key, int64_t *value);

/* vns_bind_stream — run all later work on `hip_stream` (a hipStream_t; NULL = the context's own stream).
 * The caller keeps ownership and must keep it alive while the context uses it. */
vns_status vns_bind_stream(vns_ctx *ctx, void *hip_stream);

/*
 * Workspace: device memory that a call's kernels use only while the call runs.  By default the context
 * allocates it itself (hipMalloc, kept for later calls).  A caller that manages device memory (a framework's
 * caching allocator) can bind a buffer it owns instead; the flags say which calls take their scratch from it:
 *   VNS_WS_RUN          vns_run's speculative-iteration and best-of-G buffers (per chain a 128-byte control
 *                       line, per chain and slot a summary and 40 bytes per product), sized for the current
 *                       VNS_OPT_SPEC_ITERS / VNS_OPT_BEST_OF; nothing when neither is on;
 *   VNS_WS_EVAL         vns_eval_neighbourhood's table of pricing workgroups (40 bytes per (chain, product),
 *                       the most any chain range or VNS_OPT_EVAL_GROUP needs);
 *   VNS_WS_EVAL_PRICES  as VNS_WS_EVAL, plus the staging of slot prices for every chain (8 bytes per slot).
 * vns_workspace_bytes — bytes a workspace bound with `flags` must have under the current options (0 for no
 * flags).  vns_bind_workspace — bind `dev_ptr` (device memory of the context's device, 256-byte aligned,
 * `bytes` long) for the calls in `flags`; VNS_EINVAL if it is smaller than vns_workspace_bytes(flags), badly
 * aligned, or flags has unknown bits.  dev_ptr = NULL (or flags = 0) unbinds: the context allocates again.
 * The caller keeps ownership, must keep the buffer alive while it is bound, and must not touch it while a
 * call of this context runs.  A call whose scratch outgrows the bound buffer (options changed after the bind)
 * returns VNS_EINVAL without running; query the size again and rebind.
 */
#define VNS_WS_RUN 1u
#define VNS_WS_EVAL 2u
#define VNS_WS_EVAL_PRICES 4u
vns_status vns_workspace_bytes(const vns_ctx *ctx, uint32_t flags, size_t *bytes);
vns_status vns_bind_workspace(vns_ctx *ctx, void *dev_ptr, size_t bytes, uint32_t flags);

/*
 * vns_eval_neighbourhood — exact pricing of every move of the neighbourhoods in nb_mask (an OR of VNS_NB_*)
 * for the current solution of one chain, or of every chain (chain = VNS_ALL_CHAINS).  For a move of product
 * k, price = F - cost_k + cost_k(after the move), the objective the move would give (Section 3: the new
 * objective value of each product is computed independently).  Pads, swaps of equal bits, slots outside
 * nb_mask and moves that make the product infeasible get VNS_PRICE_INF.
 * Outputs (each may be NULL; per chain, chains concatenated in global chain order for VNS_ALL_CHAINS):
 *   slot_price     [4*K*T] int64 per chain
 *   prod_best      [K] int64: the lowest price of each product (VNS_PRICE_INF if none)
 *   prod_best_slot [K] int32: its local slot (lowest on ties), -1 if none
 *   best           [1] int64: the lowest price over the instance
 *   best_slot      [1] int32: its global slot 4T*k + l (lowest on ties), -1 if none
 */
vns_status vns_eval_neighbourhood(vns_ctx *ctx, uint32_t nb_mask, int32_t chain, int64_t *slot_price,
                                  int64_t *prod_best, int32_t *prod_best_slot, int64_t *best,
                                  int32_t *best_slot);

/*
 * vns_eval_neighbourhood_noalloc — for callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same pricing as vns_eval_neighbourhood, with
 * the same arguments, outputs (host pointers) and results, but it allocates nothing, on the device or on the
 * host.  Its scratch (evaluation counters, per-product argmin keys, the table of pricing workgroups, built on
 * the device, and the slot-price staging) lives in one static 8 MiB device array per GPU, held until the
 * process ends.  Limits: 56 bytes per (chain, product) priced, plus 8 bytes per slot when slot_price is
 * requested, plus 16 KiB, within the 8 MiB (for example every slot of one chain of 300 x 52, or the argmins
 * of 64 chains of 100 x 52); a larger request returns VNS_EINVAL without running.  Every call on a GPU shares
 * that GPU's array and it keeps the last call's contents (the call clears what must start at zero): calls
 * that overlap on one GPU, from several threads or streams, race.  It always decodes every move in full
 * (VNS_OPT_EVAL_INCREMENTAL is not used); prices and counted evaluations equal vns_eval_neighbourhood's.
 */
vns_status vns_eval_neighbourhood_noalloc(vns_ctx *ctx, uint32_t nb_mask, int32_t chain, int64_t *slot_price,
                                          int64_t *prod_best, int32_t *prod_best_slot, int64_t *best,
                                          int32_t *best_slot);

/*
 * vns_run — every chain advances `iters` GVNS iterations (Algorithm 2): Shake(x, k) with Philox4x64-10
 * (key (seed, chain), counter (iteration, draw, 0, 0)), VND (Algorithm 1) with the neighbourhood list,
 * accept if F strictly drops (k = 1), else k = k + 1 wrapping after k_max.  iters >= 0.  The whole run is
 * one device launch; with VNS_OPT_TRACE the records of this call replace those of the previous one.
 */
vns_status vns_run(vns_ctx *ctx, int32_t iters);

/* vns_get_cost — current objective F and the best objective seen, of one chain (either may be NULL). */
vns_status vns_get_cost(vns_ctx *ctx, int32_t chain, int64_t *F, int64_t *F_best);

/* vns_get_costs — F and the best objective of every chain, [vns_num_chains] int64 each (either may be
 * NULL): one device-to-host copy instead of one call per chain. */
vns_status vns_get_costs(vns_ctx *ctx, int64_t *F, int64_t *F_best);

/*
 * vns_get_solution — setup rows of one chain, [K*T] uint8 0/1 each, row-major [k][t]:
 *   which = VNS_SOLUTION_CURRENT: the current solution x;
 *   which = VNS_SOLUTION_BEST: the cheapest solution the chain has held (objective F_best of vns_get_cost),
 *   tracked on the device at every acceptance.  Under Algorithm 2's accept-if-better rule it is x itself;
 *   it differs from x only after best-of-G as printed (VNS_OPT_BEST_OF_LITERAL), whose selected result
 *   replaces x even when it is worse.  VNS_EINVAL for any other `which`.
 */
#define VNS_SOLUTION_CURRENT 0
#define VNS_SOLUTION_BEST 1
vns_status vns_get_solution(vns_ctx *ctx, int32_t chain, int32_t which, uint8_t *zM, uint8_t *zR);

/* vns_set_solution — replace the current solution of one chain ([K*T] uint8, nonzero = setup).  The
 * chain's search state restarts from it: best solution = x, best objective = the new F, shake size 1.
 * VNS_ERANGE if a product would be infeasible: x is then left unchanged and the search state restarts from
 * it in the same way. */
vns_status vns_set_solution(vns_ctx *ctx, int32_t chain, const uint8_t *zM, const uint8_t *zR);

/* vns_get_trajectory — records of the last vns_run for one chain: up to `cap` records into `rec`, the
 * number available into *n (both may be NULL/0 to query the count). */
vns_status vns_get_trajectory(vns_ctx *ctx, int32_t chain, vns_record *rec, int64_t cap, int64_t *n);

/* vns_get_stats — counters and device times, see vns_stats. */
vns_status vns_get_stats(const vns_ctx *ctx, vns_stats *out);

/*
 * Learned move scorer (an MLP 16 -> 64 -> 64 -> 1 with ReLU, bfloat16 weights and layer inputs on the
 * matrix cores, float32 accumulation) that ranks moves so that only the best-ranked are priced exactly.
 * Features of a move at period t (float32): one-hot type (flip zM, flip zR, swap zM, swap zR); zM(t), zR(t);
 * D(t)/200, R(t)/200, D(t-1)/200, D(t+1)/200 (0 outside the horizon); kM/2000, kR/2000, hM/8, hR/8;
 * (t - last setup <= t)/T (1 if none); (next setup > t - t)/T (T if none).
 * Parameters: VNS_MLP_PARAMS float32 = W1 [16][64] row-major, b1 [64], W2 [64][64], b2 [64], W3 [64], b3.
 * A new context starts from vns_mlp_init(ctx, seed of the context).
 */
vns_status vns_mlp_set_params(vns_ctx *ctx, const float *params);   /* also resets the Adam state       */
/* vns_mlp_init — He-uniform weights (U(-sqrt(6/fan_in), +sqrt(6/fan_in)) per layer), zero biases, Adam
 * state reset; the uniforms come from splitmix64 of seed + parameter index + 1 Weyl steps, so a seed gives
 * the same weights on every host. */
vns_status vns_mlp_init(vns_ctx *ctx, uint64_t seed);
vns_status vns_mlp_get_params(vns_ctx *ctx, float *params);
/* Scores of n feature rows ([n][16] float32) into scores [n]. */
vns_status vns_mlp_score(vns_ctx *ctx, const float *feats, int64_t n, float *scores);
/* Gradient (VNS_MLP_PARAMS float32, may be NULL) and value (may be NULL) of the mean squared error of the
 * scores of n rows against targets [n]. */
vns_status vns_mlp_grad(vns_ctx *ctx, const float *feats, const float *targets, int64_t n, float *grads, float *loss);
/* Adam (lr, betas 0.9 / 0.999, eps 1e-8) over `epochs` passes of minibatches of `batch` rows, each epoch in
 * the order (m*i + a_e) mod n with m coprime to n and a_e drawn from seed; *last_loss (may be NULL) receives
 * the last minibatch's loss.  The data are copied to the device for the call. */
vns_status vns_mlp_train(vns_ctx *ctx, const float *feats, const float *targets, int64_t n, int32_t epochs,
                         int32_t batch, float lr, uint64_t seed, float *last_loss);
/* Move log of plain runs (VNS_OPT_LOG): up to cap records into feats [cap][16] and targets [cap] (cost
 * change / 1000); *n receives the number stored.  Record order depends on chain scheduling. */
vns_status vns_get_move_log(vns_ctx *ctx, float *feats, float *targets, int64_t cap, int64_t *n);
/*
 * vns_eval_learned — the learned choice of one neighbourhood's move (nb: one VNS_NB_* id) for every product
 * of one chain's current solution, as the learned VND makes it: scores of every move, the best-ranked
 * ceil(top_permille*n/1000) priced exactly, the whole neighbourhood when none of those improves.
 * Outputs (each may be NULL): scores [4KT] (NaN where not a move), selected [4KT] (1 = priced before any
 * fallback), prod_best [K] price of the chosen move (VNS_PRICE_INF if none), prod_best_slot [K] its local
 * slot (-1), fallback [K] (1 = the whole neighbourhood was priced).
 */
vns_status vns_eval_learned(vns_ctx *ctx, uint32_t nb, int32_t chain, int32_t top_permille, float *scores,
                            uint8_t *selected, int64_t *prod_best, int32_t *prod_best_slot, uint8_t *fallback);

/* vns_instance_size — K and T of instance `inst`; vns_num_chains — total number of chains. */
vns_status vns_instance_size(const vns_ctx *ctx, int32_t inst, int32_t *K, int32_t *T);
int64_t vns_num_chains(const vns_ctx *ctx);

/* vns_last_error — text of the last error of the context (or of the last failed create when ctx is NULL);
 * valid until the next call on the same context. */
const char *vns_last_error(const vns_ctx *ctx);

/*
 * vns_test_inject_failure — for tests of the error paths, without a real device fault (per calling thread):
 *   kind = VNS_INJECT_ALLOC:  the `countdown`-th device allocation from now (1 = the next) fails as out of
 *                             memory, so the call making it returns VNS_ENOMEM;
 *   kind = VNS_INJECT_DEVICE: the `countdown`-th call on a live context from now reports a HIP failure, so it
 *                             returns VNS_EDEVICE and the context is dead (later calls: VNS_ESTATE);
 *   countdown = 0 clears the injection of that kind.  VNS_EINVAL for another kind or a negative countdown.
 */
#define VNS_INJECT_ALLOC 1
#define VNS_INJECT_DEVICE 2
vns_status vns_test_inject_failure(int32_t kind, int32_t countdown);

#ifdef __cplusplus
}
#endif

#endif /* VNS_H */
