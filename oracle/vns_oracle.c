/*
 * CPU oracle for the VNS of Antoniadis & Sifaleras (2017) on the uncapacitated multi-item economic
 * lot-sizing problem with remanufacturing.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the HIP path is checked
 * against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never links, calls or falls back to it.  It shares no code, header or table with
 * the HIP path.
 *
 * Everything is int64.  Bit rows are uint8 0/1 arrays laid out [k][t].  Nothing is blocked, fused or
 * reordered beyond the steps named in each comment:
 *   - problem data and objective: Section 2 of the paper, with the unit costs p_M, p_R that Algorithm 1's
 *     signature carries (zero unless given) (the decode itself is not printed there; the
 *     rules followed are the look-ahead decode of the lot-sizing reading: a setup covers demand until the
 *     next setup of either type, remanufacture first, carry a shortfall back to the last manufacturing lot);
 *   - VND: Algorithm 1 (per-product best move of one neighbourhood at a time, reduction of the gains,
 *     repeat until no improvement);
 *   - GVNS: Algorithm 2 and the VNS description of Section 1 (shake, VND, accept if better);
 *   - best-of-G GVNS: Algorithm 2 with the selection Section 3 describes for its two GPUs (G shakes of x
 *     with the same k, one VND each, the minimum kept), in the GVNS form and as printed;
 *   - Philox4x64-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF INT64_MAX

/* The reading of a remanufacture-only shortfall in force for this thread's calls:
 *   0 (default) carry-back (R5): the last manufacturing lot makes the shortfall and holds it;
 *   1 strict (R5-alt): a shortfall makes the pattern infeasible. */
static _Thread_local int orc_strict = 0;

void orc_set_strict(int strict)
{
    orc_strict = strict ? 1 : 0;
}

/* Disposal of returns in force for this thread's calls:
 *   0 (default) no disposal (R7): every return is held as recoverable stock until it is remanufactured or
 *     the horizon ends;
 *   1 disposal (R29): returns may be disposed of at no cost.  The lots are the decode's; the stock kept at the
 *     end of period t is what a later lot still needs, yR(t) - min_{s >= t} yR(s) with yR the stock without
 *     disposal (the rest is disposed of as it arrives), and recoverable holding is charged on the kept stock. */
static _Thread_local int orc_dispose = 0;

void orc_set_dispose(int dispose)
{
    orc_dispose = dispose ? 1 : 0;
}

/* ------------------------------------------------------------------------------------------------ */
/* Decode of one product (Section 2 quantities x_M, x_R, y_M, y_R).                                  */
/* Returns the cost, or ORC_INF when the pattern cannot meet demand.  The four arrays receive the     */
/* per-period lots and end-of-period inventories (they may be NULL).                                  */
/* ------------------------------------------------------------------------------------------------ */
int64_t orc_decode(int T, const int32_t *D, const int32_t *R,
                   int64_t kM, int64_t kR, int64_t hM, int64_t hR, int64_t pM, int64_t pR,
                   const uint8_t *zM, const uint8_t *zR,
                   int64_t *xM_out, int64_t *xR_out, int64_t *yM_out, int64_t *yR_out)
{
    int64_t *xM = (int64_t *)calloc((size_t)T + 1, sizeof(int64_t));
    int64_t *xR = (int64_t *)calloc((size_t)T + 1, sizeof(int64_t));
    int64_t *yM = (int64_t *)calloc((size_t)T + 1, sizeof(int64_t));
    int64_t *yR = (int64_t *)calloc((size_t)T + 1, sizeof(int64_t));
    int64_t cost = ORC_INF;
    int feasible = 1;
    int lastM = -1;                 /* last period with a manufacturing setup, -1 = none yet */
    int64_t yM_prev = 0, yR_prev = 0;

    for (int t = 0; t < T && feasible; ++t) {
        int setup = zM[t] || zR[t];
        /* next setup period of either type */
        int nxt = t + 1;
        while (nxt < T && !(zM[nxt] || zR[nxt])) ++nxt;

        int64_t avail = yR_prev + R[t];          /* returns of period t are usable in t */
        int64_t need = 0;
        if (setup) {
            int64_t interval_demand = 0;
            for (int tau = t; tau < nxt; ++tau) interval_demand += D[tau];
            need = interval_demand - yM_prev;
            if (need < 0) need = 0;
        }
        xR[t] = zR[t] ? (avail < need ? avail : need) : 0;   /* remanufacture first */
        xM[t] = zM[t] ? need - xR[t] : 0;                    /* manufacture the rest */

        int64_t shortfall = need - xR[t] - xM[t];
        if (shortfall > 0) {
            if (lastM < 0 || orc_strict) { feasible = 0; break; }
            /* the last manufacturing lot makes the shortfall and holds it until t */
            xM[lastM] += shortfall;
            for (int tau = lastM; tau < t; ++tau) yM[tau] += shortfall;
            yM_prev += shortfall;
        }
        if (zM[t]) lastM = t;

        yR[t] = avail - xR[t];
        yM[t] = yM_prev + xR[t] + xM[t] - D[t];
        if (yM[t] < 0) { feasible = 0; break; }
        yM_prev = yM[t];
        yR_prev = yR[t];
    }

    if (feasible) {
        int64_t nM = 0, nR = 0, sYM = 0, sYR = 0, sXM = 0, sXR = 0;
        for (int t = 0; t < T; ++t) {
            nM += zM[t];
            nR += zR[t];
            sYM += yM[t];
            sYR += yR[t];
            sXM += xM[t];
            sXR += xR[t];
        }
        if (orc_dispose) {
            /* recoverable holding on the kept stock only: subtract the suffix minima of the stock path */
            int64_t suffix_min = yR[T - 1], sMin = 0;
            for (int t = T - 1; t >= 0; --t) {
                if (yR[t] < suffix_min) suffix_min = yR[t];
                sMin += suffix_min;
            }
            sYR -= sMin;
        }
        /* setups, holding, and the unit costs of the items made (p_M, p_R of Algorithm 1's signature) */
        cost = kM * nM + kR * nR + hM * sYM + hR * sYR + pM * sXM + pR * sXR;
    }
    for (int t = 0; t < T; ++t) {
        if (xM_out) xM_out[t] = xM[t];
        if (xR_out) xR_out[t] = xR[t];
        if (yM_out) yM_out[t] = yM[t];
        if (yR_out) yR_out[t] = yR[t];
    }
    free(xM); free(xR); free(yM); free(yR);
    return cost;
}

/* Cost of product k of an instance laid out [k][t]. */
static int64_t product_cost(int k, int T, const int32_t *D, const int32_t *R,
                            const int32_t *kM, const int32_t *kR, const int32_t *hM, const int32_t *hR,
                   const int32_t *pM, const int32_t *pR,
                            const uint8_t *zM, const uint8_t *zR)
{
    size_t o = (size_t)k * (size_t)T;
    return orc_decode(T, D + o, R + o, kM[k], kR[k], hM[k], hR[k], pM[k], pR[k], zM + o, zR + o,
                      NULL, NULL, NULL, NULL);
}

/* Objective F = sum of product costs (ORC_INF if any product is infeasible); cost_k may be NULL. */
int64_t orc_objective(int K, int T, const int32_t *D, const int32_t *R,
                      const int32_t *kM, const int32_t *kR, const int32_t *hM, const int32_t *hR,
                   const int32_t *pM, const int32_t *pR,
                      const uint8_t *zM, const uint8_t *zR, int64_t *cost_k)
{
    int64_t F = 0;
    int inf = 0;
    for (int k = 0; k < K; ++k) {
        int64_t c = product_cost(k, T, D, R, kM, kR, hM, hR, pM, pR, zM, zR);
        if (cost_k) cost_k[k] = c;
        if (c == ORC_INF) inf = 1; else F += c;
    }
    return inf ? ORC_INF : F;
}

/* ------------------------------------------------------------------------------------------------ */
/* Moves.  Product k owns 4T slots: [0,T) flip zM(t); [T,2T) flip zR(t); [2T,3T-1) swap zM(t),zM(t+1);  */
/* 3T-1 pad; [3T,4T-1) swap zR(t),zR(t+1); 4T-1 pad.  A swap is a move only if the two bits differ.     */
/* ------------------------------------------------------------------------------------------------ */

/* Neighbourhood a local slot belongs to: 1 flip zM, 2 flip zR, 4 shift. */
int orc_slot_nb(int T, int l)
{
    if (l < T) return 1;
    if (l < 2 * T) return 2;
    return 4;
}

/* Apply local slot l to one product's bit rows in place.  Returns 0 (and changes nothing) if the slot is
 * a pad or a swap of two equal bits. */
int orc_apply_slot(int T, uint8_t *zM, uint8_t *zR, int l)
{
    if (l < 0 || l >= 4 * T) return 0;
    if (l < T) { zM[l] ^= 1; return 1; }
    if (l < 2 * T) { zR[l - T] ^= 1; return 1; }
    uint8_t *z = (l < 3 * T) ? zM : zR;
    int t = (l < 3 * T) ? l - 2 * T : l - 3 * T;
    if (t >= T - 1) return 0;            /* pad */
    if (z[t] == z[t + 1]) return 0;      /* no-op swap */
    uint8_t a = z[t];
    z[t] = z[t + 1];
    z[t + 1] = a;
    return 1;
}

/* Price every slot of every product whose neighbourhood is in nb_mask:
 * price = F - cost_k + cost_k(moved), ORC_INF for pads, no-op swaps, slots outside nb_mask and
 * infeasible results.  F and cost_k are those of the given solution (which must be feasible).
 * Returns the number of move-evaluations (valid slots priced). */
int64_t orc_price_all(int K, int T, const int32_t *D, const int32_t *R,
                      const int32_t *kM, const int32_t *kR, const int32_t *hM, const int32_t *hR,
                   const int32_t *pM, const int32_t *pR,
                      const uint8_t *zM, const uint8_t *zR, uint32_t nb_mask, int64_t *price)
{
    int64_t *cost = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    int64_t F = orc_objective(K, T, D, R, kM, kR, hM, hR, pM, pR, zM, zR, cost);
    uint8_t *wM = (uint8_t *)malloc((size_t)T);
    uint8_t *wR = (uint8_t *)malloc((size_t)T);
    int64_t evals = 0;
    for (int k = 0; k < K; ++k) {
        size_t o = (size_t)k * (size_t)T;
        for (int l = 0; l < 4 * T; ++l) {
            int64_t *p = &price[(size_t)k * 4 * (size_t)T + (size_t)l];
            *p = ORC_INF;
            if (!(orc_slot_nb(T, l) & nb_mask)) continue;
            memcpy(wM, zM + o, (size_t)T);
            memcpy(wR, zR + o, (size_t)T);
            if (!orc_apply_slot(T, wM, wR, l)) continue;
            ++evals;
            int64_t c = orc_decode(T, D + o, R + o, kM[k], kR[k], hM[k], hR[k], pM[k], pR[k], wM, wR,
                                   NULL, NULL, NULL, NULL);
            if (c != ORC_INF && F != ORC_INF) *p = F - cost[k] + c;
        }
    }
    free(wM); free(wR); free(cost);
    return evals;
}

/* Lexicographic (price, slot) minimum over n prices; *slot = -1 and ORC_INF when all are ORC_INF. */
int64_t orc_argmin(int64_t n, const int64_t *price, int64_t *slot)
{
    int64_t best = ORC_INF, bs = -1;
    for (int64_t i = 0; i < n; ++i)
        if (price[i] < best) { best = price[i]; bs = i; }
    *slot = bs;
    return best;
}

/* ------------------------------------------------------------------------------------------------ */
/* VND, Algorithm 1.  nb_list holds n_nb neighbourhood ids in order.  For each neighbourhood, every   */
/* product's best move (lowest slot on ties) is applied when it strictly lowers F; passes repeat until */
/* one changes nothing.  zM/zR are updated in place; returns the final F (the input must be feasible). */
/* *evals (may be NULL) accumulates the number of move-evaluations.  With trace non-NULL, every applied */
/* move appends (pass, neighbourhood id, product, local slot, F after the move), five int64 each, up   */
/* to trace_cap moves; *n_trace receives the number of moves applied.                                  */
/* ------------------------------------------------------------------------------------------------ */
int64_t orc_vnd_trace(int K, int T, const int32_t *D, const int32_t *R,
                      const int32_t *kM, const int32_t *kR, const int32_t *hM, const int32_t *hR,
                      const int32_t *pM, const int32_t *pR,
                      uint8_t *zM, uint8_t *zR, const int32_t *nb_list, int n_nb, int64_t *evals,
                      int64_t *trace, int64_t trace_cap, int64_t *n_trace)
{
    int64_t *cost = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    int64_t F = orc_objective(K, T, D, R, kM, kR, hM, hR, pM, pR, zM, zR, cost);
    uint8_t *wM = (uint8_t *)malloc((size_t)T);
    uint8_t *wR = (uint8_t *)malloc((size_t)T);
    int improvement;
    int64_t pass = 0, n_moves = 0;
    do {
        improvement = 0;
        for (int q = 0; q < n_nb; ++q) {
            for (int k = 0; k < K; ++k) {
                size_t o = (size_t)k * (size_t)T;
                /* find the best neighbour of product k in neighbourhood nb_list[q] */
                int64_t best_price = ORC_INF;
                int best_l = -1;
                for (int l = 0; l < 4 * T; ++l) {
                    if (!(orc_slot_nb(T, l) & nb_list[q])) continue;
                    memcpy(wM, zM + o, (size_t)T);
                    memcpy(wR, zR + o, (size_t)T);
                    if (!orc_apply_slot(T, wM, wR, l)) continue;
                    if (evals) ++*evals;
                    int64_t c = orc_decode(T, D + o, R + o, kM[k], kR[k], hM[k], hR[k], pM[k], pR[k], wM, wR,
                                           NULL, NULL, NULL, NULL);
                    if (c == ORC_INF) continue;
                    int64_t p = F - cost[k] + c;
                    if (p < best_price) { best_price = p; best_l = l; }
                }
                if (best_l >= 0 && best_price < F) {
                    orc_apply_slot(T, zM + o, zR + o, best_l);
                    cost[k] = cost[k] + (best_price - F);
                    F = best_price;
                    improvement = 1;
                    if (trace && n_moves < trace_cap) {
                        int64_t *r = trace + 5 * n_moves;
                        r[0] = pass; r[1] = nb_list[q]; r[2] = k; r[3] = best_l; r[4] = F;
                    }
                    ++n_moves;
                }
            }
        }
        ++pass;
    } while (improvement);
    if (n_trace) *n_trace = n_moves;
    free(wM); free(wR); free(cost);
    return F;
}

int64_t orc_vnd(int K, int T, const int32_t *D, const int32_t *R,
                const int32_t *kM, const int32_t *kR, const int32_t *hM, const int32_t *hR,
                const int32_t *pM, const int32_t *pR,
                uint8_t *zM, uint8_t *zR, const int32_t *nb_list, int n_nb, int64_t *evals)
{
    return orc_vnd_trace(K, T, D, R, kM, kR, hM, hR, pM, pR, zM, zR, nb_list, n_nb, evals, NULL, 0, NULL);
}

/* ------------------------------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC'11): 10 rounds of two 64x64->128 multiplies with the published     */
/* multipliers, key bumped by the published Weyl constants between rounds.                            */
/* ------------------------------------------------------------------------------------------------ */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t key[2], const uint64_t ctr[4], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, x0, &hi0, &lo0);
        mulhilo64(M1, x2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ x1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ x3 ^ k1;
        uint64_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Flip move f in [0, 2KT) of the shake: product f / 2T, then zM(t) for f mod 2T < T, else zR(t - T). */
static void flip_move(int T, int64_t f, int *k, int *l)
{
    *k = (int)(f / (2 * (int64_t)T));
    int r = (int)(f % (2 * (int64_t)T));
    *l = r;     /* local slot: [0,T) flip zM, [T,2T) flip zR — the same numbering as the slots */
}

/* Draw j of iteration `iter` of random stream g for chain key (seed, chain): index in [0, n).  Stream 0 is
 * the chain's own shake; the best-of-G search gives its G parallel shakes streams 0 .. G-1. */
int64_t orc_draw_stream(uint64_t seed, uint64_t chain, uint64_t iter, uint64_t j, uint64_t g, uint64_t n)
{
    uint64_t key[2] = {seed, chain};
    uint64_t ctr[4] = {iter, j, g, 0};
    uint64_t out[4];
    orc_philox4x64_10(key, ctr, out);
    return (int64_t)(((out[0] >> 32) * n) >> 32);
}

int64_t orc_draw(uint64_t seed, uint64_t chain, uint64_t iter, uint64_t j, uint64_t n)
{
    return orc_draw_stream(seed, chain, iter, j, 0, n);
}

/* Shake(x, k) with random stream g: k random flips, each skipped if it makes its product infeasible.
 * Returns the number of flips applied; applied[j] (may be NULL) receives 1/0 per draw. */
int orc_shake_stream(int K, int T, const int32_t *D, const int32_t *R,
                     const int32_t *kM, const int32_t *kR, const int32_t *hM, const int32_t *hR,
                   const int32_t *pM, const int32_t *pR,
                     uint8_t *zM, uint8_t *zR, int kshake, uint64_t seed, uint64_t chain, uint64_t iter,
                     uint64_t g, int32_t *applied)
{
    int n_applied = 0;
    uint64_t n = 2 * (uint64_t)K * (uint64_t)T;
    for (int j = 0; j < kshake; ++j) {
        int64_t f = orc_draw_stream(seed, chain, iter, (uint64_t)j, g, n);
        int k, l;
        flip_move(T, f, &k, &l);
        size_t o = (size_t)k * (size_t)T;
        orc_apply_slot(T, zM + o, zR + o, l);
        int64_t c = product_cost(k, T, D, R, kM, kR, hM, hR, pM, pR, zM, zR);
        if (c == ORC_INF) {
            orc_apply_slot(T, zM + o, zR + o, l);   /* undo: a flip is its own inverse */
            if (applied) applied[j] = 0;
        } else {
            if (applied) applied[j] = 1;
            ++n_applied;
        }
    }
    return n_applied;
}

int orc_shake(int K, int T, const int32_t *D, const int32_t *R,
              const int32_t *kM, const int32_t *kR, const int32_t *hM, const int32_t *hR,
                   const int32_t *pM, const int32_t *pR,
              uint8_t *zM, uint8_t *zR, int kshake, uint64_t seed, uint64_t chain, uint64_t iter,
              int32_t *applied)
{
    return orc_shake_stream(K, T, D, R, kM, kR, hM, hR, pM, pR, zM, zR, kshake, seed, chain, iter, 0, applied);
}

/* One trajectory record per GVNS iteration. */
typedef struct {
    int32_t iter;
    int32_t k;
    int32_t accepted;
    int32_t winner;   /* best-of-G: the stream whose result was selected (0 for a plain chain) */
    int64_t F_shaken;
    int64_t F_local;
    int64_t F_best;
} orc_record;

/* GVNS (Algorithm 2 with the accept-if-better rule of Section 1) for one chain.
 * In/out state: zM, zR (current solution x), *k (shake size), *F_best.  Iterations it0 .. it0+iters-1
 * are run; rec (may be NULL) receives one record per iteration.  Returns F(x) at the end; *evals (may be
 * NULL) accumulates move-evaluations. */
int64_t orc_gvns(int K, int T, const int32_t *D, const int32_t *R,
                 const int32_t *kM, const int32_t *kR, const int32_t *hM, const int32_t *hR,
                   const int32_t *pM, const int32_t *pR,
                 uint8_t *zM, uint8_t *zR, const int32_t *nb_list, int n_nb, int k_max,
                 uint64_t seed, uint64_t chain, int64_t it0, int64_t iters, int32_t *k_state,
                 int64_t *F_best, orc_record *rec, int64_t *evals)
{
    size_t n = (size_t)K * (size_t)T;
    uint8_t *sM = (uint8_t *)malloc(n);
    uint8_t *sR = (uint8_t *)malloc(n);
    int64_t F = orc_objective(K, T, D, R, kM, kR, hM, hR, pM, pR, zM, zR, NULL);
    for (int64_t i = 0; i < iters; ++i) {
        int64_t it = it0 + i;
        int k = *k_state;
        memcpy(sM, zM, n);
        memcpy(sR, zR, n);
        orc_shake(K, T, D, R, kM, kR, hM, hR, pM, pR, sM, sR, k, seed, chain, (uint64_t)it, NULL);
        int64_t F_shaken = orc_objective(K, T, D, R, kM, kR, hM, hR, pM, pR, sM, sR, NULL);
        int64_t F_local = orc_vnd(K, T, D, R, kM, kR, hM, hR, pM, pR, sM, sR, nb_list, n_nb, evals);
        int accepted = F_local < F;
        if (accepted) {
            memcpy(zM, sM, n);
            memcpy(zR, sR, n);
            F = F_local;
            *k_state = 1;
        } else {
            *k_state = (k >= k_max) ? 1 : k + 1;
        }
        if (F < *F_best) *F_best = F;
        if (rec) {
            rec[i].iter = (int32_t)it;
            rec[i].k = k;
            rec[i].accepted = accepted;
            rec[i].winner = 0;
            rec[i].F_shaken = F_shaken;
            rec[i].F_local = F_local;
            rec[i].F_best = *F_best;
        }
    }
    free(sM); free(sR);
    return F;
}

/* Best-of-G GVNS, the search of Algorithm 2: in every iteration G copies of x are shaken with the same k,
 * each by its own random stream g, and each runs the VND; the objective values are compared and the
 * minimum one is selected (the lowest g among equal values), as Section 3 describes for the two GPUs.
 *   literal = 0: the selected result replaces x iff it is strictly better, and k follows the GVNS rule of
 *                Section 1 (k = 1 after a move, else k + 1, back to 1 after k_max);
 *   literal = 1: Algorithm 2 as printed: k never changes, and the selected result always replaces x
 *                (accepted = 1 in every record).
 * State, records (winner = the selected stream, F_shaken / F_local of that stream) and evaluations (all G
 * VNDs) as in orc_gvns. */
int64_t orc_gvns_best_of(int K, int T, const int32_t *D, const int32_t *R,
                         const int32_t *kM, const int32_t *kR, const int32_t *hM, const int32_t *hR,
                   const int32_t *pM, const int32_t *pR,
                         uint8_t *zM, uint8_t *zR, const int32_t *nb_list, int n_nb, int k_max, int G,
                         int literal, uint64_t seed, uint64_t chain, int64_t it0, int64_t iters,
                         int32_t *k_state, int64_t *F_best, orc_record *rec, int64_t *evals)
{
    size_t n = (size_t)K * (size_t)T;
    uint8_t *sM = (uint8_t *)malloc(n), *sR = (uint8_t *)malloc(n);
    uint8_t *bM = (uint8_t *)malloc(n), *bR = (uint8_t *)malloc(n);
    int64_t F = orc_objective(K, T, D, R, kM, kR, hM, hR, pM, pR, zM, zR, NULL);
    for (int64_t i = 0; i < iters; ++i) {
        int64_t it = it0 + i;
        int k = *k_state;
        int best_g = -1;
        int64_t best_local = 0, best_shaken = 0;
        for (int g = 0; g < G; ++g) {
            memcpy(sM, zM, n);
            memcpy(sR, zR, n);
            orc_shake_stream(K, T, D, R, kM, kR, hM, hR, pM, pR, sM, sR, k, seed, chain, (uint64_t)it, (uint64_t)g, NULL);
            int64_t F_shaken = orc_objective(K, T, D, R, kM, kR, hM, hR, pM, pR, sM, sR, NULL);
            int64_t F_local = orc_vnd(K, T, D, R, kM, kR, hM, hR, pM, pR, sM, sR, nb_list, n_nb, evals);
            if (best_g < 0 || F_local < best_local) {
                best_g = g;
                best_local = F_local;
                best_shaken = F_shaken;
                memcpy(bM, sM, n);
                memcpy(bR, sR, n);
            }
        }
        int accepted = literal ? 1 : best_local < F;
        if (accepted) {
            memcpy(zM, bM, n);
            memcpy(zR, bR, n);
            F = best_local;
        }
        if (!literal) *k_state = accepted ? 1 : ((k >= k_max) ? 1 : k + 1);
        if (F < *F_best) *F_best = F;
        if (rec) {
            rec[i].iter = (int32_t)it;
            rec[i].k = k;
            rec[i].accepted = accepted;
            rec[i].winner = best_g;
            rec[i].F_shaken = best_shaken;
            rec[i].F_local = best_local;
            rec[i].F_best = *F_best;
        }
    }
    free(sM); free(sR); free(bM); free(bR);
    return F;
}
