// Host runtime of the lot-sizing VNS: the C ABI declared in include/vns.h.
//
// A context owns, for its whole life, every array of the search in device memory (instance rows, product
// parameters, current and working solutions of every chain, costs, records); calls move only their
// arguments and results across PCIe.  All work is queued on one stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "vns.h"
#include "vns_launch.hpp"
#include "vns_mlp.hpp"
#include "vns_types.hpp"

using namespace vns;

static_assert(sizeof(Record) == sizeof(vns_record), "record layout");
static_assert(sizeof(Bits) == 32, "bits layout");
static_assert(VNS_MLP_PARAMS == mlp::kParams, "scorer parameter count");

static void mlp_he_uniform(uint64_t seed, std::vector<float> &p);

// Scratch of the allocation-free pricing call (vns_eval_neighbourhood_noalloc): the evaluation counters,
// the per-product argmin keys, the pricing workgroup table and the slot-price staging.  One copy per GPU,
// held until the process ends, shared by every call on that GPU (calls that overlap on one GPU race).  Host
// code never passes the array's name to a kernel or a copy: it uses the device address that
// hipGetSymbolAddress returned for that GPU at context creation.
constexpr size_t kScratchBytes = 8u << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_create_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` on each GPU (null until resolved)

// Resolves the device address of `scratch` on `device` (which must be current) once per device.
hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

void *scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

// vns_test_inject_failure: countdowns to a simulated allocation failure / HIP failure (0 = off)
thread_local int32_t g_inject_alloc = 0;
thread_local int32_t g_inject_device = 0;

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
};

}  // namespace

struct vns_ctx {
    // instance data (host)
    int32_t n_inst = 0;
    std::vector<int32_t> K, T, prod0;
    std::vector<int32_t> prod_row;        // row offset of every product (as in the device product table)
    std::vector<ProdParams> prod_host;    // the device product table
    std::vector<int64_t> cost_bound;      // each product's worst-case cost without unit costs (< 2^47)
    int64_t n_prod = 0;
    uint64_t seed = 0;
    int device = 0;

    // options
    int64_t chains_per_inst = 1;
    int32_t kmax = 5;
    uint32_t nb_list = 0x421;
    int32_t n_nb = 3;
    int32_t trace = 1;
    int32_t run_waves = 8;
    int32_t eval_group = 4;
    int32_t eval_spread = 0;              // pricing: wavefronts per workgroup of the range form (0 = off)
    int32_t n_cu = 256;                   // compute units of the device (queried at create)
    int64_t run_lds_budget = 64 * 1024;   // bytes of LDS the search kernel may use for an instance's rows
    int32_t use_graph = 0;
    int64_t max_lds_per_wg = 65536;       // device limit on LDS per workgroup (queried at create)
    int64_t coop_wait_ticks = 0;          // steady-clock ticks of kCoopWaitSeconds (clock rate queried at create)
    int32_t permille = 0;                 // learned scorer: top permille priced exactly (0 = plain search)
    int32_t learned_pack = 0;             // learned VND: products per wavefront batch (0, 1 = one at a time)
    int32_t speculate = 0;                // plain search: speculative VND (neighbourhoods priced side by side)
    int32_t state_lds = 1;                // search kernel: chains' solution state in LDS when it fits
    int32_t vnd_memo = 0;                 // VND: skip neighbourhoods priced without improvement on this pattern
    int32_t spec_iters = 1;               // iterations speculated side by side per chain (1 = off)
    int32_t best_of = 0;                  // best-of-G search: streams per iteration (0, 1 = the plain chain)
    int32_t best_literal = 0;             //   as printed (k fixed, the minimum always kept)
    int32_t eval_inc = 0;                 // pricing sweeps decode each move only until it rejoins the base
    int32_t model = 0;                    // decode reading: kModelStrict | kModelDispose (VNS_OPT_DECODE)
    CoopCtl *d_coop_ctl = nullptr;        // speculative iterations: per-chain control, per-slot summaries and
    CoopSlot *d_coop_slot = nullptr;      //   VND results
    Bits *d_coop_res = nullptr;
    int64_t *d_coop_res_cost = nullptr;
    size_t coop_cap_ctl = 0, coop_cap_slot = 0, coop_cap_res = 0;
    int32_t spec_waves = 16;
    int64_t log_cap = 0;                  // move-log capacity in records (0 = no log)

    // chains (host mirror)
    std::vector<ChainInfo> chains;
    std::vector<int64_t> price_off;
    int64_t total_cp = 0;
    int64_t total_slots = 0;

    // device arrays
    int2 *d_rows = nullptr;
    ProdParams *d_prod = nullptr;
    ChainInfo *d_chains = nullptr;
    int32_t *d_cp_chain = nullptr;
    int64_t *d_price_off = nullptr;
    Bits *d_cur = nullptr, *d_work = nullptr;
    Bits *d_bestx = nullptr;              // each chain's best solution so far
    int64_t *d_cur_cost = nullptr, *d_work_cost = nullptr;
    ChainState *d_cs = nullptr;
    uint64_t *d_prod_key = nullptr;
    int64_t *d_prod_price = nullptr;
    int32_t *d_prod_slot = nullptr;
    int64_t *d_best = nullptr;
    int32_t *d_best_slot = nullptr;
    unsigned long long *d_evals = nullptr;
    int64_t *d_slot_price = nullptr;
    size_t slot_price_cap = 0;
    Record *d_trace = nullptr;
    size_t trace_cap = 0;
    int32_t trace_iters = 0;
    int64_t *d_iter = nullptr;            // device iteration counter (first iteration of the next run)
    float *d_mlp = nullptr;               // scorer parameters, Adam moments
    float *d_adam_m = nullptr, *d_adam_v = nullptr;
    int64_t adam_step = 0;
    float *d_log_x = nullptr, *d_log_y = nullptr;   // move log
    unsigned long long *d_log_n = nullptr;
    hipGraph_t graph = nullptr;           // captured search launch (VNS_OPT_GRAPH)
    hipGraphExec_t graph_exec = nullptr;
    int64_t graph_key[5] = {-1, -1, -1, -1, -1};  // (iters, chains, waves, LDS bytes, trace buffer)
    EvalWg *d_eval_wg = nullptr;          // k_eval workgroup table of the last chain range priced
    int64_t eval_wg_n = 0;
    int64_t eval_wg_key[4] = {-1, -1, -1, -1};  // (first chain, number of chains, group size, form: 1
                                                 // incremental, 2 + spread otherwise) of that table
                                                 // (incremental pricing takes one product per entry)

    char *ws = nullptr;                   // caller-owned workspace (vns_bind_workspace), its size and flags
    size_t ws_bytes = 0;
    uint32_t ws_flags = 0;

    hipStream_t own_stream = nullptr, stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;

    // progress and stats
    int64_t iteration = 0;
    vns_stats stats{};

    std::string err;
    bool dead = false;
};

// ---------------------------------------------------------------------------------------------------
// error helpers
// ---------------------------------------------------------------------------------------------------
static vns_status fail(vns_ctx *c, vns_status s, const std::string &msg) {
    if (c) {
        c->err = msg;
        if (s == VNS_EDEVICE) c->dead = true;
    } else {
        g_create_error = msg;
    }
    return s;
}

static vns_status hip_fail(vns_ctx *c, hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return fail(c, VNS_ENOMEM, m);
    return fail(c, VNS_EDEVICE, m);
}

#define VNS_HIP(ctx, expr)                                          \
    do {                                                            \
        hipError_t e_ = (expr);                                     \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);    \
    } while (0)

#define VNS_LIVE(ctx)                                                                          \
    do {                                                                                       \
        if (!(ctx)) return fail(nullptr, VNS_EINVAL, "null context");                          \
        if ((ctx)->dead) return fail((ctx), VNS_ESTATE, "context is dead after a device error"); \
        if (g_inject_device > 0 && --g_inject_device == 0)                                     \
            return hip_fail((ctx), hipErrorLaunchFailure, "injected failure (vns_test_inject_failure)"); \
        VNS_HIP((ctx), hipSetDevice((ctx)->device));                                          \
    } while (0)

template <class T>
static hipError_t dmalloc(T **p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    if (g_inject_alloc > 0 && --g_inject_alloc == 0) return hipErrorOutOfMemory;
    return hipMalloc((void **)p, n * sizeof(T));
}

template <class T>
static void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

static void drop_graph(vns_ctx *c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    for (int i = 0; i < 5; ++i) c->graph_key[i] = -1;
}

static void free_chains(vns_ctx *c) {
    drop_graph(c);
    dfree(c->d_iter);
    dfree(c->d_chains);
    dfree(c->d_cp_chain);
    dfree(c->d_price_off);
    dfree(c->d_cur);
    dfree(c->d_work);
    dfree(c->d_bestx);
    dfree(c->d_cur_cost);
    dfree(c->d_work_cost);
    dfree(c->d_cs);
    dfree(c->d_prod_key);
    dfree(c->d_prod_price);
    dfree(c->d_prod_slot);
    dfree(c->d_best);
    dfree(c->d_best_slot);
    dfree(c->d_slot_price);
    c->slot_price_cap = 0;
    dfree(c->d_trace);
    c->trace_cap = 0;
    c->trace_iters = 0;
    dfree(c->d_eval_wg);
    c->eval_wg_n = 0;
    c->eval_wg_key[0] = c->eval_wg_key[1] = c->eval_wg_key[2] = c->eval_wg_key[3] = -1;
}

static void free_log(vns_ctx *c) {
    dfree(c->d_log_x);
    dfree(c->d_log_y);
    dfree(c->d_log_n);
}

static void free_all(vns_ctx *c) {
    free_chains(c);
    free_log(c);
    dfree(c->d_mlp);
    dfree(c->d_adam_m);
    dfree(c->d_adam_v);
    dfree(c->d_rows);
    dfree(c->d_prod);
    dfree(c->d_evals);
    dfree(c->d_coop_ctl);
    dfree(c->d_coop_slot);
    dfree(c->d_coop_res);
    dfree(c->d_coop_res_cost);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    c->ev0 = c->ev1 = nullptr;
    c->own_stream = c->stream = nullptr;
}

// Initial solution of every chain: manufacture in every period (always feasible).
static Bits initial_bits(int T) {
    Bits b{};
    for (int t = 0; t < T; ++t) b.m[t >> 5] |= 1u << (t & 31);
    return b;
}

// (Re)build the chain arrays for chains_per_inst chains per instance and reset every chain.
static vns_status setup_chains(vns_ctx *c) {
    free_chains(c);
    const int64_t G = (int64_t)c->n_inst * c->chains_per_inst;
    if (G > (int64_t)INT32_MAX) return fail(c, VNS_EINVAL, "too many chains");
    c->chains.assign((size_t)G, ChainInfo{});
    c->price_off.assign((size_t)G, 0);
    int64_t cp = 0, slots = 0;
    for (int32_t i = 0; i < c->n_inst; ++i) {
        for (int64_t j = 0; j < c->chains_per_inst; ++j) {
            const int64_t g = (int64_t)i * c->chains_per_inst + j;
            ChainInfo &ci = c->chains[(size_t)g];
            ci.inst = i;
            ci.K = c->K[(size_t)i];
            ci.T = c->T[(size_t)i];
            ci.prod0 = c->prod0[(size_t)i];
            ci.cp0 = cp;
            c->price_off[(size_t)g] = slots;
            cp += ci.K;
            slots += 4LL * ci.K * ci.T;
        }
    }
    c->total_cp = cp;
    c->total_slots = slots;
    std::vector<int32_t> cp_chain((size_t)cp);
    std::vector<Bits> bits((size_t)cp);
    for (int64_t g = 0; g < G; ++g) {
        const ChainInfo &ci = c->chains[(size_t)g];
        const Bits b0 = initial_bits(ci.T);
        for (int32_t p = 0; p < ci.K; ++p) {
            cp_chain[(size_t)(ci.cp0 + p)] = (int32_t)g;
            bits[(size_t)(ci.cp0 + p)] = b0;
        }
    }
    VNS_HIP(c, dmalloc(&c->d_chains, (size_t)G));
    VNS_HIP(c, dmalloc(&c->d_cp_chain, (size_t)cp));
    VNS_HIP(c, dmalloc(&c->d_price_off, (size_t)G));
    VNS_HIP(c, dmalloc(&c->d_cur, (size_t)cp));
    VNS_HIP(c, dmalloc(&c->d_work, (size_t)cp));
    VNS_HIP(c, dmalloc(&c->d_bestx, (size_t)cp));
    VNS_HIP(c, dmalloc(&c->d_cur_cost, (size_t)cp));
    VNS_HIP(c, dmalloc(&c->d_work_cost, (size_t)cp));
    VNS_HIP(c, dmalloc(&c->d_cs, (size_t)G));
    VNS_HIP(c, dmalloc(&c->d_prod_key, (size_t)cp));
    VNS_HIP(c, dmalloc(&c->d_prod_price, (size_t)cp));
    VNS_HIP(c, dmalloc(&c->d_prod_slot, (size_t)cp));
    VNS_HIP(c, dmalloc(&c->d_best, (size_t)G));
    VNS_HIP(c, dmalloc(&c->d_best_slot, (size_t)G));
    VNS_HIP(c, dmalloc(&c->d_iter, 1));
    const int64_t zero = 0;
    VNS_HIP(c, hipMemcpyAsync(c->d_iter, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
    VNS_HIP(c, hipMemcpyAsync(c->d_chains, c->chains.data(), sizeof(ChainInfo) * (size_t)G, hipMemcpyHostToDevice, c->stream));
    VNS_HIP(c, hipMemcpyAsync(c->d_cp_chain, cp_chain.data(), sizeof(int32_t) * (size_t)cp, hipMemcpyHostToDevice, c->stream));
    VNS_HIP(c, hipMemcpyAsync(c->d_price_off, c->price_off.data(), sizeof(int64_t) * (size_t)G, hipMemcpyHostToDevice, c->stream));
    VNS_HIP(c, hipMemcpyAsync(c->d_cur, bits.data(), sizeof(Bits) * (size_t)cp, hipMemcpyHostToDevice, c->stream));
    InitArgs ia{c->d_chains, c->d_prod, c->d_rows, c->d_cur, c->d_cur_cost, c->d_work, c->d_work_cost, c->d_cs,
                c->d_bestx, 0};
    VNS_HIP(c, launch_init(ia, (int)G, c->stream, c->model));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    c->iteration = 0;
    c->stats = vns_stats{};
    return VNS_OK;
}

static vns_status check_chain(vns_ctx *c, int32_t chain) {
    if (chain < 0 || (size_t)chain >= c->chains.size()) return fail(c, VNS_EINVAL, "chain index out of range");
    return VNS_OK;
}

// ---------------------------------------------------------------------------------------------------
// creation
// ---------------------------------------------------------------------------------------------------
extern "C" vns_status vns_create_batch(int32_t n_inst, const int32_t *K, const int32_t *T, const int32_t *D,
                                       const int32_t *R, const int32_t *kM, const int32_t *kR, const int32_t *hM,
                                       const int32_t *hR, uint64_t seed, vns_ctx **out) {
    if (!out) return fail(nullptr, VNS_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_inst < 1) return fail(nullptr, VNS_EINVAL, "n_inst must be >= 1");
    if (!K || !T || !D || !R || !kM || !kR || !hM || !hR) return fail(nullptr, VNS_EINVAL, "NULL input array");
    int64_t n_prod = 0, n_rows = 0;
    for (int32_t i = 0; i < n_inst; ++i) {
        if (K[i] < 1 || K[i] > VNS_K_MAX) return fail(nullptr, VNS_EINVAL, "K out of range");
        if (T[i] < 1 || T[i] > VNS_T_MAX) return fail(nullptr, VNS_EINVAL, "T out of range");
        n_prod += K[i];
        n_rows += (int64_t)K[i] * T[i];
    }
    if (n_prod > (int64_t)INT32_MAX / 2) return fail(nullptr, VNS_EINVAL, "too many products");
    if (n_rows * 4 > (int64_t)INT32_MAX) return fail(nullptr, VNS_EINVAL, "too many periods in total");

    std::vector<int2> rows((size_t)n_rows);
    std::vector<ProdParams> prod((size_t)n_prod);
    std::vector<int64_t> bounds((size_t)n_prod);   // worst-case cost of each product without unit costs
    std::vector<int32_t> prod0((size_t)n_inst);
    int64_t p = 0, r = 0;
    for (int32_t i = 0; i < n_inst; ++i) {
        prod0[(size_t)i] = (int32_t)p;
        __int128 F_bound = 0;
        for (int32_t k = 0; k < K[i]; ++k, ++p) {
            const int Ti = T[i];
            if (kM[p] < 0 || kR[p] < 0 || hM[p] < 0 || hR[p] < 0)
                return fail(nullptr, VNS_EINVAL, "negative cost");
            int64_t sumD = 0, sumR = 0, maxD = 0, S_tD = 0, S_PR = 0;
            for (int t = 0; t < Ti; ++t) {
                const int64_t d = D[r + t], q = R[r + t];
                if (d < 0 || q < 0) return fail(nullptr, VNS_EINVAL, "negative demand or returns");
                if (d >= (1 << 24) || q >= (1 << 24)) return fail(nullptr, VNS_ERANGE, "demand or returns >= 2^24");
                sumD += d;
                sumR += q;
                maxD = std::max(maxD, d);
                S_tD += (int64_t)t * d;
                S_PR += sumR;
                rows[(size_t)(r + t)] = make_int2((int)d, (int)sumR);
            }
            // int32 accumulators of the forward decode: A2 <= sum D * (T-1), A1 <= sum R * (T-1),
            // XR + D <= sum R + max D.
            if (sumD * Ti >= (1LL << 31) || sumR * Ti >= (1LL << 31) || sumR + maxD >= (1LL << 31))
                return fail(nullptr, VNS_ERANGE, "a product's demand or returns over the horizon are too large");
            const __int128 bound = (__int128)Ti * ((__int128)kM[p] + kR[p]) + (__int128)hM[p] * sumD * Ti +
                                   (__int128)hR[p] * sumR * Ti;
            if (bound >= ((__int128)1 << 47)) return fail(nullptr, VNS_ERANGE, "a product's cost could reach 2^47");
            F_bound += bound;
            ProdParams &pp = prod[(size_t)p];
            pp.kM = kM[p];
            pp.kR = kR[p];
            pp.hM = hM[p];
            pp.hR = hR[p];
            pp.S_tD = S_tD;
            pp.S_PR = S_PR;
            pp.T = Ti;
            pp.row = (int32_t)r;
            pp.pM = pp.pR = 0;
            pp.SD = sumD;
            set_cost_terms(pp);
            bounds[(size_t)p] = (int64_t)bound;
            r += Ti;
        }
        if (F_bound >= ((__int128)1 << 62)) return fail(nullptr, VNS_ERANGE, "an instance's objective could reach 2^62");
    }

    vns_ctx *c = new (std::nothrow) vns_ctx();
    if (!c) return fail(nullptr, VNS_ENOMEM, "host allocation failed");
    c->n_inst = n_inst;
    c->K.assign(K, K + n_inst);
    c->T.assign(T, T + n_inst);
    c->prod0 = prod0;
    c->n_prod = n_prod;
    c->prod_row.resize((size_t)n_prod);
    for (int64_t q = 0; q < n_prod; ++q) c->prod_row[(size_t)q] = prod[(size_t)q].row;
    c->prod_host = prod;
    c->cost_bound = bounds;
    c->seed = seed;
    vns_status st = VNS_OK;
    auto bail = [&](vns_status s) {
        g_create_error = c->err;
        free_all(c);
        delete c;
        return s;
    };
#define VNS_CREATE_HIP(expr)                                     \
    do {                                                         \
        hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) return bail(hip_fail(c, e_, #expr)); \
    } while (0)
    VNS_CREATE_HIP(hipGetDevice(&c->device));
    VNS_CREATE_HIP(scratch_setup(c->device));   // the allocation-free pricing call's scratch on this GPU
    {
        int v = 0;
        VNS_CREATE_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
        c->max_lds_per_wg = v;
        VNS_CREATE_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, c->device));
        c->n_cu = std::max(v, 1);
        VNS_CREATE_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, c->device));   // kHz
        c->coop_wait_ticks = (int64_t)((double)(v > 0 ? v : 100000) * 1000.0 * kCoopWaitSeconds);
    }
    VNS_CREATE_HIP(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
    c->stream = c->own_stream;
    VNS_CREATE_HIP(hipEventCreate(&c->ev0));
    VNS_CREATE_HIP(hipEventCreate(&c->ev1));
    VNS_CREATE_HIP(dmalloc(&c->d_rows, (size_t)n_rows));
    VNS_CREATE_HIP(dmalloc(&c->d_prod, (size_t)n_prod));
    VNS_CREATE_HIP(dmalloc(&c->d_evals, (size_t)counter_words()));
    VNS_CREATE_HIP(dmalloc(&c->d_mlp, (size_t)mlp::kParams));
    VNS_CREATE_HIP(dmalloc(&c->d_adam_m, (size_t)mlp::kParams));
    VNS_CREATE_HIP(dmalloc(&c->d_adam_v, (size_t)mlp::kParams));
    std::vector<float> init_params;
    mlp_he_uniform(seed, init_params);
    VNS_CREATE_HIP(hipMemcpyAsync(c->d_mlp, init_params.data(), sizeof(float) * mlp::kParams, hipMemcpyHostToDevice,
                                  c->stream));
    VNS_CREATE_HIP(hipMemsetAsync(c->d_adam_m, 0, sizeof(float) * mlp::kParams, c->stream));
    VNS_CREATE_HIP(hipMemsetAsync(c->d_adam_v, 0, sizeof(float) * mlp::kParams, c->stream));
    VNS_CREATE_HIP(hipMemcpyAsync(c->d_rows, rows.data(), sizeof(int2) * (size_t)n_rows, hipMemcpyHostToDevice, c->stream));
    VNS_CREATE_HIP(hipMemcpyAsync(c->d_prod, prod.data(), sizeof(ProdParams) * (size_t)n_prod, hipMemcpyHostToDevice, c->stream));
#undef VNS_CREATE_HIP
    st = setup_chains(c);
    if (st != VNS_OK) return bail(st);
    *out = c;
    return VNS_OK;
}

extern "C" vns_status vns_create(int32_t K, int32_t T, const int32_t *D, const int32_t *R, const int32_t *kM,
                                 const int32_t *kR, const int32_t *hM, const int32_t *hR, uint64_t seed, vns_ctx **out) {
    return vns_create_batch(1, &K, &T, D, R, kM, kR, hM, hR, seed, out);
}

extern "C" void vns_destroy(vns_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (!c->dead && c->stream) (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

// ---------------------------------------------------------------------------------------------------
// options
// ---------------------------------------------------------------------------------------------------
extern "C" vns_status vns_set_option(vns_ctx *c, int32_t key, int64_t v) {
    VNS_LIVE(c);
    drop_graph(c);   // a captured launch holds the previous options in its arguments
    switch (key) {
        case VNS_OPT_CHAINS:
            if (v < 1 || v > 65536) return fail(c, VNS_EINVAL, "chains out of range");
            c->chains_per_inst = v;
            return setup_chains(c);
        case VNS_OPT_KMAX:
            if (v < 1 || v > VNS_KSHAKE_MAX) return fail(c, VNS_EINVAL, "k_max out of range");
            c->kmax = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_NB_LIST: {
            int n = 0;
            uint64_t x = (uint64_t)v;
            if (v <= 0 || x > 0xFFFFu) return fail(c, VNS_EINVAL, "neighbourhood list out of range");
            while (x) {
                const uint64_t nb = x & 0xF;
                if (nb != VNS_NB_FLIP_M && nb != VNS_NB_FLIP_R && nb != VNS_NB_SHIFT)
                    return fail(c, VNS_EINVAL, "unknown neighbourhood id in list");
                ++n;
                x >>= 4;
            }
            c->nb_list = (uint32_t)v;
            c->n_nb = n;
            return VNS_OK;
        }
        case VNS_OPT_TRACE:
            if (v != 0 && v != 1) return fail(c, VNS_EINVAL, "trace must be 0 or 1");
            c->trace = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_RUN_WAVES:
            if (v < 1 || v > 8) return fail(c, VNS_EINVAL, "run waves out of range");
            c->run_waves = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_EVAL_GROUP:
            if (v < 1 || v > kEvalGroup) return fail(c, VNS_EINVAL, "eval group out of range");
            c->eval_group = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_EVAL_SPREAD:
            if (v != 0 && v != 4 && v != 8 && v != 12 && v != 16)
                return fail(c, VNS_EINVAL, "eval spread must be 0, 4, 8, 12 or 16");
            c->eval_spread = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_RUN_LDS:
            if (v < 0 || v > kRunLdsMax) return fail(c, VNS_EINVAL, "search kernel LDS budget out of range");
            c->run_lds_budget = v;
            return VNS_OK;
        case VNS_OPT_GRAPH:
            if (v != 0 && v != 1) return fail(c, VNS_EINVAL, "graph must be 0 or 1");
            c->use_graph = (int32_t)v;
            if (!v) drop_graph(c);
            return VNS_OK;
        case VNS_OPT_SPECULATE:
            if (v != 0 && v != 1) return fail(c, VNS_EINVAL, "speculate must be 0 or 1");
            c->speculate = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_SPEC_WAVES:
            if (v < 1 || v > kMaxWaves) return fail(c, VNS_EINVAL, "speculative waves out of range");
            c->spec_waves = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_STATE_LDS:
            if (v != 0 && v != 1) return fail(c, VNS_EINVAL, "state_lds must be 0 or 1");
            c->state_lds = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_VND_MEMO:
            if (v != 0 && v != 1) return fail(c, VNS_EINVAL, "vnd_memo must be 0 or 1");
            c->vnd_memo = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_SPEC_ITERS:
            if (v < 1 || v > 16) return fail(c, VNS_EINVAL, "spec_iters must be in 1..16");
            c->spec_iters = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_BEST_OF:
            if (v < 0 || v > 16) return fail(c, VNS_EINVAL, "best_of must be in 0..16");
            c->best_of = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_BEST_OF_LITERAL:
            if (v != 0 && v != 1) return fail(c, VNS_EINVAL, "best_of_literal must be 0 or 1");
            c->best_literal = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_EVAL_INCREMENTAL:
            if (v != 0 && v != 1) return fail(c, VNS_EINVAL, "eval_incremental must be 0 or 1");
            c->eval_inc = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_DECODE:
            if (v < 0 || v >= kModels) return fail(c, VNS_EINVAL, "decode reading must be in 0..3");
            c->model = (int32_t)v;
            return setup_chains(c);   // every chain restarts from the initial solution under the new costs
        case VNS_OPT_LEARNED:
            if (v < 0 || v > 1000) return fail(c, VNS_EINVAL, "learned permille must be in 0..1000");
            c->permille = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_LEARNED_PACK:
            if (v < 0 || v > kPackMax) return fail(c, VNS_EINVAL, "learned pack must be in 0..8");
            c->learned_pack = (int32_t)v;
            return VNS_OK;
        case VNS_OPT_LOG: {
            if (v < 0 || v > ((int64_t)1 << 31)) return fail(c, VNS_EINVAL, "move-log capacity out of range");
            free_log(c);
            c->log_cap = 0;
            if (v > 0) {
                VNS_HIP(c, dmalloc(&c->d_log_x, (size_t)v * mlp::kF));
                VNS_HIP(c, dmalloc(&c->d_log_y, (size_t)v));
                VNS_HIP(c, dmalloc(&c->d_log_n, 1));
                VNS_HIP(c, hipMemsetAsync(c->d_log_n, 0, sizeof(unsigned long long), c->stream));
                VNS_HIP(c, hipStreamSynchronize(c->stream));
            }
            c->log_cap = v;
            return VNS_OK;
        }
        default:
            return fail(c, VNS_EINVAL, "unknown option");
    }
}

extern "C" vns_status vns_get_option(const vns_ctx *c, int32_t key, int64_t *v) {
    if (!c || !v) return fail(nullptr, VNS_EINVAL, "null argument");
    switch (key) {
        case VNS_OPT_CHAINS: *v = c->chains_per_inst; return VNS_OK;
        case VNS_OPT_KMAX: *v = c->kmax; return VNS_OK;
        case VNS_OPT_NB_LIST: *v = c->nb_list; return VNS_OK;
        case VNS_OPT_TRACE: *v = c->trace; return VNS_OK;
        case VNS_OPT_RUN_WAVES: *v = c->run_waves; return VNS_OK;
        case VNS_OPT_EVAL_GROUP: *v = c->eval_group; return VNS_OK;
        case VNS_OPT_EVAL_SPREAD: *v = c->eval_spread; return VNS_OK;
        case VNS_OPT_RUN_LDS: *v = c->run_lds_budget; return VNS_OK;
        case VNS_OPT_GRAPH: *v = c->use_graph; return VNS_OK;
        case VNS_OPT_LEARNED: *v = c->permille; return VNS_OK;
        case VNS_OPT_LEARNED_PACK: *v = c->learned_pack; return VNS_OK;
        case VNS_OPT_SPECULATE: *v = c->speculate; return VNS_OK;
        case VNS_OPT_SPEC_WAVES: *v = c->spec_waves; return VNS_OK;
        case VNS_OPT_STATE_LDS: *v = c->state_lds; return VNS_OK;
        case VNS_OPT_VND_MEMO: *v = c->vnd_memo; return VNS_OK;
        case VNS_OPT_SPEC_ITERS: *v = c->spec_iters; return VNS_OK;
        case VNS_OPT_BEST_OF: *v = c->best_of; return VNS_OK;
        case VNS_OPT_BEST_OF_LITERAL: *v = c->best_literal; return VNS_OK;
        case VNS_OPT_EVAL_INCREMENTAL: *v = c->eval_inc; return VNS_OK;
        case VNS_OPT_DECODE: *v = c->model; return VNS_OK;
        case VNS_OPT_LOG: *v = c->log_cap; return VNS_OK;
        default: return fail(const_cast<vns_ctx *>(c), VNS_EINVAL, "unknown option");
    }
}

extern "C" vns_status vns_bind_stream(vns_ctx *c, void *s) {
    VNS_LIVE(c);
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    c->stream = s ? (hipStream_t)s : c->own_stream;
    return VNS_OK;
}

// ---------------------------------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Layout of a workspace bound with `flags` under the current options: the pricing workgroup table at 0, then
// the slot-price staging, then vns_run's buffers (the only part whose size depends on options, so last).
struct WsLayout {
    size_t eval_off = 0, eval_bytes = 0;
    size_t price_off = 0, price_bytes = 0;
    size_t run_off = 0, ctl_bytes = 0, slot_bytes = 0, res_bytes = 0, res_cost_bytes = 0;
    size_t total = 0;
};

static int64_t max_products(const vns_ctx *c) {
    int64_t m = 0;
    for (int32_t i = 0; i < c->n_inst; ++i) m = std::max<int64_t>(m, c->K[(size_t)i]);
    return m;
}

// Slots per chain of vns_run's cooperative launch under the current options (0: no cooperative launch).
static int32_t coop_slots(const vns_ctx *c) {
    const bool best = c->best_of >= 2 || c->best_literal;
    if (best) return std::max<int32_t>(c->best_of, 1);
    return c->spec_iters > 1 ? c->spec_iters : 0;
}

static WsLayout ws_layout(const vns_ctx *c, uint32_t flags) {
    WsLayout L;
    size_t off = 0;
    if (flags & (VNS_WS_EVAL | VNS_WS_EVAL_PRICES)) {
        L.eval_off = off;
        L.eval_bytes = align256(sizeof(EvalWg) * (size_t)std::max<int64_t>(c->total_cp, 1));
        off += L.eval_bytes;
    }
    if (flags & VNS_WS_EVAL_PRICES) {
        L.price_off = off;
        L.price_bytes = align256(sizeof(int64_t) * (size_t)std::max<int64_t>(c->total_slots, 1));
        off += L.price_bytes;
    }
    if (flags & VNS_WS_RUN) {
        const size_t G = c->chains.size(), m = (size_t)coop_slots(c), n_res = G * m * (size_t)max_products(c);
        L.run_off = off;
        if (m > 0) {
            L.ctl_bytes = align256(sizeof(CoopCtl) * G);
            L.slot_bytes = align256(sizeof(CoopSlot) * G * m);
            L.res_bytes = align256(sizeof(Bits) * n_res);
            L.res_cost_bytes = align256(sizeof(int64_t) * n_res);
        }
        off += L.ctl_bytes + L.slot_bytes + L.res_bytes + L.res_cost_bytes;
    }
    L.total = off;
    return L;
}

extern "C" vns_status vns_workspace_bytes(const vns_ctx *c, uint32_t flags, size_t *bytes) {
    if (!c || !bytes) return fail(nullptr, VNS_EINVAL, "null argument");
    if (flags & ~(VNS_WS_RUN | VNS_WS_EVAL | VNS_WS_EVAL_PRICES))
        return fail(const_cast<vns_ctx *>(c), VNS_EINVAL, "unknown workspace flags");
    *bytes = ws_layout(c, flags).total;
    return VNS_OK;
}

extern "C" vns_status vns_bind_workspace(vns_ctx *c, void *p, size_t bytes, uint32_t flags) {
    VNS_LIVE(c);
    if (flags & ~(VNS_WS_RUN | VNS_WS_EVAL | VNS_WS_EVAL_PRICES)) return fail(c, VNS_EINVAL, "unknown workspace flags");
    VNS_HIP(c, hipStreamSynchronize(c->stream));   // no running call still uses the previous buffer
    drop_graph(c);
    c->eval_wg_key[0] = c->eval_wg_key[1] = c->eval_wg_key[2] = c->eval_wg_key[3] = -1;   // the cached table lives in one of them
    if (!p || flags == 0) {
        c->ws = nullptr;
        c->ws_bytes = 0;
        c->ws_flags = 0;
        return VNS_OK;
    }
    if (((uintptr_t)p & 255u) != 0) return fail(c, VNS_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < ws_layout(c, flags).total) return fail(c, VNS_EINVAL, "workspace smaller than vns_workspace_bytes");
    c->ws = (char *)p;
    c->ws_bytes = bytes;
    c->ws_flags = flags;
    return VNS_OK;
}

// The bound workspace's layout for its flags, or an error when the current options outgrew it.
static vns_status ws_check(vns_ctx *c, WsLayout *L) {
    *L = ws_layout(c, c->ws_flags);
    if (L->total > c->ws_bytes)
        return fail(c, VNS_EINVAL, "the bound workspace is smaller than this call needs under the current options: "
                                   "query vns_workspace_bytes and rebind");
    return VNS_OK;
}

// ---------------------------------------------------------------------------------------------------
// pricing
// ---------------------------------------------------------------------------------------------------
// Sums of the spread workgroup counters (waits for the stream).
static hipError_t read_counters(vns_ctx *c, unsigned long long (&ev)[3]) {
    std::vector<unsigned long long> h((size_t)counter_words());
    hipError_t e = hipMemcpyAsync(h.data(), c->d_evals, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    ev[0] = ev[1] = ev[2] = 0;
    for (int s = 0; s < kCounterSlots; ++s) {
        ev[0] += h[(size_t)s * kCounterStride];
        ev[1] += h[(size_t)s * kCounterStride + 1];
        ev[2] += h[(size_t)s * kCounterStride + 2];
    }
    return e;
}

extern "C" vns_status vns_eval_neighbourhood(vns_ctx *c, uint32_t nb_mask, int32_t chain, int64_t *slot_price,
                                             int64_t *prod_best, int32_t *prod_best_slot, int64_t *best,
                                             int32_t *best_slot) {
    VNS_LIVE(c);
    if (nb_mask == 0 || (nb_mask & ~7u)) return fail(c, VNS_EINVAL, "bad neighbourhood mask");
    if (c->eval_inc && c->model != 0)
        return fail(c, VNS_EINVAL, "incremental pricing takes only the default decode reading (VNS_OPT_DECODE = 0)");
    int32_t g0, ng;
    if (chain == VNS_ALL_CHAINS) {
        g0 = 0;
        ng = (int32_t)c->chains.size();
    } else {
        vns_status s = check_chain(c, chain);
        if (s != VNS_OK) return s;
        g0 = chain;
        ng = 1;
    }
    const ChainInfo &first = c->chains[(size_t)g0];
    const ChainInfo &last = c->chains[(size_t)(g0 + ng - 1)];
    const int64_t cp_begin = first.cp0, n_cp = last.cp0 + last.K - first.cp0;
    const int64_t slot_begin = c->price_off[(size_t)g0];
    const int64_t n_slots = c->price_off[(size_t)(g0 + ng - 1)] + 4LL * last.K * last.T - slot_begin;
    const bool ws_tab = c->ws && (c->ws_flags & (VNS_WS_EVAL | VNS_WS_EVAL_PRICES));
    const bool ws_price = c->ws && (c->ws_flags & VNS_WS_EVAL_PRICES);
    WsLayout wl;
    if (ws_tab) {
        vns_status s = ws_check(c, &wl);
        if (s != VNS_OK) return s;
    }
    int64_t *d_sp = ws_price ? reinterpret_cast<int64_t *>(c->ws + wl.price_off) : c->d_slot_price;
    if (slot_price && !ws_price && (size_t)n_slots > c->slot_price_cap) {
        dfree(c->d_slot_price);
        c->slot_price_cap = 0;
        VNS_HIP(c, dmalloc(&c->d_slot_price, (size_t)n_slots));
        c->slot_price_cap = (size_t)n_slots;
        d_sp = c->d_slot_price;
    }
    // workgroup table: for each run of up to eval_group consecutive chains of one instance, one workgroup
    // per product (incremental pricing: at most as many chains as the snapshots' LDS allows)
    int32_t maxT = 1;
    for (int32_t g = g0; g < g0 + ng; ++g) maxT = std::max<int32_t>(maxT, c->chains[(size_t)g].T);
    const int32_t group = c->eval_inc ? std::max<int32_t>(1, std::min<int32_t>(c->eval_group,
                                                                              kSnapLdsMax / ((maxT + 1) * kSnapBytes)))
                                      : c->eval_group;
    const int32_t spread = c->eval_inc ? 0 : c->eval_spread;
    const int64_t key[4] = {g0, ng, group, c->eval_inc ? 1 : 2 + spread};
    EvalWg *d_tab = ws_tab ? reinterpret_cast<EvalWg *>(c->ws + wl.eval_off) : c->d_eval_wg;
    if (!(key[0] == c->eval_wg_key[0] && key[1] == c->eval_wg_key[1] && key[2] == c->eval_wg_key[2] &&
          key[3] == c->eval_wg_key[3])) {
        std::vector<EvalWg> tab;
        int32_t g = g0;
        // range form: 24 wavefronts per compute unit (the pricing kernel's register bound), so n_cu * (24 / spread)
        // workgroups; each instance gets its share of them by pairs, split into near-equal ranges
        double per = 1.0;
        if (spread) {
            int64_t pairs = 0;
            for (int32_t h = g0; h < g0 + ng; ++h) pairs += c->chains[(size_t)h].K;
            per = std::max(1.0, (double)pairs / ((double)c->n_cu * std::max(1, 24 / spread)));
        }
        while (spread && g < g0 + ng) {
            const ChainInfo &ci = c->chains[(size_t)g];
            int32_t G = 1;
            while (g + G < g0 + ng && c->chains[(size_t)(g + G)].inst == ci.inst) ++G;
            // a range's moves (at most 4T per pair) fit the item table, its products' rows the row buffer
            const int64_t len_max = std::max<int64_t>(1, std::min<int64_t>(kEvalPairs, kEvalItems / (4 * ci.T)));
            const int32_t span_max = std::max<int32_t>(1, std::min<int32_t>(kEvalProds, kTMax / ci.T));
            const int64_t P = (int64_t)G * ci.K;
            const int64_t nr = std::max<int64_t>(1, std::llround((double)P / per));
            for (int64_t r = 0; r < nr; ++r) {
                const int64_t q_end = P * (r + 1) / nr;
                for (int64_t q = P * r / nr; q < q_end;) {
                    int64_t len = std::min<int64_t>(len_max, q_end - q);
                    const int32_t p0 = (int32_t)(q / G);
                    if ((q + len - 1) / G - p0 + 1 > span_max) len = (int64_t)(p0 + span_max) * G - q;
                    EvalWg w{};
                    w.cp = ci.cp0 + p0;
                    w.g0 = g;
                    w.n = (int32_t)len;
                    w.K = ci.K;
                    w.T = ci.T;
                    w.p = p0;
                    w.prod = ci.prod0 + p0;
                    w.row = c->prod_row[(size_t)(ci.prod0 + p0)];
                    w.np = (int32_t)((q + len - 1) / G - p0 + 1);
                    w.q0 = (int32_t)q;
                    w.G = G;
                    tab.push_back(w);
                    q += len;
                }
            }
            g += G;
        }
        while (!spread && g < g0 + ng) {
            const ChainInfo &ci = c->chains[(size_t)g];
            int32_t n = 1;
            while (n < group && g + n < g0 + ng && c->chains[(size_t)(g + n)].inst == ci.inst) ++n;
            // short horizons (T <= 32): several products per workgroup, so that a workgroup prices about 1024
            // moves (about 3T per pair) and its set-up is shared; their rows, pairs and moves must fit its LDS.
            // Longer horizons keep one product per workgroup: fewer, larger workgroups made the 100 x 52 sweep
            // (1300 workgroups) slower.
            int32_t np = 1;
            if (!c->eval_inc && ci.T <= kEvalShortT) {
                const int32_t want = (kEvalTargetMoves + 3 * n * ci.T - 1) / (3 * n * ci.T);
                np = std::max<int32_t>(1, std::min({want, kTMax / ci.T, kEvalPairs / n, kEvalProds,
                                                    kEvalItems / (4 * n * ci.T)}));
            }
            for (int32_t p = 0; p < ci.K; p += np) {
                EvalWg w{};
                w.cp = ci.cp0 + p;
                w.g0 = g;
                w.n = n;
                w.K = ci.K;
                w.T = ci.T;
                w.p = p;
                w.prod = ci.prod0 + p;
                w.row = c->prod_row[(size_t)(ci.prod0 + p)];
                w.np = std::min<int32_t>(np, ci.K - p);
                tab.push_back(w);
            }
            g += n;
        }
        c->eval_wg_n = 0;
        c->eval_wg_key[0] = c->eval_wg_key[1] = c->eval_wg_key[2] = c->eval_wg_key[3] = -1;
        if (!ws_tab) {
            dfree(c->d_eval_wg);
            VNS_HIP(c, dmalloc(&c->d_eval_wg, tab.size()));
            d_tab = c->d_eval_wg;
        }
        VNS_HIP(c, hipMemcpyAsync(d_tab, tab.data(), sizeof(EvalWg) * tab.size(), hipMemcpyHostToDevice, c->stream));
        c->eval_wg_n = (int64_t)tab.size();
        for (int i = 0; i < 4; ++i) c->eval_wg_key[i] = key[i];
    }
    EvalArgs ea{};
    ea.cp_chain = c->d_cp_chain;
    ea.chains = c->d_chains;
    ea.prod = c->d_prod;
    ea.rows = c->d_rows;
    ea.cur = c->d_cur;
    ea.cur_cost = c->d_cur_cost;
    ea.cstate = c->d_cs;
    ea.slot_price = slot_price ? d_sp - slot_begin : nullptr;
    ea.price_off = c->d_price_off;
    ea.prod_key = c->d_prod_key;
    ea.evals = c->d_evals;
    ea.nb_mask = nb_mask;
    VNS_HIP(c, hipMemsetAsync(c->d_evals, 0, sizeof(unsigned long long) * counter_words(), c->stream));
    VNS_HIP(c, hipEventRecord(c->ev0, c->stream));
    if (c->eval_inc)
        VNS_HIP(c, launch_eval_inc(ea, d_tab, c->eval_wg_n, (size_t)group * (size_t)(maxT + 1) * kSnapBytes,
                                   c->stream));
    else
        VNS_HIP(c, launch_eval(ea, d_tab, c->eval_wg_n, c->stream, c->model, spread ? spread : 4));
    VNS_HIP(c, hipEventRecord(c->ev1, c->stream));
    ChainBestArgs cb{c->d_chains, c->d_cs, c->d_cur_cost, c->d_prod_key, c->d_prod_price, c->d_prod_slot,
                     c->d_best, c->d_best_slot, g0};
    VNS_HIP(c, launch_chain_best(cb, ng, c->stream));
    if (slot_price)
        VNS_HIP(c, hipMemcpyAsync(slot_price, d_sp, sizeof(int64_t) * (size_t)n_slots, hipMemcpyDeviceToHost, c->stream));
    if (prod_best)
        VNS_HIP(c, hipMemcpyAsync(prod_best, c->d_prod_price + cp_begin, sizeof(int64_t) * (size_t)n_cp, hipMemcpyDeviceToHost, c->stream));
    if (prod_best_slot)
        VNS_HIP(c, hipMemcpyAsync(prod_best_slot, c->d_prod_slot + cp_begin, sizeof(int32_t) * (size_t)n_cp, hipMemcpyDeviceToHost, c->stream));
    if (best) VNS_HIP(c, hipMemcpyAsync(best, c->d_best, sizeof(int64_t) * (size_t)ng, hipMemcpyDeviceToHost, c->stream));
    if (best_slot)
        VNS_HIP(c, hipMemcpyAsync(best_slot, c->d_best_slot, sizeof(int32_t) * (size_t)ng, hipMemcpyDeviceToHost, c->stream));
    unsigned long long ev[3] = {0, 0, 0};
    VNS_HIP(c, read_counters(c, ev));
    float ms = 0.f;
    VNS_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->stats.last_eval_evals = (int64_t)ev[0];
    c->stats.last_eval_period_steps = (int64_t)ev[1];
    c->stats.last_eval_decoded_steps = (int64_t)ev[2];
    c->stats.last_eval_ms = ms;
    return VNS_OK;
}

// The same pricing with its scratch in the per-GPU static array: no device or host allocation.  The table
// of pricing workgroups is built on the device (one entry per (chain, product), empty for chains that do
// not lead a group), and every move is decoded in full.
extern "C" vns_status vns_eval_neighbourhood_noalloc(vns_ctx *c, uint32_t nb_mask, int32_t chain, int64_t *slot_price,
                                                     int64_t *prod_best, int32_t *prod_best_slot, int64_t *best,
                                                     int32_t *best_slot) {
    VNS_LIVE(c);
    if (nb_mask == 0 || (nb_mask & ~7u)) return fail(c, VNS_EINVAL, "bad neighbourhood mask");
    int32_t g0, ng;
    if (chain == VNS_ALL_CHAINS) {
        g0 = 0;
        ng = (int32_t)c->chains.size();
    } else {
        vns_status s = check_chain(c, chain);
        if (s != VNS_OK) return s;
        g0 = chain;
        ng = 1;
    }
    const ChainInfo &first = c->chains[(size_t)g0];
    const ChainInfo &last = c->chains[(size_t)(g0 + ng - 1)];
    const int64_t cp_begin = first.cp0, n_cp = last.cp0 + last.K - first.cp0;
    const int64_t slot_begin = c->price_off[(size_t)g0];
    const int64_t n_slots = c->price_off[(size_t)(g0 + ng - 1)] + 4LL * last.K * last.T - slot_begin;
    // scratch layout: counters, argmin keys, workgroup table, slot prices (each 256-byte aligned)
    const size_t ctr_bytes = align256(sizeof(unsigned long long) * (size_t)counter_words());
    const size_t key_bytes = align256(sizeof(uint64_t) * (size_t)n_cp);
    const size_t tab_bytes = align256(sizeof(EvalWg) * (size_t)n_cp);
    const size_t sp_bytes = slot_price ? align256(sizeof(int64_t) * (size_t)n_slots) : 0;
    if (ctr_bytes + key_bytes + tab_bytes + sp_bytes > kScratchBytes)
        return fail(c, VNS_EINVAL, "vns_eval_neighbourhood_noalloc: the chains priced need more than its 8 MiB static "
                                   "scratch (56 bytes per (chain, product), plus 8 per slot with slot prices); "
                                   "price fewer chains per call or use vns_eval_neighbourhood");
    unsigned char *base = static_cast<unsigned char *>(scratch_of(c->device));
    if (!base) return fail(c, VNS_EDEVICE, "the static scratch of this GPU has no device address");
    unsigned long long *ctr = reinterpret_cast<unsigned long long *>(base);
    uint64_t *keys = reinterpret_cast<uint64_t *>(base + ctr_bytes);
    EvalWg *tab = reinterpret_cast<EvalWg *>(base + ctr_bytes + key_bytes);
    int64_t *sp = reinterpret_cast<int64_t *>(base + ctr_bytes + key_bytes + tab_bytes);

    EvalPrepArgs pa{};
    pa.chains = c->d_chains;
    pa.prod = c->d_prod;
    pa.cp_chain = c->d_cp_chain;
    pa.cp_begin = cp_begin;
    pa.n_cp = n_cp;
    pa.g0 = g0;
    pa.ng = ng;
    pa.group = c->eval_group;
    pa.chains_per_inst = (int32_t)c->chains_per_inst;
    pa.table = tab;
    pa.counters = ctr;
    VNS_HIP(c, launch_eval_prep(pa, c->stream));
    EvalArgs ea{};
    ea.cp_chain = c->d_cp_chain;
    ea.chains = c->d_chains;
    ea.prod = c->d_prod;
    ea.rows = c->d_rows;
    ea.cur = c->d_cur;
    ea.cur_cost = c->d_cur_cost;
    ea.cstate = c->d_cs;
    ea.slot_price = slot_price ? sp - slot_begin : nullptr;   // indexed by absolute slot offset
    ea.price_off = c->d_price_off;
    ea.prod_key = keys - cp_begin;                           // indexed by absolute (chain, product)
    ea.evals = ctr;
    ea.nb_mask = nb_mask;
    VNS_HIP(c, hipEventRecord(c->ev0, c->stream));
    VNS_HIP(c, launch_eval(ea, tab, n_cp, c->stream, c->model));
    VNS_HIP(c, hipEventRecord(c->ev1, c->stream));
    ChainBestArgs cb{c->d_chains, c->d_cs, c->d_cur_cost, keys - cp_begin, c->d_prod_price, c->d_prod_slot, c->d_best,
                     c->d_best_slot, g0};
    VNS_HIP(c, launch_chain_best(cb, ng, c->stream));
    if (slot_price)
        VNS_HIP(c, hipMemcpyAsync(slot_price, sp, sizeof(int64_t) * (size_t)n_slots, hipMemcpyDeviceToHost, c->stream));
    if (prod_best)
        VNS_HIP(c, hipMemcpyAsync(prod_best, c->d_prod_price + cp_begin, sizeof(int64_t) * (size_t)n_cp, hipMemcpyDeviceToHost, c->stream));
    if (prod_best_slot)
        VNS_HIP(c, hipMemcpyAsync(prod_best_slot, c->d_prod_slot + cp_begin, sizeof(int32_t) * (size_t)n_cp, hipMemcpyDeviceToHost, c->stream));
    if (best) VNS_HIP(c, hipMemcpyAsync(best, c->d_best, sizeof(int64_t) * (size_t)ng, hipMemcpyDeviceToHost, c->stream));
    if (best_slot)
        VNS_HIP(c, hipMemcpyAsync(best_slot, c->d_best_slot, sizeof(int32_t) * (size_t)ng, hipMemcpyDeviceToHost, c->stream));
    unsigned long long h[counter_words()];
    VNS_HIP(c, hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    unsigned long long ev[3] = {0, 0, 0};
    for (int q = 0; q < kCounterSlots; ++q)
        for (int w = 0; w < 3; ++w) ev[w] += h[(size_t)q * kCounterStride + (size_t)w];
    float ms = 0.f;
    VNS_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->stats.last_eval_evals = (int64_t)ev[0];
    c->stats.last_eval_period_steps = (int64_t)ev[1];
    c->stats.last_eval_decoded_steps = (int64_t)ev[2];
    c->stats.last_eval_ms = ms;
    return VNS_OK;
}

// ---------------------------------------------------------------------------------------------------
// search
// ---------------------------------------------------------------------------------------------------
extern "C" vns_status vns_run(vns_ctx *c, int32_t iters) {
    VNS_LIVE(c);
    if (iters < 0) return fail(c, VNS_EINVAL, "iters must be >= 0");
    if (c->iteration + iters > (int64_t)INT32_MAX) return fail(c, VNS_ERANGE, "iteration counter would overflow");
    if (iters == 0) return VNS_OK;
    const int64_t G = (int64_t)c->chains.size();
    if (c->trace) {
        const size_t need = (size_t)G * (size_t)iters;
        if (need > c->trace_cap) {
            dfree(c->d_trace);
            c->trace_cap = 0;
            VNS_HIP(c, dmalloc(&c->d_trace, need));
            c->trace_cap = need;
        }
        c->trace_iters = iters;
    } else {
        c->trace_iters = 0;
    }
    RunArgs ra{};
    ra.chains = c->d_chains;
    ra.prod = c->d_prod;
    ra.rows = c->d_rows;
    ra.cur = c->d_cur;
    ra.cur_cost = c->d_cur_cost;
    ra.work = c->d_work;
    ra.work_cost = c->d_work_cost;
    ra.cstate = c->d_cs;
    ra.best = c->d_bestx;
    ra.trace = c->trace ? c->d_trace : nullptr;
    ra.it0 = c->d_iter;
    ra.seed = c->seed;
    ra.iters = iters;
    ra.kmax = c->kmax;
    ra.nb_list = c->nb_list;
    ra.n_nb = c->n_nb;
    ra.permille = c->permille;
    ra.learned_pack = c->permille > 0 ? c->learned_pack : 0;
    ra.mlp = c->d_mlp;
    ra.log_x = c->log_cap > 0 ? c->d_log_x : nullptr;
    ra.log_y = c->d_log_y;
    ra.log_n = c->d_log_n;
    ra.log_cap = c->log_cap;
    ra.memo = c->vnd_memo;
    int64_t max_rows = 0;
    for (int32_t i = 0; i < c->n_inst; ++i) max_rows = std::max<int64_t>(max_rows, (int64_t)c->K[(size_t)i] * c->T[(size_t)i]);
    // instance rows in LDS for every chain whose instance fits the budget; the others stage one row per wave
    // speculative VND for plain runs (one wavefront per neighbourhood of each product), else one wavefront
    // per product
    const bool spec = c->speculate && c->permille == 0 && c->spec_waves >= c->n_nb;
    const RunKind kind = c->permille > 0 ? (c->learned_pack > 1 ? RunKind::kLearnedPacked : RunKind::kLearned)
                         : spec          ? RunKind::kSpec
                                         : RunKind::kPlain;
    const int waves = spec ? c->spec_waves : c->run_waves;
    size_t static_lds = 0;
    if (c->model != 0 && kind != RunKind::kPlain)
        return fail(c, VNS_EINVAL, "the learned search and the speculative VND take only the default decode reading "
                                   "(VNS_OPT_DECODE = 0)");
    // the one-workgroup plain search has a variant for batches with a short horizon
    int32_t min_T = kTMax;
    for (int32_t i = 0; i < c->n_inst; ++i) min_T = std::min<int32_t>(min_T, c->T[(size_t)i]);
    const RunKind run_k = (kind == RunKind::kPlain && min_T <= kMultiMaxT) ? RunKind::kPlainShort : kind;
    VNS_HIP(c, run_kernel_lds(run_k, &static_lds, 0, c->model));
    const bool packed = c->permille > 0 && c->learned_pack > 1;
    const int64_t learned = c->permille <= 0 ? 0
                            : packed         ? (int64_t)pack_region_bytes(waves, c->learned_pack)
                                             : (int64_t)waves * kLearnedWaveBytes;
    const int64_t room = c->max_lds_per_wg - (int64_t)static_lds - learned;   // dynamic LDS left for rows
    const int64_t slices = (int64_t)waves * kTMax;                   // per-wave rows when the instance does not fit
    if (room < slices * (int64_t)sizeof(int2)) return fail(c, VNS_EINVAL, "not enough LDS for the search kernel");
    // the chains' solution state (80 bytes per product) when it fits beside the per-wave row slices
    int64_t max_K = 0;
    for (int32_t i = 0; i < c->n_inst; ++i) max_K = std::max<int64_t>(max_K, c->K[(size_t)i]);
    int64_t state_bytes = c->state_lds ? (int64_t)(2 * sizeof(Bits) + 2 * sizeof(int64_t)) * max_K : 0;
    if (room - state_bytes < slices * (int64_t)sizeof(int2)) state_bytes = 0;
    const int64_t budget = std::min<int64_t>(c->run_lds_budget, room - state_bytes) / (int64_t)sizeof(int2);
    // no LDS for rows when not even the smallest instance fits: the per-wave slices suffice, and the
    // workgroups stay small enough to share a compute unit
    int64_t min_rows = max_rows;
    for (int32_t i = 0; i < c->n_inst; ++i) min_rows = std::min<int64_t>(min_rows, (int64_t)c->K[(size_t)i] * c->T[(size_t)i]);
    ra.lds_rows = min_rows > budget ? 0 : (int32_t)std::min<int64_t>(max_rows, budget);
    const size_t rows_bytes = (size_t)run_rows_entries(ra.lds_rows, waves) * sizeof(int2);
    ra.state_off = state_bytes > 0 ? (int32_t)(rows_bytes + (size_t)learned) : -1;
    const size_t lds = rows_bytes + (size_t)learned + (size_t)state_bytes;
    VNS_HIP(c, run_kernel_lds(run_k, &static_lds, lds, c->model));
    // speculative iterations: plain search without the move log (a discarded iteration's moves must not be
    // logged), not captured, and every workgroup of the launch resident at once
    // best-of-G (Algorithm 2): the same cooperative launch with G workgroups per chain, one per random stream
    const bool best = c->best_of >= 2 || c->best_literal;
    const int m = best ? std::max<int>(c->best_of, 1) : c->spec_iters;
    bool coop = false;
    // x stays in device memory: no state region; the learned search keeps its per-wavefront tiles
    const size_t lds_coop = rows_bytes + (size_t)learned;
    if (best) {
        if (kind != RunKind::kPlain || c->use_graph || ra.log_x != nullptr || c->spec_iters > 1)
            return fail(c, VNS_EINVAL, "best-of-G runs the plain search alone: no learned scorer, speculative VND or "
                                       "iterations, move log or graph capture");
        VNS_HIP(c, coop_fits(waves, lds_coop, G * m, &coop, RunKind::kPlain, c->model));
        if (!coop)
            return fail(c, VNS_EINVAL, "best-of-G needs its G workgroups per chain resident at once: use fewer "
                                       "chains, wavefronts per workgroup or streams");
    } else if (m > 1 && kind != RunKind::kSpec && !c->use_graph && ra.log_x == nullptr) {
        VNS_HIP(c, coop_fits(waves, lds_coop, G * m, &coop, kind, c->model));
    }
    c->stats.last_run_spec_iters = coop && !best ? m : 1;
    CoopCtl *d_ctl = c->d_coop_ctl;
    CoopSlot *d_slot = c->d_coop_slot;
    Bits *d_res = c->d_coop_res;
    int64_t *d_res_cost = c->d_coop_res_cost;
    if (coop && c->ws && (c->ws_flags & VNS_WS_RUN)) {   // from the caller's workspace
        WsLayout wl;
        vns_status s = ws_check(c, &wl);
        if (s != VNS_OK) return s;
        char *base = c->ws + wl.run_off;
        d_ctl = reinterpret_cast<CoopCtl *>(base);
        d_slot = reinterpret_cast<CoopSlot *>(base + wl.ctl_bytes);
        d_res = reinterpret_cast<Bits *>(base + wl.ctl_bytes + wl.slot_bytes);
        d_res_cost = reinterpret_cast<int64_t *>(base + wl.ctl_bytes + wl.slot_bytes + wl.res_bytes);
    } else if (coop) {
        const size_t n_res = (size_t)G * (size_t)m * (size_t)max_K;
        if ((size_t)G > c->coop_cap_ctl) {
            dfree(c->d_coop_ctl);
            c->coop_cap_ctl = 0;
            VNS_HIP(c, dmalloc(&c->d_coop_ctl, (size_t)G));
            c->coop_cap_ctl = (size_t)G;
        }
        if ((size_t)(G * m) > c->coop_cap_slot) {
            dfree(c->d_coop_slot);
            c->coop_cap_slot = 0;
            VNS_HIP(c, dmalloc(&c->d_coop_slot, (size_t)(G * m)));
            c->coop_cap_slot = (size_t)(G * m);
        }
        if (n_res > c->coop_cap_res) {
            dfree(c->d_coop_res);
            dfree(c->d_coop_res_cost);
            c->coop_cap_res = 0;
            VNS_HIP(c, dmalloc(&c->d_coop_res, n_res));
            VNS_HIP(c, dmalloc(&c->d_coop_res_cost, n_res));
            c->coop_cap_res = n_res;
        }
        d_ctl = c->d_coop_ctl;
        d_slot = c->d_coop_slot;
        d_res = c->d_coop_res;
        d_res_cost = c->d_coop_res_cost;
    }
    if (coop) {
        VNS_HIP(c, hipMemsetAsync(d_ctl, 0, sizeof(CoopCtl) * (size_t)G, c->stream));
        // the slots' round stamps: one left by an earlier launch must not match a round of this one
        VNS_HIP(c, hipMemsetAsync(d_slot, 0, sizeof(CoopSlot) * (size_t)(G * m), c->stream));
        ra.state_off = -1;
        ra.coop_m = m;
        ra.coop_xcd = G % 8 == 0;
        ra.coop_kmax = (int32_t)max_K;
        ra.coop_ctl = d_ctl;
        ra.coop_slot = d_slot;
        ra.coop_res = d_res;
        ra.coop_res_cost = d_res_cost;
        ra.coop_wait_ticks = c->coop_wait_ticks;
        ra.best_of = best ? 1 : 0;
        ra.best_literal = c->best_literal;
        VNS_HIP(c, hipEventRecord(c->ev0, c->stream));
        VNS_HIP(c, launch_run_coop(ra, (int)G, waves, lds_coop, c->d_iter, c->stream, kind, c->model));
        VNS_HIP(c, hipEventRecord(c->ev1, c->stream));
    } else if (c->use_graph) {
        const int64_t key[5] = {iters, G, waves * 8 + (int64_t)run_k, (int64_t)lds, (int64_t)(intptr_t)ra.trace};
        bool same = true;
        for (int i = 0; i < 5; ++i) same = same && key[i] == c->graph_key[i];
        if (!same || !c->graph_exec) {
            drop_graph(c);
            VNS_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            hipError_t le = launch_run(ra, run_k, (int)G, waves, lds, c->d_iter, c->stream, c->model);
            hipGraph_t gr = nullptr;
            hipError_t ce = hipStreamEndCapture(c->stream, &gr);
            if (le != hipSuccess) {
                if (gr) (void)hipGraphDestroy(gr);
                return hip_fail(c, le, "launch_run (capture)");
            }
            VNS_HIP(c, ce);
            c->graph = gr;
            VNS_HIP(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
            for (int i = 0; i < 5; ++i) c->graph_key[i] = key[i];
        }
        VNS_HIP(c, hipEventRecord(c->ev0, c->stream));
        VNS_HIP(c, hipGraphLaunch(c->graph_exec, c->stream));
        VNS_HIP(c, hipEventRecord(c->ev1, c->stream));
    } else {
        VNS_HIP(c, hipEventRecord(c->ev0, c->stream));
        VNS_HIP(c, launch_run(ra, run_k, (int)G, waves, lds, c->d_iter, c->stream, c->model));
        VNS_HIP(c, hipEventRecord(c->ev1, c->stream));
    }
    std::vector<ChainState> cs((size_t)G);
    VNS_HIP(c, hipMemcpyAsync(cs.data(), c->d_cs, sizeof(ChainState) * (size_t)G, hipMemcpyDeviceToHost, c->stream));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    float ms = 0.f;
    VNS_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    int64_t ev = 0, steps = 0, nbe = 0, fbs = 0, thrown = 0;
    int32_t err = 0;
    for (size_t g = 0; g < cs.size(); ++g) {
        ev += cs[g].evals;
        thrown += cs[g].discarded;
        steps += cs[g].evals * c->chains[g].T;
        nbe += cs[g].nb_evals;
        fbs += cs[g].fallbacks;
        err |= cs[g].err;
    }
    c->stats.last_run_learned_evals = nbe;
    c->stats.last_run_fallbacks = fbs;
    c->stats.last_run_discarded_evals = thrown;
    if (err & 2) return fail(c, VNS_EDEVICE, "speculative iterations: a workgroup's wait for its chain ran out");
    if (err) return fail(c, VNS_EDEVICE, "a VND exceeded its pass guard (inconsistent costs)");
    c->iteration += iters;
    c->stats.iterations = c->iteration;
    c->stats.last_run_evals = ev;
    c->stats.last_run_period_steps = steps;
    c->stats.move_evals += ev;
    c->stats.last_run_ms = ms;
    return VNS_OK;
}

// ---------------------------------------------------------------------------------------------------
// state access
// ---------------------------------------------------------------------------------------------------
extern "C" vns_status vns_get_cost(vns_ctx *c, int32_t chain, int64_t *F, int64_t *F_best) {
    VNS_LIVE(c);
    vns_status s = check_chain(c, chain);
    if (s != VNS_OK) return s;
    ChainState cs;
    VNS_HIP(c, hipMemcpyAsync(&cs, c->d_cs + chain, sizeof(cs), hipMemcpyDeviceToHost, c->stream));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    if (F) *F = cs.F;
    if (F_best) *F_best = cs.F_best;
    return VNS_OK;
}

extern "C" vns_status vns_get_costs(vns_ctx *c, int64_t *F, int64_t *F_best) {
    VNS_LIVE(c);
    std::vector<ChainState> cs(c->chains.size());
    VNS_HIP(c, hipMemcpyAsync(cs.data(), c->d_cs, sizeof(ChainState) * cs.size(), hipMemcpyDeviceToHost, c->stream));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    for (size_t g = 0; g < cs.size(); ++g) {
        if (F) F[g] = cs[g].F;
        if (F_best) F_best[g] = cs[g].F_best;
    }
    return VNS_OK;
}

extern "C" vns_status vns_get_solution(vns_ctx *c, int32_t chain, int32_t which, uint8_t *zM, uint8_t *zR) {
    VNS_LIVE(c);
    vns_status s = check_chain(c, chain);
    if (s != VNS_OK) return s;
    if (which != VNS_SOLUTION_CURRENT && which != VNS_SOLUTION_BEST) return fail(c, VNS_EINVAL, "which must be 0 or 1");
    if (!zM || !zR) return fail(c, VNS_EINVAL, "NULL output");
    const ChainInfo &ci = c->chains[(size_t)chain];
    std::vector<Bits> b((size_t)ci.K);
    const Bits *src = (which == VNS_SOLUTION_BEST ? c->d_bestx : c->d_cur) + ci.cp0;
    VNS_HIP(c, hipMemcpyAsync(b.data(), src, sizeof(Bits) * (size_t)ci.K, hipMemcpyDeviceToHost, c->stream));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    for (int32_t k = 0; k < ci.K; ++k)
        for (int32_t t = 0; t < ci.T; ++t) {
            zM[(size_t)k * ci.T + t] = (uint8_t)((b[(size_t)k].m[t >> 5] >> (t & 31)) & 1u);
            zR[(size_t)k * ci.T + t] = (uint8_t)((b[(size_t)k].r[t >> 5] >> (t & 31)) & 1u);
        }
    return VNS_OK;
}

extern "C" vns_status vns_set_unit_costs(vns_ctx *c, const int32_t *pM, const int32_t *pR) {
    VNS_LIVE(c);
    if (!pM || !pR) return fail(c, VNS_EINVAL, "NULL input");
    std::vector<ProdParams> prod = c->prod_host;
    size_t p = 0;
    for (int32_t i = 0; i < c->n_inst; ++i) {
        __int128 F_bound = 0;
        for (int32_t k = 0; k < c->K[(size_t)i]; ++k, ++p) {
            if (pM[p] < 0 || pR[p] < 0 || pM[p] >= (1 << 16) || pR[p] >= (1 << 16))
                return fail(c, VNS_EINVAL, "unit costs must be in [0, 2^16)");
            const __int128 bound = (__int128)c->cost_bound[p] + (__int128)std::max(pM[p], pR[p]) * prod[p].SD;
            if (bound >= ((__int128)1 << 47)) return fail(c, VNS_ERANGE, "a product's cost could reach 2^47");
            F_bound += bound;
            prod[p].pM = pM[p];
            prod[p].pR = pR[p];
            set_cost_terms(prod[p]);
        }
        if (F_bound >= ((__int128)1 << 62)) return fail(c, VNS_ERANGE, "an instance's objective could reach 2^62");
    }
    drop_graph(c);
    VNS_HIP(c, hipMemcpyAsync(c->d_prod, prod.data(), sizeof(ProdParams) * prod.size(), hipMemcpyHostToDevice, c->stream));
    // every chain's costs from its current solution, as at creation: F = best = the new objective, k = 1
    InitArgs ia{c->d_chains, c->d_prod, c->d_rows, c->d_cur, c->d_cur_cost, c->d_work, c->d_work_cost, c->d_cs,
                c->d_bestx, 0};
    VNS_HIP(c, launch_init(ia, (int)c->chains.size(), c->stream, c->model));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    c->prod_host = prod;
    return VNS_OK;
}

static vns_status reinit_chain(vns_ctx *c, int32_t chain) {
    InitArgs ia{c->d_chains, c->d_prod, c->d_rows, c->d_cur, c->d_cur_cost, c->d_work, c->d_work_cost, c->d_cs,
                c->d_bestx, chain};
    VNS_HIP(c, launch_init(ia, 1, c->stream, c->model));
    return VNS_OK;
}

extern "C" vns_status vns_set_solution(vns_ctx *c, int32_t chain, const uint8_t *zM, const uint8_t *zR) {
    VNS_LIVE(c);
    vns_status s = check_chain(c, chain);
    if (s != VNS_OK) return s;
    if (!zM || !zR) return fail(c, VNS_EINVAL, "NULL input");
    const ChainInfo &ci = c->chains[(size_t)chain];
    std::vector<Bits> nb((size_t)ci.K), old((size_t)ci.K);
    for (int32_t k = 0; k < ci.K; ++k) {
        Bits b{};
        for (int32_t t = 0; t < ci.T; ++t) {
            if (zM[(size_t)k * ci.T + t]) b.m[t >> 5] |= 1u << (t & 31);
            if (zR[(size_t)k * ci.T + t]) b.r[t >> 5] |= 1u << (t & 31);
        }
        nb[(size_t)k] = b;
    }
    VNS_HIP(c, hipMemcpyAsync(old.data(), c->d_cur + ci.cp0, sizeof(Bits) * (size_t)ci.K, hipMemcpyDeviceToHost, c->stream));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    VNS_HIP(c, hipMemcpyAsync(c->d_cur + ci.cp0, nb.data(), sizeof(Bits) * (size_t)ci.K, hipMemcpyHostToDevice, c->stream));
    s = reinit_chain(c, chain);
    if (s != VNS_OK) return s;
    ChainState cs;
    VNS_HIP(c, hipMemcpyAsync(&cs, c->d_cs + chain, sizeof(cs), hipMemcpyDeviceToHost, c->stream));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    if (cs.F == kInf) {
        VNS_HIP(c, hipMemcpyAsync(c->d_cur + ci.cp0, old.data(), sizeof(Bits) * (size_t)ci.K, hipMemcpyHostToDevice, c->stream));
        s = reinit_chain(c, chain);
        if (s != VNS_OK) return s;
        VNS_HIP(c, hipStreamSynchronize(c->stream));
        return fail(c, VNS_ERANGE, "the solution leaves a product infeasible");
    }
    return VNS_OK;
}

extern "C" vns_status vns_get_trajectory(vns_ctx *c, int32_t chain, vns_record *rec, int64_t cap, int64_t *n) {
    VNS_LIVE(c);
    vns_status s = check_chain(c, chain);
    if (s != VNS_OK) return s;
    const int64_t avail = c->trace_iters;
    if (n) *n = avail;
    const int64_t m = std::min<int64_t>(avail, cap < 0 ? 0 : cap);
    if (rec && m > 0) {
        VNS_HIP(c, hipMemcpyAsync(rec, c->d_trace + (int64_t)chain * c->trace_iters, sizeof(vns_record) * (size_t)m,
                                  hipMemcpyDeviceToHost, c->stream));
        VNS_HIP(c, hipStreamSynchronize(c->stream));
    }
    return VNS_OK;
}

extern "C" vns_status vns_get_stats(const vns_ctx *c, vns_stats *out) {
    if (!c || !out) return fail(nullptr, VNS_EINVAL, "null argument");
    *out = c->stats;
    return VNS_OK;
}

extern "C" vns_status vns_instance_size(const vns_ctx *c, int32_t inst, int32_t *K, int32_t *T) {
    if (!c) return fail(nullptr, VNS_EINVAL, "null context");
    if (inst < 0 || inst >= c->n_inst) return fail(const_cast<vns_ctx *>(c), VNS_EINVAL, "instance out of range");
    if (K) *K = c->K[(size_t)inst];
    if (T) *T = c->T[(size_t)inst];
    return VNS_OK;
}

extern "C" int64_t vns_num_chains(const vns_ctx *c) { return c ? (int64_t)c->chains.size() : 0; }

extern "C" const char *vns_last_error(const vns_ctx *c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

extern "C" vns_status vns_test_inject_failure(int32_t kind, int32_t countdown) {
    if (countdown < 0) return fail(nullptr, VNS_EINVAL, "negative countdown");
    if (kind == VNS_INJECT_ALLOC) g_inject_alloc = countdown;
    else if (kind == VNS_INJECT_DEVICE) g_inject_device = countdown;
    else return fail(nullptr, VNS_EINVAL, "unknown injection kind");
    return VNS_OK;
}

// ---------------------------------------------------------------------------------------------------
// learned scorer
// ---------------------------------------------------------------------------------------------------
// He-uniform initial weights (He et al. 2015, uniform form: U(-sqrt(6/fan_in), +sqrt(6/fan_in))), zero
// biases.  Parameter i draws its uniform from splitmix64 (Steele, Lea & Flood, OOPSLA 2014) of seed + i + 1
// steps of the generator's Weyl sequence, top 53 bits.
static void mlp_he_uniform(uint64_t seed, std::vector<float> &p) {
    p.assign((size_t)mlp::kParams, 0.f);
    auto uniform = [seed](uint64_t i) {
        uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * 0x1.0p-53;
    };
    const struct { int off, fan_in, n; } layers[3] = {
        {mlp::oW1, mlp::kF, mlp::kF * mlp::kH}, {mlp::oW2, mlp::kH, mlp::kH * mlp::kH}, {mlp::oW3, mlp::kH, mlp::kH}};
    for (const auto &L : layers) {
        const double lim = std::sqrt(6.0 / (double)L.fan_in);
        for (int j = 0; j < L.n; ++j) p[(size_t)(L.off + j)] = (float)(lim * (2.0 * uniform((uint64_t)(L.off + j)) - 1.0));
    }
}

static vns_status upload_mlp(vns_ctx *c, const float *params) {
    VNS_HIP(c, hipMemcpyAsync(c->d_mlp, params, sizeof(float) * mlp::kParams, hipMemcpyHostToDevice, c->stream));
    VNS_HIP(c, hipMemsetAsync(c->d_adam_m, 0, sizeof(float) * mlp::kParams, c->stream));
    VNS_HIP(c, hipMemsetAsync(c->d_adam_v, 0, sizeof(float) * mlp::kParams, c->stream));
    c->adam_step = 0;
    drop_graph(c);
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    return VNS_OK;
}

extern "C" vns_status vns_mlp_init(vns_ctx *c, uint64_t seed) {
    VNS_LIVE(c);
    std::vector<float> p;
    mlp_he_uniform(seed, p);
    return upload_mlp(c, p.data());
}

extern "C" vns_status vns_mlp_set_params(vns_ctx *c, const float *params) {
    VNS_LIVE(c);
    if (!params) return fail(c, VNS_EINVAL, "NULL params");
    for (int i = 0; i < mlp::kParams; ++i)
        if (!(params[i] == params[i]) || params[i] > 1e30f || params[i] < -1e30f)
            return fail(c, VNS_EINVAL, "non-finite scorer parameter");
    return upload_mlp(c, params);
}

extern "C" vns_status vns_mlp_get_params(vns_ctx *c, float *params) {
    VNS_LIVE(c);
    if (!params) return fail(c, VNS_EINVAL, "NULL params");
    VNS_HIP(c, hipMemcpyAsync(params, c->d_mlp, sizeof(float) * mlp::kParams, hipMemcpyDeviceToHost, c->stream));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    return VNS_OK;
}

template <class T>
struct Scoped {
    T *p = nullptr;
    ~Scoped() { dfree(p); }
};

// Device time between the context's two events (recorded around a scorer call's kernels) into the stats.
static vns_status record_mlp_time(vns_ctx *c, int64_t rows) {
    float ms = 0.f;
    VNS_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->stats.last_mlp_ms = (double)ms;
    c->stats.last_mlp_rows = rows;
    return VNS_OK;
}

extern "C" vns_status vns_mlp_score(vns_ctx *c, const float *feats, int64_t n, float *scores) {
    VNS_LIVE(c);
    if (n < 0 || (n > 0 && (!feats || !scores))) return fail(c, VNS_EINVAL, "bad arguments");
    if (n == 0) return VNS_OK;
    Scoped<float> X, S;
    VNS_HIP(c, dmalloc(&X.p, (size_t)n * mlp::kF));
    VNS_HIP(c, dmalloc(&S.p, (size_t)n));
    VNS_HIP(c, hipMemcpyAsync(X.p, feats, sizeof(float) * mlp::kF * (size_t)n, hipMemcpyHostToDevice, c->stream));
    VNS_HIP(c, hipEventRecord(c->ev0, c->stream));
    VNS_HIP(c, launch_mlp_score(c->d_mlp, X.p, n, S.p, c->stream));
    VNS_HIP(c, hipEventRecord(c->ev1, c->stream));
    VNS_HIP(c, hipMemcpyAsync(scores, S.p, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, c->stream));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    return record_mlp_time(c, n);
}

// Device scratch of one gradient evaluation over up to n rows.
struct GradScratch {
    Scoped<float> part, grad;
    vns_status alloc(vns_ctx *c, int64_t n) {
        const int64_t nb = mlp_grad_partials(n);
        VNS_HIP(c, dmalloc(&part.p, (size_t)(nb * (mlp::kParams + 1))));
        VNS_HIP(c, dmalloc(&grad.p, (size_t)(mlp::kParams + 1)));
        return VNS_OK;
    }
};

extern "C" vns_status vns_mlp_grad(vns_ctx *c, const float *feats, const float *targets, int64_t n, float *grads,
                                   float *loss) {
    VNS_LIVE(c);
    if (n <= 0 || !feats || !targets) return fail(c, VNS_EINVAL, "bad arguments");
    Scoped<float> X, Y;
    VNS_HIP(c, dmalloc(&X.p, (size_t)n * mlp::kF));
    VNS_HIP(c, dmalloc(&Y.p, (size_t)n));
    VNS_HIP(c, hipMemcpyAsync(X.p, feats, sizeof(float) * mlp::kF * (size_t)n, hipMemcpyHostToDevice, c->stream));
    VNS_HIP(c, hipMemcpyAsync(Y.p, targets, sizeof(float) * (size_t)n, hipMemcpyHostToDevice, c->stream));
    GradScratch gs;
    vns_status st = gs.alloc(c, n);
    if (st != VNS_OK) return st;
    VNS_HIP(c, hipEventRecord(c->ev0, c->stream));
    VNS_HIP(c, launch_mlp_grad(c->d_mlp, X.p, Y.p, nullptr, n, gs.part.p, gs.grad.p,
                               c->stream));
    VNS_HIP(c, hipEventRecord(c->ev1, c->stream));
    std::vector<float> g((size_t)mlp::kParams + 1);
    VNS_HIP(c, hipMemcpyAsync(g.data(), gs.grad.p, sizeof(float) * g.size(), hipMemcpyDeviceToHost, c->stream));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    if (grads) std::memcpy(grads, g.data(), sizeof(float) * mlp::kParams);
    if (loss) *loss = g[(size_t)mlp::kParams];
    return record_mlp_time(c, n);
}

extern "C" vns_status vns_mlp_train(vns_ctx *c, const float *feats, const float *targets, int64_t n, int32_t epochs,
                                    int32_t batch, float lr, uint64_t seed, float *last_loss) {
    VNS_LIVE(c);
    if (n <= 0 || !feats || !targets || epochs < 0 || batch < 1 || !(lr > 0.f)) return fail(c, VNS_EINVAL, "bad arguments");
    Scoped<float> X, Y;
    VNS_HIP(c, dmalloc(&X.p, (size_t)n * mlp::kF));
    VNS_HIP(c, dmalloc(&Y.p, (size_t)n));
    VNS_HIP(c, hipMemcpyAsync(X.p, feats, sizeof(float) * mlp::kF * (size_t)n, hipMemcpyHostToDevice, c->stream));
    VNS_HIP(c, hipMemcpyAsync(Y.p, targets, sizeof(float) * (size_t)n, hipMemcpyHostToDevice, c->stream));
    const int64_t bmax = std::min<int64_t>(batch, n);
    GradScratch gs;
    vns_status st = gs.alloc(c, bmax);
    if (st != VNS_OK) return st;
    // rows of each epoch in the order (mul * i + add) mod n, mul coprime to n, add drawn per epoch
    uint64_t mul = 1000003ull;
    auto gcd = [](uint64_t a, uint64_t b) { while (b) { uint64_t t = a % b; a = b; b = t; } return a; };
    while (gcd(mul, (uint64_t)n) != 1) mul += 2;
    uint64_t state = seed * 0x9E3779B97F4A7C15ull + 1;
    float loss = 0.f;
    VNS_HIP(c, hipEventRecord(c->ev0, c->stream));
    for (int32_t e = 0; e < epochs; ++e) {
        state ^= state >> 33; state *= 0xFF51AFD7ED558CCDull; state ^= state >> 33;
        const uint64_t add = state % (uint64_t)n;
        for (int64_t s0 = 0; s0 < n; s0 += bmax) {
            const int64_t cnt = std::min<int64_t>(bmax, n - s0);
            // the minibatch's rows (mul i + add) mod n, i = s0 .. s0 + cnt - 1, are computed in the gradient kernel
            VNS_HIP(c, launch_mlp_train_step(c->d_mlp, c->d_adam_m, c->d_adam_v, X.p, Y.p, RowPerm{mul, add, s0, n}, cnt,
                                             gs.part.p, gs.grad.p, lr, ++c->adam_step, c->stream));
        }
    }
    VNS_HIP(c, hipEventRecord(c->ev1, c->stream));
    if (epochs > 0) {
        VNS_HIP(c, hipMemcpyAsync(&loss, gs.grad.p + mlp::kParams, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    }
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    if (last_loss) *last_loss = loss;
    return record_mlp_time(c, n * (int64_t)epochs);
}

extern "C" vns_status vns_get_move_log(vns_ctx *c, float *feats, float *targets, int64_t cap, int64_t *n) {
    VNS_LIVE(c);
    if (c->log_cap <= 0) {
        if (n) *n = 0;
        return VNS_OK;
    }
    unsigned long long cnt = 0;
    VNS_HIP(c, hipMemcpyAsync(&cnt, c->d_log_n, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    const int64_t avail = std::min<int64_t>((int64_t)cnt, c->log_cap);
    if (n) *n = avail;
    const int64_t m = std::min<int64_t>(avail, cap < 0 ? 0 : cap);
    if (m > 0 && feats)
        VNS_HIP(c, hipMemcpyAsync(feats, c->d_log_x, sizeof(float) * mlp::kF * (size_t)m, hipMemcpyDeviceToHost, c->stream));
    if (m > 0 && targets)
        VNS_HIP(c, hipMemcpyAsync(targets, c->d_log_y, sizeof(float) * (size_t)m, hipMemcpyDeviceToHost, c->stream));
    VNS_HIP(c, hipStreamSynchronize(c->stream));
    return VNS_OK;
}

__global__ void k_fill_nan(float *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = __int_as_float(0x7FC00000);
}

extern "C" vns_status vns_eval_learned(vns_ctx *c, uint32_t nb, int32_t chain, int32_t top_permille, float *scores,
                                       uint8_t *selected, int64_t *prod_best, int32_t *prod_best_slot, uint8_t *fallback) {
    VNS_LIVE(c);
    if (nb != VNS_NB_FLIP_M && nb != VNS_NB_FLIP_R && nb != VNS_NB_SHIFT) return fail(c, VNS_EINVAL, "nb must be one neighbourhood");
    if (c->model != 0)
        return fail(c, VNS_EINVAL, "the learned choice takes only the default decode reading (VNS_OPT_DECODE = 0)");
    if (top_permille < 1 || top_permille > 1000) return fail(c, VNS_EINVAL, "top_permille must be in 1..1000");
    vns_status st = check_chain(c, chain);
    if (st != VNS_OK) return st;
    const ChainInfo &ci = c->chains[(size_t)chain];
    const int64_t n_slots = 4LL * ci.K * ci.T, slot0 = c->price_off[(size_t)chain];
    Scoped<float> S;
    Scoped<uint8_t> Sel, Fb;
    Scoped<int64_t> PP;
    Scoped<int32_t> PS;
    VNS_HIP(c, dmalloc(&S.p, (size_t)n_slots));
    VNS_HIP(c, dmalloc(&Sel.p, (size_t)n_slots));
    VNS_HIP(c, dmalloc(&Fb.p, (size_t)ci.K));
    hipLaunchKernelGGL(k_fill_nan, dim3((unsigned)((n_slots + 255) / 256)), dim3(256), 0, c->stream, S.p, n_slots);
    VNS_HIP(c, hipGetLastError());
    VNS_HIP(c, hipMemsetAsync(Sel.p, 0, (size_t)n_slots, c->stream));
    VNS_HIP(c, hipMemsetAsync(c->d_evals, 0, sizeof(unsigned long long) * counter_words(), c->stream));
    EvalLearnedArgs a{};
    a.cp_chain = c->d_cp_chain;
    a.chains = c->d_chains;
    a.prod = c->d_prod;
    a.rows = c->d_rows;
    a.cur = c->d_cur;
    a.cur_cost = c->d_cur_cost;
    a.cstate = c->d_cs;
    a.mlp = c->d_mlp;
    a.slot_off = c->d_price_off;
    a.scores = S.p - slot0;
    a.selected = Sel.p - slot0;
    a.prod_price = c->d_prod_price;
    a.prod_slot = c->d_prod_slot;
    a.fallback = Fb.p - ci.cp0;
    a.evals = c->d_evals;
    a.nb = nb;
    a.permille = top_permille;
    VNS_HIP(c, launch_eval_learned(a, ci.cp0, ci.K, c->stream));
    if (scores) VNS_HIP(c, hipMemcpyAsync(scores, S.p, sizeof(float) * (size_t)n_slots, hipMemcpyDeviceToHost, c->stream));
    if (selected) VNS_HIP(c, hipMemcpyAsync(selected, Sel.p, (size_t)n_slots, hipMemcpyDeviceToHost, c->stream));
    if (prod_best) VNS_HIP(c, hipMemcpyAsync(prod_best, c->d_prod_price + ci.cp0, sizeof(int64_t) * (size_t)ci.K, hipMemcpyDeviceToHost, c->stream));
    if (prod_best_slot) VNS_HIP(c, hipMemcpyAsync(prod_best_slot, c->d_prod_slot + ci.cp0, sizeof(int32_t) * (size_t)ci.K, hipMemcpyDeviceToHost, c->stream));
    if (fallback) VNS_HIP(c, hipMemcpyAsync(fallback, Fb.p, (size_t)ci.K, hipMemcpyDeviceToHost, c->stream));
    unsigned long long ev[3] = {0, 0, 0};
    VNS_HIP(c, read_counters(c, ev));
    c->stats.last_eval_evals = (int64_t)ev[0];
    c->stats.last_eval_period_steps = (int64_t)ev[0] * ci.T;
    return VNS_OK;
}
