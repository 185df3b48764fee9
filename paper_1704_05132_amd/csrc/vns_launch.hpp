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

hipError_t launch_init(const InitArgs &a, int n_chains, hipStream_t s);
hipError_t launch_eval(const EvalArgs &a, const EvalWg *wg, int64_t n_wg, hipStream_t s);
hipError_t launch_chain_best(const ChainBestArgs &a, int n_chains, hipStream_t s);
hipError_t launch_run(const RunArgs &a, int n_chains, int waves, size_t lds_bytes, hipStream_t s);

}  // namespace vns
