// Issue-rate probe for the integer VALU operations of the decode's period-step, on gfx950.
//
// The pricing kernels are bound by integer vector ALU issue, not by HBM.  Their peak is derived from the
// chip's unit counts and clock (256 compute units x 4 SIMDs x 16 lanes at 2.4 GHz = 64 lane-operations per
// CU per clock for a single-rate operation) and from the rate class of each operation of the step.  This
// probe measures each class on the device: every lane runs eight independent dependency chains of one
// operation (so issue, not latency, limits it) in a grid that fills every SIMD, and the rate is reported as
// lane-operations per CU per nominal clock.  A last kernel runs the decode's own period-step on independent
// states with operands in registers, giving the achievable rate of the whole 14-operation mix.
//
// Built into its own library (libvaluprobe.so); bench.py --valu-probe calls it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vns_device.hpp"

namespace {

constexpr int kChains = 8;

enum Op {
    kAdd = 0, kSub, kBitop3, kBfi, kBfe, kMad24, kMin, kAndOr, kDecodeStep, kNumOps
};

template <int OP>
__device__ __forceinline__ void step_op(uint32_t &x, uint32_t a, uint32_t b) {
    if constexpr (OP == kAdd) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x) : "v"(a));
    else if constexpr (OP == kSub) asm volatile("v_sub_u32 %0, %0, %1" : "+v"(x) : "v"(a));
    else if constexpr (OP == kBitop3) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x6c" : "+v"(x) : "v"(a), "v"(b));
    else if constexpr (OP == kBfi) asm volatile("v_bfi_b32 %0, %1, %2, %0" : "+v"(x) : "v"(a), "v"(b));
    else if constexpr (OP == kBfe) asm volatile("v_bfe_i32 %0, %0, %1, 1" : "+v"(x) : "v"(a));
    else if constexpr (OP == kMad24) asm volatile("v_mad_u32_u24 %0, %1, %2, %0" : "+v"(x) : "v"(a), "v"(b));
    else if constexpr (OP == kMin) asm volatile("v_min_i32 %0, %0, %1" : "+v"(x) : "v"(a));
    else if constexpr (OP == kAndOr) asm volatile("v_and_or_b32 %0, %1, %2, %0" : "+v"(x) : "v"(a), "v"(b));
}

// iters x 16 steps of kChains independent chains; ops per lane = iters * 16 * kChains.
template <int OP>
__global__ __launch_bounds__(256) void k_probe(uint32_t *out, int iters, uint32_t seed) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = tid * 2654435761u + c + seed;
    const uint32_t a = tid ^ seed, b = (tid << 3) | 5u;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int c = 0; c < kChains; ++c) step_op<OP>(x[c], a, b);
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r ^= x[c];
    out[tid] = r;
}

// The decode's period-step (vns::decode_chunk, four vns::decode_step) on two independent states per lane,
// with the period offset a run-time scalar as in the pricing loop; setup words change every iteration and
// the rows stay in registers, so only the step's own arithmetic is issued.  Period-steps per lane =
// iters * 32 * 2.
__global__ __launch_bounds__(256) void k_probe_decode(uint32_t *out, int iters, uint32_t seed) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    vns::DecodeState s0, s1;
    int32_t m = (int32_t)(tid * 2654435761u ^ seed), r = (int32_t)(tid * 40503u + seed);
    int32_t m1 = (int32_t)(tid * 2246822519u + seed), r1 = (int32_t)(tid * 3266489917u ^ seed);
    int2 c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) c[q] = make_int2((int)((tid + q) & 127), (int)(((tid >> 7) + 50 * q) & 1023));
    for (int i = 0; i < iters; ++i) {
        const int base = __builtin_amdgcn_readfirstlane((int)((i + seed) & 7)) * 4;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            vns::decode_chunk(s0, m, r, base + 4 * q, c);
            vns::decode_chunk(s1, m1, r1, base + 4 * q, c);
        }
        m = (int32_t)__builtin_amdgcn_alignbit((uint32_t)m, (uint32_t)r, 7);
        m1 = (int32_t)__builtin_amdgcn_alignbit((uint32_t)m1, (uint32_t)r1, 5);
    }
    out[tid] = (uint32_t)(s0.A1 ^ s0.A2 ^ s0.XR ^ s0.bad ^ s1.A1 ^ s1.A2 ^ s1.XR ^ s1.bad);
}

template <int OP>
hipError_t launch(uint32_t *out, int grid, int iters, hipStream_t s) {
    hipLaunchKernelGGL(k_probe<OP>, dim3(grid), dim3(256), 0, s, out, iters, 12345u);
    return hipGetLastError();
}

}  // namespace

// Names of the probed operations, in the order of the op index.
extern "C" const char *valu_probe_name(int op) {
    static const char *names[kNumOps] = {"v_add_u32", "v_sub_u32", "v_bitop3_b32", "v_bfi_b32", "v_bfe_i32",
                                         "v_mad_u32_u24", "v_min_i32", "v_and_or_b32", "decode_step"};
    return (op >= 0 && op < kNumOps) ? names[op] : nullptr;
}

extern "C" int valu_probe_count() { return kNumOps; }

// Runs probe `op` once on the current device: grid workgroups of 256 lanes, `iters` outer iterations.
// *ms receives the kernel time (HIP events), *lane_ops the lane-operations it executed (for decode_step:
// lane period-steps).  Returns 0, or the hipError_t of the first failing call.
extern "C" int valu_probe_run(int op, int grid, int iters, double *ms, double *lane_ops) {
    if (op < 0 || op >= kNumOps || grid < 1 || iters < 1 || !ms || !lane_ops) return (int)hipErrorInvalidValue;
    uint32_t *out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void **)&out, sizeof(uint32_t) * (size_t)grid * 256);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) {
        switch (op) {
            case kAdd: e = launch<kAdd>(out, grid, iters, s); break;
            case kSub: e = launch<kSub>(out, grid, iters, s); break;
            case kBitop3: e = launch<kBitop3>(out, grid, iters, s); break;
            case kBfi: e = launch<kBfi>(out, grid, iters, s); break;
            case kBfe: e = launch<kBfe>(out, grid, iters, s); break;
            case kMad24: e = launch<kMad24>(out, grid, iters, s); break;
            case kMin: e = launch<kMin>(out, grid, iters, s); break;
            case kAndOr: e = launch<kAndOr>(out, grid, iters, s); break;
            default:
                hipLaunchKernelGGL(k_probe_decode, dim3(grid), dim3(256), 0, s, out, iters, 12345u);
                e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    *ms = t;
    const double lanes = (double)grid * 256.0;
    *lane_ops = op == kDecodeStep ? lanes * iters * 64.0 : lanes * iters * 16.0 * kChains;
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (s) (void)hipStreamDestroy(s);
    if (out) (void)hipFree(out);
    return (int)e;
}
