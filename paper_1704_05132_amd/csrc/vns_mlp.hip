// Kernels of the learned move scorer: batch scoring, forward with saved pre-activations, backward,
// deterministic gradient reduction and the Adam update (Kingma & Ba 2015).
//
// Training objective: mean squared error between the score and the target over a minibatch.  Gradients
// treat the bfloat16-rounded weights and layer inputs as their float values (straight-through), the usual
// mixed-precision rule; the backward pass runs in float32.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "vns_launch.hpp"
#include "vns_mlp.hpp"

namespace vns {
namespace mlp {

// Scores of n feature rows (X 16-byte aligned): each wavefront loads the weight fragments once and scores
// tiles of 64 rows blockIdx.x, blockIdx.x + gridDim.x, ...; the next tile's rows (one 64-byte row per lane,
// four 16-byte loads) are in flight while the current tile is scored.
__global__ __launch_bounds__(64) void k_mlp_score(const float *__restrict__ P, const float *__restrict__ X, int64_t n,
                                                  float *__restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) __bf16 s_mlp[];
    __bf16 *sx = s_mlp;
    const int lane = threadIdx.x & 63;
    const float4 zero4 = {0.f, 0.f, 0.f, 0.f};
    float4 v[4];
    auto fetch = [&](int64_t tile) {   // rows past n read row n-1 and score zeros
        const int64_t row = tile * 64 + lane;
        const float4 *src = reinterpret_cast<const float4 *>(X + (row < n ? row : n - 1) * kF);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 w = src[q];
            v[q] = row < n ? w : zero4;
        }
    };
    int64_t tile = blockIdx.x;
    if (tile * 64 < n) fetch(tile);
    Frags fr;
    load_frags(P, fr);
    for (; tile * 64 < n; tile += gridDim.x) {
        bf8 lo, hi;
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                lo[4 * q + e] = (__bf16)v[q][e];
                hi[4 * q + e] = (__bf16)v[2 + q][e];
            }
        *reinterpret_cast<bf8 *>(sx + lane * kF) = lo;
        *reinterpret_cast<bf8 *>(sx + lane * kF + 8) = hi;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if ((tile + gridDim.x) * 64 < n) fetch(tile + gridDim.x);
        const float s = forward64(sx, fr);   // ends with a wavefront barrier: sx may be rewritten
        const int64_t row = tile * 64 + lane;
        if (row < n) out[row] = s;
    }
}

// The same forward pass for the rows idx[0..n) of a training set (all rows when idx is null): stores the rows
// in minibatch order in Xb, the scores in s_out and the hidden pre-activations in z1, z2 (float32).  Xb, z1
// and z2 are sized for whole blocks of 64 rows.
__global__ __launch_bounds__(64) void k_mlp_fwd_cache(const float *__restrict__ P, const float *__restrict__ X,
                                                      const int64_t *__restrict__ idx, int64_t n, float *__restrict__ Xb,
                                                      float *__restrict__ s_out, float *__restrict__ z1,
                                                      float *__restrict__ z2) {
    extern __shared__ __attribute__((aligned(16))) __bf16 s_mlp[];
    __bf16 *sx = s_mlp;
    Frags fr;
    load_frags(P, fr);
    const int lane = threadIdx.x & 63;
    const int64_t base = (int64_t)blockIdx.x * 64, r = base + lane;
    const int64_t src = r < n ? (idx ? idx[r] : r) : 0;
#pragma unroll
    for (int f = 0; f < kF; ++f) {
        const float v = r < n ? X[src * kF + f] : 0.f;
        sx[lane * kF + f] = (__bf16)v;
        Xb[r * kF + f] = v;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float s = forward64(sx, fr, z1 + base * kH, z2 + base * kH);
    if (r < n) s_out[r] = s;
}

// Backward: one workgroup of 64 lanes per 64 rows writes its partial gradients (and partial loss) to
// part[blockIdx.x][kParams + 1].
__global__ __launch_bounds__(256) void k_mlp_bwd(const float *__restrict__ P, const float *__restrict__ Xb,
                                                 const float *__restrict__ y, const int64_t *__restrict__ idx,
                                                 const float *__restrict__ s, const float *__restrict__ z1,
                                                 const float *__restrict__ z2, int64_t n, float inv_n,
                                                 float *__restrict__ part) {
    __shared__ float a0[64][kF];
    __shared__ float a1[64][kH];
    __shared__ float a2[64][kH];
    __shared__ float dz1[64][kH];
    __shared__ float dz2[64][kH];
    __shared__ float ds[64];
    __shared__ float w2q[kH][kH + 1];
    __shared__ float w3q[kH];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * 64;
    for (int i = tid; i < kH * kH; i += blockDim.x) w2q[i / kH][i % kH] = (float)(__bf16)P[oW2 + i];
    for (int i = tid; i < kH; i += blockDim.x) w3q[i] = (float)(__bf16)P[oW3 + i];
    for (int i = tid; i < 64 * kF; i += blockDim.x) {
        const int b = i / kF;
        a0[b][i % kF] = base + b < n ? (float)(__bf16)Xb[(base + b) * kF + i % kF] : 0.f;
    }
    for (int i = tid; i < 64 * kH; i += blockDim.x) {
        const int b = i / kH, j = i % kH;
        const bool in = base + b < n;
        const float v1 = in ? z1[(base + b) * kH + j] : 0.f, v2 = in ? z2[(base + b) * kH + j] : 0.f;
        a1[b][j] = (float)(__bf16)fmaxf(v1, 0.f);
        a2[b][j] = (float)(__bf16)fmaxf(v2, 0.f);
        dz1[b][j] = v1;   // pre-activation for now (its sign gives the ReLU mask)
        dz2[b][j] = v2;
    }
    if (tid < 64) {
        const int64_t r = base + tid;
        const float t = r < n ? y[idx ? idx[r] : r] : 0.f;
        ds[tid] = r < n ? 2.f * (s[r] - t) * inv_n : 0.f;
    }
    __syncthreads();
    for (int i = tid; i < 64 * kH; i += blockDim.x) {
        const int b = i / kH, j = i % kH;
        dz2[b][j] = dz2[b][j] > 0.f ? ds[b] * w3q[j] : 0.f;
    }
    __syncthreads();
    for (int i = tid; i < 64 * kH; i += blockDim.x) {
        const int b = i / kH, j = i % kH;
        float acc = 0.f;
        for (int q = 0; q < kH; ++q) acc += dz2[b][q] * w2q[j][q];
        dz1[b][j] = dz1[b][j] > 0.f ? acc : 0.f;
    }
    __syncthreads();
    float *out = part + (int64_t)blockIdx.x * (kParams + 1);
    for (int e = tid; e < kParams + 1; e += blockDim.x) {
        float acc = 0.f;
        if (e < oB1) {                       // W1[f][i]
            const int f = e / kH, i = e % kH;
            for (int b = 0; b < 64; ++b) acc += a0[b][f] * dz1[b][i];
        } else if (e < oW2) {                // b1
            for (int b = 0; b < 64; ++b) acc += dz1[b][e - oB1];
        } else if (e < oB2) {                // W2[i][j]
            const int i = (e - oW2) / kH, j = (e - oW2) % kH;
            for (int b = 0; b < 64; ++b) acc += a1[b][i] * dz2[b][j];
        } else if (e < oW3) {                // b2
            for (int b = 0; b < 64; ++b) acc += dz2[b][e - oB2];
        } else if (e < oB3) {                // W3
            for (int b = 0; b < 64; ++b) acc += a2[b][e - oW3] * ds[b];
        } else if (e == oB3) {               // b3
            for (int b = 0; b < 64; ++b) acc += ds[b];
        } else {                             // loss contribution
            for (int b = 0; b < 64; ++b) {
                const int64_t r = base + b;
                if (r < n) {
                    const float d = s[r] - y[idx ? idx[r] : r];
                    acc += d * d * inv_n;
                }
            }
        }
        out[e] = acc;
    }
}

// Fixed-order sum of the partial gradients of nb workgroups: out[e] = sum_b part[b][e].
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ part, int64_t nb, float *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e > kParams) return;
    float acc = 0.f;
    for (int64_t b = 0; b < nb; ++b) acc += part[b * (kParams + 1) + e];
    out[e] = acc;
}

// Adam on the float32 master parameters.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ P, const float *__restrict__ grad, float *__restrict__ m,
                                              float *__restrict__ v, float lr, float beta1, float beta2, float eps,
                                              float corr1, float corr2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kParams) return;
    const float g = grad[e];
    const float mm = beta1 * m[e] + (1.f - beta1) * g;
    const float vv = beta2 * v[e] + (1.f - beta2) * g * g;
    m[e] = mm;
    v[e] = vv;
    P[e] -= lr * (mm / corr1) / (sqrtf(vv / corr2) + eps);
}

}  // namespace mlp

hipError_t launch_mlp_score(const float *P, const float *X, int64_t n, float *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (n + 63) / 64;
    const unsigned grid = (unsigned)std::min<int64_t>(tiles, 256 * 8);   // 8 wavefronts per CU, each many tiles
    hipLaunchKernelGGL(mlp::k_mlp_score, dim3(grid), dim3(64), mlp::kWaveLdsBytes, s, P, X, n, out);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *P, const float *X, const float *y, const int64_t *idx, int64_t n, float *Xb,
                           float *sc, float *z1, float *z2, float *part, float *grad_out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(mlp::k_mlp_fwd_cache, dim3(nb), dim3(64), mlp::kWaveLdsBytes, s, P, X, idx, n, Xb, sc, z1, z2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp::k_mlp_bwd, dim3(nb), dim3(256), 0, s, P, Xb, y, idx, sc, z1, z2, n, 1.f / (float)n, part);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp::k_mlp_reduce, dim3((mlp::kParams + 1 + 255) / 256), dim3(256), 0, s, part, (int64_t)nb, grad_out);
    return hipGetLastError();
}

hipError_t launch_adam(float *P, const float *grad, float *m, float *v, float lr, int64_t step, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(mlp::k_adam, dim3((mlp::kParams + 255) / 256), dim3(256), 0, s, P, grad, m, v, 1.f * lr, b1, b2,
                       1e-8f, c1, c2);
    return hipGetLastError();
}

}  // namespace vns
