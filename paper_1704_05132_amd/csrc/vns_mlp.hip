// Kernels of the learned move scorer: batch scoring, the gradient (forward and backward in one pass),
// deterministic gradient reduction and the Adam update (Kingma & Ba 2015).
//
// Training objective: mean squared error between the score and the target over a minibatch.  Gradients
// treat the bfloat16-rounded weights and layer inputs as their float values (straight-through), the usual
// mixed-precision rule.  The backward pass runs on the matrix cores like the forward one: bfloat16 operands
// (weights, layer inputs, deltas), float32 accumulation; bias gradients are float32 sums.
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
        const float s = forward64<4>(sx, fr);   // ends with a wavefront barrier: sx may be rewritten
        const int64_t row = tile * 64 + lane;
        if (row < n) out[row] = s;
    }
}

// Gradient of the mean squared error on the matrix cores, forward and backward in one pass.  One wavefront
// per workgroup takes the 64-row tiles blockIdx.x, blockIdx.x + gridDim.x, ... of the rows idx[0..n) (all rows
// when idx is null) and writes its partial gradients (and partial loss) to part[blockIdx.x][kParams + 1].
//
// Per 16 rows the forward pass is forward64's (bfloat16 operands, float32 accumulation), and the deltas stay
// in its fragment layout: dz2 = [z2 > 0] ds w3 and dz1 = [z1 > 0] (W2 dz2), the latter on the matrix cores
// with dz2's D fragments taken, in the order pi, as B fragments (as layer 2 takes layer 1's).  The tile's
// layer inputs and deltas go to LDS transposed (unit-major, rows contiguous), so that dW2 = sum over rows of
// h1 dz2^T and dW1 = x dz1^T are products with the rows as K.  Weight gradients accumulate in registers over
// the wavefront's tiles; bias gradients as per-lane sums over rows, added across lanes at the end.
constexpr int kGradLd = 64 + 8;   // padded row (bfloat16) of the transposed tiles: 16-byte reads stay aligned

__global__ __launch_bounds__(64) void k_mlp_grad(const float *__restrict__ P, const float *__restrict__ X,
                                                 const float *__restrict__ y, const int64_t *__restrict__ idx,
                                                 RowPerm perm, int64_t n, float inv_n, float *__restrict__ part) {
    __shared__ __attribute__((aligned(16))) __bf16 sx[64 * kF];        // [row][feature]: forward input
    __shared__ __attribute__((aligned(16))) __bf16 xT[kF * kGradLd];   // [feature][row]
    __shared__ __attribute__((aligned(16))) __bf16 hT[kH * kGradLd];   // [unit][row]: relu(z1)
    __shared__ __attribute__((aligned(16))) __bf16 d2T[kH * kGradLd];  // [unit][row]: dz2
    __shared__ __attribute__((aligned(16))) __bf16 d1T[kH * kGradLd];  // [unit][row]: dz1
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
    Frags fr;
    load_frags(P, fr);
    bf8 w2b[4][2];   // A fragments of W2 for W2 dz2: rows i = 16 mi + c, inputs j in the order pi(kt, 8g + e)
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int e = 0; e < 8; ++e)
                w2b[mi][kt][e] = (__bf16)P[oW2 + (16 * mi + c) * kH + 32 * kt + 16 * (e >> 2) + 4 * g + (e & 3)];
    const f4 z4 = {0.f, 0.f, 0.f, 0.f};
    const bf8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
    f4 gW2[4][4];                  // [mi][nj]: dW2[16 mi + 4g + e][16 nj + c]
    f4 gW1[4];                     // [ni]: dW1[4g + e][16 ni + c]
    f4 gb1[4], gb2[4], gw3[4];     // [t]: this lane's rows' sums for unit 16 t + 4g + e
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        gW1[t] = gb1[t] = gb2[t] = gw3[t] = z4;
#pragma unroll
        for (int u = 0; u < 4; ++u) gW2[t][u] = z4;
    }
    float gb3 = 0.f, gloss = 0.f;

    for (int64_t tile = blockIdx.x; tile * 64 < n; tile += gridDim.x) {
        // lane l stages row 64 tile + l (zeros past n: such rows have ds = 0 and add nothing)
        const int64_t r = tile * 64 + lane;
        const bool in = r < n;
        const int64_t src = !in ? 0
                            : idx ? idx[r]
                            : perm.n > 0 ? (int64_t)(((unsigned __int128)perm.mul * (uint64_t)(perm.start + r) + perm.add) %
                                                     (uint64_t)perm.n)
                                         : r;
        const float yl = in ? y[src] : 0.f;
        const float4 *xs = reinterpret_cast<const float4 *>(X + src * kF);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 v = in ? xs[q] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const __bf16 b = (__bf16)vv[e];
                sx[lane * kF + 4 * q + e] = b;
                xT[(4 * q + e) * kGradLd + lane] = b;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 1
        for (int nt = 0; nt < 4; ++nt) {   // 16 rows at a time
            const int row = 16 * nt + c;
            const bf8 xb = g < 2 ? *reinterpret_cast<const bf8 *>(sx + row * kF + 8 * g) : zero8;
            f4 d1[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) d1[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.w1t[mt], xb, fr.b1[mt], 0, 0, 0);
            bf8 h[2];
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int e = 0; e < 4; e += 2) {
                    const bf2 lo = relu_pack(d1[2 * kt][e], d1[2 * kt][e + 1]);
                    const bf2 hi = relu_pack(d1[2 * kt + 1][e], d1[2 * kt + 1][e + 1]);
                    h[kt][e] = lo[0];
                    h[kt][e + 1] = lo[1];
                    h[kt][4 + e] = hi[0];
                    h[kt][4 + e + 1] = hi[1];
                    hT[(32 * kt + 4 * g + e) * kGradLd + row] = lo[0];
                    hT[(32 * kt + 4 * g + e + 1) * kGradLd + row] = lo[1];
                    hT[(32 * kt + 16 + 4 * g + e) * kGradLd + row] = hi[0];
                    hT[(32 * kt + 16 + 4 * g + e + 1) * kGradLd + row] = hi[1];
                }
            f4 d2[4];
            float acc3 = 0.f;
#pragma unroll
            for (int mo = 0; mo < 4; ++mo) {
                d2[mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.w2t[mo][0], h[0], fr.b2[mo], 0, 0, 0);
                d2[mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.w2t[mo][1], h[1], d2[mo], 0, 0, 0);
                acc3 = __builtin_amdgcn_fdot2_f32_bf16(relu_pack(d2[mo][0], d2[mo][1]), fr.w3[mo][0], acc3, false);
                acc3 = __builtin_amdgcn_fdot2_f32_bf16(relu_pack(d2[mo][2], d2[mo][3]), fr.w3[mo][1], acc3, false);
            }
            acc3 += __shfl_xor(acc3, 16, 64);
            acc3 += __shfl_xor(acc3, 32, 64);
            const float sc = fr.b3 + acc3;                 // score of row 16 nt + c (in every lane group)
            const float yr = __shfl(yl, row, 64);
            const bool rin = tile * 64 + row < n;
            const float dsr = rin ? 2.f * (sc - yr) * inv_n : 0.f;
            if (g == 0 && rin) {
                gb3 += dsr;
                gloss += (sc - yr) * (sc - yr) * inv_n;
            }
            // dz2 = [z2 > 0] ds w3, with dW3 and db2's row sums
            f4 dz2[4];
#pragma unroll
            for (int mo = 0; mo < 4; ++mo) {
                const bf2 a01 = relu_pack(d2[mo][0], d2[mo][1]), a23 = relu_pack(d2[mo][2], d2[mo][3]);
                const float a2[4] = {(float)a01[0], (float)a01[1], (float)a23[0], (float)a23[1]};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float w3v = (float)fr.w3[mo][e >> 1][e & 1];
                    const float dz = d2[mo][e] > 0.f ? dsr * w3v : 0.f;
                    dz2[mo][e] = dz;
                    gb2[mo][e] += dz;
                    gw3[mo][e] += a2[e] * dsr;
                    d2T[(16 * mo + 4 * g + e) * kGradLd + row] = (__bf16)dz;
                }
            }
            // dz1 = [z1 > 0] (W2 dz2) on the matrix cores
            bf8 dzb[2];
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    dzb[kt][e] = (__bf16)dz2[2 * kt][e];
                    dzb[kt][4 + e] = (__bf16)dz2[2 * kt + 1][e];
                }
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) {
                f4 dh = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2b[mi][0], dzb[0], z4, 0, 0, 0);
                dh = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2b[mi][1], dzb[1], dh, 0, 0, 0);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float dz = d1[mi][e] > 0.f ? dh[e] : 0.f;
                    gb1[mi][e] += dz;
                    d1T[(16 * mi + 4 * g + e) * kGradLd + row] = (__bf16)dz;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // weight gradients of the tile: the 64 rows as K, in two slices of 32
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            const int k0 = 32 * kt + 8 * g;
            bf8 bd2[4];
#pragma unroll
            for (int nj = 0; nj < 4; ++nj) bd2[nj] = *reinterpret_cast<const bf8 *>(d2T + (16 * nj + c) * kGradLd + k0);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) {
                const bf8 ah = *reinterpret_cast<const bf8 *>(hT + (16 * mi + c) * kGradLd + k0);
#pragma unroll
                for (int nj = 0; nj < 4; ++nj) gW2[mi][nj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bd2[nj], gW2[mi][nj], 0, 0, 0);
            }
            const bf8 ax = *reinterpret_cast<const bf8 *>(xT + c * kGradLd + k0);
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) {
                const bf8 bd1 = *reinterpret_cast<const bf8 *>(d1T + (16 * ni + c) * kGradLd + k0);
                gW1[ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, bd1, gW1[ni], 0, 0, 0);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // the next tile rewrites the LDS tiles
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // this wavefront's partial, in the parameters' order
    float *out = part + (int64_t)blockIdx.x * (kParams + 1);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
#pragma unroll
            for (int u = 0; u < 4; ++u) out[oW2 + (16 * t + 4 * g + e) * kH + 16 * u + c] = gW2[t][u][e];
            out[oW1 + (4 * g + e) * kH + 16 * t + c] = gW1[t][e];
            // bias and W3 gradients: the sum over the 16 lanes (rows) of each lane group
            float b1 = gb1[t][e], b2 = gb2[t][e], w3 = gw3[t][e];
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                b1 += __shfl_xor(b1, off, 64);
                b2 += __shfl_xor(b2, off, 64);
                w3 += __shfl_xor(w3, off, 64);
            }
            if (c == 0) {
                out[oB1 + 16 * t + 4 * g + e] = b1;
                out[oB2 + 16 * t + 4 * g + e] = b2;
                out[oW3 + 16 * t + 4 * g + e] = w3;
            }
        }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        gb3 += __shfl_xor(gb3, off, 64);
        gloss += __shfl_xor(gloss, off, 64);
    }
    if (lane == 0) {
        out[oB3] = gb3;
        out[kParams] = gloss;
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

// The fixed-order sum of the partial gradients (as k_mlp_reduce) and the Adam step on each parameter, in one
// pass: thread e sums parameter e's partials, stores the gradient (and the loss at e = kParams) and updates
// the parameter and its moments.
__global__ __launch_bounds__(256) void k_mlp_reduce_adam(const float *__restrict__ part, int64_t nb, float *__restrict__ out,
                                                         float *__restrict__ P, float *__restrict__ m,
                                                         float *__restrict__ v, float lr, float beta1, float beta2,
                                                         float eps, float corr1, float corr2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e > kParams) return;
    float g = 0.f;
    for (int64_t b = 0; b < nb; ++b) g += part[b * (kParams + 1) + e];
    out[e] = g;
    if (e == kParams) return;
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

hipError_t launch_mlp_grad(const float *P, const float *X, const float *y, const int64_t *idx, int64_t n, float *part,
                           float *grad_out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = mlp_grad_partials(n);
    hipLaunchKernelGGL(mlp::k_mlp_grad, dim3((unsigned)nb), dim3(64), 0, s, P, X, y, idx, RowPerm{0, 0, 0, 0}, n,
                       1.f / (float)n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp::k_mlp_reduce, dim3((mlp::kParams + 1 + 255) / 256), dim3(256), 0, s, part, nb, grad_out);
    return hipGetLastError();
}

int64_t mlp_grad_partials(int64_t n) { return std::min<int64_t>((n + 63) / 64, mlp::kGradWaves); }

hipError_t launch_mlp_train_step(float *P, float *m, float *v, const float *X, const float *y, const RowPerm &perm,
                                 int64_t cnt, float *part, float *grad_out, float lr, int64_t step, hipStream_t s) {
    if (cnt <= 0) return hipSuccess;
    const int64_t nb = mlp_grad_partials(cnt);
    hipLaunchKernelGGL(mlp::k_mlp_grad, dim3((unsigned)nb), dim3(64), 0, s, P, X, y, nullptr, perm, cnt,
                       1.f / (float)cnt, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(mlp::k_mlp_reduce_adam, dim3((mlp::kParams + 1 + 255) / 256), dim3(256), 0, s, part, nb, grad_out,
                       P, m, v, lr, b1, b2, 1e-8f, c1, c2);
    return hipGetLastError();
}

}  // namespace vns
