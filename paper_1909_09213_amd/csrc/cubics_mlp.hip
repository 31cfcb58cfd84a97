// Training and evaluation kernels of the branching-policy network (forward
// with BF16 MFMA / FP32 accumulation, backward with wave reductions, Adam on
// FP32 master weights, BF16 re-rounding of the weights the MFMAs read).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cubics_internal.h"
#include "cubics_mlp.h"

namespace cubics {

// bf16 copies of W1 (padded to 16 inputs) and w2 from the fp32 master theta
__global__ void policy_round_kernel(const float *theta, uint16_t *w1b, uint16_t *w2b) {
    const int h = threadIdx.x;
    if (h >= POLICY_H) return;
    for (int k = 0; k < MLP_FPAD; ++k)
        w1b[h * MLP_FPAD + k] = k < POLICY_F ? f2bf(theta[OFF_W1 + h * POLICY_F + k]) : (uint16_t)0;
    w2b[h] = f2bf(theta[OFF_W2 + h]);
}

// bf16 B operand of layer 1 for row s of X (fp32 rows of stride ld, features
// in columns 0..POLICY_F-1): lane holds features 4 (lane / 16) + j
__device__ __forceinline__ bf16x4 load_xT(const float *X, int ld, long long s, long long N, int kq) {
    bf16x4 xT;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = 4 * kq + j;
        xT[j] = (short)((s < N && k < POLICY_F) ? f2bf(X[s * ld + k]) : (uint16_t)0);
    }
    return xT;
}

// y[s] for N rows of X
__global__ __launch_bounds__(256) void mlp_forward_kernel(PolicyDev P, const float *X, int ld, long long N, float *y) {
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    for (long long tile = (long long)blockIdx.x * 4 + wave; tile * 16 < N; tile += (long long)gridDim.x * 4) {
        const long long s = tile * 16 + row;
        const bf16x4 xT = load_xT(X, ld, s, N, kq);
        const f32x4 acc = mlp_tile(P, xT, lane, nullptr);
        if (row == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long ss = tile * 16 + 4 * kq + r;
                if (ss < N) y[ss] = acc[r] + *P.b2;
            }
        }
    }
}

__device__ __forceinline__ float sum16(float v) {  // sum over the 16 lanes sharing lane / 16
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Gradients of the mean squared error over N rows (added into grad[449] and
// *loss).  The rounding of weights and activations to bf16 is treated as the
// identity in the backward pass (straight-through).
__global__ __launch_bounds__(256) void mlp_grad_kernel(PolicyDev P, const float *X, int ld, const float *T,
                                                       int ldt, long long N, float *grad, float *loss) {
    __shared__ float g[POLICY_NP + 1];
    __shared__ float sdy[4][16];
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    for (int i = threadIdx.x; i <= POLICY_NP; i += blockDim.x) g[i] = 0.f;
    __syncthreads();
    const float invN = 1.0f / (float)N;
    for (long long tile = (long long)blockIdx.x * 4 + wave; tile * 16 < N; tile += (long long)gridDim.x * 4) {
        const long long s = tile * 16 + row;
        const bool valid = s < N;
        const bf16x4 xT = load_xT(X, ld, s, N, kq);
        float pre[16];
        const f32x4 acc = mlp_tile(P, xT, lane, pre);
        float lsum = 0.f;
        if (row == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long ss = tile * 16 + 4 * kq + r;
                float dy = 0.f;
                if (ss < N) {
                    const float e = acc[r] + *P.b2 - T[ss * ldt];
                    dy = 2.f * e * invN;
                    lsum += e * e * invN;
                }
                sdy[wave][4 * kq + r] = dy;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        const float dyv = sdy[wave][row];
        float x[POLICY_F];
#pragma unroll
        for (int k = 0; k < POLICY_F; ++k) x[k] = valid ? bf2f(f2bf(X[s * ld + k])) : 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int h = 16 * t + 4 * kq + r;
                const float p = pre[4 * t + r];
                const float hb = bf2f(f2bf(p > 0.f ? p : 0.f));
                const float dpre = p > 0.f ? dyv * bf2f(P.w2[h]) : 0.f;
                const float gw2 = sum16(dyv * hb);
                const float gb1 = sum16(dpre);
                float gw1[POLICY_F];
#pragma unroll
                for (int k = 0; k < POLICY_F; ++k) gw1[k] = sum16(dpre * x[k]);
                if (row == 0) {
                    atomicAdd(&g[OFF_W2 + h], gw2);
                    atomicAdd(&g[OFF_B1 + h], gb1);
#pragma unroll
                    for (int k = 0; k < POLICY_F; ++k) atomicAdd(&g[OFF_W1 + h * POLICY_F + k], gw1[k]);
                }
            }
        }
        const float gb2 = sum16(dyv);
        if (lane == 0) {
            atomicAdd(&g[OFF_B2], gb2);
        }
        if (row == 0) atomicAdd(&g[POLICY_NP], lsum);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    }
    __syncthreads();
    for (int i = threadIdx.x; i < POLICY_NP; i += blockDim.x) atomicAdd(&grad[i], g[i]);
    if (threadIdx.x == 0) atomicAdd(loss, g[POLICY_NP]);
}

__global__ void fill_kernel(float *p, int n, float v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Adam (Kingma & Ba) on the fp32 master parameters.
__global__ void adam_kernel(float *theta, float *m, float *v, const float *grad, float lr, float beta1,
                            float beta2, float eps, int step) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= POLICY_NP) return;
    const float gi = grad[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.f - powf(beta1, (float)step));
    const float vh = vi / (1.f - powf(beta2, (float)step));
    theta[i] -= lr * mh / (sqrtf(vh) + eps);
}

hipError_t launch_policy_round(const float *theta, uint16_t *w1b, uint16_t *w2b, hipStream_t st) {
    hipLaunchKernelGGL(policy_round_kernel, dim3(1), dim3(64), 0, st, theta, w1b, w2b);
    return hipGetLastError();
}
hipError_t launch_mlp_forward(const PolicyDev &P, const float *X, int ld, long long N, float *y, hipStream_t st) {
    long long tiles = (N + 15) / 16;
    int blocks = (int)((tiles + 3) / 4);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks), dim3(256), 0, st, P, X, ld, N, y);
    return hipGetLastError();
}
hipError_t launch_mlp_grad(const PolicyDev &P, const float *X, int ld, const float *T, int ldt, long long N,
                           float *grad, float *loss, hipStream_t st) {
    hipLaunchKernelGGL(fill_kernel, dim3(2), dim3(256), 0, st, grad, POLICY_NP, 0.f);
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, st, loss, 1, 0.f);
    long long tiles = (N + 15) / 16;
    int blocks = (int)((tiles + 3) / 4);
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(blocks), dim3(256), 0, st, P, X, ld, T, ldt, N, grad, loss);
    return hipGetLastError();
}
hipError_t launch_adam(float *theta, float *m, float *v, const float *grad, float lr, int step, hipStream_t st) {
    hipLaunchKernelGGL(adam_kernel, dim3(2), dim3(256), 0, st, theta, m, v, grad, lr, 0.9f, 0.999f, 1e-8f, step);
    return hipGetLastError();
}
hipError_t launch_fill(float *p, int n, float v, hipStream_t st) {
    hipLaunchKernelGGL(fill_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace cubics
