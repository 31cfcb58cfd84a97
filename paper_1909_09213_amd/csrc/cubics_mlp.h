// Branching-policy network on CDNA4 matrix cores: a 2-layer MLP
// (F inputs zero-padded to 16, 64 hidden ReLU units, 1 output) with BF16
// weights and activations and FP32 accumulation, evaluated 16 rows at a time
// with v_mfma_f32_16x16x16_bf16.
//
// Layer 1 is computed transposed, D1 = W1 * X^T (rows of D1 = hidden units,
// columns = the 16 input rows), so that each lane's accumulator already holds
// the A-operand layout layer 2 needs: for the 16x16x16 MFMA, lane l supplies
// A[l % 16][4 (l / 16) + j], B[4 (l / 16) + j][l % 16] and receives
// D[4 (l / 16) + r][l % 16] (j, r = 0..3).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cubics_internal.h"

namespace cubics {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MLP_FPAD = 16;  // padded input width (the MFMA K of layer 1)

// fp32 -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// One 16-row tile.  xT: this lane's B operand of layer 1, i.e. the bf16 bits
// of X[row = lane % 16][feature = 4 (lane / 16) + j].  Returns layer 2's
// accumulator: lanes with lane % 16 == 0 hold y (without b2) of rows
// 4 (lane / 16) + r.  If pre != nullptr, pre[4 t + r] receives the layer-1
// pre-activation (with b1) of hidden unit 16 t + 4 (lane / 16) + r for row
// lane % 16.
// COMPACT: keep one hidden tile in flight at a time (fewer live registers,
// for callers embedded in a larger kernel).
template <bool COMPACT = false>
__device__ __forceinline__ f32x4 mlp_tile(const PolicyDev &P, bf16x4 xT, int lane, float *pre) {
    const int col = lane & 15, kq = lane >> 4;
    f32x4 acc2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll(COMPACT ? 1 : 4)
    for (int t = 0; t < 4; ++t) {
        bf16x4 a1;
        const uint16_t *w = P.w1 + (size_t)(16 * t + col) * MLP_FPAD + 4 * kq;
#pragma unroll
        for (int j = 0; j < 4; ++j) a1[j] = (short)w[j];
        const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
        const f32x4 d1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, xT, zero, 0, 0, 0);
        bf16x4 a2, b2;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int h = 16 * t + 4 * kq + r;
            const float p = d1[r] + P.b1[h];
            if (pre) pre[4 * t + r] = p;
            a2[r] = (short)f2bf(p > 0.f ? p : 0.f);
            b2[r] = (short)(col == 0 ? P.w2[h] : (uint16_t)0);
        }
        acc2 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, b2, acc2, 0, 0, 0);
    }
    return acc2;
}

}  // namespace cubics
