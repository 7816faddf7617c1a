// Matrix-core helpers shared by the separable map (kde_sep.hip) and the
// matrix-core VJP (kde_vjp_mfma.hip): 8-element FP16 / BF16 operand words and
// the 32 x 32 x 16 MFMA.
//
// Operand word: 8 consecutive values along the contraction (k) axis, 16 bytes.
// v_mfma_f32_32x32x16_{f16,bf16}: lane l supplies A[l % 32][8 (l / 32) .. +8] and
// B[8 (l / 32) .. +8][l % 32]; accumulator register r of lane l holds
// C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
#pragma once

#include <hip/hip_runtime.h>

namespace kde {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Rounds 8 floats to FP16 or BF16 (nearest even) and packs them into a word.
template <bool kBf16>
__device__ __forceinline__ uint4 pack8(const float (&v)[8]) {
    uint4 r;
    if constexpr (kBf16) {
        bf16x8 h;
#pragma unroll
        for (int k = 0; k < 8; ++k) h[k] = (__bf16)v[k];
        r = __builtin_bit_cast(uint4, h);
    } else {
        half8 h;
#pragma unroll
        for (int k = 0; k < 8; ++k) h[k] = (_Float16)v[k];
        r = __builtin_bit_cast(uint4, h);
    }
    return r;
}

// Residual v - (float)round16(v), for the lo half of a split.
template <bool kBf16>
__device__ __forceinline__ void residual8(const float (&v)[8], uint4 hi, float (&lo)[8]) {
    if constexpr (kBf16) {
        const bf16x8 h = __builtin_bit_cast(bf16x8, hi);
#pragma unroll
        for (int k = 0; k < 8; ++k) lo[k] = v[k] - (float)h[k];
    } else {
        const half8 h = __builtin_bit_cast(half8, hi);
#pragma unroll
        for (int k = 0; k < 8; ++k) lo[k] = v[k] - (float)h[k];
    }
}

template <bool kBf16>
__device__ __forceinline__ f32x16 mfma(uint4 a, uint4 b, f32x16 c) {
    if constexpr (kBf16)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c,
                                                      0, 0, 0);
}

}  // namespace kde
