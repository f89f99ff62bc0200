// bf16 limbs of FP64 operands for the split-precision MFMA forms: every
// operand x is split into bf16 limbs x = x0 + x1 (+ x2) by round-to-nearest
// on the successive residuals, and a product a b is formed from the limb
// products of the same order of magnitude (two limbs: a0 b0 + a0 b1 + a1 b0;
// three limbs add a1 b1 + a0 b2 + a2 b0).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pufe {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two FP32 values -> a packed pair of bf16 (low half: the first), rounded to
// nearest even by the hardware conversion (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
    const f32x2 f = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));
}

// Limbs of two values x0, x1 as packed bf16 pairs: the first limb from the
// FP64 values, the others from the residuals, which are exact in FP64 and
// carried on in FP32 (their FP32 rounding, below 2^-32 |x|, is far under the
// last limb).
template <int NL>
__device__ __forceinline__ void split_limbs2(double x0, double x1, uint32_t *h) {
    h[0] = bf16_pair((float)x0, (float)x1);
    float r0 = (float)(x0 - (double)__uint_as_float(h[0] << 16));
    float r1 = (float)(x1 - (double)__uint_as_float(h[0] & 0xffff0000u));
#pragma unroll
    for (int j = 1; j < NL; ++j) {
        h[j] = bf16_pair(r0, r1);
        r0 -= __uint_as_float(h[j] << 16);
        r1 -= __uint_as_float(h[j] & 0xffff0000u);
    }
}

// Limbs of eight consecutive values as one bf16x8 per limb (the operand of
// one lane of a 16x16x32 bf16 MFMA).
template <int NL>
__device__ __forceinline__ void split_limbs8(const double *x, bf16x8 *h) {
    uint32_t w[4][NL];
#pragma unroll
    for (int p = 0; p < 4; ++p) split_limbs2<NL>(x[2 * p], x[2 * p + 1], w[p]);
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const uint4 v = make_uint4(w[0][j], w[1][j], w[2][j], w[3][j]);
        h[j] = __builtin_bit_cast(bf16x8, v);
    }
}

// One K-block of a split product: acc += sum over the kept limb products of
// A and B, smallest first.
template <int NL>
__device__ __forceinline__ f32x4 mfma_limbs(const bf16x8 *A, const bf16x8 *B, f32x4 acc) {
    if (NL == 3) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2], B[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[1], acc, 0, 0, 0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[0], acc, 0, 0, 0);
    return acc;
}

}  // namespace pufe
