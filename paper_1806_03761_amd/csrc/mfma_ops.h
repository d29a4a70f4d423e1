// Matrix-core operand types and the 16x16x4 MFMA step shared by the contraction kernels.
//
// A 16x16x4 MFMA adds its four products into each output in k order with one rounding per
// product, like a chain of fma, so a sum split over MFMAs that take k = 4s .. 4s+3 in
// step s keeps the ascending order of a plain fma loop: every kernel built on these
// gives the same bits for the same operands and k order.
#pragma once

#include "common.h"

namespace peps {

typedef double mf64x4 __attribute__((ext_vector_type(4)));
typedef float mf32x4 __attribute__((ext_vector_type(4)));

template <Arith AR> struct MT;
template <> struct MT<Arith::F64> { using In = double; using Acc = mf64x4; };
template <> struct MT<Arith::F32> { using In = float; using Acc = mf32x4; };
template <> struct MT<Arith::BF16> { using In = float; using Acc = mf32x4; };

template <Arith AR>
__device__ __forceinline__ typename MT<AR>::In to_mt(double x) {
    if constexpr (AR == Arith::F64) {
        return x;
    } else if constexpr (AR == Arith::F32) {
        return (float)x;
    } else {
        // operands rounded to bfloat16 (nearest-even); their products are exact in float32
        return __bfloat162float(__float2bfloat16((float)x));
    }
}

template <Arith AR>
__device__ __forceinline__ typename MT<AR>::Acc mfma(typename MT<AR>::In a, typename MT<AR>::In b,
                                                     typename MT<AR>::Acc c) {
    if constexpr (AR == Arith::F64) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

}  // namespace peps
