// Shared declarations of the PEPS HIP library (host and device side).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace peps {

// Compute type of a GEMM launch.
enum class Arith : int { F64 = 0, F32 = 1, BF16 = 2 };

// A linear index i split as (i / inner, i % inner), each part with its own stride.
struct Idx2 {
    int inner;
    long long s_outer, s_inner;
};

// Gather of an operand by spin: base += ((sel[b*sel_bs + sel_off] ^ flip) & 1) * slice.
struct Gather {
    const int8_t* sel;   // nullptr: no gather
    long long sel_bs;
    int flip;
    long long slice;
};

// Batched C(b) = alpha * A(b) x B(b) (+ beta * C(b)) on strided multi-index operands.
// Element offsets (in elements of the operand's storage type):
//   A(m,k) = A + b*a_bs + gather + off(m; am) + off(k; ak)
//   B(k,n) = B + b*b_bs + gather + off(k; bk) + off(n; bn)
//   C(m,n) = C + b*c_bs + gather + off(m; cm) + off(n; cn)
struct GemmArgs {
    int M, N, K, batch;
    Idx2 am, ak, bk, bn, cm, cn;
    long long a_bs, b_bs, c_bs;
    Gather ga, gb, gc;
    const double* A;
    const double* B;
    double* C;
    double alpha, beta;
};

__host__ __device__ inline long long idx_off(const Idx2& x, int i) {
    return (long long)(i / x.inner) * x.s_outer + (long long)(i % x.inner) * x.s_inner;
}

__device__ inline long long gather_off(const Gather& g, int b) {
    if (!g.sel) return 0;
    return (long long)((g.sel[(long long)b * g.sel_bs] ^ g.flip) & 1) * g.slice;
}

}  // namespace peps
