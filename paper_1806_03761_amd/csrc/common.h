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
    // storage type of each operand: 0 = float64, 1 = float32 (the pointer then addresses
    // floats and every offset above counts floats)
    int a_f32, b_f32, c_f32;
    // optional per-sample predicate: sample b is skipped (C left untouched) when
    // skip[b * skip_bs] == 0
    const int8_t* skip = nullptr;
    long long skip_bs = 0;
};

__host__ __device__ inline long long idx_off(const Idx2& x, int i) {
    return (long long)(i / x.inner) * x.s_outer + (long long)(i % x.inner) * x.s_inner;
}

__device__ inline long long gather_off(const Gather& g, int b) {
    if (!g.sel) return 0;
    return (long long)((g.sel[(long long)b * g.sel_bs] ^ g.flip) & 1) * g.slice;
}

// p[off] when ok, else zero, read without a branch: the load always goes to p[ok ? off : 0]
// (p[0] must be readable), so a run of these issues back to back and waits once, where a
// guarded load compiles to a branch that waits for its own result before the next one.
template <class T>
__device__ __forceinline__ T ld_or0(bool ok, const T* p, long long off) {
    const T v = p[ok ? off : 0];
    return ok ? v : T(0);
}

// dst[i] = src[i] for i in [0, n), by threads tid, tid + nth, ...: each thread issues its
// loads in groups of 8 before storing them, instead of a load, wait and store per
// element (a strided loop of unknown trip count is not unrolled by the compiler).
__device__ inline void copy_strided(double* dst, const double* src, long long n, int tid, int nth) {
    for (long long b0 = 0; b0 < n; b0 += 8LL * nth) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const long long i = b0 + tid + (long long)u * nth;
            v[u] = src[i < n ? i : 0];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const long long i = b0 + tid + (long long)u * nth;
            if (i < n) dst[i] = v[u];
        }
    }
}

// One DPP lane permutation of a double (both 32-bit halves moved alike).  Controls used:
// 0xB1 swaps lanes 2i <-> 2i+1, 0x4E swaps pairs within a quad, 0x141 mirrors each half
// row of 8 lanes, 0x140 mirrors each row of 16 lanes.
template <int CTRL>
__device__ inline double dpp_perm(double x) {
    const long long b = __double_as_longlong(x);
    // every control used here gives each lane a valid source lane, so no "old" value is
    // ever kept: the plain DPP move needs no copy of the destination first
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// v plus the value of lane l ^ 16 (l ^ 32): v_permlane16_swap (32_swap) with both operands
// v hands every lane its own row's (half's) value and the partner row's (half's) value at
// the same position, a plain VALU exchange.  Their sum is the same in every lane of the
// pair, and equal to v + v[l ^ 16] since the addition commutes.
__device__ inline double add_xor16(double v) {
    const long long b = __double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    return __longlong_as_double(((long long)hi[0] << 32) | lo[0]) +
           __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}
__device__ inline double add_xor32(double v) {
    const long long b = __double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    return __longlong_as_double(((long long)hi[0] << 32) | lo[0]) +
           __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

// Sum over aligned groups of `width` lanes (a power of two up to 64); every lane of a
// group gets the bitwise-same total.  Inside a row of 16 lanes the partner values come
// from DPP permutations, across rows and wave halves from the permlane swaps: all VALU,
// no LDS round trip.  All lanes of a group must be active.
__device__ inline double lane_group_sum(double v, int width) {
    if (width >= 2) v += dpp_perm<0xB1>(v);
    if (width >= 4) v += dpp_perm<0x4E>(v);
    if (width >= 8) v += dpp_perm<0x141>(v);
    if (width >= 16) v += dpp_perm<0x140>(v);
    if (width >= 32) v = add_xor16(v);
    if (width >= 64) v = add_xor32(v);
    return v;
}

}  // namespace peps
