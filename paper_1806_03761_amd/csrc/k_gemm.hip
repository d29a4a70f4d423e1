// Batched strided multi-index GEMM: the one contraction primitive of the library.
//
// Every contraction of the path (boundary apply, single- and two-row sandwich
// steps, environment tensors) is written as C = A x B where each of M, N, K is a
// pair of tensor legs with its own strides, so no permutation is ever
// materialised.  Operand tiles are staged through LDS in the compute type
// (float64, float32, or bfloat16-rounded with float32 accumulation).
#include "common.h"
#include "kernels.h"

namespace peps {

template <Arith AR> struct ArithT;
template <> struct ArithT<Arith::F64> { using In = double; using Acc = double; };
template <> struct ArithT<Arith::F32> { using In = float; using Acc = float; };
template <> struct ArithT<Arith::BF16> { using In = float; using Acc = float; };

template <Arith AR>
__device__ inline typename ArithT<AR>::In to_in(double x) {
    if constexpr (AR == Arith::F64) {
        return x;
    } else if constexpr (AR == Arith::F32) {
        return (float)x;
    } else {
        // round to bfloat16 (nearest-even) and back to float32: the product of two
        // such values is exact in float32, as in a bf16 matrix core with fp32 accumulation
        return __bfloat162float(__float2bfloat16((float)x));
    }
}

// Row kernel for skinny products (N <= 64, K <= kRowsMaxK): the TPR threads of a row own
// CPT consecutive columns each and accumulate them in registers, reading the A row
// straight from memory with KC loads in flight (k in order, as in the tiled kernel, so
// the results are identical); B is staged once per block and C leaves through LDS so
// that consecutive threads store consecutive columns.
static constexpr int kRowsMaxK = 64;

template <int CPT, int TPR, Arith AR>
__global__ __launch_bounds__(256) void k_gemm_rows(GemmArgs g, int blocks_m) {
    using In = typename ArithT<AR>::In;
    using Acc = typename ArithT<AR>::Acc;
    constexpr int KC = 16;               // A loads in flight per thread
    constexpr int RPB = 256 / TPR;       // rows per block
    constexpr int NC = CPT * TPR;        // columns per block
    __shared__ In Bs[kRowsMaxK][NC];
    __shared__ Acc Cs[RPB][NC + 1];
    __shared__ long long koff[kRowsMaxK], coff_n[NC], coff_m[RPB];
    const int b = blockIdx.x / blocks_m, m0 = (blockIdx.x % blocks_m) * RPB, tid = threadIdx.x;
    if (b >= g.batch) return;
    const long long a0 = (long long)b * g.a_bs + gather_off(g.ga, b);
    const long long b0 = (long long)b * g.b_bs + gather_off(g.gb, b);
    const long long c0 = (long long)b * g.c_bs + gather_off(g.gc, b);
    // B staged in rounds of 8 loads per thread, each round's loads issued together
    for (int e0 = 0; e0 < g.K * NC; e0 += 8 * 256) {
        long long o[8];
        bool ok[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = e0 + tid + 256 * i, k = e / NC, n = e % NC;
            ok[i] = e < g.K * NC && n < g.N;
            o[i] = b0 + (ok[i] ? idx_off(g.bk, k) + idx_off(g.bn, n) : 0);
        }
        In v[8];
        if (g.b_f32) {
            float x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = reinterpret_cast<const float*>(g.B)[o[i]];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = ok[i] ? to_in<AR>((double)x[i]) : In(0);
        } else {
            double x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = g.B[o[i]];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = ok[i] ? to_in<AR>(x[i]) : In(0);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = e0 + tid + 256 * i;
            if (e < g.K * NC) Bs[e / NC][e % NC] = v[i];
        }
    }
    for (int k = tid; k < g.K; k += 256) koff[k] = idx_off(g.ak, k);
    for (int n = tid; n < NC; n += 256) coff_n[n] = n < g.N ? idx_off(g.cn, n) : 0;
    const int r = tid / TPR, cg = (tid % TPR) * CPT;
    const int m = m0 + r;
    if (tid < RPB) coff_m[tid] = m0 + tid < g.M ? idx_off(g.cm, m0 + tid) : 0;
    __syncthreads();
    Acc acc[CPT];
#pragma unroll
    for (int n = 0; n < CPT; ++n) acc[n] = Acc(0);
    if (m < g.M) {
        const long long am = a0 + idx_off(g.am, m);
        const float* Af = reinterpret_cast<const float*>(g.A) + am;
        const double* Ad = g.A + am;
        for (int k0 = 0; k0 < g.K; k0 += KC) {
            In av[KC];
            if (g.a_f32) {
                float x[KC];
#pragma unroll
                for (int u = 0; u < KC; ++u) x[u] = Af[koff[k0 + u < g.K ? k0 + u : 0]];
#pragma unroll
                for (int u = 0; u < KC; ++u) av[u] = k0 + u < g.K ? to_in<AR>((double)x[u]) : In(0);
            } else {
                double x[KC];
#pragma unroll
                for (int u = 0; u < KC; ++u) x[u] = Ad[koff[k0 + u < g.K ? k0 + u : 0]];
#pragma unroll
                for (int u = 0; u < KC; ++u) av[u] = k0 + u < g.K ? to_in<AR>(x[u]) : In(0);
            }
#pragma unroll
            for (int u = 0; u < KC; ++u) {
                if (k0 + u >= g.K) break;
#pragma unroll
                for (int n = 0; n < CPT; ++n) acc[n] = fma((Acc)av[u], (Acc)Bs[k0 + u][cg + n], acc[n]);
            }
        }
    }
#pragma unroll
    for (int n = 0; n < CPT; ++n) Cs[r][cg + n] = acc[n];
    __syncthreads();
    float* Cf = reinterpret_cast<float*>(g.C) + c0;
    double* Cd = g.C + c0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int e = tid + 256 * j, rr = e / NC, n = e % NC;
        if (n >= g.N || m0 + rr >= g.M) continue;
        const long long o = coff_m[rr] + coff_n[n];
        double v = g.alpha * (double)Cs[rr][n];
        if (g.c_f32) {
            if (g.beta != 0.0) v += g.beta * (double)Cf[o];
            Cf[o] = (float)v;
        } else {
            if (g.beta != 0.0) v += g.beta * Cd[o];
            Cd[o] = v;
        }
    }
}

template <int CPT, int TPR>
static hipError_t launch_rows_t(const GemmArgs& g, Arith ar, hipStream_t st) {
    constexpr int RPB = 256 / TPR;
    const int bm = (g.M + RPB - 1) / RPB;
    const long long blocks = (long long)bm * g.batch;
    if (blocks == 0) return hipSuccess;
    switch (ar) {
        case Arith::F64: hipLaunchKernelGGL((k_gemm_rows<CPT, TPR, Arith::F64>), dim3((unsigned)blocks), dim3(256), 0, st, g, bm); break;
        case Arith::F32: hipLaunchKernelGGL((k_gemm_rows<CPT, TPR, Arith::F32>), dim3((unsigned)blocks), dim3(256), 0, st, g, bm); break;
        case Arith::BF16: hipLaunchKernelGGL((k_gemm_rows<CPT, TPR, Arith::BF16>), dim3((unsigned)blocks), dim3(256), 0, st, g, bm); break;
    }
    return hipGetLastError();
}

bool gemm_rows_fits(const GemmArgs& g) { return g.N <= 64 && g.K <= kRowsMaxK; }

hipError_t launch_gemm_rows(const GemmArgs& g, Arith ar, hipStream_t st) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    if (!gemm_rows_fits(g)) return hipErrorInvalidValue;
    if (g.N <= 4) return launch_rows_t<4, 1>(g, ar, st);
    if (g.N <= 8) return launch_rows_t<8, 1>(g, ar, st);
    if (g.N <= 16) return launch_rows_t<16, 1>(g, ar, st);
    if (g.N <= 32) return launch_rows_t<16, 2>(g, ar, st);
    return launch_rows_t<16, 4>(g, ar, st);
}

// the same product as C^T = B^T A^T (M and N, A and B swapped)
GemmArgs gemm_transposed(const GemmArgs& g) {
    GemmArgs t = g;
    t.M = g.N; t.N = g.M;
    t.A = g.B; t.B = g.A;
    t.am = g.bn; t.ak = g.bk; t.bk = g.ak; t.bn = g.am;
    t.cm = g.cn; t.cn = g.cm;
    t.a_bs = g.b_bs; t.b_bs = g.a_bs;
    t.ga = g.gb; t.gb = g.ga;
    t.a_f32 = g.b_f32; t.b_f32 = g.a_f32;
    return t;
}

hipError_t launch_gemm(const GemmArgs& g, Arith ar, hipStream_t st, int tile) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    // 1..kMfmaTiles: matrix-core tiles; kMfmaTiles + 1: row kernel; kMfmaTiles + 2: row kernel
    // on the transposed product (each falls back to the heuristic tile when the shape does
    // not fit it).  Every form sums the products of an output in ascending k with one
    // rounding per product (a 16x16x4 MFMA adds its four products in k order, like a chain
    // of fma), so all of them give the same results.
    if (tile == kMfmaTiles + 1 && gemm_rows_fits(g)) return launch_gemm_rows(g, ar, st);
    if (tile == kMfmaTiles + 2) {
        const GemmArgs t = gemm_transposed(g);
        if (gemm_rows_fits(t)) return launch_gemm_rows(t, ar, st);
    }
    return launch_mgemm(g, ar, st, tile > kMfmaTiles ? 0 : tile);
}

}  // namespace peps
