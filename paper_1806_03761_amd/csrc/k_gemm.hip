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

// WG of 256 threads as a 16x16 grid; each thread owns a (TM/16) x (TN/16) micro-tile.
template <int TM, int TN, int TK, Arith AR>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g, int tiles_m, int tiles_n) {
    using In = typename ArithT<AR>::In;
    using Acc = typename ArithT<AR>::Acc;
    constexpr int RM = TM / 16, RN = TN / 16;
    __shared__ In As[TK][TM + 1];
    __shared__ In Bs[TK][TN + 1];
    __shared__ long long aoff_m[TM], boff_n[TN], coff_m[TM], coff_n[TN];
    __shared__ long long aoff_k[TK], boff_k[TK];

    const int tiles = tiles_m * tiles_n;
    const long long blk = blockIdx.x;
    const int b = (int)(blk / tiles);
    const int t = (int)(blk % tiles);
    const int m0 = (t / tiles_n) * TM;
    const int n0 = (t % tiles_n) * TN;
    const int tid = threadIdx.x;
    if (b >= g.batch) return;

    // element offsets of this batch entry (in the operand's own storage type)
    const long long a0 = (long long)b * g.a_bs + gather_off(g.ga, b);
    const long long b0 = (long long)b * g.b_bs + gather_off(g.gb, b);
    const long long c0 = (long long)b * g.c_bs + gather_off(g.gc, b);
    const double* Ab = g.A + a0;
    const double* Bb = g.B + b0;
    double* Cb = g.C + c0;
    const float* Af = reinterpret_cast<const float*>(g.A) + a0;
    const float* Bf = reinterpret_cast<const float*>(g.B) + b0;
    float* Cf = reinterpret_cast<float*>(g.C) + c0;

    for (int i = tid; i < TM; i += 256) {
        int m = m0 + i;
        aoff_m[i] = m < g.M ? idx_off(g.am, m) : -1;
        coff_m[i] = m < g.M ? idx_off(g.cm, m) : -1;
    }
    for (int i = tid; i < TN; i += 256) {
        int n = n0 + i;
        boff_n[i] = n < g.N ? idx_off(g.bn, n) : -1;
        coff_n[i] = n < g.N ? idx_off(g.cn, n) : -1;
    }

    Acc acc[RM][RN];
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) acc[i][j] = Acc(0);

    const int tx = tid % 16, ty = tid / 16;
    for (int k0 = 0; k0 < g.K; k0 += TK) {
        __syncthreads();
        for (int i = tid; i < TK; i += 256) {
            int k = k0 + i;
            aoff_k[i] = k < g.K ? idx_off(g.ak, k) : -1;
            boff_k[i] = k < g.K ? idx_off(g.bk, k) : -1;
        }
        __syncthreads();
        // A tile: TK x TM, consecutive threads walk m (operand layouts vary, so no
        // single order is coalesced for all of them)
        for (int e = tid; e < TK * TM; e += 256) {
            int kk = e / TM, mm = e % TM;
            long long om = aoff_m[mm], ok = aoff_k[kk];
            As[kk][mm] = (om >= 0 && ok >= 0) ? to_in<AR>(g.a_f32 ? (double)Af[om + ok] : Ab[om + ok]) : In(0);
        }
        for (int e = tid; e < TK * TN; e += 256) {
            int kk = e / TN, nn = e % TN;
            long long on = boff_n[nn], ok = boff_k[kk];
            Bs[kk][nn] = (on >= 0 && ok >= 0) ? to_in<AR>(g.b_f32 ? (double)Bf[on + ok] : Bb[on + ok]) : In(0);
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < TK; ++kk) {
            Acc av[RM], bv[RN];
#pragma unroll
            for (int i = 0; i < RM; ++i) av[i] = (Acc)As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < RN; ++j) bv[j] = (Acc)Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int j = 0; j < RN; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < RM; ++i) {
        long long om = coff_m[ty + 16 * i];
        if (om < 0) continue;
#pragma unroll
        for (int j = 0; j < RN; ++j) {
            long long on = coff_n[tx + 16 * j];
            if (on < 0) continue;
            double v = g.alpha * (double)acc[i][j];
            if (g.c_f32) {
                if (g.beta != 0.0) v += g.beta * (double)Cf[om + on];
                Cf[om + on] = (float)v;
            } else {
                if (g.beta != 0.0) v += g.beta * Cb[om + on];
                Cb[om + on] = v;
            }
        }
    }
}

template <int TM, int TN, int TK>
static hipError_t launch_t(const GemmArgs& g, Arith ar, hipStream_t st) {
    int tm = (g.M + TM - 1) / TM, tn = (g.N + TN - 1) / TN;
    long long blocks = (long long)tm * tn * g.batch;
    if (blocks == 0) return hipSuccess;
    dim3 grid((unsigned)blocks), block(256);
    switch (ar) {
        case Arith::F64: hipLaunchKernelGGL((k_gemm<TM, TN, TK, Arith::F64>), grid, block, 0, st, g, tm, tn); break;
        case Arith::F32: hipLaunchKernelGGL((k_gemm<TM, TN, TK, Arith::F32>), grid, block, 0, st, g, tm, tn); break;
        case Arith::BF16: hipLaunchKernelGGL((k_gemm<TM, TN, TK, Arith::BF16>), grid, block, 0, st, g, tm, tn); break;
    }
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& g, Arith ar, hipStream_t st, int tile) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    if (tile <= 0 || tile > kGemmTiles) {
        // heuristic: smallest tile that covers small problems
        if (g.M <= 16 && g.N <= 16) tile = 1;
        else if (g.M <= 32 && g.N <= 32) tile = 2;
        else if (g.N <= 16) tile = 3;
        else if (g.M <= 16) tile = 4;
        else tile = 5;
    }
    switch (tile) {
        case 1: return launch_t<16, 16, 16>(g, ar, st);
        case 2: return launch_t<32, 32, 16>(g, ar, st);
        case 3: return launch_t<64, 16, 16>(g, ar, st);
        case 4: return launch_t<16, 64, 16>(g, ar, st);
        case 5: return launch_t<64, 64, 16>(g, ar, st);
        case 6: return launch_t<32, 16, 32>(g, ar, st);
        case 7: return launch_t<16, 32, 32>(g, ar, st);
        default: return launch_t<64, 64, 16>(g, ar, st);
    }
}

}  // namespace peps
