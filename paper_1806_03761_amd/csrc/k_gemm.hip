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
// Cooperative load of a TK x TW tile (rows of TW + 1 in LDS): entry (kk, ww) = src[off_w[ww] + off_k[kk]] (zero where
// either offset is negative), threads striding over the TK * TW entries.  Every load
// reads a valid address (entry 0 of the operand for padding) and all are issued before
// the first conversion, so they overlap instead of each waiting on its own.
template <int TK, int TW, Arith AR>
__device__ __forceinline__ void tile_load(typename ArithT<AR>::In* dst, const long long* off_w,
                                          const long long* off_k, int f32, const double* srcd,
                                          const float* srcf, int tid) {
    using In = typename ArithT<AR>::In;
    constexpr int NE = TK * TW, NI = (NE + 255) / 256;
    long long o[NI];
    bool ok[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = tid + 256 * i;
        const bool in = NE % 256 == 0 || e < NE;
        const long long ow = in ? off_w[e % TW] : -1, ok_ = in ? off_k[e / TW] : -1;
        ok[i] = ow >= 0 && ok_ >= 0;
        o[i] = ok[i] ? ow + ok_ : 0;
    }
    In v[NI];
    if (f32) {
        float x[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) x[i] = srcf[o[i]];
#pragma unroll
        for (int i = 0; i < NI; ++i) v[i] = ok[i] ? to_in<AR>((double)x[i]) : In(0);
    } else {
        double x[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) x[i] = srcd[o[i]];
#pragma unroll
        for (int i = 0; i < NI; ++i) v[i] = ok[i] ? to_in<AR>(x[i]) : In(0);
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = tid + 256 * i;
        if (NE % 256 == 0 || e < NE) dst[(e / TW) * (TW + 1) + e % TW] = v[i];   // rows padded by one
    }
}

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
        // single order is coalesced for all of them); B tile likewise.  All loads of a
        // tile are issued before any is used.
        tile_load<TK, TM, AR>(&As[0][0], aoff_m, aoff_k, g.a_f32, Ab, Af, tid);
        tile_load<TK, TN, AR>(&Bs[0][0], boff_n, boff_k, g.b_f32, Bb, Bf, tid);
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
static GemmArgs transposed(const GemmArgs& g) {
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
    // 14: row kernel; 15: row kernel on the transposed product (each falls back to the
    // heuristic tile when the shape does not fit it)
    if (tile == 14 && gemm_rows_fits(g)) return launch_gemm_rows(g, ar, st);
    if (tile == 15) {
        const GemmArgs t = transposed(g);
        if (gemm_rows_fits(t)) return launch_gemm_rows(t, ar, st);
    }
    if (tile >= 14) tile = 0;
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
        case 8: return launch_t<128, 16, 16>(g, ar, st);
        case 9: return launch_t<256, 16, 16>(g, ar, st);
        case 10: return launch_t<16, 128, 16>(g, ar, st);
        case 11: return launch_t<16, 256, 16>(g, ar, st);
        case 12: return launch_t<128, 32, 16>(g, ar, st);
        case 13: return launch_t<32, 128, 16>(g, ar, st);
        default: return launch_t<64, 64, 16>(g, ar, st);
    }
}

}  // namespace peps
