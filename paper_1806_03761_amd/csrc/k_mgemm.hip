// Batched strided multi-index GEMM on the matrix cores (the contraction primitive of
// the boundary apply, the single- and two-row sandwich steps and the environment
// tensors).
//
// C(b) = A(b) x B(b) with each of M, N, K a pair of tensor legs with its own strides
// (no permutation is materialised), an optional spin-selected operand slice, and an
// optional per-sample predicate that skips samples whose result is not needed.
//
// A workgroup of four waves computes a TM x TN tile; wave (wm, wn) owns BM x BN blocks
// of 16 x 16, each accumulated by 16x16x4 MFMAs (float64: v_mfma_f64_16x16x4f64,
// float32: v_mfma_f32_16x16x4f32).  Operand tiles of TK k values (16, or 12, 32, 36 where
// they divide K) are staged through LDS in the compute type; the next stage's global
// loads are issued before the current stage's MFMAs so their latency overlaps.  Every output sums its products in ascending
// k (MFMA s takes k = 4s..4s+3), with no split of K over waves, so all tile shapes give
// bitwise-identical results and the autotuner may pick any of them.
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "mfma_ops.h"

namespace peps {

namespace {

// Per-thread share of one operand tile (TK x TW entries): NI loads.  Entry e of the tile
// maps to (k, w) either w-fastest (consecutive threads walk the free index) or k-fastest,
// whichever index has unit stride in memory, so the loads coalesce.  TK = 16, or 12, 32
// or 36 where it divides K (no padded k stage).
template <int TK, int TW>
struct TileLd {
    static constexpr int NE = TK * TW, NI = (NE + 255) / 256;
};

// Offsets of this thread's tile entries along the free index (fixed for the whole K
// loop, so read from LDS once; 32-bit, as the launcher checks that every in-sample
// offset fits), and the entry's k within a stage.
template <int TK, int TW, int NI>
__device__ __forceinline__ void tile_map(int (&ow)[NI], int (&kk)[NI], const long long* off_w, bool kfast, int tid) {
    constexpr int NE = TK * TW;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = tid + 256 * i;
        const bool in = NE % 256 == 0 || e < NE;
        kk[i] = kfast ? e % TK : e / TW;
        const int w = kfast ? e / TK : e % TW;
        ow[i] = in ? (int)off_w[w] : -1;
    }
}

// Global loads of one stage: entry i at ow[i] + koff[kk[i]] (koff: the stage's k offsets,
// -1 past K), zero where either is absent (bit i of ok clear).  The raw 64 or 32 bits
// are kept until the LDS store, so one register pair serves both storage types and no
// instruction waits on a load before the next stage's MFMAs.
template <int NI>
__device__ __forceinline__ void tile_issue(unsigned long long (&x)[NI], unsigned& ok, const int (&ow)[NI],
                                           const int (&kk)[NI], const long long* koff, int f32, const double* srcd,
                                           const float* srcf) {
    long long o[NI];
    ok = 0;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const long long ko = koff[kk[i]];
        const bool v = ow[i] >= 0 && ko >= 0;
        ok |= (unsigned)v << i;
        o[i] = v ? ow[i] + ko : 0;
    }
    if (f32) {
#pragma unroll
        for (int i = 0; i < NI; ++i) x[i] = __float_as_uint(srcf[o[i]]);
    } else {
#pragma unroll
        for (int i = 0; i < NI; ++i) x[i] = (unsigned long long)__double_as_longlong(srcd[o[i]]);
    }
}

// k offsets of stage k0 of both operands (threads 0 .. 2 TK - 1): the only divisions of
// the multi-index k, once per stage and workgroup
template <int TK>
__device__ __forceinline__ void stage_koff(long long* ka, long long* kb, const Idx2& ak, const Idx2& bk, int k0,
                                           int K, int tid) {
    if (tid < 2 * TK) {
        const int kk = tid % TK, k = k0 + kk;
        const long long v = k < K ? idx_off(tid < TK ? ak : bk, k) : -1;
        (tid < TK ? ka : kb)[kk] = v;
    }
}

template <int TK, int TW, int NI, Arith AR>
__device__ __forceinline__ void tile_store(typename MT<AR>::In* dst, const unsigned long long (&x)[NI], unsigned ok,
                                           bool kfast, int f32, int tid) {
    using In = typename MT<AR>::In;
    constexpr int NE = TK * TW;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = tid + 256 * i;
        if (NE % 256 != 0 && e >= NE) continue;
        const int kk = kfast ? e % TK : e / TW, w = kfast ? e / TK : e % TW;
        const double d = f32 ? (double)__uint_as_float((unsigned)x[i]) : __longlong_as_double((long long)x[i]);
        dst[kk * (TW + 1) + w] = ((ok >> i) & 1) ? to_mt<AR>(d) : In(0);
    }
}

// Output of one wave's blocks: C = alpha acc (+ beta C).  Lane (li, gq) holds column li of
// each 16 x 16 block, rows 4 gq + r (float32 MFMA) or gq + 4 r (float64 MFMA).  With
// beta != 0 and GATHER (the float64 factorisation updates), all of the lane's old values are
// loaded before any is used (read without a branch, p[ok ? o : 0]), so their latencies
// overlap instead of adding up; the other launches keep those registers free.
template <int BM, int BN, Arith AR, bool GATHER, class Acc>
__device__ __forceinline__ void tile_out(const Acc (&acc)[BM][BN], const GemmArgs& g, long long c0,
                                         const long long* coff_m, const long long* coff_n, int wm, int wn, int li,
                                         int gq) {
    double* Cd = g.C + c0;
    float* Cf = reinterpret_cast<float*>(g.C) + c0;
    auto off = [&](int i, int j, int r) -> long long {
        const int row = AR == Arith::F64 ? gq + 4 * r : 4 * gq + r;
        const long long om = coff_m[(wm * BM + i) * 16 + row], on = coff_n[(wn * BN + j) * 16 + li];
        return (om < 0 || on < 0) ? -1 : om + on;
    };
    double old[GATHER ? BM : 1][GATHER ? BN : 1][4];
#pragma unroll
    for (int i = 0; i < (GATHER ? BM : 1); ++i)
#pragma unroll
        for (int j = 0; j < (GATHER ? BN : 1); ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) old[i][j][r] = 0.0;
    if (GATHER && g.beta != 0.0) {
#pragma unroll
        for (int i = 0; i < BM; ++i)
#pragma unroll
            for (int j = 0; j < BN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const long long o = off(i, j, r);
                    const long long oo = o >= 0 ? o : 0;
                    old[GATHER ? i : 0][GATHER ? j : 0][r] = g.c_f32 ? (double)Cf[oo] : Cd[oo];
                }
    }
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long o = off(i, j, r);
                if (o < 0) continue;
                double v = g.alpha * (double)acc[i][j][r];
                if (g.beta != 0.0)
                    v += g.beta * (GATHER ? old[GATHER ? i : 0][GATHER ? j : 0][r] : (g.c_f32 ? (double)Cf[o] : Cd[o]));
                if (g.c_f32) Cf[o] = (float)v;
                else Cd[o] = v;
            }
}

template <int WM, int WN, int BM, int BN, int TK, Arith AR, bool GATHER = false>
__global__ __launch_bounds__(256) void k_mgemm(GemmArgs g, int tiles_m, int tiles_n) {
    using In = typename MT<AR>::In;
    using Acc = typename MT<AR>::Acc;
    constexpr int TM = 16 * WM * BM, TN = 16 * WN * BN;
    __shared__ In As[TK * (TM + 1)];
    __shared__ In Bs[TK * (TN + 1)];
    __shared__ long long aoff_m[TM], boff_n[TN], coff_m[TM], coff_n[TN];
    __shared__ long long koff[2][2][TK];   // [stage parity][operand][k in stage]

    const int tiles = tiles_m * tiles_n;
    const long long blk = blockIdx.x;
    const int b = (int)(blk / tiles);
    const int t = (int)(blk % tiles);
    const int m0 = (t / tiles_n) * TM;
    const int n0 = (t % tiles_n) * TN;
    const int tid = threadIdx.x;
    if (b >= g.batch) return;
    if (g.skip && g.skip[(long long)b * g.skip_bs] == 0) return;

    const long long a0 = (long long)b * g.a_bs + gather_off(g.ga, b);
    const long long b0 = (long long)b * g.b_bs + gather_off(g.gb, b);
    const long long c0 = (long long)b * g.c_bs + gather_off(g.gc, b);
    const double* Ab = g.A + a0;
    const double* Bb = g.B + b0;
    const float* Af = reinterpret_cast<const float*>(g.A) + a0;
    const float* Bf = reinterpret_cast<const float*>(g.B) + b0;

    for (int i = tid; i < TM; i += 256) {
        const int m = m0 + i;
        aoff_m[i] = m < g.M ? idx_off(g.am, m) : -1;
        coff_m[i] = m < g.M ? idx_off(g.cm, m) : -1;
    }
    for (int i = tid; i < TN; i += 256) {
        const int n = n0 + i;
        boff_n[i] = n < g.N ? idx_off(g.bn, n) : -1;
        coff_n[i] = n < g.N ? idx_off(g.cn, n) : -1;
    }
    // unit stride along k (and not along the free index): walk k fastest
    const bool akf = g.ak.s_inner == 1 && !(g.am.s_inner == 1 && g.am.inner > 1);
    const bool bkf = g.bk.s_inner == 1 && !(g.bn.s_inner == 1 && g.bn.inner > 1);
    __syncthreads();

    const int lane = tid & 63, w = tid >> 6;
    const int wm = w % WM, wn = w / WM;
    const int li = lane & 15, gq = lane >> 4;
    Acc acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

    constexpr int NIA = TileLd<TK, TM>::NI, NIB = TileLd<TK, TN>::NI;
    static_assert(NIA <= 32 && NIB <= 32, "tile share exceeds the load mask");
    unsigned long long xa[NIA], xb[NIB];
    unsigned oka, okb;
    int owa[NIA], owb[NIB];
    int kka[NIA], kkb[NIB];
    tile_map<TK, TM, NIA>(owa, kka, aoff_m, akf, tid);
    tile_map<TK, TN, NIB>(owb, kkb, boff_n, bkf, tid);
    stage_koff<TK>(koff[0][0], koff[0][1], g.ak, g.bk, 0, g.K, tid);
    __syncthreads();
    tile_issue<NIA>(xa, oka, owa, kka, koff[0][0], g.a_f32, Ab, Af);
    tile_issue<NIB>(xb, okb, owb, kkb, koff[0][1], g.b_f32, Bb, Bf);
    int stg = 0;
    for (int k0 = 0; k0 < g.K; k0 += TK, ++stg) {
        // the next stage's k offsets go to the other buffer, last read two stages ago
        const int nb = (stg + 1) & 1;
        if (k0 + TK < g.K) stage_koff<TK>(koff[nb][0], koff[nb][1], g.ak, g.bk, k0 + TK, g.K, tid);
        __syncthreads();
        tile_store<TK, TM, NIA, AR>(As, xa, oka, akf, g.a_f32, tid);
        tile_store<TK, TN, NIB, AR>(Bs, xb, okb, bkf, g.b_f32, tid);
        __syncthreads();
        if (k0 + TK < g.K) {
            tile_issue<NIA>(xa, oka, owa, kka, koff[nb][0], g.a_f32, Ab, Af);
            tile_issue<NIB>(xb, okb, owb, kkb, koff[nb][1], g.b_f32, Bb, Bf);
        }
#pragma unroll
        for (int s = 0; s < TK / 4; ++s) {
            In av[BM], bv[BN];
#pragma unroll
            for (int i = 0; i < BM; ++i) av[i] = As[(4 * s + gq) * (TM + 1) + (wm * BM + i) * 16 + li];
#pragma unroll
            for (int j = 0; j < BN; ++j) bv[j] = Bs[(4 * s + gq) * (TN + 1) + (wn * BN + j) * 16 + li];
#pragma unroll
            for (int i = 0; i < BM; ++i)
#pragma unroll
                for (int j = 0; j < BN; ++j) acc[i][j] = mfma<AR>(av[i], bv[j], acc[i][j]);
        }
    }
    tile_out<BM, BN, AR, GATHER>(acc, g, c0, coff_m, coff_n, wm, wn, li, gq);
}

// Persistent form of k_mgemm for the short-K products that bound the contraction chain
// by memory: each workgroup walks the tiles blockIdx.x, blockIdx.x + gridDim.x, ... as
// one flattened sequence of (tile, k stage) steps, so the global loads of the next
// step (the next tile's first stage included) are in flight during the current step's
// MFMAs and the previous tile's output stores.  The LDS operand tiles are double
// buffered (one barrier per step), the k offsets of a stage double buffered, and the
// row / column offset tables of a tile triple buffered (a tile of one stage has its
// table rewritten one step after its output is stored).  Per output the products are
// summed exactly as in k_mgemm (ascending k, one MFMA chain), so results are equal bit
// for bit.
template <int TM, int TN>
__device__ __forceinline__ void tile_tables(const GemmArgs& g, int m0, int n0, long long* ao, long long* bo,
                                            long long* co_m, long long* co_n, int tid) {
    for (int i = tid; i < TM; i += 256) {
        const int m = m0 + i;
        ao[i] = m < g.M ? idx_off(g.am, m) : -1;
        co_m[i] = m < g.M ? idx_off(g.cm, m) : -1;
    }
    for (int i = tid; i < TN; i += 256) {
        const int n = n0 + i;
        bo[i] = n < g.N ? idx_off(g.bn, n) : -1;
        co_n[i] = n < g.N ? idx_off(g.cn, n) : -1;
    }
}

// next tile of this workgroup after t whose sample is not skipped (total when none)
__device__ __forceinline__ long long next_tile(const GemmArgs& g, long long t, int tiles, long long total) {
    for (t += gridDim.x; t < total; t += gridDim.x)
        if (!g.skip || g.skip[(t / tiles) * g.skip_bs] != 0) break;
    return t;
}

template <int WM, int WN, int BM, int BN, int TK, Arith AR>
__global__ __launch_bounds__(256) void k_mgemm_p(GemmArgs g, int tiles_m, int tiles_n) {
    using In = typename MT<AR>::In;
    using Acc = typename MT<AR>::Acc;
    constexpr int TM = 16 * WM * BM, TN = 16 * WN * BN;
    __shared__ In As[2][TK * (TM + 1)];
    __shared__ In Bs[2][TK * (TN + 1)];
    __shared__ long long aoff_m[3][TM], boff_n[3][TN], coff_m[3][TM], coff_n[3][TN];
    __shared__ long long koff[2][2][TK];   // [step parity][operand][k in stage]

    const int tiles = tiles_m * tiles_n;
    const long long total = (long long)tiles * g.batch;
    const int nst = (g.K + TK - 1) / TK;
    const int tid = threadIdx.x;
    long long it = blockIdx.x;                      // tile of the loads in flight
    if (g.skip && it < total && g.skip[(it / tiles) * g.skip_bs] == 0) it = next_tile(g, it, tiles, total);
    if (it >= total) return;                        // uniform over the workgroup

    const bool akf = g.ak.s_inner == 1 && !(g.am.s_inner == 1 && g.am.inner > 1);
    const bool bkf = g.bk.s_inner == 1 && !(g.bn.s_inner == 1 && g.bn.inner > 1);
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w % WM, wn = w / WM;
    const int li = lane & 15, gq = lane >> 4;
    constexpr int NIA = TileLd<TK, TM>::NI, NIB = TileLd<TK, TN>::NI;
    static_assert(NIA <= 32 && NIB <= 32, "tile share exceeds the load mask");
    unsigned long long xa[NIA], xb[NIB];
    unsigned oka, okb;
    int owa[NIA], owb[NIB];
    int kka[NIA], kkb[NIB];
    Acc acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

    // operand bases of tile t (sample t / tiles, spin-selected slices)
    auto bases = [&](long long t, const double*& Ab, const double*& Bb) {
        const int b = (int)(t / tiles);
        Ab = g.A + (long long)b * g.a_bs + gather_off(g.ga, b);
        Bb = g.B + (long long)b * g.b_bs + gather_off(g.gb, b);
    };
    auto issue = [&](long long t, int tb, int stage, int kb) {
        const double *Ab, *Bb;
        bases(t, Ab, Bb);
        const long long abs_ = Ab - g.A, bbs = Bb - g.B;
        tile_issue<NIA>(xa, oka, owa, kka, koff[kb][0], g.a_f32, Ab, reinterpret_cast<const float*>(g.A) + abs_);
        tile_issue<NIB>(xb, okb, owb, kkb, koff[kb][1], g.b_f32, Bb, reinterpret_cast<const float*>(g.B) + bbs);
        (void)tb;
        (void)stage;
    };

    // prologue: tables of the first tile, its first stage in flight
    int tb_i = 0;                                   // table buffer of the in-flight tile
    {
        const int t = (int)(it % tiles);
        tile_tables<TM, TN>(g, (t / tiles_n) * TM, (t % tiles_n) * TN, aoff_m[0], boff_n[0], coff_m[0], coff_n[0], tid);
        stage_koff<TK>(koff[0][0], koff[0][1], g.ak, g.bk, 0, g.K, tid);
    }
    __syncthreads();
    tile_map<TK, TM, NIA>(owa, kka, aoff_m[0], akf, tid);
    tile_map<TK, TN, NIB>(owb, kkb, boff_n[0], bkf, tid);
    issue(it, 0, 0, 0);

    long long ct = it;                              // tile of the step being computed
    int cs = 0, tb_c = 0;                           // its stage and table buffer
    int is = 0;                                     // stage of the loads in flight
    for (int step = 0;; ++step) {
        // where the next loads come from: the next stage, or the next tile's first
        long long nt = it;
        int ns = is + 1;
        if (ns == nst) {
            nt = next_tile(g, it, tiles, total);
            ns = 0;
        }
        const bool more = nt < total;
        const int kb = (step + 1) & 1;
        int tb_n = tb_i;
        if (more) {
            stage_koff<TK>(koff[kb][0], koff[kb][1], g.ak, g.bk, ns * TK, g.K, tid);
            if (ns == 0) {
                tb_n = tb_i == 2 ? 0 : tb_i + 1;
                const int t = (int)(nt % tiles);
                tile_tables<TM, TN>(g, (t / tiles_n) * TM, (t % tiles_n) * TN, aoff_m[tb_n], boff_n[tb_n],
                                    coff_m[tb_n], coff_n[tb_n], tid);
            }
        }
        In* as = As[step & 1];
        In* bs = Bs[step & 1];
        tile_store<TK, TM, NIA, AR>(as, xa, oka, akf, g.a_f32, tid);
        tile_store<TK, TN, NIB, AR>(bs, xb, okb, bkf, g.b_f32, tid);
        __syncthreads();
        if (more) {
            if (ns == 0) {
                tile_map<TK, TM, NIA>(owa, kka, aoff_m[tb_n], akf, tid);
                tile_map<TK, TN, NIB>(owb, kkb, boff_n[tb_n], bkf, tid);
            }
            issue(nt, tb_n, ns, kb);
        }
#pragma unroll
        for (int s = 0; s < TK / 4; ++s) {
            In av[BM], bv[BN];
#pragma unroll
            for (int i = 0; i < BM; ++i) av[i] = as[(4 * s + gq) * (TM + 1) + (wm * BM + i) * 16 + li];
#pragma unroll
            for (int j = 0; j < BN; ++j) bv[j] = bs[(4 * s + gq) * (TN + 1) + (wn * BN + j) * 16 + li];
#pragma unroll
            for (int i = 0; i < BM; ++i)
#pragma unroll
                for (int j = 0; j < BN; ++j) acc[i][j] = mfma<AR>(av[i], bv[j], acc[i][j]);
        }
        if (cs == nst - 1) {
            // output of tile ct, then the accumulators restart for the next tile
            const int b = (int)(ct / tiles);
            const long long c0 = (long long)b * g.c_bs + gather_off(g.gc, b);
            tile_out<BM, BN, AR, false>(acc, g, c0, coff_m[tb_c], coff_n[tb_c], wm, wn, li, gq);
#pragma unroll
            for (int i = 0; i < BM; ++i)
#pragma unroll
                for (int j = 0; j < BN; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;
        }
        if (!more) break;
        ct = nt;
        cs = ns;
        tb_c = tb_n;
        it = nt;
        is = ns;
        tb_i = tb_n;
    }
}

template <int WM, int WN, int BM, int BN, int TK, Arith AR>
int persistent_grid(long long total) {
    static int per_cu = -1;
    static int cus = 0;
    if (per_cu < 0) {
        int n = 0, dev = 0;
        hipGetDevice(&dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mgemm_p<WM, WN, BM, BN, TK, AR>, 256, 0) != hipSuccess ||
            n < 1)
            n = 1;
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 256;
        cus = c;
        per_cu = n;
    }
    return (int)std::min<long long>(total, (long long)per_cu * cus);
}

template <int WM, int WN, int BM, int BN, int TK = 16>
hipError_t launch_p(const GemmArgs& g, Arith ar, hipStream_t st) {
    constexpr int TM = 16 * WM * BM, TN = 16 * WN * BN;
    const int tm = (g.M + TM - 1) / TM, tn = (g.N + TN - 1) / TN;
    const long long total = (long long)tm * tn * g.batch;
    if (total == 0) return hipSuccess;
    const dim3 block(256);
    switch (ar) {
        case Arith::F64:
            hipLaunchKernelGGL((k_mgemm_p<WM, WN, BM, BN, TK, Arith::F64>),
                               dim3(persistent_grid<WM, WN, BM, BN, TK, Arith::F64>(total)), block, 0, st, g, tm, tn);
            break;
        case Arith::F32:
            hipLaunchKernelGGL((k_mgemm_p<WM, WN, BM, BN, TK, Arith::F32>),
                               dim3(persistent_grid<WM, WN, BM, BN, TK, Arith::F32>(total)), block, 0, st, g, tm, tn);
            break;
        case Arith::BF16:
            hipLaunchKernelGGL((k_mgemm_p<WM, WN, BM, BN, TK, Arith::BF16>),
                               dim3(persistent_grid<WM, WN, BM, BN, TK, Arith::BF16>(total)), block, 0, st, g, tm, tn);
            break;
    }
    return hipGetLastError();
}

template <int WM, int WN, int BM, int BN, int TK = 16>
hipError_t launch_m(const GemmArgs& g, Arith ar, hipStream_t st) {
    constexpr int TM = 16 * WM * BM, TN = 16 * WN * BN;
    const int tm = (g.M + TM - 1) / TM, tn = (g.N + TN - 1) / TN;
    const long long blocks = (long long)tm * tn * g.batch;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(256);
    switch (ar) {
        case Arith::F64:
            // the factorisation updates (beta != 0) read their old values all at once
            if (g.beta != 0.0)
                hipLaunchKernelGGL((k_mgemm<WM, WN, BM, BN, TK, Arith::F64, true>), grid, block, 0, st, g, tm, tn);
            else
                hipLaunchKernelGGL((k_mgemm<WM, WN, BM, BN, TK, Arith::F64>), grid, block, 0, st, g, tm, tn);
            break;
        case Arith::F32: hipLaunchKernelGGL((k_mgemm<WM, WN, BM, BN, TK, Arith::F32>), grid, block, 0, st, g, tm, tn); break;
        case Arith::BF16: hipLaunchKernelGGL((k_mgemm<WM, WN, BM, BN, TK, Arith::BF16>), grid, block, 0, st, g, tm, tn); break;
    }
    return hipGetLastError();
}

// largest offset of a multi-index over [0, n) (strides must not be negative)
long long idx_bound(const Idx2& x, int n) {
    if (n <= 0) return 0;
    if (x.s_outer < 0 || x.s_inner < 0 || x.inner <= 0) return -1;
    const long long lo = std::min<long long>(n - 1, x.inner - 1);
    return (long long)((n - 1) / x.inner) * x.s_outer + lo * x.s_inner;
}

}  // namespace

// tiles 1..kMfmaTiles (TM x TN, k stage): 32x32, 64x16, 16x64, 64x64, 128x16, 16x128, 64x32, 32x64,
// 128x64, 64x128, 128x32, 32x128 (k stage 16); 64x48, 128x48, 48x64, 48x128 (16); 64x48, 128x48,
// 48x64, 64x64 (k stage 12: no padded stage when K is a multiple of 12, e.g. 36 or 216);
// 64x48, 128x48, 48x64, 64x64, 32x64 (k stage 36: a K of 36 in one stage, one barrier pair);
// 64x64, 32x64 (k stage 32); persistent pipelined forms (k_mgemm_p): 64x48, 64x64, 48x64,
// 128x48 (k stage 12), 64x64, 32x64, 64x48, 48x64 (16)
hipError_t launch_mgemm(const GemmArgs& g, Arith ar, hipStream_t st, int tile) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    // consecutive lanes write consecutive N: a result with unit stride along M instead (the
    // column-major updates of the QR and of the application of Q) runs as the transposed
    // product, whose stores then coalesce.  Same products, same ascending k: same bits.
    auto unit = [](const Idx2& x) { return x.s_inner == 1 && x.inner > 1; };
    if (unit(g.cm) && !unit(g.cn)) return launch_mgemm(gemm_transposed(g), ar, st, tile);
    // the kernels hold the free-index offsets of A and B in 32 bits
    const long long ma = idx_bound(g.am, g.M), nb = idx_bound(g.bn, g.N);
    if (ma < 0 || nb < 0 || ma > 0x7fffffffLL || nb > 0x7fffffffLL) return hipErrorInvalidValue;
    if (tile <= 0 || tile > kMfmaTiles) {
        // heuristic: the smallest tile that covers small products, 48-wide where a leg of
        // 36 or 48 would leave a 64-wide tile part-empty, else 64 x 64 (64 x 48 with a
        // 12-deep stage); a k stage of 36 for K = 36 or 72, of 12 where it divides K, else 16
        const bool k36 = g.K % 36 == 0 && g.K <= 72;   // longer K: the 36-deep tiles hold too many registers
        const bool k12 = !k36 && g.K % 12 == 0 && g.K % 16 != 0;
        if (g.M <= 32 && g.N <= 32) tile = 1;
        else if (g.N <= 16) tile = g.M >= 128 ? 5 : 2;
        else if (g.M <= 16) tile = g.N >= 128 ? 6 : 3;
        else if (g.M <= 32) tile = k36 ? 25 : (g.K % 32 == 0 ? 27 : 8);
        else if (g.N <= 48 && g.N > 32) tile = k36 ? 21 : k12 ? 18 : 14;
        else if (g.M <= 48 && g.M > 32) tile = k36 ? 23 : k12 ? 19 : 15;
        else if (g.N <= 32) tile = 7;
        else tile = k36 ? 24 : k12 ? 17 : 4;
    }
    switch (tile) {
        case 1: return launch_m<2, 2, 1, 1>(g, ar, st);
        case 2: return launch_m<4, 1, 1, 1>(g, ar, st);
        case 3: return launch_m<1, 4, 1, 1>(g, ar, st);
        case 4: return launch_m<2, 2, 2, 2>(g, ar, st);
        case 5: return launch_m<4, 1, 2, 1>(g, ar, st);
        case 6: return launch_m<1, 4, 1, 2>(g, ar, st);
        case 7: return launch_m<2, 2, 2, 1>(g, ar, st);
        case 8: return launch_m<2, 2, 1, 2>(g, ar, st);
        case 9: return launch_m<2, 2, 4, 2>(g, ar, st);
        case 10: return launch_m<2, 2, 2, 4>(g, ar, st);
        case 11: return launch_m<4, 1, 2, 2>(g, ar, st);
        case 12: return launch_m<1, 4, 2, 2>(g, ar, st);
        case 13: return launch_m<4, 1, 1, 3>(g, ar, st);
        case 14: return launch_m<4, 1, 2, 3>(g, ar, st);
        case 15: return launch_m<1, 4, 3, 1>(g, ar, st);
        case 16: return launch_m<1, 4, 3, 2>(g, ar, st);
        case 17: return launch_m<4, 1, 1, 3, 12>(g, ar, st);
        case 18: return launch_m<4, 1, 2, 3, 12>(g, ar, st);
        case 19: return launch_m<1, 4, 3, 1, 12>(g, ar, st);
        case 20: return launch_m<2, 2, 2, 2, 12>(g, ar, st);
        case 21: return launch_m<4, 1, 1, 3, 36>(g, ar, st);
        case 22: return launch_m<4, 1, 2, 3, 36>(g, ar, st);
        case 23: return launch_m<1, 4, 3, 1, 36>(g, ar, st);
        case 24: return launch_m<2, 2, 2, 2, 36>(g, ar, st);
        case 25: return launch_m<2, 2, 1, 2, 36>(g, ar, st);
        case 26: return launch_m<2, 2, 2, 2, 32>(g, ar, st);
        case 27: return launch_m<2, 2, 1, 2, 32>(g, ar, st);
        case 28: return launch_p<4, 1, 1, 3, 12>(g, ar, st);
        case 29: return launch_p<2, 2, 2, 2, 12>(g, ar, st);
        case 30: return launch_p<1, 4, 3, 1, 12>(g, ar, st);
        case 31: return launch_p<4, 1, 2, 3, 12>(g, ar, st);
        case 32: return launch_p<2, 2, 2, 2, 16>(g, ar, st);
        case 33: return launch_p<2, 2, 1, 2, 16>(g, ar, st);
        case 34: return launch_p<4, 1, 1, 3, 16>(g, ar, st);
        default: return launch_p<1, 4, 3, 1, 16>(g, ar, st);
    }
}

}  // namespace peps
