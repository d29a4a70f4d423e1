// Truncation step of the right-to-left sweep through a symmetric eigenproblem.
//
// For the centre M (m' x n', formed as Q G with the reflectors of the QR sweep)
// the leading t = min(Dc, m', n') right singular vectors are the leading
// eigenvectors of the Gram matrix M^T M (or, when n' > m', they follow from those
// of M M^T).  In exact arithmetic this is the same truncation as an SVD of M; the
// kept subspace is accurate to about eps * sigma_1^2 / (sigma_t^2 - sigma_{t+1}^2).
//
//   k_eig_prep  one workgroup per matrix: Z = Q G, Gram A, Householder reduction
//               of A to tridiagonal form (d, e); reflectors kept for later.
//   k_eig_tri   one lane per (matrix, eigenvalue): bisection with Sturm counts for
//               the l-th largest eigenvalue, then inverse iteration on the
//               tridiagonal matrix (LDL^T recurrences).
//   k_eig_fin   one workgroup per matrix: modified Gram-Schmidt (twice) on the t
//               tridiagonal eigenvectors, back-transformation by the reflectors,
//               then the new boundary tensor V_t^T and U_t Sigma_t.
#include "common.h"
#include "kernels.h"

namespace peps {

static constexpr int NT = 256;
static constexpr int kQc = 4;    // reflectors staged per chunk in the implicit-Q phase

__device__ inline double e_wave_sum(double v, int width) { return lane_group_sum(v, width); }
__device__ inline double e_block_sum(double v, double* red) {
    v = e_wave_sum(v, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}
__host__ __device__ inline int e_tpc(int ncols) {
    int p = 1;
    while (p < ncols) p <<= 1;
    const int t = NT / p;
    return t < 1 ? 1 : (t > 64 ? 64 : t);
}
__host__ __device__ inline int e_pad(int tpc) { return tpc == 16 ? 2 : 4; }

// Block order of the register-resident tridiagonalisation: the 16 x 16 thread grid holds
// A in RB x RB blocks, so orders up to 64 stay in registers (RB = 8 would spill);
// 0 = the LDS/global variant.
__host__ __device__ inline int tri_rb(int ns) {
    return ns <= 16 ? 1 : ns <= 32 ? 2 : ns <= 64 ? 4 : 0;
}

// Per-matrix global scratch (doubles): everything the three kernels hand over.
__host__ __device__ inline EigLayout eig_layout(int mz, int tin, int p, int Dc) {
    EigLayout L;
    L.mp = mz / p;
    L.np = p * tin;
    L.gram_right = L.np <= L.mp;             // A = M^T M (n' x n'), else A = M M^T
    L.ns = L.gram_right ? L.np : L.mp;
    L.tk = Dc < L.ns ? Dc : L.ns;
    L.ldz = mz + e_pad(e_tpc(tin));
    L.lda = L.ns + 1;
    L.ldx = L.ns + 1;
    L.oZ = 0;
    L.oA = L.oZ + (long long)L.ldz * tin;
    L.oD = L.oA + (long long)L.lda * L.ns;
    L.oE = L.oD + L.ns;
    L.oT = L.oE + L.ns;
    L.oX = L.oT + L.ns;
    L.oL = L.oX + (long long)L.ldx * L.tk;
    L.oP = L.oL + L.tk;
    L.nv = 3 * L.ns + 2 > kQc * mz ? 3 * L.ns + 2 : kQc * mz;   // work vectors of the prep kernel
    if (L.nv < 48 * tri_rb(L.ns)) L.nv = 48 * tri_rb(L.ns);
    L.oW = L.oP + (long long)L.ldx * L.tk;
    L.nm = 0;
    L.oM = L.oW + L.nv;
    L.oY = L.oM;                                   // refinement: Y (mp x tk) and W (np x tk)
    L.oV = L.oY + (long long)L.mp * L.tk;
    L.oQ = L.oV + (long long)L.np * L.tk;          // W blocks of the GEMM application of Q
    L.total = L.oQ + 64LL * tin;
    // LDS needs of the two workgroup kernels
    L.lds_prep = (long long)L.ldz * tin + (long long)L.lda * L.ns + 3LL * L.ns + L.nv + 8;
    // k_eig_fin stages X, tau and the eigenvalues; the reflectors and Z stay in global
    // scratch, where they are L2-resident (the reflectors are read by every vector group
    // alike, Z only by the output products): about 9 KB of LDS per block instead of 76 KB
    // at the bulk shape, so more blocks share a CU
    L.lds_fin = (long long)L.ldx * L.tk + L.ns + L.tk + 8;
    return L;
}

// ---------------------------------------------------------------------------
// A: centre, Gram, tridiagonalisation
// ---------------------------------------------------------------------------

// Householder reduction of the symmetric A (order ns <= 16 RB, full storage in Am) to
// tridiagonal form with A held in registers.  Thread (ti, tj) of the 16 x 16 grid (ti =
// 4 wave + lane / 16, tj = lane % 16) owns rows ti RB .. ti RB + RB - 1 and the same
// range of columns; padding rows and columns up to 16 RB stay exactly zero.  Step k:
//   pivot   the 16 lanes of the row group holding row k (== column k) form the
//           reflector H_k = I - tau v v^T from entries k+1.. of that row (v_{k+1} = 1);
//   p       = tau A v, row sums reduced over the 16 lanes of a segment;
//   update  A <- A - v w^T - w v^T with w = p - (tau/2)(p.v) v on the whole register
//           matrix.  That is the similarity H A H: it leaves the finished diagonal
//           entries alone (v vanishes on indices <= k) and takes the rest of row and
//           column k to (e_k, 0, ...) up to rounding; those entries are never read
//           again, and the live trailing block gets exactly the masked update's values.
// Entries beyond k+1 of v_k are stored in row k of Am for the back-transformation.
// Two barriers per step; v and tau are double-buffered so the next pivot can run
// while other waves still finish their update.
// G x G threads (G = 16: four waves; G = 8: one wave holding 8x8 blocks, whose row
// sums then take three lane stages instead of four and need no barrier between waves).
template <int RB, int G = 16>
__device__ __forceinline__ void tri_reg(double* Am, double* d, double* e, double* tau, double* vbuf, int ns, int lda) {
    constexpr int W = G * RB, NW = G * G / 64;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ti = tid / G, tj = tid % G;
    const int r0 = ti * RB, c0 = tj * RB;
    double* pb = vbuf + 2 * W;
    __shared__ double s_tau2[2];
    __shared__ double s_red[NW];
    double A[RB][RB];
#pragma unroll
    for (int u = 0; u < RB; ++u)
#pragma unroll
        for (int w = 0; w < RB; ++w)
            A[u][w] = (r0 + u < ns && c0 + w < ns) ? Am[(long long)(c0 + w) * lda + r0 + u] : 0.0;
    __syncthreads();   // Am rows are overwritten by reflectors below
    auto pivot = [&](int kp) {
        // the same for every active lane (the row group holding row kp)
        const int ku = __builtin_amdgcn_readfirstlane(kp - r0);
        double rv[RB];
#pragma unroll
        for (int u = 0; u < RB; ++u)
            if (u == ku)   // a uniform branch: one row of registers copied
#pragma unroll
                for (int w = 0; w < RB; ++w) rv[w] = A[u][w];
        double sq = 0.0, al = 0.0;
#pragma unroll
        for (int w = 0; w < RB; ++w) {
            const int j = c0 + w;
            if (j >= kp + 2) sq = fma(rv[w], rv[w], sq);
            if (j == kp + 1) al = rv[w];
        }
        sq = e_wave_sum(sq, G);
        al = e_wave_sum(al, G);
        double tk, be, sc;
        if (sq == 0.0) {
            tk = 0.0; be = al; sc = 0.0;
        } else {
            be = -copysign(sqrt(al * al + sq), al);
            tk = (be - al) / be;
            sc = 1.0 / (al - be);
        }
        double* vb = vbuf + (kp & 1) * W;
#pragma unroll
        for (int w = 0; w < RB; ++w) {
            const int j = c0 + w;
            const double v = (j >= kp + 2) ? sc * rv[w] : (j == kp + 1 ? 1.0 : 0.0);
            vb[j] = v;
            if (tk != 0.0 && j >= kp + 2 && j < ns) Am[(long long)kp * lda + j] = v;
        }
        if (tj == 0) {
            s_tau2[kp & 1] = tk;
            tau[kp] = tk;
            e[kp] = be;
        }
    };
    if (ns > 2 && ti == 0) pivot(0);
    __syncthreads();
    for (int k = 0; k + 2 < ns; ++k) {
        const int par = k & 1;
        const double tk = s_tau2[par];
        // rows 0..k are final: v is zero there, so a wave whose rows all lie in that range
        // adds exact zeros to p and to v.p, and the trailing matrix never reads the entries
        // it would update; such a wave only publishes its zeros (the test is wave-uniform)
        const bool fin = (wave + 1) * (64 / G) * RB <= k + 1;
        if (tk != 0.0) {
            const double* vb = vbuf + par * W;
            double vr[RB], vc[RB], pr[RB];
            if (!fin) {
#pragma unroll
                for (int u = 0; u < RB; ++u) vr[u] = vb[r0 + u];
#pragma unroll
                for (int w = 0; w < RB; ++w) vc[w] = vb[c0 + w];
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    double acc = 0.0;
#pragma unroll
                    for (int w = 0; w < RB; ++w) acc = fma(A[u][w], vc[w], acc);
                    pr[u] = tk * e_wave_sum(acc, G);
                }
                double pv = 0.0;
#pragma unroll
                for (int u = 0; u < RB; ++u) pv = fma(pr[u], vr[u], pv);
                // one value per row group of G lanes: sum over the row groups of the wave
                if (G == 8) pv += dpp_perm<0x140>(pv);   // the other row group of the 16 lanes
                if (G <= 16) pv = add_xor16(pv);
                pv = add_xor32(pv);
                if (lane == 0) s_red[wave] = pv;
            } else {
#pragma unroll
                for (int u = 0; u < RB; ++u) pr[u] = 0.0;
                if (lane == 0) s_red[wave] = 0.0;
            }
            if (tj == 0)
#pragma unroll
                for (int u = 0; u < RB; ++u) pb[r0 + u] = pr[u];
            __syncthreads();
            if (!fin) {
                double pc[RB];
#pragma unroll
                for (int w = 0; w < RB; ++w) pc[w] = pb[c0 + w];
                double sp = 0.0;
#pragma unroll
                for (int i = 0; i < NW; ++i) sp += s_red[i];
                const double K = 0.5 * tk * sp;
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    const double wr = pr[u] - K * vr[u];
#pragma unroll
                    for (int w = 0; w < RB; ++w) {
                        const double wc = pc[w] - K * vc[w];
                        A[u][w] -= vr[u] * wc + wr * vc[w];
                    }
                }
            }
        }
        if (k + 3 < ns && ti == (k + 1) / RB) pivot(k + 1);
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < RB; ++u)
#pragma unroll
        for (int w = 0; w < RB; ++w) {
            const int i = r0 + u, j = c0 + w;
            if (i == j && i < ns) d[i] = A[u][w];
            if (i == ns - 2 && j == ns - 1) e[ns - 2] = A[u][w];
        }
    if (tid == 0) {
        if (ns >= 2) tau[ns - 2] = 0.0;
        if (ns >= 1) tau[ns - 1] = 0.0;
    }
    __syncthreads();
}

// The same reduction for orders up to GR RBR = GC RBC (224 with the 32 x 16 grid of 7 x 14
// blocks below), where a square grid would not fit the register file: thread (ti, tj) of
// the GR x GC grid (tj fastest, so a row group is GC lanes of one wave) owns rows ti RBR ..
// and columns tj RBC ..; the column entries of v and p are read from LDS inside the loops
// instead of being held in registers.  Same steps, outputs and reflector storage as tri_reg.
template <int RBR, int RBC, int GR, int GC>
__device__ __forceinline__ void tri_reg_rect(double* Am, double* d, double* e, double* tau, double* vbuf, int ns,
                                             int lda) {
    constexpr int W = GR * RBR, NW = GR * GC / 64;
    static_assert(GR * RBR == GC * RBC, "square coverage");
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ti = tid / GC, tj = tid % GC;
    const int r0 = ti * RBR, c0 = tj * RBC;
    double* pb = vbuf + 2 * W;
    __shared__ double s_tau2[2];
    __shared__ double s_red[NW];
    double A[RBR][RBC];
#pragma unroll
    for (int u = 0; u < RBR; ++u)
#pragma unroll
        for (int w = 0; w < RBC; ++w)
            A[u][w] = (r0 + u < ns && c0 + w < ns) ? Am[(long long)(c0 + w) * lda + r0 + u] : 0.0;
    __syncthreads();   // Am rows are overwritten by reflectors below
    auto pivot = [&](int kp) {
        const int ku = __builtin_amdgcn_readfirstlane(kp - r0);
        double sq = 0.0, al = 0.0;
#pragma unroll
        for (int u = 0; u < RBR; ++u)
            if (u == ku) {
#pragma unroll
                for (int w = 0; w < RBC; ++w) {
                    const int j = c0 + w;
                    if (j >= kp + 2) sq = fma(A[u][w], A[u][w], sq);
                    if (j == kp + 1) al = A[u][w];
                }
            }
        sq = e_wave_sum(sq, GC);
        al = e_wave_sum(al, GC);
        double tk, be, sc;
        if (sq == 0.0) {
            tk = 0.0; be = al; sc = 0.0;
        } else {
            be = -copysign(sqrt(al * al + sq), al);
            tk = (be - al) / be;
            sc = 1.0 / (al - be);
        }
        double* vb = vbuf + (kp & 1) * W;
#pragma unroll
        for (int u = 0; u < RBR; ++u)
            if (u == ku) {
#pragma unroll
                for (int w = 0; w < RBC; ++w) {
                    const int j = c0 + w;
                    const double v = (j >= kp + 2) ? sc * A[u][w] : (j == kp + 1 ? 1.0 : 0.0);
                    vb[j] = v;
                    if (tk != 0.0 && j >= kp + 2 && j < ns) Am[(long long)kp * lda + j] = v;
                }
            }
        if (tj == 0) {
            s_tau2[kp & 1] = tk;
            tau[kp] = tk;
            e[kp] = be;
        }
    };
    if (ns > 2 && ti == 0) pivot(0);
    __syncthreads();
    for (int k = 0; k + 2 < ns; ++k) {
        const int par = k & 1;
        const double tk = s_tau2[par];
        const bool fin = (wave + 1) * (64 / GC) * RBR <= k + 1;
        if (tk != 0.0) {
            const double* vb = vbuf + par * W;
            double vr[RBR], pr[RBR];
            if (!fin) {
#pragma unroll
                for (int u = 0; u < RBR; ++u) {
                    vr[u] = vb[r0 + u];
                    pr[u] = 0.0;
                }
#pragma unroll
                for (int w = 0; w < RBC; ++w) {
                    const double vc = vb[c0 + w];
#pragma unroll
                    for (int u = 0; u < RBR; ++u) pr[u] = fma(A[u][w], vc, pr[u]);
                }
#pragma unroll
                for (int u = 0; u < RBR; ++u) pr[u] = tk * e_wave_sum(pr[u], GC);
                double pv = 0.0;
#pragma unroll
                for (int u = 0; u < RBR; ++u) pv = fma(pr[u], vr[u], pv);
                // one value per row group of GC lanes: sum over the row groups of the wave
                if (GC <= 16) pv = add_xor16(pv);
                pv = add_xor32(pv);
                if (lane == 0) s_red[wave] = pv;
            } else {
#pragma unroll
                for (int u = 0; u < RBR; ++u) {
                    pr[u] = 0.0;
                    vr[u] = 0.0;
                }
                if (lane == 0) s_red[wave] = 0.0;
            }
            if (tj == 0)
#pragma unroll
                for (int u = 0; u < RBR; ++u) pb[r0 + u] = pr[u];
            __syncthreads();
            if (!fin) {
                double sp = 0.0;
#pragma unroll
                for (int i = 0; i < NW; ++i) sp += s_red[i];
                const double K = 0.5 * tk * sp;
                // A -= v w^T + w v^T with w = p - K v, written as v (p - 2 K v)^T + p v^T on
                // the block so that no w is held in registers
#pragma unroll
                for (int w = 0; w < RBC; ++w) {
                    const double vc = vb[c0 + w];
                    const double yc = pb[c0 + w] - 2.0 * K * vc;
#pragma unroll
                    for (int u = 0; u < RBR; ++u) A[u][w] -= vr[u] * yc + pr[u] * vc;
                }
            }
        }
        if (k + 3 < ns && ti == (k + 1) / RBR) pivot(k + 1);
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < RBR; ++u)
#pragma unroll
        for (int w = 0; w < RBC; ++w) {
            const int i = r0 + u, j = c0 + w;
            if (i == j && i < ns) d[i] = A[u][w];
            if (i == ns - 2 && j == ns - 1) e[ns - 2] = A[u][w];
        }
    if (tid == 0) {
        if (ns >= 2) tau[ns - 2] = 0.0;
        if (ns >= 1) tau[ns - 1] = 0.0;
    }
    __syncthreads();
}

// Gram matrix of M (full symmetric storage, stride lda) with 4x4 register blocks per
// thread, read straight from Z (column-major, stride ldz):
//   gram_right: A[c1][c2] = sum_ar M[ar][c1] M[ar][c2]   (x = column c, y = row ar)
//   else:       A[a1][a2] = sum_col M[a1][col] M[a2][col] (x = row a, y = column col)
// M[ar][col] = Z[t][ar*p+d] with col = d*tin + t, i.e. element (x, y) = Z[bx(x) + by(y)].
__device__ inline void gram_4x4(const double* Z, int ldz, double* Am, int lda, const EigLayout& L, int tin,
                                int p) {
    const int tid = threadIdx.x, ns = L.ns;
    const int ny = L.gram_right ? L.mp : L.np;
    auto bx = [&](int x) -> int {
        return L.gram_right ? (x % tin) * ldz + x / tin : x * p;
    };
    auto by = [&](int y) -> int {
        return L.gram_right ? y * p : (y % tin) * ldz + y / tin;
    };
    const int nb = (ns + 3) / 4;                 // 4x4 blocks per dimension
    for (int blk = tid; blk < nb * nb; blk += NT) {
        const int bi = blk / nb, bj = blk % nb;
        if (bj < bi) continue;
        double acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int w = 0; w < 4; ++w) acc[u][w] = 0.0;
        int oi[4], oj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            oi[u] = bx(min(bi * 4 + u, ns - 1));
            oj[u] = bx(min(bj * 4 + u, ns - 1));
        }
#pragma unroll 4
        for (int y = 0; y < ny; ++y) {   // unrolled: four rows' LDS reads in flight
            const double* zy = Z + by(y);
            double a4[4], b4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a4[u] = zy[oi[u]];
                b4[u] = zy[oj[u]];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int w = 0; w < 4; ++w) acc[u][w] = fma(a4[u], b4[w], acc[u][w]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int ii = bi * 4 + u, jj = bj * 4 + w;
                if (ii < ns && jj < ns && jj >= ii) {
                    Am[(long long)ii * lda + jj] = acc[u][w];
                    Am[(long long)jj * lda + ii] = acc[u][w];
                }
            }
    }
}

// Z = Q [G; 0] with Z held in registers: group g of TPC lanes owns the columns g, g + NG, ...
// (NG = NT / TPC), lane l the row pairs (2l, 2l+1) + 2 TPC j, so one 16-byte LDS read of a
// reflector serves CPG columns.  Reflectors are staged kc at a time through LDS, zero
// below their first row and with the unit leading entry written out (one barrier per
// chunk).  The result goes to the Z slot of the per-matrix scratch.
static constexpr int kMaxKc = 32;

template <int TPC>
__device__ __forceinline__ int zq_row(int q, int l) {
    return (q >> 1) * (2 * TPC) + 2 * l + (q & 1);
}

template <int RPT, int TPC, int CPG>
__global__ __launch_bounds__(NT) void k_eig_applyq(EigArgs a, int kc) {
    extern __shared__ __align__(16) double vsh[];
    __shared__ double s_tq[kMaxKc];
    constexpr int NG = NT / TPC, LDV = RPT * TPC;
    const EigLayout L = eig_layout(a.mz, a.tin, a.p, a.Dc);
    const int b = blockIdx.x, tid = threadIdx.x, g = tid / TPC, l = tid % TPC;
    const int mz = a.mz, tin = a.tin, r = a.r, ldz = L.ldz;
    const double* G = a.G + (long long)b * a.gs;
    const double* V = a.V + (long long)b * a.vs;
    const double* tq = a.tau + (long long)b * a.ts;
    double z[CPG][RPT];
#pragma unroll
    for (int s = 0; s < CPG; ++s) {
        const int c = g + s * NG;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = zq_row<TPC>(q, l);
            z[s][q] = (c < tin && i < r) ? G[(long long)i * tin + c] : 0.0;
        }
    }
    for (int k1 = r - 1; k1 >= 0; k1 -= kc) {
        const int k0 = k1 - kc + 1 > 0 ? k1 - kc + 1 : 0, nk = k1 - k0 + 1;
        __syncthreads();
        // reflectors k0..k1 zero-padded with the unit entry written out; loads in groups
        for (int e0 = 0; e0 < nk * LDV; e0 += 8 * NT) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + tid + u * NT, kk = e / LDV, i = e % LDV, k = k0 + kk;
                const bool in = e < nk * LDV;
                const double raw = ld_or0(in && i > k && i < mz, V, (long long)k * mz + i);
                v[u] = (in && i == k) ? 1.0 : raw;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + tid + u * NT;
                if (e < nk * LDV) vsh[e] = v[u];
            }
        }
        if (tid < nk) s_tq[tid] = tq[k0 + tid];
        __syncthreads();
        for (int k = k1; k >= k0; --k) {
            const double tk = s_tq[k - k0];
            if (tk == 0.0) continue;
            const double* vk = vsh + (k - k0) * LDV;
            double v[RPT];
#pragma unroll
            for (int q = 0; q < RPT; q += 2) {
                const double2 t = *reinterpret_cast<const double2*>(vk + zq_row<TPC>(q, l));
                v[q] = t.x;
                v[q + 1] = t.y;
            }
#pragma unroll
            for (int s = 0; s < CPG; ++s) {
                if (g + s * NG >= tin) continue;
                double d0 = 0.0, d1 = 0.0;
#pragma unroll
                for (int q = 0; q < RPT; q += 2) {
                    d0 = fma(v[q], z[s][q], d0);
                    d1 = fma(v[q + 1], z[s][q + 1], d1);
                }
                const double f = tk * lane_group_sum(d0 + d1, TPC);
#pragma unroll
                for (int q = 0; q < RPT; ++q) z[s][q] = fma(-f, v[q], z[s][q]);
            }
        }
    }
    double* gsb = a.scratch + (long long)b * a.ss;
    double* Z = gsb + L.oZ;
    if (a.gram_ready) __syncthreads();   // the staging buffer now takes Z
#pragma unroll
    for (int s = 0; s < CPG; ++s) {
        const int c = g + s * NG;
        if (c >= tin) continue;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = zq_row<TPC>(q, l);
            if (i < mz) {
                Z[(long long)c * ldz + i] = z[s][q];
                if (a.gram_ready) vsh[(long long)c * ldz + i] = z[s][q];
            }
        }
    }
    if (a.gram_ready) {
        // Gram matrix of the reshaped centre, from the LDS copy of Z, into the Am slot
        __syncthreads();
        gram_4x4(vsh, ldz, gsb + L.oA, L.lda, L, tin, a.p);
    }
}

// Householder tridiagonalisation of the Gram matrix formed by k_eig_applyq (order
// <= G RB), A in registers; reflectors, d, e and tau go straight to the scratch slots.
template <int RB, int G = 16>
__global__ __launch_bounds__(G * G) void k_eig_tridiag(EigArgs a) {
    __shared__ __align__(16) double vbuf[3 * G * RB];
    const EigLayout L = eig_layout(a.mz, a.tin, a.p, a.Dc);
    double* gs = a.scratch + (long long)blockIdx.x * a.ss;
    tri_reg<RB, G>(gs + L.oA, gs + L.oD, gs + L.oE, gs + L.oT, vbuf, L.ns, L.lda);
}

// tridiagonalisation of a Gram matrix of order <= 224 already in the Am slot (formed on
// the matrix cores by launch_eig), 512 threads
__global__ __launch_bounds__(512) void k_eig_tridiag_big(EigArgs a) {
    __shared__ __align__(16) double vbuf[3 * 224];
    const EigLayout L = eig_layout(a.mz, a.tin, a.p, a.Dc);
    double* gs = a.scratch + (long long)blockIdx.x * a.ss;
    tri_reg_rect<7, 14, 32, 16>(gs + L.oA, gs + L.oD, gs + L.oE, gs + L.oT, vbuf, L.ns, L.lda);
}

// launch k_eig_applyq for the first lane-group width (16, 32, 64) whose register
// blocking fits mz x tin (16 measured fastest at mz = 256, tin = 16); false when none
// does (the prep kernel then applies Q itself)
template <int TPC>
static bool applyq_t(const EigArgs& a, size_t cap, size_t zbytes, hipStream_t st) {
    constexpr int NG = NT / TPC;
    int rpt = (a.mz + TPC - 1) / TPC;
    rpt += rpt & 1;
    const int cpg = (a.tin + NG - 1) / NG;
#define AQ_LAUNCH(RPT_, CPG_)                                                                   \
    if (rpt <= RPT_ && cpg <= CPG_) {                                                             \
        const size_t ldv = (size_t)RPT_ * TPC;                                                    \
        int kc = (int)(cap / (ldv * sizeof(double)));                                             \
        kc = kc > kMaxKc ? kMaxKc : kc;                                                           \
        kc = kc > a.r ? a.r : kc;                                                                 \
        if (kc < 1) return false;                                                                 \
        size_t bytes = (size_t)kc * ldv * sizeof(double);                                         \
        if (a.gram_ready && bytes < zbytes) bytes = zbytes;                                       \
        hipLaunchKernelGGL((k_eig_applyq<RPT_, TPC, CPG_>), dim3(a.batch), dim3(NT), bytes, st,   \
                           a, kc);                                                                \
        return true;                                                                              \
    }
    AQ_LAUNCH(2, 1)
    AQ_LAUNCH(4, 1)
    AQ_LAUNCH(2, 2)
    AQ_LAUNCH(8, 1)
    AQ_LAUNCH(4, 2)
    AQ_LAUNCH(2, 4)
    AQ_LAUNCH(16, 1)
    AQ_LAUNCH(8, 2)
    AQ_LAUNCH(4, 4)
    AQ_LAUNCH(16, 2)
    AQ_LAUNCH(8, 4)
#undef AQ_LAUNCH
    return false;
}

static bool launch_applyq(const EigArgs& a, size_t cap, size_t zbytes, hipStream_t st) {
    if (!a.V || a.r <= 0) return false;
    return applyq_t<16>(a, cap, zbytes, st) || applyq_t<32>(a, cap, zbytes, st) ||
           applyq_t<64>(a, cap, zbytes, st);
}

template <bool kLds, int RB>
__device__ void prep_body(const EigArgs& a, double* Z, double* Am, double* d, double* e, double* tau,
                          double* vbuf, const EigLayout& L, double* red) {
    const int b = blockIdx.x, tid = threadIdx.x;
    const int mz = a.mz, tin = a.tin, p = a.p, ns = L.ns, lda = L.lda, ldz = L.ldz;
    // Z = [G; 0] then Z <- Q Z (reflectors of the QR of this column, applied last to first).
    // Group c owns column c of Z.
    const double* G = a.G + (long long)b * a.gs;
    const int r = a.V ? a.r : mz;
    if (a.z_ready) {
        // Z = Q [G; 0] was formed by k_eig_applyq in global scratch
        if constexpr (kLds) {
            const double* zg = a.scratch + (long long)b * a.ss + L.oZ;
            copy_strided(Z, zg, (long long)ldz * tin, tid, NT);
        }
    } else {
        for (int e2 = tid; e2 < mz * tin; e2 += NT) {
            const int c = e2 / mz, i = e2 % mz;
            Z[(long long)c * ldz + i] = (i < r) ? G[(long long)i * tin + c] : 0.0;
        }
    }
    __syncthreads();
    if (a.V && !a.z_ready) {
        const double* V = a.V + (long long)b * a.vs;
        const double* tq = a.tau + (long long)b * a.ts;
        const int tpc = e_tpc(tin), ngroups = NT / tpc, g = tid / tpc, l = tid % tpc;
        // lane l always owns the rows i = l (mod tpc) of its group's column; reflectors
        // are staged through LDS kQc at a time (one barrier per chunk)
        double* vs = vbuf;                      // kQc reflectors of length mz
        __shared__ double s_tq[kQc];
        for (int k1 = r - 1; k1 >= 0; k1 -= kQc) {
            const int k0 = k1 - kQc + 1 > 0 ? k1 - kQc + 1 : 0;
            __syncthreads();
            copy_strided(vs, V + (long long)k0 * mz, (long long)(k1 - k0 + 1) * mz, tid, NT);
            if (tid <= k1 - k0) s_tq[tid] = tq[k0 + tid];
            __syncthreads();
            for (int c0 = 0; c0 < tin; c0 += ngroups) {
                const int c = c0 + g;
                const bool act = c < tin;
                double* zc = Z + (long long)(act ? c : 0) * ldz;
                for (int k = k1; k >= k0; --k) {
                    const double tk = s_tq[k - k0];
                    if (tk == 0.0) continue;
                    const double* vk = vs + (k - k0) * mz;
                    const int i0 = k + (((l - k) % tpc) + tpc) % tpc;     // first own row >= k
                    double dot = 0.0;
                    if (act)
                        for (int i = i0; i < mz; i += tpc) dot += ((i == k) ? 1.0 : vk[i]) * zc[i];
                    dot = e_wave_sum(dot, tpc);
                    if (act) {
                        const double f = tk * dot;
                        for (int i = i0; i < mz; i += tpc) zc[i] -= f * ((i == k) ? 1.0 : vk[i]);
                    }
                }
            }
        }
        __syncthreads();
    }
    gram_4x4(Z, ldz, Am, lda, L, tin, p);
    if constexpr (RB > 0) {
        __syncthreads();
        tri_reg<RB>(Am, d, e, tau, vbuf, ns, lda);
        return;
    }
    // Householder tridiagonalisation in full symmetric storage (row c == column c).
    // At step k, group g updates column c = k+1+g (+ multiples of the group count),
    // lane l the rows i = k+1+l (mod tpc); group 0 therefore holds column k+1 right
    // after step k and computes the next reflector from its own lanes' rows (no
    // cross-lane reads).  Reflector k (v_{k+1} = 1 implicit) is kept in column k,
    // rows > k+1, for the back-transformation.  Two barriers per step.
    __shared__ double s_tau[2];
    double* vb0 = vbuf;                 // two reflector buffers of length ns
    double* vb1 = vbuf + ns;
    double* pb = vbuf + 2 * ns;         // p = tau A v
    // orders above 128 (the matrix in global memory): a whole wave per column, so every
    // column is read in coalesced 64-row runs (one lane per column would stream 256
    // separate columns)
    const int tpc = ns > 128 ? 64 : e_tpc(ns), ngroups = NT / tpc, g = tid / tpc, l = tid % tpc;
    __syncthreads();
    auto pivot = [&](int kp, double* vb) {
        double* ck = Am + (long long)kp * lda;
        double sq = 0.0, al = 0.0;
        for (int i = kp + l; i < ns; i += tpc) {
            const double x = ck[i];
            if (i >= kp + 2) sq += x * x;
            if (i == kp + 1) al = x;
        }
        sq = e_wave_sum(sq, tpc);
        al = e_wave_sum(al, tpc);
        double tk, be, sc;
        if (sq == 0.0) {
            tk = 0.0; be = al; sc = 0.0;
        } else {
            be = -copysign(sqrt(al * al + sq), al);
            tk = (be - al) / be;
            sc = 1.0 / (al - be);
        }
        for (int i = kp + l; i < ns; i += tpc) {
            if (i >= kp + 2) {
                const double v = sc * ck[i];
                if (tk != 0.0) ck[i] = v;
                vb[i] = v;
            } else {
                vb[i] = (i == kp + 1) ? 1.0 : 0.0;
            }
        }
        for (int i = l; i < kp; i += tpc) vb[i] = 0.0;
        if (l == 0) {
            s_tau[kp & 1] = tk;
            tau[kp] = tk;
            e[kp] = be;
        }
    };
    if (ns > 2 && g == 0) pivot(0, vb0);
    __syncthreads();
    for (int k = 0; k + 2 < ns; ++k) {
        const double tk = s_tau[k & 1];
        const double* v = (k & 1) ? vb1 : vb0;
        if (tk != 0.0) {
            // p_c = tau * (A v)_c for c > k
            for (int c0 = k + 1; c0 < ns; c0 += ngroups) {
                const int c = c0 + g;
                const bool act = c < ns;
                const double* col = Am + (long long)(act ? c : 0) * lda;
                double dot = 0.0;
                if (act)
                    for (int i = k + 1 + l; i < ns; i += tpc) dot += col[i] * v[i];
                dot = e_wave_sum(dot, tpc);
                if (act && l == 0) pb[c] = tk * dot;
            }
            __syncthreads();
            // K = tau/2 (p . v), w = p - K v ; column c -= v w_c + w v_c
            double pv = 0.0;
            for (int i = k + 1 + l; i < ns; i += tpc) pv += pb[i] * v[i];
            pv = e_wave_sum(pv, tpc);
            const double K = 0.5 * tk * pv;
            for (int c0 = k + 1; c0 < ns; c0 += ngroups) {
                const int c = c0 + g;
                if (c >= ns) continue;
                double* col = Am + (long long)c * lda;
                const double vc = v[c], wc = pb[c] - K * vc;
                for (int i = k + 1 + l; i < ns; i += tpc) col[i] -= v[i] * wc + (pb[i] - K * v[i]) * vc;
            }
        }
        if (k + 3 < ns && g == 0) pivot(k + 1, (k & 1) ? vb0 : vb1);
        __syncthreads();
    }
    if (tid == 0) {
        if (ns >= 2) {
            e[ns - 2] = Am[(long long)(ns - 2) * lda + (ns - 1)];
            tau[ns - 2] = 0.0;
        }
        if (ns >= 1) tau[ns - 1] = 0.0;
    }
    for (int k = tid; k < ns; k += NT) d[k] = Am[(long long)k * lda + k];
    __syncthreads();
}

template <bool kLds, int RB>
__global__ __launch_bounds__(NT) void k_eig_prep(EigArgs a) {
    extern __shared__ double lds[];
    __shared__ double red[NT / 64];
    const EigLayout L = eig_layout(a.mz, a.tin, a.p, a.Dc);
    const int b = blockIdx.x;
    double* gs = a.scratch + (long long)b * a.ss;
    if constexpr (kLds) {
        double* Z = lds;
        double* Am = Z + (long long)L.ldz * a.tin;
        double* d = Am + (long long)L.lda * L.ns;
        double* e = d + L.ns;
        double* tau = e + L.ns;
        double* vbuf = tau + L.ns;
        prep_body<true, RB>(a, Z, Am, d, e, tau, vbuf, L, red);
        // hand over Z, reflectors, d, e, tau
        const int tid = threadIdx.x;
        if (!a.z_ready)
            for (long long i = tid; i < (long long)L.ldz * a.tin; i += NT) gs[L.oZ + i] = Z[i];
        for (long long i = tid; i < (long long)L.lda * L.ns; i += NT) gs[L.oA + i] = Am[i];
        for (int i = tid; i < L.ns; i += NT) {
            gs[L.oD + i] = d[i];
            gs[L.oE + i] = e[i];
            gs[L.oT + i] = tau[i];
        }
    } else {
        // everything in global scratch
        prep_body<false, RB>(a, gs + L.oZ, gs + L.oA, gs + L.oD, gs + L.oE, gs + L.oT, gs + L.oW, L, red);
    }
}

// ---------------------------------------------------------------------------
// B: eigenvalues and tridiagonal eigenvectors, one lane each
// ---------------------------------------------------------------------------
__device__ inline unsigned hash_u32(unsigned x) {
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    return x;
}

// 1/q by the hardware reciprocal estimate refined with one Newton-Raphson step
// (r <- r + r (1 - q r)), which roughly doubles the estimate's correct bits.  Used in the
// Sturm recurrence, whose sign count is backward stable to such rounding, and for the
// pivots of inverse iteration (bounded away from zero there), which corrects itself.
__device__ inline double sturm_rcp(double q) {
    const double r = __builtin_amdgcn_rcp(q);
    return fma(fma(-q, r, 1.0), r, r);
}

// Block = mats_per_block matrices x tk eigenvalues x S sub-lanes.  The S sub-lanes of an
// eigenvalue (aligned, consecutive lanes) evaluate the Sturm count at S interior points
// of the common interval, which therefore shrinks by S + 1 per step (multisection); all
// of them then hold the same interval.  Sub-lane 0 runs the inverse iteration.
__global__ __launch_bounds__(256) void k_eig_tri(EigArgs a, int S, int mats_per_block, int tri_lanes_in_lds) {
    extern __shared__ double tri_lds[];
    const EigLayout L = eig_layout(a.mz, a.tin, a.p, a.Dc);
    const int n = L.ns, tk = L.tk;
    const int lpm = tk * S;
    const int mi = threadIdx.x / lpm, le = threadIdx.x % lpm, l = le / S, sub = le % S;
    const int b = blockIdx.x * mats_per_block + mi;
    // d, e and e^2 of this block's matrices in LDS (every Sturm step reads them)
    for (int e2 = threadIdx.x; e2 < mats_per_block * n; e2 += blockDim.x) {
        const int m2 = e2 / n, i = e2 % n;
        const int b2 = blockIdx.x * mats_per_block + m2;
        const double* g2 = a.scratch + (long long)(b2 < a.batch ? b2 : 0) * a.ss;
        const double dv = ld_or0(b2 < a.batch, g2, L.oD + i);
        const double ev = ld_or0(b2 < a.batch && i + 1 < n, g2, L.oE + i);
        tri_lds[(3 * m2) * n + i] = dv;
        tri_lds[(3 * m2 + 1) * n + i] = ev;
        tri_lds[(3 * m2 + 2) * n + i] = ev * ev;
    }
    __syncthreads();
    if (b >= a.batch || mi >= mats_per_block) return;
    double* gs = a.scratch + (long long)b * a.ss;
    const double* d = tri_lds + (3 * mi) * n;
    const double* e = tri_lds + (3 * mi + 1) * n;
    const double* e2 = tri_lds + (3 * mi + 2) * n;
    // Gershgorin interval and pivot floor
    double lo = 0.0, hi = 0.0, emax2 = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
        lo = (i == 0) ? d[i] - r : fmin(lo, d[i] - r);
        hi = (i == 0) ? d[i] + r : fmax(hi, d[i] + r);
        if (i + 1 < n) emax2 = fmax(emax2, e2[i]);
    }
    const double tnorm = fmax(fabs(lo), fabs(hi));
    const double pivmin = 1e-300 * fmax(1.0, emax2);
    const int kidx = n - 1 - l;   // l-th largest = kidx-th smallest
    const int base = threadIdx.x - sub;
    // count(x) = number of eigenvalues < x
    for (int it = 0; it < 128; ++it) {
        // to the accuracy the tridiagonal supports (about eps times its norm), so that inverse
        // iteration separates every eigenvalue the Gram matrix resolves
        if (hi - lo <= 4.5e-16 * tnorm + pivmin) break;
        const double h = (hi - lo) / (double)(S + 1);
        const double x = lo + (double)(sub + 1) * h;
        int cnt = 0;
        double q = d[0] - x;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
        for (int i = 1; i < n; ++i) {
            q = d[i] - x - e2[i - 1] * sturm_rcp(q);
            if (fabs(q) < pivmin) q = -pivmin;
            cnt += q < 0.0;
        }
        // the first point with more than kidx eigenvalues below it bounds lambda above
        double nlo = lo, nhi = hi;
        bool found = false;
        for (int s2 = 0; s2 < S; ++s2) {
            const int c2 = __shfl(cnt, base + s2, 64);
            const double x2 = lo + (double)(s2 + 1) * h;
            if (!found) {
                if (c2 > kidx) {
                    nhi = x2;
                    found = true;
                } else {
                    nlo = x2;
                }
            }
        }
        lo = nlo;
        hi = nhi;
    }
    if (sub != 0 || l >= tk) return;
    const double lam = 0.5 * (lo + hi);
    // the lane's iterate: in LDS after the d/e block when it fits, element i of every
    // vector lane side by side (stride mats_per_block * tk), its pivots then side by side in
    // global scratch (stride tk: coalesced, and half the LDS, so more blocks share a CU);
    // else both in global scratch, one row per lane
    const int vl = mi * tk + l, nvl = mats_per_block * tk;
    double* x;
    double* piv;
    int xs, ps;
    if (tri_lanes_in_lds) {
        xs = nvl;
        x = tri_lds + 3LL * mats_per_block * n + vl;
        piv = gs + L.oP + l;
        ps = tk;
    } else {
        xs = 1;
        ps = 1;
        x = gs + L.oX + (long long)l * L.ldx;
        piv = gs + L.oP + (long long)l * L.ldx;
    }
    // inverse iteration (T - lam I) x = b with T - lam I = L D L^T
    const double ptol = fmax(2.220446049250313e-16 * tnorm, 1e-300);
    for (int i = 0; i < n; ++i)
        x[i * xs] = (double)(hash_u32((unsigned)(l * 7919 + i * 104729 + 17)) & 0xffffff) / 16777216.0 - 0.5;
    // Per sweep: one pass factors and solves L y = b together (both run upwards), one
    // solves L^T x = D^-1 y and finds max |x_i|, one forms the norm of x / max, one scales.
    // Each recurrence carries its previous term in a register (LDS stays off the
    // dependency chain); the reciprocal pivots come from the hardware estimate plus one
    // Newton step, the pivots being bounded away from zero by ptol.
    for (int it = 0; it < 3; ++it) {
        double q = d[0] - lam;
        if (fabs(q) < ptol) q = (q < 0.0) ? -ptol : ptol;
        double pp = sturm_rcp(q);
        piv[0] = pp;
        double y = x[0];
        for (int i = 1; i < n; ++i) {
            y = x[i * xs] - (e[i - 1] * pp) * y;   // pp = 1 / pivot i-1
            x[i * xs] = y;
            q = d[i] - lam - e2[i - 1] * pp;
            if (fabs(q) < ptol) q = (q < 0.0) ? -ptol : ptol;
            pp = sturm_rcp(q);
            piv[i * ps] = pp;
        }
        double xn = x[(n - 1) * xs] * pp;
        x[(n - 1) * xs] = xn;
        double mx = fabs(xn);
        for (int i = n - 2; i >= 0; --i) {
            xn = (x[i * xs] - e[i] * xn) * piv[i * ps];
            x[i * xs] = xn;
            mx = fmax(mx, fabs(xn));
        }
        const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) {
            const double t = x[i * xs] * inv;
            nrm += t * t;
        }
        const double sn = nrm > 0.0 ? 1.0 / sqrt(nrm) : 1.0;
        for (int i = 0; i < n; ++i) x[i * xs] = (x[i * xs] * inv) * sn;
    }
    // eigenvalue from the Rayleigh quotient of the converged unit vector
    double rq = d[0] * x[0] * x[0];
    for (int i = 1; i < n; ++i) rq += d[i] * x[i * xs] * x[i * xs] + 2.0 * e[i - 1] * x[(i - 1) * xs] * x[i * xs];
    gs[L.oL + l] = (fabs(rq - lam) <= 1e-8 * tnorm + pivmin) ? rq : lam;
    if (tri_lanes_in_lds) {
        double* xo = gs + L.oX + (long long)l * L.ldx;
        for (int i = 0; i < n; ++i) xo[i] = x[i * xs];
    }
}

// ---------------------------------------------------------------------------
// C: orthonormalise, back-transform, outputs
// ---------------------------------------------------------------------------
// Orthonormalisation and back-transformation with the t vectors in registers: group g
// of TPC lanes owns the vectors g, g + NG, ... (NG = NT / TPC), lane l the row pairs
// (2l, 2l+1) + 2 TPC j.
//   modified Gram-Schmidt, twice, right-looking: the group of vector j normalises it and
//   publishes it (double-buffered LDS), every later vector then removes its component
//   (one barrier per vector);
//   back-transformation X <- H_0 ... H_{ns-3} X with the reflectors read from Am rows
//   (no barriers: X stays in registers).
// X (LDS or global, stride ldx) holds the result on return.
template <int RPT, int TPC, int CPG>
__device__ __forceinline__ void fin_vectors(double* X, const double* Am, const double* tau, int ns, int tk,
                                            int ldx, int lda) {
    constexpr int NG = NT / TPC, LDQ = RPT * TPC;
    __shared__ __align__(16) double qbuf[2][LDQ];
    const int tid = threadIdx.x, g = tid / TPC, l = tid % TPC;
    double x[CPG][RPT];
#pragma unroll
    for (int s = 0; s < CPG; ++s) {
        const int c = g + s * NG;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = zq_row<TPC>(q, l);
            x[s][q] = (c < tk && i < ns) ? X[(long long)c * ldx + i] : 0.0;
        }
    }
    for (int pass = 0; pass < 2; ++pass) {
        for (int j = 0; j < tk; ++j) {
            double* qj = qbuf[j & 1];
            if (g == j % NG) {
                const int sj = j / NG;
#pragma unroll
                for (int s = 0; s < CPG; ++s) {
                    if (s != sj) continue;
                    double n0 = 0.0, n1 = 0.0;
#pragma unroll
                    for (int q = 0; q < RPT; q += 2) {
                        n0 = fma(x[s][q], x[s][q], n0);
                        n1 = fma(x[s][q + 1], x[s][q + 1], n1);
                    }
                    const double nr = lane_group_sum(n0 + n1, TPC);
                    const double sc = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
#pragma unroll
                    for (int q = 0; q < RPT; q += 2) {
                        x[s][q] *= sc;
                        x[s][q + 1] *= sc;
                        *reinterpret_cast<double2*>(qj + zq_row<TPC>(q, l)) = make_double2(x[s][q], x[s][q + 1]);
                    }
                }
            }
            __syncthreads();
            double qv[RPT];
#pragma unroll
            for (int q = 0; q < RPT; q += 2) {
                const double2 t = *reinterpret_cast<const double2*>(qj + zq_row<TPC>(q, l));
                qv[q] = t.x;
                qv[q + 1] = t.y;
            }
#pragma unroll
            for (int s = 0; s < CPG; ++s) {
                const int c = g + s * NG;
                if (c <= j || c >= tk) continue;
                double d0 = 0.0, d1 = 0.0;
#pragma unroll
                for (int q = 0; q < RPT; q += 2) {
                    d0 = fma(qv[q], x[s][q], d0);
                    d1 = fma(qv[q + 1], x[s][q + 1], d1);
                }
                const double dot = lane_group_sum(d0 + d1, TPC);
#pragma unroll
                for (int q = 0; q < RPT; ++q) x[s][q] = fma(-dot, qv[q], x[s][q]);
            }
        }
    }
    // reflector k: unit entry at row k+1, entries beyond it in row k of Am.  Its entries
    // are read without branches (row k's entry 0 stands in for the rows outside it), and
    // those of reflector k - 1 are already in flight while reflector k is applied.
    double vn[RPT], tn = 0.0;
    const auto load_v = [&](int k, double (&v)[RPT], double& t) {
        const double* vk = Am + (long long)k * lda;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = zq_row<TPC>(q, l);
            const bool in = i > k + 1 && i < ns;
            const double raw = vk[in ? i : 0];
            v[q] = i == k + 1 ? 1.0 : (in ? raw : 0.0);
        }
        t = tau[k];
    };
    if (ns >= 3) load_v(ns - 3, vn, tn);
    for (int k = ns - 3; k >= 0; --k) {
        double v[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) v[q] = vn[q];
        const double tq = tn;
        if (k > 0) load_v(k - 1, vn, tn);
        if (tq == 0.0) continue;
#pragma unroll
        for (int s = 0; s < CPG; ++s) {
            if (g + s * NG >= tk) continue;
            double d0 = 0.0, d1 = 0.0;
#pragma unroll
            for (int q = 0; q < RPT; q += 2) {
                d0 = fma(v[q], x[s][q], d0);
                d1 = fma(v[q + 1], x[s][q + 1], d1);
            }
            const double f = tq * lane_group_sum(d0 + d1, TPC);
#pragma unroll
            for (int q = 0; q < RPT; ++q) x[s][q] = fma(-f, v[q], x[s][q]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < CPG; ++s) {
        const int c = g + s * NG;
        if (c >= tk) continue;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = zq_row<TPC>(q, l);
            if (i < ns) X[(long long)c * ldx + i] = x[s][q];
        }
    }
    __syncthreads();
}

template <bool kLds, int RPT, int TPC, int CPG>
__global__ __launch_bounds__(NT) void k_eig_fin(EigArgs a) {
    extern __shared__ double lds[];
    const EigLayout L = eig_layout(a.mz, a.tin, a.p, a.Dc);
    const int b = blockIdx.x, tid = threadIdx.x;
    const int ns = L.ns, tk = L.tk, ldx = L.ldx, lda = L.lda, ldz = L.ldz, tin = a.tin, p = a.p;
    double* gs = a.scratch + (long long)b * a.ss;
    double *X, *Am, *tau, *Z, *lam;
    if constexpr (kLds) {
        X = lds;
        Am = gs + L.oA;
        tau = X + (long long)ldx * tk;
        Z = gs + L.oZ;
        lam = tau + ns;
        copy_strided(X, gs + L.oX, (long long)ldx * tk, tid, NT);
        copy_strided(tau, gs + L.oT, ns, tid, NT);
        copy_strided(lam, gs + L.oL, tk, tid, NT);
        __syncthreads();
    } else {
        X = gs + L.oX; Am = gs + L.oA; tau = gs + L.oT; Z = gs + L.oZ; lam = gs + L.oL;
    }
    if constexpr (RPT > 0) {
        fin_vectors<RPT, TPC, CPG>(X, Am, tau, ns, tk, ldx, lda);
    } else {
        // modified Gram-Schmidt, twice, by wave 0 (lanes own rows)
        if (tid < 64) {
            for (int pass = 0; pass < 2; ++pass)
                for (int j = 0; j < tk; ++j) {
                    double* xj = X + (long long)j * ldx;
                    for (int i = 0; i < j; ++i) {
                        const double* xi = X + (long long)i * ldx;
                        double dot = 0.0;
                        for (int r = tid; r < ns; r += 64) dot += xi[r] * xj[r];
                        dot = e_wave_sum(dot, 64);
                        for (int r = tid; r < ns; r += 64) xj[r] -= dot * xi[r];
                    }
                    double nr = 0.0;
                    for (int r = tid; r < ns; r += 64) nr += xj[r] * xj[r];
                    nr = e_wave_sum(nr, 64);
                    const double s = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
                    for (int r = tid; r < ns; r += 64) xj[r] *= s;
                }
        }
        __syncthreads();
        // back-transformation: X <- H_0 ... H_{ns-3} X (reflector k acts on rows k+1..; its
        // entries beyond k+1 are stored in Am row k).  Group c owns vector c, lane l the rows
        // i = l (mod tpc), so no barrier is needed between reflectors.
        {
            const int tpc = e_tpc(tk), ngroups = NT / tpc, g = tid / tpc, l = tid % tpc;
            for (int c0 = 0; c0 < tk; c0 += ngroups) {
                const int c = c0 + g;
                const bool act = c < tk;
                double* xc = X + (long long)(act ? c : 0) * ldx;
                for (int k = ns - 3; k >= 0; --k) {
                    const double tq = tau[k];
                    if (tq == 0.0) continue;
                    const double* vk = Am + (long long)k * lda;
                    const int i0 = (k + 1) + (((l - k - 1) % tpc) + tpc) % tpc;   // first own row > k
                    double dot = 0.0;
                    if (act)
                        for (int i = i0; i < ns; i += tpc) dot += ((i == k + 1) ? 1.0 : vk[i]) * xc[i];
                    dot = e_wave_sum(dot, tpc);
                    if (act) {
                        const double f = tq * dot;
                        for (int i = i0; i < ns; i += tpc) xc[i] -= f * ((i == k + 1) ? 1.0 : vk[i]);
                    }
                }
            }
            __syncthreads();
        }
    }
    double* U = a.newU + (long long)b * a.us;
    double* Go = a.Gout + (long long)b * a.gos;
    const int mp = L.mp, np = L.np;
    if (L.gram_right) {
        // X columns are the right singular vectors: V_t^T rows, and U_t Sigma_t = M V_t
        for (int e2 = tid; e2 < tk * np; e2 += NT) {
            const int rr = e2 / np, c = e2 % np;
            U[e2] = X[(long long)rr * ldx + c];
        }
        for (int e2 = tid; e2 < mp * tk; e2 += NT) {
            const int ar = e2 / tk, rr = e2 % tk;
            const double* vk = X + (long long)rr * ldx;
            double acc = 0.0;
            for (int dd = 0; dd < p; ++dd) {
                const double* zrow = Z + ar * p + dd;
#pragma unroll 4
                for (int t = 0; t < tin; ++t) acc += zrow[(long long)t * ldz] * vk[dd * tin + t];
            }
            Go[e2] = acc;
        }
    } else {
        // X columns are left singular vectors u_k; sigma_k = sqrt(lambda_k);
        // U_t Sigma_t = u_k sigma_k and v_k = M^T u_k / sigma_k (renormalised)
        const double lmax = lam[0] > 0.0 ? lam[0] : 0.0;
        for (int e2 = tid; e2 < mp * tk; e2 += NT) {
            const int ar = e2 / tk, rr = e2 % tk;
            const double sg = sqrt(fmax(lam[rr], 0.0));
            Go[e2] = X[(long long)rr * ldx + ar] * sg;
        }
        const int tpc = e_tpc(tk), ngroups = NT / tpc, g = tid / tpc, l = tid % tpc;
        for (int r0 = 0; r0 < tk; r0 += ngroups) {
            const int rr = r0 + g;
            const bool act = rr < tk;
            const double* uk = X + (long long)(act ? rr : 0) * ldx;
            double nr = 0.0;
            if (act) {
                for (int c = l; c < np; c += tpc) {
                    const int dd = c / tin, t = c % tin;
                    const double* zt = Z + (long long)t * ldz + dd;
                    double acc = 0.0;
#pragma unroll 4
                    for (int ar = 0; ar < mp; ++ar) acc += zt[ar * p] * uk[ar];
                    U[(long long)rr * np + c] = acc;
                    nr += acc * acc;
                }
            }
            nr = e_wave_sum(nr, tpc);
            const bool keep = act && lam[rr] > 1e-28 * lmax && nr > 0.0;
            const double s = keep ? 1.0 / sqrt(nr) : 0.0;
            if (act)
                for (int c = l; c < np; c += tpc) U[(long long)rr * np + c] *= s;
        }
    }
}

// ---------------------------------------------------------------------------
// D: refinement of the kept subspace without squaring
// ---------------------------------------------------------------------------
// The Gram eigenvectors locate the kept right singular subspace only to about
// eps sigma_1^2 / (sigma_t^2 - sigma_{t+1}^2), which is too coarse when the boundary spectrum
// decays steeply.  One step of orthogonal iteration on M itself, Y = M V_t, Q = orth(Y),
// V' = orth(M^T Q), rounds to about eps sigma_1 / (sigma_t - sigma_{t+1}) (every product
// acts on orthonormal vectors) and contracts the starting error by (sigma_{t+1}/sigma_t)^2.
// Only the subspace matters: the truncated state M V V^T is the same for any orthonormal
// basis of it.  Outputs: the new tensor V'^T and U_t Sigma_t = M V' (the carried matrix).
//
__device__ inline double e_block_max(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) s = fmax(s, red[i]);
    return s;
}

// Orthonormal basis of the n x t column-major block X (stride n, t <= n) in place, by
// Householder QR followed by the explicit Q = H_0 ... H_{t-1} [I; 0] (LAPACK's dgeqr2 /
// dorg2r steps; the reflectors are scaled by the column's largest entry so no squared norm
// underflows).  Q is orthonormal to working precision whatever the rank of X, and its
// first columns span X's first columns when those are independent.  tq: t doubles.
__device__ inline void hh_orth(double* X, int n, int t, double* tq, double* h, double* red) {
    const int tid = threadIdx.x;
    const int g = tid >> 2, l = tid & 3;
    for (int k = 0; k < t; ++k) {
        double* xk = X + (long long)k * n;
        double mx = 0.0;
        for (int r = k + tid; r < n; r += NT) mx = fmax(mx, fabs(xk[r]));
        mx = e_block_max(mx, red);
        double sq = 0.0;
        const double inv = mx > 0.0 ? 1.0 / mx : 0.0;
        for (int r = k + 1 + tid; r < n; r += NT) {
            const double y = xk[r] * inv;
            sq = fma(y, y, sq);
        }
        sq = e_block_sum(sq, red);
        const double al = xk[k] * inv;
        double tk = 0.0, be = al, sc = 0.0;
        if (mx > 0.0 && sq > 0.0) {
            be = -copysign(sqrt(al * al + sq), al);
            tk = (be - al) / be;
            sc = inv / (al - be);
        }
        __syncthreads();
        if (tk != 0.0)
            for (int r = k + 1 + tid; r < n; r += NT) xk[r] *= sc;   // v below the pivot
        if (tid == 0) tq[k] = tk;
        __syncthreads();
        if (tk != 0.0) {
            // w_c = v^T X[k:, c] for the later columns, 4 lanes per column
            for (int c0 = k + 1; c0 < t; c0 += NT / 4) {
                const int c = c0 + g;
                double dot = 0.0;
                if (c < t) {
                    const double* xc = X + (long long)c * n;
                    if (l == 0) dot = xc[k];
                    for (int r = k + 1 + l; r < n; r += 4) dot = fma(xk[r], xc[r], dot);
                }
                dot = e_wave_sum(dot, 4);
                if (c < t && l == 0) h[c] = tk * dot;
            }
            __syncthreads();
            for (long long e2 = tid; e2 < (long long)(t - k - 1) * (n - k); e2 += NT) {
                const int c = k + 1 + (int)(e2 / (n - k)), r = k + (int)(e2 % (n - k));
                const double v = r == k ? 1.0 : xk[r];
                X[(long long)c * n + r] -= h[c] * v;
            }
            __syncthreads();
        }
    }
    // explicit Q, last reflector first; column k is formed after H_k has acted on the later ones
    for (int k = t - 1; k >= 0; --k) {
        double* xk = X + (long long)k * n;
        const double tk = tq[k];
        if (tk != 0.0 && k + 1 < t) {
            for (int c0 = k + 1; c0 < t; c0 += NT / 4) {
                const int c = c0 + g;
                double dot = 0.0;
                if (c < t) {
                    const double* xc = X + (long long)c * n;
                    for (int r = k + 1 + l; r < n; r += 4) dot = fma(xk[r], xc[r], dot);   // Q[k][c] = 0 here
                }
                dot = e_wave_sum(dot, 4);
                if (c < t && l == 0) h[c] = tk * dot;
            }
            __syncthreads();
            for (long long e2 = tid; e2 < (long long)(t - k - 1) * (n - k); e2 += NT) {
                const int c = k + 1 + (int)(e2 / (n - k)), r = k + (int)(e2 % (n - k));
                const double v = r == k ? 1.0 : xk[r];
                X[(long long)c * n + r] -= h[c] * v;
            }
            __syncthreads();
        }
        for (int r = tid; r < n; r += NT) {
            double q;
            if (r < k) q = 0.0;
            else if (r == k) q = 1.0 - tk;
            else q = -tk * xk[r];
            xk[r] = q;
        }
        __syncthreads();
    }
}

template <bool kLds>
__global__ __launch_bounds__(NT) void k_eig_refine(EigArgs a) {
    extern __shared__ double lds[];
    __shared__ double h[NT];
    __shared__ double red[NT / 64];
    const EigLayout L = eig_layout(a.mz, a.tin, a.p, a.Dc);
    const int b = blockIdx.x, tid = threadIdx.x;
    const int mp = L.mp, np = L.np, tk = L.tk, tin = a.tin, p = a.p, ldz = L.ldz;
    double* gs = a.scratch + (long long)b * a.ss;
    const double* Z = gs + L.oZ;
    double* U = a.newU + (long long)b * a.us;
    double* Go = a.Gout + (long long)b * a.gos;
    // the Gram route already resolves the subspace when every kept eigenvalue is within 1e-6
    // of the largest (sigma_t >= 1e-3 sigma_1): its angle error, about eps lambda_1 / gap, then
    // moves the state by less than 1e-13 relative.  Only steeper spectra are refined.
    {
        const double l0 = gs[L.oL], lt = gs[L.oL + (tk > 0 ? tk - 1 : 0)];
        if (tk <= 0 || !(l0 > 0.0) || lt >= 1e-6 * l0) return;
    }
    double* Y = kLds ? lds : gs + L.oY;                    // mp x tk, column-major
    double* Wv = kLds ? lds + (long long)mp * tk : gs + L.oV;   // np x tk, column-major
    auto Mel = [&](int ar, int c) { return Z[(long long)(c % tin) * ldz + (long long)ar * p + c / tin]; };
    // Y = M V_t (V_t^T is the current tensor, row-major tk x np)
    for (int e2 = tid; e2 < mp * tk; e2 += NT) {
        const int ar = e2 % mp, k = e2 / mp;
        const double* vk = U + (long long)k * np;
        double acc = 0.0;
        for (int c = 0; c < np; ++c) acc = fma(Mel(ar, c), vk[c], acc);
        Y[(long long)k * mp + ar] = acc;
    }
    __syncthreads();
    __shared__ double tq[NT];
    hh_orth(Y, mp, tk, tq, h, red);
    // W = M^T Q
    for (int e2 = tid; e2 < np * tk; e2 += NT) {
        const int c = e2 % np, k = e2 / np;
        const double* qk = Y + (long long)k * mp;
        double acc = 0.0;
        for (int ar = 0; ar < mp; ++ar) acc = fma(Mel(ar, c), qk[ar], acc);
        Wv[(long long)k * np + c] = acc;
    }
    __syncthreads();
    hh_orth(Wv, np, tk, tq, h, red);
    // outputs: V'^T and M V'
    for (int e2 = tid; e2 < tk * np; e2 += NT) {
        const int k = e2 / np, c = e2 % np;
        U[e2] = Wv[(long long)k * np + c];
    }
    for (int e2 = tid; e2 < mp * tk; e2 += NT) {
        const int ar = e2 / tk, k = e2 % tk;
        const double* vk = Wv + (long long)k * np;
        double acc = 0.0;
        for (int c = 0; c < np; ++c) acc = fma(Mel(ar, c), vk[c], acc);
        Go[e2] = acc;
    }
}

// k_eig_fin with register-resident vectors (16-lane groups) when ns and tk fit one of the
// blockings; false when none does
template <int RPT, int CPG>
static bool fin_try(const EigArgs& a, int rpt, int cpg, size_t bf, size_t cap, hipStream_t st) {
    if (rpt > RPT || cpg > CPG) return false;
    const size_t stat = 2 * (size_t)RPT * 16 * sizeof(double);   // the qbuf double buffer
    if (bf + stat <= cap) hipLaunchKernelGGL((k_eig_fin<true, RPT, 16, CPG>), dim3(a.batch), dim3(NT), bf, st, a);
    else hipLaunchKernelGGL((k_eig_fin<false, RPT, 16, CPG>), dim3(a.batch), dim3(NT), 0, st, a);
    return true;
}

static bool launch_fin_reg(const EigArgs& a, const EigLayout& L, size_t bf, size_t cap, hipStream_t st) {
    constexpr int NG = NT / 16;
    int rpt = (L.ns + 15) / 16;
    rpt += rpt & 1;
    const int cpg = (L.tk + NG - 1) / NG;
    return fin_try<2, 1>(a, rpt, cpg, bf, cap, st) || fin_try<4, 1>(a, rpt, cpg, bf, cap, st) ||
           fin_try<2, 2>(a, rpt, cpg, bf, cap, st) || fin_try<8, 1>(a, rpt, cpg, bf, cap, st) ||
           fin_try<4, 2>(a, rpt, cpg, bf, cap, st) || fin_try<8, 2>(a, rpt, cpg, bf, cap, st) ||
           fin_try<4, 4>(a, rpt, cpg, bf, cap, st) || fin_try<16, 1>(a, rpt, cpg, bf, cap, st) ||
           fin_try<16, 2>(a, rpt, cpg, bf, cap, st) || fin_try<8, 4>(a, rpt, cpg, bf, cap, st) ||
           fin_try<16, 4>(a, rpt, cpg, bf, cap, st);
}

// ---------------------------------------------------------------------------
size_t eig_scratch_doubles(int mz, int tin, int p, int Dc) {
    return (size_t)eig_layout(mz, tin, p, Dc).total;
}

hipError_t launch_eig(const double* V, long long vs, const double* tau, long long ts, const double* G,
                      long long gs, int mz, int r, int tin, int p, int Dc, double* newU, long long us,
                      double* Gout, long long gos, double* scratch, long long ss, int batch,
                      hipStream_t st, const double* wyT, long long wys) {
    if (batch <= 0) return hipSuccess;
    EigArgs a;
    a.V = V; a.vs = vs; a.tau = tau; a.ts = ts; a.G = G; a.gs = gs;
    a.mz = mz; a.r = r; a.tin = tin; a.p = p; a.Dc = Dc;
    a.newU = newU; a.us = us; a.Gout = Gout; a.gos = gos;
    a.scratch = scratch; a.ss = ss; a.batch = batch; a.z_ready = 0; a.gram_ready = 0;
    const EigLayout L = eig_layout(mz, tin, p, Dc);
    const size_t cap = get_lds_cap() - 1024;
    // staging for k_eig_applyq: at most a quarter of the LDS so several blocks share a CU;
    // when the tridiagonalisation fits registers it also forms the Gram matrix (its
    // staging buffer then has to hold Z)
    const int rb = tri_rb(L.ns);
    const size_t zbytes = (size_t)L.ldz * tin * sizeof(double);
    a.gram_ready = (rb > 0 && zbytes <= cap / 4) ? 1 : 0;
    if (wyT && V && r > 0) {
        // reflectors of the blocked QR: Z = Q [G; 0] by its WY blocks on the matrix cores
        a.gram_ready = 0;
        hipError_t ez = launch_applyq_blocked(V, vs, mz, r, wyT, wys, G, gs, r, tin, scratch + L.oZ, ss, L.ldz,
                                              scratch + L.oQ, ss, batch, st);
        if (ez != hipSuccess) return ez;
        a.z_ready = 1;
    } else {
        a.z_ready = launch_applyq(a, cap / 4, zbytes, st) ? 1 : 0;
    }
    if (!a.z_ready) a.gram_ready = 0;
    if (a.z_ready) {
        hipError_t e0 = hipGetLastError();
        if (e0 != hipSuccess) return e0;
    }
    const size_t bp = (size_t)L.lds_prep * sizeof(double), bf = (size_t)L.lds_fin * sizeof(double);
    const bool in_lds_prep = bp <= cap;
    const size_t bpl = in_lds_prep ? bp : 0;
    if (rb == 0 && a.z_ready && L.ns <= 224) {
        // orders 65..224: the Gram matrix of the reshaped centre on the matrix cores, then the
        // 512-thread register tridiagonalisation.  M[ar][c] = Z[(c % tin) ldz + ar p + c / tin].
        GemmArgs g{};
        const Idx2 col{tin, 1, (long long)L.ldz}, row{1 << 30, 0, (long long)p};
        g.M = g.N = L.ns;
        g.K = L.gram_right ? L.mp : L.np;
        g.batch = batch;
        g.am = L.gram_right ? col : row;
        g.ak = L.gram_right ? row : col;
        g.bk = g.ak;
        g.bn = g.am;
        g.cm = Idx2{1 << 30, 0, (long long)L.lda};
        g.cn = Idx2{1 << 30, 0, 1};
        g.a_bs = g.b_bs = g.c_bs = ss;
        g.A = g.B = scratch + L.oZ;
        g.C = scratch + L.oA;
        g.alpha = 1.0;
        g.beta = 0.0;
        hipError_t eg = launch_mgemm(g, Arith::F64, st, 0);
        if (eg != hipSuccess) return eg;
        hipLaunchKernelGGL(k_eig_tridiag_big, dim3(batch), dim3(512), 0, st, a);
    } else
    switch (a.gram_ready ? -rb : tri_rb(L.ns) * 2 + (in_lds_prep ? 1 : 0)) {
        case -1: hipLaunchKernelGGL((k_eig_tridiag<2, 8>), dim3(batch), dim3(64), 0, st, a); break;
        case -2: hipLaunchKernelGGL((k_eig_tridiag<4, 8>), dim3(batch), dim3(64), 0, st, a); break;
        case -4: hipLaunchKernelGGL((k_eig_tridiag<8, 8>), dim3(batch), dim3(64), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_eig_prep<false, 1>), dim3(batch), dim3(NT), bpl, st, a); break;
        case 3: hipLaunchKernelGGL((k_eig_prep<true, 1>), dim3(batch), dim3(NT), bpl, st, a); break;
        case 4: hipLaunchKernelGGL((k_eig_prep<false, 2>), dim3(batch), dim3(NT), bpl, st, a); break;
        case 5: hipLaunchKernelGGL((k_eig_prep<true, 2>), dim3(batch), dim3(NT), bpl, st, a); break;
        case 8: hipLaunchKernelGGL((k_eig_prep<false, 4>), dim3(batch), dim3(NT), bpl, st, a); break;
        case 9: hipLaunchKernelGGL((k_eig_prep<true, 4>), dim3(batch), dim3(NT), bpl, st, a); break;
        case 1: hipLaunchKernelGGL((k_eig_prep<true, 0>), dim3(batch), dim3(NT), bpl, st, a); break;
        default: hipLaunchKernelGGL((k_eig_prep<false, 0>), dim3(batch), dim3(NT), bpl, st, a); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (L.tk > NT) return hipErrorInvalidValue;   // one lane per kept value, at most NT per matrix
    const int tkk = L.tk > 0 ? L.tk : 1;
    // multisection sub-lanes: two points per eigenvalue and step (measured against one, four
    // and eight: the bisection is issue-bound, and fewer points cost fewer Sturm sweeps in
    // all while keeping the chain of steps short)
    const int S = 2 * tkk <= 64 ? 2 : 1;
    const int lpm = tkk * S;
    const int mpb = 64 / lpm > 0 ? 64 / lpm : 1;
    size_t tri_bytes = (size_t)3 * mpb * L.ns * sizeof(double);
    const size_t lane_bytes = (size_t)mpb * tkk * L.ns * sizeof(double);   // the iterates
    const int in_lds = tri_bytes + lane_bytes <= cap ? 1 : 0;
    if (in_lds) tri_bytes += lane_bytes;
    hipLaunchKernelGGL(k_eig_tri, dim3((unsigned)((batch + mpb - 1) / mpb)), dim3(mpb * lpm), tri_bytes, st,
                       a, S, mpb, in_lds);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!launch_fin_reg(a, L, bf, cap, st)) {
        if (bf <= cap) hipLaunchKernelGGL((k_eig_fin<true, 0, 0, 0>), dim3(batch), dim3(NT), bf, st, a);
        else hipLaunchKernelGGL((k_eig_fin<false, 0, 0, 0>), dim3(batch), dim3(NT), 0, st, a);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;

    const size_t br = (size_t)(L.mp + L.np) * L.tk * sizeof(double);
    if (br <= cap / 2) hipLaunchKernelGGL(k_eig_refine<true>, dim3(batch), dim3(NT), br, st, a);
    else hipLaunchKernelGGL(k_eig_refine<false>, dim3(batch), dim3(NT), 0, st, a);
    return hipGetLastError();
}

}  // namespace peps
