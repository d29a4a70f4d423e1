// Blocked Householder QR of tall column tensors (the left-to-right canonicalisation
// sweep of the boundary-MPS truncation, Fig. 1(c); QR as in Sec. II-C) and the blocked
// application of its Q, for matrices too large to stay on chip.
//
// The reflectors are grouped in panels of NB = 16 columns in compact WY form,
// Q_b = H_k0 ... H_{k0+15} = I - V T V^T (T upper triangular, LAPACK's forward
// column-wise convention), and every reflector keeps the dlarfg convention of the
// register kernels (v_k = 1 at the pivot, stored below the diagonal of X, tau[k]).
//
//   k_qrb_panel   one workgroup per matrix: the 16 columns of the panel (already
//                 updated by the earlier panels) factorised in registers, T formed
//                 from the reflectors' inner products;
//   k_qrb_update  one workgroup per (matrix, block of 16 trailing columns): A <- Q_b^T A
//                 as W = V^T A, W <- T^T W, A -= V W, on the matrix cores
//                 (v_mfma_f64_16x16x4f64);
//   k_qrb_applyq  Z = Q [G; 0] = Q_1 (Q_2 (... Q_p [G; 0])) for the right-to-left sweep,
//                 one workgroup per (matrix, block of 16 columns of Z), all panels in
//                 one launch;
//   k_qrb_r       R (row-major, zeros below the diagonal) from the upper triangle.
#include "common.h"
#include "kernels.h"

namespace peps {

namespace {

constexpr int NB = 16;
typedef double d4v __attribute__((ext_vector_type(4)));

// reflector j of a panel starting at column k0: entry i (row) of v_j
__device__ __forceinline__ double v_at(const double* V, long long ldv, int k0, int j, int nref, int i, int m) {
    const int piv = k0 + j;
    if (j >= nref || i < piv || i >= m) return 0.0;
    return i == piv ? 1.0 : V[(long long)piv * ldv + i];
}

// Sum over the workgroup of NV values per thread; red holds (WG / 64) * NV doubles.
// Every thread gets all NV totals in out.  Two barriers.
template <int WG, int NV>
__device__ __forceinline__ void block_sums(const double (&x)[NV], double (&out)[NV], double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double s = lane_group_sum(x[v], 64);
        if (lane == 0) red[w * NV + v] = s;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < WG / 64; ++u) s += red[u * NV + v];
        out[v] = s;
    }
    __syncthreads();
}

// Thread t owns rows k0 + t + WG q (q < RPT) of the PW panel columns (PW = 16, or 8
// for the tallest matrices so the panel stays in registers).  The WY blocks are always
// stored as 16 x 16 T matrices (zero beyond the panel's reflectors), T of panel p at p*256.
template <int RPT, int WG, int PW>
__device__ __forceinline__ void qrb_panel(double* X, long long xs, int m, int n, int k0, double* tau, long long ts,
                                          double* Tw, long long tws) {
    __shared__ double red[(WG / 64) * PW];
    __shared__ double vtv[4 * 256];
    __shared__ double Ts[NB * NB];
    __shared__ double tvs[NB];
    const int b = blockIdx.x, tid = threadIdx.x;
    double* Xb = X + (long long)b * xs;
    const int r = min(m, n);
    const int nc = min(PW, n - k0);          // panel columns
    const int nref = min(PW, r - k0);        // reflectors of this panel
    double a[RPT][PW];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = k0 + tid + WG * q;
#pragma unroll
        for (int j = 0; j < PW; ++j) a[q][j] = (i < m && j < nc) ? Xb[(long long)(k0 + j) * m + i] : 0.0;
    }
    // the step loop is unrolled so that every register column index is a constant
    const int lane = tid & 63, wv = tid >> 6;
#pragma clang loop unroll(full)
    for (int j = 0; j < PW; ++j) {
        if (j >= nref) continue;   // uniform
        const int c = k0 + j;
        // squared norm below the pivot and the pivot entry
        double x0 = 0.0, x1 = 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = k0 + tid + WG * q;
            x0 += (i > c && i < m) ? a[q][j] * a[q][j] : 0.0;
            x1 += (i == c) ? a[q][j] : 0.0;
        }
        x0 = lane_group_sum(x0, 64);
        x1 = lane_group_sum(x1, 64);
        if (lane == 0) {
            red[wv * 2] = x0;
            red[wv * 2 + 1] = x1;
        }
        __syncthreads();
        double s = 0.0, al = 0.0;
#pragma unroll
        for (int u = 0; u < WG / 64; ++u) {
            s += red[u * 2];
            al += red[u * 2 + 1];
        }
        __syncthreads();
        double tk, be, sc;
        if (s == 0.0) {
            tk = 0.0; be = al; sc = 0.0;
        } else {
            be = -copysign(sqrt(al * al + s), al);
            tk = (be - al) / be;
            sc = 1.0 / (al - be);
        }
        if (tid == 0) tvs[j] = tk;
        // v (unit pivot) replaces column j below the pivot; beta is the diagonal of R
        double vq[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = k0 + tid + WG * q;
            const double v = (i < c || i >= m) ? 0.0 : (i == c ? 1.0 : (tk != 0.0 ? sc * a[q][j] : 0.0));
            vq[q] = v;
            if (i == c) a[q][j] = be;
            else if (i > c && i < m && tk != 0.0) a[q][j] = v;
        }
        if (tk == 0.0 || j + 1 >= nc) continue;     // uniform over the workgroup
        // the reflector applied to the remaining panel columns: their dot products with v
        // summed over the workgroup in one pass
#pragma unroll
        for (int jj = j + 1; jj < PW; ++jj) {
            double d = 0.0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) d = fma(vq[q], a[q][jj], d);
            d = lane_group_sum(d, 64);
            if (lane == 0) red[wv * PW + jj] = d;
        }
        __syncthreads();
#pragma unroll
        for (int jj = j + 1; jj < PW; ++jj) {
            double d = 0.0;
#pragma unroll
            for (int u = 0; u < WG / 64; ++u) d += red[u * PW + jj];
            const double f = tk * d;
#pragma unroll
            for (int q = 0; q < RPT; ++q) a[q][jj] = fma(-f, vq[q], a[q][jj]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = k0 + tid + WG * q;
        if (i >= m) continue;
#pragma unroll
        for (int j = 0; j < PW; ++j)
            if (j < nc) Xb[(long long)(k0 + j) * m + i] = a[q][j];
    }
    __syncthreads();
    // V^T V of the reflectors (unit pivots, zeros above) on the matrix cores, rows split
    // over the first four waves, read back from X
    if (tid < 256) {
        const int lane = tid & 63, w = tid >> 6, li = lane & 15, gq = lane >> 4;
        d4v acc = {0.0, 0.0, 0.0, 0.0};
        for (int r0 = k0 + 32 * w; r0 < m; r0 += 128) {
            double va[8];
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) va[s8] = v_at(Xb, m, k0, li, nref, r0 + 8 * gq + s8, m);
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[s8], va[s8], acc, 0, 0, 0);
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) vtv[w * 256 + (gq + 4 * rr) * 16 + li] = acc[rr];
    }
    __syncthreads();
    // T (upper triangular): T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^T v_j).
    // Row i of T only needs its own earlier entries, so lane i of the first wave forms it.
    if (tid < 256) vtv[tid] = vtv[tid] + vtv[256 + tid] + vtv[512 + tid] + vtv[768 + tid];
    __syncthreads();
    if (tid < NB) {
        const int i = tid;
        double row[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) row[j] = 0.0;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j >= nref || j < i) continue;
            if (j == i) {
                row[j] = tvs[j];
            } else {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    if (k >= i && k < j) s = fma(row[k], vtv[k * 16 + j], s);
                row[j] = -tvs[j] * s;
            }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) Ts[i * NB + j] = row[j];
    }
    __syncthreads();
    if (tid < 256) Tw[(long long)b * tws + (long long)(k0 / PW) * NB * NB + tid] = Ts[tid];
    if (tid < nref) tau[(long long)b * ts + k0 + tid] = tvs[tid];
}

template <int RPT, int WG, int PW>
__global__ __launch_bounds__(WG) void k_qrb_panel(double* X, long long xs, int m, int n, int k0, double* tau,
                                                  long long ts, double* Tw, long long tws) {
    qrb_panel<RPT, WG, PW>(X, xs, m, n, k0, tau, ts, Tw, tws);
}

// A <- op(Q_b)^T-style update of columns [c0, c0 + 16) of A over rows [k0, m):
//   W = V^T A;  W <- T^T W (trans = 1, the QR) or T W (trans = 0, applying Q);  A -= V W.
// V: reflectors of the panel at column k0 (ld ldv, unit pivots implicit), T row-major 16 x 16.
// Four waves split the rows; W is reduced through LDS.
__device__ __forceinline__ void wy_block(const double* V, long long ldv, int k0, int nref, const double* T,
                                         int trans, double* A, long long lda, int c0, int ncols, int m,
                                         double* sh /* 4*256 + 256 + 256 doubles */) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, gq = lane >> 4;
    // phase 1: W[j][c] = sum_i V[i][j] A[i][c0 + c], rows in chunks of 32 (lane: 8 rows)
    d4v acc = {0.0, 0.0, 0.0, 0.0};
    const bool colok = li < ncols;
    for (int r0 = k0 + 32 * w; r0 < m; r0 += 128) {
        double va[8], aa[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int i = r0 + 8 * gq + s;
            va[s] = v_at(V, ldv, k0, li, nref, i, m);
            aa[s] = (colok && i < m) ? A[(long long)(c0 + li) * lda + i] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 8; s += 2) {
            // MFMA s: k index gq <-> row r0 + 8 gq + s (a permutation of the rows of the chunk)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[s], aa[s], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[s + 1], aa[s + 1], acc, 0, 0, 0);
        }
    }
    // lane holds W[j = gq + 4 rr][c = li]
    double* red = sh;                 // [4][256]
    double* Wm = sh + 4 * 256;        // [16][16]
    double* W2 = sh + 5 * 256;        // [16][16]
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) red[w * 256 + (gq + 4 * rr) * 16 + li] = acc[rr];
    __syncthreads();
    {
        const double s = red[tid] + red[256 + tid] + red[512 + tid] + red[768 + tid];
        Wm[tid] = s;
    }
    __syncthreads();
    {
        const int aa = tid >> 4, c = tid & 15;
        double s = 0.0;
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
            const double t = trans ? T[bb * NB + aa] : T[aa * NB + bb];
            s = fma(t, Wm[bb * 16 + c], s);
        }
        W2[tid] = s;
    }
    __syncthreads();
    // phase 3: A[i][c0 + c] -= sum_j V[i][j] W2[j][c]; computed transposed so that lane
    // (li, gq) holds A[r0 + li][c0 + gq + 4 rr] (consecutive lanes, consecutive rows)
    for (int r0 = k0 + 16 * w; r0 < m; r0 += 64) {
        const int i = r0 + li;
        d4v cacc;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int c = gq + 4 * rr;
            cacc[rr] = (c < ncols && i < m) ? A[(long long)(c0 + c) * lda + i] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int j = 4 * s + gq;
            const double aop = -W2[j * 16 + li];          // (W2^T)[c = li][j]
            const double bop = v_at(V, ldv, k0, j, nref, i, m);   // (V^T)[j][row li]
            cacc = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop, cacc, 0, 0, 0);
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int c = gq + 4 * rr;
            if (c < ncols && i < m) A[(long long)(c0 + c) * lda + i] = cacc[rr];
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_qrb_update(double* X, long long xs, int m, int n, int k0, int pw,
                                                    const double* Tw, long long tws, int cblocks) {
    __shared__ double sh[6 * 256];
    const int b = blockIdx.x / cblocks, cb = blockIdx.x % cblocks;
    double* Xb = X + (long long)b * xs;
    const int r = min(m, n);
    const int nref = min(pw, r - k0);
    const int c0 = k0 + pw + 16 * cb;
    const int ncols = min(16, n - c0);
    if (ncols <= 0) return;
    const double* T = Tw + (long long)b * tws + (long long)(k0 / pw) * NB * NB;
    wy_block(Xb, m, k0, nref, T, 1, Xb, m, c0, ncols, m, sh);
}

// Z (column-major, ld ldz, mz rows, tin columns) = Q [G; 0] with G row-major rin x tin.
__global__ __launch_bounds__(256) void k_qrb_applyq(const double* V, long long vs, int mz, int nrefl, int pw,
                                                    const double* Tw, long long tws, const double* G, long long gs,
                                                    int rin, int tin, double* Z, long long zs, int ldz,
                                                    int cblocks) {
    __shared__ double sh[6 * 256];
    const int b = blockIdx.x / cblocks, cb = blockIdx.x % cblocks;
    const int c0 = 16 * cb, ncols = min(16, tin - c0);
    const double* Vb = V + (long long)b * vs;
    const double* Gb = G + (long long)b * gs;
    double* Zb = Z + (long long)b * zs;
    const int tid = threadIdx.x;
    for (int e = tid; e < 16 * mz; e += 256) {
        const int c = e / mz, i = e % mz;
        if (c < ncols) Zb[(long long)(c0 + c) * ldz + i] = i < rin ? Gb[(long long)i * tin + c0 + c] : 0.0;
    }
    __syncthreads();
    const int np = (nrefl + pw - 1) / pw;
    for (int p = np - 1; p >= 0; --p) {
        const int k0 = p * pw;
        const int nref = min(pw, nrefl - k0);
        wy_block(Vb, mz, k0, nref, Tw + (long long)b * tws + (long long)p * NB * NB, 0, Zb, ldz, c0, ncols, mz, sh);
    }
}

__global__ __launch_bounds__(256) void k_qrb_r(const double* X, long long xs, int m, int n, double* R, long long rs) {
    const int b = blockIdx.y;
    const int r = min(m, n);
    const double* Xb = X + (long long)b * xs;
    double* Rb = R + (long long)b * rs;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < (long long)r * n; e += 256LL * gridDim.x) {
        const int i = (int)(e / n), c = (int)(e % n);
        Rb[e] = i <= c ? Xb[(long long)c * m + i] : 0.0;
    }
}

// The reflectors of the 32 columns [k0, k0 + 32) as a plain column-major matrix Vc
// (rows [k0, m), stride ldc = m - k0 rounded up): zero above the pivot, one on it.
__global__ __launch_bounds__(256) void k_qrb_vclean(const double* X, long long xs, int m, int k0, int nref,
                                                    double* Vc, long long vcs, int ldc) {
    const int b = blockIdx.y;
    const double* Xb = X + (long long)b * xs;
    double* Vb = Vc + (long long)b * vcs;
    const int rows = m - k0;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < 32LL * rows; e += 256LL * gridDim.x) {
        const int j = (int)(e / rows), i = k0 + (int)(e % rows);
        const int piv = k0 + j;
        double v = 0.0;
        if (j < nref && i >= piv) v = i == piv ? 1.0 : Xb[(long long)piv * m + i];
        Vb[(long long)j * ldc + (i - k0)] = v;
    }
}

// T of the 32 reflectors: [[T1, -T1 (V1^T V2) T2], [0, T2]] from the two 16-column blocks
// (Q = Q1 Q2 = I - V T V^T).  V1^T V2 over the rows of Vc on the matrix cores.
__global__ __launch_bounds__(256) void k_qrb_t32(const double* Vc, long long vcs, int rows, int ldc,
                                                 const double* T16, double* T32, long long tws) {
    __shared__ double red[4 * 256];
    __shared__ double S[256], P[256];
    const int b = blockIdx.x, tid = threadIdx.x;
    const double* Vb = Vc + (long long)b * vcs;
    const double* T1 = T16 + (long long)b * tws;
    const double* T2 = T1 + 256;
    double* To = T32 + (long long)b * tws;
    const int lane = tid & 63, w = tid >> 6, li = lane & 15, gq = lane >> 4;
    d4v acc = {0.0, 0.0, 0.0, 0.0};
    for (int r0 = 32 * w; r0 < rows; r0 += 128) {
#pragma unroll
        for (int s8 = 0; s8 < 8; ++s8) {
            const int i = r0 + 8 * gq + s8;
            const double a1 = i < rows ? Vb[(long long)li * ldc + i] : 0.0;          // V1^T[li][i]
            const double a2 = i < rows ? Vb[(long long)(16 + li) * ldc + i] : 0.0;   // V2[i][li]
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a2, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) red[w * 256 + (gq + 4 * rr) * 16 + li] = acc[rr];
    __syncthreads();
    S[tid] = red[tid] + red[256 + tid] + red[512 + tid] + red[768 + tid];   // (V1^T V2)[a][c]
    __syncthreads();
    const int a = tid >> 4, c = tid & 15;
    double x = 0.0;
    for (int k = 0; k < 16; ++k) x = fma(S[a * 16 + k], T2[k * 16 + c], x);
    P[tid] = x;                                                            // (V1^T V2) T2
    __syncthreads();
    x = 0.0;
    for (int k = 0; k < 16; ++k) x = fma(T1[a * 16 + k], P[k * 16 + c], x);
    // 32 x 32 row-major
    To[a * 32 + c] = T1[a * 16 + c];
    To[a * 32 + 16 + c] = -x;
    To[(16 + a) * 32 + c] = 0.0;
    To[(16 + a) * 32 + 16 + c] = T2[a * 16 + c];
}

// T of a lone last 16-column panel in the 32 x 32 slot: [[T1, 0], [0, 0]]
__global__ __launch_bounds__(256) void k_qrb_t32_single(const double* T16, double* T32, long long tws) {
    const int b = blockIdx.x, tid = threadIdx.x;
    const double* T1 = T16 + (long long)b * tws;
    double* To = T32 + (long long)b * tws;
    for (int e = tid; e < 1024; e += 256) {
        const int a = e / 32, c = e % 32;
        To[e] = (a < 16 && c < 16) ? T1[a * 16 + c] : 0.0;
    }
}

// After R has been copied out: the reflector columns of X become plain unit lower
// trapezoidal vectors (zero above the pivot, one on it), so the application of Q can
// read them as a GEMM operand.
__global__ __launch_bounds__(256) void k_qrb_clean(double* X, long long xs, int m, int r) {
    const int b = blockIdx.y;
    double* Xb = X + (long long)b * xs;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < (long long)r * r; e += 256LL * gridDim.x) {
        const int j = (int)(e / r), i = (int)(e % r);   // column j, row i <= pivot rows
        if (i < j) Xb[(long long)j * m + i] = 0.0;
        else if (i == j) Xb[(long long)j * m + i] = 1.0;
    }
}

// Z = [G; 0] (column-major, ld ldz) from G row-major rin x tin
__global__ __launch_bounds__(256) void k_qrb_zinit(const double* G, long long gs, int rin, int tin, double* Z,
                                                   long long zs, int ldz, int mz) {
    const int b = blockIdx.y;
    const double* Gb = G + (long long)b * gs;
    double* Zb = Z + (long long)b * zs;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < (long long)mz * tin; e += 256LL * gridDim.x) {
        const int c = (int)(e / mz), i = (int)(e % mz);
        Zb[(long long)c * ldz + i] = i < rin ? Gb[(long long)i * tin + c] : 0.0;
    }
}

template <int RPT, int WG, int PW>
void panel_t(double* X, long long xs, int m, int n, int k0, double* tau, long long ts, double* Tw, long long tws,
             int batch, hipStream_t st) {
    hipLaunchKernelGGL((k_qrb_panel<RPT, WG, PW>), dim3(batch), dim3(WG), 0, st, X, xs, m, n, k0, tau, ts, Tw, tws);
}

}  // namespace

// panel width of the blocked QR of an m-row matrix (8 for the tallest, so the panel
// stays in registers)
int qrb_panel_width(int m) { return m <= 1536 ? 16 : 8; }

long long qrb_wy_doubles(int m, int n) {
    const int r = m < n ? m : n, pw = qrb_panel_width(m);
    return (long long)((r + pw - 1) / pw) * NB * NB + (long long)((r + 31) / 32) * 1024;
}

// per-matrix scratch of the 32-reflector updates: Vc (rows rounded to 16, 32 columns) and W
// (two 32 x n blocks)
long long qrb_vc_doubles(int m) { return (long long)((m + 15) / 16 * 16) * 32; }
long long qrb_wq_doubles(int n) { return 64LL * n; }

bool qrb_fits(int m, int n) { return m <= 4096 && n >= 1; }

hipError_t launch_qr_blocked(double* X, long long xs, int m, int n, double* R, long long rs, double* tau, long long ts,
                             double* Tw, long long tws, double* Vc, long long vcs, double* Wq, long long wqs, int batch,
                             hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    if (!qrb_fits(m, n)) return hipErrorInvalidValue;
    const int r = m < n ? m : n, pw = qrb_panel_width(m);
    const long long nt16 = (long long)((r + pw - 1) / pw) * NB * NB;   // 16-column T blocks, then 32-column ones
    auto panel = [&](int k0) {
        const int rows = m - k0;
        if (rows <= 256 * 2) panel_t<2, 256, 16>(X, xs, m, n, k0, tau, ts, Tw, tws, batch, st);
        else if (rows <= 256 * 6) panel_t<6, 256, 16>(X, xs, m, n, k0, tau, ts, Tw, tws, batch, st);
        else panel_t<8, 512, 8>(X, xs, m, n, k0, tau, ts, Tw, tws, batch, st);
    };
    auto update16 = [&](int k0, int cend) {
        // columns [k0 + pw, cend) with the WY block of the panel at k0
        const int trail = cend - (k0 + pw);
        if (trail <= 0) return;
        const int cblocks = (trail + 15) / 16;
        hipLaunchKernelGGL(k_qrb_update, dim3((unsigned)(batch * cblocks)), dim3(256), 0, st, X, xs, m, cend, k0, pw,
                           Tw, tws, cblocks);
    };
    for (int k0 = 0; k0 < r; k0 += 2 * pw) {
        panel(k0);
        if (pw != 16 || k0 + pw >= r || !Vc) {
            // a single panel (the last one, or narrow panels): its own trailing update
            if (pw == 16 && k0 + pw >= r)
                hipLaunchKernelGGL(k_qrb_t32_single, dim3(batch), dim3(256), 0, st, Tw + (long long)(k0 / pw) * NB * NB,
                                   Tw + nt16 + (long long)(k0 / 32) * 1024, tws);
            update16(k0, n);
            if (k0 + pw < r) {
                panel(k0 + pw);
                update16(k0 + pw, n);
            }
            continue;
        }
        // two 16-column panels: the second is updated by the first, factorised, then the
        // trailing columns take both at once as one 32-reflector WY update, two GEMMs on the
        // matrix cores: W = T^T (V^T A), A -= V W
        update16(k0, std::min(n, k0 + 2 * pw));
        panel(k0 + pw);
        const int c0 = k0 + 2 * pw, nt = n - c0, rows = m - k0;
        const int nref = std::min(2 * pw, r - k0);
        const int ldc = (rows + 15) / 16 * 16;
        // the 32-reflector T is also what the later application of Q uses, so it is formed
        // even when no trailing column is left
        hipLaunchKernelGGL(k_qrb_vclean, dim3((unsigned)std::min(((long long)32 * rows + 255) / 256, 512LL), batch),
                           dim3(256), 0, st, X, xs, m, k0, nref, Vc, vcs, ldc);
        double* T32 = Tw + nt16 + (long long)(k0 / 32) * 1024;
        hipLaunchKernelGGL(k_qrb_t32, dim3(batch), dim3(256), 0, st, Vc, vcs, rows, ldc,
                           Tw + (long long)(k0 / pw) * NB * NB, T32, tws);
        if (nt <= 0) continue;
        GemmArgs g{};
        // W0 (32 x nt, row-major) = Vc^T A[k0:, c0:]
        g.M = 32; g.N = nt; g.K = rows; g.batch = batch;
        g.am = Idx2{1 << 30, 0, ldc}; g.ak = Idx2{1 << 30, 0, 1};
        g.bk = Idx2{1 << 30, 0, 1}; g.bn = Idx2{1 << 30, 0, m};
        g.cm = Idx2{1 << 30, 0, nt}; g.cn = Idx2{1 << 30, 0, 1};
        g.a_bs = vcs; g.b_bs = xs; g.c_bs = wqs;
        g.A = Vc; g.B = X + (long long)c0 * m + k0; g.C = Wq;
        g.alpha = 1.0; g.beta = 0.0;
        hipError_t e = launch_mgemm(g, Arith::F64, st, 0);
        if (e != hipSuccess) return e;
        // W (32 x nt, after W0) = T^T W0
        GemmArgs h{};
        h.M = 32; h.N = nt; h.K = 32; h.batch = batch;
        h.am = Idx2{1 << 30, 0, 1}; h.ak = Idx2{1 << 30, 0, 32};       // T^T[a][k] = T[k][a]
        h.bk = Idx2{1 << 30, 0, nt}; h.bn = Idx2{1 << 30, 0, 1};
        h.cm = Idx2{1 << 30, 0, nt}; h.cn = Idx2{1 << 30, 0, 1};
        h.a_bs = tws; h.b_bs = wqs; h.c_bs = wqs;
        h.A = T32; h.B = Wq; h.C = Wq + 32LL * nt;
        h.alpha = 1.0; h.beta = 0.0;
        e = launch_mgemm(h, Arith::F64, st, 0);
        if (e != hipSuccess) return e;
        // A[k0:, c0:] -= Vc W
        GemmArgs u{};
        u.M = rows; u.N = nt; u.K = 32; u.batch = batch;
        u.am = Idx2{1 << 30, 0, 1}; u.ak = Idx2{1 << 30, 0, ldc};
        u.bk = Idx2{1 << 30, 0, nt}; u.bn = Idx2{1 << 30, 0, 1};
        u.cm = Idx2{1 << 30, 0, 1}; u.cn = Idx2{1 << 30, 0, m};
        u.a_bs = vcs; u.b_bs = wqs; u.c_bs = xs;
        u.A = Vc; u.B = Wq + 32LL * nt; u.C = X + (long long)c0 * m + k0;
        u.alpha = -1.0; u.beta = 1.0;
        e = launch_mgemm(u, Arith::F64, st, 0);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_qrb_r, dim3((unsigned)std::min<long long>(((long long)r * n + 255) / 256, 1024), batch),
                       dim3(256), 0, st, X, xs, m, n, R, rs);
    if (pw == 16)
        hipLaunchKernelGGL(k_qrb_clean, dim3((unsigned)std::min<long long>(((long long)r * r + 255) / 256, 1024), batch),
                           dim3(256), 0, st, X, xs, m, r);
    return hipGetLastError();
}

hipError_t launch_applyq_blocked(const double* V, long long vs, int mz, int nrefl, const double* Tw, long long tws,
                                 const double* G, long long gs, int rin, int tin, double* Z, long long zs, int ldz,
                                 double* Wq, long long wqs, int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    const int pw = qrb_panel_width(mz);
    if (pw != 16 || !Wq) {
        const int cblocks = (tin + 15) / 16;
        hipLaunchKernelGGL(k_qrb_applyq, dim3((unsigned)(batch * cblocks)), dim3(256), 0, st, V, vs, mz, nrefl, pw,
                           Tw, tws, G, gs, rin, tin, Z, zs, ldz, cblocks);
        return hipGetLastError();
    }
    // Z = [G; 0], then Q_p ... applied last block first as GEMMs on the plain reflectors of
    // X (k_qrb_clean): W0 = V^T Z, W = T W0, Z -= V W, 32 reflectors at a time
    hipLaunchKernelGGL(k_qrb_zinit, dim3((unsigned)std::min<long long>(((long long)mz * tin + 255) / 256, 512), batch),
                       dim3(256), 0, st, G, gs, rin, tin, Z, zs, ldz, mz);
    const long long nt16 = (long long)((nrefl + pw - 1) / pw) * NB * NB;
    for (int k0 = (nrefl - 1) / 32 * 32; k0 >= 0; k0 -= 32) {
        const int nref = std::min(32, nrefl - k0), rows = mz - k0;
        const double* T32 = Tw + nt16 + (long long)(k0 / 32) * 1024;
        GemmArgs g{};
        g.M = nref; g.N = tin; g.K = rows; g.batch = batch;
        g.am = Idx2{1 << 30, 0, mz}; g.ak = Idx2{1 << 30, 0, 1};
        g.bk = Idx2{1 << 30, 0, 1}; g.bn = Idx2{1 << 30, 0, ldz};
        g.cm = Idx2{1 << 30, 0, tin}; g.cn = Idx2{1 << 30, 0, 1};
        g.a_bs = vs; g.b_bs = zs; g.c_bs = wqs;
        g.A = V + (long long)k0 * mz + k0; g.B = Z + k0; g.C = Wq;
        g.alpha = 1.0; g.beta = 0.0;
        hipError_t e = launch_mgemm(g, Arith::F64, st, 0);
        if (e != hipSuccess) return e;
        GemmArgs h{};
        h.M = nref; h.N = tin; h.K = nref; h.batch = batch;
        h.am = Idx2{1 << 30, 0, 32}; h.ak = Idx2{1 << 30, 0, 1};
        h.bk = Idx2{1 << 30, 0, tin}; h.bn = Idx2{1 << 30, 0, 1};
        h.cm = Idx2{1 << 30, 0, tin}; h.cn = Idx2{1 << 30, 0, 1};
        h.a_bs = tws; h.b_bs = wqs; h.c_bs = wqs;
        h.A = T32; h.B = Wq; h.C = Wq + 32LL * tin;
        h.alpha = 1.0; h.beta = 0.0;
        e = launch_mgemm(h, Arith::F64, st, 0);
        if (e != hipSuccess) return e;
        GemmArgs u{};
        u.M = rows; u.N = tin; u.K = nref; u.batch = batch;
        u.am = Idx2{1 << 30, 0, 1}; u.ak = Idx2{1 << 30, 0, mz};
        u.bk = Idx2{1 << 30, 0, tin}; u.bn = Idx2{1 << 30, 0, 1};
        u.cm = Idx2{1 << 30, 0, 1}; u.cn = Idx2{1 << 30, 0, ldz};
        u.a_bs = vs; u.b_bs = wqs; u.c_bs = zs;
        u.A = V + (long long)k0 * mz + k0; u.B = Wq + 32LL * tin; u.C = Z + k0;
        u.alpha = -1.0; u.beta = 1.0;
        e = launch_mgemm(u, Arith::F64, st, 0);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace peps
