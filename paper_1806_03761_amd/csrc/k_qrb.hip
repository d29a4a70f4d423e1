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
__global__ __launch_bounds__(WG) void k_qrb_panel(double* X, long long xs, int m, int n, int k0, double* tau,
                                                  long long ts, double* Tw, long long tws) {
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
    for (int j = 0; j < nref; ++j) {
        const int c = k0 + j;
        // squared norm below the pivot and the pivot entry
        double x2[2] = {0.0, 0.0}, s2[2];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = k0 + tid + WG * q;
#pragma unroll
            for (int jj = 0; jj < PW; ++jj) {
                if (jj != j) continue;
                x2[0] += (i > c && i < m) ? a[q][jj] * a[q][jj] : 0.0;
                x2[1] += (i == c) ? a[q][jj] : 0.0;
            }
        }
        block_sums<WG, 2>(x2, s2, red);
        const double s = s2[0], al = s2[1];
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
#pragma unroll
            for (int jj = 0; jj < PW; ++jj) {
                if (jj != j) continue;
                const double v = (i < c || i >= m) ? 0.0 : (i == c ? 1.0 : (tk != 0.0 ? sc * a[q][jj] : 0.0));
                vq[q] = v;
                if (i == c) a[q][jj] = be;
                else if (i > c && i < m && tk != 0.0) a[q][jj] = v;
            }
        }
        if (tk == 0.0 || j + 1 >= nc) continue;     // uniform over the workgroup
        // the reflector applied to the remaining panel columns
        double d[PW];
#pragma unroll
        for (int jj = 0; jj < PW; ++jj) {
            d[jj] = 0.0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) d[jj] = fma(vq[q], a[q][jj], d[jj]);
        }
        block_sums<WG, PW>(d, d, red);
#pragma unroll
        for (int jj = 0; jj < PW; ++jj) {
            if (jj <= j) continue;
            const double f = tk * d[jj];
#pragma unroll
            for (int q = 0; q < RPT; ++q) a[q][jj] = fma(-f, vq[q], a[q][jj]);
        }
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
    // T (upper triangular): T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^T v_j)
    if (tid < 256) Ts[tid] = 0.0;
    __syncthreads();
    if (tid == 0) {
        for (int j = 0; j < nref; ++j) {
            Ts[j * NB + j] = tvs[j];
            for (int i = 0; i < j; ++i) {
                double s = 0.0;
                for (int k = i; k < j; ++k) {
                    const int e = k * 16 + j;
                    s += Ts[i * NB + k] * (vtv[e] + vtv[256 + e] + vtv[512 + e] + vtv[768 + e]);
                }
                Ts[i * NB + j] = -tvs[j] * s;
            }
        }
    }
    __syncthreads();
    if (tid < 256) Tw[(long long)b * tws + (long long)(k0 / PW) * NB * NB + tid] = Ts[tid];
    if (tid < nref) tau[(long long)b * ts + k0 + tid] = tvs[tid];
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
    return (long long)((r + pw - 1) / pw) * NB * NB;
}

bool qrb_fits(int m, int n) { return m <= 4096 && n >= 1; }

hipError_t launch_qr_blocked(double* X, long long xs, int m, int n, double* R, long long rs, double* tau, long long ts,
                             double* Tw, long long tws, int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    if (!qrb_fits(m, n)) return hipErrorInvalidValue;
    const int r = m < n ? m : n, pw = qrb_panel_width(m);
    for (int k0 = 0; k0 < r; k0 += pw) {
        const int rows = m - k0;
        if (rows <= 256 * 2) panel_t<2, 256, 16>(X, xs, m, n, k0, tau, ts, Tw, tws, batch, st);
        else if (rows <= 512 * 3) panel_t<3, 512, 16>(X, xs, m, n, k0, tau, ts, Tw, tws, batch, st);
        else panel_t<8, 512, 8>(X, xs, m, n, k0, tau, ts, Tw, tws, batch, st);
        const int trail = n - (k0 + pw);
        if (trail > 0) {
            const int cblocks = (trail + 15) / 16;
            hipLaunchKernelGGL(k_qrb_update, dim3((unsigned)(batch * cblocks)), dim3(256), 0, st, X, xs, m, n, k0, pw,
                               Tw, tws, cblocks);
        }
    }
    hipLaunchKernelGGL(k_qrb_r, dim3((unsigned)std::min<long long>(((long long)r * n + 255) / 256, 1024), batch),
                       dim3(256), 0, st, X, xs, m, n, R, rs);
    return hipGetLastError();
}

hipError_t launch_applyq_blocked(const double* V, long long vs, int mz, int nrefl, const double* Tw, long long tws,
                                 const double* G, long long gs, int rin, int tin, double* Z, long long zs, int ldz,
                                 int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    const int cblocks = (tin + 15) / 16;
    hipLaunchKernelGGL(k_qrb_applyq, dim3((unsigned)(batch * cblocks)), dim3(256), 0, st, V, vs, mz, nrefl,
                       qrb_panel_width(mz), Tw, tws, G, gs, rin, tin, Z, zs, ldz, cblocks);
    return hipGetLastError();
}

}  // namespace peps
