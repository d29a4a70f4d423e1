// Kernels of the variational boundary compression (one-site alternating least squares,
// the truncation alternative of Sec. II-A): the thin QR that turns an updated site
// tensor into an isometry, and the normalisation of the final site.  The contractions
// of the sweeps are batched GEMMs (k_mgemm.hip).
#include "common.h"
#include "kernels.h"

namespace peps {

static constexpr int VT = 256;           // threads of the small kernels
static constexpr int kThinqMaxN = 128;   // columns

__device__ inline double vq_wsum(double v) { return lane_group_sum(v, 64); }

template <int NT>
__device__ inline double vq_bsum(double v, double* red) {
    v = vq_wsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}

// One wave applies H = I - tk v v^T (v_k = 1, v_i = a[k m + i] below row k) to the up to
// G columns j0..j0+G-1 (< n) of a, rows k..m-1: the G dot products share every load of v
// and are reduced together.
template <int G>
__device__ inline void vq_reflect(double* a, int m, int n, int k, int j0, double tk, int lane) {
    const double* vk = a + (long long)k * m;
    double* c0 = a + (long long)j0 * m;
    const int nc = min(G, n - j0);
    double d[G];
#pragma unroll
    for (int c = 0; c < G; ++c) d[c] = (lane == 0 && c < nc) ? c0[(long long)c * m + k] : 0.0;
    for (int i = k + 1 + lane; i < m; i += 64) {
        const double v = vk[i];
#pragma unroll
        for (int c = 0; c < G; ++c)
            if (c < nc) d[c] += v * c0[(long long)c * m + i];
    }
#pragma unroll
    for (int c = 0; c < G; ++c) d[c] = vq_wsum(d[c]) * tk;
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < G; ++c)
            if (c < nc) c0[(long long)c * m + k] -= d[c];
    }
    for (int i = k + 1 + lane; i < m; i += 64) {
        const double v = vk[i];
#pragma unroll
        for (int c = 0; c < G; ++c)
            if (c < nc) c0[(long long)c * m + i] -= d[c] * v;
    }
}

// Thin Householder QR of one m x n matrix (m >= n) per workgroup of NT threads, held in
// LDS (IN_LDS) or in the workgroup's slice of a global scratch buffer (W + b ws, m n
// doubles; the waves of a workgroup share one CU, so its barriers order those accesses as
// they do LDS ones):
//   X: column-major, leading dimension m, stride xs per matrix (may equal Q: every
//      element is read before any is written);
//   Q: the m x n factor with the signs fixed so that diag(R) >= 0, element (i, k) at
//      Q + b qs + i q_row + k q_col;
//   R: when not null, the n x n factor (row-major, zeros below the diagonal), stride rs.
// Reflectors follow the usual convention (beta = -sign(alpha) ||x||, tau = (beta -
// alpha) / beta); a column with nothing below the diagonal gives tau = 0.  Q is formed
// in place by applying the reflectors backwards to the leading n columns of I.  Each
// wave updates groups of G trailing columns.
template <int NT, bool IN_LDS, int G>
__global__ __launch_bounds__(NT) void k_thinq(const double* X, long long xs, int m, int n, double* Q,
                                              long long qs, long long q_row, long long q_col, double* R,
                                              long long rs, double* W, long long ws) {
    constexpr int NW = NT / 64;
    extern __shared__ double lds[];
    __shared__ double tau[kThinqMaxN], sg[kThinqMaxN], red[NW];
    const int b = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
    double* a = IN_LDS ? lds : W + (long long)b * ws;
    const double* Xb = X + (long long)b * xs;
    const int mn = m * n;
    for (int i = t; i < mn; i += NT) a[i] = Xb[i];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        double* ak = a + (long long)k * m;
        double s = 0.0;
        for (int i = k + 1 + t; i < m; i += NT) s += ak[i] * ak[i];
        s = vq_bsum<NT>(s, red);
        const double alpha = ak[k];
        double tk = 0.0, beta = alpha;
        if (s > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + s), alpha);
            tk = (beta - alpha) / beta;
            const double sc = 1.0 / (alpha - beta);
            for (int i = k + 1 + t; i < m; i += NT) ak[i] *= sc;
        }
        __syncthreads();
        if (t == 0) {
            ak[k] = beta;
            tau[k] = tk;
        }
        if (tk != 0.0)
            for (int j0 = k + 1 + G * w; j0 < n; j0 += G * NW) vq_reflect<G>(a, m, n, k, j0, tk, lane);
        __syncthreads();
    }
    for (int k = t; k < n; k += NT) sg[k] = a[k + (long long)k * m] < 0.0 ? -1.0 : 1.0;
    __syncthreads();
    if (R) {
        double* Rb = R + (long long)b * rs;
        for (int idx = t; idx < n * n; idx += NT) {
            const int k = idx / n, j = idx - k * n;
            Rb[idx] = j >= k ? sg[k] * a[k + (long long)j * m] : 0.0;
        }
    }
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
        double* ak = a + (long long)k * m;
        const double tk = tau[k];
        if (tk != 0.0)
            for (int j0 = k + 1 + G * w; j0 < n; j0 += G * NW) vq_reflect<G>(a, m, n, k, j0, tk, lane);
        __syncthreads();
        for (int i = t; i < m; i += NT) ak[i] = i < k ? 0.0 : (i == k ? 1.0 - tk : -tk * ak[i]);
        __syncthreads();
    }
    double* Qb = Q + (long long)b * qs;
    if (q_row == 1) {
        for (int idx = t; idx < mn; idx += NT) {
            const int k = idx / m, i = idx - k * m;
            Qb[i + (long long)k * q_col] = sg[k] * a[idx];
        }
    } else {
        for (int idx = t; idx < mn; idx += NT) {
            const int i = idx / n, k = idx - i * n;
            Qb[(long long)i * q_row + (long long)k * q_col] = sg[k] * a[i + (long long)k * m];
        }
    }
}

// The same factorisation with the matrix in registers: column j belongs to wave j % NW
// (slot j / NW), its rows i = lane + 64 r (r < RPL) to that wave's lanes, so m <= 64 RPL
// and n <= NW * SL.  Only the current reflector v_k is shared, through a double-buffered
// LDS vector (one barrier per step): the owner of column k forms it with wave reductions,
// every wave applies it to its own trailing columns.  Q is formed in the registers the same
// way, backwards, and stored with the signs that make diag(R) >= 0.
template <int NW, int SL, int RPL>
__global__ __launch_bounds__(NW * 64) void k_thinq_reg(const double* X, long long xs, int m, int n, double* Q,
                                                       long long qs, long long q_row, long long q_col, double* R,
                                                       long long rs) {
    __shared__ double vbuf[2][64 * RPL];
    __shared__ double tau[NW * SL], sg[NW * SL];
    const int b = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double* Xb = X + (long long)b * xs;
    double a[SL][RPL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int j = s * NW + w;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + 64 * r;
            a[s][r] = (j < n && i < m) ? Xb[i + (long long)j * m] : 0.0;
        }
    }
    for (int k = 0; k < n; ++k) {
        double* v = vbuf[k & 1];
        if (w == k % NW) {
            const int sk = k / NW;
            double x[RPL];
#pragma unroll
            for (int s = 0; s < SL; ++s)
                if (s == sk) {
#pragma unroll
                    for (int r = 0; r < RPL; ++r) x[r] = a[s][r];
                }
            double ss = 0.0, al = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                if (i > k && i < m) ss += x[r] * x[r];
                if (i == k) al = x[r];
            }
            ss = vq_wsum(ss);
            al = vq_wsum(al);
            double tk = 0.0, beta = al, sc = 0.0;
            if (ss > 0.0) {
                beta = -copysign(sqrt(al * al + ss), al);
                tk = (beta - al) / beta;
                sc = 1.0 / (al - beta);
            }
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                double vi = 0.0;
                if (i == k) {
                    vi = 1.0;
                    x[r] = beta;
                } else if (i > k && i < m) {
                    vi = ss > 0.0 ? x[r] * sc : 0.0;
                    x[r] = vi;
                }
                v[i] = vi;
            }
#pragma unroll
            for (int s = 0; s < SL; ++s)
                if (s == sk) {
#pragma unroll
                    for (int r = 0; r < RPL; ++r) a[s][r] = x[r];
                }
            if (lane == 0) tau[k] = tk;
        }
        __syncthreads();
        const double tk = tau[k];
        if (tk != 0.0) {
            double vr[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) vr[r] = v[lane + 64 * r];
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const int j = s * NW + w;
                if (j > k && j < n) {
                    double d = 0.0;
#pragma unroll
                    for (int r = 0; r < RPL; ++r) d += vr[r] * a[s][r];
                    d = vq_wsum(d) * tk;
#pragma unroll
                    for (int r = 0; r < RPL; ++r) a[s][r] -= d * vr[r];
                }
            }
        }
    }
    // signs of diag(R) and R itself
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int j = s * NW + w;
#pragma unroll
        for (int r = 0; r < RPL; ++r)
            if (j < n && lane + 64 * r == j) sg[j] = a[s][r] < 0.0 ? -1.0 : 1.0;
    }
    __syncthreads();
    if (R) {
        double* Rb = R + (long long)b * rs;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int j = s * NW + w;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                if (j < n && i < n) Rb[(long long)i * n + j] = i <= j ? sg[i] * a[s][r] : 0.0;
            }
        }
    }
    // Q, backwards: H_k applied to the columns right of k, then column k becomes e_k - tau_k v_k
    for (int k = n - 1; k >= 0; --k) {
        double* v = vbuf[k & 1];
        const double tk = tau[k];
        if (w == k % NW) {
            const int sk = k / NW;
#pragma unroll
            for (int s = 0; s < SL; ++s)
                if (s == sk) {
#pragma unroll
                    for (int r = 0; r < RPL; ++r) {
                        const int i = lane + 64 * r;
                        const double vi = i == k ? 1.0 : (i > k && i < m ? a[s][r] : 0.0);
                        v[i] = vi;
                        a[s][r] = i < k ? 0.0 : (i == k ? 1.0 - tk : -tk * vi);
                    }
                }
        }
        __syncthreads();
        if (tk != 0.0) {
            double vr[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) vr[r] = v[lane + 64 * r];
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const int j = s * NW + w;
                if (j > k && j < n) {
                    double d = 0.0;
#pragma unroll
                    for (int r = 0; r < RPL; ++r) d += vr[r] * a[s][r];
                    d = vq_wsum(d) * tk;
#pragma unroll
                    for (int r = 0; r < RPL; ++r) a[s][r] -= d * vr[r];
                }
            }
        }
    }
    double* Qb = Q + (long long)b * qs;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int j = s * NW + w;
        if (j >= n) continue;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + 64 * r;
            if (i < m) Qb[(long long)i * q_row + (long long)j * q_col] = sg[j] * a[s][r];
        }
    }
}

bool thinq_shape_ok(int m, int n) { return n >= 1 && m >= n && n <= kThinqMaxN; }
bool thinq_fits(int m, int n) {
    return thinq_shape_ok(m, n) && (size_t)m * n * sizeof(double) + 4096 <= get_lds_cap();
}
bool thinq_needs_scratch(int m, int n) {
    return !(m <= 256 && n <= 40) && !(m <= 512 && n <= 64) && !thinq_fits(m, n);
}

// Up to 256 x 40 and 512 x 64: in registers (512 and 1024 threads); beyond, in LDS where
// it fits (256 threads, one column per wave at a time), else in global scratch (1024
// threads and four columns per wave, so that every trailing column group of a step has a
// wave of its own and each load of v serves four columns)
hipError_t launch_thinq(const double* X, long long xs, int m, int n, double* Q, long long qs, long long q_row,
                        long long q_col, double* R, long long rs, double* W, long long ws, int batch,
                        hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    if (!thinq_shape_ok(m, n)) return hipErrorInvalidValue;
    if (m <= 256 && n <= 40) {
        hipLaunchKernelGGL((k_thinq_reg<8, 5, 4>), dim3(batch), dim3(512), 0, st, X, xs, m, n, Q, qs, q_row, q_col,
                           R, rs);
    } else if (m <= 512 && n <= 64) {
        hipLaunchKernelGGL((k_thinq_reg<16, 4, 8>), dim3(batch), dim3(1024), 0, st, X, xs, m, n, Q, qs, q_row, q_col,
                           R, rs);
    } else if (thinq_fits(m, n)) {
        hipLaunchKernelGGL((k_thinq<256, true, 1>), dim3(batch), dim3(256), (size_t)m * n * sizeof(double), st, X, xs,
                           m, n, Q, qs, q_row, q_col, R, rs, nullptr, 0LL);
    } else {
        if (!W || ws < (long long)m * n) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_thinq<1024, false, 4>), dim3(batch), dim3(1024), 0, st, X, xs, m, n, Q, qs, q_row,
                           q_col, R, rs, W, ws);
    }
    return hipGetLastError();
}

// x /= ||x||_2 and lout = lin + ln ||x||_2; a zero x is left as it is with lout = -inf.
__global__ __launch_bounds__(VT) void k_vc_norm(double* x, long long xs, int n, const double* lin,
                                                double* lout) {
    __shared__ double red[VT / 64];
    const int b = blockIdx.x;
    double* xb = x + (long long)b * xs;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += VT) s += xb[i] * xb[i];
    s = vq_bsum<VT>(s, red);
    const double nu = sqrt(s);
    if (nu > 0.0) {
        const double inv = 1.0 / nu;
        for (int i = threadIdx.x; i < n; i += VT) xb[i] *= inv;
    }
    if (threadIdx.x == 0) lout[b] = nu > 0.0 ? (lin ? lin[b] : 0.0) + log(nu) : -INFINITY;
}

hipError_t launch_vc_norm(double* x, long long xs, int n, const double* lin, double* lout, int batch,
                          hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_vc_norm, dim3(batch), dim3(VT), 0, st, x, xs, n, lin, lout);
    return hipGetLastError();
}

}  // namespace peps
