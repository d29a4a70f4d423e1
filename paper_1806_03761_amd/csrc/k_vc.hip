// Kernels of the variational boundary compression (one-site alternating least squares,
// the truncation alternative of Sec. II-A): the thin QR that turns an updated site
// tensor into an isometry, and the normalisation of the final site.  The contractions
// of the sweeps are batched GEMMs (k_mgemm.hip).
#include "common.h"
#include "kernels.h"

namespace peps {

static constexpr int VT = 256;           // threads per matrix
static constexpr int kThinqMaxN = 128;   // columns

__device__ inline double vq_wsum(double v) { return lane_group_sum(v, 64); }

__device__ inline double vq_bsum(double v, double* red) {
    v = vq_wsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < VT / 64; ++i) s += red[i];
    return s;
}

// One wave applies H = I - tk v v^T (v_k = 1, v_i = vk[i] below row k) to column aj,
// rows k..m-1.
__device__ inline void vq_reflect(const double* vk, double* aj, int k, int m, double tk, int lane) {
    double d = lane == 0 ? aj[k] : 0.0;
    for (int i = k + 1 + lane; i < m; i += 64) d += vk[i] * aj[i];
    d = vq_wsum(d) * tk;
    if (lane == 0) aj[k] -= d;
    for (int i = k + 1 + lane; i < m; i += 64) aj[i] -= d * vk[i];
}

// Thin Householder QR of one m x n matrix (m >= n) per workgroup, in LDS:
//   X: column-major, leading dimension m, stride xs per matrix (may equal Q: every
//      element is read before any is written);
//   Q: the m x n factor with the signs fixed so that diag(R) >= 0, element (i, k) at
//      Q + b qs + i q_row + k q_col;
//   R: when not null, the n x n factor (row-major, zeros below the diagonal), stride rs.
// Reflectors follow the usual convention (beta = -sign(alpha) ||x||, tau = (beta -
// alpha) / beta); a column with nothing below the diagonal gives tau = 0.  Q is formed
// in place by applying the reflectors backwards to the leading n columns of I.
__global__ __launch_bounds__(VT) void k_thinq(const double* X, long long xs, int m, int n, double* Q,
                                              long long qs, long long q_row, long long q_col, double* R,
                                              long long rs) {
    extern __shared__ double a[];
    __shared__ double tau[kThinqMaxN], sg[kThinqMaxN], red[VT / 64];
    const int b = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
    const double* Xb = X + (long long)b * xs;
    const int mn = m * n;
    for (int i = t; i < mn; i += VT) a[i] = Xb[i];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        double* ak = a + (long long)k * m;
        double s = 0.0;
        for (int i = k + 1 + t; i < m; i += VT) s += ak[i] * ak[i];
        s = vq_bsum(s, red);
        const double alpha = ak[k];
        double tk = 0.0, beta = alpha;
        if (s > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + s), alpha);
            tk = (beta - alpha) / beta;
            const double sc = 1.0 / (alpha - beta);
            for (int i = k + 1 + t; i < m; i += VT) ak[i] *= sc;
        }
        __syncthreads();
        if (t == 0) {
            ak[k] = beta;
            tau[k] = tk;
        }
        if (tk != 0.0)
            for (int j = k + 1 + w; j < n; j += VT / 64) vq_reflect(ak, a + (long long)j * m, k, m, tk, lane);
        __syncthreads();
    }
    for (int k = t; k < n; k += VT) sg[k] = a[k + (long long)k * m] < 0.0 ? -1.0 : 1.0;
    __syncthreads();
    if (R) {
        double* Rb = R + (long long)b * rs;
        for (int idx = t; idx < n * n; idx += VT) {
            const int k = idx / n, j = idx - k * n;
            Rb[idx] = j >= k ? sg[k] * a[k + (long long)j * m] : 0.0;
        }
    }
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
        double* ak = a + (long long)k * m;
        const double tk = tau[k];
        if (tk != 0.0)
            for (int j = k + 1 + w; j < n; j += VT / 64) vq_reflect(ak, a + (long long)j * m, k, m, tk, lane);
        __syncthreads();
        for (int i = t; i < m; i += VT) ak[i] = i < k ? 0.0 : (i == k ? 1.0 - tk : -tk * ak[i]);
        __syncthreads();
    }
    double* Qb = Q + (long long)b * qs;
    if (q_row == 1) {
        for (int idx = t; idx < mn; idx += VT) {
            const int k = idx / m, i = idx - k * m;
            Qb[i + (long long)k * q_col] = sg[k] * a[idx];
        }
    } else {
        for (int idx = t; idx < mn; idx += VT) {
            const int i = idx / n, k = idx - i * n;
            Qb[(long long)i * q_row + (long long)k * q_col] = sg[k] * a[i + (long long)k * m];
        }
    }
}

bool thinq_fits(int m, int n) {
    return n >= 1 && m >= n && n <= kThinqMaxN && (size_t)m * n * sizeof(double) + 4096 <= get_lds_cap();
}

hipError_t launch_thinq(const double* X, long long xs, int m, int n, double* Q, long long qs, long long q_row,
                        long long q_col, double* R, long long rs, int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    if (!thinq_fits(m, n)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_thinq, dim3(batch), dim3(VT), (size_t)m * n * sizeof(double), st, X, xs, m, n, Q, qs,
                       q_row, q_col, R, rs);
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
    s = vq_bsum(s, red);
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
