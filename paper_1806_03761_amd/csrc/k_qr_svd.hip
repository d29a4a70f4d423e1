// Batched float64 factorisations of the boundary-MPS truncation (Fig. 1(c)).
//
//  k_qr      Householder QR of one column tensor X (rows (a,phys), cols right bond),
//            one workgroup per matrix, column-major, LDS-resident when it fits.
//            The reflectors stay in X (below the diagonal) for the later
//            implicit application of Q; R is written to its own buffer.
//  k_center0 the same centre formation for the first column, then the norm is
//            pulled out into the running log scale.
#include "common.h"
#include "kernels.h"

namespace peps {

static constexpr int NT = 256;

__device__ inline double wave_sum(double v, int width) { return lane_group_sum(v, width); }

// Sum over the whole workgroup; every thread gets the result.
__device__ inline double block_sum(double v, double* red) {
    v = wave_sum(v, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}

// Max over the whole workgroup; every thread gets the result.
__device__ inline double block_max(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) s = fmax(s, red[i]);
    return s;
}


// ---------------------------------------------------------------------------
// LDS strides.  A wave reads tpc consecutive rows of several columns at once; a
// column stride that is a multiple of 32 doubles puts every column on the same
// banks (8- to 16-way conflicts).  Padding the stride by 4 (or 2) doubles spreads
// the groups over the banks (2-way, the minimum for 64 lanes of 8 bytes).
// ---------------------------------------------------------------------------
__host__ __device__ inline int tpc_for(int ncols) {
    int p = 1;
    while (p < ncols) p <<= 1;
    const int t = NT / p;
    return t < 1 ? 1 : (t > 64 ? 64 : t);
}
__host__ __device__ inline int pad_for(int tpc) { return tpc == 16 ? 2 : 4; }

// ---------------------------------------------------------------------------
// QR
// ---------------------------------------------------------------------------
// X: column-major m x n per batch item (stride xs); in place -> reflectors + R.
// R: row-major r x n (zeros below the diagonal), r = min(m, n); tau: [r].
__global__ __launch_bounds__(NT) void k_qr(double* X, long long xs, int m, int n,
                                           double* R, long long rs, double* tau, long long ts,
                                           int use_lds) {
    extern __shared__ double lds[];
    __shared__ double red[NT / 64];
    __shared__ double s_beta, s_tau, s_scal;
    const int b = blockIdx.x, tid = threadIdx.x;
    double* Xg = X + (long long)b * xs;
    const int ldw = use_lds ? m + 4 : m;
    double* W = use_lds ? lds : Xg;
    const int r = min(m, n);
    if (use_lds) {
        for (int e = tid; e < m * n; e += NT) W[(e / m) * ldw + e % m] = Xg[e];
        __syncthreads();
    }
    for (int k = 0; k < r; ++k) {
        double* colk = W + (long long)k * ldw;
        double part = 0.0;
        for (int i = k + 1 + tid; i < m; i += NT) part += colk[i] * colk[i];
        const double s = block_sum(part, red);
        if (tid == 0) {
            const double alpha = colk[k];
            if (s == 0.0) {
                s_tau = 0.0;
                s_beta = alpha;
                s_scal = 0.0;
            } else {
                const double beta = -copysign(sqrt(alpha * alpha + s), alpha);
                s_tau = (beta - alpha) / beta;
                s_scal = 1.0 / (alpha - beta);
                s_beta = beta;
            }
        }
        __syncthreads();
        const double tk = s_tau;
        if (tk != 0.0) {
            const double sc = s_scal;
            for (int i = k + 1 + tid; i < m; i += NT) colk[i] *= sc;
        }
        __syncthreads();
        if (tid == 0) {
            colk[k] = s_beta;
            tau[(long long)b * ts + k] = tk;
        }
        if (tk != 0.0) {
            const int ncols = n - k - 1;
            if (ncols > 0) {
                const int tpc = tpc_for(ncols);
                const int ngroups = NT / tpc;
                const int g = tid / tpc, l = tid % tpc;
                for (int c0 = k + 1; c0 < n; c0 += ngroups) {
                    const int c = c0 + g;
                    const bool act = c < n;
                    double* colc = W + (long long)(act ? c : k) * ldw;
                    double dot = 0.0;
                    if (act) {
                        for (int i = k + 1 + l; i < m; i += tpc) dot += colk[i] * colc[i];
                        if (l == 0) dot += colc[k];
                    }
                    dot = wave_sum(dot, tpc);
                    if (act) {
                        const double f = tk * dot;
                        if (l == 0) colc[k] -= f;
                        for (int i = k + 1 + l; i < m; i += tpc) colc[i] -= f * colk[i];
                    }
                }
            }
        }
        __syncthreads();
    }
    // R (row-major r x n) and write-back of the reflectors
    double* Rb = R + (long long)b * rs;
    for (int e = tid; e < r * n; e += NT) {
        const int i = e / n, c = e % n;
        Rb[e] = (i <= c) ? W[(long long)c * ldw + i] : 0.0;
    }
    if (use_lds) {
        for (int e = tid; e < m * n; e += NT) Xg[e] = W[(e / m) * ldw + e % m];
    }
}

// ---------------------------------------------------------------------------
// Register-resident QR for matrices of up to RPT*tpc rows and up to 256 columns.
// Column c lives in the registers of thread group c (tpc lanes, lane l holds rows
// l, l+tpc, ...).  Step k: the group of column k has published its column (after
// all earlier reflections), its squared norm below the diagonal and its diagonal
// entry in a double-buffered LDS slot; every thread derives the same reflector
// from them, groups c > k apply it to their own column, and group k+1 publishes
// the next pivot column.  One barrier per step; the pivot column reads are LDS
// broadcasts.  Same arithmetic as k_qr (LAPACK dlarfg convention).
// ---------------------------------------------------------------------------
template <int RPT, int TPC>
__device__ inline void qr_reg_pivot(double (&a)[RPT], int k, int m, int l, double* vslot,
                                    double* tslot, double* tau_out) {
    // column k of this group: reflector with v_k = 1 (LAPACK dlarfg convention),
    // published zero-padded (v_i = 0 for i < k and i >= m) together with tau
    double s = 0.0, al = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = l + q * TPC;
        const double x = a[q];
        s += (i > k && i < m) ? x * x : 0.0;
        al += (i == k) ? x : 0.0;
    }
    s = wave_sum(s, TPC);
    al = wave_sum(al, TPC);
    double tk, be, sc;
    if (s == 0.0) {
        tk = 0.0; be = al; sc = 0.0;
    } else {
        be = -copysign(sqrt(al * al + s), al);
        tk = (be - al) / be;
        sc = 1.0 / (al - be);
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = l + q * TPC;
        const double v = (i < k || i >= m) ? 0.0 : (i == k ? 1.0 : sc * a[q]);
        vslot[i] = v;
        a[q] = (i == k) ? be : ((i > k && tk != 0.0) ? v : a[q]);
    }
    if (l == 0) {
        *tslot = tk;
        *tau_out = tk;
    }
}

// RPT rows per lane, TPC lanes per column, WG threads (WG / TPC >= n columns).
template <int RPT, int TPC, int WG>
__global__ __launch_bounds__(WG) void k_qr_reg(double* X, long long xs, int m, int n, double* R,
                                               long long rs, double* tau, long long ts) {
    __shared__ double xcol[2][RPT * TPC];
    __shared__ double sh_t[2];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int g = tid / TPC, l = tid % TPC;
    const int r = min(m, n);
    double* Xg = X + (long long)b * xs;
    double* taub = tau + (long long)b * ts;
    const bool own = g < n;
    double a[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = l + q * TPC;
        a[q] = (own && i < m) ? Xg[(long long)g * m + i] : 0.0;
    }
    // iteration k: apply the reflector of step k-1, then group k publishes step k
    for (int k = 0; k <= r; ++k) {
        if (k > 0) {
            const int bk = (k - 1) & 1;
            const double tk = sh_t[bk];
            if (own && g >= k && tk != 0.0) {
                const double* vs = xcol[bk];
                double v[RPT];
                double dot = 0.0;
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    v[q] = vs[l + q * TPC];
                    dot += v[q] * a[q];
                }
                dot = wave_sum(dot, TPC);
                const double f = tk * dot;
#pragma unroll
                for (int q = 0; q < RPT; ++q) a[q] -= f * v[q];
            }
        }
        if (k < r && g == k) qr_reg_pivot<RPT, TPC>(a, k, m, l, xcol[k & 1], &sh_t[k & 1], &taub[k]);
        __syncthreads();
    }
    // write back: reflectors + R in X (column-major), R row-major r x n
    if (own) {
        double* Rb = R + (long long)b * rs;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = l + q * TPC;
            if (i < m) Xg[(long long)g * m + i] = a[q];
            if (i < r) Rb[(long long)i * n + g] = (i <= g) ? a[q] : 0.0;
        }
    }
}

template <int TPC, int WG>
static bool launch_qr_reg_t(double* X, long long xs, int m, int n, double* R, long long rs,
                            double* tau, long long ts, int batch, hipStream_t st) {
    const int need = (m + TPC - 1) / TPC;
    if (need <= 4) hipLaunchKernelGGL((k_qr_reg<4, TPC, WG>), dim3(batch), dim3(WG), 0, st, X, xs, m, n, R, rs, tau, ts);
    else if (need <= 16) hipLaunchKernelGGL((k_qr_reg<16, TPC, WG>), dim3(batch), dim3(WG), 0, st, X, xs, m, n, R, rs, tau, ts);
    else if (need <= 32) hipLaunchKernelGGL((k_qr_reg<32, TPC, WG>), dim3(batch), dim3(WG), 0, st, X, xs, m, n, R, rs, tau, ts);
    else return false;
    return true;
}

template <int WG>
static bool launch_qr_reg_wg(double* X, long long xs, int m, int n, double* R, long long rs,
                             double* tau, long long ts, int batch, hipStream_t st) {
    int p2 = 1;
    while (p2 < n) p2 <<= 1;
    int tpc = WG / p2;
    tpc = tpc > 64 ? 64 : tpc;
    if ((m + tpc - 1) / tpc > 32) return false;
    switch (tpc) {
        case 4: return WG == 256 && launch_qr_reg_t<4, 256>(X, xs, m, n, R, rs, tau, ts, batch, st);
        case 8: return WG == 256 ? launch_qr_reg_t<8, 256>(X, xs, m, n, R, rs, tau, ts, batch, st)
                                 : launch_qr_reg_t<8, 512>(X, xs, m, n, R, rs, tau, ts, batch, st);
        case 16: return WG == 256 ? launch_qr_reg_t<16, 256>(X, xs, m, n, R, rs, tau, ts, batch, st)
                                  : launch_qr_reg_t<16, 512>(X, xs, m, n, R, rs, tau, ts, batch, st);
        case 32: return WG == 256 ? launch_qr_reg_t<32, 256>(X, xs, m, n, R, rs, tau, ts, batch, st)
                                  : launch_qr_reg_t<32, 512>(X, xs, m, n, R, rs, tau, ts, batch, st);
        case 64: return WG == 256 ? launch_qr_reg_t<64, 256>(X, xs, m, n, R, rs, tau, ts, batch, st)
                                  : launch_qr_reg_t<64, 512>(X, xs, m, n, R, rs, tau, ts, batch, st);
        default: return false;
    }
}

// ---------------------------------------------------------------------------
// Column-group QR: each group of TPC lanes owns CPG columns (c = g, g + NG, ...; NG =
// WG / TPC groups), lane l the row pairs (2l, 2l+1) + 2 TPC j, so one reflector read
// (a 16-byte LDS load per row pair) serves CPG columns and every dependent chain is
// RPT long.  Step k: groups apply reflector k-1 to their columns >= k; the group of
// column k then forms reflector k (LAPACK dlarfg convention, v_k = 1) and publishes it
// zero-padded with tau in a double-buffered LDS slot.  One barrier per step.
// ---------------------------------------------------------------------------
template <int TPC>
__device__ __forceinline__ int qc_row(int q, int l) {
    return (q >> 1) * (2 * TPC) + 2 * l + (q & 1);
}

template <int RPT, int TPC>
__device__ __forceinline__ void qc_pivot(double (&a)[RPT], int k, int m, int l, double* vslot,
                                         double* tslot, double* tau_out) {
    double s0 = 0.0, s1 = 0.0, al = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = qc_row<TPC>(q, l);
        const double x = (i > k) ? a[q] : 0.0;
        if (q & 1) s1 = fma(x, x, s1);
        else s0 = fma(x, x, s0);
        al = (i == k) ? a[q] : al;
    }
    const double s = lane_group_sum(s0 + s1, TPC);
    al = lane_group_sum(al, TPC);
    double tk, be, sc;
    if (s == 0.0) {
        tk = 0.0; be = al; sc = 0.0;
    } else {
        be = -copysign(sqrt(al * al + s), al);
        tk = (be - al) / be;
        sc = 1.0 / (al - be);
    }
#pragma unroll
    for (int q = 0; q < RPT; q += 2) {
        const int i = qc_row<TPC>(q, l);
        const double v0 = (i < k || i >= m) ? 0.0 : (i == k ? 1.0 : sc * a[q]);
        const double v1 = (i + 1 < k || i + 1 >= m) ? 0.0 : (i + 1 == k ? 1.0 : sc * a[q + 1]);
        *reinterpret_cast<double2*>(vslot + i) = make_double2(v0, v1);
        a[q] = (i == k) ? be : ((i > k && tk != 0.0) ? v0 : a[q]);
        a[q + 1] = (i + 1 == k) ? be : ((i + 1 > k && tk != 0.0) ? v1 : a[q + 1]);
    }
    if (l == 0) {
        *tslot = tk;
        *tau_out = tk;
    }
}

template <int RPT, int TPC, int CPG, int WG>
__global__ __launch_bounds__(WG) void k_qr_cols(double* X, long long xs, int m, int n, double* R,
                                                long long rs, double* tau, long long ts) {
    constexpr int NG = WG / TPC;
    __shared__ __align__(16) double xcol[2][RPT * TPC];
    __shared__ double sh_t[2];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int g = tid / TPC, l = tid % TPC;
    const int r = min(m, n);
    double* Xg = X + (long long)b * xs;
    double* taub = tau + (long long)b * ts;
    double a[CPG][RPT];
#pragma unroll
    for (int s = 0; s < CPG; ++s) {
        const int c = g + s * NG;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = qc_row<TPC>(q, l);
            a[s][q] = (c < n && i < m) ? Xg[(long long)c * m + i] : 0.0;
        }
    }
    for (int k = 0; k <= r; ++k) {
        if (k > 0) {
            const int bk = (k - 1) & 1;
            const double tk = sh_t[bk];
            if (tk != 0.0 && g + (CPG - 1) * NG >= k) {
                double v[RPT];
#pragma unroll
                for (int q = 0; q < RPT; q += 2) {
                    const double2 t = *reinterpret_cast<const double2*>(xcol[bk] + qc_row<TPC>(q, l));
                    v[q] = t.x;
                    v[q + 1] = t.y;
                }
#pragma unroll
                for (int s = 0; s < CPG; ++s) {
                    const int c = g + s * NG;
                    if (c >= k && c < n) {
                        double d0 = 0.0, d1 = 0.0;
#pragma unroll
                        for (int q = 0; q < RPT; q += 2) {
                            d0 = fma(v[q], a[s][q], d0);
                            d1 = fma(v[q + 1], a[s][q + 1], d1);
                        }
                        const double f = tk * lane_group_sum(d0 + d1, TPC);
#pragma unroll
                        for (int q = 0; q < RPT; ++q) a[s][q] = fma(-f, v[q], a[s][q]);
                    }
                }
            }
        }
        if (k < r && g == k % NG) {
            const int sk = k / NG;
#pragma unroll
            for (int s = 0; s < CPG; ++s)
                if (s == sk) qc_pivot<RPT, TPC>(a[s], k, m, l, xcol[k & 1], &sh_t[k & 1], &taub[k]);
        }
        __syncthreads();
    }
    double* Rb = R + (long long)b * rs;
#pragma unroll
    for (int s = 0; s < CPG; ++s) {
        const int c = g + s * NG;
        if (c >= n) continue;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = qc_row<TPC>(q, l);
            if (i < m) Xg[(long long)c * m + i] = a[s][q];
            if (i < r) Rb[(long long)i * n + c] = (i <= c) ? a[s][q] : 0.0;
        }
    }
}

template <int RPT, int CPG, int TPC, int WG>
static bool qc_try(int rpt, int cpg, double* X, long long xs, int m, int n, double* R, long long rs,
                   double* tau, long long ts, int batch, hipStream_t st) {
    if constexpr (WG >= 1024 && (RPT * CPG > 32 || RPT * CPG + RPT > 40)) {
        return false;   // would spill at the 128-register limit of 1024-thread groups
    } else {
        if (rpt > RPT || cpg > CPG) return false;
        hipLaunchKernelGGL((k_qr_cols<RPT, TPC, CPG, WG>), dim3(batch), dim3(WG), 0, st, X, xs, m, n, R,
                           rs, tau, ts);
        return true;
    }
}

template <int TPC, int WG>
static bool launch_qr_cols_t(double* X, long long xs, int m, int n, double* R, long long rs,
                             double* tau, long long ts, int batch, hipStream_t st) {
    constexpr int NG = WG / TPC;
    const int cpg = (n + NG - 1) / NG;
    int rpt = (m + TPC - 1) / TPC;
    rpt += rpt & 1;
#define QC(RPT_, CPG_) qc_try<RPT_, CPG_, TPC, WG>(rpt, cpg, X, xs, m, n, R, rs, tau, ts, batch, st)
    return QC(4, 1) || QC(8, 1) || QC(4, 2) || QC(16, 1) || QC(8, 2) || QC(4, 4) || QC(16, 2) ||
           QC(8, 4) || QC(32, 1) || QC(2, 8) || QC(4, 8) || QC(16, 4) || QC(8, 8);
#undef QC
}

bool launch_qr_cols(double* X, long long xs, int m, int n, double* R, long long rs, double* tau,
                    long long ts, int batch, int tpc, int wg, hipStream_t st) {
    if (m <= 0 || n <= 0) return false;
    if (wg == 256) {
        switch (tpc) {
            case 8: return launch_qr_cols_t<8, 256>(X, xs, m, n, R, rs, tau, ts, batch, st);
            case 16: return launch_qr_cols_t<16, 256>(X, xs, m, n, R, rs, tau, ts, batch, st);
            case 32: return launch_qr_cols_t<32, 256>(X, xs, m, n, R, rs, tau, ts, batch, st);
            case 64: return launch_qr_cols_t<64, 256>(X, xs, m, n, R, rs, tau, ts, batch, st);
        }
    } else if (wg == 512) {
        switch (tpc) {
            case 16: return launch_qr_cols_t<16, 512>(X, xs, m, n, R, rs, tau, ts, batch, st);
            case 32: return launch_qr_cols_t<32, 512>(X, xs, m, n, R, rs, tau, ts, batch, st);
            case 64: return launch_qr_cols_t<64, 512>(X, xs, m, n, R, rs, tau, ts, batch, st);
        }
    } else if (wg == 1024) {
        switch (tpc) {
            case 32: return launch_qr_cols_t<32, 1024>(X, xs, m, n, R, rs, tau, ts, batch, st);
            case 64: return launch_qr_cols_t<64, 1024>(X, xs, m, n, R, rs, tau, ts, batch, st);
        }
    }
    return false;
}

// ---------------------------------------------------------------------------
// implicit Q: Z (column-major mz x tin, stride ldz) <- H_0 H_1 ... H_{r-1} Z
// V column-major mz x r (reflector k in column k below the diagonal, unit diagonal).
// ---------------------------------------------------------------------------
__device__ void apply_q(const double* V, const double* tau, int mz, int r, double* Z, int ldz,
                        int tin, double* vbuf) {
    const int tid = threadIdx.x;
    const int tpc = tpc_for(tin);
    const int ngroups = NT / tpc;
    const int g = tid / tpc, l = tid % tpc;
    for (int k = r - 1; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;
        __syncthreads();
        for (int i = k + 1 + tid; i < mz; i += NT) vbuf[i] = V[(long long)k * mz + i];
        __syncthreads();
        for (int c0 = 0; c0 < tin; c0 += ngroups) {
            const int c = c0 + g;
            const bool act = c < tin;
            double* zc = Z + (long long)(act ? c : 0) * ldz;
            double dot = 0.0;
            if (act) {
                for (int i = k + 1 + l; i < mz; i += tpc) dot += vbuf[i] * zc[i];
                if (l == 0) dot += zc[k];
            }
            dot = wave_sum(dot, tpc);
            if (act) {
                const double f = tk * dot;
                if (l == 0) zc[k] -= f;
                for (int i = k + 1 + l; i < mz; i += tpc) zc[i] -= f * vbuf[i];
            }
        }
    }
    __syncthreads();
}

// Load Z = [G; 0] column-major (mz x tin, stride ldz) from G row-major (r x tin), then apply Q.
__device__ void form_center(const double* V, const double* tau, const double* G, int mz, int r,
                            int tin, double* Z, int ldz, double* vbuf) {
    for (int e = threadIdx.x; e < mz * tin; e += NT) {
        const int c = e / mz, i = e % mz;
        Z[(long long)c * ldz + i] = (i < r) ? G[(long long)i * tin + c] : 0.0;
    }
    __syncthreads();
    if (V) apply_q(V, tau, mz, r, Z, ldz, tin, vbuf);
}

// First column: Z = Q_0 G_1 (mz x tin), nu = ||Z||, newU_0 = Z / nu (row-major mz x tin),
// logs[b] = logs_in[b] + ln nu.
__global__ __launch_bounds__(NT) void k_center0(const double* V, long long vs, const double* tau,
                                                long long ts, const double* G, long long gs, int mz,
                                                int r, int tin, double* newU, long long us,
                                                const double* logs_in, double* logs_out,
                                                double* scratch, long long ss, int use_lds) {
    extern __shared__ double lds[];
    __shared__ double red[NT / 64];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int ldz = mz + pad_for(tpc_for(tin));
    double* Z = use_lds ? lds : scratch + (long long)b * ss;
    double* vbuf = Z + (long long)ldz * tin;
    form_center(V ? V + (long long)b * vs : nullptr, tau + (long long)b * ts, G + (long long)b * gs,
                mz, V ? r : mz, tin, Z, ldz, vbuf);
    double part = 0.0;
    for (int e = tid; e < mz * tin; e += NT) {
        const double z = Z[(long long)(e / mz) * ldz + e % mz];
        part += z * z;
    }
    const double nu = sqrt(block_sum(part, red));
    const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
    double* U = newU + (long long)b * us;
    for (int e = tid; e < mz * tin; e += NT) {
        const int i = e / tin, c = e % tin;
        U[e] = Z[(long long)c * ldz + i] * inv;
    }
    if (tid == 0) logs_out[b] = (logs_in ? logs_in[b] : 0.0) + (nu > 0.0 ? log(nu) : -INFINITY);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static size_t lds_cap() { return get_lds_cap(); }

hipError_t launch_qr(double* X, long long xs, int m, int n, double* R, long long rs, double* tau,
                     long long ts, int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    // column groups of 16 lanes in 256-thread blocks up to 128 rows (four-stage lane sums),
    // 32 lanes in 512-thread blocks above: the faster of the launch shapes measured at
    // each height
    if (m <= 128 && launch_qr_cols(X, xs, m, n, R, rs, tau, ts, batch, 16, 256, st)) return hipGetLastError();
    if (launch_qr_cols(X, xs, m, n, R, rs, tau, ts, batch, 32, 512, st)) return hipGetLastError();
    if (n <= 64) {
        if (launch_qr_reg_wg<256>(X, xs, m, n, R, rs, tau, ts, batch, st) ||
            launch_qr_reg_wg<512>(X, xs, m, n, R, rs, tau, ts, batch, st))
            return hipGetLastError();
    }
    const size_t bytes = (size_t)(m + 4) * n * sizeof(double);
    const int use = bytes <= lds_cap() - 1024;
    hipLaunchKernelGGL(k_qr, dim3(batch), dim3(NT), use ? bytes : 0, st, X, xs, m, n, R, rs, tau,
                       ts, use);
    return hipGetLastError();
}

size_t center0_scratch_doubles(int mz, int tin) {
    return (size_t)(mz + pad_for(tpc_for(tin))) * tin + mz + 8;
}

hipError_t launch_center0(const double* V, long long vs, const double* tau, long long ts,
                          const double* G, long long gs, int mz, int r, int tin, double* newU,
                          long long us, const double* logs_in, double* logs_out, double* scratch,
                          long long ss, int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    const size_t bytes = center0_scratch_doubles(mz, tin) * sizeof(double);
    const int use = bytes <= lds_cap() - 1024;
    hipLaunchKernelGGL(k_center0, dim3(batch), dim3(NT), use ? bytes : 0, st, V, vs, tau, ts, G, gs,
                       mz, r, tin, newU, us, logs_in, logs_out, scratch, ss, use);
    return hipGetLastError();
}

}  // namespace peps
