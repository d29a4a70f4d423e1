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

__device__ inline double e_wave_sum(double v, int width) {
    for (int o = width / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
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
    L.nv = mz > 2 * L.ns ? mz : 2 * L.ns;     // work vector of the prep kernel
    L.oW = L.oP + (long long)L.ldx * L.tk;
    L.total = L.oW + L.nv;
    // LDS needs of the two workgroup kernels
    L.lds_prep = (long long)L.ldz * tin + (long long)L.lda * L.ns + 3LL * L.ns + L.nv + 8;
    L.lds_fin = (long long)L.ldx * L.tk + (long long)L.lda * L.ns + L.ns + (long long)L.ldz * tin + L.tk + 8;
    return L;
}

// ---------------------------------------------------------------------------
// A: centre, Gram, tridiagonalisation
// ---------------------------------------------------------------------------
template <bool kLds>
__device__ void prep_body(const EigArgs& a, double* Z, double* Am, double* d, double* e, double* tau,
                          double* vbuf, const EigLayout& L, double* red) {
    const int b = blockIdx.x, tid = threadIdx.x;
    const int mz = a.mz, tin = a.tin, p = a.p, ns = L.ns, lda = L.lda, ldz = L.ldz;
    // Z = [G; 0] then Z <- Q Z (reflectors of the QR of this column)
    const double* G = a.G + (long long)b * a.gs;
    const int r = a.V ? a.r : mz;
    for (int e2 = tid; e2 < mz * tin; e2 += NT) {
        const int c = e2 / mz, i = e2 % mz;
        Z[(long long)c * ldz + i] = (i < r) ? G[(long long)i * tin + c] : 0.0;
    }
    __syncthreads();
    if (a.V) {
        const double* V = a.V + (long long)b * a.vs;
        const double* tq = a.tau + (long long)b * a.ts;
        const int tpc = e_tpc(tin), ngroups = NT / tpc, g = tid / tpc, l = tid % tpc;
        for (int k = r - 1; k >= 0; --k) {
            const double tk = tq[k];
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
                dot = e_wave_sum(dot, tpc);
                if (act) {
                    const double f = tk * dot;
                    if (l == 0) zc[k] -= f;
                    for (int i = k + 1 + l; i < mz; i += tpc) zc[i] -= f * vbuf[i];
                }
            }
        }
        __syncthreads();
    }
    // Gram matrix.  M[ar][col] = Z[t][ar*p+d] with col = d*tin + t.
    // gram_right: A[c1][c2] = sum_ar M[ar][c1] M[ar][c2];  else A[a1][a2] = sum_col M[a1][col] M[a2][col]
    for (int e2 = tid; e2 < ns * ns; e2 += NT) {
        const int i = e2 / ns, j = e2 % ns;
        if (j < i) continue;
        double acc = 0.0;
        if (L.gram_right) {
            const int d1 = i / tin, t1 = i % tin, d2 = j / tin, t2 = j % tin;
            const double* z1 = Z + (long long)t1 * ldz + d1;
            const double* z2 = Z + (long long)t2 * ldz + d2;
            for (int ar = 0; ar < L.mp; ++ar) acc += z1[ar * p] * z2[ar * p];
        } else {
            for (int col = 0; col < L.np; ++col) {
                const int dd = col / tin, t = col % tin;
                const double* zt = Z + (long long)t * ldz + dd;
                acc += zt[i * p] * zt[j * p];
            }
        }
        Am[(long long)i * lda + j] = acc;
        Am[(long long)j * lda + i] = acc;
    }
    __syncthreads();
    // Householder tridiagonalisation (lower part keeps the reflectors)
    __shared__ double s_beta, s_tau, s_scal, s_K;
    for (int k = 0; k + 2 < ns; ++k) {
        double part = 0.0;
        for (int i = k + 2 + tid; i < ns; i += NT) {
            const double x = Am[(long long)i * lda + k];
            part += x * x;
        }
        const double s = e_block_sum(part, red);
        if (tid == 0) {
            const double al = Am[(long long)(k + 1) * lda + k];
            if (s == 0.0) {
                s_tau = 0.0; s_beta = al; s_scal = 0.0;
            } else {
                const double be = -copysign(sqrt(al * al + s), al);
                s_tau = (be - al) / be; s_scal = 1.0 / (al - be); s_beta = be;
            }
        }
        __syncthreads();
        const double tk = s_tau;
        if (tid == 0) {
            tau[k] = tk;
            e[k] = s_beta;
        }
        if (tk == 0.0) {
            __syncthreads();
            continue;
        }
        // v (length ns-k-1, v[0] = 1) kept in column k below the subdiagonal
        for (int i = k + 2 + tid; i < ns; i += NT) Am[(long long)i * lda + k] *= s_scal;
        __syncthreads();
        // p = tau * A22 v  (vbuf holds p), A22 = rows/cols k+1..ns-1
        const int n2 = ns - k - 1;
        {
            const int tpr = e_tpc(n2), ngr = NT / tpr, g = tid / tpr, l = tid % tpr;
            for (int i0 = 0; i0 < n2; i0 += ngr) {
                const int ii = i0 + g;
                const bool act = ii < n2;
                double acc = 0.0;
                if (act) {
                    const double* row = Am + (long long)(k + 1 + ii) * lda + (k + 1);
                    for (int jj = l; jj < n2; jj += tpr) {
                        const double vj = (jj == 0) ? 1.0 : Am[(long long)(k + 1 + jj) * lda + k];
                        acc += row[jj] * vj;
                    }
                }
                acc = e_wave_sum(acc, tpr);
                if (act && l == 0) vbuf[ii] = tk * acc;
            }
        }
        __syncthreads();
        // K = tau/2 (p . v); w = p - K v
        double pv = 0.0;
        for (int jj = tid; jj < n2; jj += NT) {
            const double vj = (jj == 0) ? 1.0 : Am[(long long)(k + 1 + jj) * lda + k];
            pv += vbuf[jj] * vj;
        }
        pv = e_block_sum(pv, red);
        const double K = 0.5 * tk * pv;
        for (int jj = tid; jj < n2; jj += NT) {
            const double vj = (jj == 0) ? 1.0 : Am[(long long)(k + 1 + jj) * lda + k];
            vbuf[n2 + jj] = vbuf[jj] - K * vj;     // w
        }
        __syncthreads();
        // A22 -= v w^T + w v^T (upper triangle and diagonal, mirrored)
        for (int e2 = tid; e2 < n2 * n2; e2 += NT) {
            const int ii = e2 / n2, jj = e2 % n2;
            if (jj < ii) continue;
            const double vi = (ii == 0) ? 1.0 : Am[(long long)(k + 1 + ii) * lda + k];
            const double vj = (jj == 0) ? 1.0 : Am[(long long)(k + 1 + jj) * lda + k];
            const double wi = vbuf[n2 + ii], wj = vbuf[n2 + jj];
            const double nv = Am[(long long)(k + 1 + ii) * lda + (k + 1 + jj)] - vi * wj - wi * vj;
            Am[(long long)(k + 1 + ii) * lda + (k + 1 + jj)] = nv;
            if (jj != ii) Am[(long long)(k + 1 + jj) * lda + (k + 1 + ii)] = nv;
        }
        __syncthreads();
    }
    if (tid == 0) {
        for (int k = ns - 2; k >= 0 && k + 2 >= ns; --k) {   // last (or only) off-diagonal
            e[k] = Am[(long long)(k + 1) * lda + k];
            tau[k] = 0.0;
        }
        if (ns >= 1) tau[ns - 1] = 0.0;
    }
    for (int k = tid; k < ns; k += NT) d[k] = Am[(long long)k * lda + k];
    __syncthreads();
}

template <bool kLds>
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
        prep_body<true>(a, Z, Am, d, e, tau, vbuf, L, red);
        // hand over Z, reflectors, d, e, tau
        const int tid = threadIdx.x;
        for (long long i = tid; i < (long long)L.ldz * a.tin; i += NT) gs[L.oZ + i] = Z[i];
        for (long long i = tid; i < (long long)L.lda * L.ns; i += NT) gs[L.oA + i] = Am[i];
        for (int i = tid; i < L.ns; i += NT) {
            gs[L.oD + i] = d[i];
            gs[L.oE + i] = e[i];
            gs[L.oT + i] = tau[i];
        }
    } else {
        // everything in global scratch
        prep_body<false>(a, gs + L.oZ, gs + L.oA, gs + L.oD, gs + L.oE, gs + L.oT, gs + L.oW, L, red);
    }
}

// ---------------------------------------------------------------------------
// B: eigenvalues and tridiagonal eigenvectors, one lane each
// ---------------------------------------------------------------------------
__device__ inline unsigned hash_u32(unsigned x) {
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    return x;
}

__global__ __launch_bounds__(64) void k_eig_tri(EigArgs a, int lanes_per_matrix) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const EigLayout L = eig_layout(a.mz, a.tin, a.p, a.Dc);
    const int b = (int)(gid / lanes_per_matrix), l = (int)(gid % lanes_per_matrix);
    if (b >= a.batch || l >= L.tk) return;
    double* gs = a.scratch + (long long)b * a.ss;
    const double* d = gs + L.oD;
    const double* e = gs + L.oE;
    double* x = gs + L.oX + (long long)l * L.ldx;
    double* piv = gs + L.oP + (long long)l * L.ldx;
    const int n = L.ns;
    // Gershgorin interval and pivot floor
    double lo = 0.0, hi = 0.0, emax2 = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
        lo = (i == 0) ? d[i] - r : fmin(lo, d[i] - r);
        hi = (i == 0) ? d[i] + r : fmax(hi, d[i] + r);
        if (i + 1 < n) emax2 = fmax(emax2, e[i] * e[i]);
    }
    const double tnorm = fmax(fabs(lo), fabs(hi));
    const double pivmin = 1e-300 * fmax(1.0, emax2);
    const int kidx = n - 1 - l;   // l-th largest = kidx-th smallest
    // bisection: count(x) = number of eigenvalues < x
    for (int it = 0; it < 128; ++it) {
        if (hi - lo <= 4.440892098500626e-16 * tnorm + pivmin) break;
        const double mid = 0.5 * (lo + hi);
        int cnt = 0;
        double q = d[0] - mid;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
        for (int i = 1; i < n; ++i) {
            q = d[i] - mid - e[i - 1] * e[i - 1] / q;
            if (fabs(q) < pivmin) q = -pivmin;
            cnt += q < 0.0;
        }
        if (cnt > kidx) hi = mid;
        else lo = mid;
    }
    const double lam = 0.5 * (lo + hi);
    // inverse iteration (T - lam I) x = b with T - lam I = L D L^T
    const double ptol = fmax(2.220446049250313e-16 * tnorm, 1e-300);
    for (int i = 0; i < n; ++i)
        x[i] = (double)(hash_u32((unsigned)(l * 7919 + i * 104729 + 17)) & 0xffffff) / 16777216.0 - 0.5;
    for (int it = 0; it < 3; ++it) {
        double q = d[0] - lam;
        if (fabs(q) < ptol) q = (q < 0.0) ? -ptol : ptol;
        piv[0] = q;
        for (int i = 1; i < n; ++i) {
            q = d[i] - lam - e[i - 1] * e[i - 1] / q;
            if (fabs(q) < ptol) q = (q < 0.0) ? -ptol : ptol;
            piv[i] = q;
        }
        // L y = b (in place), then L^T x = D^-1 y
        for (int i = 1; i < n; ++i) x[i] -= (e[i - 1] / piv[i - 1]) * x[i - 1];
        x[n - 1] /= piv[n - 1];
        for (int i = n - 2; i >= 0; --i) x[i] = (x[i] - e[i] * x[i + 1]) / piv[i];
        double mx = 0.0;
        for (int i = 0; i < n; ++i) mx = fmax(mx, fabs(x[i]));
        const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) {
            x[i] *= inv;
            nrm += x[i] * x[i];
        }
        const double s = nrm > 0.0 ? 1.0 / sqrt(nrm) : 1.0;
        for (int i = 0; i < n; ++i) x[i] *= s;
    }
    gs[L.oL + l] = lam;
}

// ---------------------------------------------------------------------------
// C: orthonormalise, back-transform, outputs
// ---------------------------------------------------------------------------
template <bool kLds>
__global__ __launch_bounds__(NT) void k_eig_fin(EigArgs a) {
    extern __shared__ double lds[];
    const EigLayout L = eig_layout(a.mz, a.tin, a.p, a.Dc);
    const int b = blockIdx.x, tid = threadIdx.x;
    const int ns = L.ns, tk = L.tk, ldx = L.ldx, lda = L.lda, ldz = L.ldz, tin = a.tin, p = a.p;
    double* gs = a.scratch + (long long)b * a.ss;
    double *X, *Am, *tau, *Z, *lam;
    if constexpr (kLds) {
        X = lds;
        Am = X + (long long)ldx * tk;
        tau = Am + (long long)lda * ns;
        Z = tau + ns;
        lam = Z + (long long)ldz * tin;
        for (long long i = tid; i < (long long)ldx * tk; i += NT) X[i] = gs[L.oX + i];
        for (long long i = tid; i < (long long)lda * ns; i += NT) Am[i] = gs[L.oA + i];
        for (int i = tid; i < ns; i += NT) tau[i] = gs[L.oT + i];
        for (long long i = tid; i < (long long)ldz * tin; i += NT) Z[i] = gs[L.oZ + i];
        for (int i = tid; i < tk; i += NT) lam[i] = gs[L.oL + i];
        __syncthreads();
    } else {
        X = gs + L.oX; Am = gs + L.oA; tau = gs + L.oT; Z = gs + L.oZ; lam = gs + L.oL;
    }
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
    // back-transformation: X <- H_0 ... H_{ns-3} X (reflector k acts on rows k+1..)
    {
        const int tpc = e_tpc(tk), ngroups = NT / tpc, g = tid / tpc, l = tid % tpc;
        for (int k = ns - 3; k >= 0; --k) {
            const double tq = tau[k];
            if (tq == 0.0) continue;
            for (int c0 = 0; c0 < tk; c0 += ngroups) {
                const int c = c0 + g;
                const bool act = c < tk;
                double* xc = X + (long long)(act ? c : 0) * ldx;
                double dot = 0.0;
                if (act) {
                    for (int i = k + 2 + l; i < ns; i += tpc) dot += Am[(long long)i * lda + k] * xc[i];
                    if (l == 0) dot += xc[k + 1];
                }
                dot = e_wave_sum(dot, tpc);
                if (act) {
                    const double f = tq * dot;
                    if (l == 0) xc[k + 1] -= f;
                    for (int i = k + 2 + l; i < ns; i += tpc) xc[i] -= f * Am[(long long)i * lda + k];
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
size_t eig_scratch_doubles(int mz, int tin, int p, int Dc) {
    return (size_t)eig_layout(mz, tin, p, Dc).total;
}

hipError_t launch_eig(const double* V, long long vs, const double* tau, long long ts, const double* G,
                      long long gs, int mz, int r, int tin, int p, int Dc, double* newU, long long us,
                      double* Gout, long long gos, double* scratch, long long ss, int batch,
                      hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    EigArgs a;
    a.V = V; a.vs = vs; a.tau = tau; a.ts = ts; a.G = G; a.gs = gs;
    a.mz = mz; a.r = r; a.tin = tin; a.p = p; a.Dc = Dc;
    a.newU = newU; a.us = us; a.Gout = Gout; a.gos = gos;
    a.scratch = scratch; a.ss = ss; a.batch = batch;
    const EigLayout L = eig_layout(mz, tin, p, Dc);
    const size_t cap = get_lds_cap() - 1024;
    const size_t bp = (size_t)L.lds_prep * sizeof(double), bf = (size_t)L.lds_fin * sizeof(double);
    if (bp <= cap) hipLaunchKernelGGL(k_eig_prep<true>, dim3(batch), dim3(NT), bp, st, a);
    else hipLaunchKernelGGL(k_eig_prep<false>, dim3(batch), dim3(NT), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int lpm = L.tk > 0 ? L.tk : 1;
    const long long lanes = (long long)batch * lpm;
    hipLaunchKernelGGL(k_eig_tri, dim3((unsigned)((lanes + 63) / 64)), dim3(64), 0, st, a, lpm);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (bf <= cap) hipLaunchKernelGGL(k_eig_fin<true>, dim3(batch), dim3(NT), bf, st, a);
    else hipLaunchKernelGGL(k_eig_fin<false>, dim3(batch), dim3(NT), 0, st, a);
    return hipGetLastError();
}

}  // namespace peps
