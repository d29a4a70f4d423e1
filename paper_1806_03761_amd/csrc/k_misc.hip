// Small per-sample kernels: validation, rescaling of partial contractions,
// spin-flip amplitude ratios, local-energy assembly and log-derivative output.
#include "common.h"
#include "kernels.h"

namespace peps {

static constexpr int NT = 256;

__device__ inline double wsum(double v) { return lane_group_sum(v, 64); }
__device__ inline double wmax(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double bsum(double v, double* red) {
    v = wsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}
__device__ inline double bmax(double v, double* red) {
    v = wmax(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < NT / 64; ++i) s = fmax(s, red[i]);
    return s;
}

__global__ void k_fill(double* x, long long n, double v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}
__global__ void k_fill_i8(int8_t* x, long long n, int8_t v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

hipError_t launch_fill(double* x, long long n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_i8(int8_t* x, long long n, int8_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, v);
    return hipGetLastError();
}

__global__ void k_copy_i8(const int8_t* src, int8_t* dst, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}
hipError_t launch_copy_i8(const int8_t* src, int8_t* dst, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_i8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

// flags[b] = 1 if any S[b][m] is outside {0, 1}, else 0.
__global__ void k_check_configs(const int8_t* S, int N, int batch, int8_t* flags) {
    const int b = blockIdx.x;
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        const int8_t v = S[(long long)b * N + m];
        if (v != 0 && v != 1) bad = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) flags[b] = bad ? 1 : 0;
}
hipError_t launch_check_configs(const int8_t* S, int N, int batch, int8_t* flags, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_configs, dim3(batch), dim3(256), 0, st, S, N, batch, flags);
    return hipGetLastError();
}

// x /= max|x|, lout = lin + ln max|x| (unchanged when x is all zero or not finite).
__global__ __launch_bounds__(NT) void k_rescale(double* x, long long xs, int n, const double* lin,
                                                double* lout) {
    __shared__ double red[NT / 64];
    const int b = blockIdx.x;
    double* xb = x + (long long)b * xs;
    double mx = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) mx = fmax(mx, fabs(xb[i]));
    mx = bmax(mx, red);
    const bool ok = mx > 0.0 && isfinite(mx);
    if (ok) {
        const double inv = 1.0 / mx;
        for (int i = threadIdx.x; i < n; i += NT) xb[i] *= inv;
    }
    if (threadIdx.x == 0) lout[b] = (lin ? lin[b] : 0.0) + (ok ? log(mx) : 0.0);
}
hipError_t launch_rescale(double* x, long long xs, int n, const double* lin, double* lout,
                          int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rescale, dim3(batch), dim3(NT), 0, st, x, xs, n, lin, lout);
    return hipGetLastError();
}

// ratio[b][bond] = <F,G> exp(la + lb - lnW) * sgW: W(S')/W(S) from partial contractions.
__global__ __launch_bounds__(NT) void k_ratio(const double* F, long long fs, const double* G,
                                              long long gs, int n, const double* la,
                                              const double* lb, const double* lnW,
                                              const double* sgW, double* ratio, int nbonds,
                                              int bond, const int8_t* skip) {
    __shared__ double red[NT / 64];
    const int b = blockIdx.x;
    // a bond of equal spins has no exchange term: its flipped partials were not formed
    if (skip && skip[(long long)b * nbonds + bond] == 0) {
        if (threadIdx.x == 0) ratio[(long long)b * nbonds + bond] = 0.0;
        return;
    }
    const double* Fb = F + (long long)b * fs;
    const double* Gb = G + (long long)b * gs;
    // each thread's terms in ascending i, their loads issued 8 strides at a time
    double d = 0.0;
    for (int i0 = 0; i0 < n; i0 += 8 * NT) {
        double f[8], g[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + threadIdx.x + u * NT;
            f[u] = Fb[i < n ? i : 0];
            g[u] = Gb[i < n ? i : 0];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + threadIdx.x + u * NT < n) d += f[u] * g[u];
    }
    d = bsum(d, red);
    if (threadIdx.x == 0) {
        double r;
        if (d == 0.0) {
            r = 0.0;
        } else {
            const double sg = sgW[b];
            r = (sg == 0.0) ? NAN : copysign(exp(log(fabs(d)) + la[b] + lb[b] - lnW[b]), d) * sg;
        }
        ratio[(long long)b * nbonds + bond] = r;
    }
}
hipError_t launch_ratio(const double* F, long long fs, const double* G, long long gs, int n,
                        const double* la, const double* lb, const double* lnW, const double* sgW,
                        double* ratio, int nbonds, int bond, int batch, hipStream_t st,
                        const int8_t* skip) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ratio, dim3(batch), dim3(NT), 0, st, F, fs, G, gs, n, la, lb, lnW, sgW,
                       ratio, nbonds, bond, skip);
    return hipGetLastError();
}

// Full sandwich value from the last (1x1x...) partial: ln|W| = lam + ln|P|, sign.
__global__ void k_sandwich_value(const double* P, long long ps, const double* lam, double* lnW,
                                 double* sgW, int batch) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const double v = P[(long long)b * ps];
    if (v == 0.0 || !isfinite(v)) {
        lnW[b] = (v == 0.0) ? -INFINITY : NAN;
        sgW[b] = (v == 0.0) ? 0.0 : NAN;
    } else {
        lnW[b] = lam[b] + log(fabs(v));
        sgW[b] = v > 0.0 ? 1.0 : -1.0;
    }
}
hipError_t launch_sandwich_value(const double* P, long long ps, const double* lam, double* lnW,
                                 double* sgW, int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sandwich_value, dim3((batch + 255) / 256), dim3(256), 0, st, P, ps, lam,
                       lnW, sgW, batch);
    return hipGetLastError();
}

// act[b][bond] = [the two spins of the bond differ], bonds in the order of k_eloc
__global__ void k_bond_active(const int8_t* S, int Lx, int Ly, int8_t* act, int nbonds, int batch) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)batch * nbonds) return;
    const int b = (int)(e / nbonds), k = (int)(e % nbonds);
    const int nH = Ly * (Lx - 1), nV = (Ly - 1) * Lx, nD = (Ly - 1) * (Lx - 1);
    int m, n;
    if (k < nH) {
        m = (k / (Lx - 1)) * Lx + k % (Lx - 1); n = m + 1;
    } else if (k < nH + nV) {
        m = k - nH; n = m + Lx;
    } else if (k < nH + nV + nD) {
        const int q = k - nH - nV; m = (q / (Lx - 1)) * Lx + q % (Lx - 1); n = m + Lx + 1;
    } else {
        const int q = k - nH - nV - nD; m = (q / (Lx - 1)) * Lx + q % (Lx - 1) + 1; n = m + Lx - 1;
    }
    const int8_t* s = S + (long long)b * Lx * Ly;
    act[e] = s[m] != s[n] ? 1 : 0;
}
hipError_t launch_bond_active(const int8_t* S, int Lx, int Ly, int8_t* act, int nbonds, int batch, hipStream_t st) {
    const long long n = (long long)batch * nbonds;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bond_active, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, S, Lx, Ly, act, nbonds,
                       batch);
    return hipGetLastError();
}

// E(S) = sum_bonds J [sigma sigma'/4 + 1/2 [s != s'] ratio]; bonds in the fixed order
// J1 horizontal (i, j<Lx-1), J1 vertical (i<Ly-1, j), J2 (i,j)-(i+1,j+1), J2 (i,j+1)-(i+1,j).
__global__ void k_eloc(ElocArgs a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.batch) return;
    const int Lx = a.Lx, Ly = a.Ly, N = Lx * Ly;
    const int8_t* s = a.S + (long long)b * N;
    const double* rt = a.ratio + (long long)b * a.nbonds;
    if (a.flags[b] != 0) {
        a.e_loc[b] = NAN;
        return;
    }
    double E = 0.0;
    int id = 0;
    auto term = [&](int m, int n, double J, int bid) {
        const int sm = s[m], sn = s[n];
        E += J * ((sm == sn) ? 0.25 : -0.25);
        if (sm != sn) E += J * 0.5 * rt[bid];
    };
    for (int i = 0; i < Ly; ++i)
        for (int j = 0; j + 1 < Lx; ++j) term(i * Lx + j, i * Lx + j + 1, a.J1, id++);
    for (int i = 0; i + 1 < Ly; ++i)
        for (int j = 0; j < Lx; ++j) term(i * Lx + j, (i + 1) * Lx + j, a.J1, id++);
    for (int i = 0; i + 1 < Ly; ++i)
        for (int j = 0; j + 1 < Lx; ++j) term(i * Lx + j, (i + 1) * Lx + j + 1, a.J2, id++);
    for (int i = 0; i + 1 < Ly; ++i)
        for (int j = 0; j + 1 < Lx; ++j) term(i * Lx + j + 1, (i + 1) * Lx + j, a.J2, id++);
    a.e_loc[b] = E;
}
hipError_t launch_eloc(const ElocArgs& a, hipStream_t st) {
    if (a.batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eloc, dim3((a.batch + 127) / 128), dim3(128), 0, st, a);
    return hipGetLastError();
}

// log_abs = logU + lnW, sign; zero amplitude -> flag 2, non-finite -> flag 3.
__global__ void k_amp_out(const double* logU, const double* lnW, const double* sgW,
                          int8_t* flags, double* log_abs, int8_t* sign, int batch) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    int8_t f = flags[b];
    double la = logU[b] + lnW[b];
    double sg = sgW[b];
    if (f == 0) {
        if (sg == 0.0 || la == -INFINITY) {
            f = 2;
        } else if (!isfinite(la) || !isfinite(sg)) {
            f = 3;
        }
    }
    if (f == 1 || f == 3) {
        la = NAN;
        sg = 0.0;
    } else if (f == 2) {
        la = -INFINITY;
        sg = 0.0;
    }
    flags[b] = f;
    if (log_abs) log_abs[b] = la;
    if (sign) sign[b] = (int8_t)(sg > 0.0 ? 1 : (sg < 0.0 ? -1 : 0));
}
hipError_t launch_amp_out(const double* logU, const double* lnW, const double* sgW,
                          int8_t* flags, double* log_abs, int8_t* sign, int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_amp_out, dim3((batch + 255) / 256), dim3(256), 0, st, logU, lnW, sgW,
                       flags, log_abs, sign, batch);
    return hipGetLastError();
}

__global__ void k_nan_flagged(const int8_t* flags, double* log_abs, int8_t* sign, double* e_loc,
                              int batch) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    if (flags[b] == 1 || flags[b] == 3) {
        if (e_loc) e_loc[b] = NAN;
        if (log_abs) log_abs[b] = NAN;
        if (sign) sign[b] = 0;
    }
}
hipError_t launch_nan_flagged(const int8_t* flags, double* log_abs, int8_t* sign, double* e_loc,
                              int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nan_flagged, dim3((batch + 255) / 256), dim3(256), 0, st, flags, log_abs,
                       sign, e_loc, batch);
    return hipGetLastError();
}

// Delta = B / <B, T> over the live block (l<Dl, u<Du, r<Dr, d<Dd) of site `site`.
// Dsite points at the site's D^4 block of sample 0; samples are `bs` doubles apart.
__global__ __launch_bounds__(NT) void k_grad_site(double* Dsite, long long bs, const double* A,
                                                  const int8_t* S, int site, int N, int D, int Dl,
                                                  int Du, int Dr, int Dd) {
    __shared__ double red[NT / 64];
    const int b = blockIdx.x;
    const int D2 = D * D, D3 = D2 * D, D4 = D3 * D;
    double* Bb = Dsite + (long long)b * bs;
    const int s = S[(long long)b * N + site] & 1;
    const double* T = A + ((long long)site * 2 + s) * D4;
    const int nl = Dl * Du * Dr * Dd;
    double w = 0.0;
    for (int e = threadIdx.x; e < nl; e += NT) {
        int x = e;
        const int d = x % Dd; x /= Dd;
        const int r = x % Dr; x /= Dr;
        const int u = x % Du;
        const int l = x / Du;
        const int o = l * D3 + u * D2 + r * D + d;
        w += Bb[o] * T[o];
    }
    w = bsum(w, red);
    const double inv = (w != 0.0) ? 1.0 / w : 0.0;
    for (int e = threadIdx.x; e < D4; e += NT) Bb[e] *= inv;
}
hipError_t launch_grad_site(double* Dsite, long long bs, const double* A, const int8_t* S, int site,
                            int N, int D, int Dl, int Du, int Dr, int Dd, int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_site, dim3(batch), dim3(NT), 0, st, Dsite, bs, A, S, site, N, D, Dl,
                       Du, Dr, Dd);
    return hipGetLastError();
}

// out[b][m][s][e] from Delta[b][m][e] (the slice s = S[b][m]; the other slice is zero).
__global__ void k_grad_store(const double* Dall, const int8_t* S, int N, int D4,
                             const int8_t* flags, double* out) {
    const int b = blockIdx.y;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = 2LL * N * D4;
    if (e >= per) return;
    const int m = (int)(e / (2 * D4));
    const int rem = (int)(e % (2 * D4));
    const int slice = rem / D4, k = rem % D4;
    const int s = S[(long long)b * N + m] & 1;
    const int8_t f = flags[b];
    double v = 0.0;
    if (f == 1 || f == 3) {
        v = NAN;
    } else if (f == 0 && slice == s) {
        v = Dall[((long long)b * N + m) * D4 + k];
    }
    out[(long long)b * per + e] = v;
}
hipError_t launch_grad_store(const double* Dall, const int8_t* S, int N, int D4, const int8_t* flags,
                             double* out, int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    const long long per = 2LL * N * D4;
    hipLaunchKernelGGL(k_grad_store, dim3((unsigned)((per + 255) / 256), batch), dim3(256), 0, st,
                       Dall, S, N, D4, flags, out);
    return hipGetLastError();
}

// out[m][s][e] (+)= sum over b in order of w_b [S_b[m] = s] Delta_b[m][e]; flagged samples skipped.
// Batch sums of Eq. (5), in two passes so the whole grid reads Delta once: pass one,
// block row p adds samples [p per, (p+1) per) in order, thread (m, e) keeping both the
// weighted and the plain sum for each spin value of S_b[m]; pass two adds the partitions
// in order.  Fixed partitions and orders make the result deterministic.
__global__ void k_grad_partial(const double* Dall, const int8_t* S, int N, int D4, const int8_t* flags,
                               const double* w, int batch, int per, double* ws1, double* ws0) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nd = (long long)N * D4;
    if (e >= nd) return;
    const int m = (int)(e / D4), k = (int)(e % D4);
    double a1[2] = {0.0, 0.0}, a0[2] = {0.0, 0.0};
    const int b0 = blockIdx.y * per, b1 = min(batch, b0 + per);
    for (int b = b0; b < b1; ++b) {
        if (flags[b] != 0) continue;
        const int s = S[(long long)b * N + m] & 1;
        const double d = Dall[((long long)b * N + m) * D4 + k];
        const double wb = w ? w[b] : 1.0;
        if (s) { a1[1] += wb * d; a0[1] += d; }
        else { a1[0] += wb * d; a0[0] += d; }
    }
    const long long o = (long long)blockIdx.y * 2 * nd + (long long)m * 2 * D4 + k;
    ws1[o] = a1[0]; ws1[o + D4] = a1[1];
    if (ws0) { ws0[o] = a0[0]; ws0[o + D4] = a0[1]; }
}
__global__ void k_grad_parts_sum(const double* ws, int parts, long long n, int accumulate, double* out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int p = 0; p < parts; ++p) acc += ws[(long long)p * n + i];
    out[i] = accumulate ? out[i] + acc : acc;
}
int grad_parts(int batch) { return batch / 64 < 1 ? 1 : (batch / 64 > kGradParts ? kGradParts : batch / 64); }
hipError_t launch_grad_reduce(const double* Dall, const int8_t* S, int N, int D4, const int8_t* flags,
                              const double* w, int accumulate, double* out1, double* out0, double* ws,
                              int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    const int parts = grad_parts(batch), per = (batch + parts - 1) / parts;
    const long long nd = (long long)N * D4, n = 2 * nd;
    double* ws1 = ws;
    double* ws0 = out0 ? ws + (long long)parts * n : nullptr;
    hipLaunchKernelGGL(k_grad_partial, dim3((unsigned)((nd + 255) / 256), parts), dim3(256), 0, st, Dall, S, N,
                       D4, flags, w, batch, per, ws1, ws0);
    hipLaunchKernelGGL(k_grad_parts_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ws1, parts, n,
                       accumulate, out1);
    if (out0)
        hipLaunchKernelGGL(k_grad_parts_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ws0, parts,
                           n, accumulate, out0);
    return hipGetLastError();
}

// acc[0] (+)= sum of e_loc over flag-0 samples, acc[1] (+)= their count: 256 threads each
// sum a contiguous run in order, thread 0 adds the runs in order.
__global__ void k_energy_sums(const double* e_loc, const int8_t* flags, int batch, double* acc,
                              int accumulate) {
    __shared__ double ps[256], pc[256];
    const int t = threadIdx.x, per = (batch + 255) / 256;
    double s = 0.0, c = 0.0;
    for (int b = t * per; b < batch && b < (t + 1) * per; ++b)
        if (flags[b] == 0) {
            s += e_loc[b];
            c += 1.0;
        }
    ps[t] = s;
    pc[t] = c;
    __syncthreads();
    if (t != 0) return;
    s = 0.0;
    c = 0.0;
    for (int i = 0; i < 256; ++i) {
        s += ps[i];
        c += pc[i];
    }
    acc[0] = accumulate ? acc[0] + s : s;
    acc[1] = accumulate ? acc[1] + c : c;
}
hipError_t launch_energy_sums(const double* e_loc, const int8_t* flags, int batch, double* acc,
                              int accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_sums, dim3(1), dim3(256), 0, st, e_loc, flags, batch, acc, accumulate);
    return hipGetLastError();
}

// Metropolis step (Sec. II-B, steps 1-3 of the sampling loop), per sample (one thread):
// bond k = min(floor(u0 nb), nb - 1) of the J1 and J2 bonds in the order horizontal,
// vertical, diagonal (i,j)-(i+1,j+1), anti-diagonal (i,j+1)-(i+1,j).
__device__ inline void mc_bond(int k, int Lx, int Ly, int* m, int* n) {
    const int nh = Ly * (Lx - 1), nv = (Ly - 1) * Lx, nd = (Ly - 1) * (Lx - 1);
    if (k < nh) {
        const int i = k / (Lx - 1), j = k % (Lx - 1);
        *m = i * Lx + j; *n = *m + 1;
    } else if (k < nh + nv) {
        k -= nh;
        *m = k; *n = k + Lx;
    } else if (k < nh + nv + nd) {
        k -= nh + nv;
        const int i = k / (Lx - 1), j = k % (Lx - 1);
        *m = i * Lx + j; *n = (i + 1) * Lx + j + 1;
    } else {
        k -= nh + nv + nd;
        const int i = k / (Lx - 1), j = k % (Lx - 1);
        *m = i * Lx + j + 1; *n = (i + 1) * Lx + j;
    }
}

// The drawn bond of chain b (u[2b] picks it) and whether its two spins differ.
__device__ inline void mc_draw(const double* u, int b, int Lx, int Ly, int* m, int* n) {
    const int nb = Ly * (Lx - 1) + (Ly - 1) * Lx + 2 * (Ly - 1) * (Lx - 1);
    const double kf = floor(u[2LL * b] * nb);
    const int k = kf < (double)(nb - 1) ? (int)kf : nb - 1;
    mc_bond(k, Lx, Ly, m, n);
}

__global__ void k_mc_mark(const int8_t* S, const double* u, int Lx, int Ly, int batch, int8_t* moved) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    int m, n;
    mc_draw(u, b, Lx, Ly, &m, &n);
    const int8_t* s = S + (long long)b * Lx * Ly;
    moved[b] = s[m] != s[n];
}

// pos[b] = number of moved chains before b, count = all of them: one block of 1024
// threads, each summing a contiguous run of chains, then a scan of the run totals in LDS
// (deterministic: the proposals are packed in chain order).
__global__ __launch_bounds__(1024) void k_mc_scan(const int8_t* moved, int batch, int* pos, int* count) {
    __shared__ int run[1024];
    const int t = threadIdx.x, per = (batch + 1023) / 1024;
    const long long lo = (long long)t * per, hi = lo + per < batch ? lo + per : batch;
    int c = 0;
    for (long long b = lo; b < hi; ++b) c += moved[b];
    run[t] = c;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {      // inclusive Hillis-Steele scan
        const int v = t >= off ? run[t - off] : 0;
        __syncthreads();
        run[t] += v;
        __syncthreads();
    }
    int p = run[t] - c;
    for (long long b = lo; b < hi; ++b) {
        pos[b] = p;
        p += moved[b];
    }
    if (t == 1023) *count = run[1023];
}

// the proposal of every moved chain at its packed position: S with the bond's spins
// exchanged (S^z is kept)
__global__ void k_mc_build(const int8_t* S, const double* u, const int8_t* moved, const int* pos, int Lx, int Ly,
                           int batch, int8_t* Sp) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch || !moved[b]) return;
    const int N = Lx * Ly;
    int m, n;
    mc_draw(u, b, Lx, Ly, &m, &n);
    const int8_t* s = S + (long long)b * N;
    int8_t* sp = Sp + (long long)pos[b] * N;
    for (int i = 0; i < N; ++i) sp[i] = s[i];
    sp[m] = s[n];
    sp[n] = s[m];
}

hipError_t launch_mc_propose(const int8_t* S, const double* u, int Lx, int Ly, int batch, int8_t* moved, int* pos,
                             int* count, int8_t* Sp, int* hcount, hipStream_t st) {
    *hcount = 0;
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mc_mark, dim3((batch + 127) / 128), dim3(128), 0, st, S, u, Lx, Ly, batch, moved);
    hipLaunchKernelGGL(k_mc_scan, dim3(1), dim3(1024), 0, st, moved, batch, pos, count);
    hipLaunchKernelGGL(k_mc_build, dim3((batch + 127) / 128), dim3(128), 0, st, S, u, moved, pos, Lx, Ly, batch,
                       Sp);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(hcount, count, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

// accept when the chain moved, its proposal has flag 0 and
// u1 < W(S')^2 / W(S)^2 = exp(2 (ln|W(S')| - ln|W(S)|)); proposal data at the packed position
__global__ void k_mc_accept(int8_t* S, const int8_t* Sp, const int8_t* moved, const int* pos, const double* u,
                            const double* lap, const int8_t* sgp, const int8_t* flp, double* log_abs,
                            int8_t* sign, int8_t* accepted, int N, int batch) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    bool acc = false;
    if (moved[b]) {
        const int k = pos[b];
        acc = flp[k] == 0 && u[2LL * b + 1] < exp(2.0 * (lap[k] - log_abs[b]));
        if (acc) {
            for (int i = 0; i < N; ++i) S[(long long)b * N + i] = Sp[(long long)k * N + i];
            log_abs[b] = lap[k];
            sign[b] = sgp[k];
        }
    }
    if (accepted) accepted[b] = acc ? 1 : 0;
}
hipError_t launch_mc_accept(int8_t* S, const int8_t* Sp, const int8_t* moved, const int* pos, const double* u,
                            const double* lap, const int8_t* sgp, const int8_t* flp, double* log_abs,
                            int8_t* sign, int8_t* accepted, int N, int batch, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mc_accept, dim3((batch + 127) / 128), dim3(128), 0, st, S, Sp, moved, pos, u, lap, sgp,
                       flp, log_abs, sign, accepted, N, batch);
    return hipGetLastError();
}

// Sampled energy of Eq. (3) from the ordered sums of k_energy_sums: out = {mean, count}
// (NaN mean when no sample has flag 0).
__global__ void k_energy_mean(const double* acc, double* out) {
    if (threadIdx.x != 0) return;
    out[0] = acc[1] == 0.0 ? __longlong_as_double(0x7ff8000000000000LL) : acc[0] / acc[1];
    out[1] = acc[1];
}
hipError_t launch_energy_mean(const double* acc, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_mean, dim3(1), dim3(64), 0, st, acc, out);
    return hipGetLastError();
}

// Gradient-optimisation update: A[i] moves against the sign of grad[i] by p[i] * dt; a
// zero or NaN derivative leaves it.  The step p * dt is rounded on its own before the
// addition (no fused multiply-add), so the result is the exactly rounded rule.
__global__ void k_go_update(double* A, const double* grad, const double* p, double dt, long long n) {
#pragma clang fp contract(off)
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double g = grad[i], step = p[i] * dt, a = A[i];
    A[i] = g > 0.0 ? a - step : (g < 0.0 ? a + step : a);
}
hipError_t launch_go_update(double* A, const double* grad, const double* p, double dt, long long n,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_go_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, grad, p, dt, n);
    return hipGetLastError();
}

// Eq. (5): dE/dA = 2 <Delta E> - 2 <Delta><E> with <.> the mean over flag-0 samples.
__global__ void k_energy_grad_combine(const double* G1, const double* G0, const double* acc,
                                      long long n, double* out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double cnt = acc[1];
    if (cnt == 0.0) {
        out[i] = 0.0;
        return;
    }
    const double Em = acc[0] / cnt;
    out[i] = 2.0 * G1[i] / cnt - 2.0 * (G0[i] / cnt) * Em;
}
hipError_t launch_energy_grad_combine(const double* G1, const double* G0, const double* acc,
                                      long long n, double* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_energy_grad_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       G1, G0, acc, n, out);
    return hipGetLastError();
}

}  // namespace peps
