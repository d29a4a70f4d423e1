// Spin-spin correlation estimator (Sec. III-A): local value of S_m . S_n at a sampled
// configuration, sigma_m sigma_n / 4 plus half the ratio W(S')/W(S) of the configuration
// S' with the two spins exchanged (only where they differ), and the structure factor
// m_s^2(k) of a block of sites.
#include "common.h"
#include "kernels.h"

namespace peps {

// Exchanged configurations of every anti-parallel pair of every sample, packed in the
// order they are claimed: slot[b*P + p] = their index in Sx, or -1 (no contraction
// needed: equal spins or m == n).  One thread per (sample, pair).
__global__ void k_corr_pack(const int8_t* S, const int* pairs, int P, int N, int batch, int8_t* Sx,
                            int* slot, int* count) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)batch * P) return;
    const int b = (int)(t / P), p = (int)(t % P);
    const int m = pairs[2 * p], n = pairs[2 * p + 1];
    const int8_t* s = S + (long long)b * N;
    if (m == n || s[m] == s[n]) {
        slot[t] = -1;
        return;
    }
    const int k = atomicAdd(count, 1);
    slot[t] = k;
    int8_t* x = Sx + (long long)k * N;
    for (int i = 0; i < N; ++i) x[i] = s[i];
    x[m] = s[n];
    x[n] = s[m];
}
hipError_t launch_corr_pack(const int8_t* S, const int* pairs, int P, int N, int batch, int8_t* Sx, int* slot,
                            int* count, hipStream_t st) {
    const long long n = (long long)batch * P;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_corr_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, S, pairs, P, N, batch,
                       Sx, slot, count);
    return hipGetLastError();
}

// Local values v[b][p] and the sample flags: the flag of S, or 3 when the contraction
// of an exchanged configuration is not finite (a zero W(S') gives a zero ratio).
__global__ void k_corr_values(const int8_t* S, const int* pairs, int P, int N, int batch, const double* la,
                              const int8_t* sg, const int8_t* fl, const int* slot, const double* lax,
                              const int8_t* sgx, const int8_t* flx, double* v, int8_t* flags) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const int8_t* s = S + (long long)b * N;
    int8_t f = fl[b];
    for (int p = 0; p < P; ++p) {
        const int m = pairs[2 * p], n = pairs[2 * p + 1];
        double x;
        if (m == n) {
            x = 0.75;
        } else {
            x = 0.25 * (double)((1 - 2 * s[m]) * (1 - 2 * s[n]));
            const int k = slot[(long long)b * P + p];
            if (k >= 0 && f == 0) {
                if (flx[k] == 0)
                    x += 0.5 * (double)(sgx[k] * sg[b]) * exp(lax[k] - la[b]);
                else if (flx[k] != 2)
                    f = 3;
            }
        }
        v[(long long)b * P + p] = f == 0 ? x : __longlong_as_double(0x7ff8000000000000LL);
    }
    if (flags) flags[b] = f;
}
hipError_t launch_corr_values(const int8_t* S, const int* pairs, int P, int N, int batch, const double* la,
                              const int8_t* sg, const int8_t* fl, const int* slot, const double* lax,
                              const int8_t* sgx, const int8_t* flx, double* v, int8_t* flags, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_corr_values, dim3((batch + 127) / 128), dim3(128), 0, st, S, pairs, P, N, batch, la, sg,
                       fl, slot, lax, sgx, flx, v, flags);
    return hipGetLastError();
}

// means[p] = mean of v[b][p] over the samples with flag 0: 256 ordered runs of samples
// per pair, then the runs in order (deterministic).  One block per pair.
__global__ void k_corr_means(const double* v, const int8_t* flags, int P, int batch, double* means) {
    __shared__ double ps[256], pc[256];
    const int p = blockIdx.x, t = threadIdx.x, per = (batch + 255) / 256;
    double s = 0.0, c = 0.0;
    for (int b = t * per; b < batch && b < (t + 1) * per; ++b)
        if (flags[b] == 0) {
            s += v[(long long)b * P + p];
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
    means[p] = c == 0.0 ? __longlong_as_double(0x7ff8000000000000LL) : s / c;
}
hipError_t launch_corr_means(const double* v, const int8_t* flags, int P, int batch, double* means,
                             hipStream_t st) {
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_corr_means, dim3(P), dim3(256), 0, st, v, flags, P, batch, means);
    return hipGetLastError();
}

// m_s^2(k) = (1/Nb^2) sum_{i,j} C[i][j] cos(k . (r_i - r_j)), r = (column, row): the real
// part of the Fourier sum (C real).  One thread per k, terms in row-major order.
__global__ void k_structure_factor(int Lx, int nb, const int* sites, const double* C, int nk, const double* kv,
                                   double* out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nk) return;
    const double kx = kv[2 * q], ky = kv[2 * q + 1];
    double s = 0.0;
    for (int i = 0; i < nb; ++i) {
        const int xi = sites[i] % Lx, yi = sites[i] / Lx;
        for (int j = 0; j < nb; ++j) {
            const int dx = xi - sites[j] % Lx, dy = yi - sites[j] / Lx;
            s += C[(long long)i * nb + j] * cos(kx * dx + ky * dy);
        }
    }
    out[q] = s / ((double)nb * nb);
}
hipError_t launch_structure_factor(int Lx, int nb, const int* sites, const double* C, int nk, const double* kv,
                                   double* out, hipStream_t st) {
    if (nk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_structure_factor, dim3((nk + 63) / 64), dim3(64), 0, st, Lx, nb, sites, C, nk, kv, out);
    return hipGetLastError();
}

}  // namespace peps
