// Fused two-row sandwich step in float32 (Sec. 3, Eq. (4): the two-row transfer that
// carries the partial contraction of rows i and i+1 between the boundary MPSs across
// one column).
//
// Unfused, the step is four batched GEMMs whose three temporaries (each Dc^2 D^3 per
// sample) make the round trip through HBM.  Here one workgroup owns one sample: the
// incoming partial, the two environment tensors and the two spin-selected site tensors
// are staged once into LDS, thread (l, c') (lower-left and upper-right boundary bonds,
// the indices that stay free through the first three contractions) keeps its D^3 slice
// of each temporary in registers, and the last contraction, which sums over l (forward)
// or c' (backward), goes through an LDS copy of the third temporary.  Every product
// accumulates in the order its unfused GEMM uses (fma, k ascending, operands rounded
// to float32 first), so the result equals the unfused float32 path value for value.
//
// Index names (forward):  P[c][b][b'][l] -> Pout[c'][a][a'][l']
//   U[c][u][c'] upper environment, L[l][q][l'] lower environment,
//   S1[b][u][a][m] site (i,j), S2[b'][m][a'][q] site (i+1,j) (left, up, right, down).
// Backward: Q[c'][a][a'][l'] -> Qout[c][b][b'][l] with the same tensors.
#include "common.h"
#include "kernels.h"

namespace peps {

static constexpr int kPD = 4;    // PEPS legs (horizontal and vertical) of the fused path
static constexpr int kPX = 16;   // boundary bonds of the fused path
static constexpr int kPairLds = 2 * 256 + 2 * 1024 + 16384;   // floats

bool pair_step_fits(const PairArgs& a) {
    const int legs[5] = {a.h, a.h1, a.Du, a.Dm, a.Dq};
    const int bonds[4] = {a.cu, a.cu1, a.cl, a.cl1};
    for (int v : legs)
        if (v < 1 || v > kPD) return false;
    for (int v : bonds)
        if (v < 1 || v > kPX) return false;
    return kPairLds * sizeof(float) <= get_lds_cap() - 1024;
}

__device__ inline float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }

template <bool FWD>
__global__ __launch_bounds__(256) void k_pair_step(PairArgs a) {
    extern __shared__ __align__(16) float sm[];
    float* Sa = sm;              // site (i,j), 4^4, zero padded
    float* Sb = Sa + 256;        // site (i+1,j)
    float* Ue = Sb + 256;        // upper environment, 16 x 16 x 4
    float* Le = Ue + 1024;       // lower environment
    float* Big = Le + 1024;      // incoming partial, later the third temporary
    const int b = blockIdx.x, tid = threadIdx.x;
    if (b >= a.batch) return;
    const int cu = a.cu, cu1 = a.cu1, cl = a.cl, cl1 = a.cl1;
    const int Du = a.Du, Dm = a.Dm, Dq = a.Dq, h = a.h, h1 = a.h1;
    const double* X = a.X + (long long)b * a.xs;
    const double* U = a.U + (long long)b * a.us;
    const double* L = a.L + (long long)b * a.ls;
    const double* s1 = a.site1 + (long long)((a.sel1[(long long)b * a.sel_bs] ^ a.flip1) & 1) * a.slice;
    const double* s2 = a.site2 + (long long)((a.sel2[(long long)b * a.sel_bs] ^ a.flip2) & 1) * a.slice;

    // ---- staging (float32, zero padded) ----
    {
        const int x0 = tid >> 6, x1 = (tid >> 4) & 3, x2 = (tid >> 2) & 3, x3 = tid & 3;
        // FWD: Sa[b][u][a][m], Sb[b'][m][a'][q];  BWD: Sa[a][m][b][u], Sb[a'][q][b'][m]
        int lb, up, rt, dn;
        if (FWD) { lb = x0; up = x1; rt = x2; dn = x3; }
        else { rt = x0; dn = x1; lb = x2; up = x3; }
        Sa[tid] = (lb < h && up < Du && rt < h1 && dn < Dm)
                      ? (float)s1[lb * a.D3 + up * a.D2 + rt * a.D + dn] : 0.f;
        if (FWD) { lb = x0; up = x1; rt = x2; dn = x3; }
        else { rt = x0; dn = x1; lb = x2; up = x3; }
        Sb[tid] = (lb < h && up < Dm && rt < h1 && dn < Dq)
                      ? (float)s2[lb * a.D3 + up * a.D2 + rt * a.D + dn] : 0.f;
    }
    for (int e = tid; e < 1024; e += 256) {
        int c, u, cp;
        if (FWD) { c = e >> 6; cp = (e >> 2) & 15; u = e & 3; }     // Ue[c][c'][u]
        else { u = e >> 8; cp = (e >> 4) & 15; c = e & 15; }        // Ue[u][c'][c]
        Ue[e] = (c < cu && u < Du && cp < cu1) ? (float)U[((long long)c * Du + u) * cu1 + cp] : 0.f;
        int l, q, lp;
        if (FWD) { l = e >> 6; q = (e >> 4) & 3; lp = e & 15; }     // Le[l][q][l']
        else { lp = e >> 6; l = (e >> 2) & 15; q = e & 3; }         // Le[l'][l][q]
        Le[e] = (l < cl && q < Dq && lp < cl1) ? (float)L[((long long)l * Dq + q) * cl1 + lp] : 0.f;
    }
    for (int e = tid; e < 4096; e += 256) {
        if (FWD) {   // Big[c][l][b][b'] = P[c][b][b'][l]
            const int c = e >> 8, l = (e >> 4) & 15, bb = (e >> 2) & 3, bp = e & 3;
            Big[e] = (c < cu && l < cl && bb < h && bp < h)
                         ? (float)X[(long long)c * h * h * cl + ((long long)bb * h + bp) * cl + l] : 0.f;
        } else {     // Big[l'][c'][a][a'] = Q[c'][a][a'][l']
            const int lp = e >> 8, cp = (e >> 4) & 15, aa = (e >> 2) & 3, ap = e & 3;
            Big[e] = (lp < cl1 && cp < cu1 && aa < h1 && ap < h1)
                         ? (float)X[(((long long)cp * h1 + aa) * h1 + ap) * cl1 + lp] : 0.f;
        }
    }
    __syncthreads();

    // ---- three contractions with the slice of thread (l, c') in registers ----
    const int l = tid >> 4, cp = tid & 15;
    float T1[kPD][kPD][kPD], T2[kPD][kPD][kPD];
#pragma unroll
    for (int x = 0; x < kPD; ++x)
#pragma unroll
        for (int y = 0; y < kPD; ++y)
#pragma unroll
            for (int z = 0; z < kPD; ++z) T1[x][y][z] = 0.f;
    if (FWD) {
        // T1[b][b'][u] = sum_c P[c][b][b'][l] U[c][u][c']
        for (int c = 0; c < cu; ++c) {
            float pv[kPD][kPD];
#pragma unroll
            for (int x = 0; x < kPD; ++x) {
                const float4 t = ld4(Big + ((c * kPX + l) * kPD + x) * kPD);
                pv[x][0] = t.x; pv[x][1] = t.y; pv[x][2] = t.z; pv[x][3] = t.w;
            }
            const float4 uu = ld4(Ue + (c * kPX + cp) * kPD);
            const float uv[kPD] = {uu.x, uu.y, uu.z, uu.w};
#pragma unroll
            for (int x = 0; x < kPD; ++x)
#pragma unroll
                for (int y = 0; y < kPD; ++y)
#pragma unroll
                    for (int z = 0; z < kPD; ++z) T1[x][y][z] = fmaf(pv[x][y], uv[z], T1[x][y][z]);
        }
    } else {
        // T1[q][a][a'] = sum_l' L[l][q][l'] Q[c'][a][a'][l']
        for (int lp = 0; lp < cl1; ++lp) {
            float qv[kPD][kPD];
#pragma unroll
            for (int x = 0; x < kPD; ++x) {
                const float4 t = ld4(Big + ((lp * kPX + cp) * kPD + x) * kPD);
                qv[x][0] = t.x; qv[x][1] = t.y; qv[x][2] = t.z; qv[x][3] = t.w;
            }
            const float4 ll = ld4(Le + (lp * kPX + l) * kPD);
            const float lv[kPD] = {ll.x, ll.y, ll.z, ll.w};
#pragma unroll
            for (int x = 0; x < kPD; ++x)
#pragma unroll
                for (int y = 0; y < kPD; ++y)
#pragma unroll
                    for (int z = 0; z < kPD; ++z) T1[x][y][z] = fmaf(lv[x], qv[y][z], T1[x][y][z]);
        }
    }
#pragma unroll
    for (int x = 0; x < kPD; ++x)
#pragma unroll
        for (int y = 0; y < kPD; ++y)
#pragma unroll
            for (int z = 0; z < kPD; ++z) T2[x][y][z] = 0.f;
    // FWD: T2[b'][a][m] = sum_{b,u} T1[b][b'][u] S1[b][u][a][m]
    // BWD: T2[b'][m][a] = sum_{a',q} S2[b'][m][a'][q] T1[q][a][a']
#pragma unroll
    for (int x = 0; x < kPD; ++x)
#pragma unroll
        for (int y = 0; y < kPD; ++y) {
            float sv[kPD][kPD];
            const float* sp = (FWD ? Sa : Sb) + (x * kPD + y) * 16;
#pragma unroll
            for (int r = 0; r < kPD; ++r) {
                const float4 t = ld4(sp + r * kPD);
                sv[r][0] = t.x; sv[r][1] = t.y; sv[r][2] = t.z; sv[r][3] = t.w;
            }
#pragma unroll
            for (int p = 0; p < kPD; ++p)
#pragma unroll
                for (int r = 0; r < kPD; ++r)
#pragma unroll
                    for (int s = 0; s < kPD; ++s) {
                        if (FWD) T2[p][r][s] = fmaf(T1[x][p][y], sv[r][s], T2[p][r][s]);
                        else T2[r][s][p] = fmaf(sv[r][s], T1[y][p][x], T2[r][s][p]);
                    }
        }
    // reuse T1 for the third temporary
    // FWD: T3[a][a'][q] = sum_{b',m} T2[b'][a][m] S2[b'][m][a'][q]
    // BWD: T3[b][u][b'] = sum_{a,m} S1[b][u][a][m] T2[b'][m][a]
#pragma unroll
    for (int x = 0; x < kPD; ++x)
#pragma unroll
        for (int y = 0; y < kPD; ++y)
#pragma unroll
            for (int z = 0; z < kPD; ++z) T1[x][y][z] = 0.f;
#pragma unroll
    for (int x = 0; x < kPD; ++x)
#pragma unroll
        for (int y = 0; y < kPD; ++y) {
            float sv[kPD][kPD];
            const float* sp = (FWD ? Sb : Sa) + (x * kPD + y) * 16;
#pragma unroll
            for (int r = 0; r < kPD; ++r) {
                const float4 t = ld4(sp + r * kPD);
                sv[r][0] = t.x; sv[r][1] = t.y; sv[r][2] = t.z; sv[r][3] = t.w;
            }
#pragma unroll
            for (int p = 0; p < kPD; ++p)
#pragma unroll
                for (int r = 0; r < kPD; ++r)
#pragma unroll
                    for (int s = 0; s < kPD; ++s) {
                        if (FWD) T1[p][r][s] = fmaf(T2[x][p][y], sv[r][s], T1[p][r][s]);
                        else T1[r][s][p] = fmaf(sv[r][s], T2[p][y][x], T1[r][s][p]);
                    }
        }
    __syncthreads();   // everyone is done with the incoming partial
    // ---- third temporary to LDS ----
    if (FWD) {
        // Big[l][c'][a][a'][q]
        float* dst = Big + (l * kPX + cp) * 64;
#pragma unroll
        for (int x = 0; x < kPD; ++x)
#pragma unroll
            for (int y = 0; y < kPD; ++y)
                *reinterpret_cast<float4*>(dst + (x * kPD + y) * kPD) =
                    make_float4(T1[x][y][0], T1[x][y][1], T1[x][y][2], T1[x][y][3]);
    } else {
        // Big[l][b][b'][u][c']
#pragma unroll
        for (int x = 0; x < kPD; ++x)
#pragma unroll
            for (int y = 0; y < kPD; ++y)
#pragma unroll
                for (int z = 0; z < kPD; ++z) Big[(((l * kPD + x) * kPD + z) * kPD + y) * kPX + cp] = T1[x][y][z];
    }
    __syncthreads();
    // ---- last contraction ----
    double* Y = a.Y + (long long)b * a.ys;
    float acc[kPX];
#pragma unroll
    for (int n = 0; n < kPX; ++n) acc[n] = 0.f;
    if (FWD) {
        // thread (c', a, a'): Pout[c'][a][a'][l'] = sum_{l,q} T3[l][c'][a][a'][q] L[l][q][l']
        const int c2 = tid >> 4, aa = (tid >> 2) & 3, ap = tid & 3;
        for (int l2 = 0; l2 < cl; ++l2) {
            const float4 t = ld4(Big + ((l2 * kPX + c2) * kPD + aa) * 16 + ap * kPD);
            const float tv[kPD] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int q = 0; q < kPD; ++q) {
                const float* lr = Le + (l2 * kPD + q) * kPX;
#pragma unroll
                for (int n4 = 0; n4 < kPX / 4; ++n4) {
                    const float4 lv = ld4(lr + n4 * 4);
                    acc[n4 * 4 + 0] = fmaf(tv[q], lv.x, acc[n4 * 4 + 0]);
                    acc[n4 * 4 + 1] = fmaf(tv[q], lv.y, acc[n4 * 4 + 1]);
                    acc[n4 * 4 + 2] = fmaf(tv[q], lv.z, acc[n4 * 4 + 2]);
                    acc[n4 * 4 + 3] = fmaf(tv[q], lv.w, acc[n4 * 4 + 3]);
                }
            }
        }
        if (c2 < cu1 && aa < h1 && ap < h1) {
            double* yo = Y + (((long long)c2 * h1 + aa) * h1 + ap) * cl1;
#pragma unroll
            for (int n = 0; n < kPX; ++n)
                if (n < cl1) yo[n] = (double)acc[n];
        }
    } else {
        // thread (b, b', l): Qout[c][b][b'][l] = sum_{u,c'} U[c][u][c'] T3[b][u][b'][l][c']
        const int bb = tid >> 6, bp = (tid >> 4) & 3, l2 = tid & 15;
#pragma unroll
        for (int u = 0; u < kPD; ++u) {
            const float* tr = Big + ((l2 * kPD + bb) * kPD + bp) * 64 + u * kPX;
            for (int c2 = 0; c2 < cu1; ++c2) {
                const float tv = tr[c2];
                const float* ur = Ue + (u * kPX + c2) * kPX;
#pragma unroll
                for (int n4 = 0; n4 < kPX / 4; ++n4) {
                    const float4 uv = ld4(ur + n4 * 4);
                    acc[n4 * 4 + 0] = fmaf(uv.x, tv, acc[n4 * 4 + 0]);
                    acc[n4 * 4 + 1] = fmaf(uv.y, tv, acc[n4 * 4 + 1]);
                    acc[n4 * 4 + 2] = fmaf(uv.z, tv, acc[n4 * 4 + 2]);
                    acc[n4 * 4 + 3] = fmaf(uv.w, tv, acc[n4 * 4 + 3]);
                }
            }
        }
        if (bb < h && bp < h && l2 < cl) {
            const long long m = ((long long)bb * h + bp) * cl + l2, ms = (long long)h * h * cl;
#pragma unroll
            for (int n = 0; n < kPX; ++n)
                if (n < cu) Y[(long long)n * ms + m] = (double)acc[n];
        }
    }
}

hipError_t launch_pair_step(const PairArgs& a, bool fwd, hipStream_t st) {
    if (a.batch <= 0) return hipSuccess;
    if (!pair_step_fits(a)) return hipErrorInvalidValue;
    const size_t bytes = kPairLds * sizeof(float);
    if (fwd) hipLaunchKernelGGL(k_pair_step<true>, dim3(a.batch), dim3(256), bytes, st, a);
    else hipLaunchKernelGGL(k_pair_step<false>, dim3(a.batch), dim3(256), bytes, st, a);
    return hipGetLastError();
}

}  // namespace peps
