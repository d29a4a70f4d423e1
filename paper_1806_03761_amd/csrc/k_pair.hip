// Fused two-row sandwich step in float32 (Sec. 3, Eq. (4): the two-row transfer that
// carries the partial contraction of rows i and i+1 between the boundary MPSs across
// one column).
//
// Unfused, the step is four batched GEMMs whose three temporaries (each Dc^2 D^3 per
// sample) make the round trip through HBM.  Here one workgroup owns one sample: the
// incoming partial and the two environment tensors are staged once into LDS, thread
// (l, c') (lower-left and upper-right boundary bonds, the indices that stay free through
// the first three contractions) keeps its D^3 slice of each temporary in registers, the
// spin-selected site tensors come from a zero-padded float32 table through the scalar
// cache (uniform operands, no LDS traffic), and the last contraction, which sums over l
// (forward) or c' (backward), goes through an LDS copy of the third temporary with each
// thread producing a 4 x 4 block of outputs.  Every product
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

bool pair_step_fits(const PairArgs& a) {
    const int legs[5] = {a.h, a.h1, a.Du, a.Dm, a.Dq};
    const int bonds[4] = {a.cu, a.cu1, a.cl, a.cl1};
    for (int v : legs)
        if (v < 1 || v > kPD) return false;
    for (int v : bonds)
        if (v < 1 || v > kPX) return false;
    return true;
}

// Site tensors of the whole lattice as float32, zero padded to 4 per leg, in the two
// leg orders the fused step reads: [left][up][right][down] and [right][down][left][up].
// T[((site * 2 + spin) * 2 + order) * 256 + index].
__global__ void k_site_tables(const double* A, float* T, int Lx, int Ly, int D) {
    const int s = blockIdx.x, tid = threadIdx.x;   // 256 threads: one padded entry each
    const int i = s / Lx, j = s % Lx;
    const int left = j == 0 ? 1 : D, right = j == Lx - 1 ? 1 : D;
    const int up = i == 0 ? 1 : D, down = i == Ly - 1 ? 1 : D;
    const long long D2 = (long long)D * D, D3 = D2 * D, D4 = D3 * D;
    const int x0 = tid >> 6, x1 = (tid >> 4) & 3, x2 = (tid >> 2) & 3, x3 = tid & 3;
    for (int sp = 0; sp < 2; ++sp) {
        const double* a = A + ((long long)s * 2 + sp) * D4;
        float* t = T + ((long long)s * 2 + sp) * 512;
        // natural order: (x0, x1, x2, x3) = (left, up, right, down)
        t[tid] = (float)ld_or0(x0 < left && x1 < up && x2 < right && x3 < down, a, x0 * D3 + x1 * D2 + x2 * D + x3);
        // second order: (x0, x1, x2, x3) = (right, down, left, up)
        t[256 + tid] = (float)ld_or0(x2 < left && x3 < up && x0 < right && x1 < down, a, x2 * D3 + x3 * D2 + x0 * D + x1);
    }
}

hipError_t launch_site_tables(const double* A, float* T, int Lx, int Ly, int D, hipStream_t st) {
    if (D > kPD) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_site_tables, dim3(Lx * Ly), dim3(256), 0, st, A, T, Lx, Ly, D);
    return hipGetLastError();
}

__device__ inline float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }

// Max-abs rescaling of the step's output, as the separate rescale kernel does it: the
// largest |entry| of the sample over the whole workgroup, entries multiplied by its
// reciprocal, its log added to the running log.  Returns the factor (1 when the max is
// 0 or not finite).
__device__ inline double step_rescale(double local_max, const double* lin, double* lout, int b,
                                      double* red) {
    double m = local_max;
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const bool ok = m > 0.0 && isfinite(m);
    if (threadIdx.x == 0) lout[b] = (lin ? lin[b] : 0.0) + (ok ? log(m) : 0.0);
    return ok ? 1.0 / m : 1.0;
}

// Fused single-row sandwich step (three GEMMs: environment, site, environment) in
// float32: thread (l, c') holds its D^2 slices of the two temporaries in registers,
// the last contraction goes through LDS, every sum keeps the order of its unfused GEMM.
//   FWD: P[c][b][l] -> Pout[c'][a][l'];  BWD: Q[c'][a][l'] -> Qout[c][b][l]
//   U[c][u][c'], L[l][d][l'], S[b][u][a][d] site (i,j) (left, up, right, down).
static constexpr int kRowLds = 3 * 1024 + 4096;   // floats

bool row_step_fits(const RowArgs& a) {
    const int legs[4] = {a.h, a.h1, a.Du, a.Dd};
    const int bonds[4] = {a.cu, a.cu1, a.cl, a.cl1};
    for (int v : legs)
        if (v < 1 || v > kPD) return false;
    for (int v : bonds)
        if (v < 1 || v > kPX) return false;
    return true;
}

template <bool FWD>
__global__ __launch_bounds__(256) void k_row_step(RowArgs a) {
    extern __shared__ __align__(16) float sm[];
    float* Xs = sm;              // incoming partial
    float* Ue = Xs + 1024;       // upper environment
    float* Le = Ue + 1024;       // lower environment
    float* Ts = Le + 1024;       // second temporary
    const int b = blockIdx.x, tid = threadIdx.x;
    if (b >= a.batch) return;
    if (a.skip && a.skip[(long long)b * a.skip_bs] == 0) return;
    const int cu = a.cu, cu1 = a.cu1, cl = a.cl, cl1 = a.cl1, Du = a.Du, Dd = a.Dd, h = a.h, h1 = a.h1;
    const double* X = a.X + (long long)b * a.xs;
    const double* U = a.U + (long long)b * a.us;
    const double* L = a.L + (long long)b * a.ls;
    const float* S = a.site + (long long)((a.sel[(long long)b * a.sel_bs] ^ a.flip) & 1) * 512 + (FWD ? 0 : 256);
#pragma unroll
    for (int it = 0; it < 4; ++it) {   // constant trip count: all loads issued together
        const int e = tid + 256 * it;
        if (FWD) {
            {   // Xs[c][l][b] = P[c][b][l]
                const int c = e >> 6, l = (e >> 2) & 15, bb = e & 3;
                Xs[e] = (float)ld_or0(c < cu && l < cl && bb < h, X, ((long long)c * h + bb) * cl + l);
            }
            {   // Ue[c][c'][u]
                const int c = e >> 6, cp = (e >> 2) & 15, u = e & 3;
                Ue[e] = (float)ld_or0(c < cu && cp < cu1 && u < Du, U, ((long long)c * Du + u) * cu1 + cp);
            }
            {   // Le[l][d][l']
                const int l = e >> 6, d = (e >> 4) & 3, lp = e & 15;
                Le[e] = (float)ld_or0(l < cl && d < Dd && lp < cl1, L, ((long long)l * Dd + d) * cl1 + lp);
            }
        } else {
            {   // Xs[l'][c'][a] = Q[c'][a][l']
                const int lp = e >> 6, cp = (e >> 2) & 15, aa = e & 3;
                Xs[e] = (float)ld_or0(lp < cl1 && cp < cu1 && aa < h1, X, ((long long)cp * h1 + aa) * cl1 + lp);
            }
            {   // Ue[u][c'][c]
                const int u = e >> 8, cp = (e >> 4) & 15, c = e & 15;
                Ue[e] = (float)ld_or0(c < cu && cp < cu1 && u < Du, U, ((long long)c * Du + u) * cu1 + cp);
            }
            {   // Le[l'][l][d]
                const int lp = e >> 6, l = (e >> 2) & 15, d = e & 3;
                Le[e] = (float)ld_or0(l < cl && d < Dd && lp < cl1, L, ((long long)l * Dd + d) * cl1 + lp);
            }
        }
    }
    __syncthreads();
    const int l = tid >> 4, cp = tid & 15;
    float T1[kPD][kPD], T2[kPD][kPD];
#pragma unroll
    for (int x = 0; x < kPD; ++x)
#pragma unroll
        for (int y = 0; y < kPD; ++y) T1[x][y] = T2[x][y] = 0.f;
    if (FWD) {
        // T1[b][u] = sum_c P[c][b][l] U[c][u][c']
        for (int c = 0; c < cu; ++c) {
            const float4 p4 = ld4(Xs + (c * kPX + l) * kPD), u4 = ld4(Ue + (c * kPX + cp) * kPD);
            const float pv[kPD] = {p4.x, p4.y, p4.z, p4.w}, uv[kPD] = {u4.x, u4.y, u4.z, u4.w};
#pragma unroll
            for (int x = 0; x < kPD; ++x)
#pragma unroll
                for (int y = 0; y < kPD; ++y) T1[x][y] = fmaf(pv[x], uv[y], T1[x][y]);
        }
        // T2[a][d] = sum_{b,u} T1[b][u] S[b][u][a][d]
#pragma unroll
        for (int x = 0; x < kPD; ++x)
#pragma unroll
            for (int y = 0; y < kPD; ++y) {
                const float* sp = S + (x * kPD + y) * 16;
#pragma unroll
                for (int r = 0; r < kPD; ++r)
#pragma unroll
                    for (int q = 0; q < kPD; ++q) T2[r][q] = fmaf(T1[x][y], sp[r * kPD + q], T2[r][q]);
            }
        // Ts[l][d][c'][a]
#pragma unroll
        for (int q = 0; q < kPD; ++q)
            *reinterpret_cast<float4*>(Ts + ((l * kPD + q) * kPX + cp) * kPD) = make_float4(T2[0][q], T2[1][q], T2[2][q], T2[3][q]);
    } else {
        // T1[d][a] = sum_l' L[l][d][l'] Q[c'][a][l']
        for (int lp = 0; lp < cl1; ++lp) {
            const float4 q4 = ld4(Xs + (lp * kPX + cp) * kPD), l4 = ld4(Le + (lp * kPX + l) * kPD);
            const float qv[kPD] = {q4.x, q4.y, q4.z, q4.w}, lv[kPD] = {l4.x, l4.y, l4.z, l4.w};
#pragma unroll
            for (int x = 0; x < kPD; ++x)
#pragma unroll
                for (int y = 0; y < kPD; ++y) T1[x][y] = fmaf(lv[x], qv[y], T1[x][y]);
        }
        // T2[b][u] = sum_{a,d} S[b][u][a][d] T1[d][a]   (S in the order [a][d][b][u])
#pragma unroll
        for (int x = 0; x < kPD; ++x)
#pragma unroll
            for (int y = 0; y < kPD; ++y) {
                const float* sp = S + (x * kPD + y) * 16;
#pragma unroll
                for (int r = 0; r < kPD; ++r)
#pragma unroll
                    for (int q = 0; q < kPD; ++q) T2[r][q] = fmaf(sp[r * kPD + q], T1[y][x], T2[r][q]);
            }
        // Ts[u][c'][l][b]
#pragma unroll
        for (int q = 0; q < kPD; ++q)
            *reinterpret_cast<float4*>(Ts + ((q * kPX + cp) * kPX + l) * kPD) = make_float4(T2[0][q], T2[1][q], T2[2][q], T2[3][q]);
    }
    __syncthreads();
    float acc[kPD] = {0.f, 0.f, 0.f, 0.f};
    double* Y = a.Y + (long long)b * a.ys;
    __shared__ double red[4];
    if (FWD) {
        // thread (c', a, l' group): Pout[c'][a][l'] = sum_{l,d} T2[l][c'][a][d] L[l][d][l']
        const int c2 = tid >> 4, aa = (tid >> 2) & 3, lg = tid & 3;
        for (int l2 = 0; l2 < cl; ++l2)
#pragma unroll
            for (int d = 0; d < kPD; ++d) {
                const float t = Ts[((l2 * kPD + d) * kPX + c2) * kPD + aa];
                const float4 w = ld4(Le + (l2 * kPD + d) * kPX + lg * kPD);
                acc[0] = fmaf(t, w.x, acc[0]);
                acc[1] = fmaf(t, w.y, acc[1]);
                acc[2] = fmaf(t, w.z, acc[2]);
                acc[3] = fmaf(t, w.w, acc[3]);
            }
        double scale = 1.0;
        if (a.lout) {
            double mx = 0.0;
#pragma unroll
            for (int y = 0; y < kPD; ++y) mx = fmax(mx, fabs((double)acc[y]));
            scale = step_rescale(mx, a.lin, a.lout, b, red);
        }
        // through LDS (padded [c'][a][l'] in the incoming-partial and environment tiles,
        // free now) so the global stores go out in output order
        __syncthreads();
        double* Ys = reinterpret_cast<double*>(sm);
#pragma unroll
        for (int y = 0; y < kPD; ++y) Ys[(c2 * kPD + aa) * kPX + lg * kPD + y] = (double)acc[y] * scale;
        __syncthreads();
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int e = tid + 256 * it, c = e >> 6, x = (e >> 4) & 3, lp = e & 15;
            if (c < cu1 && x < h1 && lp < cl1) Y[((long long)c * h1 + x) * cl1 + lp] = Ys[e];
        }
    } else {
        // thread (l, b, c group): Qout[c][b][l] = sum_{u,c'} U[c][u][c'] T2[b][u][l][c']
        const int l2 = tid >> 4, bb = (tid >> 2) & 3, cg = tid & 3;
#pragma unroll
        for (int u = 0; u < kPD; ++u)
            for (int c2 = 0; c2 < cu1; ++c2) {
                const float t = Ts[((u * kPX + c2) * kPX + l2) * kPD + bb];
                const float4 w = ld4(Ue + (u * kPX + c2) * kPX + cg * kPD);
                acc[0] = fmaf(w.x, t, acc[0]);
                acc[1] = fmaf(w.y, t, acc[1]);
                acc[2] = fmaf(w.z, t, acc[2]);
                acc[3] = fmaf(w.w, t, acc[3]);
            }
        double scale = 1.0;
        if (a.lout) {
            double mx = 0.0;
#pragma unroll
            for (int y = 0; y < kPD; ++y) mx = fmax(mx, fabs((double)acc[y]));
            scale = step_rescale(mx, a.lin, a.lout, b, red);
        }
        // through LDS (padded [c][b][l]) so the global stores go out in output order
        __syncthreads();
        double* Ys = reinterpret_cast<double*>(sm);
#pragma unroll
        for (int y = 0; y < kPD; ++y) Ys[((cg * kPD + y) * kPD + bb) * kPX + l2] = (double)acc[y] * scale;
        __syncthreads();
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int e = tid + 256 * it, c = e >> 6, x = (e >> 4) & 3, l = e & 15;
            if (c < cu && x < h && l < cl) Y[((long long)c * h + x) * cl + l] = Ys[e];
        }
    }
}

hipError_t launch_row_step(const RowArgs& a, bool fwd, hipStream_t st) {
    if (a.batch <= 0) return hipSuccess;
    if (!row_step_fits(a)) return hipErrorInvalidValue;
    const size_t bytes = kRowLds * sizeof(float);
    if (fwd) hipLaunchKernelGGL(k_row_step<true>, dim3(a.batch), dim3(256), bytes, st, a);
    else hipLaunchKernelGGL(k_row_step<false>, dim3(a.batch), dim3(256), bytes, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The fused two-row step on the matrix cores: the four contractions of the unfused
// chain (upper environment, two site tensors, lower environment) as 16x16x4 float32
// MFMA tiles.  A 16x16x4 MFMA accumulates its four products into
// each output in k order with one rounding per product, like a chain of fma, so a
// 16-long sum split over four MFMAs keeps ascending k order when MFMA s takes
// k = 4s .. 4s+3, i.e. lane (i, g) supplies k = 4s + g as element s of its operand.
// Sums longer than 16 chain the MFMAs block by block, and padding adds exact zeros, so
// every output is the unfused GEMM chain's value bit for bit.
//
// Work split (one sample per workgroup, four waves): a free bond is taken in chunks of
// four (c' forward, l backward: free through all four contractions), and inside a
// chunk wave w owns a second free index for the first three contractions (l in
// [4w, 4w+4) forward, c' = w mod 4 backward), so those three run wave-locally through
// the wave's own LDS tiles with no workgroup barrier.  Only the last contraction, which
// sums over that index, reads the whole third temporary (one barrier per chunk: the
// third temporary is double-buffered, and each wave's first and second temporaries
// share one tile, every operand of the second contraction read before its results
// overwrite them).  The
// first contraction's operand rows and the last one's B operand sit in registers for
// the whole kernel, loaded straight from the float64 inputs.
//
// Tile rows are chosen so each MFMA result (lane (li, g), register r = row 4g + r,
// column li) lands as four consecutive k entries of the next contraction: one 16-byte
// LDS store per lane.  LDS positions are XOR-swizzled (t12_at, t3_at) so that these
// stores and the 16-byte operand reads hit 16 distinct bank quads per 16 lanes.
// ---------------------------------------------------------------------------
typedef float mfma4_t __attribute__((ext_vector_type(4)));
// LDS (floats): per-wave T1/T2 tiles, then T3 -- single-buffered forward (32 KB: four
// workgroups per CU at the 128 registers the forward form fits in), double-buffered
// backward (48 KB, one barrier per chunk; it also holds the staged output block)
template <bool FWD>
constexpr int pair_mfma_lds() { return 4 * 1024 + (FWD ? 1 : 2) * 4096; }

__device__ __forceinline__ mfma4_t mfma_k16(const float4& av, const float4& bv, mfma4_t acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv.w, acc, 0, 0, 0);
    return acc;
}

// row R (of 64) of a 16-wide temporary, k quad q (k % 4 = q, k / 4 = offset in the quad)
__device__ __forceinline__ int t12_at(int R, int q) { return R * 16 + 4 * (q ^ ((R >> 4) & 3)); }
// row R of the 64-wide third temporary, k block kb, quad q
__device__ __forceinline__ int t3_at(int R, int kb, int q) {
    return R * 64 + 16 * (kb ^ (R & 3)) + 4 * (q ^ (((R >> 4) ^ (R >> 2)) & 3));
}
__device__ __forceinline__ void st4(float* p, const mfma4_t& v) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
// LDS written by other lanes of this wave becomes readable: no reordering across this
// point, and the wave's LDS stores complete first
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// B operand from a site table row (16 k entries in natural order): k = 4 s + g
__device__ __forceinline__ float4 site_b(const float* row, int g) {
    return make_float4(row[g], row[4 + g], row[8 + g], row[12 + g]);
}

template <bool FWD>
__global__ __launch_bounds__(256, FWD ? 4 : 3) void k_pair_mfma(PairArgs a) {
    extern __shared__ __align__(16) float sm[];
    const int b = blockIdx.x, tid = threadIdx.x;
    if (b >= a.batch) return;
    if (a.skip && a.skip[(long long)b * a.skip_bs] == 0) return;
    const int w = tid >> 6, li = tid & 15, g = (tid >> 4) & 3;
    float* T12 = sm + w * 1024;   // this wave's first, then second temporary, 64 rows x 16
    const int cu = a.cu, cu1 = a.cu1, cl = a.cl, cl1 = a.cl1;
    const int Du = a.Du, Dq = a.Dq, h = a.h, h1 = a.h1;
    const double* X = a.X + (long long)b * a.xs;
    const double* U = a.U + (long long)b * a.us;
    const double* L = a.L + (long long)b * a.ls;
    // site tables: FWD reads the second leg order ([right][down][left][up]), BWD the natural one
    const float* S1 = a.site1 + (long long)((a.sel1[(long long)b * a.sel_bs] ^ a.flip1) & 1) * 512 + (FWD ? 256 : 0);
    const float* S2 = a.site2 + (long long)((a.sel2[(long long)b * a.sel_bs] ^ a.flip2) & 1) * 512 + (FWD ? 256 : 0);

    // ---- operands held in registers (element s of lane (li, g) is k = 4 s + g) ----
    float4 xa[4];   // first contraction, A rows of tile tt
    float4 wb[4];   // last contraction, B operand of k block kb
    float4 ub[4];   // first contraction, B operand of chunk ch
    // offsets (element t * 4 + s of each group) with out-of-range entries sent to 0, then all
    // loads issued before any conversion so they overlap
    int ox[16], ow[16], ou[16];
    unsigned mx = 0, mw = 0, mu = 0;   // bit t * 4 + s: entry in range
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = 4 * s + g, e = t * 4 + s;
            bool okx, okw, oku;
            int fx, fw, fu;
            if (FWD) {
                // P[c = k][b = li & 3][b' = t][l = 4w + li / 4]
                const int bb = li & 3, l = 4 * w + (li >> 2);
                okx = k < cu && bb < h && t < h && l < cl;
                fx = (k * h * h + bb * h + t) * cl + l;
                // L[l = 4t + s][q = g][l' = li]
                okw = 4 * t + s < cl && g < Dq && li < cl1;
                fw = ((4 * t + s) * Dq + g) * cl1 + li;
                // U[c = k][u = li & 3][c' = 4t + li / 4]
                const int u = li & 3, cp = 4 * t + (li >> 2);
                oku = k < cu && u < Du && cp < cu1;
                fu = (k * Du + u) * cu1 + cp;
            } else {
                // Q[c' = 4t + w][a = li / 4][a' = li & 3][l' = k]
                const int cp = 4 * t + w, aa = li >> 2, ap = li & 3;
                okx = cp < cu1 && aa < h1 && ap < h1 && k < cl1;
                fx = ((cp * h1 + aa) * h1 + ap) * cl1 + k;
                // U[c = li][u = t][c' = k]
                okw = li < cu && t < Du && k < cu1;
                fw = (li * Du + t) * cu1 + k;
                // L[l = 4t + li / 4][q = li & 3][l' = k]
                const int l = 4 * t + (li >> 2), q = li & 3;
                oku = l < cl && q < Dq && k < cl1;
                fu = (l * Dq + q) * cl1 + k;
            }
            ox[e] = okx ? fx : 0; ow[e] = okw ? fw : 0; ou[e] = oku ? fu : 0;
            mx |= (unsigned)okx << e; mw |= (unsigned)okw << e; mu |= (unsigned)oku << e;
        }
    const double* Wsrc = FWD ? L : U;
    const double* Usrc = FWD ? U : L;
    {
        double rx[16], rw[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) rx[e] = X[ox[e]];
#pragma unroll
        for (int e = 0; e < 16; ++e) rw[e] = Wsrc[ow[e]];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float v[4], x[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                v[s] = (mx >> (t * 4 + s)) & 1 ? (float)rx[t * 4 + s] : 0.f;
                x[s] = (mw >> (t * 4 + s)) & 1 ? (float)rw[t * 4 + s] : 0.f;
            }
            xa[t] = make_float4(v[0], v[1], v[2], v[3]);
            wb[t] = make_float4(x[0], x[1], x[2], x[3]);
        }
    }
    {
        double ru[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) ru[e] = Usrc[ou[e]];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float y[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) y[s] = (mu >> (t * 4 + s)) & 1 ? (float)ru[t * 4 + s] : 0.f;
            ub[t] = make_float4(y[0], y[1], y[2], y[3]);
        }
    }
    const float4 s2b = site_b((FWD ? S1 : S2) + li * 16, g);
    const float4 s3b = site_b((FWD ? S2 : S1) + li * 16, g);

    const mfma4_t zero = {0.f, 0.f, 0.f, 0.f};
    mfma4_t out[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) out[t] = zero;
    const int nch = ((FWD ? cu1 : cl) + 3) >> 2;
    const int rread = 16 * (li & 3) + (li >> 2);   // operand row of a 16-wide temporary, tile 0
    for (int ch = 0; ch < nch; ++ch) {
        float* T3 = sm + 4096 + (FWD ? 0 : 4096 * (ch & 1));   // third temporary, 64 x 64, shared
        const float4 ubc = ch == 0 ? ub[0] : ch == 1 ? ub[1] : ch == 2 ? ub[2] : ub[3];
        wave_lds_sync();   // the previous chunk's reads of T12 are done
        // first contraction.  FWD: T1[(b',l,cc)][(b,u)] = sum_c P[c][b][b'][l] U[c][u][c'],
        // tile t = b', result row (b, l) = (r, 4w + g), column (cc, u).
        // BWD: T1[(a,c',l)][(a',q)] = sum_l' Q[c'][a][a'][l'] L[l][q][l'], tile t: c' = 4t + w,
        // result row (a', a) = (r, g), column (ll, q).
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const mfma4_t acc = mfma_k16(xa[t], ubc, zero);
            const int R = FWD ? 16 * t + 4 * g + (li >> 2) : 16 * g + 4 * t + (li >> 2);
            st4(T12 + t12_at(R, li & 3), acc);
        }
        wave_lds_sync();
        // second contraction, tile t (FWD: l = 4w + t, BWD: c' = 4t + w).
        // FWD: T2[(l,cc,a)][(b',m)] = sum_{(b,u)} T1 S1[b][u][a][m]; result row (b', cc) = (r, g).
        // BWD: T2[(c',l,b')][(a,m)] = sum_{(a',q)} T1 S2[b'][m][a'][q]; result row (a, ll) = (r, g).
        float4 av2[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) av2[t] = ld4(T12 + t12_at(rread + 4 * t, g));
        wave_lds_sync();   // all of T1 read before T2 overwrites it
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const mfma4_t acc = mfma_k16(av2[t], s2b, zero);
            st4(T12 + t12_at(16 * t + 4 * g + (li >> 2), li & 3), acc);
        }
        wave_lds_sync();
        if (FWD) __syncthreads();   // single buffer: the previous chunk's reads of T3 are done
        // third contraction, tile t (FWD: cc = t, BWD: ll = t).
        // FWD: T3[(cc,a,a')][(l,q)] = sum_{(b',m)} T2 S2[b'][m][a'][q]; result row (l, a) = (4w + r, g).
        // BWD: T3[(b,b',l)][(u,c')] = sum_{(a,m)} T2 S1[b][u][a][m]; result row (c', b') = (4r + w, g).
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float4 av = ld4(T12 + t12_at(rread + 4 * t, g));
            const mfma4_t acc = mfma_k16(av, s3b, zero);
            if (FWD) st4(T3 + t3_at(16 * t + 4 * g + (li >> 2), w, li & 3), acc);
            else st4(T3 + t3_at(16 * (li >> 2) + 4 * g + t, li & 3, w), acc);
        }
        // T3 complete; backward, its other buffer was last read before every wave passed the
        // previous chunk's barrier, so the next chunk may refill it
        __syncthreads();
        // last contraction, rows 16 w .. 16 w + 15 of T3, k blocks in order.
        // FWD: Pout[(cc,a,a')][l'] = sum_{(l,q)} T3 L[l][q][l'];  BWD: Qout[(b,b',l)][c] = sum_{(u,c')} T3 U[c][u][c']
        mfma4_t acc = zero;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = mfma_k16(ld4(T3 + t3_at(16 * w + li, kb, g)), wb[kb], acc);
        out[ch] = acc;
    }
    // ---- optional max-abs rescale, then the store ----
    double* Y = a.Y + (long long)b * a.ys;
    double scale = 1.0;
    if (a.lout) {
        double mx = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) mx = fmax(mx, fabs((double)out[t][r]));
        __shared__ double red[4];
        scale = step_rescale(mx, a.lin, a.lout, b, red);
    }
    // chunk t, output row 16 w + 4 g + r, column li
    if (FWD) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {   // row (cc, a, a') = (w, g, r), column l' = li
                const int cp = 4 * t + w;
                if (t < nch && cp < cu1 && g < h1 && r < h1 && li < cl1)
                    Y[(((long long)cp * h1 + g) * h1 + r) * cl1 + li] = (double)out[t][r] * scale;
            }
    } else {
        // row (b, b', l) = (w, g, 4t + r), column c = li: the lane index would be the slowest
        // output index, so the block goes through LDS (padded [c][b][b'][l], c stride 257
        // doubles: the 16 lanes of a store hit distinct banks) and leaves in output order
        __syncthreads();   // every wave is done with the tiles
        double* Ys = reinterpret_cast<double*>(sm);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (t < nch) Ys[li * 257 + (w * 4 + g) * 16 + 4 * t + r] = (double)out[t][r] * scale;
        __syncthreads();
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int e = tid + 256 * it, c = e >> 8, bb = (e >> 6) & 3, bp = (e >> 4) & 3, l = e & 15;
            if (c < cu && bb < h && bp < h && l < cl)
                Y[(((long long)c * h + bb) * h + bp) * cl + l] = Ys[c * 257 + (bb * 4 + bp) * 16 + l];
        }
    }
}

hipError_t launch_pair_step(const PairArgs& a, bool fwd, hipStream_t st) {
    if (a.batch <= 0) return hipSuccess;
    if (!pair_step_fits(a)) return hipErrorInvalidValue;
    const size_t mb = (fwd ? pair_mfma_lds<true>() : pair_mfma_lds<false>()) * sizeof(float);
    if (mb + 64 > get_lds_cap()) return hipErrorInvalidValue;
    if (fwd) hipLaunchKernelGGL(k_pair_mfma<true>, dim3(a.batch), dim3(256), mb, st, a);
    else hipLaunchKernelGGL(k_pair_mfma<false>, dim3(a.batch), dim3(256), mb, st, a);
    return hipGetLastError();
}

}  // namespace peps
