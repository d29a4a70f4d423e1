// Launchers of the library's HIP kernels (all enqueue on `st`, none synchronises).
#pragma once

#include "common.h"

namespace peps {

// tile: 0 = heuristic choice, 1..kMfmaTiles = a matrix-core tile shape (k_mgemm.hip), the two
// after them = the row kernel (k_gemm.hip) on the product or its transpose
static constexpr int kMfmaTiles = 35;
static constexpr int kGemmTiles = kMfmaTiles + 2;
// row kernel for skinny products: N <= 64 and K <= 64 (gemm_rows_fits); same results as
// launch_gemm
bool gemm_rows_fits(const GemmArgs& g);
hipError_t launch_gemm_rows(const GemmArgs& g, Arith ar, hipStream_t st);
hipError_t launch_gemm(const GemmArgs& g, Arith ar, hipStream_t st, int tile = 0);
// the same product with the roles of A and B (and of M and N) exchanged: C^T = B^T A^T
GemmArgs gemm_transposed(const GemmArgs& g);
// matrix-core GEMM (k_mgemm.hip): tile 1..kMfmaTiles, 0 = heuristic
hipError_t launch_mgemm(const GemmArgs& g, Arith ar, hipStream_t st, int tile = 0);
size_t get_lds_cap();

// column-group QR with TPC lanes per column group in WG-thread workgroups; false when the
// shape does not fit that configuration (nothing launched)
bool launch_qr_cols(double* X, long long xs, int m, int n, double* R, long long rs, double* tau,
                    long long ts, int batch, int tpc, int wg, hipStream_t st);
hipError_t launch_qr(double* X, long long xs, int m, int n, double* R, long long rs, double* tau,
                     long long ts, int batch, hipStream_t st);
size_t center0_scratch_doubles(int mz, int tin);
hipError_t launch_center0(const double* V, long long vs, const double* tau, long long ts,
                          const double* G, long long gs, int mz, int r, int tin, double* newU,
                          long long us, const double* logs_in, double* logs_out, double* scratch,
                          long long ss, int batch, hipStream_t st);

// truncation SVD through the Gram eigenproblem (three launches, see k_eig.hip)
struct EigLayout {
    int mp, np, gram_right, ns, tk, ldz, lda, ldx, nv;
    long long oZ, oA, oD, oE, oT, oX, oL, oP, oW, oM, oY, oV, oQ, nm, total, lds_prep, lds_fin;
};
struct EigArgs {
    const double* V; long long vs;
    const double* tau; long long ts;
    const double* G; long long gs;
    int mz, r, tin, p, Dc;
    double* newU; long long us;
    double* Gout; long long gos;
    double* scratch; long long ss;
    int batch;
    int z_ready;      // set by the launcher: Z = Q [G; 0] already in the scratch Z slot
    int gram_ready;   // set by the launcher: the Gram matrix already in the scratch Am slot
};
size_t eig_scratch_doubles(int mz, int tin, int p, int Dc);
// wyT != nullptr: the reflectors came from the blocked QR, whose WY blocks (wyT, stride wys
// per matrix) apply Q to [G; 0] on the matrix cores
hipError_t launch_eig(const double* V, long long vs, const double* tau, long long ts, const double* G,
                      long long gs, int mz, int r, int tin, int p, int Dc, double* newU, long long us,
                      double* Gout, long long gos, double* scratch, long long ss, int batch,
                      hipStream_t st, const double* wyT = nullptr, long long wys = 0);

// blocked Householder QR (k_qrb.hip) for matrices beyond the register kernels: panels of
// qrb_panel_width(m) columns factorised in registers, trailing updates in compact WY form
// on the matrix cores.  Same reflector convention and outputs as launch_qr, plus the WY
// T blocks (qrb_wy_doubles(m, n) doubles per matrix, stride tws).
int qrb_panel_width(int m);
long long qrb_wy_doubles(int m, int n);
bool qrb_fits(int m, int n);
long long qrb_vc_doubles(int m);
long long qrb_wq_doubles(int n);
// Vc (qrb_vc_doubles(m) per matrix) and Wq (qrb_wq_doubles(n)) hold the 32-reflector updates
// (trailing columns updated by two GEMMs per pair of panels); Vc == nullptr: 16-column
// WY updates only
hipError_t launch_qr_blocked(double* X, long long xs, int m, int n, double* R, long long rs, double* tau,
                             long long ts, double* Tw, long long tws, double* Vc, long long vcs, double* Wq,
                             long long wqs, int batch, hipStream_t st);
// Z (column-major, ld ldz, stride zs per matrix) = Q [G; 0], Q from launch_qr_blocked
// Wq: 64 tin doubles per matrix (stride wqs) for the GEMM form (16-column panels)
hipError_t launch_applyq_blocked(const double* V, long long vs, int mz, int nrefl, const double* Tw,
                                 long long tws, const double* G, long long gs, int rin, int tin, double* Z,
                                 long long zs, int ldz, double* Wq, long long wqs, int batch, hipStream_t st);

// variational compression (k_vc.hip)
// thin QR of m x n matrices (m >= n, n <= 128, column-major, one per sample) into the
// sign-fixed Q (element (i, k) at Q + b qs + i q_row + k q_col) and, when R != nullptr,
// the n x n factor (row-major); X may equal Q.  Matrices up to 512 x 64 are held in
// registers, larger ones in LDS where they fit (thinq_fits), the rest in W (m n doubles
// per sample, stride ws; thinq_needs_scratch).
bool thinq_shape_ok(int m, int n);
bool thinq_fits(int m, int n);
bool thinq_needs_scratch(int m, int n);   // W is read only for these shapes
hipError_t launch_thinq(const double* X, long long xs, int m, int n, double* Q, long long qs, long long q_row,
                        long long q_col, double* R, long long rs, double* W, long long ws, int batch,
                        hipStream_t st);
// x /= ||x||, lout = lin + ln ||x|| (lout = -inf for a zero x)
hipError_t launch_vc_norm(double* x, long long xs, int n, const double* lin, double* lout, int batch,
                          hipStream_t st);

// misc
// fused two-row sandwich step (float32, legs <= 4, boundary bonds <= 16; see k_pair.hip)
struct PairArgs {
    int cu, cu1, cl, cl1, Du, Dm, Dq, h, h1;
    const double* X; long long xs;       // incoming partial (P forward, Q backward)
    const double* U; long long us;       // upper environment [cu][Du][cu1]
    const double* L; long long ls;       // lower environment [cl][Dq][cl1]
    const float* site1;                  // site tables (launch_site_tables) of (i, j)
    const float* site2;                  // and (i+1, j)
    const int8_t* sel1; const int8_t* sel2; long long sel_bs; int flip1, flip2;
    double* Y; long long ys;             // outgoing partial
    const double* lin; double* lout;     // lout != nullptr: max-abs rescale, log into lout
    int batch;
    const int8_t* skip = nullptr;        // sample b skipped when skip[b * skip_bs] == 0
    long long skip_bs = 0;
};
bool pair_step_fits(const PairArgs& a);
// fused single-row sandwich step (float32, legs <= 4, boundary bonds <= 16)
struct RowArgs {
    int cu, cu1, cl, cl1, Du, Dd, h, h1;
    const double* X; long long xs;       // incoming partial (P forward, Q backward)
    const double* U; long long us;       // upper environment [cu][Du][cu1]
    const double* L; long long ls;       // lower environment [cl][Dd][cl1]
    const float* site;                   // site table of (i, j)
    const int8_t* sel; long long sel_bs; int flip;
    double* Y; long long ys;
    const double* lin; double* lout;     // lout != nullptr: max-abs rescale, log into lout
    int batch;
    const int8_t* skip = nullptr;        // sample b skipped when skip[b * skip_bs] == 0
    long long skip_bs = 0;
};
bool row_step_fits(const RowArgs& a);
hipError_t launch_row_step(const RowArgs& a, bool fwd, hipStream_t st);
// float32 site tables of the fused step: 512 floats per (site, spin), see k_pair.hip
hipError_t launch_site_tables(const double* A, float* T, int Lx, int Ly, int D, hipStream_t st);
hipError_t launch_pair_step(const PairArgs& a, bool fwd, hipStream_t st);
hipError_t launch_fill(double* x, long long n, double v, hipStream_t st);
hipError_t launch_fill_i8(int8_t* x, long long n, int8_t v, hipStream_t st);
hipError_t launch_copy_i8(const int8_t* src, int8_t* dst, long long n, hipStream_t st);
hipError_t launch_check_configs(const int8_t* S, int N, int batch, int8_t* flags, hipStream_t st);
hipError_t launch_rescale(double* x, long long xs, int n, const double* lin, double* lout,
                          int batch, hipStream_t st);
hipError_t launch_ratio(const double* F, long long fs, const double* G, long long gs, int n,
                        const double* la, const double* lb, const double* lnW, const double* sgW,
                        double* ratio, int nbonds, int bond, int batch, hipStream_t st,
                        const int8_t* skip = nullptr);
// act[b][bond] = 1 where the two spins of the bond differ (bond order of launch_eloc)
hipError_t launch_bond_active(const int8_t* S, int Lx, int Ly, int8_t* act, int nbonds, int batch,
                              hipStream_t st);
hipError_t launch_sandwich_value(const double* P, long long ps, const double* lam, double* lnW,
                                 double* sgW, int batch, hipStream_t st);
struct ElocArgs {
    const int8_t* S; int Lx, Ly;
    double J1, J2;
    const double* ratio; int nbonds;
    const int8_t* flags;
    double* e_loc;
    int batch;
};
hipError_t launch_eloc(const ElocArgs& a, hipStream_t st);
hipError_t launch_amp_out(const double* logU, const double* lnW, const double* sgW,
                          int8_t* flags, double* log_abs, int8_t* sign, int batch, hipStream_t st);
// Delta = B / <B, T> on the live block of site `site`, in place.
hipError_t launch_grad_site(double* Dsite, long long bs, const double* A, const int8_t* S, int site,
                            int N, int D, int Dl, int Du, int Dr, int Dd, int batch, hipStream_t st);
// per-sample output out[b][m][s][D^4] (both slices written) from Delta[b][m][D^4]
hipError_t launch_grad_store(const double* Dall, const int8_t* S, int N, int D4, const int8_t* flags,
                             double* out, int batch, hipStream_t st);
// out1[m][s][e] (+)= sum_b w_b [S_b[m] = s] Delta_b[m][e] (w null: ones) and, when out0 is
// not null, out0 the same sum with unit weights.  Flagged samples are skipped.  ws holds
// 2 * grad_parts(batch) * 2 N D4 doubles.
static constexpr int kGradParts = 64;
int grad_parts(int batch);
hipError_t launch_grad_reduce(const double* Dall, const int8_t* S, int N, int D4, const int8_t* flags,
                              const double* w, int accumulate, double* out1, double* out0, double* ws,
                              int batch, hipStream_t st);
// Metropolis step (see k_misc.hip): proposal and acceptance kernels, one thread per sample
// Metropolis proposals of the moved chains packed in chain order (moved, pos per chain;
// the number of moved chains is returned in *hcount, which synchronises the stream).
hipError_t launch_mc_propose(const int8_t* S, const double* u, int Lx, int Ly, int batch, int8_t* moved, int* pos,
                             int* count, int8_t* Sp, int* hcount, hipStream_t st);
hipError_t launch_mc_accept(int8_t* S, const int8_t* Sp, const int8_t* moved, const int* pos, const double* u,
                            const double* lap, const int8_t* sgp, const int8_t* flp, double* log_abs,
                            int8_t* sign, int8_t* accepted, int N, int batch, hipStream_t st);
hipError_t launch_energy_mean(const double* acc, double* out, hipStream_t st);
hipError_t launch_go_update(double* A, const double* grad, const double* p, double dt, long long n,
                            hipStream_t st);
hipError_t launch_corr_pack(const int8_t* S, const int* pairs, int P, int N, int batch, int8_t* Sx, int* slot,
                            int* count, hipStream_t st);
hipError_t launch_corr_values(const int8_t* S, const int* pairs, int P, int N, int batch, const double* la,
                              const int8_t* sg, const int8_t* fl, const int* slot, const double* lax,
                              const int8_t* sgx, const int8_t* flx, double* v, int8_t* flags, hipStream_t st);
hipError_t launch_corr_means(const double* v, const int8_t* flags, int P, int batch, double* means,
                             hipStream_t st);
hipError_t launch_structure_factor(int Lx, int nb, const int* sites, const double* C, int nk, const double* kv,
                                   double* out, hipStream_t st);
hipError_t launch_energy_sums(const double* e_loc, const int8_t* flags, int batch, double* acc,
                              int accumulate, hipStream_t st);
hipError_t launch_energy_grad_combine(const double* G1, const double* G0, const double* acc,
                                      long long n, double* out, hipStream_t st);
hipError_t launch_nan_flagged(const int8_t* flags, double* log_abs, int8_t* sign, double* e_loc,
                              int batch, hipStream_t st);

}  // namespace peps
