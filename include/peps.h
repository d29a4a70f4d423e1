/*
 * peps.h - C ABI of the MI355X (gfx950) PEPS variational Monte Carlo hot path.
 *
 * For a batch of spin configurations S of an open Lx x Ly spin-1/2 lattice and
 * a PEPS with bond dimension D (physical dimension d = 2), the library computes
 *   - ln|W(S)| and sign W(S), the single-layer contraction of the PEPS at fixed
 *     S (Eq. (1) of the paper, the W(S) of Sec. II-A), approximated by the
 *     row-by-row boundary-MPS contraction with bond truncation Dc (Fig. 1(c));
 *   - the local energy E(S) of Eq. (4) for the J1-J2 Heisenberg model of
 *     Sec. III-A (Eq. (9)), from cached upper and lower environments;
 *   - the log-derivatives Delta = B/W of Eqs. (6)-(7), per sample or contracted
 *     with per-sample weights (the Monte Carlo gradient of Eq. (5));
 *   - around that path: a Metropolis step of many Markov chains sampling W(S)^2
 *     (Sec. II-B, steps 1-3), the gradient-optimisation update of the tensors and one
 *     iteration of the optimisation loop (Sec. II-A, II-B), and the spin-spin
 *     correlations and structure factor of Sec. III-A.
 *
 * Conventions shared by every entry point
 *   A      device, float64, [Ly*Lx][2][D][D][D][D] = [site][phys][l][u][r][d],
 *          C order, site m = i*Lx + j (row i from the top, column j from the
 *          left).  Legs that point out of the open lattice (l at j = 0, u at
 *          i = 0, r at j = Lx-1, d at i = Ly-1) are read at index 0 only; the
 *          other entries of those legs are never read.  Read-only, except for
 *          peps_go_update and peps_vmc_step, which update it in place.
 *   S      device, int8, [batch][Ly*Lx], values {0, 1}; 0 = spin up (S^z=+1/2).
 *          Read-only, except for the chains of peps_metropolis_step and
 *          peps_vmc_step, which move in place.
 *   batch  number of configurations (>= 0; 0 is a no-op that returns PEPS_OK).
 *   flags  optional device int8 [batch] (may be NULL): 0 ok, 1 configuration
 *          value outside {0,1}, 2 zero amplitude, 3 non-finite result.
 *          A flagged sample never aborts the batch: its outputs are NaN
 *          (flag 1, 3) or sign 0 / ln|W| = -inf / E = NaN / Delta = 0 (flag 2).
 *   prec   arithmetic of the contraction GEMMs.  PEPS_PREC_F64: all in float64.
 *          PEPS_PREC_F32: operands rounded to float32, float32 accumulation.
 *          PEPS_PREC_BF16: the MPO x MPS apply GEMMs of the boundary sweeps take
 *          bfloat16 operands with float32 accumulation; the sandwich and
 *          environment-tensor GEMMs run in float32.  QR, SVD, normalisation,
 *          ln|W|, sign and the energy assembly are always float64.
 *   Every buffer is owned by the caller; outputs are written asynchronously on
 *   the context's stream and are valid after that stream is synchronised.
 *   Host-detectable errors (NULL pointers, Lx < 2 or Ly < 2, D < 1, Dc < 1,
 *   batch < 0, unsupported sizes) return before anything is enqueued.
 *   A context must not be used by two host threads at once.
 */
#ifndef PEPS_H
#define PEPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PEPS_OK = 0,
    PEPS_ERR_INVALID_ARG = 1,
    PEPS_ERR_OOM = 2,
    PEPS_ERR_HIP = 3,
    PEPS_ERR_UNSUPPORTED = 4,
    PEPS_ERR_NUMERICAL = 5
} peps_status;

typedef enum { PEPS_PREC_F64 = 0, PEPS_PREC_F32 = 1, PEPS_PREC_BF16 = 2 } peps_precision;

/* Lattice Lx x Ly (open boundaries), bond dimension D, boundary-MPS truncation Dc,
 * couplings of H = J1 sum_<ij> S_i.S_j + J2 sum_<<ij>> S_i.S_j (Sec. III-A). */
typedef struct {
    int32_t Lx, Ly, D, Dc;
    double J1, J2;
} peps_lattice;

typedef struct peps_ctx peps_ctx;

/* Create a context on HIP device `device`.  It owns a lazily grown workspace and
 * the tuned launch parameters.  Returns PEPS_ERR_HIP if the device is unusable. */
peps_status peps_create(peps_ctx** ctx, int device);

/* Free the context and its workspace.  NULL is accepted. */
peps_status peps_destroy(peps_ctx* ctx);

/* Stream on which all later work is enqueued (a hipStream_t; NULL = default stream). */
peps_status peps_set_stream(peps_ctx* ctx, void* hip_stream);

/* Boundary truncation of every contraction on this context (Sec. II-A: the bond of a
 * boundary MPS is cut to Dc after each row is applied).  sweeps = 0 (default): the
 * canonical SVD truncation.  sweeps = 1..16: variational compression wherever the
 * incoming boundary already has the bond and physical dims of the outgoing one (the
 * bond has stopped growing; the SVD truncation still fixes the dims before that):
 * the outgoing boundary is fitted to the applied row by one-site alternating least
 * squares started from the incoming boundary, `sweeps` left-to-right plus
 * right-to-left passes, every factor sign-fixed (non-negative diagonal of R), the norm
 * kept as a log.  Its contractions are float64 batched GEMMs of O(D^4 Dc^2) per site
 * and pass, whatever the precision argument of a call; the result is a different
 * approximation of W than the SVD truncation's.  Site factorisations (Dc D x Dc) run in
 * LDS where they fit and from workspace memory otherwise; evaluations fail with
 * PEPS_ERR_UNSUPPORTED when a bond of a variational step exceeds 128.
 * PEPS_ERR_INVALID_ARG for sweeps outside [0, 16]. */
peps_status peps_set_truncation(peps_ctx* ctx, int32_t sweeps);

/* Fused float32 sandwich steps (enable != 0, the default): the single- and two-row steps
 * of the float32 and bfloat16 modes with legs <= 4 and boundary bonds <= 16 run as one
 * kernel each, summing every product in the order of the GEMM form, so their results
 * equal the GEMM form's bit for bit.  enable = 0 keeps the GEMM form (a comparison
 * switch; slower). */
peps_status peps_set_fused_steps(peps_ctx* ctx, int32_t enable);

/* Cap the device workspace in bytes (0 = default: 1/4 of free device memory at
 * first use).  Larger batches are processed in chunks that fit; a single sample
 * that does not fit returns PEPS_ERR_OOM. */
peps_status peps_set_workspace_limit(peps_ctx* ctx, size_t bytes);

/* Device bytes the context would use for one chunk of `batch` samples. */
peps_status peps_workspace_query(peps_ctx* ctx, const peps_lattice* lat, int64_t batch,
                                 peps_precision prec, size_t* bytes);

/* Message of the last failing call on this context ("" if none); valid until the
 * next call on the context. */
const char* peps_last_error(const peps_ctx* ctx);

/* ln|W(S)| and sign W(S) (top-down boundary-MPS contraction, then the overlap
 * with the last row).  log_abs: device float64 [batch]; sign: device int8 [batch]. */
peps_status peps_log_amplitude(peps_ctx* ctx, const peps_lattice* lat, peps_precision prec,
                               const double* A, const int8_t* S, int64_t batch,
                               double* log_abs, int8_t* sign, int8_t* flags);

/* Local energy of Eq. (4): E(S) = sum_bonds J [sigma sigma'/4 + 1/2 [s != s'] W(S')/W(S)],
 * with W(S')/W(S) from the single-row sandwich <U_i|row i|L_i> (horizontal bonds) or
 * the two-row sandwich <U_i|rows i,i+1|L_{i+1}> (vertical and diagonal bonds).
 * e_loc: device float64 [batch], total energy of the sample.  log_abs, sign as above. */
peps_status peps_local_energy(peps_ctx* ctx, const peps_lattice* lat, peps_precision prec,
                              const double* A, const int8_t* S, int64_t batch,
                              double* log_abs, int8_t* sign, double* e_loc, int8_t* flags);

/* Log-derivatives of Eqs. (6)-(7), Delta_m = (1/W_i) dW_i/dA_m with the row-i
 * environments held fixed (row i holds site m).
 * weights == NULL: out is device float64 [batch][Ly*Lx][2][D^4], per sample; only the
 *                  slice s = S[b][m] and live leg entries are non-zero.
 * weights != NULL (device float64 [batch]): out is [Ly*Lx][2][D^4] =
 *                  sum_b weights[b] * Delta_b, summed in sample order (overwritten). */
peps_status peps_log_derivative(peps_ctx* ctx, const peps_lattice* lat, peps_precision prec,
                                const double* A, const int8_t* S, int64_t batch,
                                const double* weights, double* out, double* log_abs,
                                int8_t* sign, int8_t* flags);

/* One pass of the whole path from one set of environments.  Any output may be NULL.
 * grad_mode: 0 = no gradient; 1 = per-sample Delta into `out` ([batch][N][2][D^4]);
 *            2 = out = sum_b weights[b] Delta_b ([N][2][D^4]);
 *            3 = out = dE/dA of Eq. (5) = sum_b (2/B)(E_b - mean E) Delta_b over the
 *                samples with flag 0 (B = their count); needs e_loc. */
peps_status peps_evaluate(peps_ctx* ctx, const peps_lattice* lat, peps_precision prec,
                          const double* A, const int8_t* S, int64_t batch, int32_t grad_mode,
                          const double* weights, double* log_abs, int8_t* sign,
                          double* e_loc, double* out, int8_t* flags);

/* peps_evaluate for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same arguments,
 * kernels and results (per-sample outputs bit for bit; the grad_mode 2 and 3 sums may
 * differ by rounding, as they are summed over the chunks below), with the workspace in a
 * fixed device array of peps_noalloc_scratch_bytes() bytes (64 MiB) that each device
 * holds from library load to process end, instead of the context's allocated workspace.
 * The batch is processed in chunks sized to that array; a lattice whose single sample
 * does not fit returns PEPS_ERR_INVALID_ARG with a message, before any work.
 * The call allocates no device memory (no hipMalloc or hipFree, no library routine that
 * does) and records no profiling events.  Every context and call on one device shares
 * that device's array, which keeps the last call's contents (nothing in it is assumed
 * to be zero on entry): calls whose work overlaps on one device (several streams or
 * contexts) race and must be serialised by the caller.  The caller passes inputs and
 * outputs as for peps_evaluate. */
peps_status peps_evaluate_noalloc(peps_ctx* ctx, const peps_lattice* lat, peps_precision prec,
                                  const double* A, const int8_t* S, int64_t batch,
                                  int32_t grad_mode, const double* weights, double* log_abs,
                                  int8_t* sign, double* e_loc, double* out, int8_t* flags);

/* Size in bytes of the fixed scratch array of peps_evaluate_noalloc. */
size_t peps_noalloc_scratch_bytes(void);

/* One Metropolis step of every chain: the sampling loop of Sec. II-B (steps 1-3: a
 * proposed configuration, its weight by contraction, accept or reject) for weights
 * W(S)^2, the importance sampling of the energy estimator Eq. (3).
 * Chain b draws bond k = min(floor(u[b][0] * nb), nb - 1) of the nb J1 and J2 bonds,
 * ordered: horizontal (i,j)-(i,j+1) row by row, vertical (i,j)-(i+1,j), diagonal
 * (i,j)-(i+1,j+1), anti-diagonal (i,j+1)-(i+1,j).  If its two spins differ, S' is S with
 * them exchanged (S^z is kept; the same bond undoes it), ln|W(S')| is contracted as in
 * peps_log_amplitude, and S' replaces S when it has flag 0 and
 * u[b][1] < exp(2 (ln|W(S')| - log_abs[b])).
 * S: device int8 [batch][Ly*Lx], the chains, updated in place.
 * log_abs, sign: device [batch], ln|W(S)| and sign of the chains on entry (as from
 *   peps_log_amplitude), updated with the moves.
 * u: device float64 [batch][2], uniform in [0, 1), drawn by the caller.
 * accepted: device int8 [batch] or NULL; 1 where the chain moved, else 0.
 * Only the chains whose bond holds two different spins are contracted; their number is
 * read back to the host to size that contraction, so the call synchronises the
 * context's stream once.  The context keeps its sampling buffers (about
 * batch * (N + 35) bytes) between calls. */
peps_status peps_metropolis_step(peps_ctx* ctx, const peps_lattice* lat, peps_precision prec,
                                 const double* A, int8_t* S, int64_t batch, const double* u,
                                 double* log_abs, int8_t* sign, int8_t* accepted);

/* Gradient-optimisation update of the tensors (Sec. II-A): every element moves against
 * the sign of its energy derivative, A[i] -= p[i] * dt * sign(grad[i]), with p[i] in
 * (0, 1) drawn per element by the caller and dt the step length of this iteration.  A
 * zero or NaN derivative leaves the element unchanged.
 * A: device float64 [Ly*Lx][2][D^4] (the layout of every entry point), updated in place.
 * grad, p: device float64, same layout.  dt must be finite.
 * Enqueued on the context's stream; no allocation. */
peps_status peps_go_update(peps_ctx* ctx, const peps_lattice* lat, double* A, const double* grad,
                           const double* p, double dt);

/* One iteration of the optimisation loop (Sec. II-B, Step B; Step B-a then B-b):
 *   1. ln|W| of the chains S under A (as peps_log_amplitude);
 *   2. n_mc Metropolis steps of every chain (as peps_metropolis_step, step t taking the
 *      uniforms u + 2*batch*t);
 *   3. the sampled energy (Eq. (3)) and dE/dA (Eq. (5)) over the chains' configurations,
 *      samples with a non-zero flag left out (as peps_evaluate with grad_mode 3);
 *   4. the GO update of A with p and dt (as peps_go_update).
 * A: device float64 [Ly*Lx][2][D^4], updated in place.  S: device int8 [batch][Ly*Lx],
 * the chains, updated in place.  u: device float64 [n_mc][batch][2] uniforms in [0, 1)
 * (may be NULL when n_mc is 0).  p: device float64 [Ly*Lx][2][D^4] in (0, 1).
 * energy: device float64 [2] or NULL: {sampled E, number of samples with flag 0} (E is
 * NaN when there is none).  grad: device float64 [Ly*Lx][2][D^4] or NULL: dE/dA before the
 * update (the context keeps its own copy when NULL).
 * batch must be at least 1.  Work is enqueued on the context's stream, which each
 * Metropolis step synchronises once (see peps_metropolis_step); the context keeps
 * its sampling buffers (about batch * (N + 35) bytes, plus the gradient when grad is
 * NULL) between calls. */
peps_status peps_vmc_step(peps_ctx* ctx, const peps_lattice* lat, peps_precision prec, double* A,
                          int8_t* S, int64_t batch, int32_t n_mc, const double* u, const double* p,
                          double dt, double* energy, double* grad);

/* Spin-spin correlations <S_m . S_n> by Monte Carlo (Sec. III-A): for every sample and
 * pair, the local value sigma_m sigma_n / 4 plus, where the two spins differ, half the
 * ratio W(S')/W(S) of the configuration with them exchanged (both contracted in full, as
 * in peps_log_amplitude); 3/4 when m == n.  A zero W(S') gives a zero ratio; a sample
 * whose W(S), or any of whose W(S'), has another non-zero flag is left out (flag 3 for
 * an exchanged configuration that is not finite).
 * pairs: device int32 [npairs][2] site indices in [0, Ly*Lx) (checked; read back to the
 *   host, which synchronises the context's stream).
 * means: device float64 [npairs] or NULL: mean over the samples with flag 0 (NaN when
 *   there is none).  per_sample: device float64 [batch][npairs] or NULL (NaN where the
 *   sample is left out).  flags: device int8 [batch] or NULL.
 * batch * npairs must be at most 2^30.  The context keeps a buffer of about
 * batch * npairs * (N + 22) bytes between calls. */
peps_status peps_pair_correlations(peps_ctx* ctx, const peps_lattice* lat, peps_precision prec,
                                   const double* A, const int8_t* S, int64_t batch, int32_t npairs,
                                   const int32_t* pairs, double* means, double* per_sample,
                                   int8_t* flags);

/* Structure factor of Sec. III-A over a block of nsites sites:
 * out[q] = (1/nsites^2) sum_{i,j} corr[i][j] cos(k_q . (r_i - r_j)), r = (column, row) of
 * the site, which is the real part of the Fourier sum for a real correlation matrix
 * (M^2 = out at k = (pi, pi) with the central (L-4) x (L-4) block).
 * sites: device int32 [nsites] (checked; read back to the host).  corr: device float64
 * [nsites][nsites], <S_i . S_j> of those sites.  k: device float64 [nk][2].  out: device
 * float64 [nk]. */
peps_status peps_structure_factor(peps_ctx* ctx, const peps_lattice* lat, int32_t nsites,
                                  const int32_t* sites, const double* corr, int32_t nk,
                                  const double* k, double* out);

/* One job of a heterogeneous batch (peps_eval_jobs): a lattice with its own tensors,
 * configurations and outputs, with the meanings of peps_evaluate.  A NULL e_loc skips
 * the local energy (unless grad_mode is 3). */
typedef struct {
    peps_lattice lat;
    const double* A;
    const int8_t* S;
    int64_t batch;
    int32_t grad_mode;
    const double* weights;
    double* log_abs;
    int8_t* sign;
    double* e_loc;
    double* out;
    int8_t* flags;
} peps_job;

enum { PEPS_JOBS_GRAPH = 1 };

/* Evaluate several lattices (sizes, D, Dc may differ) in one call, for example the
 * mixed batches of a Monte Carlo run over several lattices.  Every job gets its own
 * workspace region, so the whole batch of each job must fit the workspace limit
 * together (PEPS_ERR_OOM otherwise).  With PEPS_JOBS_GRAPH the launch sequence of all
 * jobs is captured once into a HIP graph, one branch per job, and launched as a single
 * graph on the context stream; a later call with the same job list (same pointers,
 * sizes and precision) replays the cached graph.  Results equal those of separate
 * peps_evaluate calls.  At most 64 jobs. */
peps_status peps_eval_jobs(peps_ctx* ctx, const peps_job* jobs, int32_t njobs,
                           peps_precision prec, uint32_t flags);

/* Autotuner of the contraction GEMM tiles.  Runs one evaluation (local energy and the
 * Eq. (5) gradient) of the given lattice and batch; every GEMM shape not yet in the
 * context's table is launched once with each candidate tile shape, timed with HIP events
 * (this synchronises), and the fastest tile is recorded.  All tiles accumulate in the
 * same order, so results do not depend on the choice.  Later calls on the context use
 * the table.  *tuned (may be NULL) receives the number of shapes added.  If the
 * environment variable PEPS_TUNE_CACHE names a file, peps_create loads it and
 * peps_autotune saves the table there. */
peps_status peps_autotune(peps_ctx* ctx, const peps_lattice* lat, peps_precision prec,
                          const double* A, const int8_t* S, int64_t batch, int32_t* tuned);

/* Save / load the tile table as text lines "M,N,K,batch,arith,f32mask tile" (f32mask: bit 0/1/2
   set when operand A/B/C is a float32 temporary).  Loading adds or replaces entries; tile 0
   selects the built-in heuristic for that shape, and numbers past the last tile are ignored. */
peps_status peps_tune_save(peps_ctx* ctx, const char* path);
peps_status peps_tune_load(peps_ctx* ctx, const char* path);

/* Kernel classes for the profiling calls below. */
enum { PEPS_KC_GEMM = 0, PEPS_KC_QR = 1, PEPS_KC_SVD = 2, PEPS_KC_FUSED = 3 };

/* Start timing the launches of the kernel classes in `class_mask` (bit 1 << PEPS_KC_*):
 * each such launch is bracketed by two HIP events on the context's stream, together
 * with its algorithmic flop count (GEMM 2MNK; fused single-/two-row sandwich step: the
 * 2MNK of the three / four GEMMs it replaces; QR 2 r^2 (max(m,n) - r/3), and for the
 * thin QR of the variational compression 4 m n^2 - 4 n^3 / 3 (factor and explicit Q);
 * truncation step: implicit-Q apply 4 t (mz r - r^2/2) plus a thin SVD
 * min(14 a b^2 + 8 b^3, 6 a b^2 + 20 b^3) plus U_t Sigma_t 2 m n t).  Clears earlier
 * records; 0 turns timing off. */
peps_status peps_profile_enable(peps_ctx* ctx, uint32_t class_mask);

/* Synchronise the context's stream and report, for one kernel class, the summed
 * device time (ms), the number of timed launches and their summed algorithmic flops
 * since the last peps_profile_enable. */
peps_status peps_profile_read(peps_ctx* ctx, int32_t kernel_class, double* total_ms,
                              int64_t* launches, double* flops);

/* The summed algorithmic HBM bytes of one kernel class's timed launches since the last
 * peps_profile_enable (call after peps_profile_read, which synchronises).  Counted for the
 * GEMM class only (0 for the others): per launch, every operand read once and the result
 * written once for each active sample, in its storage type; an operand shared by all
 * samples (the site tensors, the ones vector) once per launch, both spin slices of a
 * gathered one.  The minimum traffic of the product, for a bandwidth roofline. */
peps_status peps_profile_read_bytes(peps_ctx* ctx, int32_t kernel_class, double* bytes);

/* Diagnostic, no device work: lay out the workspace of one chunk of `batch` samples
 * and walk the whole launch sequence of an evaluation (want_eloc, grad_mode as in
 * peps_evaluate; sweeps as in peps_set_truncation) without launching anything,
 * checking on the host that every operand offset stays inside its buffer.  Returns
 * PEPS_OK and the chunk's workspace bytes, PEPS_ERR_INVALID_ARG if a check fails, or
 * PEPS_ERR_UNSUPPORTED as peps_set_truncation's evaluations would.  Needs no GPU. */
peps_status peps_plan_check(const peps_lattice* lat, int64_t batch, int32_t grad_mode,
                            int32_t want_eloc, int32_t sweeps, size_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* PEPS_H */
