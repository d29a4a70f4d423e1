// Host side of the PEPS library: argument checks, the per-lattice plan (bond
// dimensions of every boundary MPS and truncation), workspace layout, and the
// launch sequence of one evaluation.  Every arithmetic step runs in the HIP
// kernels; this file only computes shapes, offsets and strides.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "peps.h"
#include "common.h"
#include "kernels.h"

// one timed launch: events recorded on the context stream around it
struct ProfRec {
    hipEvent_t a, b;
    int cls;
    double flops;
    double bytes;   // algorithmic HBM bytes (GEMMs: operands read once, result written once)
};

// a captured job list of peps_eval_jobs, replayed when the same list comes again
struct CachedGraph {
    std::string key;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

static constexpr int kMaxSweeps = 16;

struct peps_ctx {
    int device = 0;
    std::vector<CachedGraph> graphs;          // captured job lists (peps_eval_jobs)
    std::vector<hipStream_t> job_streams;
    std::vector<hipEvent_t> job_events;
    std::map<std::string, int> tune;          // GEMM shape -> tile (autotuner)
    bool tune_mode = false;
    int tuned_now = 0;
    uint32_t prof_mask = 0;          // bit per kernel class (PEPS_KC_*) to time
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> ev_pool;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    size_t ws_limit = 0;
    double* ones = nullptr;   // 4096 ones
    char* scratch = nullptr;  // device address of this device's fixed scratch array
    bool fused_steps = true;  // fused float32 sandwich steps where they fit (else the GEMM form)
    int vc_sweeps = 0;        // 0: SVD truncation; n > 0: variational compression, n sweeps
    char* mc = nullptr;       // sampling buffers (peps_metropolis_step, peps_vmc_step)
    size_t mc_bytes = 0;
    char* corr = nullptr;     // exchanged configurations and their amplitudes (peps_pair_correlations)
    size_t corr_bytes = 0;
    std::string err;
};

static void drop_graphs(peps_ctx* c) {
    for (auto& g : c->graphs) {
        hipGraphExecDestroy(g.exec);
        hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
}

// Fixed device scratch of the allocation-free evaluation (peps_evaluate_noalloc): each
// device that loads the library holds its own copy until the process ends, shared by
// every context and call on that device.  Host code never passes `scratch` itself (in
// host code the name is a stand-in, not a device address): it takes this device's
// address from hipGetSymbolAddress once, with the device current (scratch_address).
static constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, char*> g_scratch_ptr;   // device -> address of its scratch copy

// this device's scratch address; the device must be current
static char* scratch_address(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) return it->second;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[device] = static_cast<char*>(p);
    return static_cast<char*>(p);
}

namespace peps {

void set_lds_cap(size_t bytes);

namespace {

constexpr int kOnes = 4096;

struct Op {
    double* p;
    long long bs;      // batch stride in elements
    long long ext;     // elements addressable from p for one sample (host-side bounds check)
    bool f32 = false;  // float32 storage (GEMM temporaries): p then addresses floats
    Op at(long long off) const {
        double* q = f32 ? reinterpret_cast<double*>(reinterpret_cast<float*>(p) + off) : p + off;
        return Op{q, bs, ext - off, f32};
    }
};

inline Idx2 I1(long long s) { return Idx2{1 << 30, 0, s}; }
inline Idx2 I2(int inner, long long so, long long si) { return Idx2{inner, so, si}; }

struct Trunc {
    std::vector<int> chi, K, rho, tau;
    int pin = 1, p = 1;
};

struct Layout {
    // per-chunk byte offsets of each buffer and per-sample strides (doubles)
    size_t bytes = 0;
    int Bc = 0;
    size_t alloc(long long per_sample, long long fixed = 0) {
        size_t off = bytes;
        size_t n = (size_t)(per_sample * Bc + fixed) * sizeof(double);
        bytes += (n + 255) / 256 * 256;
        return off;
    }
};

class Runner {
public:
    Runner(peps_ctx* c, const peps_lattice& l, peps_precision pr)
        : ctx(c), lat(l), prec(pr) {
        Lx = l.Lx; Ly = l.Ly; D = l.D; Dc = l.Dc; N = Lx * Ly;
        D2 = D * D; D3 = D2 * D; D4 = D3 * D;
        // bf16 applies to the MPO x MPS apply GEMMs of the boundary sweeps; the sandwich and
        // environment-tensor GEMMs then run in f32 (f32 and f64 use one type throughout)
        ar = prec == PEPS_PREC_F64 ? Arith::F64 : (prec == PEPS_PREC_F32 ? Arith::F32 : Arith::BF16);
        ar_sw = prec == PEPS_PREC_F64 ? Arith::F64 : Arith::F32;
        // fused single- and two-row sandwich steps in float32 (peps_set_fused_steps(ctx, 0)
        // keeps the GEMM form, with the same results)
        fuse_pairs = ar_sw == Arith::F32 && D <= 4 && c->fused_steps;
        Dh.assign(Lx + 1, D); Dh[0] = Dh[Lx] = 1;
        Dv.assign(Ly + 1, D); Dv[0] = Dv[Ly] = 1;
        chiU.assign(Ly, std::vector<int>(Lx + 1, 1));
        chiL.assign(Ly, std::vector<int>(Lx + 1, 1));
        tU.resize(Ly);
        tL.resize(Ly);
        for (int i = 0; i + 1 < Ly; ++i) {
            tU[i] = make_trunc(chiU[i], Dv[i], Dv[i + 1]);
            chiU[i + 1] = tU[i].tau;
        }
        for (int i = Ly - 1; i >= 1; --i) {
            tL[i] = make_trunc(chiL[i], Dv[i + 1], Dv[i]);
            chiL[i - 1] = tL[i].tau;
        }
        sweeps = c->vc_sweeps;
        vcU.assign(Ly, 0);
        vcL.assign(Ly, 0);
        for (int i = 0; i + 1 < Ly; ++i) vcU[i] = use_vc(tU[i]);
        for (int i = Ly - 1; i >= 1; --i) vcL[i] = use_vc(tL[i]);
    }

    // Variational compression replaces the SVD truncation of a boundary wherever the
    // incoming boundary (its guess) already has the bond and physical dims of the result.
    bool use_vc(const Trunc& t) const { return sweeps > 0 && t.pin == t.p && t.chi == t.tau; }
    // the reason a planned variational step cannot run ("" when every one can)
    std::string vc_unsupported() const {
        auto check = [&](const Trunc& t) -> std::string {
            for (int j = 0; j < Lx; ++j) {
                const int a = t.chi[j], b = t.chi[j + 1];
                if (!thinq_shape_ok(a * t.p, b) || !thinq_shape_ok(t.p * b, a)) {
                    char m[160];
                    snprintf(m, sizeof m, "variational compression: bond %d exceeds the 128 columns of the "
                             "site factorisation", std::max(a, b));
                    return m;
                }
            }
            return "";
        };
        for (int i = 0; i + 1 < Ly; ++i)
            if (vcU[i]) {
                std::string m = check(tU[i]);
                if (!m.empty()) return m;
            }
        for (int i = Ly - 1; i >= 1; --i)
            if (vcL[i]) {
                std::string m = check(tL[i]);
                if (!m.empty()) return m;
            }
        return "";
    }

    Trunc make_trunc(const std::vector<int>& chi, int pin, int p) const {
        Trunc t;
        t.chi = chi; t.pin = pin; t.p = p;
        t.K.resize(Lx + 1); t.rho.resize(Lx + 1); t.tau.resize(Lx + 1);
        for (int c = 0; c <= Lx; ++c) t.K[c] = chi[c] * Dh[c];
        t.rho[0] = 1;
        for (int j = 0; j + 1 < Lx; ++j) t.rho[j + 1] = std::min(t.rho[j] * p, t.K[j + 1]);
        t.rho[Lx] = 1;
        t.tau[Lx] = 1;
        for (int j = Lx - 1; j >= 1; --j) t.tau[j] = std::min(std::min(Dc, t.rho[j]), p * t.tau[j + 1]);
        t.tau[0] = 1;
        return t;
    }

    long long env_row_size(const std::vector<int>& chi, int phys) const {
        long long s = 0;
        for (int j = 0; j < Lx; ++j) s += (long long)chi[j] * phys * chi[j + 1];
        return s;
    }
    long long env_off(const std::vector<int>& chi, int phys, int j) const {
        long long s = 0;
        for (int c = 0; c < j; ++c) s += (long long)chi[c] * phys * chi[c + 1];
        return s;
    }

    // ---- workspace layout for a chunk of Bc samples ----
    void layout(int Bc_, bool want_e, bool want_g) {
        L = Layout();
        L.Bc = Bc_;
        Bc = Bc_;
        want_eloc = want_e; want_grad = want_g;
        o_envU.resize(Ly); o_envL.resize(Ly); o_logU.resize(Ly); o_logL.resize(Ly);
        s_envU.resize(Ly); s_envL.resize(Ly);
        for (int i = 0; i < Ly; ++i) {
            s_envU[i] = env_row_size(chiU[i], Dv[i]);
            o_envU[i] = L.alloc(s_envU[i]);
            o_logU[i] = L.alloc(1);
        }
        const bool need_L = want_e || want_g;
        for (int i = 0; i < Ly; ++i) {
            s_envL[i] = env_row_size(chiL[i], Dv[i + 1]);
            o_envL[i] = (need_L || i == Ly - 1) ? L.alloc(s_envL[i]) : 0;
            o_logL[i] = (need_L || i == Ly - 1) ? L.alloc(1) : 0;
        }
        // truncation buffers (max over every truncation of the plan)
        s_X.assign(Lx, 1); s_tau.assign(Lx, 1); s_wy.assign(Lx, 0);
        s_vc = 0; s_wq = 0;
        s_R = 1; s_Y = 1; s_G = 1; s_svd = 0;
        auto visit = [&](const Trunc& t) {
            for (int j = 0; j < Lx; ++j) {
                const long long rows = (long long)t.rho[j] * t.p, cols = t.K[j + 1];
                s_X[j] = std::max(s_X[j], rows * cols);
                s_tau[j] = std::max<long long>(s_tau[j], std::min(rows, cols));
                if (j + 1 < Lx && use_qrb((int)rows, (int)cols)) {
                    s_wy[j] = std::max(s_wy[j], qrb_wy_doubles((int)rows, (int)cols));
                    s_vc = std::max(s_vc, qrb_vc_doubles((int)rows));
                    s_wq = std::max(s_wq, qrb_wq_doubles((int)cols));
                }
                if (j + 1 < Lx) s_R = std::max(s_R, (long long)t.rho[j + 1] * t.K[j + 1]);
                s_Y = std::max(s_Y, (long long)t.rho[j] * Dh[j] * t.pin * t.chi[j + 1]);
                s_G = std::max(s_G, (long long)t.rho[j] * t.tau[j]);
                const int tin = t.tau[j + 1];
                const long long mz = rows;
                const size_t sc = center0_scratch_doubles((int)mz, tin);
                if (j == 0 && sc * sizeof(double) > lds_cap_bytes()) s_svd = std::max<long long>(s_svd, sc);
            }
        };
        for (int i = 0; i + 1 < Ly; ++i)
            if (!vcU[i]) visit(tU[i]);
        if (need_L)
            for (int i = Ly - 1; i >= 1; --i)
                if (!vcL[i]) visit(tL[i]);
        // variational compression: overlap environments L_c and R_c per cut c ([c][a][l],
        // bond x bond x horizontal leg), two contraction temporaries, the updated site
        // tensor and the triangular factor of the guess's canonicalisation
        vc_eoff.assign(Lx + 2, 0);
        {
            std::vector<long long> e(Lx + 1, 0);
            s_vZ1 = s_vZ2 = s_vM = s_vRf = s_vW = 0;
            auto visit_vc = [&](const Trunc& t) {
                for (int c = 0; c <= Lx; ++c) e[c] = std::max<long long>(e[c], (long long)t.chi[c] * t.chi[c] * Dh[c]);
                for (int j = 0; j < Lx; ++j) {
                    const long long a = t.chi[j], b = t.chi[j + 1], hl = Dh[j], hr = Dh[j + 1], p = t.p;
                    s_vZ1 = std::max({s_vZ1, a * hl * p * b, b * hr * a * p});
                    s_vZ2 = std::max({s_vZ2, a * b * hr * p, b * a * hl * p});
                    s_vM = std::max(s_vM, a * p * b);
                    s_vRf = std::max({s_vRf, a * a, b * b});
                    if (thinq_needs_scratch((int)(a * p), (int)b) || thinq_needs_scratch((int)(p * b), (int)a))
                        s_vW = std::max(s_vW, a * p * b);
                }
            };
            bool any = false;
            for (int i = 0; i + 1 < Ly; ++i)
                if (vcU[i]) { visit_vc(tU[i]); any = true; }
            if (need_L)
                for (int i = Ly - 1; i >= 1; --i)
                    if (vcL[i]) { visit_vc(tL[i]); any = true; }
            for (int c = 0; c <= Lx; ++c) vc_eoff[c + 1] = vc_eoff[c] + e[c];
            s_vE = vc_eoff[Lx + 1];
            o_vL = any ? L.alloc(s_vE) : 0;
            o_vR = any ? L.alloc(s_vE) : 0;
            o_vZ1 = any ? L.alloc(s_vZ1) : 0;
            o_vZ2 = any ? L.alloc(s_vZ2) : 0;
            o_vM = any ? L.alloc(s_vM) : 0;
            o_vRf = any ? L.alloc(s_vRf) : 0;
            o_vW = s_vW > 0 ? L.alloc(s_vW) : 0;   // factorisations beyond LDS
        }
        o_X.resize(Lx); o_tau.resize(Lx); o_wy.assign(Lx, 0);
        for (int j = 0; j < Lx; ++j) {
            o_X[j] = L.alloc(s_X[j]);
            o_tau[j] = L.alloc(s_tau[j]);
            if (s_wy[j] > 0) o_wy[j] = L.alloc(s_wy[j]);
        }
        o_vc = s_vc > 0 ? L.alloc(s_vc) : 0;
        o_wq = s_wq > 0 ? L.alloc(s_wq) : 0;
        o_R[0] = L.alloc(s_R); o_R[1] = L.alloc(s_R);
        o_Y = L.alloc(s_Y);
        o_G[0] = L.alloc(s_G); o_G[1] = L.alloc(s_G);
        o_svd = s_svd ? L.alloc(s_svd) : 0;
        s_eig = 1;
        auto visit_eig = [&](const Trunc& t) {
            for (int j = 1; j < Lx; ++j) {
                const int mz = t.rho[j] * t.p, tin = (j + 1 < Lx) ? t.tau[j + 1] : 1;
                s_eig = std::max<long long>(s_eig, (long long)eig_scratch_doubles(mz, tin, t.p, Dc));
            }
        };
        for (int i = 0; i + 1 < Ly; ++i)
            if (!vcU[i]) visit_eig(tU[i]);
        if (need_L)
            for (int i = Ly - 1; i >= 1; --i)
                if (!vcL[i]) visit_eig(tL[i]);
        o_eig = L.alloc(s_eig);
        // single-row partials
        s_P.assign(Lx + 1, 1);
        for (int i = 0; i < Ly; ++i)
            for (int j = 0; j <= Lx; ++j)
                s_P[j] = std::max(s_P[j], (long long)chiU[i][j] * Dh[j] * chiL[i][j]);
        o_P.resize(Lx + 1); o_Q.resize(Lx + 1); o_lP.resize(Lx + 1); o_lQ.resize(Lx + 1);
        for (int j = 0; j <= Lx; ++j) {
            o_P[j] = L.alloc(s_P[j]);
            o_Q[j] = (need_L) ? L.alloc(s_P[j]) : 0;
            o_lP[j] = L.alloc(1);
            o_lQ[j] = L.alloc(1);
        }
        long long sT = 1, sF = 1;
        for (int i = 0; i < Ly; ++i)
            for (int j = 0; j < Lx; ++j) {
                const long long cu = chiU[i][j], cu1 = chiU[i][j + 1], cl = chiL[i][j], cl1 = chiL[i][j + 1];
                const long long Du = Dv[i], Dd = Dv[i + 1], h = Dh[j], h1 = Dh[j + 1];
                sT = std::max({sT, h * cl * Du * cu1, cl * cu1 * h1 * Dd, cl * Dd * cu1 * h1,
                               h * Du * cl * cu1});
                sF = std::max(sF, cu1 * h1 * cl1);
            }
        // two-row partials
        s_P2.assign(Lx + 1, 1);
        if (want_e) {
            for (int i = 0; i + 1 < Ly; ++i)
                for (int j = 0; j <= Lx; ++j)
                    s_P2[j] = std::max(s_P2[j], (long long)chiU[i][j] * Dh[j] * Dh[j] * chiL[i + 1][j]);
            for (int i = 0; i + 1 < Ly; ++i)
                for (int j = 0; j < Lx; ++j) {
                    const long long cu = chiU[i][j], cu1 = chiU[i][j + 1], cl = chiL[i + 1][j],
                                    cl1 = chiL[i + 1][j + 1];
                    const long long Du = Dv[i], Dm = Dv[i + 1], Dq = Dv[i + 2], h = Dh[j], h1 = Dh[j + 1];
                    sT = std::max({sT, h * h * cl * Du * cu1, h * cl * cu1 * h1 * Dm,
                                   cl * cu1 * h1 * h1 * Dq, cl * Dq * cu1 * h1 * h1,
                                   h * Dm * cl * cu1 * h1, h * Du * h * cl * cu1});
                    sF = std::max(sF, cu1 * h1 * h1 * cl1);
                    (void)cu;
                }
            o_P2.resize(Lx + 1); o_Q2.resize(Lx + 1); o_lP2.resize(Lx + 1); o_lQ2.resize(Lx + 1);
            for (int j = 0; j <= Lx; ++j) {
                o_P2[j] = L.alloc(s_P2[j]);
                o_Q2[j] = L.alloc(s_P2[j]);
                o_lP2[j] = L.alloc(1);
                o_lQ2[j] = L.alloc(1);
            }
        }
        s_T = sT; s_F = sF;
        for (int k = 0; k < 3; ++k) o_T[k] = L.alloc(s_T);
        o_F = L.alloc(s_F);
        o_Gf = L.alloc(s_F);
        o_lnW = L.alloc(1); o_sgW = L.alloc(1);
        o_lnW2 = L.alloc(1); o_sgW2 = L.alloc(1);
        o_lnWf = L.alloc(1); o_sgWf = L.alloc(1);
        o_zero = L.alloc(1);
        o_site32 = fuse_pairs ? L.alloc(0, (long long)N * 512) : 0;   // float32 site tables
        nbonds = Ly * (Lx - 1) + (Ly - 1) * Lx + 2 * (Ly - 1) * (Lx - 1);
        o_ratio = want_e ? L.alloc(nbonds) : 0;
        o_act = want_e ? L.alloc(0, ((long long)Bc * nbonds + 7) / 8) : 0;   // int8 [Bc][nbonds]
        o_delta = want_g ? L.alloc((long long)N * D4) : 0;
        o_flags = L.alloc(1);   // int8 flags in a double-sized slot per sample
        o_eloc = L.alloc(1);
        o_acc = L.alloc(0, 8);
        o_G1 = want_g ? L.alloc(0, 2LL * N * D4) : 0;
        o_G0 = want_g ? L.alloc(0, 2LL * N * D4) : 0;
        // partial sums of the batch reduction: 2 x grad_parts(Bc) partitions of 2 N D^4
        o_gws = want_g ? L.alloc((4LL * N * D4 + kGradParts - 1) / kGradParts + 1, 4LL * N * D4) : 0;
    }

    static size_t lds_cap_bytes();

    double* buf(size_t off) const { return (double*)(base_ + off); }
    Op op(size_t off, long long per) const { return Op{buf(off), per, per}; }
    // a GEMM-to-GEMM temporary: float32 storage when its GEMMs accumulate in float32 (their
    // outputs are then exact float32 values, so nothing is rounded by the narrower storage)
    Op tmp(size_t off, long long per, Arith a) const { return Op{buf(off), per, per, a != Arith::F64}; }
    Op ones() const { return Op{ctx->ones, 0, kOnes}; }

    // largest element offset an Idx2 can produce over [0, n) (an upper bound)
    static long long idx_max(const Idx2& x, int n) {
        if (n <= 0) return 0;
        const long long outer = (long long)(n - 1) / x.inner;
        const long long inner = std::min<long long>(n, x.inner) - 1;
        return outer * x.s_outer + inner * x.s_inner;
    }
    bool bounds_ok(const char* what, const Op& o, long long maxoff, long long slice) {
        if (maxoff + slice < o.ext) return true;
        char b[256];
        snprintf(b, sizeof b, "internal bounds check failed in %s: offset %lld + %lld >= extent %lld",
                 what, maxoff, slice, o.ext);
        bounds_msg = b;
        return false;
    }

    // ---- launch helpers ----
    hipError_t gemm(int M, int Nn, int K, Op A, Idx2 am, Idx2 ak, Gather ga, Op B, Idx2 bk, Idx2 bn,
                    Gather gb, Op C, Idx2 cm, Idx2 cn) {
        return gemm_a(ar_sw, M, Nn, K, A, am, ak, ga, B, bk, bn, gb, C, cm, cn);
    }
    hipError_t gemm_a(Arith arith, int M, int Nn, int K, Op A, Idx2 am, Idx2 ak, Gather ga, Op B,
                      Idx2 bk, Idx2 bn, Gather gb, Op C, Idx2 cm, Idx2 cn) {
        if (!bounds_ok("gemm A", A, idx_max(am, M) + idx_max(ak, K), ga.sel ? ga.slice : 0) ||
            !bounds_ok("gemm B", B, idx_max(bk, K) + idx_max(bn, Nn), gb.sel ? gb.slice : 0) ||
            !bounds_ok("gemm C", C, idx_max(cm, M) + idx_max(cn, Nn), 0))
            return hipErrorInvalidValue;
        if (dry) return hipSuccess;
        GemmArgs g;
        const double ns = (double)active_samples();
        const double fl = 2.0 * M * Nn * K * ns;
        // algorithmic bytes: each operand read once and the result written once per active
        // sample; an operand shared by all samples (batch stride 0) once per launch, both
        // spin slices of a gathered one
        auto obytes = [&](const Op& o, double elems, const Gather& gt) {
            const double w = o.f32 ? 4.0 : 8.0;
            return o.bs == 0 ? elems * w * (gt.sel ? 2.0 : 1.0) : elems * w * ns;
        };
        const double by = obytes(A, (double)M * K, ga) + obytes(B, (double)K * Nn, gb) +
                          obytes(C, (double)M * Nn, Gather{});
        g.M = M; g.N = Nn; g.K = K; g.batch = Bcur;
        g.am = am; g.ak = ak; g.bk = bk; g.bn = bn; g.cm = cm; g.cn = cn;
        g.a_bs = A.bs; g.b_bs = B.bs; g.c_bs = C.bs;
        g.ga = ga; g.gb = gb; g.gc = Gather{nullptr, 0, 0, 0};
        g.A = A.p; g.B = B.p; g.C = C.p;
        g.alpha = 1.0; g.beta = 0.0;
        g.a_f32 = A.f32; g.b_f32 = B.f32; g.c_f32 = C.f32;
        g.skip = skip_; g.skip_bs = skip_bs_;
        char kb[96];
        snprintf(kb, sizeof kb, "%d,%d,%d,%d,%d,%d", M, Nn, K, Bcur, (int)arith,
                 (int)A.f32 | ((int)B.f32 << 1) | ((int)C.f32 << 2));
        const std::string key(kb);
        int tile = 0;
        auto it = ctx->tune.find(key);
        if (it != ctx->tune.end()) {
            tile = it->second;
        } else if (ctx->tune_mode) {
            // time every tile on this very launch (all tiles give identical results, and the
            // product has beta = 0, so repeating it changes nothing): one untimed launch
            // first, so a kernel's first-use cost does not count against it
            hipEvent_t ev[2];
            if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
                return hipErrorUnknown;
            float best = 1e30f;
            int best_t = 0;
            for (int t = 1; t <= kGemmTiles; ++t) {
                hipError_t e0 = launch_gemm(g, arith, st_, t);
                if (e0 != hipSuccess) return e0;
                hipEventRecord(ev[0], st_);
                hipError_t e = launch_gemm(g, arith, st_, t);
                hipEventRecord(ev[1], st_);
                if (e != hipSuccess) return e;
                hipEventSynchronize(ev[1]);
                float ms = 0.f;
                hipEventElapsedTime(&ms, ev[0], ev[1]);
                if (ms < best) {
                    best = ms;
                    best_t = t;
                }
            }
            hipEventDestroy(ev[0]);
            hipEventDestroy(ev[1]);
            ctx->tune[key] = best_t;
            ctx->tuned_now++;
            return hipSuccess;
        }
        return timed(PEPS_KC_GEMM, fl, [&] { return launch_gemm(g, arith, st_, tile); }, by);
    }
    Gather site_gather(int i, int j, int flip) const {
        return Gather{Scur + (long long)i * Lx + j, (long long)N, flip, (long long)D4};
    }
    Op site_op(int i, int j) const {
        const long long off = ((long long)(i * Lx + j) * 2) * D4;
        return Op{const_cast<double*>(Ad) + off, 0, (long long)N * 2 * D4 - off};
    }
    Op envU(int i, int j) const {
        if (i == 0) return ones();
        return op(o_envU[i], s_envU[i]).at(env_off(chiU[i], Dv[i], j));
    }
    Op envL(int i, int j) const {
        if (i == Ly - 1) return ones();
        return op(o_envL[i], s_envL[i]).at(env_off(chiL[i], Dv[i + 1], j));
    }
    Op logU(int i) const { return op(o_logU[i], 1); }
    Op logL(int i) const { return op(o_logL[i], 1); }

#define CK(x)                                  \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return e_;       \
    } while (0)
// a kernel launch: skipped in a dry run, which only walks the plan and checks bounds
#define KL(x)                                  \
    do {                                       \
        if (!dry) {                            \
            hipError_t e_ = (x);               \
            if (e_ != hipSuccess) return e_;   \
        }                                      \
    } while (0)

    // One truncation: new env = Trunc(Apply(env, row)), top-down (down) or bottom-up.
    hipError_t trunc_step(bool down, int row) {
        const Trunc& t = down ? tU[row] : tL[row];
        const long long s_in = down ? D2 : 1, s_out = down ? 1 : D2;
        const int pin = t.pin, p = t.p;
        for (int j = 0; j < Lx; ++j) {
            const int chj = t.chi[j], chj1 = t.chi[j + 1], Dl = Dh[j], Dr = Dh[j + 1];
            const int rho = t.rho[j];
            Op Rin = (j == 0) ? ones() : op(o_R[(j - 1) & 1], s_R);
            const long long ldR = t.K[j];
            Op Ein = down ? envU(row, j) : envL(row, j);
            Op Y = tmp(o_Y, s_Y, ar);
            // Y[(a',l),(u,b)] = sum_a R[a', a*Dl+l] E[a,(u,b)]
            CK(gemm_a(ar, rho * Dl, pin * chj1, chj, Rin, I2(Dl, ldR, 1), I1(Dl), Gather{},
                    Ein, I1((long long)pin * chj1), I1(1), Gather{},
                    Y, I1((long long)pin * chj1), I1(1)));
            // X[(a',d),(b,r)] (column-major) = sum_{l,u} Y[a',l,u,b] T[l,u,r,d]
            const long long rows = (long long)rho * p;
            Op X = op(o_X[j], s_X[j]);
            CK(gemm_a(ar, rho * chj1, Dr * p, Dl * pin, Y, I2(chj1, (long long)Dl * pin * chj1, 1),
                    I2(pin, (long long)pin * chj1, chj1), Gather{},
                    site_op(row, j), I2(pin, D3, s_in), I2(p, D, s_out), site_gather(row, j, 0),
                    X, I2(chj1, p, Dr * rows), I2(p, rows, 1)));
            if (j + 1 < Lx) {
                if (rows * t.K[j + 1] > s_X[j] || std::min<long long>(rows, t.K[j + 1]) > s_tau[j] ||
                    (long long)t.rho[j + 1] * t.K[j + 1] > s_R) {
                    bounds_msg = "internal bounds check failed in qr";
                    return hipErrorInvalidValue;
                }
                const bool blocked = use_qrb((int)rows, t.K[j + 1]);
                if (blocked && (qrb_wy_doubles((int)rows, t.K[j + 1]) > s_wy[j] ||
                                qrb_vc_doubles((int)rows) > s_vc || qrb_wq_doubles(t.K[j + 1]) > s_wq)) {
                    bounds_msg = "internal bounds check failed in blocked qr";
                    return hipErrorInvalidValue;
                }
                KL(timed(PEPS_KC_QR, Bcur * qr_flops((double)rows, t.K[j + 1]), [&] {
                    if (blocked)
                        return launch_qr_blocked(X.p, X.bs, (int)rows, t.K[j + 1], buf(o_R[j & 1]), s_R,
                                                 buf(o_tau[j]), s_tau[j], buf(o_wy[j]), s_wy[j], buf(o_vc), s_vc,
                                                 buf(o_wq), s_wq, Bcur, st_);
                    return launch_qr(X.p, X.bs, (int)rows, t.K[j + 1], buf(o_R[j & 1]), s_R,
                                     buf(o_tau[j]), s_tau[j], Bcur, st_);
                }));
            }
        }
        // right-to-left SVD sweep (bounds of every factorisation buffer checked first)
        for (int j = 0; j < Lx; ++j) {
            const long long mz = (long long)t.rho[j] * p;
            const int tin = t.tau[j + 1];
            const size_t sc = center0_scratch_doubles((int)mz, tin);
            const bool in_lds = sc * sizeof(double) <= lds_cap_bytes();
            const long long rin = (j + 1 < Lx) ? t.rho[j + 1] : mz;     // rows of G / reflectors
            bool ok = j == 0 ? (in_lds || (long long)sc <= s_svd)
                             : (long long)eig_scratch_doubles((int)mz, tin, p, Dc) <= s_eig;
            ok = ok && mz * (j + 1 < Lx ? t.K[j + 1] : 1) <= s_X[j];
            ok = ok && (j + 1 == Lx || (rin <= s_tau[j] && rin * tin <= s_G));
            ok = ok && (long long)t.rho[j] * t.tau[j] <= s_G;
            const std::vector<int>& chn = down ? chiU[row + 1] : chiL[row - 1];
            ok = ok && chn[j] == t.tau[j] && chn[j + 1] == t.tau[j + 1];
            if (!ok) {
                bounds_msg = "internal bounds check failed in svd";
                return hipErrorInvalidValue;
            }
        }
        int cur = 0;
        {
            const int j = Lx - 1;
            Op Eout = down ? envU(row + 1, j) : envL(row - 1, j);
            const int mz = t.rho[j] * p;
            KL(timed(PEPS_KC_SVD, Bcur * svd_flops(mz, 0, 1, p, t.tau[j]), [&] {
                return launch_eig(nullptr, 0, buf(o_tau[0]), 0, buf(o_X[j]), s_X[j], mz, mz, 1, p, Dc,
                                  Eout.p, Eout.bs, buf(o_G[0]), s_G, buf(o_eig), s_eig, Bcur, st_);
            }));
        }
        for (int j = Lx - 2; j >= 1; --j) {
            Op Eout = down ? envU(row + 1, j) : envL(row - 1, j);
            const int mz = t.rho[j] * p;
            KL(timed(PEPS_KC_SVD, Bcur * svd_flops(mz, t.rho[j + 1], t.tau[j + 1], p, t.tau[j]), [&] {
                const bool blocked = use_qrb(mz, t.K[j + 1]);
                return launch_eig(buf(o_X[j]), s_X[j], buf(o_tau[j]), s_tau[j], buf(o_G[cur]), s_G, mz,
                                  t.rho[j + 1], t.tau[j + 1], p, Dc, Eout.p, Eout.bs, buf(o_G[cur ^ 1]), s_G,
                                  buf(o_eig), s_eig, Bcur, st_, blocked ? buf(o_wy[j]) : nullptr, s_wy[j]);
            }));
            cur ^= 1;
        }
        {
            Op Eout = down ? envU(row + 1, 0) : envL(row - 1, 0);
            Op lin = down ? logU(row) : logL(row);
            Op lout = down ? logU(row + 1) : logL(row - 1);
            KL(launch_center0(buf(o_X[0]), s_X[0], buf(o_tau[0]), s_tau[0], buf(o_G[cur]), s_G, p,
                              t.rho[1], t.tau[1], Eout.p, Eout.bs, lin.p, lout.p, buf(o_svd), s_svd,
                              Bcur, st_));
        }
        return hipSuccess;
    }

    // One variational compression: new env = the one-site least-squares fit of
    // Apply(env, row) started from env itself (same bond and physical dims), in `sweeps`
    // sweeps, never forming the applied MPS.  Indices of site j: a = bond at cut j,
    // b = bond at cut j+1 (incoming and outgoing boundaries alike), l / r = the row's
    // horizontal legs (Dh), u / d = its incoming / outgoing physical leg (p each).
    // Overlap environments: L_j[c][a][l] = <C| rows |E> left of cut j, R_j the same right
    // of it.  Every contraction is a float64 GEMM; every QR a thin QR with explicit Q
    // (launch_thinq: in registers, LDS or, for the largest, global scratch).
    hipError_t vc_step(bool down, int row) {
        const Trunc& t = down ? tU[row] : tL[row];
        const long long s_in = down ? D2 : 1, s_out = down ? 1 : D2;
        const int p = t.p;
        const Arith F = Arith::F64;
        auto Ein = [&](int j) { return down ? envU(row, j) : envL(row, j); };
        auto Cout = [&](int j) { return down ? envU(row + 1, j) : envL(row - 1, j); };
        auto Lenv = [&](int c) { return c == 0 ? ones() : op(o_vL, s_vE).at(vc_eoff[c]); };
        auto Renv = [&](int c) { return c == Lx ? ones() : op(o_vR, s_vE).at(vc_eoff[c]); };
        const Op Z1 = op(o_vZ1, s_vZ1), Z2 = op(o_vZ2, s_vZ2), Mb = op(o_vM, s_vM), Rf = op(o_vRf, s_vRf);
        const Op lin = down ? logU(row) : logL(row), lout = down ? logU(row + 1) : logL(row - 1);
        // thin QR of an m x n column-major matrix at X into Q (rows q_row, columns q_col apart)
        auto thinq = [&](const Op& X, int m, int n, const Op& Q, long long q_row, long long q_col,
                         bool with_r) -> hipError_t {
            const bool on_chip = !thinq_needs_scratch(m, n);   // registers or LDS: no scratch
            const Op Wq = op(o_vW, s_vW);
            if (!bounds_ok("vc qr in", X, (long long)m * n - 1, 0) ||
                !bounds_ok("vc qr out", Q, (long long)(m - 1) * q_row + (long long)(n - 1) * q_col, 0) ||
                (with_r && !bounds_ok("vc qr R", Rf, (long long)n * n - 1, 0)) ||
                (!on_chip && (s_vW < (long long)m * n || !bounds_ok("vc qr scratch", Wq, (long long)m * n - 1, 0))))
                return hipErrorInvalidValue;
            const double fl = (4.0 * m * n * n - 4.0 / 3.0 * n * n * n) * Bcur;
            KL(timed(PEPS_KC_QR, fl, [&] {
                return launch_thinq(X.p, X.bs, m, n, Q.p, Q.bs, q_row, q_col, with_r ? Rf.p : nullptr, Rf.bs,
                                    on_chip ? nullptr : Wq.p, on_chip ? 0 : Wq.bs, Bcur, st_);
            }));
            return hipSuccess;
        };
        // W2[c'][a][l][d] = sum_{a',r,u} R_{j+1}[c',a',r] E_j[a,u,a'] T_j[l,u,r,d] (in Z2)
        auto right_part = [&](int j) -> hipError_t {
            const int a = t.chi[j], b = t.chi[j + 1], hl = Dh[j], hr = Dh[j + 1];
            CK(gemm_a(F, b * hr, a * p, b, Renv(j + 1), I2(hr, (long long)b * hr, 1), I1(hr), Gather{},
                      Ein(j), I1(1), I1(b), Gather{}, Z1, I1((long long)a * p), I1(1)));
            CK(gemm_a(F, b * a, hl * p, hr * p, Z1, I2(a, (long long)hr * a * p, p), I2(p, (long long)a * p, 1),
                      Gather{}, site_op(row, j), I2(p, D, s_in), I2(p, D3, s_out), site_gather(row, j, 0),
                      Z2, I1((long long)hl * p), I1(1)));
            return hipSuccess;
        };
        // R_j[c][a][l] = sum_{d,c'} C_j[c,d,c'] W2[c',a,l,d]
        auto right_env = [&](int j) -> hipError_t {
            const int a = t.chi[j], b = t.chi[j + 1], hl = Dh[j];
            CK(gemm_a(F, a, a * hl, p * b, Cout(j), I1((long long)p * b), I1(1), Gather{}, Z2,
                      I2(b, 1, (long long)a * hl * p), I1(p), Gather{}, Renv(j), I1((long long)a * hl), I1(1)));
            return hipSuccess;
        };
        // C_j (row layout [c][d][c']) = sum_{a,l} L_j[c,a,l] W2[c',a,l,d]: the update seen from the right
        auto update_right = [&](int j) -> hipError_t {
            const int a = t.chi[j], b = t.chi[j + 1], hl = Dh[j];
            CK(gemm_a(F, a, p * b, a * hl, Lenv(j), I1((long long)a * hl), I1(1), Gather{}, Z2, I1(p),
                      I2(b, 1, (long long)a * hl * p), Gather{}, Cout(j), I1((long long)p * b), I1(1)));
            return hipSuccess;
        };

        // 1. the guess in right-canonical form: LQ of every site from the right (a QR of its
        //    transpose, which is the row layout read column-major), the factor pushed left
        for (int j = Lx - 1; j >= 1; --j) {
            const int a = t.chi[j], b = t.chi[j + 1];
            Op src = Ein(j);
            if (j < Lx - 1) {
                // C_j[(a,u)][k] = sum_a' E_j[(a,u), a'] R[k][a']
                CK(gemm_a(F, a * p, b, b, Ein(j), I1(b), I1(1), Gather{}, Rf, I1(1), I1(b), Gather{}, Cout(j),
                          I1(b), I1(1)));
                src = Cout(j);
            }
            CK(thinq(src, p * b, a, Cout(j), 1, (long long)p * b, true));
        }
        for (int j = Lx - 1; j >= 1; --j) {
            CK(right_part(j));
            CK(right_env(j));
        }
        // 2. the sweeps
        for (int s = 0; s < sweeps; ++s) {
            for (int j = 0; j + 1 < Lx; ++j) {
                const int a = t.chi[j], b = t.chi[j + 1], hl = Dh[j], hr = Dh[j + 1];
                // Z1[c][l][u][a'] = sum_a L_j[c,a,l] E_j[a,u,a']
                CK(gemm_a(F, a * hl, p * b, a, Lenv(j), I2(hl, (long long)a * hl, 1), I1(hl), Gather{}, Ein(j),
                          I1((long long)p * b), I1(1), Gather{}, Z1, I1((long long)p * b), I1(1)));
                // Z2[c][a'][r][d] = sum_{l,u} Z1[c,l,u,a'] T_j[l,u,r,d]
                CK(gemm_a(F, a * b, hr * p, hl * p, Z1, I2(b, (long long)hl * p * b, 1), I1(b), Gather{},
                          site_op(row, j), I2(p, D3, s_in), I2(p, D, s_out), site_gather(row, j, 0), Z2,
                          I1((long long)hr * p), I1(1)));
                // M[(c,d)][c'] (column-major) = sum_{a',r} Z2[c,a',r,d] R_{j+1}[c',a',r]
                CK(gemm_a(F, a * p, b, b * hr, Z2, I2(p, (long long)b * hr * p, 1), I1(p), Gather{}, Renv(j + 1),
                          I1(1), I1((long long)b * hr), Gather{}, Mb, I1(1), I1((long long)a * p)));
                CK(thinq(Mb, a * p, b, Cout(j), b, 1, false));
                // L_{j+1}[c'][a'][r] = sum_{c,d} C_j[c,d,c'] Z2[c,a',r,d]
                CK(gemm_a(F, b, b * hr, a * p, Cout(j), I1(1), I1(b), Gather{}, Z2,
                          I2(p, (long long)b * hr * p, 1), I1(p), Gather{}, Lenv(j + 1), I1((long long)b * hr),
                          I1(1)));
            }
            for (int j = Lx - 1; j >= 1; --j) {
                const int a = t.chi[j], b = t.chi[j + 1];
                CK(right_part(j));
                CK(update_right(j));
                CK(thinq(Cout(j), p * b, a, Cout(j), 1, (long long)p * b, false));
                CK(right_env(j));
            }
        }
        // 3. the last update of site 0 carries the norm
        CK(right_part(0));
        CK(update_right(0));
        const Op C0 = Cout(0);
        const int n0 = p * t.chi[1];
        if (!bounds_ok("vc norm", C0, n0 - 1, 0)) return hipErrorInvalidValue;
        KL(launch_vc_norm(C0.p, C0.bs, n0, lin.p, lout.p, Bcur, st_));
        return hipSuccess;
    }

    // the single-row step as one fused kernel when it fits (done = false: use the GEMMs)
    hipError_t row_fused(int i, int j, Op X, int flip, Op Y, bool fwd, bool& done, const double* lin,
                         double* lout) {
        done = false;
        step_rescaled = false;
        if (!fuse_pairs) return hipSuccess;
        RowArgs a;
        a.cu = chiU[i][j]; a.cu1 = chiU[i][j + 1]; a.cl = chiL[i][j]; a.cl1 = chiL[i][j + 1];
        a.Du = Dv[i]; a.Dd = Dv[i + 1]; a.h = Dh[j]; a.h1 = Dh[j + 1];
        if (!row_step_fits(a)) return hipSuccess;
        const long long nl = (long long)a.cu * a.h * a.cl, nr = (long long)a.cu1 * a.h1 * a.cl1;
        const Op U = envU(i, j), L = envL(i, j);
        if (!bounds_ok("row in", X, (fwd ? nl : nr) - 1, 0) || !bounds_ok("row out", Y, (fwd ? nr : nl) - 1, 0) ||
            !bounds_ok("row U", U, (long long)a.cu * a.Du * a.cu1 - 1, 0) ||
            !bounds_ok("row L", L, (long long)a.cl * a.Dd * a.cl1 - 1, 0))
            return hipErrorInvalidValue;
        if (X.f32 || Y.f32) return hipSuccess;
        done = true;
        if (dry) return hipSuccess;
        a.X = X.p; a.xs = X.bs; a.U = U.p; a.us = U.bs; a.L = L.p; a.ls = L.bs;
        a.site = reinterpret_cast<const float*>(buf(o_site32)) + ((long long)i * Lx + j) * 1024;
        a.sel = Scur + (long long)i * Lx + j; a.sel_bs = N; a.flip = flip;
        a.Y = Y.p; a.ys = Y.bs; a.batch = Bcur;
        a.lin = lin; a.lout = lout;
        a.skip = skip_; a.skip_bs = skip_bs_;
        step_rescaled = lout != nullptr;
        const double fl = 2.0 * active_samples() *
                          ((double)a.h * a.cl * a.Du * a.cu1 * a.cu + (double)a.cl * a.cu1 * a.h1 * a.Dd * a.h * a.Du +
                           (double)a.cu1 * a.h1 * a.cl1 * a.cl * a.Dd);
        return timed(PEPS_KC_FUSED, fl, [&] { return launch_row_step(a, fwd, st_); });
    }

    // P_{j+1} = step(P_j) of the row-i sandwich <U_i| row i |L_i>
    hipError_t row_fwd(int i, int j, Op P, int flip, Op Pout, const double* lin = nullptr,
                       double* lout = nullptr) {
        bool done = false;
        CK(row_fused(i, j, P, flip, Pout, true, done, lin, lout));
        if (done) return hipSuccess;
        step_rescaled = false;
        const long long cu = chiU[i][j], cu1 = chiU[i][j + 1], cl = chiL[i][j], cl1 = chiL[i][j + 1];
        const long long Du = Dv[i], Dd = Dv[i + 1], h = Dh[j], h1 = Dh[j + 1];
        Op T1 = tmp(o_T[0], s_T, ar_sw), T2 = tmp(o_T[1], s_T, ar_sw);
        CK(gemm((int)(h * cl), (int)(Du * cu1), (int)cu, P, I1(1), I1(h * cl), Gather{},
                envU(i, j), I1(Du * cu1), I1(1), Gather{}, T1, I1(Du * cu1), I1(1)));
        CK(gemm((int)(cl * cu1), (int)(h1 * Dd), (int)(h * Du), T1, I2((int)cu1, Du * cu1, 1),
                I2((int)Du, cl * Du * cu1, cu1), Gather{}, site_op(i, j), I2((int)Du, D3, D2),
                I2((int)Dd, D, 1), site_gather(i, j, flip), T2, I1(h1 * Dd), I1(1)));
        CK(gemm((int)(cu1 * h1), (int)cl1, (int)(cl * Dd), T2, I1(Dd), I2((int)Dd, cu1 * h1 * Dd, 1),
                Gather{}, envL(i, j), I1(cl1), I1(1), Gather{}, Pout, I1(cl1), I1(1)));
        return hipSuccess;
    }

    // Q_j = step(Q_{j+1}) from the right
    hipError_t row_bwd(int i, int j, Op Q, int flip, Op Qout, const double* lin = nullptr,
                       double* lout = nullptr) {
        bool done = false;
        CK(row_fused(i, j, Q, flip, Qout, false, done, lin, lout));
        if (done) return hipSuccess;
        step_rescaled = false;
        const long long cu = chiU[i][j], cu1 = chiU[i][j + 1], cl = chiL[i][j], cl1 = chiL[i][j + 1];
        const long long Du = Dv[i], Dd = Dv[i + 1], h = Dh[j], h1 = Dh[j + 1];
        Op T1 = tmp(o_T[0], s_T, ar_sw), T2 = tmp(o_T[1], s_T, ar_sw);
        CK(gemm((int)(cl * Dd), (int)(cu1 * h1), (int)cl1, envL(i, j), I1(cl1), I1(1), Gather{}, Q,
                I1(1), I1(cl1), Gather{}, T1, I1(cu1 * h1), I1(1)));
        CK(gemm((int)(h * Du), (int)(cl * cu1), (int)(h1 * Dd), site_op(i, j), I2((int)Du, D3, D2),
                I2((int)Dd, D, 1), site_gather(i, j, flip), T1, I2((int)Dd, 1, cu1 * h1),
                I2((int)cu1, Dd * cu1 * h1, h1), Gather{}, T2, I1(cl * cu1), I1(1)));
        CK(gemm((int)cu, (int)(h * cl), (int)(Du * cu1), envU(i, j), I1(Du * cu1), I1(1), Gather{},
                T2, I2((int)cu1, cl * cu1, 1), I2((int)cl, Du * cl * cu1, cu1), Gather{}, Qout,
                I1(h * cl), I1(1)));
        return hipSuccess;
    }

    // two-row sandwich <U_i| rows i, i+1 |L_{i+1}>, forward step
    // the two-row step as one fused kernel when it fits (done = false: use the GEMMs)
    hipError_t pair_fused(int i, int j, Op X, int f1, int f2, Op Y, bool fwd, bool& done, const double* lin,
                          double* lout) {
        done = false;
        step_rescaled = false;
        if (!fuse_pairs) return hipSuccess;
        PairArgs a;
        a.cu = chiU[i][j]; a.cu1 = chiU[i][j + 1]; a.cl = chiL[i + 1][j]; a.cl1 = chiL[i + 1][j + 1];
        a.Du = Dv[i]; a.Dm = Dv[i + 1]; a.Dq = Dv[i + 2]; a.h = Dh[j]; a.h1 = Dh[j + 1];
        if (!pair_step_fits(a)) return hipSuccess;
        const long long nl = (long long)a.cu * a.h * a.h * a.cl, nr = (long long)a.cu1 * a.h1 * a.h1 * a.cl1;
        const Op U = envU(i, j), L = envL(i + 1, j);
        if (!bounds_ok("pair in", X, (fwd ? nl : nr) - 1, 0) || !bounds_ok("pair out", Y, (fwd ? nr : nl) - 1, 0) ||
            !bounds_ok("pair U", U, (long long)a.cu * a.Du * a.cu1 - 1, 0) ||
            !bounds_ok("pair L", L, (long long)a.cl * a.Dq * a.cl1 - 1, 0))
            return hipErrorInvalidValue;
        if (X.f32 || Y.f32) return hipSuccess;
        done = true;
        if (dry) return hipSuccess;
        a.X = X.p; a.xs = X.bs; a.U = U.p; a.us = U.bs; a.L = L.p; a.ls = L.bs;
        const float* tab = reinterpret_cast<const float*>(buf(o_site32));
        a.site1 = tab + ((long long)i * Lx + j) * 1024;
        a.site2 = tab + ((long long)(i + 1) * Lx + j) * 1024;
        a.sel1 = Scur + (long long)i * Lx + j; a.sel2 = Scur + (long long)(i + 1) * Lx + j; a.sel_bs = N;
        a.flip1 = f1; a.flip2 = f2;
        a.Y = Y.p; a.ys = Y.bs; a.batch = Bcur;
        a.lin = lin; a.lout = lout;
        a.skip = skip_; a.skip_bs = skip_bs_;
        step_rescaled = lout != nullptr;
        const double fl = 2.0 * active_samples() *
                          ((double)a.h * a.h * a.cl * a.Du * a.cu1 * a.cu + (double)a.h * a.cl * a.cu1 * a.h1 * a.Dm * a.h * a.Du +
                           (double)a.cl * a.cu1 * a.h1 * a.h1 * a.Dq * a.h * a.Dm + (double)a.cu1 * a.h1 * a.h1 * a.cl1 * a.cl * a.Dq);
        return timed(PEPS_KC_FUSED, fl, [&] { return launch_pair_step(a, fwd, st_); });
    }

    hipError_t pair_fwd(int i, int j, Op P, int f1, int f2, Op Pout, const double* lin = nullptr,
                        double* lout = nullptr) {
        bool done = false;
        CK(pair_fused(i, j, P, f1, f2, Pout, true, done, lin, lout));
        if (done) return hipSuccess;
        step_rescaled = false;
        const long long cu = chiU[i][j], cu1 = chiU[i][j + 1], cl = chiL[i + 1][j], cl1 = chiL[i + 1][j + 1];
        const long long Du = Dv[i], Dm = Dv[i + 1], Dq = Dv[i + 2], h = Dh[j], h1 = Dh[j + 1];
        Op T1 = tmp(o_T[0], s_T, ar_sw), T2 = tmp(o_T[1], s_T, ar_sw), T3 = tmp(o_T[2], s_T, ar_sw);
        CK(gemm((int)(h * h * cl), (int)(Du * cu1), (int)cu, P, I1(1), I1(h * h * cl), Gather{},
                envU(i, j), I1(Du * cu1), I1(1), Gather{}, T1, I1(Du * cu1), I1(1)));
        CK(gemm((int)(h * cl * cu1), (int)(h1 * Dm), (int)(h * Du), T1, I2((int)cu1, Du * cu1, 1),
                I2((int)Du, h * cl * Du * cu1, cu1), Gather{}, site_op(i, j), I2((int)Du, D3, D2),
                I2((int)Dm, D, 1), site_gather(i, j, f1), T2, I1(h1 * Dm), I1(1)));
        CK(gemm((int)(cl * cu1 * h1), (int)(h1 * Dq), (int)(h * Dm), T2, I1(Dm),
                I2((int)Dm, cl * cu1 * h1 * Dm, 1), Gather{}, site_op(i + 1, j), I2((int)Dm, D3, D2),
                I2((int)Dq, D, 1), site_gather(i + 1, j, f2), T3, I1(h1 * Dq), I1(1)));
        CK(gemm((int)(cu1 * h1 * h1), (int)cl1, (int)(cl * Dq), T3, I1(Dq),
                I2((int)Dq, cu1 * h1 * h1 * Dq, 1), Gather{}, envL(i + 1, j), I1(cl1), I1(1),
                Gather{}, Pout, I1(cl1), I1(1)));
        return hipSuccess;
    }

    hipError_t pair_bwd(int i, int j, Op Q, int f1, int f2, Op Qout, const double* lin = nullptr,
                        double* lout = nullptr) {
        bool done = false;
        CK(pair_fused(i, j, Q, f1, f2, Qout, false, done, lin, lout));
        if (done) return hipSuccess;
        step_rescaled = false;
        const long long cu = chiU[i][j], cu1 = chiU[i][j + 1], cl = chiL[i + 1][j], cl1 = chiL[i + 1][j + 1];
        const long long Du = Dv[i], Dm = Dv[i + 1], Dq = Dv[i + 2], h = Dh[j], h1 = Dh[j + 1];
        Op T1 = tmp(o_T[0], s_T, ar_sw), T2 = tmp(o_T[1], s_T, ar_sw), T3 = tmp(o_T[2], s_T, ar_sw);
        CK(gemm((int)(cl * Dq), (int)(cu1 * h1 * h1), (int)cl1, envL(i + 1, j), I1(cl1), I1(1),
                Gather{}, Q, I1(1), I1(cl1), Gather{}, T1, I1(cu1 * h1 * h1), I1(1)));
        CK(gemm((int)(h * Dm), (int)(cl * cu1 * h1), (int)(h1 * Dq), site_op(i + 1, j),
                I2((int)Dm, D3, D2), I2((int)Dq, D, 1), site_gather(i + 1, j, f2), T1,
                I2((int)Dq, 1, cu1 * h1 * h1), I2((int)(cu1 * h1), Dq * cu1 * h1 * h1, h1), Gather{},
                T2, I1(cl * cu1 * h1), I1(1)));
        CK(gemm((int)(h * Du), (int)(h * cl * cu1), (int)(h1 * Dm), site_op(i, j), I2((int)Du, D3, D2),
                I2((int)Dm, D, 1), site_gather(i, j, f1), T2, I2((int)Dm, 1, cl * cu1 * h1),
                I2((int)(cl * cu1), Dm * cl * cu1 * h1, h1), Gather{}, T3, I1(h * cl * cu1), I1(1)));
        CK(gemm((int)cu, (int)(h * h * cl), (int)(Du * cu1), envU(i, j), I1(Du * cu1), I1(1), Gather{},
                T3, I2((int)cu1, h * cl * cu1, 1), I2((int)(h * cl), Du * h * cl * cu1, cu1), Gather{},
                Qout, I1(h * h * cl), I1(1)));
        return hipSuccess;
    }

    // B_m = dW_i/dT_m (unnormalised), into the per-sample Delta buffer at site m
    hipError_t site_env(int i, int j) {
        const long long cu1 = chiU[i][j + 1], cl = chiL[i][j], cl1 = chiL[i][j + 1];
        const long long cu = chiU[i][j];
        const long long Du = Dv[i], Dd = Dv[i + 1], h = Dh[j], h1 = Dh[j + 1];
        Op T1 = tmp(o_T[0], s_T, ar_sw), T2 = tmp(o_T[1], s_T, ar_sw);
        Op P = (j == 0) ? ones() : op(o_P[j], s_P[j]);
        Op Q = (j + 1 == Lx) ? ones() : op(o_Q[j + 1], s_P[j + 1]);
        CK(gemm((int)(h * cl), (int)(Du * cu1), (int)cu, P, I1(1), I1(h * cl), Gather{},
                envU(i, j), I1(Du * cu1), I1(1), Gather{}, T1, I1(Du * cu1), I1(1)));
        CK(gemm((int)(cl * Dd), (int)(cu1 * h1), (int)cl1, envL(i, j), I1(cl1), I1(1), Gather{}, Q,
                I1(1), I1(cl1), Gather{}, T2, I1(cu1 * h1), I1(1)));
        Op Dl = op(o_delta, (long long)N * D4).at((long long)(i * Lx + j) * D4);
        CK(gemm((int)(h * Du), (int)(h1 * Dd), (int)(cl * cu1), T1, I2((int)Du, cl * Du * cu1, cu1),
                I2((int)cu1, Du * cu1, 1), Gather{}, T2, I2((int)cu1, Dd * cu1 * h1, h1),
                I2((int)Dd, 1, cu1 * h1), Gather{}, Dl, I2((int)Du, D3, D2), I2((int)Dd, D, 1)));
        if (dry) return hipSuccess;
        return launch_grad_site(Dl.p, Dl.bs, Ad, Scur, i * Lx + j, N, D, (int)h, (int)Du, (int)h1,
                                (int)Dd, Bcur, st_);
    }

    int8_t* flags() const { return (int8_t*)buf(o_flags); }
    int8_t* act() const { return (int8_t*)buf(o_act); }
    // the GEMMs and fused steps launched between skip_on(bond) and skip_off() leave out the
    // samples whose two spins on `bond` are equal (no exchange term, so no flipped partial)
    void skip_on(int bond) {
        skip_ = act() + bond;
        skip_bs_ = nbonds;
        skip_bond_ = bond;
    }
    void skip_off() {
        skip_ = nullptr;
        skip_bs_ = 0;
        skip_bond_ = -1;
    }
    // samples a launch works on, for the algorithmic flop counts of the profiling records
    // (the active-bond table is read back only while kernel classes are being timed)
    double active_samples() const {
        if (skip_bond_ < 0 || act_host_.empty()) return (double)Bcur;
        long long n = 0;
        for (int b = 0; b < Bcur; ++b) n += act_host_[(size_t)b * nbonds + skip_bond_] != 0;
        return (double)n;
    }

    // launch `f` between two events when its kernel class is being profiled
    template <class F>
    hipError_t timed(int cls, double flops, F f, double bytes = 0.0) {
        if (dry || quiet || !(ctx->prof_mask & (1u << cls))) return f();
        hipEvent_t ev[2];
        for (int k = 0; k < 2; ++k) {
            if (!ctx->ev_pool.empty()) {
                ev[k] = ctx->ev_pool.back();
                ctx->ev_pool.pop_back();
            } else {
                hipError_t e = hipEventCreate(&ev[k]);
                if (e != hipSuccess) return e;
            }
        }
        hipError_t e = hipEventRecord(ev[0], st_);
        if (e == hipSuccess) e = f();
        if (e == hipSuccess) e = hipEventRecord(ev[1], st_);
        ctx->prof.push_back(ProfRec{ev[0], ev[1], cls, flops, bytes});
        return e;
    }
    // algorithmic flop models (documented in the design notes)
    static double qr_flops(double m, double n) {
        const double r = std::min(m, n);
        return 2.0 * r * r * (std::max(m, n) - r / 3.0);
    }
    // truncation step of one centre: the implicit-Q application forming it (4 tin (mz r - r^2/2)),
    // a thin SVD of the m' x n' centre counted as min(14 m n^2 + 8 n^3, 6 m n^2 + 20 n^3)
    // (m = max, n = min; the Golub-Kahan-Reinsch and R-bidiagonalisation counts), and the
    // carried U_t Sigma_t (2 m' n' t)
    static double svd_flops(double mz, double r, double tin, double p, double tk) {
        const double mp = mz / p, np = p * tin;
        const double a = std::max(mp, np), b = std::min(mp, np);
        const double svd = std::min(14.0 * a * b * b + 8.0 * b * b * b, 6.0 * a * b * b + 20.0 * b * b * b);
        return 4.0 * tin * (mz * r - 0.5 * r * r) + svd + 2.0 * mp * np * tk;
    }

    // ---- one chunk ----
    hipError_t run_chunk(const int8_t* S, int Bn, double* log_abs, int8_t* sign, double* e_loc,
                         int grad_mode, const double* weights, double* out, int8_t* flags_out,
                         bool first_chunk) {
        Bcur = Bn;
        Scur = S;
        hipStream_t st = st_;
        KL(launch_check_configs(S, N, Bn, flags(), st));
        if (want_eloc) KL(launch_bond_active(S, Lx, Ly, act(), nbonds, Bn, st));
        act_host_.clear();
        if (want_eloc && !dry && !quiet && ctx->prof_mask) {
            act_host_.resize((size_t)Bn * nbonds);
            CK(hipMemcpyAsync(act_host_.data(), act(), act_host_.size(), hipMemcpyDeviceToHost, st));
            CK(hipStreamSynchronize(st));
        }
        KL(launch_fill(buf(o_zero), Bn, 0.0, st));
        if (fuse_pairs) KL(launch_site_tables(Ad, reinterpret_cast<float*>(buf(o_site32)), Lx, Ly, D, st));
        KL(launch_fill(buf(o_logU[0]), Bn, 0.0, st));
        for (int i = 0; i + 1 < Ly; ++i) CK(vcU[i] ? vc_step(true, i) : trunc_step(true, i));
        const bool need_L = want_eloc || want_grad;
        if (need_L) {
            KL(launch_fill(buf(o_logL[Ly - 1]), Bn, 0.0, st));
            for (int i = Ly - 1; i >= 1; --i) CK(vcL[i] ? vc_step(false, i) : trunc_step(false, i));
        }
        if (want_grad) KL(launch_fill(buf(o_delta), (long long)Bn * N * D4, 0.0, st));
        const int nH = Ly * (Lx - 1), nV = (Ly - 1) * Lx, nD = (Ly - 1) * (Lx - 1);
        const int row_first = need_L ? 0 : Ly - 1;
        for (int i = row_first; i < Ly; ++i) {
            // forward partials of row i
            KL(launch_fill(buf(o_lP[0]), Bn, 0.0, st));
            for (int j = 0; j < Lx; ++j) {
                Op P = (j == 0) ? ones() : op(o_P[j], s_P[j]);
                Op Po = op(o_P[j + 1], s_P[j + 1]);
                CK(row_fwd(i, j, P, 0, Po, buf(o_lP[j]), buf(o_lP[j + 1])));
                if (!step_rescaled)
                    KL(launch_rescale(Po.p, Po.bs, (int)(chiU[i][j + 1] * Dh[j + 1] * chiL[i][j + 1]),
                                      buf(o_lP[j]), buf(o_lP[j + 1]), Bn, st));
            }
            KL(launch_sandwich_value(buf(o_P[Lx]), s_P[Lx], buf(o_lP[Lx]), buf(o_lnW), buf(o_sgW), Bn, st));
            if (i == Ly - 1) {
                KL(launch_amp_out(buf(o_logU[Ly - 1]), buf(o_lnW), buf(o_sgW), flags(), log_abs,
                                  sign, Bn, st));
            }
            if (!need_L) break;
            // backward partials
            KL(launch_fill(buf(o_lQ[Lx]), Bn, 0.0, st));
            for (int j = Lx - 1; j >= 1; --j) {
                Op Q = (j + 1 == Lx) ? ones() : op(o_Q[j + 1], s_P[j + 1]);
                Op Qo = op(o_Q[j], s_P[j]);
                CK(row_bwd(i, j, Q, 0, Qo, buf(o_lQ[j + 1]), buf(o_lQ[j])));
                if (!step_rescaled)
                    KL(launch_rescale(Qo.p, Qo.bs, (int)(chiU[i][j] * Dh[j] * chiL[i][j]),
                                      buf(o_lQ[j + 1]), buf(o_lQ[j]), Bn, st));
            }
            if (want_eloc) {
                for (int j = 0; j + 1 < Lx; ++j) {
                    Op P = (j == 0) ? ones() : op(o_P[j], s_P[j]);
                    Op Q = (j + 2 == Lx) ? ones() : op(o_Q[j + 2], s_P[j + 2]);
                    Op F = op(o_F, s_F), G = op(o_Gf, s_F);
                    const int bond = i * (Lx - 1) + j;
                    skip_on(bond);
                    CK(row_fwd(i, j, P, 1, F));
                    CK(row_bwd(i, j + 1, Q, 1, G));
                    skip_off();
                    const int n = (int)(chiU[i][j + 1] * Dh[j + 1] * chiL[i][j + 1]);
                    KL(launch_ratio(F.p, F.bs, G.p, G.bs, n, buf(o_lP[j]), buf(o_lQ[j + 2]),
                                    buf(o_lnW), buf(o_sgW), buf(o_ratio), nbonds, bond, Bn, st, act()));
                }
            }
            if (want_grad)
                for (int j = 0; j < Lx; ++j) CK(site_env(i, j));
        }
        if (want_eloc) {
            for (int i = 0; i + 1 < Ly; ++i) {
                KL(launch_fill(buf(o_lP2[0]), Bn, 0.0, st));
                for (int j = 0; j < Lx; ++j) {
                    Op P = (j == 0) ? ones() : op(o_P2[j], s_P2[j]);
                    Op Po = op(o_P2[j + 1], s_P2[j + 1]);
                    CK(pair_fwd(i, j, P, 0, 0, Po, buf(o_lP2[j]), buf(o_lP2[j + 1])));
                    if (!step_rescaled)
                        KL(launch_rescale(Po.p, Po.bs,
                                          (int)(chiU[i][j + 1] * Dh[j + 1] * Dh[j + 1] * chiL[i + 1][j + 1]),
                                          buf(o_lP2[j]), buf(o_lP2[j + 1]), Bn, st));
                }
                KL(launch_sandwich_value(buf(o_P2[Lx]), s_P2[Lx], buf(o_lP2[Lx]), buf(o_lnW2),
                                         buf(o_sgW2), Bn, st));
                KL(launch_fill(buf(o_lQ2[Lx]), Bn, 0.0, st));
                for (int j = Lx - 1; j >= 1; --j) {
                    Op Q = (j + 1 == Lx) ? ones() : op(o_Q2[j + 1], s_P2[j + 1]);
                    Op Qo = op(o_Q2[j], s_P2[j]);
                    CK(pair_bwd(i, j, Q, 0, 0, Qo, buf(o_lQ2[j + 1]), buf(o_lQ2[j])));
                    if (!step_rescaled)
                        KL(launch_rescale(Qo.p, Qo.bs,
                                          (int)(chiU[i][j] * Dh[j] * Dh[j] * chiL[i + 1][j]),
                                          buf(o_lQ2[j + 1]), buf(o_lQ2[j]), Bn, st));
                }
                for (int j = 0; j < Lx; ++j) {
                    Op P = (j == 0) ? ones() : op(o_P2[j], s_P2[j]);
                    Op F = op(o_F, s_F), G = op(o_Gf, s_F);
                    const int n1 = (int)(chiU[i][j + 1] * Dh[j + 1] * Dh[j + 1] * chiL[i + 1][j + 1]);
                    // vertical bond (i,j)-(i+1,j)
                    Op Q1 = (j + 1 == Lx) ? ones() : op(o_Q2[j + 1], s_P2[j + 1]);
                    // flipped partials only for the samples whose two spins differ
                    const int bv = nH + i * Lx + j;
                    skip_on(bv);
                    CK(pair_fwd(i, j, P, 1, 1, F));
                    skip_off();
                    KL(launch_ratio(F.p, F.bs, Q1.p, Q1.bs, n1, buf(o_lP2[j]), buf(o_lQ2[j + 1]),
                                    buf(o_lnW2), buf(o_sgW2), buf(o_ratio), nbonds, bv, Bn, st, act()));
                    if (j + 1 < Lx) {
                        Op Q2 = (j + 2 == Lx) ? ones() : op(o_Q2[j + 2], s_P2[j + 2]);
                        // diagonal (i,j)-(i+1,j+1)
                        const int bd = nH + nV + i * (Lx - 1) + j;
                        skip_on(bd);
                        CK(pair_fwd(i, j, P, 1, 0, F));
                        CK(pair_bwd(i, j + 1, Q2, 0, 1, G));
                        skip_off();
                        KL(launch_ratio(F.p, F.bs, G.p, G.bs, n1, buf(o_lP2[j]), buf(o_lQ2[j + 2]),
                                        buf(o_lnW2), buf(o_sgW2), buf(o_ratio), nbonds, bd, Bn, st, act()));
                        // anti-diagonal (i,j+1)-(i+1,j)
                        const int ba = nH + nV + nD + i * (Lx - 1) + j;
                        skip_on(ba);
                        CK(pair_fwd(i, j, P, 0, 1, F));
                        CK(pair_bwd(i, j + 1, Q2, 1, 0, G));
                        skip_off();
                        KL(launch_ratio(F.p, F.bs, G.p, G.bs, n1, buf(o_lP2[j]), buf(o_lQ2[j + 2]),
                                        buf(o_lnW2), buf(o_sgW2), buf(o_ratio), nbonds, ba, Bn, st, act()));
                    }
                }
            }
            ElocArgs ea;
            ea.S = S; ea.Lx = Lx; ea.Ly = Ly; ea.J1 = lat.J1; ea.J2 = lat.J2;
            ea.ratio = buf(o_ratio); ea.nbonds = nbonds; ea.flags = flags();
            ea.e_loc = e_loc ? e_loc : buf(o_eloc); ea.batch = Bn;
            KL(launch_eloc(ea, st));
        }
        KL(launch_nan_flagged(flags(), log_abs, sign, want_eloc ? (e_loc ? e_loc : buf(o_eloc)) : nullptr,
                              Bn, st));
        if (want_grad) {
            const double* eptr = e_loc ? e_loc : buf(o_eloc);
            if (grad_mode == 1) {
                KL(launch_grad_store(buf(o_delta), S, N, (int)D4, flags(), out, Bn, st));
            } else if (grad_mode == 2) {
                KL(launch_grad_reduce(buf(o_delta), S, N, (int)D4, flags(), weights, !first_chunk, out,
                                      nullptr, buf(o_gws), Bn, st));
            } else if (grad_mode == 3) {
                KL(launch_grad_reduce(buf(o_delta), S, N, (int)D4, flags(), eptr, !first_chunk, buf(o_G1),
                                      buf(o_G0), buf(o_gws), Bn, st));
                KL(launch_energy_sums(eptr, flags(), Bn, buf(o_acc), !first_chunk, st));
            }
        }
        if (flags_out) KL(launch_copy_i8(flags(), flags_out, Bn, st));
        return hipSuccess;
    }

    peps_ctx* ctx;
    peps_lattice lat;
    peps_precision prec;
    Arith ar, ar_sw;
    int Lx, Ly, D, Dc, N;
    long long D2, D3, D4;
    std::vector<int> Dh, Dv;
    std::vector<std::vector<int>> chiU, chiL;
    std::vector<Trunc> tU, tL;
    Layout L;
    int Bc = 0, Bcur = 0, nbonds = 0;
    std::string bounds_msg;
    bool dry = false;
    hipStream_t st_ = nullptr;   // stream this runner enqueues on
    char* base_ = nullptr;       // its workspace
    bool want_eloc = false, want_grad = false;
    const double* Ad = nullptr;
    const int8_t* Scur = nullptr;
    std::vector<size_t> o_envU, o_envL, o_logU, o_logL, o_X, o_tau, o_P, o_Q, o_lP, o_lQ, o_P2, o_Q2,
        o_lP2, o_lQ2;
    std::vector<long long> s_envU, s_envL, s_X, s_tau, s_P, s_P2, s_wy;
    std::vector<size_t> o_wy;
    size_t o_vc = 0, o_wq = 0;
    long long s_vc = 0, s_wq = 0;
    // the blocked QR (matrix-core WY updates) for matrices beyond the register kernels
    static bool use_qrb(int rows, int cols) { return (rows > 512 || cols > 128) && qrb_fits(rows, cols); }
    size_t o_site32 = 0, o_act = 0;
    const int8_t* skip_ = nullptr;
    long long skip_bs_ = 0;
    int skip_bond_ = -1;
    std::vector<int8_t> act_host_;
    bool quiet = false;       // no profiling events (the allocation-free entry point)
    size_t o_R[2], o_G[2], o_Y, o_svd, o_T[3], o_F, o_Gf, o_lnW, o_sgW, o_lnW2, o_sgW2, o_lnWf, o_sgWf,
        o_zero, o_ratio, o_delta, o_flags, o_eloc, o_acc, o_G1, o_G0, o_gws;
    long long s_R, s_Y, s_G, s_svd, s_T, s_F, s_eig = 1;
    size_t o_eig = 0;
    bool fuse_pairs = false;
    int sweeps = 0;                         // variational compression sweeps (0: SVD truncation)
    std::vector<char> vcU, vcL;             // which truncations are variational
    std::vector<long long> vc_eoff;         // offset of cut c's overlap environment
    size_t o_vL = 0, o_vR = 0, o_vZ1 = 0, o_vZ2 = 0, o_vM = 0, o_vRf = 0, o_vW = 0;
    long long s_vE = 0, s_vZ1 = 0, s_vZ2 = 0, s_vM = 0, s_vRf = 0, s_vW = 0;
    bool step_rescaled = false;   // the last sandwich step also applied the max-abs rescale
};

size_t g_lds_cap = 160 * 1024;   // gfx950; replaced by the device attribute at peps_create
size_t Runner::lds_cap_bytes() { return g_lds_cap - 1024; }

}  // namespace

void set_lds_cap(size_t bytes) { g_lds_cap = bytes; }
size_t get_lds_cap() { return g_lds_cap; }

}  // namespace peps

using namespace peps;

static peps_status fail(peps_ctx* c, peps_status s, const char* fmt, ...) {
    char b[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(b, sizeof b, fmt, ap);
    va_end(ap);
    if (c) c->err = b;
    return s;
}

static peps_status check_lat(peps_ctx* c, const peps_lattice* lat) {
    if (!lat) return fail(c, PEPS_ERR_INVALID_ARG, "lattice is NULL");
    if (lat->Lx < 2 || lat->Ly < 2) return fail(c, PEPS_ERR_INVALID_ARG, "Lx and Ly must be >= 2");
    if (lat->D < 1 || lat->Dc < 1) return fail(c, PEPS_ERR_INVALID_ARG, "D and Dc must be >= 1");
    if (lat->Lx > 4096 || lat->Ly > 4096) return fail(c, PEPS_ERR_UNSUPPORTED, "lattice too large");
    if (lat->D > 16) return fail(c, PEPS_ERR_UNSUPPORTED, "D > 16 is not supported");
    if (lat->Dc > 256) return fail(c, PEPS_ERR_UNSUPPORTED, "Dc > 256 is not supported");
    return PEPS_OK;
}

extern "C" {

peps_status peps_create(peps_ctx** ctx, int device) {
    if (!ctx) return PEPS_ERR_INVALID_ARG;
    *ctx = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return PEPS_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return PEPS_ERR_HIP;
    peps_ctx* c = new peps_ctx();
    c->device = device;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
        lds > 0)
        set_lds_cap((size_t)lds);
    if (hipMalloc(&c->ones, kOnes * sizeof(double)) != hipSuccess) {
        delete c;
        return PEPS_ERR_OOM;
    }
    launch_fill(c->ones, kOnes, 1.0, nullptr);
    c->scratch = scratch_address(device);
    if (!c->scratch || hipDeviceSynchronize() != hipSuccess) {
        hipFree(c->ones);
        delete c;
        return PEPS_ERR_HIP;
    }
    const char* tp = getenv("PEPS_TUNE_CACHE");
    if (tp && *tp) peps_tune_load(c, tp);
    *ctx = c;
    return PEPS_OK;
}

peps_status peps_destroy(peps_ctx* c) {
    if (!c) return PEPS_OK;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    drop_graphs(c);
    for (auto s2 : c->job_streams) hipStreamDestroy(s2);
    for (auto e2 : c->job_events) hipEventDestroy(e2);
    if (c->ws) hipFree(c->ws);
    if (c->ones) hipFree(c->ones);
    if (c->mc) hipFree(c->mc);
    if (c->corr) hipFree(c->corr);
    for (auto& r : c->prof) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (auto e : c->ev_pool) hipEventDestroy(e);
    delete c;
    return PEPS_OK;
}

peps_status peps_set_stream(peps_ctx* c, void* s) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    c->stream = (hipStream_t)s;
    return PEPS_OK;
}

peps_status peps_set_truncation(peps_ctx* c, int32_t sweeps) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    if (sweeps < 0 || sweeps > kMaxSweeps) return fail(c, PEPS_ERR_INVALID_ARG, "sweeps must be in [0, %d]", kMaxSweeps);
    c->vc_sweeps = sweeps;
    return PEPS_OK;
}

peps_status peps_set_fused_steps(peps_ctx* c, int32_t enable) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    c->fused_steps = enable != 0;
    return PEPS_OK;
}

peps_status peps_set_workspace_limit(peps_ctx* c, size_t bytes) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    c->ws_limit = bytes;
    return PEPS_OK;
}

const char* peps_last_error(const peps_ctx* c) { return c ? c->err.c_str() : "no context"; }

static size_t default_limit(peps_ctx* c) {
    if (c->ws_limit) return c->ws_limit;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return (size_t)1 << 30;
    return (fr + c->ws_bytes) / 4;
}

peps_status peps_workspace_query(peps_ctx* c, const peps_lattice* lat, int64_t batch,
                                 peps_precision prec, size_t* bytes) {
    if (!c || !bytes) return fail(c, PEPS_ERR_INVALID_ARG, "NULL argument");
    peps_status s = check_lat(c, lat);
    if (s != PEPS_OK) return s;
    Runner r(c, *lat, prec);
    const std::string vm = r.vc_unsupported();
    if (!vm.empty()) return fail(c, PEPS_ERR_UNSUPPORTED, "%s", vm.c_str());
    r.layout((int)std::max<int64_t>(batch, 1), true, true);
    *bytes = r.L.bytes;
    return PEPS_OK;
}

// One evaluation request: a lattice, its tensors and configurations, and the outputs.
struct JobIn {
    peps_lattice lat;
    const double* A;
    const int8_t* S;
    int64_t batch;
    bool want_e;
    int grad_mode;
    const double* weights;
    double* log_abs;
    int8_t* sign;
    double* e_loc;
    double* out;
    int8_t* flags;
};

static peps_status check_job(peps_ctx* c, JobIn& j, peps_precision prec) {
    peps_status st = check_lat(c, &j.lat);
    if (st != PEPS_OK) return st;
    if (prec < PEPS_PREC_F64 || prec > PEPS_PREC_BF16) return fail(c, PEPS_ERR_INVALID_ARG, "bad precision");
    if (j.batch < 0) return fail(c, PEPS_ERR_INVALID_ARG, "batch < 0");
    if (j.grad_mode < 0 || j.grad_mode > 3) return fail(c, PEPS_ERR_INVALID_ARG, "bad grad_mode");
    if (j.batch == 0) return PEPS_OK;
    if (!j.A || !j.S) return fail(c, PEPS_ERR_INVALID_ARG, "A or S is NULL");
    if (j.grad_mode && !j.out) return fail(c, PEPS_ERR_INVALID_ARG, "gradient requested but out is NULL");
    if (j.grad_mode == 2 && !j.weights) return fail(c, PEPS_ERR_INVALID_ARG, "weights is NULL");
    if (j.grad_mode == 3) j.want_e = true;
    return PEPS_OK;
}

// bytes per sample and fixed bytes of one chunk of this job
static void job_sizes(Runner& r, const JobIn& j, size_t* per, size_t* fixed) {
    r.layout(1, j.want_e, j.grad_mode != 0);
    const size_t per1 = r.L.bytes;
    r.layout(2, j.want_e, j.grad_mode != 0);
    *per = r.L.bytes - per1;
    *fixed = per1 > *per ? per1 - *per : 0;
}

static peps_status ensure_ws(peps_ctx* c, size_t bytes) {
    if (bytes <= c->ws_bytes) return PEPS_OK;
    if (c->ws) {
        if (c->stream) hipStreamSynchronize(c->stream);
        else hipDeviceSynchronize();
        drop_graphs(c);
        hipFree(c->ws);
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    if (hipMalloc(&c->ws, bytes) != hipSuccess) {
        c->ws = nullptr;
        return fail(c, PEPS_ERR_OOM, "hipMalloc of %zu bytes failed", bytes);
    }
    c->ws_bytes = bytes;
    return PEPS_OK;
}

// Enqueue every chunk of one job on r.st_ (workspace r.base_, laid out for Bc samples).
static hipError_t enqueue_job(Runner& r, const JobIn& j, int64_t Bc) {
    const int N = j.lat.Lx * j.lat.Ly;
    const long long D4 = (long long)j.lat.D * j.lat.D * j.lat.D * j.lat.D;
    r.Ad = j.A;
    for (int64_t b0 = 0; b0 < j.batch; b0 += Bc) {
        const int Bn = (int)std::min<int64_t>(Bc, j.batch - b0);
        hipError_t e = r.run_chunk(j.S + b0 * N, Bn, j.log_abs ? j.log_abs + b0 : nullptr,
                                   j.sign ? j.sign + b0 : nullptr, j.e_loc ? j.e_loc + b0 : nullptr,
                                   j.grad_mode, j.weights ? j.weights + b0 : nullptr,
                                   (j.grad_mode == 1) ? j.out + b0 * N * 2 * D4 : j.out,
                                   j.flags ? j.flags + b0 : nullptr, b0 == 0);
        if (e != hipSuccess) return e;
    }
    if (j.grad_mode == 3)
        return launch_energy_grad_combine(r.buf(r.o_G1), r.buf(r.o_G0), r.buf(r.o_acc),
                                          (long long)N * 2 * D4, j.out, r.st_);
    return hipSuccess;
}

// noalloc: the workspace is this device's fixed scratch array (chunks sized to fit it);
// no device allocation and no profiling events
static peps_status run_all(peps_ctx* c, const peps_lattice* lat, peps_precision prec, const double* A,
                           const int8_t* S, int64_t batch, bool want_e, int grad_mode,
                           const double* weights, double* log_abs, int8_t* sign, double* e_loc,
                           double* out, int8_t* flags, bool noalloc = false) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    c->err.clear();
    if (!lat) return fail(c, PEPS_ERR_INVALID_ARG, "lattice is NULL");
    JobIn j{*lat, A, S, batch, want_e, grad_mode, weights, log_abs, sign, e_loc, out, flags};
    peps_status st = check_job(c, j, prec);
    if (st != PEPS_OK || batch == 0) return st;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, PEPS_ERR_HIP, "hipSetDevice failed");
    Runner r(c, *lat, prec);
    const std::string vm = r.vc_unsupported();
    if (!vm.empty()) return fail(c, PEPS_ERR_UNSUPPORTED, "%s", vm.c_str());
    size_t per, fixed;
    job_sizes(r, j, &per, &fixed);
    const size_t limit = noalloc ? kScratchBytes : default_limit(c);
    if (per + fixed > limit) {
        if (noalloc)
            return fail(c, PEPS_ERR_INVALID_ARG, "one sample needs %zu bytes > the fixed scratch of %zu bytes",
                        per + fixed, limit);
        return fail(c, PEPS_ERR_OOM, "one sample needs %zu bytes > limit %zu", per + fixed, limit);
    }
    int64_t Bc = std::min<int64_t>(batch, (int64_t)((limit - fixed) / per));
    Bc = std::max<int64_t>(1, std::min<int64_t>(Bc, 1 << 20));
    r.layout((int)Bc, j.want_e, grad_mode != 0);
    if (noalloc) {
        while (r.L.bytes > limit && Bc > 1) {   // alignment padding can add a little
            --Bc;
            r.layout((int)Bc, j.want_e, grad_mode != 0);
        }
        if (r.L.bytes > limit || !c->scratch)
            return fail(c, PEPS_ERR_INVALID_ARG, "workspace of %zu bytes > the fixed scratch of %zu bytes",
                        r.L.bytes, limit);
        r.base_ = c->scratch;
        r.quiet = true;
    } else {
        st = ensure_ws(c, r.L.bytes);
        if (st != PEPS_OK) return st;
        r.base_ = c->ws;
    }
    r.st_ = c->stream;
    hipError_t e = enqueue_job(r, j, Bc);
    if (e != hipSuccess)
        return fail(c, PEPS_ERR_HIP, "HIP error: %s %s", hipGetErrorString(e), r.bounds_msg.c_str());
    return PEPS_OK;
}

// ---------------------------------------------------------------------------
// heterogeneous batches: several lattices in one graph launch
// ---------------------------------------------------------------------------
static std::string jobs_key(const peps_job* jobs, int njobs, peps_precision prec, const void* ws,
                            bool fused, int sweeps) {
    std::string k;
    auto add = [&](const void* p, size_t n) { k.append((const char*)p, n); };
    add(&prec, sizeof prec);
    add(&ws, sizeof ws);
    add(&fused, sizeof fused);    // the captured kernels differ with the step form
    add(&sweeps, sizeof sweeps);  // and with the truncation
    for (int i = 0; i < njobs; ++i) add(&jobs[i], sizeof(peps_job));
    return k;
}

peps_status peps_eval_jobs(peps_ctx* c, const peps_job* jobs, int32_t njobs, peps_precision prec,
                           uint32_t flags) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    c->err.clear();
    if (njobs < 0 || (njobs > 0 && !jobs)) return fail(c, PEPS_ERR_INVALID_ARG, "bad job list");
    if (njobs > 64) return fail(c, PEPS_ERR_UNSUPPORTED, "at most 64 jobs per call");
    std::vector<JobIn> js;
    for (int i = 0; i < njobs; ++i) {
        const peps_job& q = jobs[i];
        JobIn j{q.lat, q.A, q.S, q.batch, q.e_loc != nullptr, q.grad_mode, q.weights, q.log_abs,
                q.sign, q.e_loc, q.out, q.flags};
        peps_status st = check_job(c, j, prec);
        if (st != PEPS_OK) return fail(c, st, "job %d: %s", i, c->err.c_str());
        if (j.batch > 0) js.push_back(j);
    }
    if (js.empty()) return PEPS_OK;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, PEPS_ERR_HIP, "hipSetDevice failed");
    // every job gets its own workspace region, sized for its whole batch in one chunk
    std::vector<Runner> rs;
    rs.reserve(js.size());
    std::vector<size_t> offs;
    size_t total = 0;
    for (auto& j : js) {
        rs.emplace_back(c, j.lat, prec);
        const std::string vm = rs.back().vc_unsupported();
        if (!vm.empty()) return fail(c, PEPS_ERR_UNSUPPORTED, "%s", vm.c_str());
        rs.back().layout((int)std::min<int64_t>(j.batch, 1 << 20), j.want_e, j.grad_mode != 0);
        offs.push_back(total);
        total += (rs.back().L.bytes + 255) / 256 * 256;
    }
    if (total > default_limit(c))
        return fail(c, PEPS_ERR_OOM, "jobs need %zu bytes of workspace > limit %zu", total, default_limit(c));
    peps_status st = ensure_ws(c, total);
    if (st != PEPS_OK) return st;
    const bool use_graph = (flags & PEPS_JOBS_GRAPH) != 0;
    const std::string key = jobs_key(jobs, njobs, prec, c->ws, c->fused_steps, c->vc_sweeps);
    if (use_graph) {
        for (auto& g : c->graphs)
            if (g.key == key) {
                if (hipGraphLaunch(g.exec, c->stream) != hipSuccess) return fail(c, PEPS_ERR_HIP, "hipGraphLaunch failed");
                return PEPS_OK;
            }
    }
    // streams: one per job inside the capture (fork/join), or the context stream
    hipStream_t cs = c->stream;
    if (use_graph) {
        while (c->job_streams.size() < js.size() + 1) {
            hipStream_t s;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(c, PEPS_ERR_HIP, "stream");
            c->job_streams.push_back(s);
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(c, PEPS_ERR_HIP, "event");
            c->job_events.push_back(e);
        }
        cs = c->job_streams[0];
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(c, PEPS_ERR_HIP, "hipStreamBeginCapture failed");
        hipEventRecord(c->job_events[0], cs);
    }
    const uint32_t saved_mask = c->prof_mask;
    if (use_graph) c->prof_mask = 0;     // no timing events inside a captured graph
    hipError_t err = hipSuccess;
    for (size_t i = 0; i < js.size() && err == hipSuccess; ++i) {
        Runner& r = rs[i];
        r.base_ = c->ws + offs[i];
        r.st_ = cs;
        if (use_graph) {
            r.st_ = c->job_streams[i + 1];
            hipStreamWaitEvent(r.st_, c->job_events[0], 0);
        }
        err = enqueue_job(r, js[i], std::min<int64_t>(js[i].batch, 1 << 20));
        if (use_graph && err == hipSuccess) {
            hipEventRecord(c->job_events[i + 1], r.st_);
            hipStreamWaitEvent(cs, c->job_events[i + 1], 0);
        }
    }
    c->prof_mask = saved_mask;
    if (use_graph) {
        hipGraph_t graph = nullptr;
        hipError_t ec = hipStreamEndCapture(cs, &graph);
        if (err != hipSuccess || ec != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return fail(c, PEPS_ERR_HIP, "graph capture failed: %s", hipGetErrorString(err != hipSuccess ? err : ec));
        }
        hipGraphExec_t exec = nullptr;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(graph);
            return fail(c, PEPS_ERR_HIP, "hipGraphInstantiate failed");
        }
        if (c->graphs.size() >= 16) {
            hipGraphExecDestroy(c->graphs.front().exec);
            hipGraphDestroy(c->graphs.front().graph);
            c->graphs.erase(c->graphs.begin());
        }
        c->graphs.push_back(CachedGraph{key, graph, exec});
        if (hipGraphLaunch(exec, c->stream) != hipSuccess) return fail(c, PEPS_ERR_HIP, "hipGraphLaunch failed");
        return PEPS_OK;
    }
    if (err != hipSuccess) return fail(c, PEPS_ERR_HIP, "HIP error: %s", hipGetErrorString(err));
    return PEPS_OK;
}

peps_status peps_autotune(peps_ctx* c, const peps_lattice* lat, peps_precision prec, const double* A,
                          const int8_t* S, int64_t batch, int32_t* tuned) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    double* out = nullptr;
    if (lat && batch > 0 && A && S) {
        const long long D4 = (long long)lat->D * lat->D * lat->D * lat->D;
        if (hipMalloc(&out, sizeof(double) * (2 * (size_t)lat->Lx * lat->Ly * D4 + 2 * (size_t)batch)) != hipSuccess)
            return fail(c, PEPS_ERR_OOM, "autotune scratch");
    }
    c->tune_mode = true;
    c->tuned_now = 0;
    const uint32_t mask = c->prof_mask;
    c->prof_mask = 0;
    const long long nout = lat ? 2LL * lat->Lx * lat->Ly * lat->D * lat->D * lat->D * lat->D : 0;
    peps_status st = run_all(c, lat, prec, A, S, batch, true, 3, nullptr, out ? out + nout : nullptr,
                             nullptr, out ? out + nout + batch : nullptr, out, nullptr);
    c->prof_mask = mask;
    c->tune_mode = false;
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    if (out) hipFree(out);
    if (tuned) *tuned = c->tuned_now;
    if (st == PEPS_OK) {
        const char* path = getenv("PEPS_TUNE_CACHE");
        if (path && *path) peps_tune_save(c, path);
    }
    return st;
}

peps_status peps_tune_save(peps_ctx* c, const char* path) {
    if (!c || !path) return PEPS_ERR_INVALID_ARG;
    std::ofstream f(path);
    if (!f) return fail(c, PEPS_ERR_INVALID_ARG, "cannot write %s", path);
    f << "# peps GEMM tiles: M,N,K,batch,arith,float32-operand-mask tile\n";
    for (auto& kv : c->tune) f << kv.first << " " << kv.second << "\n";
    return PEPS_OK;
}

peps_status peps_tune_load(peps_ctx* c, const char* path) {
    if (!c || !path) return PEPS_ERR_INVALID_ARG;
    std::ifstream f(path);
    if (!f) return fail(c, PEPS_ERR_INVALID_ARG, "cannot read %s", path);
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream ss(line);
        std::string key;
        int tile = 0;
        if (ss >> key >> tile && tile >= 0 && tile <= kGemmTiles) c->tune[key] = tile;   // 0: heuristic
    }
    return PEPS_OK;
}

peps_status peps_profile_enable(peps_ctx* c, uint32_t class_mask) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    for (auto& r : c->prof) {
        c->ev_pool.push_back(r.a);
        c->ev_pool.push_back(r.b);
    }
    c->prof.clear();
    c->prof_mask = class_mask;
    return PEPS_OK;
}

peps_status peps_profile_read(peps_ctx* c, int32_t kernel_class, double* total_ms, int64_t* launches,
                              double* flops) {
    if (!c || kernel_class < 0 || kernel_class >= 32) return PEPS_ERR_INVALID_ARG;
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    double ms = 0.0, fl = 0.0;
    int64_t n = 0;
    for (auto& r : c->prof) {
        if (r.cls != kernel_class) continue;
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(c, PEPS_ERR_HIP, "event timing failed");
        ms += t;
        fl += r.flops;
        ++n;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    if (flops) *flops = fl;
    return PEPS_OK;
}

peps_status peps_profile_read_bytes(peps_ctx* c, int32_t kernel_class, double* bytes) {
    if (!c || !bytes || kernel_class < 0 || kernel_class >= 32) return PEPS_ERR_INVALID_ARG;
    double by = 0.0;
    for (auto& r : c->prof)
        if (r.cls == kernel_class) by += r.bytes;
    *bytes = by;
    return PEPS_OK;
}

peps_status peps_plan_check(const peps_lattice* lat, int64_t batch, int32_t grad_mode,
                            int32_t want_eloc, int32_t sweeps, size_t* bytes) {
    peps_status st = check_lat(nullptr, lat);
    if (st != PEPS_OK) return st;
    if (batch < 1 || grad_mode < 0 || grad_mode > 3 || sweeps < 0 || sweeps > kMaxSweeps)
        return PEPS_ERR_INVALID_ARG;
    peps_ctx dummy;
    dummy.vc_sweeps = sweeps;
    Runner r(&dummy, *lat, PEPS_PREC_F64);
    if (!r.vc_unsupported().empty()) return PEPS_ERR_UNSUPPORTED;
    r.dry = true;
    const bool want_e = want_eloc || grad_mode == 3;
    r.layout((int)std::min<int64_t>(batch, 1 << 20), want_e, grad_mode != 0);
    if (bytes) *bytes = r.L.bytes;
    static const double a0 = 0.0;
    static const int8_t s0 = 0;
    r.Ad = &a0;
    double* dptr = (double*)&a0;
    const int64_t Bn = std::min<int64_t>(batch, 1 << 20);
    hipError_t e = r.run_chunk(&s0, (int)Bn, dptr, (int8_t*)&s0, want_e ? dptr : nullptr, grad_mode,
                               dptr, dptr, nullptr, true);
    return e == hipSuccess ? PEPS_OK : PEPS_ERR_INVALID_ARG;
}

peps_status peps_log_amplitude(peps_ctx* c, const peps_lattice* lat, peps_precision prec,
                               const double* A, const int8_t* S, int64_t batch, double* log_abs,
                               int8_t* sign, int8_t* flags) {
    return run_all(c, lat, prec, A, S, batch, false, 0, nullptr, log_abs, sign, nullptr, nullptr, flags);
}

peps_status peps_local_energy(peps_ctx* c, const peps_lattice* lat, peps_precision prec,
                              const double* A, const int8_t* S, int64_t batch, double* log_abs,
                              int8_t* sign, double* e_loc, int8_t* flags) {
    return run_all(c, lat, prec, A, S, batch, true, 0, nullptr, log_abs, sign, e_loc, nullptr, flags);
}

peps_status peps_log_derivative(peps_ctx* c, const peps_lattice* lat, peps_precision prec,
                                const double* A, const int8_t* S, int64_t batch,
                                const double* weights, double* out, double* log_abs, int8_t* sign,
                                int8_t* flags) {
    if (!out) return fail(c, PEPS_ERR_INVALID_ARG, "out is NULL");
    return run_all(c, lat, prec, A, S, batch, false, weights ? 2 : 1, weights, log_abs, sign, nullptr,
                   out, flags);
}

}  // extern "C"

// Buffers of the sampling and optimisation entry points, carved from one per-context
// allocation that grows on demand: the packed proposals S' [batch][N] with ln|W(S')|,
// sign and flag; moved and packed position per chain; the chains' ln|W|, sign, E(S),
// flags [batch]; the energy sums; the gradient [N][2][D^4]; the moved-chain count.
struct McBuffers {
    int8_t* Sp; double* lap; int8_t* sgp; int8_t* flp; int8_t* moved;
    double* la; int8_t* sg; double* e; int8_t* fl; double* acc; double* grad; int* pos; int* count;
};

// Grows a per-context device buffer to at least `need` bytes (contents not kept).
static peps_status grow_buffer(peps_ctx* c, char** buf, size_t* bytes, size_t need) {
    if (need <= *bytes) return PEPS_OK;
    if (*buf) {
        if (c->stream) hipStreamSynchronize(c->stream);
        else hipDeviceSynchronize();
        hipFree(*buf);
        *buf = nullptr;
        *bytes = 0;
    }
    if (hipMalloc(buf, need) != hipSuccess) {
        *buf = nullptr;
        return fail(c, PEPS_ERR_OOM, "hipMalloc of %zu bytes failed", need);
    }
    *bytes = need;
    return PEPS_OK;
}

static peps_status mc_buffers(peps_ctx* c, int64_t batch, int N, long long ngrad, McBuffers* m) {
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t B = (size_t)batch;
    size_t off[13], need = 0;
    const size_t sz[13] = {B * N, B * 8, B, B, B, B * 8, B, B * 8, B, 16, (size_t)ngrad * 8, B * 4, 4};
    for (int k = 0; k < 13; ++k) {
        off[k] = need;
        need += up(sz[k]);
    }
    peps_status st = grow_buffer(c, &c->mc, &c->mc_bytes, need);
    if (st != PEPS_OK) return st;
    char* b = c->mc;
    *m = McBuffers{reinterpret_cast<int8_t*>(b + off[0]), reinterpret_cast<double*>(b + off[1]),
                   reinterpret_cast<int8_t*>(b + off[2]), reinterpret_cast<int8_t*>(b + off[3]),
                   reinterpret_cast<int8_t*>(b + off[4]), reinterpret_cast<double*>(b + off[5]),
                   reinterpret_cast<int8_t*>(b + off[6]), reinterpret_cast<double*>(b + off[7]),
                   reinterpret_cast<int8_t*>(b + off[8]), reinterpret_cast<double*>(b + off[9]),
                   reinterpret_cast<double*>(b + off[10]), reinterpret_cast<int*>(b + off[11]),
                   reinterpret_cast<int*>(b + off[12])};
    return PEPS_OK;
}

// One Metropolis step of every chain on validated arguments: propose, contract W(S'),
// accept (Sec. II-B steps 1-3).  Only the chains whose drawn bond holds two different
// spins have a proposal to contract; those are packed in chain order first (each
// sample's contraction is independent of the others in the batch, so packing changes no
// result).
static peps_status mc_step(peps_ctx* c, const peps_lattice* lat, peps_precision prec, const double* A,
                           int8_t* S, int64_t batch, const double* u, double* log_abs, int8_t* sign,
                           int8_t* accepted, const McBuffers& m) {
    const int N = lat->Lx * lat->Ly;
    int nmoved = 0;
    hipError_t e = launch_mc_propose(S, u, lat->Lx, lat->Ly, (int)batch, m.moved, m.pos, m.count, m.Sp, &nmoved,
                                     c->stream);
    if (e != hipSuccess) return fail(c, PEPS_ERR_HIP, "HIP error: %s", hipGetErrorString(e));
    if (nmoved < 0 || nmoved > batch) return fail(c, PEPS_ERR_HIP, "moved-chain count out of range");
    if (nmoved > 0) {
        peps_status st = run_all(c, lat, prec, A, m.Sp, nmoved, false, 0, nullptr, m.lap, m.sgp, nullptr, nullptr,
                                 m.flp);
        if (st != PEPS_OK) return st;
    }
    e = launch_mc_accept(S, m.Sp, m.moved, m.pos, u, m.lap, m.sgp, m.flp, log_abs, sign, accepted, N, (int)batch,
                         c->stream);
    if (e != hipSuccess) return fail(c, PEPS_ERR_HIP, "HIP error: %s", hipGetErrorString(e));
    return PEPS_OK;
}

static peps_status check_batch_call(peps_ctx* c, const peps_lattice* lat, int64_t batch) {
    peps_status st = check_lat(c, lat);
    if (st != PEPS_OK) return st;
    if (batch < 0) return fail(c, PEPS_ERR_INVALID_ARG, "batch < 0");
    if (batch > (1LL << 30)) return fail(c, PEPS_ERR_INVALID_ARG, "batch too large");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, PEPS_ERR_HIP, "hipSetDevice failed");
    return PEPS_OK;
}

extern "C" {

peps_status peps_metropolis_step(peps_ctx* c, const peps_lattice* lat, peps_precision prec,
                                 const double* A, int8_t* S, int64_t batch, const double* u,
                                 double* log_abs, int8_t* sign, int8_t* accepted) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    c->err.clear();
    peps_status st = check_batch_call(c, lat, batch);
    if (st != PEPS_OK || batch == 0) return st;
    if (!A || !S || !u || !log_abs || !sign) return fail(c, PEPS_ERR_INVALID_ARG, "NULL argument");
    McBuffers m;
    st = mc_buffers(c, batch, lat->Lx * lat->Ly, 0, &m);
    if (st != PEPS_OK) return st;
    return mc_step(c, lat, prec, A, S, batch, u, log_abs, sign, accepted, m);
}

peps_status peps_go_update(peps_ctx* c, const peps_lattice* lat, double* A, const double* grad,
                           const double* p, double dt) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    c->err.clear();
    peps_status st = check_batch_call(c, lat, 0);
    if (st != PEPS_OK) return st;
    if (!A || !grad || !p) return fail(c, PEPS_ERR_INVALID_ARG, "NULL argument");
    if (!std::isfinite(dt)) return fail(c, PEPS_ERR_INVALID_ARG, "dt is not finite");
    const long long n = (long long)lat->Lx * lat->Ly * 2 * lat->D * lat->D * lat->D * lat->D;
    hipError_t e = launch_go_update(A, grad, p, dt, n, c->stream);
    if (e != hipSuccess) return fail(c, PEPS_ERR_HIP, "HIP error: %s", hipGetErrorString(e));
    return PEPS_OK;
}

peps_status peps_vmc_step(peps_ctx* c, const peps_lattice* lat, peps_precision prec, double* A, int8_t* S,
                          int64_t batch, int32_t n_mc, const double* u, const double* p, double dt,
                          double* energy, double* grad) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    c->err.clear();
    peps_status st = check_batch_call(c, lat, batch);
    if (st != PEPS_OK) return st;
    if (batch == 0) return fail(c, PEPS_ERR_INVALID_ARG, "batch is 0: no samples to estimate from");
    if (n_mc < 0) return fail(c, PEPS_ERR_INVALID_ARG, "n_mc < 0");
    if (!A || !S || !p || (n_mc > 0 && !u)) return fail(c, PEPS_ERR_INVALID_ARG, "NULL argument");
    if (!std::isfinite(dt)) return fail(c, PEPS_ERR_INVALID_ARG, "dt is not finite");
    const int N = lat->Lx * lat->Ly;
    const long long ng = (long long)N * 2 * lat->D * lat->D * lat->D * lat->D;
    McBuffers m;
    st = mc_buffers(c, batch, N, grad ? 0 : ng, &m);
    if (st != PEPS_OK) return st;
    double* g = grad ? grad : m.grad;
    // ln|W| of the chains under the current tensors, then the Metropolis steps
    st = run_all(c, lat, prec, A, S, batch, false, 0, nullptr, m.la, m.sg, nullptr, nullptr, m.fl);
    if (st != PEPS_OK) return st;
    for (int t = 0; t < n_mc; ++t) {
        st = mc_step(c, lat, prec, A, S, batch, u + 2LL * batch * t, m.la, m.sg, nullptr, m);
        if (st != PEPS_OK) return st;
    }
    // Eqs. (3) and (5) over the chains, then the GO update of A
    st = run_all(c, lat, prec, A, S, batch, true, 3, nullptr, m.la, m.sg, m.e, g, m.fl);
    if (st != PEPS_OK) return st;
    hipError_t e = hipSuccess;
    if (energy) {
        e = launch_energy_sums(m.e, m.fl, (int)batch, m.acc, 0, c->stream);
        if (e == hipSuccess) e = launch_energy_mean(m.acc, energy, c->stream);
    }
    if (e == hipSuccess) e = launch_go_update(A, g, p, dt, ng, c->stream);
    if (e != hipSuccess) return fail(c, PEPS_ERR_HIP, "HIP error: %s", hipGetErrorString(e));
    return PEPS_OK;
}

peps_status peps_pair_correlations(peps_ctx* c, const peps_lattice* lat, peps_precision prec, const double* A,
                                   const int8_t* S, int64_t batch, int32_t npairs, const int32_t* pairs,
                                   double* means, double* per_sample, int8_t* flags) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    c->err.clear();
    peps_status st = check_batch_call(c, lat, batch);
    if (st != PEPS_OK) return st;
    if (npairs < 1) return fail(c, PEPS_ERR_INVALID_ARG, "npairs < 1");
    if (!A || !S || !pairs) return fail(c, PEPS_ERR_INVALID_ARG, "NULL argument");
    if (batch * (int64_t)npairs > (1LL << 30)) return fail(c, PEPS_ERR_INVALID_ARG, "batch * npairs too large");
    const int N = lat->Lx * lat->Ly, P = npairs;
    // the site indices are checked on the host before any kernel reads them
    std::vector<int32_t> hp(2 * (size_t)P);
    if (hipStreamSynchronize(c->stream) != hipSuccess || hipMemcpy(hp.data(), pairs, hp.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, PEPS_ERR_HIP, "cannot read the pair list");
    for (int32_t x : hp)
        if (x < 0 || x >= N) return fail(c, PEPS_ERR_INVALID_ARG, "pair site %d outside [0, %d)", x, N);
    if (batch == 0) return PEPS_OK;
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t B = (size_t)batch, BP = B * P;
    const size_t sz[10] = {BP * N, BP * 4, 256, BP * 8, BP, BP, B * 8, B, B, per_sample ? 0 : BP * 8};
    size_t off[10], need = 0;
    for (int k = 0; k < 10; ++k) {
        off[k] = need;
        need += up(sz[k]);
    }
    st = grow_buffer(c, &c->corr, &c->corr_bytes, need);
    if (st != PEPS_OK) return st;
    char* base = c->corr;
    int8_t* Sx = reinterpret_cast<int8_t*>(base + off[0]);
    int* slot = reinterpret_cast<int*>(base + off[1]);
    int* count = reinterpret_cast<int*>(base + off[2]);
    double* lax = reinterpret_cast<double*>(base + off[3]);
    int8_t* sgx = reinterpret_cast<int8_t*>(base + off[4]);
    int8_t* flx = reinterpret_cast<int8_t*>(base + off[5]);
    double* la = reinterpret_cast<double*>(base + off[6]);
    int8_t* sg = reinterpret_cast<int8_t*>(base + off[7]);
    int8_t* fl = reinterpret_cast<int8_t*>(base + off[8]);
    double* v = per_sample ? per_sample : reinterpret_cast<double*>(base + off[9]);
    st = run_all(c, lat, prec, A, S, batch, false, 0, nullptr, la, sg, nullptr, nullptr, fl);
    if (st != PEPS_OK) return st;
    hipError_t e = hipMemsetAsync(count, 0, sizeof(int), c->stream);
    if (e == hipSuccess) e = launch_corr_pack(S, pairs, P, N, (int)batch, Sx, slot, count, c->stream);
    int hcount = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hcount, count, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, PEPS_ERR_HIP, "HIP error: %s", hipGetErrorString(e));
    if (hcount < 0 || (size_t)hcount > BP) return fail(c, PEPS_ERR_HIP, "exchanged-configuration count out of range");
    if (hcount > 0) {
        st = run_all(c, lat, prec, A, Sx, hcount, false, 0, nullptr, lax, sgx, nullptr, nullptr, flx);
        if (st != PEPS_OK) return st;
    }
    int8_t* fo = flags ? flags : fl;
    e = launch_corr_values(S, pairs, P, N, (int)batch, la, sg, fl, slot, lax, sgx, flx, v, fo, c->stream);
    if (e == hipSuccess && means) e = launch_corr_means(v, fo, P, (int)batch, means, c->stream);
    if (e != hipSuccess) return fail(c, PEPS_ERR_HIP, "HIP error: %s", hipGetErrorString(e));
    return PEPS_OK;
}

peps_status peps_structure_factor(peps_ctx* c, const peps_lattice* lat, int32_t nsites, const int32_t* sites,
                                  const double* corr, int32_t nk, const double* k, double* out) {
    if (!c) return PEPS_ERR_INVALID_ARG;
    c->err.clear();
    peps_status st = check_batch_call(c, lat, 0);
    if (st != PEPS_OK) return st;
    if (nsites < 1 || nk < 0) return fail(c, PEPS_ERR_INVALID_ARG, "nsites < 1 or nk < 0");
    if (nk == 0) return PEPS_OK;
    if (!sites || !corr || !k || !out) return fail(c, PEPS_ERR_INVALID_ARG, "NULL argument");
    const int N = lat->Lx * lat->Ly;
    std::vector<int32_t> hs((size_t)nsites);
    if (hipStreamSynchronize(c->stream) != hipSuccess || hipMemcpy(hs.data(), sites, hs.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, PEPS_ERR_HIP, "cannot read the site list");
    for (int32_t x : hs)
        if (x < 0 || x >= N) return fail(c, PEPS_ERR_INVALID_ARG, "site %d outside [0, %d)", x, N);
    hipError_t e = launch_structure_factor(lat->Lx, nsites, sites, corr, nk, k, out, c->stream);
    if (e != hipSuccess) return fail(c, PEPS_ERR_HIP, "HIP error: %s", hipGetErrorString(e));
    return PEPS_OK;
}

peps_status peps_evaluate(peps_ctx* c, const peps_lattice* lat, peps_precision prec, const double* A,
                          const int8_t* S, int64_t batch, int32_t grad_mode, const double* weights,
                          double* log_abs, int8_t* sign, double* e_loc, double* out, int8_t* flags) {
    return run_all(c, lat, prec, A, S, batch, e_loc != nullptr, grad_mode, weights, log_abs, sign, e_loc,
                   out, flags);
}

peps_status peps_evaluate_noalloc(peps_ctx* c, const peps_lattice* lat, peps_precision prec, const double* A,
                                  const int8_t* S, int64_t batch, int32_t grad_mode, const double* weights,
                                  double* log_abs, int8_t* sign, double* e_loc, double* out, int8_t* flags) {
    return run_all(c, lat, prec, A, S, batch, e_loc != nullptr, grad_mode, weights, log_abs, sign, e_loc,
                   out, flags, true);
}

size_t peps_noalloc_scratch_bytes(void) { return kScratchBytes; }

}  // extern "C"
