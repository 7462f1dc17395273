// Host side of the library: argument checks, workspace planning, the batched
// inexact-ALM loop over the DFC blocks, the column-projection combine, and the
// extern "C" entry points declared in include/lrr.h.
//
// ALM for one block (observations X, dictionary A = M), from the augmented
// Lagrangian of the split Z = J of Eq. (2):
//   J  = SVT_{1/mu}(Z + Y2/mu)
//   Z  = (I + A^T A)^{-1} (A^T (X - E + Y1/mu) + J - Y2/mu)
//   E  = column l2 shrinkage of X - A Z + Y1/mu by lam/mu
//   Y1 += mu (X - A Z - E),  Y2 += mu (Z - J),  mu = min(rho mu, mu_max)
//   stop when both residual max-norms are below tol.
// The Z-step is evaluated in push-through form: with P = X - E + Y1/mu and
// Q = J - Y2/mu,  V = (I + A A^T)^{-1} (P - A Q),  Z = Q + A^T V  and
// X - A Z + Y1/mu = E + V, so the m x m inverse is the only factorisation and no
// product A Z is needed.
//
// All t blocks run in the same launches: the state of block b is the column
// range [boff[b], boff[b+1]) of column-concatenated matrices, the dictionary
// products cover all columns at once, and the per-block steps (Gram, eigensolve,
// reconstruction) are batched launches with one descriptor per block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <initializer_list>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "../../include/lrr.h"
#include "../../include/lrr_diag.h"
#include "host.hpp"

// Opt-in per-kernel timing with HIP events on the solve's stream.
struct LrrProf {
    struct Entry {
        std::string name;
        double ms = 0.0;
        long long launches = 0;
        double flops = 0.0, bytes = 0.0;
    };
    struct Pending {
        int idx;
        hipEvent_t a, b;
        double flops, bytes;
    };
    bool on = false;
    std::string filter;          // time only kernels whose name starts with this (empty: all)
    std::vector<Entry> entries;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;

    int index(const char* name) {
        for (size_t i = 0; i < entries.size(); ++i)
            if (entries[i].name == name) return (int)i;
        entries.push_back(Entry{name});
        return (int)entries.size() - 1;
    }
    hipEvent_t get() {
        if (pool.empty()) {
            hipEvent_t e;
            LRR_HIP(hipEventCreate(&e));
            return e;
        }
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    bool wants(const char* name) const {
        return on && (filter.empty() || std::strncmp(name, filter.c_str(), filter.size()) == 0);
    }
    template <class F>
    void run(hipStream_t s, const char* name, double flops, double bytes, F&& f) {
        if (!wants(name)) { f(); return; }
        hipEvent_t a = get(), b = get();
        LRR_HIP(hipEventRecord(a, s));
        f();
        LRR_HIP(hipEventRecord(b, s));
        pending.push_back(Pending{index(name), a, b, flops, bytes});
    }
    // call after the stream has been synchronised
    void flush() {
        for (const Pending& p : pending) {
            float ms = 0.f;
            LRR_HIP(hipEventElapsedTime(&ms, p.a, p.b));
            Entry& e = entries[p.idx];
            e.ms += ms;
            e.launches += 1;
            e.flops += p.flops;
            e.bytes += p.bytes;
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
    void release() {
        for (const Pending& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pending.clear();
        pool.clear();
    }
};

struct Tape;   // record of the last dfc_lrr_solve for dfc_lrr_backward

// One line of the autotuner's schedule table.
struct lrr_ctx {
    LrrProf prof;
    int device = 0;
    std::string err;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    void* pinned = nullptr;      // small pinned host area for flag read-back
    size_t pinned_bytes = 0;
    int* dflag = nullptr;        // device flag for the input check
    unsigned long long* dwork = nullptr;   // operation counters of the Jacobi kernels
    Tape* tape = nullptr;
    hipStream_t capture = nullptr;         // private stream for graph capture
    void* seg_ws = nullptr;                // workspace of lrr_segment (kept apart from the solver's)
    void* io_ws = nullptr;                 // FP64 copies of FP32 arguments (opts.io_type)
    size_t io_bytes = 0;
    size_t seg_bytes = 0;
    std::vector<lrr::host::TuneEntry> tune;           // schedule table (lrr_tune_load)
};

namespace {

using lrr::BlockState;
using lrr::DevIter;
using lrr::EigDesc;
using lrr::GemmDesc;
using lrr::SvtDesc;
using lrr::RefDesc;

thread_local std::string g_last_error;

lrr_status fail(lrr_ctx* ctx, lrr_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    g_last_error = msg;
    return st;
}

// bump allocator over the workspace (256-byte aligned slices)
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += sizeof(T) * std::max<size_t>(count, 1);
        return p;
    }
};

// Arithmetic (GemmMode) of each large product of an iteration, and whether the
// product is carried in difference form (reduced precision only).
struct ProductModes {
    int MQ = 0;         // M Q of the Z-step
    int MtV = 0;        // M^T V
    int comb = 0;       // U1^T J and U1 H of the combine
    bool dMQ = false;   // M Q carried as a sum of M dQ
};

struct Plan {
    int m = 0, n = 0, ncols = 0, t = 0;
    int bs = 16;                 // Jacobi block width
    std::vector<int> boff;       // t + 1 column offsets
    std::vector<int> L;          // padded Gram order per block
    int maxL = 0, maxl = 0;
    int n_iter = 0;
    ProductModes pm;             // arithmetic of each large product
    // coordinates of the n-row iterates (Z, J, Y2 and their temporaries): n rows,
    // or nr <= min(m, n) coefficients on an orthonormal basis Qm of range(M^T)
    bool reduced = false;
    int nrb = 0;                 // rows the layout reserves (n, or min(m, n))
    int nr = 0;                  // rows in use (n, or the numerical rank of M)
    int Lm = 0, bq = 16;         // padded order / Jacobi block of the M M^T eigensolve
    // every block its own dictionary (the observations C_b, Section 2.2 footnote):
    // the iterates of block b use rows [0, l_b) of maxl rows, K is per block
    bool local = false;
    // Z-step in the literal form: the n x n inverse of I + A^T A (full
    // coordinates, FP64 products) instead of the m x m one of I + A A^T
    bool literal = false;
    int ks = 0;                  // order of the factored matrix (m, or n when literal)
};

struct Buffers {
    double *X, *Z, *J, *Y2, *Y, *Q, *MtV, *E, *Y1, *T, *V;
    double *K, *Lb, *Linv, *Tb, *Dinv;
    double* F1;                  // literal form: (I + A^T A)^{-1} A^T (n x m); K then holds K^{-1} - I
    double *colsq, *mu_sched;
    double *Dn, *MQacc;          // difference form of M Q only
    // reduced coordinates only
    double *Qm, *Qtmp, *Mr, *R2r, *R2full, *Ur, *Gb, *Wq, *Rq, *lamq, *scaleq, *Gq, *Tq;
    int *protq, *loq, *stq, *runq, *idxq, *expand;
    unsigned long long* r2nrm;
    EigDesc* eq;
    GemmDesc *g_red, *g_exp;
    int *colblk, *boff, *perm;
    int *active, *svt_run, *eig_run, *iters, *rank, *eigst, *n_active, *eig_any, *flag;
    std::vector<int*> prot;
    double *res1, *res2, *eigscale;
    unsigned long long *r1max, *r2max;
    double *colr1, *colr2;       // per-column residual maxima (reduced per block without atomics)
    DevIter* it;
    std::vector<double*> Bm, Wm, Wg, Pm, Rm, lam, h, TX, SG, Eb, XE, Bq;
    std::vector<int*> lo;
    int *warm, *ref_run, *ref_unres, *ref_cont, *ref_clean, *ref_nsskip, *passes;
    unsigned long long* ref_rdev;
    int *need_all, *sched_all;   // targeted Jacobi rounds: check marks and round schedules, all blocks
    int *jac_offs, *jac_brounds; // persistent eigensolve: per-block item prefixes, planned rounds
    lrr::JacCtl* jac_ctl;
    double* locut;
    double *ref_eprev, *ref_scale;
    unsigned long long* ref_emax;
    GemmDesc *g_gram, *g_refT, *g_refSG, *g_refXE, *g_orthG, *g_Bq, *g_P, *g_J, *g_MQ, *g_MQa, *g_KV, *g_MtV, *g_U, *g_H,
        *g_Z, *g_spd, *g_KK, *g_F1T, *g_F2Q, *g_AZ, *g_F1;
    RefDesc* ref;
    EigDesc* eig;
    SvtDesc* svt;
    // combine
    double *U, *H;
};

constexpr int kRefSteps = 10;  // cap on refinement steps per thresholding step
constexpr double kPreWarm = 0.5;   // ||Y||_F / tau above which a block is decomposed ahead of time
constexpr int kBlindSteps = 3;   // refinement steps launched before the host reads the flags
constexpr int kMaxTargeted = 60;   // cap on targeted Jacobi passes per eigensolve
constexpr int kAnchorEvery = 16;   // FP64 re-anchoring period of the carried product M Q

int jacobi_bs(int maxl, int requested) {
    if (requested == 16 || requested == 32) return requested;
    return 16;
}

int round_up(int x, int a) { return ((x + a - 1) / a) * a; }

// Lay out every buffer; with a null base only the size is computed.
size_t layout(const Plan& p, char* base, Buffers& b, int with_combine, bool need_X) {
    Arena a{base, 0};
    const size_t m = p.m, c = p.ncols, t = p.t;
    const size_t n = p.nrb;      // rows of the iterates
    const size_t nfull = p.n;
    b.X = a.take<double>(m * c);
    b.Z = a.take<double>(n * c);
    b.J = a.take<double>(n * c);
    b.Y2 = a.take<double>(n * c);
    b.Y = a.take<double>(n * c);
    b.Q = a.take<double>(n * c);
    b.MtV = a.take<double>(n * c);
    b.E = a.take<double>(m * c);
    b.Y1 = a.take<double>(m * c);
    b.T = a.take<double>(m * c);
    b.V = a.take<double>(m * c);
    const size_t ks = p.ks;      // order of the factored matrix
    b.K = a.take<double>((p.local ? t : 1) * ks * ks);   // K^{-1}, one per block in local mode
    b.Lb = a.take<double>(ks * ks);
    b.Linv = a.take<double>(ks * ks);
    b.Tb = a.take<double>(ks * ks);
    b.Dinv = a.take<double>(ks * 32);
    b.F1 = p.literal ? a.take<double>(nfull * m) : nullptr;
    b.Dn = p.pm.dMQ ? a.take<double>(n * c) : nullptr;
    b.MQacc = p.pm.dMQ ? a.take<double>(m * c) : nullptr;
    b.colsq = a.take<double>(c);
    b.mu_sched = a.take<double>(p.n_iter + 2);
    b.colblk = a.take<int>(c);
    b.boff = a.take<int>(t + 1);
    b.perm = a.take<int>(c);
    b.active = a.take<int>(t);
    b.svt_run = a.take<int>(t);
    b.eig_run = a.take<int>(t);
    b.iters = a.take<int>(t);
    b.rank = a.take<int>(t);
    b.eigst = a.take<int>(2 * t);
    b.n_active = a.take<int>(1);
    b.eig_any = a.take<int>(1);
    b.flag = a.take<int>(1);
    b.res1 = a.take<double>(t);
    b.res2 = a.take<double>(t);
    b.eigscale = a.take<double>(t);
    b.r1max = a.take<unsigned long long>(t);
    b.r2max = a.take<unsigned long long>(t);
    b.colr1 = a.take<double>(c);
    b.colr2 = a.take<double>(c);
    b.it = a.take<DevIter>(1);
    for (auto* v : {&b.Bm, &b.Wm, &b.Wg, &b.Pm, &b.Rm, &b.lam, &b.h, &b.TX, &b.SG, &b.Eb, &b.XE, &b.Bq})
        v->assign(t, nullptr);
    b.prot.assign(t, nullptr);
    b.lo.assign(t, nullptr);
    for (size_t i = 0; i < t; ++i) {
        const size_t L = p.L[i];
        b.Bm[i] = a.take<double>(L * L);
        b.TX[i] = a.take<double>(2 * L * L);
        b.Wm[i] = b.TX[i] + L * L;          // eigenvector estimate X = right half of [T | X]
        b.SG[i] = a.take<double>(2 * L * L);
        b.Eb[i] = a.take<double>(L * L);
        b.XE[i] = a.take<double>(L * L);
        b.Bq[i] = a.take<double>(L * L);
        b.Wg[i] = a.take<double>(L * L);
        b.Pm[i] = a.take<double>(L * L);
        b.Rm[i] = a.take<double>(L * 2 * p.bs);
        b.lam[i] = a.take<double>(L);
        b.h[i] = a.take<double>(L);
        b.lo[i] = a.take<int>(L);
        b.prot[i] = a.take<int>(L / (2 * p.bs) + 1);
    }
    {
        size_t nneed = 0, nsched = 0;
        for (size_t i = 0; i < t; ++i) {
            const size_t nb = p.L[i] / p.bs;
            nneed += nb * nb;
            nsched += (nb - 1) * (nb / 2);
        }
        b.need_all = a.take<int>(nneed);
        b.sched_all = a.take<int>(nsched);
    }
    b.jac_offs = a.take<int>(3 * (t + 1));
    b.jac_brounds = a.take<int>(t);
    b.jac_ctl = a.take<lrr::JacCtl>(1);
    b.warm = a.take<int>(t);
    b.passes = a.take<int>(t);
    b.locut = a.take<double>(t);
    b.ref_run = a.take<int>(t);
    b.ref_cont = a.take<int>(t);
    b.ref_clean = a.take<int>(t);
    b.ref_nsskip = a.take<int>(t);
    b.ref_rdev = a.take<unsigned long long>(t);
    b.ref_unres = a.take<int>(t);
    b.ref_eprev = a.take<double>(t);
    b.ref_scale = a.take<double>(t);
    b.ref_emax = a.take<unsigned long long>(t);
    b.g_gram = a.take<GemmDesc>(t);
    b.g_refT = a.take<GemmDesc>(t);
    b.g_refSG = a.take<GemmDesc>(t);
    b.g_refXE = a.take<GemmDesc>(t);
    b.g_orthG = a.take<GemmDesc>(t);
    b.g_Bq = a.take<GemmDesc>(t);
    b.ref = a.take<RefDesc>(t);
    b.g_P = a.take<GemmDesc>(t);
    b.g_J = a.take<GemmDesc>(t);
    b.g_MQ = a.take<GemmDesc>(t);
    b.g_MQa = a.take<GemmDesc>(t);
    b.g_KV = a.take<GemmDesc>(t);
    b.g_MtV = a.take<GemmDesc>(t);

    b.g_U = a.take<GemmDesc>(1);
    b.g_H = a.take<GemmDesc>(1);
    b.g_Z = a.take<GemmDesc>(1);
    b.g_KK = a.take<GemmDesc>(p.local ? t : 1);
    b.g_spd = a.take<GemmDesc>(lrr::spd_inverse_desc_count(p.ks));
    b.g_F1T = a.take<GemmDesc>(t);
    b.g_F2Q = a.take<GemmDesc>(t);
    b.g_AZ = a.take<GemmDesc>(t);
    b.g_F1 = a.take<GemmDesc>(1);
    b.eig = a.take<EigDesc>(t);
    b.svt = a.take<SvtDesc>(t);
    if (with_combine) {
        b.U = a.take<double>(nfull * p.L[0]);
        b.H = a.take<double>((size_t)p.L[0] * c);
    } else {
        b.U = b.H = nullptr;
    }
    if (p.reduced) {
        const size_t Lm = p.Lm;
        b.Qm = a.take<double>(nfull * n);
        b.Qtmp = a.take<double>(nfull * n);
        b.Mr = a.take<double>(m * n);
        b.R2r = a.take<double>(n * c);
        b.R2full = a.take<double>(nfull * c);
        b.Ur = with_combine ? a.take<double>(n * p.L[0]) : nullptr;
        b.Gb = a.take<double>(Lm * Lm);
        b.Wq = a.take<double>(Lm * Lm);
        b.Rq = a.take<double>(Lm * 2 * p.bq);
        b.lamq = a.take<double>(Lm);
        b.scaleq = a.take<double>(1);
        b.Gq = a.take<double>(n * n);
        b.Tq = a.take<double>(n * n);
        b.protq = a.take<int>(Lm / (2 * p.bq) + 1);
        b.loq = a.take<int>(Lm);
        b.stq = a.take<int>(2);
        b.runq = a.take<int>(1);
        b.idxq = a.take<int>(m);
        b.expand = a.take<int>(t);
        b.r2nrm = a.take<unsigned long long>(t);
        b.eq = a.take<EigDesc>(1);
        b.g_red = a.take<GemmDesc>(5);
        b.g_exp = a.take<GemmDesc>(t);
    } else {
        b.Qm = b.Qtmp = b.Mr = b.R2r = b.R2full = b.Ur = b.Gb = b.Wq = b.Rq = b.lamq = b.scaleq = nullptr;
        b.Gq = b.Tq = nullptr;
        b.protq = b.loq = b.stq = b.runq = b.idxq = b.expand = nullptr;
        b.r2nrm = nullptr;
        b.eq = nullptr;
        b.g_red = b.g_exp = nullptr;
    }
    (void)need_X;
    return a.off + 256;
}

// Arithmetic of the large products (Gram, reconstruction, dictionary
// products, combine) for a precision form.  The Cholesky factorisation, the
// eigen-decomposition of the Gram matrix and every residual stay in FP64.
int gemm_mode(int precision) {
    if (precision == LRR_FP32) return lrr::kGemmFP32;
    if (precision == LRR_MIXED_BF16) return lrr::kGemmBF16X3;
    return lrr::kGemmFP64;
}

// Products of each precision form.  Only the two dictionary products of the
// Z-step (M Q and M^T V, 4 m n l of the iteration's flops) and the last two
// products of the combine run in reduced precision.  FP64 stays where rounding
// is amplified:
//  - the Gram matrix Y^T Y, whose eigenvalues are thresholded at tau^2, far
//    below FP32 resolution once mu is large;
//  - the reconstruction J = Y P, whose rounding error lands in the directions
//    the thresholding has just removed, where the multipliers accumulate it;
//  - K^{-1} T, whose entries cancel heavily when M is ill-conditioned;
//  - the combine basis U1 = Y W diag(1/sigma), which divides by sigma ~ tau;
//  - the Cholesky factorisation, the eigen-decomposition and every residual.
// M Q, whose operand does not vanish at convergence, is carried as a sum of
// products of the changes of Q, so that its rounding error vanishes as the
// iteration converges; M^T V acts on V -> 0 and is formed directly.
ProductModes product_modes(int precision) {
    ProductModes m;
    const int g = gemm_mode(precision);
    if (g == lrr::kGemmFP64) return m;
    m.MQ = g;
    m.MtV = g;
    m.comb = g;
    m.dMQ = true;
    return m;
}

bool opts_valid(const lrr_opts& o, std::string& why) {
    if (o.precision != LRR_FP64 && o.precision != LRR_FP32 && o.precision != LRR_MIXED_BF16) {
        why = "unknown precision";
        return false;
    }
    if (o.solve_form < 0 || o.solve_form > 2) { why = "unknown solve_form"; return false; }
    if (!(o.mu0 > 0) || !std::isfinite(o.mu0)) { why = "mu0 must be positive"; return false; }
    if (!(o.rho >= 1.0) || !std::isfinite(o.rho)) { why = "rho must be >= 1"; return false; }
    if (!(o.mu_max >= o.mu0) || !std::isfinite(o.mu_max)) { why = "mu_max must be >= mu0"; return false; }
    if (!(o.tol > 0)) { why = "tol must be positive"; return false; }
    if (o.max_iter <= 0 && o.fixed_iters <= 0) { why = "max_iter must be positive"; return false; }
    if (o.fixed_iters < 0) { why = "fixed_iters must be >= 0"; return false; }
    if (o.check_every < 0 || o.max_sweeps < 0 || o.checkpoint_every < 0) {
        why = "negative count"; return false;
    }
    if (o.eig_block != 0 && o.eig_block != 16 && o.eig_block != 32) { why = "eig_block must be 0, 16 or 32"; return false; }
    if (o.use_graph < 0 || o.use_graph > 3) { why = "use_graph must be 0, 1, 2 or 3"; return false; }
    if (o.coords < 0 || o.coords > 2) { why = "unknown coords"; return false; }
    if (o.tune != 0 && o.tune != 1) { why = "tune must be 0 or 1"; return false; }
    if (o.solve_form == LRR_SOLVE_LITERAL) {
        if (o.precision != LRR_FP64) { why = "the literal solve form runs in FP64 only"; return false; }
        if (o.coords == LRR_COORDS_REDUCED) { why = "the literal solve form needs full coordinates"; return false; }
        if (o.save_for_backward) { why = "the reverse mode records the push-through solve form"; return false; }
    }
    if (o.io_type != LRR_IO_FP64 && o.io_type != LRR_IO_FP32) { why = "unknown io_type"; return false; }
    if (o.io_type == LRR_IO_FP32 && o.save_for_backward) {
        why = "the reverse mode takes FP64 buffers (io_type must be LRR_IO_FP64 with save_for_backward)";
        return false;
    }
    for (int r : o.reserved) if (r != 0) { why = "reserved fields must be zero"; return false; }
    return true;
}

// the schedule of a tuned solve: the table entry for this shape, if any
void apply_tune(const lrr_ctx* ctx, lrr_opts& o, int m, int n, int t, int maxl) {
    if (!o.tune) return;
    for (const lrr::host::TuneEntry& e : ctx->tune) {
        if (e.m == m && e.n == n && e.t == t && e.maxl == maxl && e.precision == o.precision) {
            o.eig_block = e.eig_block;
            o.use_graph = e.use_graph;
            o.check_every = e.check_every;
            o.coords = e.coords;
            return;
        }
    }
}

struct Problem {
    int m, n, ncols, t;
    const double* A; long lda;
    const double* X; long ldx;    // either X given ...
    const int* perm;              // ... or columns perm of A (host)
    const int* offsets;           // host, t + 1
    double lam;
    lrr_opts o;
    int local = 0;                // 1: block b uses its own observations as dictionary
};

struct Result {
    std::vector<int> iters, rank;
    std::vector<double> res1, res2;
    int batch_iters = 0;
    bool converged = true;
};

void ensure_ws(lrr_ctx* ctx, size_t bytes) {
    if (ctx->ws_bytes >= bytes) return;
    if (ctx->ws) { (void)hipFree(ctx->ws); ctx->ws = nullptr; ctx->ws_bytes = 0; }
    void* p = nullptr;
    if (!lrr::try_device_alloc(&p, bytes)) throw std::bad_alloc();
    ctx->ws = p;
    ctx->ws_bytes = bytes;
}

void* ensure_pinned(lrr_ctx* ctx, size_t bytes) {
    if (ctx->pinned_bytes >= bytes) return ctx->pinned;
    if (ctx->pinned) { (void)hipHostFree(ctx->pinned); ctx->pinned = nullptr; ctx->pinned_bytes = 0; }
    void* p = nullptr;
    LRR_HIP(hipHostMalloc(&p, bytes, hipHostMallocDefault));
    ctx->pinned = p;
    ctx->pinned_bytes = bytes;
    return p;
}

Plan make_plan(const Problem& pr) {
    Plan p;
    p.m = pr.m; p.n = pr.n; p.ncols = pr.ncols; p.t = pr.t;
    p.boff.assign(pr.offsets, pr.offsets + pr.t + 1);
    p.maxl = 0;
    for (int b = 0; b < pr.t; ++b) p.maxl = std::max(p.maxl, p.boff[b + 1] - p.boff[b]);
    p.bs = jacobi_bs(p.maxl, pr.o.eig_block);
    p.L.resize(pr.t);
    p.maxL = 0;
    for (int b = 0; b < pr.t; ++b) {
        p.L[b] = round_up(p.boff[b + 1] - p.boff[b], 2 * p.bs);
        p.maxL = std::max(p.maxL, p.L[b]);
    }
    p.n_iter = pr.o.fixed_iters > 0 ? pr.o.fixed_iters : pr.o.max_iter;
    p.pm = product_modes(pr.o.precision);
    // reduced coordinates: explicit request, or automatic when the dictionary is
    // wider than tall (the iterates then live in a space of dimension <= m < n);
    // the reverse-mode record keeps full coordinates
    const int coords = pr.o.coords;
    p.reduced = coords == LRR_COORDS_REDUCED ||
                (coords == LRR_COORDS_AUTO && pr.n >= 2 * pr.m && !pr.o.save_for_backward &&
                 pr.o.solve_form != LRR_SOLVE_LITERAL);
    if (pr.o.save_for_backward) p.reduced = false;
    p.nrb = p.reduced ? std::min(pr.m, pr.n) : pr.n;
    p.local = pr.local != 0;
    if (p.local) {
        // rows of a block's iterates index its own points: l_b <= maxl rows; rows
        // beyond l_b meet zero dictionary columns and stay exactly zero
        p.reduced = false;
        p.nrb = p.maxl;
    }
    // literal Z-step: on request, or automatically when the dictionary is at
    // least as tall as wide (then n x n is the smaller factorisation); the
    // reduced-precision forms, the reduced coordinates, a recorded forward and
    // the local variant use the push-through form
    if (!p.local && !p.reduced && !pr.o.save_for_backward) {
        if (pr.o.solve_form == LRR_SOLVE_LITERAL) p.literal = true;
        else if (pr.o.solve_form == LRR_SOLVE_AUTO && pr.n <= pr.m && pr.o.precision == LRR_FP64) p.literal = true;
    }
    p.ks = p.literal ? pr.n : pr.m;
    p.nr = p.nrb;
    p.bq = pr.m > 512 ? 32 : 16;
    p.Lm = round_up(pr.m, 2 * p.bq);
    return p;
}

hipStream_t ctx_capture_stream(lrr_ctx* ctx) {
    if (!ctx->capture) LRR_HIP(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
    return ctx->capture;
}


// Reduced coordinates: every iterate of the n-row state (Z, J, Y2) starts at
// zero and is updated only by products with M^T and by column operations, so
// it stays in range(M^T) (pinned on the oracle).  With Qm an orthonormal basis
// of that range (n x r, r = numerical rank of M), Z = Qm Zr exactly and the
// whole iteration runs on r-row coefficients: the Gram matrix Y^T Y equals
// Yr^T Yr, and the dictionary products use Mr = M Qm (m x r).
// Qm = M^T W diag(1/sigma) from the eigen-decomposition M M^T = W diag(sigma^2)
// W^T (kept: sigma^2 > 1e-14 sigma_max^2), then one Newton-Schulz step
// Qm <- Qm (3 I - Qm^T Qm) / 2 restores orthonormality to rounding.
constexpr double kRankCut = 1e-14;

void build_basis(const Problem& pr, Plan& p, Buffers& b, hipStream_t s) {
    const int m = p.m, n = p.n, Lm = p.Lm, bq = p.bq;
    // G = M M^T (padded to Lm), eigen-decomposition by block Jacobi from the identity
    LRR_HIP(hipMemsetAsync(b.Gb, 0, sizeof(double) * (size_t)Lm * Lm, s));
    GemmDesc gG{pr.A, pr.A, b.Gb, m, m, n, (int)pr.lda, (int)pr.lda, Lm, 1.0, 0.0, nullptr, nullptr};
    std::vector<int> lo(Lm);
    for (int i = 0; i < Lm; ++i) lo[i] = i >= m ? 1 : 0;
    const int one = 1;
    LRR_HIP(hipMemcpyAsync(b.g_red, &gG, sizeof(GemmDesc), hipMemcpyHostToDevice, s));
    LRR_HIP(hipMemcpyAsync(b.loq, lo.data(), sizeof(int) * Lm, hipMemcpyHostToDevice, s));
    LRR_HIP(hipMemcpyAsync(b.runq, &one, sizeof(int), hipMemcpyHostToDevice, s));
    EigDesc ed{b.Gb, b.Wq, b.Rq, b.lamq, Lm, m, b.runq, b.stq, b.scaleq, b.protq, b.loq, nullptr};
    LRR_HIP(hipMemcpyAsync(b.eq, &ed, sizeof(EigDesc), hipMemcpyHostToDevice, s));
    lrr::launch_dgemm(b.g_red, 1, m, m, false, true, s);
    lrr::launch_set_identity(b.Wq, Lm, s);
    lrr::launch_jacobi_init(b.eq, 1, s);
    int* any = b.idxq;     // scratch flag until the index list is written
    int h_any = 1;
    for (int sw = 0; sw < 80; ++sw) {
        LRR_HIP(hipMemsetAsync(any, 0, sizeof(int), s));
        lrr::launch_jacobi_check(b.eq, 1, Lm, any, s);
        LRR_HIP(hipMemcpyAsync(&h_any, any, sizeof(int), hipMemcpyDeviceToHost, s));
        LRR_HIP(hipStreamSynchronize(s));
        if (h_any == 0) break;
        for (int r = 0; r < Lm / bq - 1; ++r) lrr::launch_jacobi_round(b.eq, 1, Lm, bq, r, s);
    }
    lrr::launch_jacobi_eigvals(b.eq, 1, s);
    std::vector<double> lam(Lm);
    LRR_HIP(hipMemcpyAsync(lam.data(), b.lamq, sizeof(double) * Lm, hipMemcpyDeviceToHost, s));
    LRR_HIP(hipStreamSynchronize(s));
    double lmax = 0.0;
    for (int i = 0; i < m; ++i) lmax = std::max(lmax, lam[i]);
    std::vector<int> idx;
    for (int i = 0; i < m; ++i)
        if (lam[i] > kRankCut * lmax) idx.push_back(i);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return lam[x] > lam[y]; });
    if ((int)idx.size() > p.nrb) idx.resize(p.nrb);   // rank(M) <= min(m, n)
    if (idx.empty()) idx.push_back(0);     // M = 0: a single zero column (scaled by 0 below)
    const int r = (int)idx.size();
    p.nr = r;
    LRR_HIP(hipMemcpyAsync(b.idxq, idx.data(), sizeof(int) * r, hipMemcpyHostToDevice, s));
    // Wk = W_kept diag(1/sigma) (m x r, in the Gram buffer), Qm = M^T Wk, NS step, Mr = M Qm
    GemmDesc g[4] = {
        GemmDesc{pr.A, b.Gb, b.Qm, n, r, m, (int)pr.lda, m, n, 1.0, 0.0, nullptr, nullptr},
        GemmDesc{b.Qm, b.Qm, b.Gq, r, r, n, n, n, r, 1.0, 0.0, nullptr, nullptr},
        GemmDesc{b.Qm, b.Tq, b.Qtmp, n, r, r, n, r, n, 1.0, 0.0, nullptr, nullptr},
        GemmDesc{pr.A, b.Qtmp, b.Mr, m, r, n, (int)pr.lda, n, m, 1.0, 0.0, nullptr, nullptr}};
    LRR_HIP(hipMemcpyAsync(b.g_red + 1, g, sizeof(g), hipMemcpyHostToDevice, s));
    lrr::launch_gather_scaled(b.Wq, Lm, b.lamq, b.idxq, b.Gb, m, m, r, s);
    lrr::launch_dgemm(b.g_red + 1, 1, n, r, true, false, s);
    lrr::launch_dgemm(b.g_red + 2, 1, r, r, true, false, s);
    lrr::launch_ns_factor(b.Gq, b.Tq, r, s);
    lrr::launch_dgemm(b.g_red + 3, 1, n, r, false, false, s);
    lrr::launch_dgemm(b.g_red + 4, 1, m, r, false, false, s);
    std::swap(b.Qm, b.Qtmp);       // the orthonormalised basis
    LRR_HIP(hipStreamSynchronize(s));   // host descriptors go out of scope
}

// Lay out the workspace, upload the descriptors, gather the observations,
// zero the state and factor K = I + A A^T (once per solve).
void setup_alm(lrr_ctx* ctx, const Problem& pr, Plan& p, Buffers& b, hipStream_t s, bool with_combine) {
    const int m = p.m, n = p.n, c = p.ncols, t = p.t;
    const lrr_opts& o = pr.o;
    const size_t need = layout(p, nullptr, b, with_combine, true);
    ensure_ws(ctx, need);
    if (!ctx->dwork) LRR_HIP(hipMalloc((void**)&ctx->dwork, lrr::kWorkBytes));
    LRR_HIP(hipMemsetAsync(ctx->dwork, 0, lrr::kWorkBytes, s));
    layout(p, static_cast<char*>(ctx->ws), b, with_combine, true);
    ensure_pinned(ctx, sizeof(int) * (4 * (size_t)t + 16) + sizeof(double) * 2 * t);
    if (p.reduced) build_basis(pr, p, b, s);
    else if (!p.local) p.nr = n;
    const int nr = p.nr;
    // dictionary of the Z-step products: M, or Mr = M Qm in reduced coordinates
    const double* Md = p.reduced ? b.Mr : pr.A;
    const int ldmd = p.reduced ? m : (int)pr.lda;

    // ---- host-side tables -------------------------------------------------
    std::vector<int> colblk(c);
    for (int bb = 0; bb < t; ++bb)
        for (int j = p.boff[bb]; j < p.boff[bb + 1]; ++j) colblk[j] = bb;
    std::vector<double> sched(p.n_iter + 2);
    sched[0] = o.mu0;
    for (int k = 1; k < (int)sched.size(); ++k) sched[k] = std::min(o.rho * sched[k - 1], o.mu_max);

    std::vector<GemmDesc> gram(t), gRT(t), gRSG(t), gRXE(t), gOG(t), gBq(t), gP(t), gJ(t);
    std::vector<GemmDesc> gMQ(t), gMQa(t), gKV(t), gMtV(t), gExp(t), gF1T(t), gF2Q(t), gAZ(t);
    std::vector<EigDesc> eig(t);
    std::vector<size_t> need_off(t + 1, 0), sched_off(t + 1, 0);
    for (int bb = 0; bb < t; ++bb) {
        const size_t nb = p.L[bb] / p.bs;
        need_off[bb + 1] = need_off[bb] + nb * nb;
        sched_off[bb + 1] = sched_off[bb] + (nb - 1) * (nb / 2);
    }
    std::vector<SvtDesc> svt(t);
    std::vector<RefDesc> ref(t);
    for (int bb = 0; bb < t; ++bb) {
        const int l = p.boff[bb + 1] - p.boff[bb], L = p.L[bb];
        const size_t LL = (size_t)L * L;
        double* Yb = b.Y + (size_t)p.boff[bb] * nr;
        double* Jb = b.J + (size_t)p.boff[bb] * nr;
        const int* run = b.svt_run + bb;    // thresholds this iteration
        const int* erun = b.eig_run + bb;   // needs an eigen-decomposition this iteration
        const int* rrun = b.ref_run + bb;
        double* X = b.Wm[bb];
        double* T = b.TX[bb];
        gram[bb] = GemmDesc{Yb, Yb, b.Bm[bb], l, l, nr, nr, nr, L, 1.0, 0.0, erun, nullptr};
        // refinement: T = B X, S = X^T T, G = X^T X (symmetric kernel), XE = X E
        gRT[bb] = GemmDesc{b.Bm[bb], X, T, L, L, L, L, L, L, 1.0, 0.0, rrun, nullptr};
        gRSG[bb] = GemmDesc{X, T, b.SG[bb], L, L, L, L, L, L, 1.0, 0.0, rrun, nullptr};
        gRXE[bb] = GemmDesc{X, b.Eb[bb], b.XE[bb], L, L, L, L, L, L, 1.0, 0.0, rrun, nullptr};
        // orthogonalisation: G = X^T X;  Jacobi matrix Bq = X^T (B X)
        gOG[bb] = GemmDesc{X, X, b.SG[bb] + LL, L, L, L, L, L, L, 1.0, 0.0, rrun, nullptr};
        gBq[bb] = GemmDesc{X, T, b.Bq[bb], L, L, L, L, L, L, 1.0, 0.0, rrun, nullptr};
        gP[bb] = GemmDesc{b.Wg[bb], X, b.Pm[bb], l, l, L, L, L, L, 1.0, 0.0, run, nullptr};
        gJ[bb] = GemmDesc{Yb, b.Pm[bb], Jb, nr, l, l, nr, L, nr, 1.0, 0.0, run, nullptr};
        const int* act = b.active + bb;
        const size_t o_n = (size_t)p.boff[bb] * nr, o_m = (size_t)p.boff[bb] * m;
        // dictionary of this block: M (or Mr), or in local mode its own columns
        // C_b (m x l, inside the gathered observations) with l inner rows
        const double* Mb = p.local ? b.X + o_m : Md;
        const int ldb_ = p.local ? m : ldmd;
        const int kin = p.local ? l : nr;
        const double* Kb = b.K + (p.local ? (size_t)bb * m * m : 0);
        if (p.pm.dMQ) {
            gMQ[bb] = GemmDesc{Mb, b.Dn + o_n, b.MQacc + o_m, m, l, kin, ldb_, nr, m, 1.0, 1.0, act, nullptr};
            // re-anchoring: the carried product replaced by an FP64 M Q
            gMQa[bb] = GemmDesc{Mb, b.Q + o_n, b.MQacc + o_m, m, l, kin, ldb_, nr, m, 1.0, 0.0, act, nullptr};
        }
        else
            gMQ[bb] = GemmDesc{Mb, b.Q + o_n, b.T + o_m, m, l, kin, ldb_, nr, m, -1.0, 1.0, act, nullptr};
        gKV[bb] = GemmDesc{Kb, b.T + o_m, b.V + o_m, m, l, m, m, m, m, 1.0, 0.0, act, nullptr};
        if (p.literal) {
            // Z = K^{-1} (A^T T + Q) = Q + [F1 T + (K^{-1} - I) Q], then T -= A Z
            gF1T[bb] = GemmDesc{b.F1, b.T + o_m, b.MtV + o_n, nr, l, m, nr, m, nr, 1.0, 0.0, act, nullptr};
            gF2Q[bb] = GemmDesc{b.K, b.Q + o_n, b.MtV + o_n, nr, l, nr, nr, nr, nr, 1.0, 1.0, act, nullptr};
            gAZ[bb] = GemmDesc{Md, b.Z + o_n, b.T + o_m, m, l, nr, ldmd, nr, m, -1.0, 1.0, act, nullptr};
        }
        gMtV[bb] = GemmDesc{Mb, b.V + o_m, b.MtV + o_n, kin, l, m, ldb_, m, nr, 1.0, 0.0, act, nullptr};
        if (p.reduced)   // expansion of the coupling residual: R2 = Qm R2r
            gExp[bb] = GemmDesc{b.Qm, b.R2r + o_n, b.R2full + (size_t)p.boff[bb] * n, n, l, nr, n, nr, n, 1.0,
                                0.0, b.expand + bb, nullptr};
        eig[bb] = EigDesc{b.Bq[bb], X, b.Rm[bb], b.lam[bb], L, l, erun, b.eigst + 2 * bb,
                          b.eigscale + bb, b.prot[bb], b.lo[bb], ctx->dwork, b.locut + bb, b.passes + bb,
                          b.need_all + need_off[bb], b.sched_all + sched_off[bb], b.ref_clean + bb};
        svt[bb] = SvtDesc{b.Bq[bb], X, b.Wg[bb], b.lam[bb], b.h[bb], L, l, run, bb};
        ref[bb] = RefDesc{b.Bm[bb], X, b.SG[bb], b.Eb[bb], b.XE[bb], b.lam[bb], b.lo[bb], b.ref_scale + bb,
                          b.ref_emax + bb, b.ref_unres + bb, b.ref_eprev + bb, b.ref_run + bb,
                          b.ref_cont + bb, b.Bq[bb], b.locut + bb, L, l, bb, b.ref_rdev + bb,
                          b.ref_nsskip + bb, b.ref_clean + bb};
    }
    std::vector<GemmDesc> gKK(p.local ? t : 1);
    if (p.literal)
        gKK[0] = GemmDesc{pr.A, pr.A, b.K, n, n, m, (int)pr.lda, (int)pr.lda, n, 1.0, 0.0, nullptr, nullptr};
    else if (p.local)
        for (int bb = 0; bb < t; ++bb)
            gKK[bb] = GemmDesc{b.X + (size_t)p.boff[bb] * m, b.X + (size_t)p.boff[bb] * m, b.K + (size_t)bb * m * m,
                               m, m, p.boff[bb + 1] - p.boff[bb], m, m, m, 1.0, 0.0, nullptr, nullptr};
    else
        gKK[0] = GemmDesc{pr.A, pr.A, b.K, m, m, n, (int)pr.lda, (int)pr.lda, m, 1.0, 0.0, nullptr, nullptr};

    auto up = [&](void* dst, const void* src, size_t bytes) {
        LRR_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    };
    up(b.colblk, colblk.data(), sizeof(int) * c);
    up(b.boff, p.boff.data(), sizeof(int) * (t + 1));
    up(b.mu_sched, sched.data(), sizeof(double) * sched.size());
    up(b.g_gram, gram.data(), sizeof(GemmDesc) * t);
    up(b.g_refT, gRT.data(), sizeof(GemmDesc) * t);
    up(b.g_refSG, gRSG.data(), sizeof(GemmDesc) * t);
    up(b.g_refXE, gRXE.data(), sizeof(GemmDesc) * t);
    up(b.g_orthG, gOG.data(), sizeof(GemmDesc) * t);
    up(b.g_Bq, gBq.data(), sizeof(GemmDesc) * t);
    up(b.ref, ref.data(), sizeof(RefDesc) * t);
    up(b.g_P, gP.data(), sizeof(GemmDesc) * t);
    up(b.g_J, gJ.data(), sizeof(GemmDesc) * t);
    up(b.g_MQ, gMQ.data(), sizeof(GemmDesc) * t);
    up(b.g_MQa, gMQa.data(), sizeof(GemmDesc) * t);
    up(b.g_KV, gKV.data(), sizeof(GemmDesc) * t);
    up(b.g_MtV, gMtV.data(), sizeof(GemmDesc) * t);
    if (p.literal) {
        up(b.g_F1T, gF1T.data(), sizeof(GemmDesc) * t);
        up(b.g_F2Q, gF2Q.data(), sizeof(GemmDesc) * t);
        up(b.g_AZ, gAZ.data(), sizeof(GemmDesc) * t);
        const GemmDesc gF1{b.K, pr.A, b.F1, n, m, n, n, (int)pr.lda, n, 1.0, 0.0, nullptr, nullptr};
        up(b.g_F1, &gF1, sizeof(GemmDesc));
    }
    if (p.reduced) up(b.g_exp, gExp.data(), sizeof(GemmDesc) * t);

    up(b.g_KK, gKK.data(), sizeof(GemmDesc) * gKK.size());
    up(b.eig, eig.data(), sizeof(EigDesc) * t);
    {
        // item prefixes of the persistent eigensolve: rows, pair slots, apply items
        std::vector<int> offs(3 * (t + 1), 0);
        for (int bb = 0; bb < t; ++bb) {
            const int L = p.L[bb], nbb = L / p.bs, np = nbb / 2;
            offs[bb + 1] = offs[bb] + L;
            offs[(t + 1) + bb + 1] = offs[(t + 1) + bb] + np;
            offs[2 * (t + 1) + bb + 1] = offs[2 * (t + 1) + bb] + np * (np + 1) / 2 + ((L + 63) / 64) * np;
        }
        up(b.jac_offs, offs.data(), sizeof(int) * offs.size());
        LRR_HIP(hipStreamSynchronize(s));   // the host table goes out of scope
    }
    up(b.svt, svt.data(), sizeof(SvtDesc) * t);
    if (pr.perm) up(b.perm, pr.perm, sizeof(int) * c);

    // ---- setup: observations, state, factorisation (once per solve) -------
    if (pr.perm) lrr::launch_gather_cols(pr.A, pr.lda, b.X, m, m, c, b.perm, s);
    else lrr::launch_copy_cols(pr.X, pr.ldx, b.X, m, m, c, s);
    const size_t nc = (size_t)nr * c, mc = (size_t)m * c;
    LRR_HIP(hipMemsetAsync(b.Z, 0, sizeof(double) * nc, s));
    LRR_HIP(hipMemsetAsync(b.J, 0, sizeof(double) * nc, s));
    LRR_HIP(hipMemsetAsync(b.Y2, 0, sizeof(double) * nc, s));
    LRR_HIP(hipMemsetAsync(b.E, 0, sizeof(double) * mc, s));
    LRR_HIP(hipMemsetAsync(b.Y1, 0, sizeof(double) * mc, s));
    // local mode: the rows of M^T V beyond a block's width are never written
    if (p.local) LRR_HIP(hipMemsetAsync(b.MtV, 0, sizeof(double) * nc, s));
    // the carried product M Q starts from Q = 0
    if (p.pm.dMQ) {
        LRR_HIP(hipMemsetAsync(b.Q, 0, sizeof(double) * nc, s));
        LRR_HIP(hipMemsetAsync(b.MQacc, 0, sizeof(double) * mc, s));
    }
    for (int bb = 0; bb < t; ++bb) {
        const size_t L = p.L[bb];
        LRR_HIP(hipMemsetAsync(b.Bm[bb], 0, sizeof(double) * L * L, s));
        LRR_HIP(hipMemsetAsync(b.TX[bb], 0, sizeof(double) * L * L, s));
        LRR_HIP(hipMemsetAsync(b.Bq[bb], 0, sizeof(double) * L * L, s));
        LRR_HIP(hipMemsetAsync(b.Pm[bb], 0, sizeof(double) * L * L, s));
        LRR_HIP(hipMemsetAsync(b.h[bb], 0, sizeof(double) * L, s));
        lrr::launch_set_identity(b.Wm[bb], (int)L, s);
    }
    std::vector<int> ones(t, 1);
    up(b.active, ones.data(), sizeof(int) * t);
    LRR_HIP(hipMemsetAsync(b.iters, 0, sizeof(int) * t, s));
    LRR_HIP(hipMemsetAsync(b.warm, 0, sizeof(int) * t, s));
    LRR_HIP(hipMemsetAsync(b.passes, 0, sizeof(int) * t, s));
    LRR_HIP(hipMemsetAsync(b.jac_ctl, 0, sizeof(lrr::JacCtl), s));
    LRR_HIP(hipMemsetAsync(b.locut, 0, sizeof(double) * t, s));   // every eigenpair resolved at first
    LRR_HIP(hipMemsetAsync(b.rank, 0, sizeof(int) * t, s));
    LRR_HIP(hipMemsetAsync(b.r1max, 0, sizeof(unsigned long long) * t, s));
    LRR_HIP(hipMemsetAsync(b.r2max, 0, sizeof(unsigned long long) * t, s));
    LRR_HIP(hipMemsetAsync(b.res1, 0, sizeof(double) * t, s));
    LRR_HIP(hipMemsetAsync(b.res2, 0, sizeof(double) * t, s));
    if (p.reduced) LRR_HIP(hipMemsetAsync(b.r2nrm, 0, sizeof(unsigned long long) * t, s));
    lrr::launch_init_iter(b.it, b.mu_sched, 0, s);

    // literal form: K = I + A^T A (n x n), K^{-1} (FP64 Cholesky, once per
    // solve), F1 = K^{-1} A^T, then K^{-1} - I in place
    if (p.literal) {
        lrr::launch_dgemm(b.g_KK, 1, n, n, true, false, s);
        lrr::launch_add_identity(b.K, n, n, 1.0, s);
        lrr::spd_inverse(b.K, n, b.Lb, b.Linv, b.Dinv, b.Tb, b.g_spd, b.flag, s);
        lrr::launch_dgemm(b.g_F1, 1, n, m, false, true, s);
        lrr::launch_add_identity(b.K, n, n, -1.0, s);
        return;
    }
    // K = I + A A^T, then K^{-1} (FP64 Cholesky, once per solve; per block in
    // local mode, A = C_b)
    for (size_t bb = 0; bb < gKK.size(); ++bb) {
        double* Kb = b.K + bb * (size_t)m * m;
        lrr::launch_dgemm(b.g_KK + bb, 1, m, m, false, true, s);
        lrr::launch_add_identity(Kb, m, m, 1.0, s);
        lrr::spd_inverse(Kb, m, b.Lb, b.Linv, b.Dinv, b.Tb, b.g_spd, b.flag, s);
    }
}

// Hooks of iterate_alm: called before iteration k starts and after it ends
// (the stream is not synchronised in between).
struct IterHooks {
    std::function<void(int)> begin;
    std::function<void(int)> end;
};

// Iterations [k0, k1) of the batched ALM over all blocks, from the state in the
// workspace (DevIter must hold iteration k0); leaves the state there.
Result iterate_alm(lrr_ctx* ctx, const Problem& pr, Plan& p, Buffers& b, hipStream_t s, int k0, int k1,
                   const IterHooks* hooks = nullptr) {
    // n: rows of the iterates (the numerical rank of M in reduced coordinates)
    const int m = p.m, n = p.nr, nfull = p.n, c = p.ncols, t = p.t;
    const lrr_opts& o = pr.o;
    // targeted Jacobi rounds: per-block offsets of the check marks and schedules
    std::vector<size_t> need_off(t + 1, 0), sched_off(t + 1, 0);
    for (int bb = 0; bb < t; ++bb) {
        const size_t nbb = p.L[bb] / p.bs;
        need_off[bb + 1] = need_off[bb] + nbb * nbb;
        sched_off[bb + 1] = sched_off[bb] + (nbb - 1) * (nbb / 2);
    }
    const size_t need_total = need_off[t];
    // pinned host area: the flags, the check marks (read back every pass) and the
    // round schedules (uploaded by targeted passes; rewritten only after the next
    // pass's synchronisation, when the previous upload has completed)
    const size_t flag_bytes = (sizeof(int) * (4 * (size_t)t + 16) + sizeof(double) * 2 * t + 255) & ~size_t(255);
    const size_t need_bytes = (sizeof(int) * need_off[t] + 255) & ~size_t(255);
    int* hp = static_cast<int*>(ensure_pinned(ctx, flag_bytes + need_bytes + sizeof(int) * sched_off[t]));
    int* h_need = reinterpret_cast<int*>(reinterpret_cast<char*>(hp) + flag_bytes);
    int* h_sched = reinterpret_cast<int*>(reinterpret_cast<char*>(hp) + flag_bytes + need_bytes);
    BlockState bst{b.active, b.svt_run, b.iters, b.rank, b.res1, b.res2, b.r1max, b.r2max, b.colr1, b.colr2};
    const ProductModes& pm = p.pm;
    const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 30;
    const int check_every = o.check_every > 0 ? o.check_every : 1;
    const int fixed = o.fixed_iters > 0 ? 1 : 0;
    // The refinement stops after a correction below ref_stop: the next one
    // (quadratic in it) would be at the rounding level of the products.  A
    // fixed-iteration solve, the form callers differentiate, uses 1e-10 so that
    // its forward map stays smooth at the scale of a central difference
    // (h = 1e-6); a solve that stops on the tolerance, whose iteration count is
    // itself a step function of the data, uses 1e-8.
    const double ref_stop = fixed ? 1e-10 : 1e-8;
    // Blocks decomposed ahead of their first thresholding step (k_eig_select):
    // ||Y||_F above this fraction of tau when another block goes cold.  Off in
    // fixed-iteration solves, whose recorded J-steps follow the thresholding
    // blocks only.
    const double prewarm = fixed ? 0.0 : kPreWarm;
    int* h_svt = hp + 3 * t + 16;   // t ints: thresholding blocks (pricing of P and J)
    int* h_run = hp;            // t ints
    int* h_misc = hp + t;       // scalars
    int* h_ref = hp + t + 16;   // t ints: refinement still running, per block
    int* h_act = hp + 2 * t + 16;   // t ints: block still iterating

    Result res;
    LrrProf& prof = ctx->prof;
    auto timed = [&](const char* name, double flops, double bytes, auto&& f) {
        prof.run(s, name, flops, bytes, f);
    };
    auto sync = [&]() {
        LRR_HIP(hipStreamSynchronize(s));
        if (prof.on) prof.flush();
    };
    std::fill(h_act, h_act + t, 1);
    long long sweeps_total = 0;
    std::vector<int> block_rounds(t, 0);
    const double D = sizeof(double);
    // use_graph 0, 1: the J-step's decisions on the host (refinement steps, Jacobi
    // passes); 2, 3: every decision on the device, one launch sequence per
    // iteration (2: replayed from a graph, 3: launched one by one)
    const bool device_loop = o.use_graph >= 2;
    // device queries of the launch shapes, made before any stream capture
    (void)lrr::gemm_grid();
    if (device_loop) (void)lrr::jacobi_solve_grid(p.bs);
    auto zstep = [&](hipStream_t st, bool anchor, auto&& tm, double cact) {
        tm("k_form_QT", 0.0, ((pm.dMQ ? 5.0 : 3.0) * n + 4.0 * m) * cact * D, [&] {
            lrr::launch_form_QT(b.J, b.Y2, b.Q, pm.dMQ ? b.Dn : nullptr, n, n, b.X, b.E, b.Y1, b.T, m, m, c,
                                b.colblk, b.active, b.it, st);
        });
        if (p.literal) {
            // Z = K^{-1} (A^T T + Q) with K = I + A^T A, written as Z = Q + W with
            // W = F1 T + (K^{-1} - I) Q; then T - A Z = X - E + Y1/mu - A Z, so
            // E + (T - A Z) is the shrinkage input: the role V plays in the
            // push-through form
            tm("k_dgemm<false, false>", 2.0 * n * m * cact, 0.0, [&] {
                lrr::launch_dgemm(b.g_F1T, t, n, p.maxl, false, false, st);
            });
            tm("k_dgemm<false, false>", 2.0 * n * n * cact, 0.0, [&] {
                lrr::launch_dgemm(b.g_F2Q, t, n, p.maxl, false, false, st);
            });
            tm("k_update_Z", 0.0, 6.0 * n * cact * D, [&] {
                lrr::launch_update_Z(b.Q, b.MtV, b.J, b.Z, b.Y2, nullptr, nullptr, n, n, c, b.colblk, bst, b.it,
                                     st);
            });
            tm("k_dgemm<false, false>", 2.0 * m * n * cact, 0.0, [&] {
                lrr::launch_dgemm(b.g_AZ, t, m, p.maxl, false, false, st);
            });
            tm("k_estep", 0.0, 5.0 * m * cact * D, [&] {
                lrr::launch_estep(b.E, b.T, b.Y1, m, m, c, pr.lam, b.colblk, bst, b.it, st);
            });
            tm("k_block_colmax", 0.0, 0.0, [&] {
                lrr::launch_block_colmax(b.colr1, b.boff, t, bst, b.r1max, st, b.colr2, b.r2max);
            });
            tm("k_check", 0.0, 0.0, [&] {
                lrr::launch_check(bst, t, b.it, b.mu_sched, o.tol, fixed, b.n_active, st);
            });
            return;
        }
        // T = P - M Q; the difference form carries M Q as a sum of products M dQ
        if (anchor) {
            // every kAnchorEvery iterations the rounding carried in the sum of
            // products is dropped: M Q is formed once in FP64
            tm("k_dgemm<false, false>", 2.0 * m * n * cact, 0.0, [&] {
                lrr::launch_dgemm(b.g_MQa, t, m, p.maxl, false, false, st);
            });
        } else {
            tm(lrr::xgemm_name(pm.MQ, false, false), 2.0 * m * n * cact, 0.0, [&] {
                lrr::launch_xgemm(b.g_MQ, t, m, p.maxl, false, false, pm.MQ, st);
            });
        }
        if (pm.dMQ)
            tm("k_sub_cols", 0.0, 3.0 * m * cact * D, [&] {
                lrr::launch_sub_cols(b.T, b.MQacc, m, m, c, b.colblk, b.active, st);
            });
        tm("k_dgemm<false, false>", 2.0 * m * m * cact, 0.0, [&] {
            lrr::launch_dgemm(b.g_KV, t, m, p.maxl, false, false, st);
        });
        tm(lrr::xgemm_name(pm.MtV, true, false), 2.0 * n * m * cact, 0.0, [&] {
            lrr::launch_xgemm(b.g_MtV, t, n, p.maxl, true, false, pm.MtV, st);
        });
        tm("k_update_Z", 0.0, (p.reduced ? 7.0 : 6.0) * n * cact * D, [&] {
            lrr::launch_update_Z(b.Q, b.MtV, b.J, b.Z, b.Y2, b.R2r, b.r2nrm, n, n, c, b.colblk, bst, b.it, st);
        });
        if (p.reduced) {
            // max-norm of R2 = Qm R2r: decided by the column 2-norm bounds, else expanded
            tm("k_block_colmax", 0.0, 0.0, [&] {
                lrr::launch_block_colmax(b.colr2, b.boff, t, bst, b.r2nrm, st);
            });
            tm("k_r2_decide", 0.0, 0.0, [&] {
                lrr::launch_r2_decide(bst, b.r2nrm, b.expand, t, o.tol, std::sqrt((double)nfull), st);
            });
            tm("k_dgemm<false, false>", 0.0, 0.0, [&] {
                lrr::launch_dgemm(b.g_exp, t, nfull, p.maxl, false, false, st);
            });
            tm("k_colmax", 0.0, 0.0, [&] {
                lrr::launch_colmax(b.R2full, nfull, nfull, c, b.colblk, b.expand, b.r2max, st);
            });
        }
        tm("k_estep", 0.0, 5.0 * m * cact * D, [&] {
            lrr::launch_estep(b.E, b.V, b.Y1, m, m, c, pr.lam, b.colblk, bst, b.it, st);
        });
        tm("k_block_colmax", 0.0, 0.0, [&] {
            if (p.reduced) lrr::launch_block_colmax(b.colr1, b.boff, t, bst, b.r1max, st);
            else lrr::launch_block_colmax(b.colr1, b.boff, t, bst, b.r1max, st, b.colr2, b.r2max);
        });
        tm("k_check", 0.0, 0.0, [&] {
            lrr::launch_check(bst, t, b.it, b.mu_sched, o.tol, fixed, b.n_active, st);
        });
    };
    // One iteration's J-step: every decision is taken on the device from per-block
    // flags (which blocks threshold, which refinement steps apply, how the
    // eigensolve proceeds), so the launches are the same in every iteration.
    // Only while profiling (`tm` times launches, prof.on) are the flags read back,
    // to price each launch with the flops of the blocks it actually covers.
    auto jstep = [&](hipStream_t st, auto&& tm, double cact) {
        const bool price = prof.on;
        auto read_flags = [&](int* dst, const int* src) {
            if (!price) return;
            LRR_HIP(hipMemcpyAsync(dst, src, sizeof(int) * t, hipMemcpyDeviceToHost, st));
            sync();
        };
        // J-step input and the exact zero test
        tm("k_form_Y", 0.0, 3.0 * n * cact * D, [&] {
            lrr::launch_form_Y(b.Z, b.Y2, b.Y, b.colsq, n, n, c, b.colblk, b.active, b.it, st);
        });
        tm("k_block_fro", 0.0, cact * D, [&] { lrr::launch_block_fro(b.colsq, b.boff, t, bst, b.it, st); });
        tm("k_zero_J", 0.0, 0.0, [&] { lrr::launch_zero_J(b.J, n, n, c, b.colblk, bst, st); });
        tm("k_eig_select", 0.0, 0.0, [&] {
            lrr::launch_eig_select(b.colsq, b.boff, t, b.active, b.svt_run, b.warm, b.eig_run, b.it, prewarm, st);
        });
        read_flags(h_run, b.eig_run);
        read_flags(h_svt, b.svt_run);
        double f_gram = 0, f_P = 0, f_J = 0, f_L3 = 0;
        for (int bb = 0; bb < t && price; ++bb) {
            const double l = p.boff[bb + 1] - p.boff[bb], L = p.L[bb];
            if (h_svt[bb]) {
                f_P += 2.0 * l * l * L;
                f_J += 2.0 * n * l * l;
            }
            if (!h_run[bb]) continue;
            f_gram += 2.0 * l * l * n;
            f_L3 += 2.0 * L * L * L;
        }
        // the symmetric kernel computes the tiles on and above the diagonal
        const double hg = lrr::dgemm_sym_tiles(t, p.maxl) ? 0.5 : 1.0, hL = lrr::dgemm_sym_tiles(t, p.maxL) ? 0.5 : 1.0;
        // Gram matrix of each block that thresholds (FP64 in every precision form)
        tm("k_dgemm_sym", hg * f_gram, 0.0, [&] { lrr::launch_dgemm_sym(b.g_gram, t, p.maxl, st); });
        // Newton refinement of the previous iteration's eigenvectors: a fixed
        // number of steps, each applied only where the per-block flags allow
        tm("k_ref_begin", 0.0, 0.0, [&] { lrr::launch_ref_begin(b.ref, t, p.maxL, b.eig_run, b.warm, st); });
        for (int step = 0; step < kRefSteps; ++step) {
            read_flags(h_ref, b.ref_run);
            double fl = 0.0;
            for (int bb = 0; bb < t && price; ++bb)
                if (h_ref[bb]) fl += 2.0 * (double)p.L[bb] * p.L[bb] * p.L[bb];
            tm("k_dgemm<false, false>", fl, 0.0, [&] {
                lrr::launch_dgemm(b.g_refT, t, p.maxL, p.maxL, false, false, st);
            });
            // S = X^T (B X) is symmetric: upper tiles, mirrored
            tm("k_dgemm_sym", hL * fl, 0.0, [&] { lrr::launch_dgemm_sym(b.g_refSG, t, p.maxL, st); });
            // the first step takes X^T X = I: X left the previous iteration orthonormal
            // to rounding (orthogonalised, or rotated by the Jacobi sweeps)
            const bool gid = step == 0;
            if (!gid) tm("k_dgemm_sym", hL * fl, 0.0, [&] { lrr::launch_dgemm_sym(b.g_orthG, t, p.maxL, st); });
            tm("k_ref_rows", 0.0, 0.0, [&] { lrr::launch_ref_rows(b.ref, t, p.maxL, b.it, st, gid); });
            tm("k_ref_E", 0.0, 0.0, [&] { lrr::launch_ref_E(b.ref, t, p.maxL, st, gid); });
            // decide before applying: only quadratically shrinking corrections
            tm("k_ref_update", 0.0, 0.0, [&] { lrr::launch_ref_update(b.ref, t, step, kRefSteps, ref_stop, st); });
            tm("k_dgemm<false, false>", fl, 0.0, [&] {
                lrr::launch_dgemm(b.g_refXE, t, p.maxL, p.maxL, false, false, st);
            });
            tm("k_ref_add", 0.0, 0.0, [&] { lrr::launch_ref_add(b.ref, t, p.maxL, st); });
            tm("k_ref_next", 0.0, 0.0, [&] { lrr::launch_ref_next(b.ref, t, st); });
        }
        // up to two Newton-Schulz steps X <- X (I + (I - X^T X)/2), the second
        // only where the first started above 1e-8; an estimate that is still far
        // from orthonormal before its last step restarts from I
        tm("k_ref_set_run", 0.0, 0.0, [&] { lrr::launch_ref_set_run_ns(b.ref, t, b.eig_run, st); });
        read_flags(h_ref, b.ref_run);
        double f_ns = 0.0;   // the orthogonalisation runs where the refinement did not measure it
        for (int bb = 0; bb < t && price; ++bb)
            if (h_ref[bb]) f_ns += 2.0 * (double)p.L[bb] * p.L[bb] * p.L[bb];
        for (int ns = 0; ns < 2; ++ns) {
            if (ns == 1 && price) {   // the second step runs where the first started above 1e-8
                read_flags(h_ref, b.ref_run);
                f_ns = 0.0;
                for (int bb = 0; bb < t; ++bb)
                    if (h_ref[bb]) f_ns += 2.0 * (double)p.L[bb] * p.L[bb] * p.L[bb];
            }
            tm("k_dgemm_sym", hL * f_ns, 0.0, [&] { lrr::launch_dgemm_sym(b.g_orthG, t, p.maxL, st); });
            tm("k_orth_E", 0.0, 0.0, [&] { lrr::launch_orth_E(b.ref, t, p.maxL, st); });
            tm("k_dgemm<false, false>", f_ns, 0.0, [&] {
                lrr::launch_dgemm(b.g_refXE, t, p.maxL, p.maxL, false, false, st);
            });
            tm("k_ref_add", 0.0, 0.0, [&] { lrr::launch_ref_add(b.ref, t, p.maxL, st); });
            if (ns == 0) tm("k_orth_decide", 0.0, 0.0, [&] { lrr::launch_orth_decide(b.ref, t, st); });
        }
        tm("k_orth_guard", 0.0, 0.0, [&] { lrr::launch_orth_guard(b.ref, t, p.maxL, b.warm, st); });
        tm("k_ref_set_run", 0.0, 0.0, [&] { lrr::launch_ref_set_run_jac(b.ref, t, b.eig_run, st); });
        read_flags(h_ref, b.ref_run);
        double f_jac = 0.0;   // the Jacobi matrix is formed for the blocks that are not clean
        for (int bb = 0; bb < t && price; ++bb)
            if (h_ref[bb]) f_jac += 2.0 * (double)p.L[bb] * p.L[bb] * p.L[bb];
        tm("k_dgemm<false, false>", f_jac, 0.0, [&] {
            lrr::launch_dgemm(b.g_refT, t, p.maxL, p.maxL, false, false, st);
        });
        tm("k_dgemm_sym", hL * f_jac, 0.0, [&] { lrr::launch_dgemm_sym(b.g_Bq, t, p.maxL, st); });
        // block-Jacobi passes for the couplings the refinement left (the whole
        // decomposition on a block's first thresholding step): one persistent launch
        tm("k_jacobi_solve", 0.0, 0.0, [&] {
            lrr::launch_jacobi_solve(b.eig, t, b.jac_offs, b.jac_brounds, b.jac_ctl, b.it, max_sweeps, kMaxTargeted,
                                     p.maxL / p.bs, p.bs, b.need_all, (long)need_total, st);
        });
        tm("k_svt_weights", 0.0, 0.0, [&] { lrr::launch_svt_weights(b.svt, t, p.maxL, b.it, bst, st); });
        tm("k_dgemm<false, true>", f_P, 0.0, [&] {
            lrr::launch_dgemm(b.g_P, t, p.maxl, p.maxl, false, true, st);
        });
        tm("k_dgemm<false, false>", f_J, 0.0, [&] {
            lrr::launch_dgemm(b.g_J, t, n, p.maxl, false, false, st);
        });
        tm("k_lo_mode", 0.0, 0.0, [&] { lrr::launch_lo_mode(b.eig_run, b.warm, b.passes, b.locut, t, st); });
        tm("k_mark_warm", 0.0, 0.0, [&] { lrr::launch_mark_warm(b.eig_run, b.warm, t, st); });
    };
    auto untimed = [](const char*, double, double, auto&& f) { f(); };
    // The J-step with its decisions on the host: which blocks threshold (one
    // read-back), each refinement step (a read-back of the continue flags), each
    // Jacobi pass (a read-back of the check marks, the round plan from the host).
    bool eig_seen = false;   // some block has been decomposed in this solve
    auto host_jstep = [&](double cact) {
        // J-step input and the exact zero test
        timed("k_form_Y", 0.0, 3.0 * n * cact * D, [&] {
            lrr::launch_form_Y(b.Z, b.Y2, b.Y, b.colsq, n, n, c, b.colblk, b.active, b.it, s);
        });
        timed("k_block_fro", 0.0, cact * D, [&] { lrr::launch_block_fro(b.colsq, b.boff, t, bst, b.it, s); });
        timed("k_zero_J", 0.0, 0.0, [&] { lrr::launch_zero_J(b.J, n, n, c, b.colblk, bst, s); });
        timed("k_eig_select", 0.0, 0.0, [&] {
            lrr::launch_eig_select(b.colsq, b.boff, t, b.active, b.svt_run, b.warm, b.eig_run, b.it, prewarm, s);
        });
        // Which blocks decompose is read back until the first eigensolve; from then
        // on the blocks keep thresholding (||Y||_F grows while tau shrinks), so the
        // J-step is launched without the read-back and the device flags gate every
        // kernel (a block that does not run is skipped, bitwise as before).  A
        // profiled solve reads them every iteration to price the products.
        int any_run = 1;
        double f_gram = 0, f_P = 0, f_J = 0;
        if (!eig_seen || prof.on) {
            LRR_HIP(hipMemcpyAsync(h_run, b.eig_run, sizeof(int) * t, hipMemcpyDeviceToHost, s));
            LRR_HIP(hipMemcpyAsync(h_svt, b.svt_run, sizeof(int) * t, hipMemcpyDeviceToHost, s));
            sync();
            any_run = 0;
            for (int bb = 0; bb < t; ++bb) {
                const double l = p.boff[bb + 1] - p.boff[bb];
                if (h_svt[bb]) {
                    f_P += 2.0 * l * l * p.L[bb];
                    f_J += 2.0 * n * l * l;
                }
                if (!h_run[bb]) continue;
                any_run = 1;
                f_gram += 2.0 * l * l * n;
            }
        }
        if (any_run) {
            eig_seen = true;
            // Gram matrix of each block that needs a decomposition (FP64 in every
            // precision form)
            // the symmetric kernel computes the tiles on and above the diagonal
            const double hg = lrr::dgemm_sym_tiles(t, p.maxl) ? 0.5 : 1.0, hL = lrr::dgemm_sym_tiles(t, p.maxL) ? 0.5 : 1.0;
            timed("k_dgemm_sym", hg * f_gram, 0.0, [&] { lrr::launch_dgemm_sym(b.g_gram, t, p.maxl, s); });
            // Newton refinement of the previous iteration's eigenvectors
            timed("k_ref_begin", 0.0, 0.0, [&] { lrr::launch_ref_begin(b.ref, t, p.maxL, b.eig_run, b.warm, s); });
            // the first kBlindSteps steps are launched without reading the flags back
            // (a warm eigensolve takes about three; the device flags decide which
            // blocks a step touches), later ones only while some block continues;
            // a profiled solve reads them every step to price the products
            for (int step = 0; step < kRefSteps; ++step) {
                double fl = 0.0;
                if (step >= kBlindSteps || prof.on) {
                    LRR_HIP(hipMemcpyAsync(h_ref, b.ref_run, sizeof(int) * t, hipMemcpyDeviceToHost, s));
                    sync();
                    int nref = 0;
                    for (int bb = 0; bb < t; ++bb)
                        if (h_ref[bb]) { fl += 2.0 * (double)p.L[bb] * p.L[bb] * p.L[bb]; ++nref; }
                    if (nref == 0) break;
                }
                timed("k_dgemm<false, false>", fl, 0.0, [&] {
                    lrr::launch_dgemm(b.g_refT, t, p.maxL, p.maxL, false, false, s);
                });
                // S = X^T (B X) is symmetric: upper tiles, mirrored
                timed("k_dgemm_sym", hL * fl, 0.0, [&] { lrr::launch_dgemm_sym(b.g_refSG, t, p.maxL, s); });
                // the first step takes X^T X = I (X left the previous iteration orthonormal)
                const bool gid = step == 0;
                if (!gid) timed("k_dgemm_sym", hL * fl, 0.0, [&] { lrr::launch_dgemm_sym(b.g_orthG, t, p.maxL, s); });
                timed("k_ref_rows", 0.0, 0.0, [&] { lrr::launch_ref_rows(b.ref, t, p.maxL, b.it, s, gid); });
                timed("k_ref_E", 0.0, 0.0, [&] { lrr::launch_ref_E(b.ref, t, p.maxL, s, gid); });
                // decide before applying: only quadratically shrinking corrections
                timed("k_ref_update", 0.0, 0.0, [&] { lrr::launch_ref_update(b.ref, t, step, kRefSteps, ref_stop, s); });
                timed("k_dgemm<false, false>", fl, 0.0, [&] {
                    lrr::launch_dgemm(b.g_refXE, t, p.maxL, p.maxL, false, false, s);
                });
                timed("k_ref_add", 0.0, 0.0, [&] { lrr::launch_ref_add(b.ref, t, p.maxL, s); });
                timed("k_ref_next", 0.0, 0.0, [&] { lrr::launch_ref_next(b.ref, t, s); });
            }
            // up to two Newton-Schulz steps X <- X (I + (I - X^T X)/2), the second
            // only where the first started above 1e-8; an estimate that is still far
            // from orthonormal before its last step restarts from I
            double f_L3 = 0.0;
            for (int bb = 0; bb < t; ++bb)
                if (h_run[bb]) f_L3 += 2.0 * (double)p.L[bb] * p.L[bb] * p.L[bb];
            timed("k_ref_set_run", 0.0, 0.0, [&] { lrr::launch_ref_set_run_ns(b.ref, t, b.eig_run, s); });
            double f_ns = f_L3;   // priced by the blocks that still orthogonalise
            if (prof.on) {
                LRR_HIP(hipMemcpyAsync(h_ref, b.ref_run, sizeof(int) * t, hipMemcpyDeviceToHost, s));
                sync();
                f_ns = 0.0;
                for (int bb = 0; bb < t; ++bb)
                    if (h_ref[bb]) f_ns += 2.0 * (double)p.L[bb] * p.L[bb] * p.L[bb];
            }
            for (int ns = 0; ns < 2; ++ns) {
                if (ns == 1 && prof.on) {   // the second step runs where the first started above 1e-8
                    LRR_HIP(hipMemcpyAsync(h_ref, b.ref_run, sizeof(int) * t, hipMemcpyDeviceToHost, s));
                    sync();
                    f_ns = 0.0;
                    for (int bb = 0; bb < t; ++bb)
                        if (h_ref[bb]) f_ns += 2.0 * (double)p.L[bb] * p.L[bb] * p.L[bb];
                }
                timed("k_dgemm_sym", hL * f_ns, 0.0, [&] { lrr::launch_dgemm_sym(b.g_orthG, t, p.maxL, s); });
                timed("k_orth_E", 0.0, 0.0, [&] { lrr::launch_orth_E(b.ref, t, p.maxL, s); });
                timed("k_dgemm<false, false>", f_ns, 0.0, [&] {
                    lrr::launch_dgemm(b.g_refXE, t, p.maxL, p.maxL, false, false, s);
                });
                timed("k_ref_add", 0.0, 0.0, [&] { lrr::launch_ref_add(b.ref, t, p.maxL, s); });
                if (ns == 0) timed("k_orth_decide", 0.0, 0.0, [&] { lrr::launch_orth_decide(b.ref, t, s); });
            }
            timed("k_orth_guard", 0.0, 0.0, [&] { lrr::launch_orth_guard(b.ref, t, p.maxL, b.warm, s); });
            timed("k_ref_set_run", 0.0, 0.0, [&] { lrr::launch_ref_set_run_jac(b.ref, t, b.eig_run, s); });
            double f_jac = f_L3;   // priced by the blocks that form the Jacobi matrix (not clean)
            if (prof.on) {
                LRR_HIP(hipMemcpyAsync(h_ref, b.ref_run, sizeof(int) * t, hipMemcpyDeviceToHost, s));
                sync();
                f_jac = 0.0;
                for (int bb = 0; bb < t; ++bb)
                    if (h_ref[bb]) f_jac += 2.0 * (double)p.L[bb] * p.L[bb] * p.L[bb];
            }
            timed("k_dgemm<false, false>", f_jac, 0.0, [&] {
                lrr::launch_dgemm(b.g_refT, t, p.maxL, p.maxL, false, false, s);
            });
            timed("k_dgemm_sym", hL * f_jac, 0.0, [&] { lrr::launch_dgemm_sym(b.g_Bq, t, p.maxL, s); });
            // block-Jacobi sweeps for the couplings the refinement left (the
            // whole decomposition on a block's first thresholding step)
            const int nb = p.maxL / p.bs;
            timed("k_jacobi_init", 0.0, 0.0, [&] { lrr::launch_jacobi_init(b.eig, t, s); });
            // A pass checks every matrix, then runs a full sweep (nb - 1 circle
            // rounds) or, when the marked index-block pairs fit into at most
            // (nb - 1) / 2 perfect matchings for every block, only those rounds.
            // At most max_sweeps full sweeps and kMaxTargeted targeted passes.
            int full = 0, targeted = 0;
            bool counted = true;   // the pass follows a full sweep (or starts the solve)
            for (;;) {
                // converged matrices are closed here; the loop ends when none is open
                timed("k_lo_rows", 0.0, 0.0, [&] { lrr::launch_lo_rows(b.eig, t, p.maxL, b.it, s, counted); });
                LRR_HIP(hipMemsetAsync(b.eig_any, 0, sizeof(int), s));
                LRR_HIP(hipMemsetAsync(b.need_all, 0, sizeof(int) * need_off[t], s));
                timed("k_jacobi_offcheck", 0.0, 0.0, [&] {
                    lrr::launch_jacobi_check(b.eig, t, p.maxL, b.eig_any, s, p.bs);
                });
                LRR_HIP(hipMemcpyAsync(h_misc, b.eig_any, sizeof(int), hipMemcpyDeviceToHost, s));
                LRR_HIP(hipMemcpyAsync(h_need, b.need_all, sizeof(int) * need_off[t],
                                       hipMemcpyDeviceToHost, s));
                sync();
                if (h_misc[0] == 0 || full == max_sweeps) break;
                ++sweeps_total;
                int rounds = targeted < kMaxTargeted ? 0 : -1;
                for (int bb = 0; bb < t && rounds >= 0; ++bb) {
                    const int nbb = p.L[bb] / p.bs;
                    // the block's schedule holds nbb - 1 rounds
                    const int rb = lrr::host::plan_rounds(h_need + need_off[bb], nbb, std::min((nb - 1) / 2, nbb - 1),
                                               h_sched + sched_off[bb]);
                    rounds = rb < 0 ? -1 : std::max(rounds, rb);
                    block_rounds[bb] = rb;
                }
                if (rounds > 0) {
                    // blocks that need fewer rounds get circle rounds (any perfect matching is valid)
                    for (int bb = 0; bb < t; ++bb) {
                        const int nbb = p.L[bb] / p.bs;
                        for (int r = block_rounds[bb]; r < std::min(rounds, nbb - 1); ++r)
                            for (int P = 0; P < nbb / 2; ++P) {
                                int a0, b0;
                                lrr::rr_pair(nbb, r, P, a0, b0);
                                h_sched[sched_off[bb] + (size_t)r * (nbb / 2) + P] = a0 | (b0 << 16);
                            }
                    }
                    LRR_HIP(hipMemcpyAsync(b.sched_all, h_sched, sizeof(int) * sched_off[t],
                                           hipMemcpyHostToDevice, s));
                    ++targeted;
                    counted = false;
                } else {
                    rounds = nb - 1;
                    ++full;
                    counted = true;
                }
                const bool sched = !counted;
                for (int r = 0; r < rounds; ++r) {
                    timed(p.bs == 16 ? "k_jacobi_pairs<16, 512>" : "k_jacobi_pairs<32, 512>", 0.0, 0.0, [&] {
                        lrr::launch_jacobi_pairs(b.eig, t, p.maxL, p.bs, r, s, sched);
                    });
                    timed(p.bs == 16 ? "k_jacobi_apply<16>" : "k_jacobi_apply<32>", 0.0, 0.0, [&] {
                        lrr::launch_jacobi_apply(b.eig, t, p.maxL, p.bs, r, s, sched);
                    });
                }
            }
            timed("k_svt_weights", 0.0, 0.0, [&] { lrr::launch_svt_weights(b.svt, t, p.maxL, b.it, bst, s); });
            timed("k_dgemm<false, true>", f_P, 0.0, [&] {
                lrr::launch_dgemm(b.g_P, t, p.maxl, p.maxl, false, true, s);
            });
            timed("k_dgemm<false, false>", f_J, 0.0, [&] {
                lrr::launch_dgemm(b.g_J, t, n, p.maxl, false, false, s);
            });
            timed("k_lo_mode", 0.0, 0.0, [&] { lrr::launch_lo_mode(b.eig_run, b.warm, b.passes, b.locut, t, s); });
            timed("k_mark_warm", 0.0, 0.0, [&] { lrr::launch_mark_warm(b.eig_run, b.warm, t, s); });
        }
    };
    // use_graph 1: the Z-/E-step chain of an iteration is captured once per solve
    // (plain and re-anchoring iterations) and replayed with hipGraphLaunch;
    // use_graph 2: one whole iteration (J-step, Z-step, E-step, multipliers, stop
    // test) is captured and replayed, and the host reads the device flags back
    // only every check_every iterations.  Per-kernel timing launches one by one
    // (the same launches).
    const bool chain_timed = prof.wants("k_form_QT") || prof.wants(lrr::xgemm_name(pm.MQ, false, false)) ||
                             prof.wants("k_dgemm<false, false>") || prof.wants(lrr::xgemm_name(pm.MtV, true, false)) ||
                             prof.wants("k_sub_cols") || prof.wants("k_update_Z") || prof.wants("k_r2_decide") ||
                             prof.wants("k_colmax") || prof.wants("k_estep") || prof.wants("k_check") ||
                             prof.wants("k_block_colmax");
    const bool use_graph = device_loop ? (o.use_graph == 2 && !prof.on) : (o.use_graph == 1 && !chain_timed);
    hipGraphExec_t g_plain = nullptr, g_anchor = nullptr;
    hipStream_t cs = use_graph ? ctx_capture_stream(ctx) : nullptr;
    struct GraphGuard {
        hipGraphExec_t* a;
        hipGraphExec_t* b;
        ~GraphGuard() {
            if (*a) (void)hipGraphExecDestroy(*a);
            if (*b) (void)hipGraphExecDestroy(*b);
        }
    } graph_guard{&g_plain, &g_anchor};
    int k = k0;
    for (k = k0; k < k1; ++k) {
        if (hooks && hooks->begin) hooks->begin(k);
        double cact = 0.0;   // columns of blocks still iterating (as of the last read-back)
        for (int bb = 0; bb < t; ++bb) if (h_act[bb]) cact += p.boff[bb + 1] - p.boff[bb];
        const bool anchor = pm.dMQ && k > 0 && k % kAnchorEvery == 0;
        if (!device_loop) host_jstep(cact);
        if (use_graph) {
            hipGraphExec_t& ex = anchor ? g_anchor : g_plain;
            if (!ex) {
                hipGraph_t graph = nullptr;
                LRR_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                if (device_loop) jstep(cs, untimed, cact);
                zstep(cs, anchor, untimed, cact);
                LRR_HIP(hipStreamEndCapture(cs, &graph));
                const hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                LRR_HIP(e);
            }
            LRR_HIP(hipGraphLaunch(ex, s));
        } else {
            if (device_loop) jstep(s, timed, cact);
            zstep(s, anchor, timed, cact);
        }
        if (hooks && hooks->end) hooks->end(k);
        if (!fixed && ((k + 1) % check_every == 0 || k + 1 == p.n_iter)) {
            LRR_HIP(hipMemcpyAsync(h_misc + 1, b.n_active, sizeof(int), hipMemcpyDeviceToHost, s));
            LRR_HIP(hipMemcpyAsync(h_act, b.active, sizeof(int) * t, hipMemcpyDeviceToHost, s));
            LRR_HIP(hipMemcpyAsync(h_misc + 2, &b.jac_ctl->err, sizeof(int), hipMemcpyDeviceToHost, s));
            sync();
            if (h_misc[2] != 0) throw lrr::HipError("eigensolver: a grid barrier wait ran out");
            if (h_misc[1] == 0) { ++k; break; }
        }
    }
    if (prof.on) {
        // operations counted on the device by the Jacobi kernels over this solve
        std::vector<unsigned long long> slots(lrr::kWorkBytes / sizeof(unsigned long long));
        LRR_HIP(hipMemcpyAsync(slots.data(), ctx->dwork, lrr::kWorkBytes, hipMemcpyDeviceToHost, s));
        sync();
        unsigned long long hw[2] = {0, 0};
        for (int kind = 0; kind < 2; ++kind)
            for (int w = 0; w < lrr::kWorkSlots; ++w) hw[kind] += slots[lrr::work_slot(kind, w)];
        const std::string sfx = p.bs == 16 ? "<16" : "<32";
        for (auto& e : prof.entries) {
            if (e.name.rfind("k_jacobi_pairs" + sfx, 0) == 0) e.flops += (double)hw[0];
            if (e.name.rfind("k_jacobi_apply" + sfx, 0) == 0) e.flops += (double)hw[1];
            if (e.name == "k_jacobi_solve") e.flops += (double)(hw[0] + hw[1]);
        }
    }
    res.batch_iters = k - k0;
    res.iters.resize(t); res.rank.resize(t); res.res1.resize(t); res.res2.resize(t);
    std::vector<int> act(t);
    LRR_HIP(hipMemcpyAsync(res.iters.data(), b.iters, sizeof(int) * t, hipMemcpyDeviceToHost, s));
    LRR_HIP(hipMemcpyAsync(res.rank.data(), b.rank, sizeof(int) * t, hipMemcpyDeviceToHost, s));
    LRR_HIP(hipMemcpyAsync(res.res1.data(), b.res1, sizeof(double) * t, hipMemcpyDeviceToHost, s));
    LRR_HIP(hipMemcpyAsync(res.res2.data(), b.res2, sizeof(double) * t, hipMemcpyDeviceToHost, s));
    LRR_HIP(hipMemcpyAsync(act.data(), b.active, sizeof(int) * t, hipMemcpyDeviceToHost, s));
    int jac_err = 0;
    LRR_HIP(hipMemcpyAsync(&jac_err, &b.jac_ctl->err, sizeof(int), hipMemcpyDeviceToHost, s));
    LRR_HIP(hipStreamSynchronize(s));
    if (jac_err != 0) throw lrr::HipError("eigensolver: a grid barrier wait ran out");
    res.converged = true;
    if (!fixed)
        for (int bb = 0; bb < t; ++bb) if (act[bb]) res.converged = false;
    return res;
}

// Run the batched ALM over all blocks; leaves the state in the workspace.
Result run_alm(lrr_ctx* ctx, const Problem& pr, Plan& p, Buffers& b, hipStream_t s, bool with_combine,
               const IterHooks* hooks = nullptr) {
    setup_alm(ctx, pr, p, b, s, with_combine);
    return iterate_alm(ctx, pr, p, b, s, 0, p.n_iter, hooks);
}

// C step of the footnote variant (Section 2.2): the best rank-k approximation
// of diag(J_1, ..., J_t).  Block b's last thresholding step left
// J_b = Y_b W_b diag(g_b) W_b^T with g = 1 - tau_b / sigma on the kept Gram
// eigenvalues sigma^2, so the singular values of J_b are sigma - tau_b and its
// right singular vectors the columns of W_b.  The k largest over all blocks are
// kept (k = 0: max_b rank(J_b); k < 0: all); each block is rebuilt as
// Y_b W_b diag(g_b m_b) W_b^T with the 0/1 mask m_b of its kept triplets, and
// the blocks are scattered to rows and columns perm of Z.  Returns k.
int combine_local(lrr_ctx* ctx, const Problem& pr, Plan& p, Buffers& b, const Result& r, int rank_req,
                  double* Zo, int ldz, hipStream_t s) {
    const int t = p.t, nr = p.nr, n = p.n, c = p.ncols;
    std::vector<double> sched(p.n_iter + 2);
    sched[0] = pr.o.mu0;
    for (size_t k = 1; k < sched.size(); ++k) sched[k] = std::min(pr.o.rho * sched[k - 1], pr.o.mu_max);
    struct Cand { double sv; int b, i; };
    std::vector<Cand> pool;
    std::vector<std::vector<double>> lam(t), h(t);
    for (int bb = 0; bb < t; ++bb) {
        lam[bb].resize(p.L[bb]);
        h[bb].resize(p.L[bb]);
        LRR_HIP(hipMemcpyAsync(lam[bb].data(), b.lam[bb], sizeof(double) * p.L[bb], hipMemcpyDeviceToHost, s));
        LRR_HIP(hipMemcpyAsync(h[bb].data(), b.h[bb], sizeof(double) * p.L[bb], hipMemcpyDeviceToHost, s));
    }
    LRR_HIP(hipStreamSynchronize(s));
    int rmax = 0;
    for (int bb = 0; bb < t; ++bb) {
        if (r.rank[bb] == 0 || r.iters[bb] == 0) continue;   // J_b = 0 (exact zero test)
        rmax = std::max(rmax, r.rank[bb]);
        const double tau = 1.0 / sched[r.iters[bb] - 1];
        const int l = p.boff[bb + 1] - p.boff[bb];
        for (int i = 0; i < l; ++i)
            if (h[bb][i] > 0.0) pool.push_back(Cand{std::sqrt(std::max(lam[bb][i], 0.0)) - tau, bb, i});
    }
    const int total = (int)pool.size();
    const int k = rank_req == 0 ? rmax : (rank_req < 0 ? total : std::min(rank_req, total));
    std::stable_sort(pool.begin(), pool.end(), [](const Cand& x, const Cand& y) { return x.sv > y.sv; });
    std::vector<std::vector<double>> mask(t);
    for (int bb = 0; bb < t; ++bb) mask[bb].assign(p.L[bb], 0.0);
    for (int q = 0; q < k; ++q) mask[pool[q].b][pool[q].i] = 1.0;
    std::vector<GemmDesc> gP(t), gJ(t);
    for (int bb = 0; bb < t; ++bb) {
        const int l = p.boff[bb + 1] - p.boff[bb], L = p.L[bb];
        // the mask goes into h (no longer needed), then Wg <- Wg diag(mask)
        LRR_HIP(hipMemcpyAsync(b.h[bb], mask[bb].data(), sizeof(double) * L, hipMemcpyHostToDevice, s));
        lrr::launch_scale_cols(b.Wg[bb], L, L, L, b.h[bb], s);
        gP[bb] = GemmDesc{b.Wg[bb], b.Wm[bb], b.Pm[bb], l, l, L, L, L, L, 1.0, 0.0, nullptr, nullptr};
        gJ[bb] = GemmDesc{b.Y + (size_t)p.boff[bb] * nr, b.Pm[bb], b.J + (size_t)p.boff[bb] * nr, nr, l, l, nr, L,
                          nr, 1.0, 0.0, nullptr, nullptr};
    }
    LRR_HIP(hipMemcpyAsync(b.g_P, gP.data(), sizeof(GemmDesc) * t, hipMemcpyHostToDevice, s));
    LRR_HIP(hipMemcpyAsync(b.g_J, gJ.data(), sizeof(GemmDesc) * t, hipMemcpyHostToDevice, s));
    LrrProf& prof = ctx->prof;
    prof.run(s, "k_dgemm<false, true>", 0.0, 0.0, [&] { lrr::launch_dgemm(b.g_P, t, p.maxl, p.maxl, false, true, s); });
    prof.run(s, "k_dgemm<false, false>", 0.0, 0.0, [&] { lrr::launch_dgemm(b.g_J, t, nr, p.maxl, false, false, s); });
    for (int j = 0; j < n; ++j) LRR_HIP(hipMemsetAsync(Zo + (size_t)j * ldz, 0, sizeof(double) * n, s));
    lrr::launch_scatter_block_diag(b.J, nr, c, b.colblk, b.boff, b.perm, Zo, ldz, s);
    LRR_HIP(hipStreamSynchronize(s));   // host masks and descriptors go out of scope
    return k;
}

void fill_info(lrr_info* info, const Result& r, int combine_rank) {
    if (!info) return;
    const int t = (int)r.iters.size();
    for (int b = 0; b < t; ++b) {
        if (info->iters) info->iters[b] = r.iters[b];
        if (info->rank) info->rank[b] = r.rank[b];
        if (info->res_primal) info->res_primal[b] = r.res1[b];
        if (info->res_coupling) info->res_coupling[b] = r.res2[b];
    }
    info->batch_iters = r.batch_iters;
    info->combine_rank = combine_rank;
}

template <class F>
lrr_status guarded(lrr_ctx* ctx, F&& f) {
    try {
        return f();
    } catch (const lrr::HipError& e) {
        return fail(ctx, LRR_EDEVICE, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(ctx, LRR_ENOMEM, "device workspace allocation failed");
    }
}

bool input_nonfinite(lrr_ctx* ctx, const double* A, long lda, int m, int n, hipStream_t s) {
    if (!ctx->dflag) LRR_HIP(hipMalloc((void**)&ctx->dflag, 256));
    int* h = static_cast<int*>(ensure_pinned(ctx, 64));
    LRR_HIP(hipMemsetAsync(ctx->dflag, 0, sizeof(int), s));
    lrr::launch_nonfinite(A, lda, m, n, ctx->dflag, s);
    LRR_HIP(hipMemcpyAsync(h, ctx->dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    LRR_HIP(hipStreamSynchronize(s));
    return h[0] != 0;
}

}  // namespace

// ============================================================================
// Reverse mode (dfc_lrr_backward): the state of the unrolled iteration is
// checkpointed every `every` iterations during the forward solve; the reverse
// sweep replays one segment at a time from its checkpoint, recording every
// state and the eigen-decomposition of every thresholding step of the segment,
// and then runs the per-iteration reverse steps (adjoint.hip) backwards
// through it.  dM collects both roles of M (dictionary and the blocks' columns).
// ============================================================================
struct Tape {
    bool valid = false;
    Problem pr{};
    lrr_opts o{};
    std::vector<int> perm, offsets;
    Plan p;
    Buffers b{};
    int K = 0, every = 0, nck = 0, rank0 = 0;
    // host tables
    std::vector<size_t> woff, loff;     // per-block offsets into the packed L x L / L arrays
    size_t sumLL = 0, sumL = 0;
    // device memory
    void* mem = nullptr;
    size_t bytes = 0;
    double *ck = nullptr, *ckW = nullptr;   // checkpoints: states and warm-start eigenvectors
    int* ckWarm = nullptr;
    double *seg = nullptr, *segW = nullptr, *segLam = nullptr;   // the replayed segment
    int* segRun = nullptr;
    double *cZ, *cE, *cY1, *cY2, *cJ, *Zt, *Jt, *Vb, *Wb, *Gm, *Mbar, *Xbar, *lamcol;
    double *Sb, *Cb, *Nb;                   // per-block L x L scratch (packed)
    double *B1, *A1, *A2, *F;               // combine reverse, n x l_1 each
    lrr::BwDesc* bwd = nullptr;
    GemmDesc* gd = nullptr;                 // backward GEMM descriptors
    size_t state_doubles() const { return (size_t)(2 * p.n + 2 * p.m) * p.ncols; }
};

enum BwG {   // indices of the single (all-column) backward GEMM descriptors
    G_MQ64, G_VBMZ, G_MBVZ, G_WB, G_ZTMW, G_MBWQ, G_G1, G_G2, G_MBGM,
    G_H, G_CJ, G_R1, G_B1, G_A1, G_A2, G_F1, G_F2, G_FP, G_F3, G_COUNT
};
enum BwGb { GB_S, GB_C1, GB_C2, GB_T1, GB_T2, GB_Y1, GB_Y2, GB_COUNT };   // per block, t each

static void tape_free(Tape* tp) {
    if (tp && tp->mem) (void)hipFree(tp->mem);
    if (tp) { tp->mem = nullptr; tp->bytes = 0; tp->valid = false; }
}

// Lay out (base == nullptr: size only) the tape memory of plan p.
static size_t tape_layout(Tape& tp, char* base) {
    Arena a{base, 0};
    const Plan& p = tp.p;
    const size_t n = p.n, m = p.m, c = p.ncols, t = p.t;
    const size_t st = tp.state_doubles();
    tp.ck = a.take<double>(st * tp.nck);
    tp.ckW = a.take<double>(tp.sumLL * tp.nck);
    tp.ckWarm = a.take<int>(t * tp.nck);
    tp.seg = a.take<double>(st * tp.every);
    tp.segW = a.take<double>(tp.sumLL * tp.every);
    tp.segLam = a.take<double>(tp.sumL * tp.every);
    tp.segRun = a.take<int>(t * tp.every);
    tp.cZ = a.take<double>(n * c);
    tp.cY2 = a.take<double>(n * c);
    tp.cJ = a.take<double>(n * c);
    tp.Zt = a.take<double>(n * c);
    tp.Jt = a.take<double>(n * c);
    tp.cE = a.take<double>(m * c);
    tp.cY1 = a.take<double>(m * c);
    tp.Vb = a.take<double>(m * c);
    tp.Wb = a.take<double>(m * c);
    tp.Xbar = a.take<double>(m * c);
    tp.Gm = a.take<double>(m * m);
    tp.Mbar = a.take<double>(m * n);
    tp.lamcol = a.take<double>(c);
    tp.Sb = a.take<double>(tp.sumLL);
    tp.Cb = a.take<double>(tp.sumLL);
    tp.Nb = a.take<double>(tp.sumLL);
    const size_t l1 = p.boff[1];
    tp.B1 = a.take<double>(std::max(n, (size_t)p.L[0]) * l1);   // also holds U1^T F (L_1 x l_1)
    tp.A1 = a.take<double>(n * l1);
    tp.A2 = a.take<double>(n * l1);
    tp.F = a.take<double>(n * l1);
    tp.bwd = a.take<lrr::BwDesc>(t);
    tp.gd = a.take<GemmDesc>(G_COUNT + GB_COUNT * t);
    return a.off + 256;
}

// Prepare the tape before a recorded forward solve (allocates its memory).
static void tape_begin(lrr_ctx* ctx, const Problem& pr, const Plan& p) {
    if (!ctx->tape) ctx->tape = new Tape();
    Tape& tp = *ctx->tape;
    tp.valid = false;
    tp.o = pr.o;
    tp.perm.assign(pr.perm, pr.perm + pr.ncols);
    tp.offsets.assign(pr.offsets, pr.offsets + pr.t + 1);
    tp.pr = pr;
    tp.pr.o = tp.o;
    tp.pr.perm = tp.perm.data();
    tp.pr.offsets = tp.offsets.data();
    tp.p = p;
    tp.K = pr.o.fixed_iters;
    tp.every = pr.o.checkpoint_every > 0 ? pr.o.checkpoint_every : 20;
    tp.every = std::min(tp.every, tp.K);
    tp.nck = (tp.K + tp.every - 1) / tp.every;
    tp.woff.assign(p.t, 0);
    tp.loff.assign(p.t, 0);
    tp.sumLL = tp.sumL = 0;
    for (int bb = 0; bb < p.t; ++bb) {
        tp.woff[bb] = tp.sumLL;
        tp.loff[bb] = tp.sumL;
        tp.sumLL += (size_t)p.L[bb] * p.L[bb];
        tp.sumL += p.L[bb];
    }
    const size_t need = tape_layout(tp, nullptr);
    if (need > tp.bytes) {
        tape_free(&tp);
        if (!lrr::try_device_alloc(&tp.mem, need)) throw std::bad_alloc();
        tp.bytes = need;
    }
    tape_layout(tp, static_cast<char*>(tp.mem));
}

// Copy the ALM state (Z, E, Y1, Y2) between the workspace and a packed slot.
static void state_copy(const Tape& tp, const Buffers& b, double* slot, bool save, hipStream_t s) {
    const size_t nc = (size_t)tp.p.n * tp.p.ncols, mc = (size_t)tp.p.m * tp.p.ncols;
    double* parts[4] = {b.Z, b.E, b.Y1, b.Y2};
    const size_t len[4] = {nc, mc, mc, nc};
    size_t off = 0;
    for (int i = 0; i < 4; ++i) {
        if (save) LRR_HIP(hipMemcpyAsync(slot + off, parts[i], sizeof(double) * len[i], hipMemcpyDeviceToDevice, s));
        else LRR_HIP(hipMemcpyAsync(parts[i], slot + off, sizeof(double) * len[i], hipMemcpyDeviceToDevice, s));
        off += len[i];
    }
}

static void eig_copy(const Tape& tp, const Buffers& b, double* W, bool save, hipStream_t s) {
    for (int bb = 0; bb < tp.p.t; ++bb) {
        const size_t LL = (size_t)tp.p.L[bb] * tp.p.L[bb];
        if (save) LRR_HIP(hipMemcpyAsync(W + tp.woff[bb], b.Wm[bb], sizeof(double) * LL, hipMemcpyDeviceToDevice, s));
        else LRR_HIP(hipMemcpyAsync(b.Wm[bb], W + tp.woff[bb], sizeof(double) * LL, hipMemcpyDeviceToDevice, s));
    }
}

// Hooks of the recorded forward: checkpoint the state every `every` iterations.
static IterHooks tape_forward_hooks(Tape& tp, Buffers& b, hipStream_t s) {
    IterHooks h;
    h.begin = [&tp, &b, s](int k) {
        if (k % tp.every) return;
        const int i = k / tp.every;
        state_copy(tp, b, tp.ck + tp.state_doubles() * i, true, s);
        eig_copy(tp, b, tp.ckW + tp.sumLL * i, true, s);
        LRR_HIP(hipMemcpyAsync(tp.ckWarm + (size_t)tp.p.t * i, b.warm, sizeof(int) * tp.p.t,
                               hipMemcpyDeviceToDevice, s));
    };
    return h;
}

// Upload the backward descriptors (after the recorded forward has laid out b).
static void tape_descriptors(Tape& tp, hipStream_t s) {
    const Plan& p = tp.p;
    const Buffers& b = tp.b;
    const int m = p.m, n = p.n, c = p.ncols, t = p.t;
    const double* M = tp.pr.A;
    const int lda = (int)tp.pr.lda;
    std::vector<GemmDesc> g(G_COUNT + GB_COUNT * t, GemmDesc{});
    g[G_MQ64] = GemmDesc{M, b.Q, b.T, m, c, n, lda, n, m, -1.0, 1.0, nullptr, nullptr};
    g[G_VBMZ] = GemmDesc{M, tp.Zt, tp.Vb, m, c, n, lda, n, m, 1.0, 1.0, nullptr, nullptr};
    g[G_MBVZ] = GemmDesc{b.V, tp.Zt, tp.Mbar, m, n, c, m, n, m, 1.0, 1.0, nullptr, nullptr};
    g[G_WB] = GemmDesc{b.K, tp.Vb, tp.Wb, m, c, m, m, m, m, 1.0, 0.0, nullptr, nullptr};
    g[G_ZTMW] = GemmDesc{M, tp.Wb, tp.Zt, n, c, m, lda, m, n, -1.0, 1.0, nullptr, nullptr};
    g[G_MBWQ] = GemmDesc{tp.Wb, b.Q, tp.Mbar, m, n, c, m, n, m, -1.0, 1.0, nullptr, nullptr};
    g[G_G1] = GemmDesc{tp.Wb, b.V, tp.Gm, m, m, c, m, m, m, 1.0, 0.0, nullptr, nullptr};
    g[G_G2] = GemmDesc{b.V, tp.Wb, tp.Gm, m, m, c, m, m, m, 1.0, 1.0, nullptr, nullptr};
    g[G_MBGM] = GemmDesc{tp.Gm, M, tp.Mbar, m, n, m, m, lda, m, -1.0, 1.0, nullptr, nullptr};
    // combine reverse (block 1 spans the projection)
    const int L0 = p.L[0], l1 = p.boff[1];
    double* Gz = tp.Zt;          // dL/dZ with the columns in block order
    g[G_H] = GemmDesc{b.U, Gz, b.H, L0, n, n, n, n, L0, 1.0, 0.0, nullptr, nullptr};
    g[G_CJ] = GemmDesc{b.U, b.H, tp.cJ, n, n, L0, n, L0, n, 1.0, 0.0, nullptr, nullptr};
    g[G_R1] = GemmDesc{tp.Sb, b.Wm[0], tp.Cb, l1, l1, L0, L0, L0, L0, 1.0, 0.0, nullptr, nullptr};
    g[G_B1] = GemmDesc{b.Y, tp.Cb, tp.B1, n, l1, l1, n, L0, n, 1.0, 0.0, nullptr, nullptr};
    g[G_A1] = GemmDesc{b.J, tp.B1, tp.A1, n, l1, n, n, n, n, 1.0, 0.0, nullptr, nullptr};
    g[G_A2] = GemmDesc{Gz, tp.B1, tp.A2, n, l1, n, n, n, n, 1.0, 0.0, nullptr, nullptr};
    g[G_F1] = GemmDesc{Gz, tp.A1, tp.F, n, l1, n, n, n, n, 1.0, 0.0, nullptr, nullptr};
    g[G_F2] = GemmDesc{b.J, tp.A2, tp.F, n, l1, n, n, n, n, 1.0, 1.0, nullptr, nullptr};
    g[G_FP] = GemmDesc{b.U, tp.F, tp.B1, L0, l1, n, n, n, L0, 1.0, 0.0, nullptr, nullptr};
    g[G_F3] = GemmDesc{b.U, tp.B1, tp.F, n, l1, L0, n, L0, n, -1.0, 1.0, nullptr, nullptr};
    std::vector<lrr::BwDesc> bw(t);
    for (int bb = 0; bb < t; ++bb) {
        const int l = p.boff[bb + 1] - p.boff[bb], L = p.L[bb];
        const size_t on = (size_t)p.boff[bb] * n;
        const int* run = b.svt_run + bb;
        double *S = tp.Sb + tp.woff[bb], *C = tp.Cb + tp.woff[bb], *N = tp.Nb + tp.woff[bb];
        const double* W = b.Wm[bb];
        GemmDesc* gb = g.data() + G_COUNT;
        gb[GB_S * t + bb] = GemmDesc{b.Y + on, tp.Jt + on, S, l, l, n, n, n, L, 1.0, 0.0, run, nullptr};
        gb[GB_C1 * t + bb] = GemmDesc{C, W, S, L, L, L, L, L, L, 1.0, 0.0, run, nullptr};
        gb[GB_C2 * t + bb] = GemmDesc{W, S, C, L, L, L, L, L, L, 1.0, 0.0, run, nullptr};
        gb[GB_T1 * t + bb] = GemmDesc{W, N, S, L, L, L, L, L, L, 1.0, 0.0, run, nullptr};
        gb[GB_T2 * t + bb] = GemmDesc{S, W, C, L, L, L, L, L, L, 1.0, 0.0, run, nullptr};
        gb[GB_Y1 * t + bb] = GemmDesc{tp.Jt + on, b.Pm[bb], tp.cZ + on, n, l, l, n, L, n, 1.0, 0.0, run, nullptr};
        gb[GB_Y2 * t + bb] = GemmDesc{b.Y + on, C, tp.cZ + on, n, l, l, n, L, n, 1.0, 1.0, run, nullptr};
        bw[bb] = lrr::BwDesc{W, b.lam[bb], b.Wg[bb], S, C, N, L, l, run};
    }
    LRR_HIP(hipMemcpyAsync(tp.gd, g.data(), sizeof(GemmDesc) * g.size(), hipMemcpyHostToDevice, s));
    LRR_HIP(hipMemcpyAsync(tp.bwd, bw.data(), sizeof(lrr::BwDesc) * t, hipMemcpyHostToDevice, s));
    LRR_HIP(hipStreamSynchronize(s));   // host vectors go out of scope
}

// The reverse sweep.  Writes dM (m x n, ld lddm) if requested and returns dlambda.
static double tape_backward(lrr_ctx* ctx, Tape& tp, const double* dZ, long lddz, double* dM, long lddm, hipStream_t s) {
    Plan& p = tp.p;
    Buffers& b = tp.b;
    const int m = p.m, n = p.n, c = p.ncols, t = p.t;
    const size_t nc = (size_t)n * c, mc = (size_t)m * c;
    GemmDesc* gd = tp.gd;
    GemmDesc* gb = tp.gd + G_COUNT;
    const int* act = b.active;
    auto zero = [&](double* x, size_t len) { LRR_HIP(hipMemsetAsync(x, 0, sizeof(double) * len, s)); };
    zero(tp.cZ, nc); zero(tp.cY2, nc); zero(tp.cJ, nc);
    zero(tp.cE, mc); zero(tp.cY1, mc); zero(tp.Xbar, mc);
    zero(tp.Mbar, (size_t)m * n); zero(tp.lamcol, c);

    // ---- combine reverse: Z = U1 U1^T [J_1 ... J_t], columns put back by perm
    if (tp.rank0 > 0) {
        const int L0 = p.L[0], l1 = p.boff[1];
        lrr::launch_init_iter(b.it, b.mu_sched, tp.K - 1, s);
        lrr::launch_gather_cols(dZ, lddz, tp.Zt, n, n, c, b.perm, s);
        lrr::launch_dgemm(gd + G_H, 1, L0, n, true, false, s);        // H = U1^T dZp
        lrr::launch_dgemm(gd + G_CJ, 1, n, n, false, false, s);       // dJcat = U1 H
        lrr::launch_bw_rdiag(b.Wm[0], b.lam[0], tp.Sb, L0, l1, b.it, s);
        lrr::launch_dgemm(gd + G_R1, 1, l1, l1, false, true, s);      // R1 = W diag(r) W^T
        lrr::launch_dgemm(gd + G_B1, 1, n, l1, false, false, s);      // (J1^+)^T = Y1 R1
        lrr::launch_dgemm(gd + G_A1, 1, n, l1, true, false, s);       // Jcat^T (J1^+)^T
        lrr::launch_dgemm(gd + G_A2, 1, n, l1, true, false, s);       // dZp^T (J1^+)^T
        lrr::launch_dgemm(gd + G_F1, 1, n, l1, false, false, s);      // F = (Pbar + Pbar^T)(J1^+)^T
        lrr::launch_dgemm(gd + G_F2, 1, n, l1, false, false, s);
        lrr::launch_dgemm(gd + G_FP, 1, L0, l1, true, false, s);      // F -= U1 (U1^T F)
        lrr::launch_dgemm(gd + G_F3, 1, n, l1, false, false, s);
        lrr::launch_add_cols(tp.cJ, n, tp.F, n, n, l1, s);
    }

    // ---- segments, last first
    const size_t st = tp.state_doubles();
    bool first = true;
    for (int sg = tp.nck - 1; sg >= 0; --sg) {
        const int k0 = sg * tp.every, k1 = std::min(tp.K, k0 + tp.every);
        // replay [k0, k1) from the checkpoint, recording states and decompositions
        state_copy(tp, b, tp.ck + st * sg, false, s);
        eig_copy(tp, b, tp.ckW + tp.sumLL * sg, false, s);
        LRR_HIP(hipMemcpyAsync(b.warm, tp.ckWarm + (size_t)t * sg, sizeof(int) * t, hipMemcpyDeviceToDevice, s));
        if (p.pm.dMQ) { zero(b.Q, nc); zero(b.MQacc, mc); }
        // the reverse step needs every eigenpair of each Gram matrix, also the
        // ones below tau^2 that the forward solve leaves unresolved
        lrr::launch_init_iter(b.it, b.mu_sched, k0, s, 1);
        IterHooks h;
        h.begin = [&](int k) { state_copy(tp, b, tp.seg + st * (k - k0), true, s); };
        h.end = [&](int k) {
            const int j = k - k0;
            eig_copy(tp, b, tp.segW + tp.sumLL * j, true, s);
            for (int bb = 0; bb < t; ++bb)
                LRR_HIP(hipMemcpyAsync(tp.segLam + tp.sumL * j + tp.loff[bb], b.lam[bb], sizeof(double) * p.L[bb],
                                       hipMemcpyDeviceToDevice, s));
            LRR_HIP(hipMemcpyAsync(tp.segRun + (size_t)t * j, b.svt_run, sizeof(int) * t, hipMemcpyDeviceToDevice, s));
        };
        iterate_alm(ctx, tp.pr, p, b, s, k0, k1, &h);

        for (int k = k1 - 1; k >= k0; --k) {
            const int j = k - k0;
            const double* Z0 = tp.seg + st * j;
            const double* E0 = Z0 + nc;
            const double* Y10 = E0 + mc;
            const double* Y20 = Y10 + mc;
            lrr::launch_init_iter(b.it, b.mu_sched, k, s);
            eig_copy(tp, b, tp.segW + tp.sumLL * j, false, s);
            for (int bb = 0; bb < t; ++bb)
                LRR_HIP(hipMemcpyAsync(b.lam[bb], tp.segLam + tp.sumL * j + tp.loff[bb], sizeof(double) * p.L[bb],
                                       hipMemcpyDeviceToDevice, s));
            LRR_HIP(hipMemcpyAsync(b.svt_run, tp.segRun + (size_t)t * j, sizeof(int) * t, hipMemcpyDeviceToDevice, s));
            // recompute the iteration's intermediates (FP64)
            lrr::launch_form_Y(Z0, Y20, b.Y, b.colsq, n, n, c, b.colblk, act, b.it, s);
            lrr::launch_bw_wg(tp.bwd, t, p.maxL, b.it, s);
            lrr::launch_dgemm(b.g_P, t, p.maxl, p.maxl, false, true, s);
            lrr::launch_dgemm(b.g_J, t, n, p.maxl, false, false, s);
            lrr::launch_zero_norun(b.J, n, n, c, b.colblk, b.svt_run, act, s);
            lrr::launch_form_QT(b.J, Y20, b.Q, nullptr, n, n, b.X, E0, Y10, b.T, m, m, c, b.colblk, act, b.it, s);
            lrr::launch_dgemm(gd + G_MQ64, 1, m, c, false, false, s);
            lrr::launch_dgemm(b.g_KV, t, m, p.maxl, false, false, s);
            // reverse step
            lrr::launch_bw_estep(E0, b.V, tp.cE, tp.cY1, tp.Vb, tp.lamcol, m, m, c, b.colblk, act, b.it,
                                 tp.pr.lam, s);
            lrr::launch_bw_zt(tp.cZ, tp.cY2, first ? tp.cJ : nullptr, tp.Zt, tp.Jt, n, n, c, b.colblk, act, b.it, s);
            first = false;
            lrr::launch_dgemm(gd + G_VBMZ, 1, m, c, false, false, s);     // Vbar += M Zt
            lrr::launch_dgemm(gd + G_MBVZ, 1, m, n, false, true, s);      // dM += V Zt^T
            lrr::launch_dgemm(gd + G_WB, 1, m, c, false, false, s);       // Wb = K^{-1} Vbar
            lrr::launch_dgemm(gd + G_ZTMW, 1, n, c, true, false, s);      // Qbar = Zt - M^T Wb
            lrr::launch_dgemm(gd + G_MBWQ, 1, m, n, false, true, s);      // dM -= Wb Q^T
            lrr::launch_dgemm(gd + G_G1, 1, m, m, false, true, s);        // G = Wb V^T + V Wb^T
            lrr::launch_dgemm(gd + G_G2, 1, m, m, false, true, s);
            lrr::launch_dgemm(gd + G_MBGM, 1, m, n, false, false, s);     // dM -= G M
            lrr::launch_bw_mid(tp.Zt, tp.Jt, tp.cY2, tp.Wb, tp.Xbar, tp.cE, tp.cY1, n, n, m, m, c, b.colblk, act,
                               b.it, s);
            // thresholding reverse per block
            lrr::launch_dgemm(gb + GB_S * t, t, p.maxl, p.maxl, true, false, s);
            lrr::launch_bw_sym(tp.bwd, t, p.maxL, s);
            lrr::launch_dgemm(gb + GB_C1 * t, t, p.maxL, p.maxL, false, false, s);
            lrr::launch_dgemm(gb + GB_C2 * t, t, p.maxL, p.maxL, true, false, s);
            lrr::launch_bw_phi(tp.bwd, t, p.maxL, b.it, s);
            lrr::launch_dgemm(gb + GB_T1 * t, t, p.maxL, p.maxL, false, false, s);
            lrr::launch_dgemm(gb + GB_T2 * t, t, p.maxL, p.maxL, false, true, s);
            lrr::launch_dgemm(gb + GB_Y1 * t, t, n, p.maxl, false, false, s);
            lrr::launch_dgemm(gb + GB_Y2 * t, t, n, p.maxl, false, false, s);
            lrr::launch_zero_norun(tp.cZ, n, n, c, b.colblk, b.svt_run, act, s);
            lrr::launch_bw_final(tp.cZ, tp.cY2, n, n, c, b.colblk, act, b.it, s);
        }
    }
    // the blocks' columns of M, then the outputs
    lrr::launch_scatter_add(tp.Xbar, m, tp.Mbar, m, m, c, b.perm, s);
    if (dM) lrr::launch_copy_cols(tp.Mbar, m, dM, lddm, m, n, s);
    std::vector<double> lc(c);
    LRR_HIP(hipMemcpyAsync(lc.data(), tp.lamcol, sizeof(double) * c, hipMemcpyDeviceToHost, s));
    LRR_HIP(hipStreamSynchronize(s));
    double dl = 0.0;
    for (int j = 0; j < c; ++j) dl += lc[j];
    tp.valid = false;   // the replay overwrote the forward's final state
    return dl;
}

namespace {
}  // namespace

namespace lrr {
lrr_status ctx_fail(lrr_ctx* ctx, lrr_status st, const std::string& msg) { return fail(ctx, st, msg); }
int ctx_device(const lrr_ctx* ctx) { return ctx ? ctx->device : 0; }
void* ctx_seg_workspace(lrr_ctx* ctx, size_t bytes) {
    if (ctx->seg_bytes < bytes) {
        if (ctx->seg_ws) { (void)hipFree(ctx->seg_ws); ctx->seg_ws = nullptr; ctx->seg_bytes = 0; }
        void* p = nullptr;
        if (!lrr::try_device_alloc(&p, bytes)) throw std::bad_alloc();
        ctx->seg_ws = p;
        ctx->seg_bytes = bytes;
    }
    return ctx->seg_ws;
}
void ctx_timed(lrr_ctx* ctx, hipStream_t s, const char* name, double flops, double bytes,
               const std::function<void()>& f) {
    ctx->prof.run(s, name, flops, bytes, f);
}
void ctx_prof_flush(lrr_ctx* ctx) { ctx->prof.flush(); }
}  // namespace lrr

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* lrr_version(void) { return "dfc-lrr-gfx950 0.1"; }

void lrr_opts_default(lrr_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = LRR_FP64;
    o->solve_form = LRR_SOLVE_AUTO;
    o->mu0 = 1e-6;
    o->rho = 1.1;
    o->mu_max = 1e10;
    o->tol = 1e-8;
    o->max_iter = 1000;
    o->fixed_iters = 0;
    o->check_every = 1;
    o->max_sweeps = 30;
    o->save_for_backward = 0;
    o->checkpoint_every = 20;
    o->use_graph = 1;
    o->eig_block = 0;
}

lrr_status lrr_ctx_create(int device, lrr_ctx** out) {
    if (!out) return fail(nullptr, LRR_EINVAL, "out must not be NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(nullptr, LRR_EDEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(nullptr, LRR_EINVAL, "device index out of range");
    lrr_ctx* c = new lrr_ctx();
    c->device = device;
    if (const char* path = std::getenv("LRR_TUNE_TABLE")) {
        std::vector<lrr::host::TuneEntry> t;
        std::string why;
        if (lrr::host::parse_tune(path, t, why)) c->tune = std::move(t);
    }
    *out = c;
    return LRR_OK;
}

lrr_status lrr_tune_load(lrr_ctx* ctx, const char* path) {
    if (!ctx) return fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    if (!path) { ctx->tune.clear(); return LRR_OK; }
    std::vector<lrr::host::TuneEntry> t;
    std::string why;
    if (!lrr::host::parse_tune(path, t, why)) return fail(ctx, LRR_EINVAL, why);
    ctx->tune = std::move(t);
    return LRR_OK;
}

void lrr_ctx_destroy(lrr_ctx* ctx) {
    if (!ctx) return;
    if (hipSetDevice(ctx->device) == hipSuccess) {
        ctx->prof.release();
        if (ctx->ws) (void)hipFree(ctx->ws);
        if (ctx->seg_ws) (void)hipFree(ctx->seg_ws);
        if (ctx->io_ws) (void)hipFree(ctx->io_ws);
        if (ctx->dflag) (void)hipFree(ctx->dflag);
        if (ctx->dwork) (void)hipFree(ctx->dwork);
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        tape_free(ctx->tape);
        if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    }
    delete ctx->tape;
    delete ctx;
}

const char* lrr_last_error(const lrr_ctx* ctx) {
    if (ctx && !ctx->err.empty()) return ctx->err.c_str();
    return g_last_error.c_str();
}

lrr_status lrr_check_partition(int n, int t, const int* perm, const int* offsets) {
    std::string why;
    lrr_status st = lrr::host::check_partition(n, t, perm, offsets, why);
    if (st != LRR_OK) return fail(nullptr, st, why);
    return LRR_OK;
}

lrr_status lrr_workspace_bytes(int m, int n, int t, const int* offsets, const lrr_opts* opts,
                               size_t* bytes) {
    if (!bytes || !offsets || !opts) return fail(nullptr, LRR_EINVAL, "NULL argument");
    if (m <= 0 || n <= 0 || t <= 0 || t > n) return fail(nullptr, LRR_EINVAL, "bad dimensions");
    Problem pr{};
    pr.m = m; pr.n = n; pr.ncols = n; pr.t = t; pr.offsets = offsets; pr.o = *opts;
    Plan p = make_plan(pr);
    Buffers b{};
    *bytes = layout(p, nullptr, b, 1, true);
    return LRR_OK;
}

static lrr_status lrr_solve_f64(lrr_ctx* ctx, int m, int n, int l, const void* A, int lda, const void* X, int ldx,
                     double lambda, const lrr_opts* opts, void* Z, int ldz, void* E, int lde,
                     lrr_info* info, void* stream) {
    if (!ctx) return fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    if (m <= 0 || n <= 0 || l <= 0) return fail(ctx, LRR_EINVAL, "dimensions must be positive");
    if (!A || !X || !Z) return fail(ctx, LRR_EINVAL, "A, X and Z must not be NULL");
    if (lda < m || ldx < m || ldz < n || (E && lde < m)) return fail(ctx, LRR_EINVAL, "leading dimension too small");
    if (lda >= lrr::kGemmMaxLd || ldx >= lrr::kGemmMaxLd || ldz >= lrr::kGemmMaxLd || (E && lde >= lrr::kGemmMaxLd))
        return fail(ctx, LRR_EINVAL, "leading dimensions must be below 4194304");
    if (!(lambda > 0) || !std::isfinite(lambda)) return fail(ctx, LRR_EINVAL, "lambda must be positive and finite");
    lrr_opts o;
    if (opts) o = *opts; else lrr_opts_default(&o);
    std::string why;
    if (!opts_valid(o, why)) return fail(ctx, LRR_EINVAL, why);
    if (ctx->tape) ctx->tape->valid = false;
    return guarded(ctx, [&]() -> lrr_status {
        LRR_HIP(hipSetDevice(ctx->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (input_nonfinite(ctx, static_cast<const double*>(A), lda, m, n, s) ||
            input_nonfinite(ctx, static_cast<const double*>(X), ldx, m, l, s))
            return fail(ctx, LRR_ENUMERIC, "non-finite value in A or X");
        int offs[2] = {0, l};
        apply_tune(ctx, o, m, n, 1, l);
        Problem pr{m, n, l, 1, static_cast<const double*>(A), lda, static_cast<const double*>(X), ldx,
                   nullptr, offs, lambda, o};
        Plan p = make_plan(pr);
        Buffers b{};
        Result r = run_alm(ctx, pr, p, b, s, false);
        if (p.reduced) {
            // Z = Qm Zr
            GemmDesc gz{b.Qm, b.Z, static_cast<double*>(Z), n, l, p.nr, n, p.nr, ldz, 1.0, 0.0, nullptr, nullptr};
            LRR_HIP(hipMemcpyAsync(b.g_U, &gz, sizeof(GemmDesc), hipMemcpyHostToDevice, s));
            lrr::launch_dgemm(b.g_U, 1, n, l, false, false, s);
        } else {
            lrr::launch_copy_cols(b.Z, n, static_cast<double*>(Z), ldz, n, l, s);
        }
        if (E) lrr::launch_copy_cols(b.E, m, static_cast<double*>(E), lde, m, l, s);
        LRR_HIP(hipStreamSynchronize(s));
        fill_info(info, r, r.rank[0]);
        return r.converged ? LRR_OK : LRR_NOT_CONVERGED;
    });
}

static lrr_status dfc_lrr_solve_f64(lrr_ctx* ctx, int m, int n, const void* M, int ldm, double lambda, int t,
                         const int* perm, const int* offsets, const lrr_opts* opts, void* Z, int ldz,
                         void* S, int lds, lrr_info* info, void* stream) {
    if (!ctx) return fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    if (m <= 0 || n <= 0) return fail(ctx, LRR_EINVAL, "dimensions must be positive");
    if (!M || !Z) return fail(ctx, LRR_EINVAL, "M and Z must not be NULL");
    if (ldm < m || ldz < n || (S && lds < m)) return fail(ctx, LRR_EINVAL, "leading dimension too small");
    if (ldm >= lrr::kGemmMaxLd || ldz >= lrr::kGemmMaxLd || (S && lds >= lrr::kGemmMaxLd))
        return fail(ctx, LRR_EINVAL, "leading dimensions must be below 4194304");
    if (!(lambda > 0) || !std::isfinite(lambda)) return fail(ctx, LRR_EINVAL, "lambda must be positive and finite");
    std::string why;
    if (lrr::host::check_partition(n, t, perm, offsets, why) != LRR_OK) return fail(ctx, LRR_EINVAL, why);
    lrr_opts o;
    if (opts) o = *opts; else lrr_opts_default(&o);
    if (!opts_valid(o, why)) return fail(ctx, LRR_EINVAL, why);
    if (ctx->tape) ctx->tape->valid = false;
    if (o.save_for_backward && o.fixed_iters <= 0)
        return fail(ctx, LRR_EINVAL, "save_for_backward needs fixed_iters > 0 (the unrolled map)");
    return guarded(ctx, [&]() -> lrr_status {
        LRR_HIP(hipSetDevice(ctx->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (input_nonfinite(ctx, static_cast<const double*>(M), ldm, m, n, s))
            return fail(ctx, LRR_ENUMERIC, "non-finite value in M");
        int maxl = 0;
        for (int b = 0; b < t; ++b) maxl = std::max(maxl, offsets[b + 1] - offsets[b]);
        apply_tune(ctx, o, m, n, t, maxl);
        Problem pr{m, n, n, t, static_cast<const double*>(M), ldm, nullptr, 0, perm, offsets, lambda, o};
        Plan p = make_plan(pr);
        Buffers b{};
        IterHooks hooks;
        if (o.save_for_backward) {
            tape_begin(ctx, pr, p);
            hooks = tape_forward_hooks(*ctx->tape, b, s);
        }
        Result r = run_alm(ctx, pr, p, b, s, true, o.save_for_backward ? &hooks : nullptr);
        // C step: U1 = Y_1 W_1 diag(h_1) spans the column space of J_1 (zero
        // columns where sigma <= tau); Z = U1 (U1^T [J_1 ... J_t]), columns put back.
        const int L0 = p.L[0], l0 = p.boff[1];
        const int r1 = r.rank[0];
        double* Zo = static_cast<double*>(Z);
        if (r1 == 0) {
            for (int j = 0; j < n; ++j)
                LRR_HIP(hipMemsetAsync(Zo + (size_t)j * ldz, 0, sizeof(double) * n, s));
        } else {
            // in reduced coordinates U1 = Qm Ur with Ur = Yr W diag(h) and
            // U1^T [J_1 ... J_t] = Ur^T [Jr_1 ... Jr_t]
            const int nr = p.nr;
            double* Uc = p.reduced ? b.Ur : b.U;
            GemmDesc gU{b.Y, b.Wm[0], Uc, nr, L0, l0, nr, L0, nr, 1.0, 0.0, nullptr, nullptr};
            GemmDesc gH{Uc, b.J, b.H, L0, n, nr, nr, nr, L0, 1.0, 0.0, nullptr, nullptr};
            GemmDesc gZ{b.U, b.H, Zo, n, n, L0, n, L0, ldz, 1.0, 0.0, nullptr, b.perm};
            GemmDesc gQU{b.Qm, b.Ur, b.U, n, L0, nr, n, nr, n, 1.0, 0.0, nullptr, nullptr};
            GemmDesc hd[3] = {gU, gH, gZ};
            LRR_HIP(hipMemcpyAsync(b.g_U, &hd[0], sizeof(GemmDesc), hipMemcpyHostToDevice, s));
            LRR_HIP(hipMemcpyAsync(b.g_H, &hd[1], sizeof(GemmDesc), hipMemcpyHostToDevice, s));
            LRR_HIP(hipMemcpyAsync(b.g_Z, &hd[2], sizeof(GemmDesc), hipMemcpyHostToDevice, s));
            if (p.reduced) LRR_HIP(hipMemcpyAsync(b.g_red, &gQU, sizeof(GemmDesc), hipMemcpyHostToDevice, s));
            LrrProf& prof = ctx->prof;
            const int gm = p.pm.comb;
            prof.run(s, "k_dgemm<false, false>", 2.0 * nr * L0 * l0, 0.0,
                     [&] { lrr::launch_dgemm(b.g_U, 1, nr, L0, false, false, s); });
            prof.run(s, "k_scale_cols", 0.0, 2.0 * nr * L0 * sizeof(double),
                     [&] { lrr::launch_scale_cols(Uc, nr, nr, L0, b.h[0], s); });
            prof.run(s, lrr::xgemm_name(gm, true, false), 2.0 * L0 * n * nr, 0.0,
                     [&] { lrr::launch_xgemm(b.g_H, 1, L0, n, true, false, gm, s); });
            if (p.reduced)
                prof.run(s, "k_dgemm<false, false>", 2.0 * n * L0 * nr, 0.0,
                         [&] { lrr::launch_dgemm(b.g_red, 1, n, L0, false, false, s); });
            prof.run(s, lrr::xgemm_name(gm, false, false), 2.0 * n * n * L0, 0.0,
                     [&] { lrr::launch_xgemm(b.g_Z, 1, n, n, false, false, gm, s); });
        }
        if (S) lrr::launch_scatter_cols(b.E, m, static_cast<double*>(S), lds, m, n, b.perm, s);
        if (o.save_for_backward) {
            Tape& tp = *ctx->tape;
            tp.b = b;
            tp.rank0 = r1;
            tape_descriptors(tp, s);
            tp.valid = true;
        }
        LRR_HIP(hipStreamSynchronize(s));
        if (ctx->prof.on) ctx->prof.flush();
        fill_info(info, r, r1);
        return r.converged ? LRR_OK : LRR_NOT_CONVERGED;
    });
}

static lrr_status dfc_lrr_solve_local_f64(lrr_ctx* ctx, int m, int n, const void* M, int ldm, double lambda, int t,
                               const int* perm, const int* offsets, int combine_rank, const lrr_opts* opts,
                               void* Z, int ldz, void* S, int lds, lrr_info* info, void* stream) {
    if (!ctx) return fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    if (m <= 0 || n <= 0) return fail(ctx, LRR_EINVAL, "dimensions must be positive");
    if (!M || !Z) return fail(ctx, LRR_EINVAL, "M and Z must not be NULL");
    if (ldm < m || ldz < n || (S && lds < m)) return fail(ctx, LRR_EINVAL, "leading dimension too small");
    if (ldm >= lrr::kGemmMaxLd || ldz >= lrr::kGemmMaxLd || (S && lds >= lrr::kGemmMaxLd))
        return fail(ctx, LRR_EINVAL, "leading dimensions must be below 4194304");
    if (!(lambda > 0) || !std::isfinite(lambda)) return fail(ctx, LRR_EINVAL, "lambda must be positive and finite");
    std::string why;
    if (lrr::host::check_partition(n, t, perm, offsets, why) != LRR_OK) return fail(ctx, LRR_EINVAL, why);
    lrr_opts o;
    if (opts) o = *opts; else lrr_opts_default(&o);
    if (!opts_valid(o, why)) return fail(ctx, LRR_EINVAL, why);
    if (o.save_for_backward) return fail(ctx, LRR_EINVAL, "the local-dictionary variant has no reverse mode");
    if (ctx->tape) ctx->tape->valid = false;
    return guarded(ctx, [&]() -> lrr_status {
        LRR_HIP(hipSetDevice(ctx->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (input_nonfinite(ctx, static_cast<const double*>(M), ldm, m, n, s))
            return fail(ctx, LRR_ENUMERIC, "non-finite value in M");
        int maxl = 0;
        for (int b = 0; b < t; ++b) maxl = std::max(maxl, offsets[b + 1] - offsets[b]);
        apply_tune(ctx, o, m, n, t, maxl);
        Problem pr{m, n, n, t, static_cast<const double*>(M), ldm, nullptr, 0, perm, offsets, lambda, o, 1};
        Plan p = make_plan(pr);
        Buffers b{};
        Result r = run_alm(ctx, pr, p, b, s, false, nullptr);
        const int k = combine_local(ctx, pr, p, b, r, combine_rank, static_cast<double*>(Z), ldz, s);
        if (S) lrr::launch_scatter_cols(b.E, m, static_cast<double*>(S), lds, m, n, b.perm, s);
        LRR_HIP(hipStreamSynchronize(s));
        if (ctx->prof.on) ctx->prof.flush();
        fill_info(info, r, k);
        return r.converged ? LRR_OK : LRR_NOT_CONVERGED;
    });
}

lrr_status lrr_prof_enable(lrr_ctx* ctx, int on) {
    if (!ctx) return fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    ctx->prof.flush();
    ctx->prof.entries.clear();
    ctx->prof.on = on != 0;
    return LRR_OK;
}

lrr_status lrr_prof_filter(lrr_ctx* ctx, const char* prefix) {
    if (!ctx) return fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    ctx->prof.filter = prefix ? prefix : "";
    return LRR_OK;
}

int lrr_prof_count(const lrr_ctx* ctx) { return ctx ? (int)ctx->prof.entries.size() : 0; }

lrr_status lrr_prof_entry(const lrr_ctx* ctx, int idx, const char** name, double* ms, long long* launches,
                          double* flops, double* bytes) {
    if (!ctx || idx < 0 || idx >= (int)ctx->prof.entries.size()) return LRR_EINVAL;
    const LrrProf::Entry& e = ctx->prof.entries[idx];
    if (name) *name = e.name.c_str();
    if (ms) *ms = e.ms;
    if (launches) *launches = e.launches;
    if (flops) *flops = e.flops;
    if (bytes) *bytes = e.bytes;
    return LRR_OK;
}

lrr_status dfc_lrr_backward(lrr_ctx* ctx, const void* dZ, int lddz, double* dlambda, void* dM, int lddm,
                            void* stream) {
    if (!ctx) return fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    if (!ctx->tape || !ctx->tape->valid)
        return fail(ctx, LRR_ENOTAPE, "no recorded forward pass on this context");
    Tape& tp = *ctx->tape;
    if (!dZ || !dlambda) return fail(ctx, LRR_EINVAL, "dZ and dlambda must not be NULL");
    if (lddz < tp.p.n || (dM && lddm < tp.p.m)) return fail(ctx, LRR_EINVAL, "leading dimension too small");
    if (lddz >= lrr::kGemmMaxLd || (dM && lddm >= lrr::kGemmMaxLd)) return fail(ctx, LRR_EINVAL, "leading dimensions must be below 4194304");
    return guarded(ctx, [&]() -> lrr_status {
        LRR_HIP(hipSetDevice(ctx->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        *dlambda = tape_backward(ctx, tp, static_cast<const double*>(dZ), lddz, static_cast<double*>(dM), lddm, s);
        return LRR_OK;
    });
}

lrr_status lrr_diag_plan_rounds(const int* need, int nb, int cap, int* out, int* rounds) {
    if (!need || !out || !rounds || nb < 2 || nb > 65534 || (nb & 1) || cap < 0) return LRR_EINVAL;
    *rounds = lrr::host::plan_rounds(need, nb, cap, out);
    return LRR_OK;
}

// ---------------------------------------------------------------- FP32 I/O
// The forward entry points with opts.io_type = LRR_IO_FP32: FP32 inputs are
// widened into FP64 copies in the ctx's I/O area, the FP64 entry point runs on
// them, and its FP64 outputs (also in the I/O area) are rounded into the
// caller's FP32 buffers.

static bool io_args_ok(lrr_ctx* ctx, std::initializer_list<std::pair<int, int>> ld_rows) {
    for (const auto& lr : ld_rows)
        if (lr.first < lr.second || lr.first >= lrr::kGemmMaxLd) {
            fail(ctx, LRR_EINVAL, "leading dimension too small or not below 4194304");
            return false;
        }
    return true;
}

static double* io_area(lrr_ctx* ctx, size_t doubles) {
    const size_t bytes = doubles * sizeof(double);
    if (ctx->io_bytes < bytes) {
        if (ctx->io_ws) { (void)hipFree(ctx->io_ws); ctx->io_ws = nullptr; ctx->io_bytes = 0; }
        void* p = nullptr;
        if (!lrr::try_device_alloc(&p, bytes)) throw std::bad_alloc();
        ctx->io_ws = p;
        ctx->io_bytes = bytes;
    }
    return static_cast<double*>(ctx->io_ws);
}

lrr_status lrr_solve(lrr_ctx* ctx, int m, int n, int l, const void* A, int lda, const void* X, int ldx,
                     double lambda, const lrr_opts* opts, void* Z, int ldz, void* E, int lde,
                     lrr_info* info, void* stream) {
    if (!opts || opts->io_type == LRR_IO_FP64 || !ctx || m <= 0 || n <= 0 || l <= 0 || !A || !X || !Z)
        return lrr_solve_f64(ctx, m, n, l, A, lda, X, ldx, lambda, opts, Z, ldz, E, lde, info, stream);
    lrr_opts o = *opts;
    std::string why;
    if (!opts_valid(o, why)) return fail(ctx, LRR_EINVAL, why);
    if (!io_args_ok(ctx, {{lda, m}, {ldx, m}, {ldz, n}, {E ? lde : m, m}})) return LRR_EINVAL;
    o.io_type = LRR_IO_FP64;
    return guarded(ctx, [&]() -> lrr_status {
        LRR_HIP(hipSetDevice(ctx->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const size_t mn = (size_t)m * n, ml = (size_t)m * l, nl = (size_t)n * l;
        double* A64 = io_area(ctx, mn + 2 * ml + nl);
        double* X64 = A64 + mn;
        double* Z64 = X64 + ml;
        double* E64 = Z64 + nl;
        lrr::launch_widen_cols(static_cast<const float*>(A), lda, A64, m, m, n, s);
        lrr::launch_widen_cols(static_cast<const float*>(X), ldx, X64, m, m, l, s);
        const lrr_status st = lrr_solve_f64(ctx, m, n, l, A64, m, X64, m, lambda, &o, Z64, n, E ? E64 : nullptr, m,
                                            info, stream);
        if (st != LRR_OK && st != LRR_NOT_CONVERGED) return st;
        lrr::launch_narrow_cols(Z64, n, static_cast<float*>(Z), ldz, n, l, s);
        if (E) lrr::launch_narrow_cols(E64, m, static_cast<float*>(E), lde, m, l, s);
        LRR_HIP(hipStreamSynchronize(s));
        return st;
    });
}

// dfc_lrr_solve and dfc_lrr_solve_local share the FP32 I/O path
extern "C++" template <typename F>
static lrr_status dfc_io32(lrr_ctx* ctx, int m, int n, const void* M, int ldm, void* Z, int ldz, void* S, int lds,
                           const lrr_opts* opts, void* stream, F&& solve64) {
    lrr_opts o = *opts;
    std::string why;
    if (!opts_valid(o, why)) return fail(ctx, LRR_EINVAL, why);
    if (!io_args_ok(ctx, {{ldm, m}, {ldz, n}, {S ? lds : m, m}})) return LRR_EINVAL;
    o.io_type = LRR_IO_FP64;
    return guarded(ctx, [&]() -> lrr_status {
        LRR_HIP(hipSetDevice(ctx->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const size_t mn = (size_t)m * n, nn = (size_t)n * n;
        double* M64 = io_area(ctx, 2 * mn + nn);
        double* S64 = M64 + mn;
        double* Z64 = S64 + mn;
        lrr::launch_widen_cols(static_cast<const float*>(M), ldm, M64, m, m, n, s);
        const lrr_status st = solve64(M64, &o, Z64, S ? S64 : nullptr);
        if (st != LRR_OK && st != LRR_NOT_CONVERGED) return st;
        lrr::launch_narrow_cols(Z64, n, static_cast<float*>(Z), ldz, n, n, s);
        if (S) lrr::launch_narrow_cols(S64, m, static_cast<float*>(S), lds, m, n, s);
        LRR_HIP(hipStreamSynchronize(s));
        return st;
    });
}

lrr_status dfc_lrr_solve(lrr_ctx* ctx, int m, int n, const void* M, int ldm, double lambda, int t,
                         const int* perm, const int* offsets, const lrr_opts* opts, void* Z, int ldz,
                         void* S, int lds, lrr_info* info, void* stream) {
    if (!opts || opts->io_type == LRR_IO_FP64 || !ctx || m <= 0 || n <= 0 || !M || !Z)
        return dfc_lrr_solve_f64(ctx, m, n, M, ldm, lambda, t, perm, offsets, opts, Z, ldz, S, lds, info, stream);
    return dfc_io32(ctx, m, n, M, ldm, Z, ldz, S, lds, opts, stream,
                    [&](const double* M64, const lrr_opts* o, double* Z64, double* S64) {
                        return dfc_lrr_solve_f64(ctx, m, n, M64, m, lambda, t, perm, offsets, o, Z64, n, S64, m,
                                                 info, stream);
                    });
}

lrr_status dfc_lrr_solve_local(lrr_ctx* ctx, int m, int n, const void* M, int ldm, double lambda, int t,
                               const int* perm, const int* offsets, int combine_rank, const lrr_opts* opts,
                               void* Z, int ldz, void* S, int lds, lrr_info* info, void* stream) {
    if (!opts || opts->io_type == LRR_IO_FP64 || !ctx || m <= 0 || n <= 0 || !M || !Z)
        return dfc_lrr_solve_local_f64(ctx, m, n, M, ldm, lambda, t, perm, offsets, combine_rank, opts, Z, ldz, S,
                                       lds, info, stream);
    return dfc_io32(ctx, m, n, M, ldm, Z, ldz, S, lds, opts, stream,
                    [&](const double* M64, const lrr_opts* o, double* Z64, double* S64) {
                        return dfc_lrr_solve_local_f64(ctx, m, n, M64, m, lambda, t, perm, offsets, combine_rank, o,
                                                       Z64, n, S64, m, info, stream);
                    });
}

}  // extern "C"
