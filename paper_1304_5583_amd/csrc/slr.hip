// SLR-graph construction (Section 4.2.2) on the GPU.
//
//   affinity     W = |Z| + |Z|^T formed once (tiled transpose through LDS), so
//                the affinities of sample i are the contiguous column i of W;
//   neighbours   one workgroup per sample: a most-significant-digit radix
//                selection over the IEEE bit patterns of column i (non-negative
//                doubles order like their bit patterns) finds the n_k-th
//                largest affinity T; the keys above T and the lowest-indexed
//                keys equal to T (ties to the lower index) are gathered into
//                LDS and ordered by a bitonic network (decreasing affinity,
//                ties by index), which is the full ordering's first n_k;
//   Gram         G = M^T M once (FP64 MFMA GEMM) into the buffer W occupied;
//                D_i^T D_i and D_i^T x_i are gathers from G;
//   Lasso        one workgroup per sample: the Lawson-Hanson active set on
//                w^T G_i w - 2 b^T w + alpha 1^T w, w >= 0, with the free set
//                P kept independent (a dependent entering column is pivoted
//                in along its dependence); the gradient over all n_k
//                coordinates is one gathered row of G per free index, the
//                factorisations of G_PP (|P| <= 32) run in LDS with all
//                threads, the triangular solves in one wave with the unknowns
//                in registers;
//   large        samples whose free set outgrows 32 are solved again by a
//                second pass that keeps the Cholesky factor of G_PP in device
//                memory and updates it as indices enter and leave.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <functional>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "../../include/lrr_slr.h"

struct lrr_ctx;   // defined in solver.hip

namespace lrr {
lrr_status ctx_fail(lrr_ctx* ctx, lrr_status st, const std::string& msg);
int ctx_device(const lrr_ctx* ctx);
void* ctx_seg_workspace(lrr_ctx* ctx, size_t bytes);
void ctx_timed(lrr_ctx* ctx, hipStream_t s, const char* name, double flops, double bytes,
               const std::function<void()>& f);
void ctx_prof_flush(lrr_ctx* ctx);
}  // namespace lrr

namespace {

constexpr int kMaxNk = 1024;
constexpr double kTol = 1e-12;       // optimality tolerance relative to the sample's scale
constexpr double kDepTol = 1e-10;    // Cholesky pivot / max diagonal below which a column is dependent
constexpr int kMaxP = 32;            // largest free set (Lasso support) held in LDS
constexpr int kTile = 64;            // affinity transpose tile

// W(r, c) = |Z(r, c)| + |Z(c, r)| (one FP64 addition, so W is exactly symmetric)
__global__ __launch_bounds__(256) void k_slr_affinity(const double* __restrict__ Z, long ldz, int n,
                                                      double* __restrict__ W, long ldw) {
    __shared__ double t[kTile][kTile + 1];
    const int r0 = blockIdx.x * kTile, c0 = blockIdx.y * kTile;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    // t[a][b] = |Z(c0 + a, r0 + b)|: the mirrored tile, read along its columns
    for (int k = ty; k < kTile; k += 4) {
        const int row = c0 + tx, col = r0 + k;
        t[tx][k] = (row < n && col < n) ? fabs(Z[row + (long)col * ldz]) : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < kTile; k += 4) {
        const int row = r0 + tx, col = c0 + k;
        if (row < n && col < n) W[row + (long)col * ldw] = fabs(Z[row + (long)col * ldz]) + t[k][tx];
    }
}

// Digits of the radix selection, most significant first: five of 12 bits and
// one of 4 (bits 63..52, 51..40, 39..28, 27..16, 15..4, 3..0).
__device__ __forceinline__ int digit_shift(int pass) { return pass < 5 ? 52 - 12 * pass : 0; }
__device__ __forceinline__ int digit_bins(int pass) { return pass < 5 ? 4096 : 16; }

// Neighbours of sample i = blockIdx.x from column i of W (entries j != i).
// Invariant of the selection: the keys whose masked bits exceed `prefix`
// number nk - need, and at least `need` keys have masked bits equal to it.
__global__ __launch_bounds__(256) void k_slr_select(const double* __restrict__ W, long ldw, int n, int nk,
                                                    int* __restrict__ nbr) {
    __shared__ unsigned hist[4096];
    __shared__ double skey[kMaxNk];
    __shared__ int sidx[kMaxNk];
    __shared__ int s_bin, s_need, s_cnt, s_gt, s_ties;
    __shared__ int wtot[4];
    const int i = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double* col = W + (long)i * ldw;
    unsigned long long prefix = 0, mask = 0;
    int need = nk;
    bool exact = true;   // false once the prefix alone isolates exactly nk keys (every key >= prefix)
    for (int pass = 0; pass < 6; ++pass) {
        const int shift = digit_shift(pass), nb = digit_bins(pass);
        for (int b = tid; b < nb; b += 256) hist[b] = 0u;
        __syncthreads();
        for (int j = tid; j < n; j += 256) {
            if (j == i) continue;
            const unsigned long long k = (unsigned long long)__double_as_longlong(col[j]);
            if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & (unsigned long long)(nb - 1)], 1u);
        }
        __syncthreads();
        if (wv == 0) {
            // lane l owns bins [lo, hi) counted from the top; the first lane whose
            // inclusive count reaches `need` walks its bins downwards
            const int chunk = (nb + 63) / 64;
            const int hi = nb - lane * chunk, lo = max(0, hi - chunk);
            int sum = 0;
            for (int b = lo; b < hi; ++b) sum += (int)hist[b];
            int incl = sum;
            for (int off = 1; off < 64; off <<= 1) {
                const int v = __shfl_up(incl, off, 64);
                if (lane >= off) incl += v;
            }
            const unsigned long long ball = __ballot(incl >= need);
            const int L = __ffsll((long long)ball) - 1;
            if (lane == L) {
                int above = incl - sum, b = hi - 1;
                for (; b > lo; --b) {
                    if (above + (int)hist[b] >= need) break;
                    above += (int)hist[b];
                }
                s_bin = b;
                s_need = need - above;
                s_cnt = (int)hist[b];
            }
        }
        __syncthreads();
        prefix |= (unsigned long long)s_bin << shift;
        mask |= (unsigned long long)(nb - 1) << shift;
        need = s_need;
        const int cnt = s_cnt;
        __syncthreads();
        if (cnt == need) { exact = false; break; }
    }
    // gather: keys above the threshold in any order, then the `need` lowest
    // indices whose key equals it (exact case), in index order
    if (tid == 0) { s_gt = 0; s_ties = 0; }
    __syncthreads();
    const int n_gt = exact ? nk - need : nk;
    for (int base = 0; base < n; base += 256) {
        const int j = base + tid;
        const bool in = j < n && j != i;
        const double v = in ? col[j] : 0.0;
        const unsigned long long k = (unsigned long long)__double_as_longlong(v);
        const bool gt = in && (exact ? k > prefix : k >= prefix);
        const bool tie = in && exact && k == prefix;
        if (gt) {
            const int slot = atomicAdd(&s_gt, 1);
            skey[slot] = v;
            sidx[slot] = j;
        }
        const unsigned long long bt = __ballot(tie);
        if (lane == 0) wtot[wv] = (int)__popcll(bt);
        __syncthreads();
        int r = s_ties + (int)__popcll(bt & ((1ull << lane) - 1ull));
        for (int q = 0; q < wv; ++q) r += wtot[q];
        if (tie && r < need) {
            skey[n_gt + r] = v;
            sidx[n_gt + r] = j;
        }
        __syncthreads();
        if (tid == 0) s_ties += wtot[0] + wtot[1] + wtot[2] + wtot[3];
        __syncthreads();
    }
    // bitonic network over the nk gathered keys; "before" = larger key, or
    // equal key and smaller index; padding (key -1, below every affinity) sinks
    int P = 1;
    while (P < nk) P <<= 1;
    for (int a = nk + tid; a < P; a += 256) {
        skey[a] = -1.0;
        sidx[a] = INT_MAX;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int st = k >> 1; st > 0; st >>= 1) {
            for (int a = tid; a < P; a += 256) {
                const int b = a ^ st;
                if (b > a) {
                    const bool up = (a & k) == 0;
                    const double ka = skey[a], kb = skey[b];
                    const int ia = sidx[a], ib = sidx[b];
                    const bool b_first = kb > ka || (kb == ka && ib < ia);
                    if (b_first == up) {
                        skey[a] = kb; skey[b] = ka;
                        sidx[a] = ib; sidx[b] = ia;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int a = tid; a < nk; a += 256) nbr[(long)i * nk + a] = sidx[a];
}

// deterministic max over the 256 threads
__device__ double block_max256(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return r;
}

__device__ double block_sum256(double v, double* red) {
    v = lrr::wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}

// (value, index) arg-min over the 256 threads: smaller value wins, ties to the lower index
__device__ void block_argmin256(double v, int i, double* sv, int* si, double& vout, int& iout) {
    sv[threadIdx.x] = v;
    si[threadIdx.x] = i;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double a = sv[threadIdx.x], b = sv[threadIdx.x + w];
            const int ia = si[threadIdx.x], ib = si[threadIdx.x + w];
            if (b < a || (b == a && ib < ia)) { sv[threadIdx.x] = b; si[threadIdx.x] = ib; }
        }
        __syncthreads();
    }
    vout = sv[0];
    iout = si[0];
    __syncthreads();
}

// Cholesky factor (lower, in place, column-major p x p) of the matrix in A; all
// threads take part; returns the last pivot (before the square root), or
// -infinity if an earlier pivot fails the threshold (the factor is then incomplete)
__device__ double chol_lds(double* A, int p, double thr, double* flag) {
    double last = 0.0;
    for (int c = 0; c < p; ++c) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const double piv = A[c + c * p];
            flag[0] = piv;
            if (c + 1 < p && !(piv > thr)) flag[0] = -1.0;
            else A[c + c * p] = piv > 0.0 ? sqrt(piv) : 0.0;
        }
        __syncthreads();
        last = flag[0];
        if (c + 1 < p && !(last > thr)) return -INFINITY;
        if (c + 1 == p) break;
        const double lcc = A[c + c * p];
        for (int r = c + 1 + threadIdx.x; r < p; r += 256) A[r + c * p] /= lcc;
        __syncthreads();
        const int q = p - c - 1;
        for (int e = threadIdx.x; e < q * q; e += 256) {
            const int rr = c + 1 + e % q, cc = c + 1 + e / q;
            if (rr >= cc) A[rr + cc * p] -= A[rr + c * p] * A[cc + c * p];
        }
    }
    __syncthreads();
    return last;
}

// wave 0 only (all 64 lanes active): x = L^-1 r over the leading p <= 64 rows of
// the factor in A (ld = ldA).  Lane q keeps x_q in a register; each row's dot
// product is a wave reduction, so no LDS traffic or barrier is needed inside.
__device__ void forward_w0(const double* A, int ldA, int p, const double* r, double* x) {
    const int lane = threadIdx.x;
    double xl = 0.0;
    for (int q = 0; q < p; ++q) {
        const double part = lrr::wave_sum(lane < q ? A[q + lane * ldA] * xl : 0.0);
        const double xq = (r[q] - part) / A[q + q * ldA];
        if (lane == q) xl = xq;
    }
    if (lane < p) x[lane] = xl;
}

// wave 0 only: x = L^-T y
__device__ void backward_w0(const double* A, int ldA, int p, const double* y, double* x) {
    const int lane = threadIdx.x;
    double xl = 0.0;
    for (int q = p - 1; q >= 0; --q) {
        const double part = lrr::wave_sum((lane > q && lane < p) ? A[lane + q * ldA] * xl : 0.0);
        const double xq = (y[q] - part) / A[q + q * ldA];
        if (lane == q) xl = xq;
    }
    if (lane < p) x[lane] = xl;
}

// non-negative Lasso of sample i = blockIdx.x: the active set of Lawson and
// Hanson in Gram form with the free set kept independent (the same steps as
// the reference solver: entering index = most negative gradient off P; a
// dependent entering column moves along its dependence and swaps out the first
// free weight that reaches zero; the face is then solved, stepping back to the
// first weight that would turn non-positive)
__global__ __launch_bounds__(256) void k_slr_lasso(const double* __restrict__ G, long ldg, int nk, double alpha,
                                                   const int* __restrict__ nbr, double* __restrict__ wout,
                                                   double* __restrict__ obj, int* __restrict__ steps_out,
                                                   double* __restrict__ kkt_out, int* __restrict__ sup_out,
                                                   int* __restrict__ big_list, int* __restrict__ big_count) {
    extern __shared__ char smem[];
    double* g = reinterpret_cast<double*>(smem);
    double* b = g + nk;
    int* nb = reinterpret_cast<int*>(b + nk);
    int* pos = nb + nk;                      // position in the free set, or -1
    __shared__ double A[kMaxP * kMaxP];
    __shared__ double wP[kMaxP], sv[kMaxP], rhs[kMaxP], ytmp[kMaxP];
    __shared__ int P[kMaxP + 1];
    __shared__ double rv[256];
    __shared__ int ri[256];
    __shared__ double red[4], flag[2];
    __shared__ int np_s, state;
    const int i = blockIdx.x;
    const int* my = nbr + (long)i * nk;
    double sc = 1.0, dm = 0.0;
    for (int a = threadIdx.x; a < nk; a += 256) {
        const int q = my[a];
        nb[a] = q;
        b[a] = G[q + (long)i * ldg];
        pos[a] = -1;
        const double d = G[q + (long)q * ldg];
        sc = fmax(sc, fmax(fabs(2.0 * b[a] - alpha), 2.0 * d));
        dm = fmax(dm, d);
    }
    if (threadIdx.x == 0) np_s = 0;
    const double scale = block_max256(sc, red);
    const double dmax = block_max256(dm, red);
    const double tol = kTol * scale, thr = kDepTol * dmax;
    int steps = 0;
    double viol = 0.0;
    int status = 0;                          // 0 running, 1 optimal, 2 gave up, 3 support above kMaxP
    while (status == 0) {
        if (threadIdx.x == 0) state = 0;
        __syncthreads();
        const int p = np_s;
        // gradient g = 2 G w - 2 b + alpha over all coordinates, and the violation
        double v = 0.0, gmin = 0.0;
        int jmin = INT_MAX;
        for (int a = threadIdx.x; a < nk; a += 256) {
            double ga = alpha - 2.0 * b[a];
            const double* row = G + nb[a];
            for (int r = 0; r < p; ++r) ga += 2.0 * wP[r] * row[(long)nb[P[r]] * ldg];
            g[a] = ga;
            if (pos[a] >= 0) v = fmax(v, fabs(ga));
            else {
                v = fmax(v, fmax(0.0, -ga));
                if (ga < gmin || (ga == gmin && ga < 0.0 && a < jmin)) { gmin = ga; jmin = a; }
            }
        }
        viol = block_max256(v, red);
        if (viol <= tol) { status = 1; break; }
        if (++steps > 10 * nk + 20) { status = 2; break; }
        double gj;
        int j;
        block_argmin256(gmin, jmin, rv, ri, gj, j);
        if (!(gj < 0.0)) j = -1;             // only free coordinates violate: solve the face again
        if (j >= 0) {
            if (p + 1 > kMaxP) { status = 3; break; }   // handed to the large-support pass
            // factor G over P + {j}; the last pivot decides dependence
            for (int e = threadIdx.x; e < (p + 1) * (p + 1); e += 256) {
                const int r = e % (p + 1), c = e / (p + 1);
                const int ar = (r < p) ? P[r] : j, ac = (c < p) ? P[c] : j;
                A[e] = G[nb[ar] + (long)nb[ac] * ldg];
            }
            const double last = chol_lds(A, p + 1, thr, flag);
            if (last == -INFINITY) { status = 2; break; }   // the free columns themselves degenerated
            if (!(last > thr)) {
                if (p == 0) { status = 2; break; }    // a zero column cannot have g_j < 0
                // D_j = D_P beta: beta = L^-T (L^-1 G_Pj), where L^-1 G_Pj is row p of the factor
                if (threadIdx.x < 64) {
                    for (int q = threadIdx.x; q < p; q += 64) rhs[q] = A[p + q * (p + 1)];
                }
                __syncthreads();
                if (threadIdx.x < 64) backward_w0(A, p + 1, p, rhs, ytmp);
                __syncthreads();
                if (threadIdx.x == 0) {
                    double t = INFINITY;
                    int out = -1;
                    for (int q = 0; q < p; ++q) {
                        if (ytmp[q] > 0.0) {
                            const double r = wP[q] / ytmp[q];
                            if (r < t || (r == t && P[q] < P[out])) { t = r; out = q; }
                        }
                    }
                    if (out < 0) state = 2;
                    else {
                        for (int q = 0; q < p; ++q) wP[q] -= t * ytmp[q];
                        pos[P[out]] = -1;
                        for (int q = out; q + 1 < p; ++q) { P[q] = P[q + 1]; wP[q] = wP[q + 1]; pos[P[q]] = q; }
                        P[p - 1] = j;
                        wP[p - 1] = t;
                        pos[j] = p - 1;
                        state = 0;
                    }
                }
                __syncthreads();
                if (state == 2) { status = 2; break; }
            } else {
                if (threadIdx.x == 0) {
                    P[p] = j;
                    wP[p] = 0.0;
                    pos[j] = p;
                    np_s = p + 1;
                }
                __syncthreads();
            }
        }
        // face solve on P, stepping back while a weight would turn non-positive
        for (int inner = 0; inner < kMaxP + 1 && np_s > 0; ++inner) {
            const int pp = np_s;
            for (int e = threadIdx.x; e < pp * pp; e += 256) {
                const int r = e % pp, c = e / pp;
                A[e] = G[nb[P[r]] + (long)nb[P[c]] * ldg];
            }
            for (int q = threadIdx.x; q < pp; q += 256) rhs[q] = b[P[q]] - 0.5 * alpha;
            const double lp = chol_lds(A, pp, 0.0, flag);
            if (!(lp > 0.0)) { if (threadIdx.x == 0) state = 2; __syncthreads(); break; }
            __syncthreads();
            if (threadIdx.x < 64) forward_w0(A, pp, pp, rhs, ytmp);
            __syncthreads();
            if (threadIdx.x < 64) backward_w0(A, pp, pp, ytmp, sv);
            __syncthreads();
            if (threadIdx.x == 0) {
                bool allpos = true;
                for (int q = 0; q < pp; ++q) allpos &= sv[q] > 0.0;
                if (allpos) {
                    for (int q = 0; q < pp; ++q) wP[q] = sv[q];
                    state = 1;
                } else {
                    // step towards the face point up to the first weight that reaches
                    // zero; every weight whose ratio attains the step leaves P
                    double t = INFINITY;
                    for (int q = 0; q < pp; ++q)
                        if (sv[q] <= 0.0) {
                            const double den = wP[q] - sv[q];
                            t = fmin(t, den > 0.0 ? wP[q] / den : 0.0);
                        }
                    int c = 0;
                    for (int q = 0; q < pp; ++q) {
                        bool gone = false;
                        if (sv[q] <= 0.0) {
                            const double den = wP[q] - sv[q];
                            gone = (den > 0.0 ? wP[q] / den : 0.0) == t;
                        }
                        const double wn = wP[q] + t * (sv[q] - wP[q]);
                        if (gone || !(wn > 0.0)) pos[P[q]] = -1;
                        else { P[c] = P[q]; wP[c] = wn; pos[P[c]] = c; ++c; }
                    }
                    np_s = c;
                    state = 0;
                }
            }
            __syncthreads();
            if (state != 0) break;
        }
        if (state == 2) { status = 2; break; }
    }
    // weights, optimal objective, statistics
    double ns = 0.0;
    for (int a = threadIdx.x; a < nk; a += 256) {
        const int q = pos[a];
        const double wa = q >= 0 ? wP[q] : 0.0;
        wout[(long)i * nk + a] = wa;
        ns += wa > 0.0 ? 1.0 : 0.0;
    }
    const double nsup = block_sum256(ns, red);
    if (obj) {
        // w^T G w = w^T (g + 2 b - alpha) / 2 with the last gradient of the free set
        double t = 0.0;
        for (int a = threadIdx.x; a < nk; a += 256) {
            const int q = pos[a];
            if (q >= 0) t += wP[q] * (0.5 * (g[a] + 2.0 * b[a] - alpha) - 2.0 * b[a] + alpha);
        }
        const double s = block_sum256(t, red);
        if (threadIdx.x == 0) obj[i] = s + G[i + (long)i * ldg];
    }
    if (threadIdx.x == 0) {
        steps_out[i] = steps;
        kkt_out[i] = status == 1 ? viol / scale : INFINITY;
        sup_out[i] = (int)nsup;
        if (status == 3) big_list[atomicAdd(big_count, 1)] = i;
    }
}

// (value, index) arg-min over the 256 threads through wave shuffles and four
// LDS slots: smaller value wins, ties to the lower index (the same result as
// block_argmin256)
__device__ void block_argmin256_w(double v, int i, double* sv, int* si, double& vout, int& iout) {
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(i, off, 64);
        if (ov < v || (ov == v && oi < i)) { v = ov; i = oi; }
    }
    if ((threadIdx.x & 63) == 0) { sv[threadIdx.x >> 6] = v; si[threadIdx.x >> 6] = i; }
    __syncthreads();
    vout = sv[0];
    iout = si[0];
    for (int w = 1; w < 4; ++w)
        if (sv[w] < vout || (sv[w] == vout && si[w] < iout)) { vout = sv[w]; iout = si[w]; }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Large supports.  A sample whose free set outgrows kMaxP is solved again from
// the start by k_slr_lasso_big with the same steps, one workgroup per sample
// over a fixed set of slots.  Each slot owns, in device memory, two pmax x pmax
// buffers for the Cholesky factor L of G_PP (column-major, ld = pmax; the
// second receives the factor after a removal) and the n_k x n_k columns of G_i
// gathered when their index first enters P.  The factor is kept up to date
// instead of recomputed: an entering index appends the row L^-1 G_Pj and its
// pivot; a leaving index is cut out and the trailing block takes a rank-one
// update with the removed column (Golub and Van Loan, Matrix Computations,
// Section 6.5.4).  z = L^-1 (b_P - alpha/2) is kept as well, so a face solve
// is one backward substitution.

constexpr int kDB = 32;          // diagonal block of the triangular solves
constexpr int kDBld = kDB + 1;   // its LDS leading dimension (odd: no bank conflicts)

__device__ double block_min256(double v, double* red) { return -block_max256(-v, red); }

// the lower part of the diagonal block L[o:o+nb, o:o+nb], four entries per
// thread, loaded into registers (so the loads can be in flight during other
// work) and then written to an LDS block of leading dimension kDBld
__device__ void diag_load(const double* L, long ld, int o, int nb, double (&v)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = threadIdx.x + 256 * u, r = e % kDB, c = e / kDB;
        v[u] = (r < nb && c <= r) ? L[(o + r) + (long)(o + c) * ld] : 0.0;
    }
}
__device__ void diag_store(double* D, const double (&v)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = threadIdx.x + 256 * u;
        D[e % kDB + (e / kDB) * kDBld] = v[u];
    }
}

__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// wave 0: x = Dl^-1 x over nb <= 32 entries (Dl the staged lower block), in
// place.  Column sweep: lane i holds x_i; step q broadcasts x_q and the lanes
// below subtract their column-q entry times it, so a step is a broadcast and
// one FMA, with no reduction.
__device__ void fwd_sweep_w0(const double* D, int nb, double* x) {
    const int lane = threadIdx.x;
    double r = lane < nb ? x[lane] : 0.0;
    const double dinv = lane < nb ? 1.0 / D[lane + lane * kDBld] : 0.0;
    for (int q = 0; q < nb; ++q) {
        const double lq = D[(lane & 31) + q * kDBld];
        const double xq = readlane_d(r, q) * readlane_d(dinv, q);
        if (lane == q) r = xq;
        else if (lane > q && lane < nb) r -= lq * xq;
    }
    if (lane < nb) x[lane] = r;
}

// wave 0: x = Dl^-T x over nb <= 32 entries, in place (row sweep from the bottom)
__device__ void bwd_sweep_w0(const double* D, int nb, double* x) {
    const int lane = threadIdx.x;
    double r = lane < nb ? x[lane] : 0.0;
    const double dinv = lane < nb ? 1.0 / D[lane + lane * kDBld] : 0.0;
    for (int q = nb - 1; q >= 0; --q) {
        const double lq = D[q + (lane & 31) * kDBld];
        const double xq = readlane_d(r, q) * readlane_d(dinv, q);
        if (lane == q) r = xq;
        else if (lane < q) r -= lq * xq;
    }
    if (lane < nb) x[lane] = r;
}

// barrier that orders LDS only: global loads in flight (prefetches) stay in
// flight, and global stores become visible to the workgroup at the next full
// __syncthreads()
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// x[i] -= sum_{c < nc} L[i, c0 + c] x[c0 + c] for rows i in [r0, p), one row per
// thread; the column entries of a batch of 8 are loaded before they are used
__device__ void big_gemv_rows(const double* L, long ld, int p, int r0, int c0, int nc, double* x) {
    for (int i = r0 + threadIdx.x; i < p; i += 256) {
        const double* li = L + i + (long)c0 * ld;
        double t = 0.0;
        int c = 0;
        for (; c + 8 <= nc; c += 8) {
            double e[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) e[u] = li[(long)(c + u) * ld];
#pragma unroll
            for (int u = 0; u < 8; ++u) t += e[u] * x[c0 + c + u];
        }
        for (; c < nc; ++c) t += li[(long)c * ld] * x[c0 + c];
        x[i] -= t;
    }
}

// x = L^-1 x over the entries [k0, p), in place, given the entries [0, k0)
// already solved.  Blocks of kDB: wave 0 solves the staged diagonal block,
// then all threads update the rows below (one row per thread, coalesced down
// the columns) while the next diagonal block's loads are in flight; D holds
// two LDS blocks used in turn.
__device__ void big_forward(const double* L, long ld, int p, int k0, double* x, double* D) {
    const int tid = threadIdx.x;
    if (k0 >= p) return;
    double dv[4];
    diag_load(L, ld, k0, min(kDB, p - k0), dv);
    if (k0 > 0) big_gemv_rows(L, ld, p, k0, 0, k0, x);
    diag_store(D, dv);
    __syncthreads();
    int buf = 0;
    for (int o = k0; o < p; o += kDB) {
        const int nb = min(kDB, p - o);
        if (tid < 64) fwd_sweep_w0(D + buf * kDB * kDBld, nb, x + o);
        __syncthreads();
        const int on = o + nb;
        if (on < p) {
            diag_load(L, ld, on, min(kDB, p - on), dv);
            big_gemv_rows(L, ld, p, on, o, nb, x);
            buf ^= 1;
            diag_store(D + buf * kDB * kDBld, dv);
            __syncthreads();
        }
    }
}

// x = L^-T x over the leading p entries, in place: blocks from the bottom; the
// entries above a solved block take its contribution, one thread per entry (a
// dot product down its column, the block's rows of it loaded at once), while
// the next diagonal block's loads are in flight
__device__ void big_backward(const double* L, long ld, int p, double* x, double* D) {
    const int tid = threadIdx.x;
    if (p <= 0) return;
    double dv[4];
    int o = ((p - 1) / kDB) * kDB;
    diag_load(L, ld, o, p - o, dv);
    diag_store(D, dv);
    __syncthreads();
    int buf = 0;
    for (; o >= 0; o -= kDB) {
        const int nb = min(kDB, p - o);
        if (tid < 64) bwd_sweep_w0(D + buf * kDB * kDBld, nb, x + o);
        __syncthreads();
        if (o > 0) {
            diag_load(L, ld, o - kDB, kDB, dv);
            for (int c = tid; c < o; c += 256) {
                const double* lc = L + o + (long)c * ld;
                double e[kDB];
#pragma unroll
                for (int r = 0; r < kDB; ++r) e[r] = r < nb ? lc[r] : 0.0;
                double t = 0.0;
#pragma unroll
                for (int r = 0; r < kDB; ++r) t += e[r] * x[o + r];
                x[c] -= t;
            }
            buf ^= 1;
            diag_store(D + buf * kDB * kDBld, dv);
            __syncthreads();
        }
    }
}

// appends index j at free position p with weight w0, given y = L^-1 G_Pj and
// the pivot d2 = G_jj - |y|^2 > 0; z gains its entry p
__device__ void big_append(double* L, long ld, int& p, int j, double w0, double d2, const double* y, short* P,
                           double* wP, short* pos, double* z, const double* b, double alpha, double* red) {
    const double piv = sqrt(d2);
    double t = 0.0;
    for (int q = threadIdx.x; q < p; q += 256) {
        L[p + (long)q * ld] = y[q];
        t += y[q] * z[q];
    }
    const double dot = block_sum256(t, red);
    if (threadIdx.x == 0) {
        L[p + (long)p * ld] = piv;
        P[p] = (short)j;
        wP[p] = w0;
        pos[j] = (short)p;
        z[p] = (b[j] - 0.5 * alpha - dot) / piv;
    }
    __syncthreads();
    ++p;
}

// removes free position k: P, wP and pos close the gap, and Lo receives the
// factor of G_PP without row and column k (then L and Lo trade places).  v is
// LDS scratch of pmax entries; z[k ..] is overwritten (the caller refreshes z
// from position k or below).
template <int NU>
__device__ void big_delete(double*& L, double*& Lo, long ld, int& p, int k, short* P, double* wP, short* pos,
                           double* v, double* z) {
    const int tid = threadIdx.x;
    const int pn = p - 1;
    const int leaving = P[k];
    for (int r = k + 1 + tid; r < p; r += 256) v[r - k - 1] = L[r + (long)k * ld];
    // the copy runs over the pn x pn square in batches of 8 entries per thread
    // (loads of a batch in flight together); entries above the diagonal are skipped
    const int tot = pn * pn;
    for (int e0 = 0; e0 < tot; e0 += 256 * 8) {
        double val[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + tid + 256 * u, r = e % pn, c = e / pn;
            val[u] = (e < tot && r >= c) ? L[(r + (r >= k)) + (long)(c + (c >= k)) * ld] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + tid + 256 * u, r = e % pn, c = e / pn;
            if (e < tot && r >= c) Lo[r + (long)c * ld] = val[u];
        }
    }
    short pr[4];
    double wr[4];
    for (int u = 0; u < 4; ++u) {
        const int q = k + tid + 256 * u;
        if (q < pn) { pr[u] = P[q + 1]; wr[u] = wP[q + 1]; }
    }
    __syncthreads();
    for (int u = 0; u < 4; ++u) {
        const int q = k + tid + 256 * u;
        if (q < pn) { P[q] = pr[u]; wP[q] = wr[u]; pos[pr[u]] = (short)q; }
    }
    if (tid == 0) pos[leaving] = -1;
    __syncthreads();
    // Lo33 Lo33^T = L33 L33^T + v v^T, one column at a time.  Thread tid owns rows
    // tid + 256 u and keeps their entries of v in registers; the entry of the next
    // pivot row goes through LDS (two slots used in turn), columns are loaded four
    // steps ahead, and the steps are ordered by LDS-only barriers.  The new pivots
    // wait in dg = z[k ..] (entries the caller recomputes) until the loop ends, so
    // no pivot is overwritten while a prefetch of it may be in flight.
    double* dg = z + k;
    double vr[NU], ring[4][NU], piv[4];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int r = tid + 256 * u;
        vr[u] = (r >= k && r < pn) ? v[r - k] : 0.0;
    }
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int col = k + d;
        piv[d] = col < pn ? Lo[col + (long)col * ld] : 1.0;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int r = tid + 256 * u;
            ring[d][u] = (r > col && r < pn) ? Lo[r + (long)col * ld] : 0.0;
        }
    }
    double* vb = v;                          // vb[(c - k) & 1]: the entry of pivot row c
    for (int c = k; c < pn; c += 4) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const int cc = c + d;
            if (cc < pn) {
                const double vc = vb[(cc - k) & 1], lcc = piv[d];
                const double rr = sqrt(lcc * lcc + vc * vc), cs = rr / lcc, ics = lcc / rr, sn = vc / lcc;
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const int r = tid + 256 * u;
                    if (r > cc && r < pn) {
                        const double ln = (ring[d][u] + sn * vr[u]) * ics;
                        vr[u] = cs * vr[u] - sn * ln;
                        Lo[r + (long)cc * ld] = ln;
                        if (r == cc + 1) vb[(cc + 1 - k) & 1] = vr[u];
                    }
                }
                if (tid == 0) dg[cc - k] = rr;
                const int cn = cc + 4;
                if (cn < pn) {
                    piv[d] = Lo[cn + (long)cn * ld];
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        const int r = tid + 256 * u;
                        ring[d][u] = (r > cn && r < pn) ? Lo[r + (long)cn * ld] : 0.0;
                    }
                }
                lds_barrier();
            }
        }
    }
    __syncthreads();
    for (int c = k + tid; c < pn; c += 256) Lo[c + (long)c * ld] = dg[c - k];
    __syncthreads();
    double* t = L;
    L = Lo;
    Lo = t;
    p = pn;
}

// z = L^-1 (b_P - alpha/2) from position k0 on
__device__ void big_refresh_z(const double* L, long ld, int p, int k0, const short* P, const double* b, double alpha,
                              double* z, double* D) {
    for (int q = k0 + threadIdx.x; q < p; q += 256) z[q] = b[P[q]] - 0.5 * alpha;
    __syncthreads();
    big_forward(L, ld, p, k0, z, D);
}

// the samples in list[0 .. *count), one per workgroup at a time; slot s of
// `scratch` (slot_doubles each) belongs to workgroup s; n_k <= 256 NU
template <int NU>
__global__ __launch_bounds__(256, NU == 2 ? 4 : 3) void k_slr_lasso_big(const double* __restrict__ G, long ldg, int nk, int pmax,
                                                       double alpha, const int* __restrict__ nbr,
                                                       const int* __restrict__ list, const int* __restrict__ count,
                                                       double* __restrict__ scratch, long slot_doubles,
                                                       double* __restrict__ wout, double* __restrict__ obj,
                                                       int* __restrict__ steps_out, double* __restrict__ kkt_out,
                                                       int* __restrict__ sup_out) {
    extern __shared__ char smem[];
    double* b = reinterpret_cast<double*>(smem);
    double* wP = b + nk;
    double* z = wP + pmax;
    double* y = z + pmax;
    int* nb = reinterpret_cast<int*>(y + pmax);
    short* pos = reinterpret_cast<short*>(nb + nk);
    short* P = pos + nk;
    unsigned char* have = reinterpret_cast<unsigned char*>(P + pmax);
    unsigned char* keep = have + nk;
    __shared__ double D[2 * kDB * kDBld];
    __shared__ double rv[4];
    __shared__ int ri[4];
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const long ld = pmax;
    double* L = scratch + (long)blockIdx.x * slot_doubles;
    double* Lo = L + ld * pmax;
    double* Gc = Lo + ld * pmax;             // column a: G_i(:, a) once a has entered P
    const long ldc = (nk + 1) & ~1;          // even, so column pairs are 16-byte aligned
    const int total = *count;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int i = list[item];
        const int* my = nbr + (long)i * nk;
        double sc = 1.0, dm = 0.0;
        for (int a = tid; a < nk; a += 256) {
            const int q = my[a];
            nb[a] = q;
            b[a] = G[q + (long)i * ldg];
            pos[a] = -1;
            have[a] = 0;
            const double d = G[q + (long)q * ldg];
            sc = fmax(sc, fmax(fabs(2.0 * b[a] - alpha), 2.0 * d));
            dm = fmax(dm, d);
        }
        const double scale = block_max256(sc, red);
        const double dmax = block_max256(dm, red);
        const double tol = kTol * scale, thr = kDepTol * dmax;
        int p = 0, steps = 0, status = 0;
        double viol = 0.0;
        double ga[NU];                       // gradient of the coordinates NU tid + u
        while (status == 0) {
            // g = alpha - 2 b + 2 G_i(:, P) w_P: NU consecutive coordinates per thread
            // (16-byte loads down the columns), the columns of a batch of 8 loaded together
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int a = NU * tid + u;
                ga[u] = a < nk ? alpha - 2.0 * b[a] : 0.0;
            }
            const bool mine = NU * tid < nk;
            int r = 0;
            for (; r + 8 <= p; r += 8) {
                double2 e[8][NU / 2];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const double2* col = reinterpret_cast<const double2*>(Gc + (long)P[r + q] * ldc) + (NU / 2) * tid;
#pragma unroll
                    for (int h = 0; h < NU / 2; ++h) e[q][h] = mine ? col[h] : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const double wr = 2.0 * wP[r + q];
#pragma unroll
                    for (int h = 0; h < NU / 2; ++h) {
                        ga[2 * h] += wr * e[q][h].x;
                        ga[2 * h + 1] += wr * e[q][h].y;
                    }
                }
            }
            for (; r < p; ++r) {
                const double wr = 2.0 * wP[r];
                const double2* col = reinterpret_cast<const double2*>(Gc + (long)P[r] * ldc) + (NU / 2) * tid;
#pragma unroll
                for (int h = 0; h < NU / 2; ++h) {
                    const double2 e = mine ? col[h] : make_double2(0.0, 0.0);
                    ga[2 * h] += wr * e.x;
                    ga[2 * h + 1] += wr * e.y;
                }
            }
            double v = 0.0, gmin = 0.0;
            int jmin = INT_MAX;
            for (int u = 0; u < NU; ++u) {
                const int a = NU * tid + u;
                if (a >= nk) continue;
                if (pos[a] >= 0) v = fmax(v, fabs(ga[u]));
                else {
                    v = fmax(v, fmax(0.0, -ga[u]));
                    if (ga[u] < gmin || (ga[u] == gmin && ga[u] < 0.0 && a < jmin)) { gmin = ga[u]; jmin = a; }
                }
            }
            viol = block_max256(v, red);
            if (viol <= tol) { status = 1; break; }
            if (++steps > 10 * nk + 20) { status = 2; break; }
            double gj;
            int j;
            block_argmin256_w(gmin, jmin, rv, ri, gj, j);
            if (!(gj < 0.0)) j = -1;
            if (j >= 0) {
                double* cj = Gc + (long)j * ldc;
                if (!have[j]) {
                    const double* src = G + (long)nb[j] * ldg;
                    for (int a = tid; a < nk; a += 256) cj[a] = src[nb[a]];
                    __syncthreads();
                    if (tid == 0) have[j] = 1;
                }
                for (int q = tid; q < p; q += 256) y[q] = cj[P[q]];
                __syncthreads();
                big_forward(L, ld, p, 0, y, D);
                double t2 = 0.0;
                for (int q = tid; q < p; q += 256) t2 += y[q] * y[q];
                const double d2 = cj[j] - block_sum256(t2, red);
                if (!(d2 > thr)) {
                    // D_j = D_P beta, beta = L^-T y: w_P -= t beta, w_j = t, until the
                    // first weight with beta > 0 reaches zero; that index leaves
                    if (p == 0) { status = 2; break; }
                    big_backward(L, ld, p, y, D);
                    double tb = INFINITY;
                    int ib = INT_MAX;
                    for (int q = tid; q < p; q += 256) {
                        if (y[q] > 0.0) {
                            const double r = wP[q] / y[q];
                            if (r < tb || (r == tb && P[q] < ib)) { tb = r; ib = P[q]; }
                        }
                    }
                    double t;
                    int out;
                    block_argmin256_w(tb, ib, rv, ri, t, out);
                    if (out == INT_MAX) { status = 2; break; }
                    for (int q = tid; q < p; q += 256) wP[q] -= t * y[q];
                    __syncthreads();
                    const int kd = pos[out];
                    big_delete<NU>(L, Lo, ld, p, kd, P, wP, pos, y, z);
                    big_refresh_z(L, ld, p, kd, P, b, alpha, z, D);
                    for (int q = tid; q < p; q += 256) y[q] = cj[P[q]];
                    __syncthreads();
                    big_forward(L, ld, p, 0, y, D);
                    t2 = 0.0;
                    for (int q = tid; q < p; q += 256) t2 += y[q] * y[q];
                    const double d2b = cj[j] - block_sum256(t2, red);
                    if (!(d2b > 0.0)) { status = 2; break; }
                    big_append(L, ld, p, j, t, d2b, y, P, wP, pos, z, b, alpha, red);
                } else {
                    if (p + 1 > pmax) { status = 2; break; }   // more independent columns than rows
                    big_append(L, ld, p, j, 0.0, d2, y, P, wP, pos, z, b, alpha, red);
                }
            }
            // face solve G_PP s = b_P - alpha/2 (s = L^-T z), stepping back while a
            // weight would turn non-positive
            for (int inner = 0; inner < pmax + 1 && p > 0; ++inner) {
                for (int q = tid; q < p; q += 256) y[q] = z[q];
                __syncthreads();
                big_backward(L, ld, p, y, D);
                double bad = 0.0;
                for (int q = tid; q < p; q += 256) bad = fmax(bad, y[q] > 0.0 ? 0.0 : 1.0);
                if (block_max256(bad, red) == 0.0) {
                    for (int q = tid; q < p; q += 256) wP[q] = y[q];
                    __syncthreads();
                    break;
                }
                double tq = INFINITY;
                for (int q = tid; q < p; q += 256) {
                    if (y[q] <= 0.0) {
                        const double den = wP[q] - y[q];
                        tq = fmin(tq, den > 0.0 ? wP[q] / den : 0.0);
                    }
                }
                const double t = block_min256(tq, red);
                if (!(t < INFINITY)) { status = 2; break; }     // the face solution is not finite
                double kmin = (double)p;
                for (int q = tid; q < p; q += 256) {
                    bool gone = false;
                    if (y[q] <= 0.0) {
                        const double den = wP[q] - y[q];
                        gone = (den > 0.0 ? wP[q] / den : 0.0) == t;
                    }
                    const double wn = wP[q] + t * (y[q] - wP[q]);
                    const bool kp = !(gone || !(wn > 0.0));
                    keep[q] = kp ? 1 : 0;
                    if (kp) wP[q] = wn;
                    else kmin = fmin(kmin, (double)q);
                }
                const int k0 = (int)block_min256(kmin, red);
                for (int q = p - 1; q >= k0; --q)
                    if (!keep[q]) big_delete<NU>(L, Lo, ld, p, q, P, wP, pos, y, z);
                if (p > 0) big_refresh_z(L, ld, p, k0, P, b, alpha, z, D);
            }
        }
        // weights, optimal objective, statistics
        double ns = 0.0, to = 0.0;
        for (int u = 0; u < NU; ++u) {
            const int a = NU * tid + u;
            if (a >= nk) continue;
            const int q = pos[a];
            const double wa = q >= 0 ? wP[q] : 0.0;
            wout[(long)i * nk + a] = wa;
            ns += wa > 0.0 ? 1.0 : 0.0;
            if (q >= 0) to += wP[q] * (0.5 * (ga[u] + 2.0 * b[a] - alpha) - 2.0 * b[a] + alpha);
        }
        const double nsup = block_sum256(ns, red);
        const double s = block_sum256(to, red);
        if (tid == 0) {
            if (obj) obj[i] = s + G[i + (long)i * ldg];
            steps_out[i] = steps;
            kkt_out[i] = status == 1 ? viol / scale : INFINITY;
            sup_out[i] = (int)nsup;
        }
        __syncthreads();
    }
}

unsigned grid1(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" lrr_status lrr_slr_graph(lrr_ctx* ctx, int m, int n, const void* Mv, int ldm, const void* Zv, int ldz,
                                    int nk, double alpha, int* nbr, double* w, double* obj, lrr_slr_info* info,
                                    void* stream) {
    if (!ctx) return lrr::ctx_fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    if (m < 1 || n < 2 || !Mv || !Zv || ldm < m || ldz < n || !nbr || !w)
        return lrr::ctx_fail(ctx, LRR_EINVAL, "bad M / Z / output arguments");
    if (ldm >= lrr::kGemmMaxLd || ldz >= lrr::kGemmMaxLd) return lrr::ctx_fail(ctx, LRR_EINVAL, "leading dimensions must be below 4194304");
    if (nk < 1 || nk > n - 1 || nk > kMaxNk) return lrr::ctx_fail(ctx, LRR_EINVAL, "nk must lie in [1, min(n-1, 1024)]");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return lrr::ctx_fail(ctx, LRR_EINVAL, "alpha must be positive");
    const double* M = static_cast<const double*>(Mv);
    const double* Z = static_cast<const double*>(Zv);
    hipStream_t s = static_cast<hipStream_t>(stream);
    try {
        if (hipSetDevice(lrr::ctx_device(ctx)) != hipSuccess)
            return lrr::ctx_fail(ctx, LRR_EDEVICE, "hipSetDevice failed");
        // workspace: W, then G (n x n, one buffer); per-sample step counts, violations and
        // support sizes; the list of samples for the large-support pass and its length;
        // one GEMM descriptor
        auto up = [](size_t o) { return (o + 255) & ~size_t(255); };
        const size_t offG = 0, offS = offG + sizeof(double) * (size_t)n * n;
        const size_t offK = up(offS + sizeof(int) * (size_t)n);
        const size_t offU = up(offK + sizeof(double) * (size_t)n);
        const size_t offL = up(offU + sizeof(int) * (size_t)n);
        const size_t offC = up(offL + sizeof(int) * (size_t)n);
        const size_t offD = up(offC + sizeof(int));
        const size_t bytes = offD + sizeof(lrr::GemmDesc);
        char* base = static_cast<char*>(lrr::ctx_seg_workspace(ctx, bytes));
        double* G = reinterpret_cast<double*>(base + offG);
        int* steps = reinterpret_cast<int*>(base + offS);
        double* kkt = reinterpret_cast<double*>(base + offK);
        int* sup = reinterpret_cast<int*>(base + offU);
        int* big_list = reinterpret_cast<int*>(base + offL);
        int* big_count = reinterpret_cast<int*>(base + offC);
        lrr::GemmDesc* gd = reinterpret_cast<lrr::GemmDesc*>(base + offD);

        const unsigned tiles = (unsigned)((n + kTile - 1) / kTile);
        lrr::ctx_timed(ctx, s, "k_slr_affinity", 0.0, 24.0 * n * (double)n, [&] {
            hipLaunchKernelGGL(k_slr_affinity, dim3(tiles, tiles), dim3(256), 0, s, Z, (long)ldz, n, G, (long)n);
        });
        lrr::ctx_timed(ctx, s, "k_slr_select", 0.0, 8.0 * n * (double)n, [&] {
            hipLaunchKernelGGL(k_slr_select, dim3(n), dim3(256), 0, s, G, (long)n, n, nk, nbr);
        });
        lrr::GemmDesc h{M, M, G, n, n, m, ldm, ldm, n, 1.0, 0.0, nullptr, nullptr};
        LRR_HIP(hipMemcpyAsync(gd, &h, sizeof(h), hipMemcpyHostToDevice, s));
        lrr::ctx_timed(ctx, s, "k_dgemm<true, false>", 2.0 * n * (double)n * m, 0.0,
                       [&] { lrr::launch_dgemm(gd, 1, n, n, true, false, s); });
        LRR_HIP(hipMemsetAsync(big_count, 0, sizeof(int), s));
        const size_t lds = (size_t)nk * (2 * sizeof(double) + 2 * sizeof(int));
        lrr::ctx_timed(ctx, s, "k_slr_lasso", 0.0, 0.0, [&] {
            hipLaunchKernelGGL(k_slr_lasso, dim3(n), dim3(256), lds, s, G, (long)n, nk, alpha, nbr, w, obj, steps,
                               kkt, sup, big_list, big_count);
        });
        LRR_HIP(hipGetLastError());
        int nbig = 0;
        LRR_HIP(hipMemcpyAsync(&nbig, big_count, sizeof(int), hipMemcpyDeviceToHost, s));
        LRR_HIP(hipStreamSynchronize(s));
        if (nbig > 0) {
            // supports above kMaxP: independent free sets hold at most min(m, nk) indices
            const int pmax = std::min(m, nk);
            const size_t lds_big = sizeof(double) * ((size_t)nk + 3 * (size_t)pmax) + sizeof(int) * (size_t)nk +
                                   sizeof(short) * ((size_t)nk + pmax) + (size_t)nk + pmax;
            const auto kern = nk <= 512 ? k_slr_lasso_big<2> : k_slr_lasso_big<4>;
            int per_cu = 0, cus = 0;
            LRR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds_big));
            LRR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, lrr::ctx_device(ctx)));
            long slots = std::min<long>(nbig, std::max(1, per_cu) * (long)std::max(1, cus));
            const long slot_doubles = ((2L * pmax * pmax + (long)nk * ((nk + 1) & ~1)) + 31) / 32 * 32;
            void* scratch = nullptr;
            while (slots >= 1 && !lrr::try_device_alloc(&scratch, sizeof(double) * slot_doubles * slots)) slots /= 2;
            if (!scratch) return lrr::ctx_fail(ctx, LRR_ENOMEM, "SLR-graph large-support workspace allocation failed");
            struct Free {
                void* p;
                ~Free() { (void)hipFree(p); }
            } release{scratch};
            lrr::ctx_timed(ctx, s, "k_slr_lasso_big", 0.0, 0.0, [&] {
                hipLaunchKernelGGL(kern, dim3((unsigned)slots), dim3(256), lds_big, s, G, (long)n, nk,
                                   pmax, alpha, nbr, big_list, big_count, static_cast<double*>(scratch),
                                   slot_doubles, w, obj, steps, kkt, sup);
            });
            LRR_HIP(hipGetLastError());
            LRR_HIP(hipStreamSynchronize(s));
        }
        std::vector<int> hs(n), hu(n);
        std::vector<double> hk(n);
        LRR_HIP(hipMemcpyAsync(hs.data(), steps, sizeof(int) * n, hipMemcpyDeviceToHost, s));
        LRR_HIP(hipMemcpyAsync(hk.data(), kkt, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        LRR_HIP(hipMemcpyAsync(hu.data(), sup, sizeof(int) * n, hipMemcpyDeviceToHost, s));
        LRR_HIP(hipStreamSynchronize(s));
        lrr::ctx_prof_flush(ctx);
        int smax = 0, nc = 0, umax = 0;
        double kmax = 0.0;
        for (int i = 0; i < n; ++i) {
            smax = std::max(smax, hs[i]);
            umax = std::max(umax, hu[i]);
            if (hk[i] <= kTol) kmax = std::max(kmax, hk[i]);
            if (!(hk[i] <= kTol)) ++nc;
        }
        if (info) {
            info->max_steps = smax;
            info->not_converged = nc;
            info->max_kkt = kmax;
            info->large_support = nbig;
            info->max_support = umax;
        }
        return nc ? LRR_NOT_CONVERGED : LRR_OK;
    } catch (const lrr::HipError& e) {
        return lrr::ctx_fail(ctx, LRR_EDEVICE, e.msg);
    } catch (const std::bad_alloc&) {
        return lrr::ctx_fail(ctx, LRR_ENOMEM, "SLR-graph workspace allocation failed");
    }
}
