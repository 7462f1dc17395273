// Subspace segmentation from a coefficient matrix (Section 4.1.2), on the GPU.
//
// Pipeline (the choices are listed in include/lrr_segment.h):
//   range of Z     Y = Z Omega (sketch) or Y = Z; eigen-decomposition of Y^T Y
//                  gives an orthonormal basis Q of range(Y) (one Newton-Schulz
//                  step restores orthonormality to rounding);
//   left vectors   B = Z^T Q, eigen-decomposition of B^T B = Q^T Z Z^T Q gives
//                  the singular values of Z and U = Q W (the rank cut is taken
//                  on sigma = sqrt(eigenvalue));
//   affinity       A = U_keep U_keep^T (MFMA FP64 GEMM), then |A| scaled by
//                  D^-1/2 on both sides in two passes over HBM;
//   embedding      Chebyshev-filtered block subspace iteration with a
//                  Rayleigh-Ritz step on L (FP64 GEMMs with the nk x nk
//                  affinity), converged when the k leading Ritz vectors satisfy
//                  |L x - theta x| <= tol;
//   k-means        farthest-point seeding (one distance pass and one arg-max
//                  per centre, chained on the device), Lloyd steps with
//                  one thread per point (assignment) and one per (cluster,
//                  coordinate) (centre update, a sequential sum in point order,
//                  so the result does not depend on scheduling);
//   labels         renumbered by first appearance in one workgroup.
// The symmetric eigenproblems use the block-Jacobi kernels of the solver from
// the identity.  Every product is FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "../../include/lrr_segment.h"

struct lrr_ctx;   // defined in solver.hip

namespace lrr {
lrr_status ctx_fail(lrr_ctx* ctx, lrr_status st, const std::string& msg);
int ctx_device(const lrr_ctx* ctx);
void* ctx_seg_workspace(lrr_ctx* ctx, size_t bytes);
void ctx_timed(lrr_ctx* ctx, hipStream_t s, const char* name, double flops, double bytes,
               const std::function<void()>& f);
void ctx_prof_flush(lrr_ctx* ctx);   // after the stream is synchronised
}  // namespace lrr

namespace {

using lrr::EigDesc;
using lrr::GemmDesc;

constexpr int kSketchExtra = 16;       // sketch columns beyond the rank bound
constexpr double kRangeCut = 1e-14;    // eigenvalue cut of Y^T Y for the range basis
constexpr double kEmbedTol = 2e-10;    // residual |L x - theta x| of the embedding
constexpr int kEmbedMaxOuter = 400;    // filter + Rayleigh-Ritz rounds
constexpr double kSpread = 1e5;        // largest amplification ratio of one filter
constexpr int kMaxDegree = 16;
constexpr int kKmeansMaxIter = 300;
constexpr int kMaxDirect = 8192;       // largest n without a sketch
constexpr int kBs = 16;                // Jacobi block size (L is a multiple of 2 kBs)
constexpr int kMaxK = 1024;
constexpr int kSeedParts = 1024;       // workgroups of one seeding step

int round_up(int x, int a) { return ((x + a - 1) / a) * a; }

// SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014) on the
// counter seed + (i + 1) * golden gamma: a reproducible stream for the sketch
// and the starting block, uniform on [-1, 1).
__device__ __forceinline__ double sm64_uniform(unsigned long long seed, unsigned long long i) {
    unsigned long long z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(256) void k_fill_uniform(double* __restrict__ A, long ld, int rows, int cols,
                                                      unsigned long long seed) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long)rows * cols) return;
    const int i = (int)(idx % rows), j = (int)(idx / rows);
    A[i + j * ld] = sm64_uniform(seed, (unsigned long long)idx);
}

__global__ __launch_bounds__(256) void k_fill_zero(double* __restrict__ A, long n) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx < n) A[idx] = 0.0;
}

// eigenvalue order (descending, ties by index) and the count above a relative
// cut: use_sqrt compares sqrt(lam_i) > cut * sqrt(lam_max), else lam_i > cut * lam_max
__global__ __launch_bounds__(1024) void k_sort_desc(const double* __restrict__ lam, int l, int* __restrict__ idx,
                                                    int* __restrict__ count, double cut, int use_sqrt) {
    __shared__ double red[1024];
    double mx = 0.0;
    for (int i = threadIdx.x; i < l; i += 1024) mx = fmax(mx, lam[i]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const double lmax = red[0];
    __syncthreads();
    int cnt = 0;
    for (int j = threadIdx.x; j < l; j += 1024) {
        const double v = lam[j];
        int rank = 0;
        for (int i = 0; i < l; ++i) {
            const double u = lam[i];
            rank += (u > v || (u == v && i < j)) ? 1 : 0;
        }
        idx[rank] = j;
        const bool keep = use_sqrt ? (sqrt(fmax(v, 0.0)) > cut * sqrt(fmax(lmax, 0.0))) : (v > cut * lmax);
        cnt += keep ? 1 : 0;
    }
    __shared__ int csum;
    if (threadIdx.x == 0) csum = 0;
    __syncthreads();
    if (cnt) atomicAdd(&csum, cnt);
    __syncthreads();
    if (threadIdx.x == 0) count[0] = csum;
}

// out[:, j] = W[0:rows, idx[j]] * (scaled ? 1/sqrt(lam[idx[j]]) (0 if lam <= 0) : 1)
__global__ __launch_bounds__(256) void k_pick_cols(const double* __restrict__ W, long ldw,
                                                   const double* __restrict__ lam, const int* __restrict__ idx,
                                                   int rows, int scaled, double* __restrict__ out, long ldo) {
    const int j = blockIdx.x;
    const int src = idx[j];
    double sc = 1.0;
    if (scaled) sc = lam[src] > 0.0 ? 1.0 / sqrt(lam[src]) : 0.0;
    for (int i = threadIdx.x; i < rows; i += 256) out[i + (long)j * ldo] = W[i + (long)src * ldw] * sc;
}

// out[i, :] = A[rows[i], :]
__global__ __launch_bounds__(256) void k_gather_rows(const double* __restrict__ A, long lda,
                                                     const int* __restrict__ rows, int nr, int ncols,
                                                     double* __restrict__ out, long ldo) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long)nr * ncols) return;
    const int i = (int)(idx % nr), j = (int)(idx / nr);
    out[i + j * ldo] = A[rows[i] + j * lda];
}

// degree of column j of |A| (A symmetric): s_j = 1/sqrt(sum_i |a_ij|), 1 for a zero sum
__global__ __launch_bounds__(256) void k_absdeg(const double* __restrict__ A, long ld, int n,
                                                double* __restrict__ s) {
    const int j = blockIdx.x;
    const double* col = A + (long)j * ld;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += fabs(col[i]);
    acc = lrr::wave_sum(acc);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double d = (red[0] + red[1]) + (red[2] + red[3]);
        s[j] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
    }
}

// A <- |A| s_i s_j (the normalised affinity D^-1/2 W D^-1/2); column j in grid row j
__global__ __launch_bounds__(256) void k_norm_aff(double* __restrict__ A, long ld, int n,
                                                  const double* __restrict__ s) {
    const int j = blockIdx.y;
    const double sj = s[j];
    double* col = A + (long)j * ld;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) col[i] = fabs(col[i]) * s[i] * sj;
}

// largest |Y_j - theta_j X_j| over the k leading columns; theta_j = lam[idx[j]]
__global__ __launch_bounds__(256) void k_resid(const double* __restrict__ Y, const double* __restrict__ X, long ld,
                                               int n, const double* __restrict__ lam, const int* __restrict__ idx,
                                               unsigned long long* __restrict__ out) {
    const int j = blockIdx.x;
    const double th = lam[idx[j]];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double r = Y[i + (long)j * ld] - th * X[i + (long)j * ld];
        acc += r * r;
    }
    acc = lrr::wave_sum(acc);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) lrr::atomic_max_nonneg(out, sqrt((red[0] + red[1]) + (red[2] + red[3])));
}

// Et[c + i k] = X[i, c] / |X[i, 0:k]| (point-major embedding; a zero row stays zero)
__global__ __launch_bounds__(256) void k_rownorm(const double* __restrict__ X, long ldx, int n, int k,
                                                 double* __restrict__ Et) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double ss = 0.0;
    for (int c = 0; c < k; ++c) {
        const double v = X[i + (long)c * ldx];
        ss += v * v;
    }
    double nrm = sqrt(ss);
    if (nrm == 0.0) nrm = 1.0;
    for (int c = 0; c < k; ++c) Et[c + (long)i * k] = X[i + (long)c * ldx] / nrm;
}

// Z = beta X + gamma Y (element-wise over n values)
__global__ __launch_bounds__(256) void k_axpby(const double* __restrict__ X, const double* __restrict__ Y,
                                               double* __restrict__ Z, long n, double beta, double gamma) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) Z[i] = beta * X[i] + gamma * Y[i];
}

__device__ __forceinline__ double sqdist(const double* __restrict__ a, const double* __restrict__ b, int k) {
    double d = 0.0;
    for (int c = 0; c < k; ++c) {
        const double t = a[c] - b[c];
        d += t * t;
    }
    return d;
}

// (value, index) arg-max over the workgroup: larger value wins, ties to the lower index
__device__ int block_argmax(double v, int i, double* sv, int* si) {
    sv[threadIdx.x] = v;
    si[threadIdx.x] = i;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double a = sv[threadIdx.x], b = sv[threadIdx.x + w];
            const int ia = si[threadIdx.x], ib = si[threadIdx.x + w];
            if (b > a || (b == a && ib < ia)) {
                sv[threadIdx.x] = b;
                si[threadIdx.x] = ib;
            }
        }
        __syncthreads();
    }
    const int r = si[0];
    __syncthreads();
    return r;
}

// mean of the embedded points, one workgroup per coordinate (fixed-order sum)
__global__ __launch_bounds__(256) void k_seed_mean(const double* __restrict__ Et, int n, int k,
                                                   double* __restrict__ mean) {
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += Et[c + (long)i * k];
    acc = lrr::wave_sum(acc);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) mean[c] = ((red[0] + red[1]) + (red[2] + red[3])) / n;
}

// one farthest-point step over the points: distance to `ref` (mode 0: the
// mean, d2 untouched; 1: the first centre, d2 = distance; 2: a further centre,
// d2 = min(d2, distance)), then the arg-max of the step's criterion per workgroup
__global__ __launch_bounds__(256) void k_seed_dist(const double* __restrict__ Et, int n, int k,
                                                   const double* __restrict__ ref, double* __restrict__ d2,
                                                   int mode, double* __restrict__ pv, int* __restrict__ pi) {
    __shared__ double sv[256];
    __shared__ int si[256];
    double best = -1.0;
    int bi = INT_MAX;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double d = sqdist(Et + (long)i * k, ref, k);
        double v = d;
        if (mode == 1) d2[i] = d;
        else if (mode == 2) { v = fmin(d2[i], d); d2[i] = v; }
        if (v > best) { best = v; bi = i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double a = sv[threadIdx.x], b = sv[threadIdx.x + w];
            const int ia = si[threadIdx.x], ib = si[threadIdx.x + w];
            if (b > a || (b == a && ib < ia)) { sv[threadIdx.x] = b; si[threadIdx.x] = ib; }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { pv[blockIdx.x] = sv[0]; pi[blockIdx.x] = si[0]; }
}

// arg-max over the workgroup partials (ties: lowest point index); the chosen
// point becomes centre s
__global__ __launch_bounds__(1024) void k_seed_pick(const double* __restrict__ pv, const int* __restrict__ pi,
                                                    int parts, const double* __restrict__ Et, int k,
                                                    double* __restrict__ Ct, int s) {
    __shared__ double sv[1024];
    __shared__ int si[1024];
    double best = -1.0;
    int bi = INT_MAX;
    for (int j = threadIdx.x; j < parts; j += 1024)
        if (pv[j] > best || (pv[j] == best && pi[j] < bi)) { best = pv[j]; bi = pi[j]; }
    const int jbest = block_argmax(best, bi, sv, si);
    for (int c = threadIdx.x; c < k; c += 1024) Ct[c + (long)s * k] = Et[c + (long)jbest * k];
}

// nearest centre of each point (ties: lowest centre); counts changed labels
__global__ __launch_bounds__(256) void k_km_assign(const double* __restrict__ Et, int n, int k,
                                                   const double* __restrict__ Ct, const int* __restrict__ old,
                                                   int* __restrict__ lab, int check, int* __restrict__ nchg) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    int changed = 0;
    if (i < n) {
        const double* p = Et + (long)i * k;
        double best = 0.0;
        int bs = 0;
        for (int s = 0; s < k; ++s) {
            const double d = sqdist(p, Ct + (long)s * k, k);
            if (s == 0 || d < best) { best = d; bs = s; }
        }
        lab[i] = bs;
        changed = check && old[i] != bs;
    }
    const unsigned long long b = __ballot(changed);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(nchg, (int)__popcll(b));
}

// centre s, coordinate c = mean over the points labelled s (sequential in point
// order); an empty cluster keeps its centre
__global__ __launch_bounds__(256) void k_km_update(const double* __restrict__ Et, int n, int k,
                                                   const int* __restrict__ lab, double* __restrict__ Ct) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= k * k) return;
    const int s = g / k, c = g % k;
    double acc = 0.0;
    int cnt = 0;
    for (int i = 0; i < n; ++i) {
        if (lab[i] == s) {
            acc += Et[c + (long)i * k];
            ++cnt;
        }
    }
    if (cnt) Ct[c + (long)s * k] = acc / cnt;
}

// labels renumbered by first appearance; out[keep[i]] = new label of point i
__global__ __launch_bounds__(1024) void k_km_relabel(const int* __restrict__ lab, const int* __restrict__ keep,
                                                     int n, int k, long long* __restrict__ out) {
    __shared__ int first[kMaxK];
    __shared__ int id[kMaxK];
    for (int s = threadIdx.x; s < k; s += 1024) first[s] = INT_MAX;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 1024) atomicMin(&first[lab[i]], i);
    __syncthreads();
    for (int s = threadIdx.x; s < k; s += 1024) {
        int r = 0;
        for (int u = 0; u < k; ++u) r += (first[u] < first[s] || (first[u] == first[s] && u < s)) ? 1 : 0;
        id[s] = r;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 1024) out[keep[i]] = id[lab[i]];
}

__global__ __launch_bounds__(256) void k_fill_i64(long long* __restrict__ a, int n, long long v) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = v;
}

unsigned grid1(long n) { return (unsigned)((n + 255) / 256); }

// Bump allocator over the segmentation workspace (256-byte aligned slices).
struct Slab {
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

// Symmetric eigensolver state for orders up to Lmax (block Jacobi from I).
struct Eig {
    double *A, *W, *R, *lam, *scale;
    int *st, *prot, *lo, *run, *any, *idx, *count;
    EigDesc* d;
    int Lmax;
};

struct Work {
    double *Om, *Y, *Q0, *Q, *Gq, *Tq, *Wk, *Bt, *Qk, *Uk, *A, *s, *X, *LX, *LQ, *B0, *B1, *B2, *Et, *d2, *Ct, *mean, *pv;
    int *pi, *keep, *labA, *labB, *nchg;
    unsigned long long* res;
    GemmDesc* g;
    Eig e;
};

size_t layout(Slab& a, Work& w, int n, int p, int nk, int k, int p2, int Lmax, bool sketch) {
    w.Om = sketch ? a.take<double>((size_t)n * p) : nullptr;
    w.Y = sketch ? a.take<double>((size_t)n * p) : nullptr;
    w.Q0 = a.take<double>((size_t)n * p);
    w.Q = a.take<double>((size_t)n * p);
    w.Gq = a.take<double>((size_t)p * p);
    w.Tq = a.take<double>((size_t)p * p);
    w.Wk = a.take<double>((size_t)Lmax * Lmax);
    w.Bt = a.take<double>((size_t)n * p);
    w.Qk = a.take<double>((size_t)nk * p);
    w.Uk = a.take<double>((size_t)nk * p);
    w.A = a.take<double>((size_t)nk * nk);
    w.s = a.take<double>(nk);
    w.X = a.take<double>((size_t)nk * p2);
    w.LX = a.take<double>((size_t)nk * p2);
    w.LQ = a.take<double>((size_t)nk * p2);
    w.B0 = a.take<double>((size_t)nk * p2);
    w.B1 = a.take<double>((size_t)nk * p2);
    w.B2 = a.take<double>((size_t)nk * p2);
    w.Et = a.take<double>((size_t)nk * k);
    w.d2 = a.take<double>(nk);
    w.mean = a.take<double>(k);
    w.pv = a.take<double>(kSeedParts);
    w.pi = a.take<int>(kSeedParts);
    w.Ct = a.take<double>((size_t)k * k);
    w.keep = a.take<int>(nk);
    w.labA = a.take<int>(nk);
    w.labB = a.take<int>(nk);
    w.nchg = a.take<int>(1);
    w.res = a.take<unsigned long long>(1);
    w.g = a.take<GemmDesc>(16);
    Eig& e = w.e;
    e.Lmax = Lmax;
    e.A = a.take<double>((size_t)Lmax * Lmax);
    e.W = a.take<double>((size_t)Lmax * Lmax);
    e.R = a.take<double>((size_t)Lmax * 2 * kBs);
    e.lam = a.take<double>(Lmax);
    e.scale = a.take<double>(1);
    e.st = a.take<int>(2);
    e.prot = a.take<int>(Lmax / (2 * kBs) + 1);
    e.lo = a.take<int>(Lmax);
    e.run = a.take<int>(1);
    e.any = a.take<int>(1);
    e.idx = a.take<int>(Lmax);
    e.count = a.take<int>(1);
    e.d = a.take<EigDesc>(1);
    return a.off;
}

struct Seg {
    lrr_ctx* ctx;
    hipStream_t s;
    Work w;
    void timed(const char* name, double flops, double bytes, const std::function<void()>& f) {
        lrr::ctx_timed(ctx, s, name, flops, bytes, f);
    }
    void sync() { LRR_HIP(hipStreamSynchronize(s)); }

    // C = alpha op(A) op(B) + beta C through descriptor slot `slot`
    void gemm(int slot, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, long lda,
              const double* B, long ldb, double beta, double* C, long ldc) {
        GemmDesc g{A, B, C, M, N, K, (int)lda, (int)ldb, (int)ldc, alpha, beta, nullptr, nullptr};
        LRR_HIP(hipMemcpyAsync(w.g + slot, &g, sizeof(GemmDesc), hipMemcpyHostToDevice, s));
        sync();   // the host descriptor goes out of scope
        const char* name = ta ? (tb ? "k_dgemm<true, true>" : "k_dgemm<true, false>")
                              : (tb ? "k_dgemm<false, true>" : "k_dgemm<false, false>");
        timed(name, 2.0 * M * N * K, 0.0, [&] { lrr::launch_dgemm(w.g + slot, 1, M, N, ta, tb, s); });
    }

    // eigen-decomposition of the l x l matrix the caller wrote into e.A (ld L);
    // e.idx = order by decreasing eigenvalue; returns the count above the cut
    int eig(int l, int L, double cut, int use_sqrt) {
        Eig& e = w.e;
        std::vector<int> lo(L);
        for (int i = 0; i < L; ++i) lo[i] = i >= l ? 1 : 0;
        const int one = 1;
        EigDesc ed{e.A, e.W, e.R, e.lam, L, l, e.run, e.st, e.scale, e.prot, e.lo, nullptr, nullptr, nullptr};
        LRR_HIP(hipMemcpyAsync(e.lo, lo.data(), sizeof(int) * L, hipMemcpyHostToDevice, s));
        LRR_HIP(hipMemcpyAsync(e.run, &one, sizeof(int), hipMemcpyHostToDevice, s));
        LRR_HIP(hipMemcpyAsync(e.d, &ed, sizeof(EigDesc), hipMemcpyHostToDevice, s));
        lrr::launch_set_identity(e.W, L, s);
        lrr::launch_jacobi_init(e.d, 1, s);
        int h_any = 1;
        for (int sw = 0; sw < 80; ++sw) {
            LRR_HIP(hipMemsetAsync(e.any, 0, sizeof(int), s));
            timed("k_jacobi_offcheck", 0.0, 0.0, [&] { lrr::launch_jacobi_check(e.d, 1, L, e.any, s); });
            LRR_HIP(hipMemcpyAsync(&h_any, e.any, sizeof(int), hipMemcpyDeviceToHost, s));
            sync();
            if (h_any == 0) break;
            for (int r = 0; r < L / kBs - 1; ++r) {
                timed("k_jacobi_pairs<16, 512>", 0.0, 0.0, [&] { lrr::launch_jacobi_pairs(e.d, 1, L, kBs, r, s); });
                timed("k_jacobi_apply<16>", 0.0, 0.0, [&] { lrr::launch_jacobi_apply(e.d, 1, L, kBs, r, s); });
            }
        }
        lrr::launch_jacobi_eigvals(e.d, 1, s);
        hipLaunchKernelGGL(k_sort_desc, dim3(1), dim3(1024), 0, s, e.lam, l, e.idx, e.count, cut, use_sqrt);
        int cnt = 0;
        LRR_HIP(hipMemcpyAsync(&cnt, e.count, sizeof(int), hipMemcpyDeviceToHost, s));
        sync();
        return cnt;
    }

    // zero the padded eigen-matrix before a product writes its l x l part
    void clear_eig(int L) {
        hipLaunchKernelGGL(k_fill_zero, dim3(grid1((long)L * L)), dim3(256), 0, s, w.e.A, (long)L * L);
    }
};

// Outlier flags from the column-sparse outlier estimate S (one wavefront per
// column, lanes stride the rows, a fixed-order wave sum): flag j when
// ||S[:, j]||_2 > delta ||M[:, j]||_2; the flagged columns are counted.
__global__ __launch_bounds__(256) void k_outlier_flags(const double* __restrict__ M, long ldm,
                                                        const double* __restrict__ S, long lds, int m, int n,
                                                        double delta, unsigned char* __restrict__ flags,
                                                        int* __restrict__ count) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n) return;
    const int lane = threadIdx.x & 63;
    double ss = 0.0, sm = 0.0;
    for (int i = lane; i < m; i += 64) {
        const double a = S[i + (long)j * lds], b = M[i + (long)j * ldm];
        ss += a * a;
        sm += b * b;
    }
    ss = lrr::wave_sum(ss);
    sm = lrr::wave_sum(sm);
    if (lane == 0) {
        const unsigned char f = sqrt(ss) > delta * sqrt(sm) ? 1 : 0;
        flags[j] = f;
        if (f) atomicAdd(count, 1);
    }
}

}  // namespace

extern "C" lrr_status lrr_outlier_flags(lrr_ctx* ctx, int m, int n, const void* M, int ldm, const void* S, int lds,
                                        double delta, unsigned char* flags, int* n_flagged, void* stream) {
    if (!ctx) return lrr::ctx_fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    if (m < 1 || n < 1 || !M || !S || !flags || ldm < m || lds < m)
        return lrr::ctx_fail(ctx, LRR_EINVAL, "bad M / S / flags arguments");
    if (!(delta >= 0.0) || !std::isfinite(delta)) return lrr::ctx_fail(ctx, LRR_EINVAL, "delta must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    try {
        if (hipSetDevice(lrr::ctx_device(ctx)) != hipSuccess)
            return lrr::ctx_fail(ctx, LRR_EDEVICE, "hipSetDevice failed");
        int* dcount = static_cast<int*>(lrr::ctx_seg_workspace(ctx, 256));
        LRR_HIP(hipMemsetAsync(dcount, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_outlier_flags, dim3((n + 3) / 4), dim3(256), 0, s, static_cast<const double*>(M),
                           (long)ldm, static_cast<const double*>(S), (long)lds, m, n, delta, flags, dcount);
        int cnt = 0;
        LRR_HIP(hipMemcpyAsync(&cnt, dcount, sizeof(int), hipMemcpyDeviceToHost, s));
        LRR_HIP(hipStreamSynchronize(s));
        if (n_flagged) *n_flagged = cnt;
        return LRR_OK;
    } catch (const lrr::HipError& e) {
        return lrr::ctx_fail(ctx, LRR_EDEVICE, e.msg);
    } catch (const std::bad_alloc&) {
        return lrr::ctx_fail(ctx, LRR_ENOMEM, "segmentation workspace allocation failed");
    }
}

extern "C" lrr_status lrr_segment(lrr_ctx* ctx, int n, const void* Zv, int ldz, int k, const unsigned char* exclude,
                                  double rank_tol, int rank_bound, long long* labels, lrr_seg_info* info,
                                  void* stream) {
    if (!ctx) return lrr::ctx_fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    if (n < 1 || !Zv || ldz < n || !labels) return lrr::ctx_fail(ctx, LRR_EINVAL, "bad Z / labels arguments");
    if (ldz >= lrr::kGemmMaxLd) return lrr::ctx_fail(ctx, LRR_EINVAL, "leading dimensions must be below 4194304");
    if (!(rank_tol > 0.0 && rank_tol < 1.0)) return lrr::ctx_fail(ctx, LRR_EINVAL, "rank_tol must lie in (0, 1)");
    if (rank_bound < 0) return lrr::ctx_fail(ctx, LRR_EINVAL, "rank_bound must be >= 0");
    if (k < 1 || k > kMaxK) return lrr::ctx_fail(ctx, LRR_EINVAL, "k must lie in [1, 1024]");
    const bool sketch = rank_bound > 0 && rank_bound + kSketchExtra < n;
    if (!sketch && n > kMaxDirect)
        return lrr::ctx_fail(ctx, LRR_EINVAL, "n > 8192 needs a rank_bound (range sketch)");
    const double* Z = static_cast<const double*>(Zv);
    hipStream_t s = static_cast<hipStream_t>(stream);
    try {
        if (hipSetDevice(lrr::ctx_device(ctx)) != hipSuccess)
            return lrr::ctx_fail(ctx, LRR_EDEVICE, "hipSetDevice failed");
        // kept points (host list from the device mask)
        std::vector<unsigned char> ex(n, 0);
        if (exclude) {
            LRR_HIP(hipMemcpyAsync(ex.data(), exclude, n, hipMemcpyDeviceToHost, s));
            LRR_HIP(hipStreamSynchronize(s));
        }
        std::vector<int> keep;
        keep.reserve(n);
        for (int i = 0; i < n; ++i)
            if (!ex[i]) keep.push_back(i);
        const int nk = (int)keep.size();
        if (k > nk) return lrr::ctx_fail(ctx, LRR_EINVAL, "k exceeds the number of kept points");
        const int p = sketch ? rank_bound + kSketchExtra : n;
        const int p2 = std::min(nk, k + std::max(16, k / 2));
        const int L1 = round_up(std::max(p, 2), 2 * kBs);
        const int L3 = round_up(std::max(p2, 2), 2 * kBs);
        const int Lmax = std::max(L1, L3);

        Slab probe;
        Work w;
        const size_t bytes = layout(probe, w, n, p, nk, k, p2, Lmax, sketch);
        Slab a;
        a.base = static_cast<char*>(lrr::ctx_seg_workspace(ctx, bytes));
        layout(a, w, n, p, nk, k, p2, Lmax, sketch);
        Seg g{ctx, s, w};
        Eig& e = g.w.e;
        LRR_HIP(hipMemcpyAsync(w.keep, keep.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
        g.sync();

        // ---- range basis Q of Z (n x q) -------------------------------------------
        const double* Y = Z;
        long ldy = ldz;
        if (sketch) {
            hipLaunchKernelGGL(k_fill_uniform, dim3(grid1((long)n * p)), dim3(256), 0, s, w.Om, (long)n, n, p,
                               0x5EEDull);
            g.gemm(0, false, false, n, p, n, 1.0, Z, ldz, w.Om, n, 0.0, w.Y, n);
            Y = w.Y;
            ldy = n;
        }
        g.clear_eig(L1);
        g.gemm(1, true, false, p, p, n, 1.0, Y, ldy, Y, ldy, 0.0, e.A, L1);
        int q = g.eig(p, L1, kRangeCut, 0);
        if (q < 1) q = 1;
        if (sketch && q >= p)
            return lrr::ctx_fail(ctx, LRR_EINVAL, "rank_bound is below the rank of Z (the range sketch has full rank)");
        hipLaunchKernelGGL(k_pick_cols, dim3(q), dim3(256), 0, s, e.W, (long)L1, e.lam, e.idx, p, 1, w.Wk, (long)p);
        g.gemm(2, false, false, n, q, p, 1.0, Y, ldy, w.Wk, p, 0.0, w.Q0, n);
        g.gemm(3, true, false, q, q, n, 1.0, w.Q0, n, w.Q0, n, 0.0, w.Gq, q);
        lrr::launch_ns_factor(w.Gq, w.Tq, q, s);
        g.gemm(4, false, false, n, q, q, 1.0, w.Q0, n, w.Tq, q, 0.0, w.Q, n);

        // ---- singular values of Z on the basis, left singular vectors U --------------
        const int L2 = round_up(std::max(q, 2), 2 * kBs);
        g.gemm(5, true, false, n, q, n, 1.0, Z, ldz, w.Q, n, 0.0, w.Bt, n);
        g.clear_eig(L2);
        g.gemm(6, true, false, q, q, n, 1.0, w.Bt, n, w.Bt, n, 0.0, e.A, L2);
        int r = g.eig(q, L2, rank_tol, 1);
        if (r < 1) r = 1;
        hipLaunchKernelGGL(k_pick_cols, dim3(r), dim3(256), 0, s, e.W, (long)L2, e.lam, e.idx, q, 0, w.Wk, (long)q);
        hipLaunchKernelGGL(k_gather_rows, dim3(grid1((long)nk * q)), dim3(256), 0, s, w.Q, (long)n, w.keep, nk, q,
                           w.Qk, (long)nk);
        g.gemm(7, false, false, nk, r, q, 1.0, w.Qk, nk, w.Wk, q, 0.0, w.Uk, nk);

        // ---- normalised affinity L = D^-1/2 |U U^T| D^-1/2 (nk x nk) -----------------
        g.gemm(8, false, true, nk, nk, r, 1.0, w.Uk, nk, w.Uk, nk, 0.0, w.A, nk);
        g.timed("k_absdeg", 0.0, 8.0 * nk * (double)nk, [&] {
            hipLaunchKernelGGL(k_absdeg, dim3(nk), dim3(256), 0, s, w.A, (long)nk, nk, w.s);
        });
        g.timed("k_norm_aff", 0.0, 16.0 * nk * (double)nk, [&] {
            const unsigned gx = (unsigned)std::min<long>(grid1(nk), 8);
            hipLaunchKernelGGL(k_norm_aff, dim3(gx, nk), dim3(256), 0, s, w.A, (long)nk, nk, w.s);
        });

        // ---- spectral embedding: k leading eigenvectors of L -------------------------
        // Chebyshev-filtered subspace iteration (Zhou and Saad, J. Comput. Phys.
        // 2007) with a Rayleigh-Ritz step on L after each filter.  L has its
        // spectrum in [-1, 1] (W >= 0 entry-wise, Perron root 1), so the filter
        // T_m((t - c) / e), c and e mapping [-1, b] onto [-1, 1] and normalised
        // to 1 at t = 1, damps everything below the smallest Ritz value b of the
        // block and amplifies the eigenvalues above it.  Its degree is capped so
        // that the filtered block stays within a condition number of about
        // kSpread, which the two Gram passes of the orthonormalisation resolve.
        double* B3[3] = {w.B0, w.B1, w.B2};
        std::vector<double> lamh(p2), th(p2);
        std::vector<int> idxh(p2);
        int products = 0;
        // Y <- orthonormal basis of span(Y) (two passes of Y W diag(lam)^-1/2); tmp is scratch
        auto orth = [&](double* Y, double* tmp) {
            double* src = Y;
            double* dst = tmp;
            for (int pass = 0; pass < 2; ++pass) {
                g.clear_eig(L3);
                g.gemm(9, true, false, p2, p2, nk, 1.0, src, nk, src, nk, 0.0, e.A, L3);
                g.eig(p2, L3, 0.0, 0);
                hipLaunchKernelGGL(k_pick_cols, dim3(p2), dim3(256), 0, s, e.W, (long)L3, e.lam, e.idx, p2, 1,
                                   w.Wk, (long)p2);
                g.gemm(10, false, false, nk, p2, p2, 1.0, src, nk, w.Wk, p2, 0.0, dst, nk);
                std::swap(src, dst);
            }
        };
        // Rayleigh-Ritz on the orthonormal block Q: X = Ritz vectors (decreasing
        // Ritz values th), LX = L X; returns the largest residual of the k leading ones
        auto rayleigh_ritz = [&](const double* Q) {
            g.gemm(11, false, false, nk, p2, nk, 1.0, w.A, nk, Q, nk, 0.0, w.LQ, nk);
            ++products;
            g.clear_eig(L3);
            g.gemm(12, true, false, p2, p2, nk, 1.0, Q, nk, w.LQ, nk, 0.0, e.A, L3);
            g.eig(p2, L3, 0.0, 0);
            hipLaunchKernelGGL(k_pick_cols, dim3(p2), dim3(256), 0, s, e.W, (long)L3, e.lam, e.idx, p2, 0, w.Wk,
                               (long)p2);
            g.gemm(13, false, false, nk, p2, p2, 1.0, Q, nk, w.Wk, p2, 0.0, w.X, nk);
            g.gemm(14, false, false, nk, p2, p2, 1.0, w.LQ, nk, w.Wk, p2, 0.0, w.LX, nk);
            LRR_HIP(hipMemsetAsync(w.res, 0, sizeof(unsigned long long), s));
            hipLaunchKernelGGL(k_resid, dim3(k), dim3(256), 0, s, w.LX, w.X, (long)nk, nk, e.lam, e.idx, w.res);
            unsigned long long rb = 0;
            LRR_HIP(hipMemcpyAsync(lamh.data(), e.lam, sizeof(double) * p2, hipMemcpyDeviceToHost, s));
            LRR_HIP(hipMemcpyAsync(idxh.data(), e.idx, sizeof(int) * p2, hipMemcpyDeviceToHost, s));
            LRR_HIP(hipMemcpyAsync(&rb, w.res, sizeof(rb), hipMemcpyDeviceToHost, s));
            g.sync();
            for (int j = 0; j < p2; ++j) th[j] = lamh[idxh[j]];
            double r;
            std::memcpy(&r, &rb, sizeof(double));
            return r;
        };
        // Y = p_m(L) X / p_m(1), three-term recurrence on ratios of T_j(x0)
        auto filter = [&](int m, double b) {
            const double a = -1.0;
            const double ee = 0.5 * (b - a), cc = 0.5 * (b + a);
            const double x0 = (1.0 - cc) / ee;
            double rp = 1.0 / x0;   // T_0(x0) / T_1(x0)
            double* prev = w.X;
            double* cur = B3[0];
            double* nxt = B3[1];
            lrr::launch_copy_cols(w.X, nk, cur, nk, nk, p2, s);
            g.gemm(15, false, false, nk, p2, nk, rp / ee, w.A, nk, w.X, nk, -cc * rp / ee, cur, nk);
            ++products;
            for (int j = 1; j < m; ++j) {
                const double rj = 1.0 / (2.0 * x0 - rp);   // T_j / T_{j+1}
                const double al = 2.0 * rj / ee;
                hipLaunchKernelGGL(k_axpby, dim3(grid1((long)nk * p2)), dim3(256), 0, s, cur, prev, nxt,
                                   (long)nk * p2, -cc * al, -rp * rj);
                g.gemm(15, false, false, nk, p2, nk, al, w.A, nk, cur, nk, 1.0, nxt, nk);
                ++products;
                rp = rj;
                if (j == 1) { prev = B3[0]; cur = B3[1]; nxt = B3[2]; }
                else { double* t0 = prev; prev = cur; cur = nxt; nxt = t0; }
            }
            return std::make_pair(cur, cur == B3[0] ? B3[1] : B3[0]);
        };
        hipLaunchKernelGGL(k_fill_uniform, dim3(grid1((long)nk * p2)), dim3(256), 0, s, B3[0], (long)nk, nk, p2,
                           0xE3B0ull);
        orth(B3[0], B3[1]);
        double resid = rayleigh_ritz(B3[0]);
        bool conv = resid <= kEmbedTol;
        int outer = 0;
        for (outer = 0; !conv && outer < kEmbedMaxOuter; ++outer) {
            double b = th[p2 - 1];
            const double gapk = th[k - 1] - b;
            if (!(gapk > 1e-12)) b = th[k - 1] - 1e-12;   // flat block: keep the interval below theta_k
            b = std::max(b, -0.999);                       // the interval [-1, b] must not be empty
            const double ee = 0.5 * (b + 1.0), cc = 0.5 * (b - 1.0);
            const double x0 = std::max((1.0 - cc) / ee, 1.0 + 1e-15);
            int m = (int)std::floor(std::log(kSpread) / std::acosh(x0));
            m = std::max(1, std::min(m, kMaxDegree));
            auto yc = filter(m, b);
            orth(yc.first, yc.second);
            resid = rayleigh_ritz(yc.first);
            conv = resid <= kEmbedTol;
        }
        const int it = products;

        // ---- k-means on the unit rows -------------------------------------------------
        g.timed("k_rownorm", 0.0, 0.0, [&] {
            hipLaunchKernelGGL(k_rownorm, dim3(grid1(nk)), dim3(256), 0, s, w.X, (long)nk, nk, k, w.Et);
        });
        {
            // farthest-point seeding: centre 0 is the point farthest from the mean,
            // centre s + 1 the point farthest from centres 0..s
            const int parts = (int)std::min<long>(grid1(nk), kSeedParts);
            g.timed("k_seed_mean", 0.0, 0.0, [&] {
                hipLaunchKernelGGL(k_seed_mean, dim3(k), dim3(256), 0, s, w.Et, nk, k, w.mean);
            });
            for (int c = 0; c < k; ++c) {
                const double* ref = (c == 0) ? w.mean : w.Ct + (long)(c - 1) * k;
                const int mode = (c == 0) ? 0 : (c == 1 ? 1 : 2);
                g.timed("k_seed_dist", 0.0, 0.0, [&] {
                    hipLaunchKernelGGL(k_seed_dist, dim3(parts), dim3(256), 0, s, w.Et, nk, k, ref, w.d2, mode,
                                       w.pv, w.pi);
                });
                g.timed("k_seed_pick", 0.0, 0.0, [&] {
                    hipLaunchKernelGGL(k_seed_pick, dim3(1), dim3(1024), 0, s, w.pv, w.pi, parts, w.Et, k, w.Ct, c);
                });
            }
        }
        int* cur = w.labA;
        int* nxt = w.labB;
        int kit = 0;
        for (kit = 0; kit < kKmeansMaxIter; ++kit) {
            LRR_HIP(hipMemsetAsync(w.nchg, 0, sizeof(int), s));
            g.timed("k_km_assign", 0.0, 0.0, [&] {
                hipLaunchKernelGGL(k_km_assign, dim3(grid1(nk)), dim3(256), 0, s, w.Et, nk, k, w.Ct, cur, nxt,
                                   kit > 0 ? 1 : 0, w.nchg);
            });
            int chg = 1;
            LRR_HIP(hipMemcpyAsync(&chg, w.nchg, sizeof(int), hipMemcpyDeviceToHost, s));
            g.sync();
            if (kit > 0 && chg == 0) break;
            std::swap(cur, nxt);
            g.timed("k_km_update", 0.0, 0.0, [&] {
                hipLaunchKernelGGL(k_km_update, dim3(grid1((long)k * k)), dim3(256), 0, s, w.Et, nk, k, cur, w.Ct);
            });
        }
        hipLaunchKernelGGL(k_fill_i64, dim3(grid1(n)), dim3(256), 0, s, labels, n, -1ll);
        hipLaunchKernelGGL(k_km_relabel, dim3(1), dim3(1024), 0, s, cur, w.keep, nk, k, labels);
        LRR_HIP(hipGetLastError());
        g.sync();
        lrr::ctx_prof_flush(ctx);
        if (info) {
            info->rank = r;
            info->range_rank = q;
            info->sketch = p;
            info->embed_iters = it;
            info->embed_resid = resid;
            info->theta_k = th[k - 1];
            info->theta_k1 = (p2 > k) ? th[k] : 0.0;
            info->kmeans_iters = std::min(kit + 1, kKmeansMaxIter);
            info->n_keep = nk;
        }
        return conv ? LRR_OK : LRR_NOT_CONVERGED;
    } catch (const lrr::HipError& e) {
        return lrr::ctx_fail(ctx, LRR_EDEVICE, e.msg);
    } catch (const std::bad_alloc&) {
        return lrr::ctx_fail(ctx, LRR_ENOMEM, "segmentation workspace allocation failed");
    }
}
