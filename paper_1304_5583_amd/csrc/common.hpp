// Shared definitions of the gfx950 DFC-LRR library (device and host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

namespace lrr {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------------------
// Batched GEMM descriptor:  C = alpha * op(A) op(B) + beta * C  (column-major).
// op(A) is M x K, op(B) is K x N, C is M x N.  If `active` is set and
// active[0] == 0 the batch item is skipped (frozen or trivial block).  If
// `colmap` is set, result column j is stored in column colmap[j] of C.
// ----------------------------------------------------------------------------
struct GemmDesc {
    const double* A;
    const double* B;
    double* C;
    int M, N, K;
    int lda, ldb, ldc;
    double alpha, beta;
    const int* active;
    const int* colmap;
};

// Arithmetic of a product (operands and result are FP64 in memory in all modes).
enum GemmMode {
    kGemmFP64 = 0,     // FP64 matrix cores, FP64 accumulation
    kGemmFP32 = 1,     // operands rounded to FP32, FP32 matrix cores and accumulation
    kGemmBF16X3 = 2    // operands split into BF16 hi + lo, three BF16 products, FP32 accumulation
};

// Device-resident iteration state of the batched ALM loop.  Kernels read the
// penalty of the current iteration from here, so a captured sequence of
// launches replays correctly.
struct DevIter {
    int k;          // iteration index (0-based) of the iteration being run
    int full;       // nonzero: the eigensolver resolves every eigenpair, also
                    // those below tau^2 (reverse-mode replay needs them)
    double mu;      // penalty mu_k of this iteration
    double tau;     // 1 / mu_k, the singular-value threshold
};

// Per-block state of the batched ALM loop (device arrays of length t).
struct BlockState {
    int* active;        // 1 while the block is iterating
    int* svt_run;       // 1 if this iteration needs the eigen-based threshold step
    int* iters;         // iterations run
    int* rank;          // rank of J
    double* res1;       // ||X - AZ - E||_max of the last iteration
    double* res2;       // ||Z - J||_max of the last iteration
    unsigned long long* r1max;  // running max (bit pattern of a non-negative double)
    unsigned long long* r2max;
    double* colr1;      // per column: max |R1| of the column (E-step)
    double* colr2;      // per column: max |R2|, or the coefficient residual's 2-norm
};

// Eigensolver descriptor of one symmetric matrix (padded size L, ld = L).
// Operation counters of the Jacobi kernels: one atomic per workgroup, spread
// over kWorkSlots counters 128 bytes apart per kind (0: pair solves, 1: tile
// updates), so that workgroups on different XCDs do not queue on one address.
constexpr int kWorkSlots = 64;
constexpr int kWorkStride = 16;   // unsigned long longs between counters
constexpr size_t kWorkBytes = 2 * kWorkSlots * kWorkStride * sizeof(unsigned long long);
__host__ __device__ __forceinline__ size_t work_slot(int kind, int wg) {
    return (size_t)(kind * kWorkSlots + wg % kWorkSlots) * kWorkStride;
}

struct EigDesc {
    double* B;          // L x L symmetric, diagonalised in place
    double* W;          // L x L, accumulates the rotations (eigenvectors)
    double* R;          // (L / (2 bs)) rotation blocks of (2 bs)^2 each
    double* lam;        // L eigenvalues (diagonal of B on exit)
    int L;              // padded order, multiple of 2 bs
    int l;              // true order (rows/cols >= l are padding)
    const int* run;     // skip the matrix if run[0] == 0
    int* st;            // [0] converged, [1] pairs that rotated in the current sweep
    double* scale;      // max |diag| of B at the start, for the absolute floor
    int* prot;          // per pair of the current round: 1 if it rotated
    int* lo;            // per index: Gershgorin disc below the cut (pairs of two such are skipped)
    unsigned long long* work;  // FP64 operation counters (may be null): pair solves, then tile
                               // updates, each spread over kWorkSlots counters (work_slot)
    const double* cut;  // cut factor nu of the block: lo when the disc lies below min(tau^2, nu * scale)
    int* passes;        // sweep-loop passes of the current eigensolve (counted while open)
    int* need;          // (L/bs)^2 flags (may be null): the check marks index-block pairs (p <= q,
                        // at p * (L/bs) + q) holding an entry that still needs a rotation
    const int* sched;   // (may be null) explicit rounds: entry r * (L/bs/2) + P is the pair
                        // p | q << 16 of slot P in round r; every round pairs all L/bs blocks
    const int* done;    // (may be null) done[0] set: the refinement left nothing to rotate; B
                        // was not formed, its diagonal is taken from lam and the matrix is
                        // closed at the start of the eigensolve
};

// Control block of the persistent eigensolve (k_jacobi_solve): its grid-wide
// barrier, an error flag (a barrier wait that ran out), the open-matrix counts of
// two consecutive passes.  Zeroed by a kernel before each launch.
struct JacCtl {
    unsigned bar_count;
    unsigned bar_gen;
    int err;
    int n_open[2];
    int pad[3];
};

// Gershgorin flag of one index: its disc lies below both tau^2 and the block's
// cut nu * scale (pairs of two such indices are never rotated)
__device__ __forceinline__ int lo_flag(double disc, double tau, double nu, double scale) {
    return disc < fmin(tau * tau * (1.0 - 1e-9), nu * scale) ? 1 : 0;
}

// Warm-started eigenvector refinement of one Gram matrix (see refsyev.hip).
struct RefDesc {
    const double* B;    // L x L Gram matrix
    double* X;          // L x L eigenvector estimate (right half of the [T | X] buffer)
    double* SG;         // L x 2L: [S | G] = X^T [B X | X]
    double* E;          // L x L correction
    double* XE;         // L x L product X E
    double* lam;        // L Rayleigh quotients
    int* lo;            // L Gershgorin flags
    double* scale;      // max |diag B|
    unsigned long long* emax;  // largest resolvable correction of the step (bits)
    int* unres;         // couplings left for the Jacobi sweeps
    double* eprev;      // previous step's largest correction
    int* run;           // refinement step applied to this matrix
    int* cont;          // refinement continues after this step
    double* Xb;         // L x L copy of X before the refinement (restored if it fails)
    const double* cut;  // cut factor of the block (as EigDesc::cut)
    int L, l, block;
    unsigned long long* rdev;  // largest |I - X^T X| seen by the step (bits)
    int* nsskip;        // the last applied step measured |I - X^T X| <= 1e-8: no orthogonalisation
    int* clean;         // the last applied step corrected by less than the stop with no unresolvable
                        // coupling, and the orthogonalisation found |I - X^T X| <= kCleanDev
};

// One block's small matrices in the reverse sweep of the thresholding step.
struct BwDesc {
    const double* W;    // L x L eigenvectors of the Gram matrix (recorded)
    const double* lam;  // L eigenvalues (recorded; zero beyond l)
    double* Wg;         // L x L  W diag(g(lam))
    double* S;          // L x L scratch
    double* C;          // L x L scratch
    double* N;          // L x L scratch
    int L, l;
    const int* run;     // thresholding step taken by this block in the recorded iteration
};

// Thresholding weights of one block after its Gram eigensolve.
struct SvtDesc {
    const double* B;    // L x L, diagonal = eigenvalues of the Gram matrix
    const double* W;    // L x L eigenvectors
    double* Wg;         // L x L, W scaled column-wise by g = (1 - tau/sigma)_+
    double* lam;        // L eigenvalues (copy)
    double* h;          // L, 1/sigma on kept columns, 0 elsewhere
    int L, l;
    const int* run;
    int block;
};

__device__ __forceinline__ unsigned long long dbl_bits(double x) {
    return (unsigned long long)__double_as_longlong(x);
}

// max of non-negative doubles through their (monotone) bit patterns: the
// result does not depend on the order of the updates.
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* addr, double v) {
    atomicMax(addr, dbl_bits(v));
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Round-robin (circle method) pairing of N players (N even) in round r of N-1:
// player N-1 is fixed, the others rotate.  Every pair meets once per sweep.
__host__ __device__ __forceinline__ void rr_pair(int N, int r, int k, int& a, int& b) {
    if (k == 0) {
        a = r;
        b = N - 1;
    } else {
        a = (r + k) % (N - 1);
        b = (r - k + (N - 1)) % (N - 1);
    }
    if (a > b) { int t = a; a = b; b = t; }
}

}  // namespace lrr

// a failing call throws; its error is also taken out of HIP's last-error
// state, so that it cannot surface at a later, unrelated error check
#define LRR_HIP(call)                                                         \
    do {                                                                      \
        hipError_t _e = (call);                                               \
        if (_e != hipSuccess) {                                               \
            (void)hipGetLastError();                                          \
            throw lrr::HipError(std::string(#call) + ": " + hipGetErrorString(_e)); \
        }                                                                     \
    } while (0)

namespace lrr {
// device allocation for the workspaces: false (and no HIP error left behind)
// when the memory is not there, which the entry points report as LRR_ENOMEM
inline bool try_device_alloc(void** p, size_t bytes) {
    if (hipMalloc(p, bytes) == hipSuccess) return true;
    *p = nullptr;
    (void)hipGetLastError();
    return false;
}
}  // namespace lrr

namespace lrr {
struct HipError {
    std::string msg;
    explicit HipError(std::string m) : msg(std::move(m)) {}
};
}  // namespace lrr
