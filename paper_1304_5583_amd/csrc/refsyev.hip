// Warm-started refinement of a symmetric eigen-decomposition (FP64).
//
// The thresholding step of iteration k needs the eigenvectors of the Gram
// matrix B_k = Y_k^T Y_k, and B_k is close to B_{k-1}.  Starting from the
// eigenvectors X of the previous iteration, each refinement step is the
// Newton-type update of Ogita and Aishima (Japan J. Indust. Appl. Math., 2018):
//   G = X^T X,  S = X^T B X,  lambda_i = s_ii / g_ii,  R = I - G,
//   E_ij = (s_ij + lambda_j r_ij) / (lambda_j - lambda_i)   (i != j, resolvable)
//   E_ij = r_ij / 2                                          (otherwise)
//   X <- X + X E
// which converges quadratically once the off-diagonal coupling is small
// against the eigenvalue gaps.  Built entirely from the MFMA GEMM plus two
// element-wise kernels, so a step is a handful of launches whatever the order.
//
// A pair (i, j) is resolvable when |s_ij + lambda_j r_ij| <= 0.1 |lambda_j -
// lambda_i| (inside the linear regime of the update) and the two Gershgorin
// discs of S are not both below the cut min(tau^2, nu scale): every eigenvalue
// whose disc lies below tau^2 is discarded by the threshold step, so rotations
// among such indices cannot change the result.  Couplings that stay
// unresolvable are left to the block-Jacobi sweeps that follow.
//
// The cut factor nu is per block and starts at 0 (every eigenpair resolved):
// the eigenvectors below tau^2 are the ones that cross the threshold as tau
// shrinks, and while the refinement carries them from one iteration to the
// next they cost nothing.  A warm eigensolve that still needs more than
// kSwitchSweeps Jacobi sweeps shows that they are not carried (a spread of
// small, drifting eigenvalues); from then on that block leaves the eigenpairs
// below min(tau^2, kLoCut scale) unresolved.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace lrr {

namespace {

constexpr double kLinCap = 0.1;
constexpr long kStatGroups = 64;         // workgroups per matrix of the kernels that also reduce statistics
constexpr long kStreamGroups = 128;      // workgroups per matrix of the element-wise passes (grid-stride)
constexpr int kRowGroups = 64;           // workgroups per matrix of the row pass
constexpr double kFirstStepCap = 0.1;    // largest correction accepted in the first step
constexpr double kOrthTol = 1e-6;         // |I - X^T X| above this after one step: restart cold
constexpr double kRelTol = 1e-15;
constexpr double kAbsFloor = 1e-14;
constexpr double kLoCut = 1e-2;           // cut factor after the switch
constexpr int kSwitchSweeps = 8;          // warm sweeps that trigger it
constexpr double kNSSecond = 1e-8;        // |I - X^T X| above which the second orthogonalisation step runs
// A block is clean (its Jacobi matrix X^T B X is not formed) when the last
// applied step's largest correction e was below the stop (at most 1e-8) with no unresolvable
// coupling above the Jacobi tolerance, and the first orthogonalisation step
// found |I - X^T X| = d <= kCleanDev (so no second step).  Write X = V (I + H)
// with V orthonormal eigenvectors up to the step's residual: the step leaves
// couplings of order e^2 times the eigenvalue gaps, and the non-orthogonality
// H (|H| ~ d / 2) couples i and j by (lambda_i + lambda_j) H_ij; the
// orthogonalisation X (I + (I - X^T X)/2) = V (I - H^2 + ...) leaves O(d^2).
// Both are below the Jacobi check's floor of 1e-14 max |diag|, and the
// Rayleigh quotients of the step's S differ from those of the final X by
// terms of the same second order.
constexpr double kCleanDev = 1e-8;


// row pass: lambda_i, Gershgorin flag lo_i of S (padding: lambda 0, lo 1)
// one row of k_ref_rows: lambda_i and the Gershgorin flag lo_i of S
__device__ void ref_row(const RefDesc& d, int i, const DevIter* it, int gid) {
    const long L = d.L;
    const double* S = d.SG;
    const double* G = d.SG + L * L;
    __shared__ double red[4];
    // Gershgorin radius from column i (S is symmetric; the column is contiguous).
    // With the cut factor at 0 the flag needs s_ii + r below 0, which a
    // non-negative s_ii never is: the radius is then summed only for s_ii < 0.
    const bool need_r = i < d.l && !it->full && (d.cut[0] != 0.0 || S[i + i * L] < 0.0);
    double r = 0.0;
    if (need_r) {
        double rs = 0.0;
        for (int j = threadIdx.x; j < d.l; j += 256)
            if (j != i) rs += fabs(S[j + i * L]);
        rs = wave_sum(rs);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rs;
        __syncthreads();
        r = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();   // red is free for the next row
    }
    if (threadIdx.x == 0) {
        const double tau = it->tau;
        if (i < d.l) {
            const double sii = S[i + i * L];
            d.lam[i] = gid ? sii : sii / G[i + i * L];
            d.lo[i] = it->full ? 0 : lo_flag(sii + r, tau, d.cut[0], d.scale[0]);
        } else {
            d.lam[i] = 0.0;
            d.lo[i] = 1;
        }
    }
}

// gid: X^T X is taken as the identity (the first step of a warm refinement,
// whose X left the previous iteration orthonormal to rounding), G not read
__global__ __launch_bounds__(256) void k_ref_rows(const RefDesc* __restrict__ descs, const DevIter* it, int gid) {
    const RefDesc d = descs[blockIdx.y];
    if (d.run[0] == 0) return;
    for (int i = blockIdx.x; i < d.L; i += gridDim.x) ref_row(d, i, it, gid);
}

// correction matrix E and per-matrix statistics
__global__ __launch_bounds__(256) void k_ref_E(const RefDesc* __restrict__ descs, int gid) {
    const RefDesc d = descs[blockIdx.y];
    if (d.run[0] == 0) return;
    const long L = d.L;
    if (blockIdx.x >= L) return;   // no column for this workgroup
    double emax = 0.0, rdev = 0.0;
    int unres = 0;
    // a few workgroups stride over the columns (rows by thread, no index
    // division): one atomic per workgroup for the statistics (one per 256
    // entries serialised on the two addresses)
    const double* S = d.SG;
    const double* G = d.SG + L * L;
    for (int j = blockIdx.x; j < L; j += gridDim.x)
    for (int i = threadIdx.x; i < L; i += 256) {
        const long idx = i + (long)j * L;
        const double gij = gid ? (i == j ? 1.0 : 0.0) : G[i + j * L];
        rdev = fmax(rdev, fabs((i == j ? 1.0 : 0.0) - gij));
        double e;
        if (i == j) {
            e = 0.5 * (1.0 - gij);
        } else {
            const double rij = -gij;
            const double sij = S[i + j * L];
            const double li = d.lam[i], lj = d.lam[j];
            const double num = sij + lj * rij;
            const double dl = lj - li;
            const bool both_lo = d.lo[i] && d.lo[j];
            const bool ok = !both_lo && dl != 0.0 && fabs(num) <= kLinCap * fabs(dl);
            if (ok) {
                e = num / dl;
                emax = fmax(emax, fabs(e));
            } else {
                e = 0.5 * rij;
                if (!both_lo && i < j && i < d.l && j < d.l) {
                    const double sii = S[i + i * L], sjj = S[j + j * L];
                    if (fabs(sij) > fmax(kRelTol * sqrt(fabs(sii * sjj)), kAbsFloor * d.scale[0])) unres += 1;
                }
            }
        }
        d.E[idx] = e;
    }
    // one atomic per workgroup (per-wave atomics on one address serialise)
    emax = wave_max(emax);
    rdev = wave_max(rdev);
    int u = unres;
    for (int off = 32; off > 0; off >>= 1) u += __shfl_xor(u, off, 64);
    __shared__ double wmax[4], wdev[4];
    __shared__ int wsum[4];
    if ((threadIdx.x & 63) == 0) {
        wmax[threadIdx.x >> 6] = emax;
        wdev[threadIdx.x >> 6] = rdev;
        wsum[threadIdx.x >> 6] = u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double r4 = fmax(fmax(wdev[0], wdev[1]), fmax(wdev[2], wdev[3]));
        if (r4 > 0.0) atomic_max_nonneg(d.rdev, r4);
        const double e4 = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
        const int u4 = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        if (e4 > 0.0) atomic_max_nonneg(d.emax, e4);
        if (u4) atomicAdd(d.unres, u4);
    }
}

// X += XE
__global__ __launch_bounds__(256) void k_ref_add(const RefDesc* __restrict__ descs) {
    const RefDesc d = descs[blockIdx.y];
    if (d.run[0] == 0) return;
    const long n = (long)d.L * d.L;
    for (long idx = (long)blockIdx.x * 256 + threadIdx.x; idx < n; idx += (long)gridDim.x * 256) d.X[idx] += d.XE[idx];
}

// after E is formed and before it is applied: apply the step only while the
// corrections do not grow; stop (without applying) otherwise
__global__ void k_ref_update(const RefDesc* __restrict__ descs, int count, int step, int max_steps, double stop) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    const RefDesc d = descs[b];
    if (d.run[0] == 0) return;
    const double e = __longlong_as_double((long long)d.emax[0]);
    const double limit = (step == 0) ? kFirstStepCap : d.eprev[0];
    const bool apply = (e <= limit);
    d.clean[0] = (apply && e < stop && d.unres[0] == 0) ? 1 : 0;
    // the step leaves |I - X^T X| of order |R| e + e^2 (E + E^T = R to first
    // order): with G measured (not the first step) and |R| <= kNSSecond the
    // orthogonalisation steps would only move rounding noise
    const double rdev = __longlong_as_double((long long)d.rdev[0]);
    d.nsskip[0] = (d.clean[0] && step > 0 && rdev <= kNSSecond) ? 1 : 0;
    d.rdev[0] = 0ull;
    // after a correction below `stop` the next one (quadratic in it) would be at
    // the rounding level; what such a step would remove is left to the Jacobi
    // check, whose tolerance decides convergence
    const bool cont = apply && e >= stop && step + 1 < max_steps;
    d.eprev[0] = e;
    d.emax[0] = 0ull;
    d.unres[0] = 0;
    d.run[0] = apply ? 1 : 0;
    d.cont[0] = cont ? 1 : 0;
}

// after the step is applied: continue only where the update asked for it
__global__ void k_ref_next(const RefDesc* __restrict__ descs, int count) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    const RefDesc d = descs[b];
    d.run[0] = d.cont[0];
}

// start of a refinement: per-matrix flags and the scale of S
__global__ void k_ref_begin(const RefDesc* __restrict__ descs, int count, const int* __restrict__ svt_run,
                            const int* __restrict__ warm) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    const RefDesc d = descs[b];
    d.run[0] = (svt_run[d.block] && warm[d.block]) ? 1 : 0;
    d.cont[0] = 0;
    d.clean[0] = 0;
    d.nsskip[0] = 0;
    d.rdev[0] = 0ull;
    d.eprev[0] = 1.0;
    d.emax[0] = 0ull;
    d.unres[0] = 0;
}

// max |diag| of the Gram matrix (scale of the absolute floor)
__global__ __launch_bounds__(256) void k_ref_scale(const RefDesc* __restrict__ descs) {
    const RefDesc d = descs[blockIdx.x];
    if (d.run[0] == 0) return;
    double mx = 0.0;
    for (int i = threadIdx.x; i < d.l; i += 256) mx = fmax(mx, fabs(d.B[i + (long)i * d.L]));
    mx = wave_max(mx);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) d.scale[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Gershgorin flags of the Jacobi matrix (for the cleanup sweeps); count_pass:
// the pass follows a full sweep (or starts the eigensolve) and is counted
__global__ __launch_bounds__(256) void k_lo_rows(const EigDesc* __restrict__ descs, const DevIter* it,
                                                 int count_pass) {
    const EigDesc d = descs[blockIdx.y];
    if (d.run[0] == 0 || d.st[0] != 0) return;
    const int i = blockIdx.x;
    if (i >= d.L) return;
    const long L = d.L;
    __shared__ double red[4];
    double rs = 0.0;   // column i of the symmetric matrix, contiguous
    for (int j = threadIdx.x; j < d.l; j += 256)
        if (j != i) rs += fabs(d.B[j + i * L]);
    rs = wave_sum(rs);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rs;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double r = (red[0] + red[1]) + (red[2] + red[3]);
        const double tau = it->tau;
        d.lo[i] = (i >= d.l) ? 1 : (it->full ? 0 : lo_flag(d.B[i + i * L] + r, tau, d.cut[0], d.scale[0]));
        if (i == 0 && count_pass) d.passes[0] += 1;
    }
}

// end of a block's eigensolve: a warm solve that needed many sweeps switches
// the block to the cut kLoCut (for the rest of the solve); counters restart
__global__ void k_lo_mode(const int* __restrict__ svt_run, const int* __restrict__ warm, int* __restrict__ passes,
                          double* __restrict__ cut, int t) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= t) return;
    // passes = sweeps + 1 (the last pass finds nothing to rotate)
    if (svt_run[b] && warm[b] && cut[b] == 0.0 && passes[b] > kSwitchSweeps + 1) cut[b] = kLoCut;
    passes[b] = 0;
}

// orthogonalisation step (Newton-Schulz for the polar factor): E = (I - G)/2,
// and the largest |I - G| of the matrix
__global__ __launch_bounds__(256) void k_orth_E(const RefDesc* __restrict__ descs) {
    const RefDesc d = descs[blockIdx.y];
    if (d.run[0] == 0) return;
    const long L = d.L;
    if ((long)blockIdx.x * 256 >= L * L) return;   // whole workgroup past the matrix
    double dev = 0.0;
    for (long idx = (long)blockIdx.x * 256 + threadIdx.x; idx < L * L; idx += (long)gridDim.x * 256) {
        const int i = (int)(idx % L), j = (int)(idx / L);
        const double g = d.SG[L * L + idx];
        const double e = (i == j) ? 0.5 * (1.0 - g) : -0.5 * g;
        d.E[idx] = e;
        dev = fmax(dev, 2.0 * fabs(e));
    }
    dev = wave_max(dev);
    __shared__ double wmax[4];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = dev;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double d4 = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
        if (d4 > 0.0) atomic_max_nonneg(d.emax, d4);
    }
}

// a matrix whose estimate lost orthogonality restarts from the identity
// A refinement that lost orthogonality is discarded: X returns to the previous
// iteration's eigenvectors (the identity on a block's first decomposition),
// from which the Jacobi sweeps finish the decomposition.
__global__ __launch_bounds__(256) void k_orth_guard(const RefDesc* __restrict__ descs, const int* __restrict__ warm) {
    const RefDesc d = descs[blockIdx.y];
    if (d.run[0] == 0) return;
    const double dev = __longlong_as_double((long long)d.emax[0]);
    if (!(dev <= kOrthTol)) {
        const long L = d.L;
        for (long idx = (long)blockIdx.x * 256 + threadIdx.x; idx < L * L; idx += (long)gridDim.x * 256)
            d.X[idx] = warm[d.block] ? d.Xb[idx] : (((idx % L) == (idx / L)) ? 1.0 : 0.0);
    }
}

// X is kept before a refinement starts
__global__ __launch_bounds__(256) void k_ref_backup(const RefDesc* __restrict__ descs) {
    const RefDesc d = descs[blockIdx.y];
    if (d.run[0] == 0) return;
    const long n = (long)d.L * d.L;
    for (long idx = (long)blockIdx.x * 256 + threadIdx.x; idx < n; idx += (long)gridDim.x * 256) d.Xb[idx] = d.X[idx];
}

__global__ void k_orth_reset(const RefDesc* __restrict__ descs, int count) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    descs[b].emax[0] = 0ull;
}

// after the first orthogonalisation step: the second runs only where the first
// started from |I - X^T X| above kNSSecond.  A step maps a deviation d to about
// 3 d^2 / 4 plus rounding, so from d <= 1e-8 the first step already reaches the
// rounding level and a second one would only move rounding noise.  (Skipping
// the first step's update as well below d = 1e-12 measured slower: workload 4
// 806 instead of 700 ms per solve at the same iteration counts.)
__global__ void k_orth_decide(const RefDesc* __restrict__ descs, int count, double thr) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    const RefDesc d = descs[b];
    if (d.run[0] == 0) return;
    const double dev = __longlong_as_double((long long)d.emax[0]);
    d.run[0] = dev > thr ? 1 : 0;
    if (!(dev <= kCleanDev)) d.clean[0] = 0;
}

// the steps after the refinement run on every matrix that needs a decomposition
__global__ void k_ref_set_run(const RefDesc* __restrict__ descs, int count, const int* __restrict__ svt_run) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    const RefDesc d = descs[b];
    d.run[0] = svt_run[d.block];
}

// the orthogonalisation steps run for the matrices that need a decomposition,
// except those whose last refinement step measured |I - X^T X| <= kNSSecond
__global__ void k_ref_set_run_ns(const RefDesc* __restrict__ descs, int count, const int* __restrict__ svt_run) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    const RefDesc d = descs[b];
    d.run[0] = (svt_run[d.block] && !d.nsskip[0]) ? 1 : 0;
}

// the Jacobi matrix X^T B X is formed for the matrices that need a decomposition
// and are not clean
__global__ void k_ref_set_run_jac(const RefDesc* __restrict__ descs, int count, const int* __restrict__ svt_run) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    const RefDesc d = descs[b];
    d.run[0] = (svt_run[d.block] && !d.clean[0]) ? 1 : 0;
}

__global__ void k_mark_warm(const int* __restrict__ svt_run, int* __restrict__ warm, int t) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < t && svt_run[b]) warm[b] = 1;
}

}  // namespace

void launch_orth_E(const RefDesc* d, int count, int maxL, hipStream_t s) {
    const long n = (long)maxL * maxL;
    hipLaunchKernelGGL(k_orth_reset, dim3((count + 63) / 64), dim3(64), 0, s, d, count);
    hipLaunchKernelGGL(k_orth_E, dim3((unsigned)std::min<long>((n + 255) / 256, kStatGroups), count), dim3(256), 0,
                       s, d);
}
void launch_orth_guard(const RefDesc* d, int count, int maxL, const int* warm, hipStream_t s) {
    const long n = (long)maxL * maxL;
    hipLaunchKernelGGL(k_orth_guard, dim3((unsigned)std::min<long>((n + 255) / 256, kStreamGroups), count), dim3(256),
                       0, s, d, warm);
}
void launch_ref_next(const RefDesc* d, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_ref_next, dim3((count + 63) / 64), dim3(64), 0, s, d, count);
}
void launch_orth_decide(const RefDesc* d, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_orth_decide, dim3((count + 63) / 64), dim3(64), 0, s, d, count, kNSSecond);
}
void launch_ref_set_run(const RefDesc* d, int count, const int* svt_run, hipStream_t s) {
    hipLaunchKernelGGL(k_ref_set_run, dim3((count + 63) / 64), dim3(64), 0, s, d, count, svt_run);
}
void launch_ref_set_run_ns(const RefDesc* d, int count, const int* svt_run, hipStream_t s) {
    hipLaunchKernelGGL(k_ref_set_run_ns, dim3((count + 63) / 64), dim3(64), 0, s, d, count, svt_run);
}
void launch_ref_set_run_jac(const RefDesc* d, int count, const int* svt_run, hipStream_t s) {
    hipLaunchKernelGGL(k_ref_set_run_jac, dim3((count + 63) / 64), dim3(64), 0, s, d, count, svt_run);
}
void launch_lo_mode(const int* svt_run, const int* warm, int* passes, double* cut, int t, hipStream_t s) {
    hipLaunchKernelGGL(k_lo_mode, dim3((t + 63) / 64), dim3(64), 0, s, svt_run, warm, passes, cut, t);
}
void launch_mark_warm(const int* svt_run, int* warm, int t, hipStream_t s) {
    hipLaunchKernelGGL(k_mark_warm, dim3((t + 63) / 64), dim3(64), 0, s, svt_run, warm, t);
}

void launch_ref_begin(const RefDesc* d, int count, int maxL, const int* svt_run, const int* warm, hipStream_t s) {
    const long n = (long)maxL * maxL;
    hipLaunchKernelGGL(k_ref_begin, dim3((count + 63) / 64), dim3(64), 0, s, d, count, svt_run, warm);
    hipLaunchKernelGGL(k_ref_scale, dim3(count), dim3(256), 0, s, d);
    hipLaunchKernelGGL(k_ref_backup, dim3((unsigned)std::min<long>((n + 255) / 256, kStreamGroups), count), dim3(256),
                       0, s, d);
}
void launch_ref_rows(const RefDesc* d, int count, int maxL, const DevIter* it, hipStream_t s, bool gid) {
    hipLaunchKernelGGL(k_ref_rows, dim3(std::min(maxL, kRowGroups), count), dim3(256), 0, s, d, it, (int)gid);
}
void launch_ref_E(const RefDesc* d, int count, int maxL, hipStream_t s, bool gid) {
    const long n = (long)maxL * maxL;
    hipLaunchKernelGGL(k_ref_E, dim3((unsigned)std::min<long>((n + 255) / 256, kStatGroups), count), dim3(256), 0,
                       s, d, (int)gid);
}
void launch_ref_add(const RefDesc* d, int count, int maxL, hipStream_t s) {
    const long n = (long)maxL * maxL;
    hipLaunchKernelGGL(k_ref_add, dim3((unsigned)std::min<long>((n + 255) / 256, kStreamGroups), count), dim3(256), 0,
                       s, d);
}
void launch_ref_update(const RefDesc* d, int count, int step, int max_steps, double stop, hipStream_t s) {
    hipLaunchKernelGGL(k_ref_update, dim3((count + 63) / 64), dim3(64), 0, s, d, count, step, max_steps, stop);
}
void launch_lo_rows(const EigDesc* d, int count, int maxL, const DevIter* it, hipStream_t s, bool count_pass) {
    hipLaunchKernelGGL(k_lo_rows, dim3(maxL, count), dim3(256), 0, s, d, it, (int)count_pass);
}

}  // namespace lrr
