// Kernels of the reverse sweep through the unrolled ALM (dfc_lrr_backward).
//
// One iteration of the forward map (push-through form, per block column):
//   Y  = Z + Y2/mu,           J = Y P,  P = W g(Lambda) W^T  (Y^T Y = W Lambda W^T,
//                                        g(lam) = (1 - tau/sqrt(lam))_+)
//   Q  = J - Y2/mu,           Pv = X - E + Y1/mu,  V = K^{-1}(Pv - M Q),  K = I + M M^T
//   Z' = Q + M^T V,           q = E + V,  E' = shrink(q, lambda/mu)
//   Y1' = mu (q - E'),        Y2' = Y2 + mu (Z' - J)
// Given the cotangents (cZ, cE, cY1, cY2, cJ) of (Z', E', Y1', Y2', J) the step
// below produces those of (Z, E, Y1, Y2) and accumulates dM, dX (the block's
// columns of M) and dlambda:
//   qbar = mu cY1 + shrink'(q)^T (cE - mu cY1),  dtheta = -q^T(cE - mu cY1)/||q||
//   Vbar = qbar + M Zt,  Zt = cZ + mu cY2,  Jt = cJ - mu cY2
//   Wb = K^{-1} Vbar;  Qbar = Zt - M^T Wb;  dX += Wb
//   dM += V Zt^T - Wb Q^T - (Wb V^T + V Wb^T) M
//   Jt += Qbar;  E_bar = qbar - Wb;  Y1_bar = Wb/mu;  Y2_bar = cY2 - Qbar/mu + Ybar/mu
//   Ybar = Jt P + Y W [phi o (W^T (Y^T Jt + Jt^T Y) W)] W^T,  Z_bar = Ybar
// where phi_ij is the divided difference of g over the eigenvalue pair
// (lam_i, lam_j) (Daleckii-Krein formula for the derivative of the matrix
// function g(Y^T Y)); this is the singular-value-thresholding derivative
// written on the Gram eigenvalues.
#include "common.hpp"
#include "kernels.hpp"

namespace lrr {

namespace {

__device__ double block_sum256b(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}

// E-step reverse: qbar (written to cE and Vb), dlambda per column
__global__ __launch_bounds__(256) void k_bw_estep(const double* __restrict__ E0, const double* __restrict__ V,
                                                   double* __restrict__ cE, const double* __restrict__ cY1,
                                                   double* __restrict__ Vb, double* __restrict__ lamcol, int m,
                                                   long ld, const int* __restrict__ colblk,
                                                   const int* __restrict__ active, const DevIter* it,
                                                   double lam) {
    __shared__ double red[4];
    const int j = blockIdx.x;
    if (!active[colblk[j]]) return;
    const double mu = it->mu;
    const double theta = lam / mu;
    const long o = j * ld;
    double nn = 0.0, dot = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        const double q = E0[o + i] + V[o + i];
        const double et = cE[o + i] - mu * cY1[o + i];
        nn += q * q;
        dot += q * et;
    }
    nn = block_sum256b(nn, red);
    dot = block_sum256b(dot, red);
    const double nq = sqrt(nn);
    const bool big = nq > theta;
    const double a = big ? 1.0 - theta / nq : 0.0;
    const double b = big ? theta * dot / (nn * nq) : 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        const double q = E0[o + i] + V[o + i];
        const double y1 = cY1[o + i];
        const double et = cE[o + i] - mu * y1;
        const double qb = mu * y1 + a * et + b * q;
        cE[o + i] = qb;
        Vb[o + i] = qb;
    }
    if (threadIdx.x == 0 && big) lamcol[j] += -dot / nq / mu;
}

// Zt = cZ + mu cY2,  Jt = cJ - mu cY2  (cJ may be null: zero)
__global__ __launch_bounds__(256) void k_bw_zt(const double* __restrict__ cZ, const double* __restrict__ cY2,
                                                const double* __restrict__ cJ, double* __restrict__ Zt,
                                                double* __restrict__ Jt, int n, long ld,
                                                const int* __restrict__ colblk, const int* __restrict__ active,
                                                const DevIter* it) {
    const int j = blockIdx.x;
    if (!active[colblk[j]]) return;
    const double mu = it->mu;
    const long o = j * ld;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double y2 = cY2[o + i];
        Zt[o + i] = cZ[o + i] + mu * y2;
        Jt[o + i] = (cJ ? cJ[o + i] : 0.0) - mu * y2;
    }
}

// Jt += Qbar, cY2 -= Qbar/mu (n rows);  dX += Wb, cE -= Wb, cY1 = Wb/mu (m rows)
__global__ __launch_bounds__(256) void k_bw_mid(const double* __restrict__ Qb, double* __restrict__ Jt,
                                                 double* __restrict__ cY2, const double* __restrict__ Wb,
                                                 double* __restrict__ Xbar, double* __restrict__ cE,
                                                 double* __restrict__ cY1, int n, long ldn, int m, long ldm,
                                                 const int* __restrict__ colblk, const int* __restrict__ active,
                                                 const DevIter* it) {
    const int j = blockIdx.x;
    if (!active[colblk[j]]) return;
    const double mu = it->mu;
    const long on = j * ldn, om = j * ldm;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double qb = Qb[on + i];
        Jt[on + i] += qb;
        cY2[on + i] -= qb / mu;
    }
    for (int i = threadIdx.x; i < m; i += 256) {
        const double w = Wb[om + i];
        Xbar[om + i] += w;
        cE[om + i] -= w;
        cY1[om + i] = w / mu;
    }
}

// cY2 += Ybar/mu (Ybar already stored as the new cZ)
__global__ __launch_bounds__(256) void k_bw_final(const double* __restrict__ Yb, double* __restrict__ cY2, int n,
                                                   long ld, const int* __restrict__ colblk,
                                                   const int* __restrict__ active, const DevIter* it) {
    const int j = blockIdx.x;
    if (!active[colblk[j]]) return;
    const double mu = it->mu;
    const long o = j * ld;
    for (int i = threadIdx.x; i < n; i += 256) cY2[o + i] += Yb[o + i] / mu;
}

// columns of active blocks that skipped the thresholding step (J = 0) are zeroed
__global__ __launch_bounds__(256) void k_zero_norun(double* __restrict__ A, int n, long ld,
                                                     const int* __restrict__ colblk, const int* __restrict__ run,
                                                     const int* __restrict__ active) {
    const int j = blockIdx.x;
    const int b = colblk[j];
    if (!active[b] || run[b]) return;
    for (int i = threadIdx.x; i < n; i += 256) A[i + j * ld] = 0.0;
}

__device__ __forceinline__ double g_of(double lam, double tau) {
    const double sig = sqrt(fmax(lam, 0.0));
    return sig > tau ? 1.0 - tau / sig : 0.0;
}

// Wg = W diag(g(lam)) on the leading L x l columns
__global__ __launch_bounds__(256) void k_bw_wg(const BwDesc* __restrict__ descs, const DevIter* it) {
    const BwDesc d = descs[blockIdx.y];
    if (!d.run[0]) return;
    const int i = blockIdx.x;
    if (i >= d.L) return;
    const double g = (i < d.l) ? g_of(d.lam[i], it->tau) : 0.0;
    const long o = (long)i * d.L;
    for (int r = threadIdx.x; r < d.L; r += 256) d.Wg[o + r] = d.W[o + r] * g;
}

// C = S + S^T on the leading l x l part, zero elsewhere
__global__ __launch_bounds__(256) void k_bw_sym(const BwDesc* __restrict__ descs) {
    const BwDesc d = descs[blockIdx.y];
    if (!d.run[0]) return;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    const int L = d.L;
    if (idx >= (long)L * L) return;
    const int i = (int)(idx % L), j = (int)(idx / L);
    d.C[idx] = (i < d.l && j < d.l) ? d.S[idx] + d.S[j + (long)i * L] : 0.0;
}

// N = phi o C, phi_ij the divided difference of g(lam) = (1 - tau/sqrt(lam))_+
// over (lam_i, lam_j), evaluated in forms without cancellation:
//   both above tau^2:  tau / (s_i s_j (s_i + s_j))     (s = sqrt(lam); i = j gives g')
//   one above (i):     g(lam_i) / (lam_i - lam_j)       (lam_j <= tau^2 < lam_i)
//   neither:           0
__global__ __launch_bounds__(256) void k_bw_phi(const BwDesc* __restrict__ descs, const DevIter* it) {
    const BwDesc d = descs[blockIdx.y];
    if (!d.run[0]) return;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    const int L = d.L;
    if (idx >= (long)L * L) return;
    const int i = (int)(idx % L), j = (int)(idx / L);
    const double tau = it->tau;
    const double li = (i < d.l) ? fmax(d.lam[i], 0.0) : 0.0;
    const double lj = (j < d.l) ? fmax(d.lam[j], 0.0) : 0.0;
    const double si = sqrt(li), sj = sqrt(lj);
    const bool ai = si > tau, aj = sj > tau;
    double phi = 0.0;
    if (ai && aj) phi = tau / (si * sj * (si + sj));
    else if (ai) phi = (1.0 - tau / si) / (li - lj);
    else if (aj) phi = (1.0 - tau / sj) / (lj - li);
    d.N[idx] = phi * d.C[idx];
}

// Wr = W diag(1/(s (s - tau))) on the kept columns (combine reverse: (J^+)^T = Y Wr W^T)
__global__ __launch_bounds__(256) void k_bw_rdiag(const double* __restrict__ W, const double* __restrict__ lam,
                                                   double* __restrict__ Wr, int L, int l, const DevIter* it) {
    const int i = blockIdx.x;
    if (i >= L) return;
    const double tau = it->tau;
    double r = 0.0;
    if (i < l) {
        const double s = sqrt(fmax(lam[i], 0.0));
        if (s > tau) r = 1.0 / (s * (s - tau));
    }
    const long o = (long)i * L;
    for (int k = threadIdx.x; k < L; k += 256) Wr[o + k] = W[o + k] * r;
}

// Mbar[:, perm[j]] += Xbar[:, j]
__global__ __launch_bounds__(256) void k_scatter_add(const double* __restrict__ Xb, long ldx,
                                                      double* __restrict__ Mb, long ldm, int m,
                                                      const int* __restrict__ perm) {
    const int j = blockIdx.x;
    const long dst = perm[j];
    for (int i = threadIdx.x; i < m; i += 256) Mb[i + dst * ldm] += Xb[i + j * ldx];
}

// A[:, j] += B[:, j] for j < ncols
__global__ __launch_bounds__(256) void k_add_cols(double* __restrict__ A, long lda, const double* __restrict__ B,
                                                   long ldb, int rows) {
    const int j = blockIdx.x;
    for (int i = threadIdx.x; i < rows; i += 256) A[i + j * lda] += B[i + j * ldb];
}

}  // namespace

void launch_bw_estep(const double* E0, const double* V, double* cE, const double* cY1, double* Vb,
                     double* lamcol, int m, long ld, int ncols, const int* colblk, const int* active,
                     const DevIter* it, double lam, hipStream_t s) {
    hipLaunchKernelGGL(k_bw_estep, dim3(ncols), dim3(256), 0, s, E0, V, cE, cY1, Vb, lamcol, m, ld, colblk,
                       active, it, lam);
}
void launch_bw_zt(const double* cZ, const double* cY2, const double* cJ, double* Zt, double* Jt, int n, long ld,
                  int ncols, const int* colblk, const int* active, const DevIter* it, hipStream_t s) {
    hipLaunchKernelGGL(k_bw_zt, dim3(ncols), dim3(256), 0, s, cZ, cY2, cJ, Zt, Jt, n, ld, colblk, active, it);
}
void launch_bw_mid(const double* Qb, double* Jt, double* cY2, const double* Wb, double* Xbar, double* cE,
                   double* cY1, int n, long ldn, int m, long ldm, int ncols, const int* colblk,
                   const int* active, const DevIter* it, hipStream_t s) {
    hipLaunchKernelGGL(k_bw_mid, dim3(ncols), dim3(256), 0, s, Qb, Jt, cY2, Wb, Xbar, cE, cY1, n, ldn, m, ldm,
                       colblk, active, it);
}
void launch_bw_final(const double* Yb, double* cY2, int n, long ld, int ncols, const int* colblk,
                     const int* active, const DevIter* it, hipStream_t s) {
    hipLaunchKernelGGL(k_bw_final, dim3(ncols), dim3(256), 0, s, Yb, cY2, n, ld, colblk, active, it);
}
void launch_zero_norun(double* A, int n, long ld, int ncols, const int* colblk, const int* run, const int* active,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_zero_norun, dim3(ncols), dim3(256), 0, s, A, n, ld, colblk, run, active);
}
void launch_bw_wg(const BwDesc* d, int count, int maxL, const DevIter* it, hipStream_t s) {
    hipLaunchKernelGGL(k_bw_wg, dim3(maxL, count), dim3(256), 0, s, d, it);
}
void launch_bw_sym(const BwDesc* d, int count, int maxL, hipStream_t s) {
    const long nn = (long)maxL * maxL;
    hipLaunchKernelGGL(k_bw_sym, dim3((unsigned)((nn + 255) / 256), count), dim3(256), 0, s, d);
}
void launch_bw_phi(const BwDesc* d, int count, int maxL, const DevIter* it, hipStream_t s) {
    const long nn = (long)maxL * maxL;
    hipLaunchKernelGGL(k_bw_phi, dim3((unsigned)((nn + 255) / 256), count), dim3(256), 0, s, d, it);
}
void launch_bw_rdiag(const double* W, const double* lam, double* Wr, int L, int l, const DevIter* it,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_bw_rdiag, dim3(L), dim3(256), 0, s, W, lam, Wr, L, l, it);
}
void launch_scatter_add(const double* Xb, long ldx, double* Mb, long ldm, int m, int ncols, const int* perm,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_add, dim3(ncols), dim3(256), 0, s, Xb, ldx, Mb, ldm, m, perm);
}
void launch_add_cols(double* A, long lda, const double* B, long ldb, int rows, int ncols, hipStream_t s) {
    hipLaunchKernelGGL(k_add_cols, dim3(ncols), dim3(256), 0, s, A, lda, B, ldb, rows);
}

}  // namespace lrr
