// Column-wise kernels of the batched inexact-ALM iteration (FP64).
//
// All t blocks of DFC-LRR share one column-concatenated layout: block b owns
// columns [boff[b], boff[b+1]) of every state matrix (Z, J, Y2 in R^{n x n};
// E, Y1 in R^{m x n}).  Each kernel here handles one column per workgroup,
// skips the columns of frozen blocks, and reads the penalty of the current
// iteration from the device-resident DevIter, so that the same launches can
// be replayed without host-side arguments changing.
//
// Per iteration (push-through form of the Z-step, see the solver):
//   k_form_Y      Y = Z + Y2/mu, column sums of squares        (J-step input)
//   k_block_fro   ||Y_b||_F per block; ||Y_b||_F <= tau => J_b = 0 exactly
//   k_form_QT     Q = J - Y2/mu,  T = X - E + Y1/mu
//                 (reduced-precision products: also dQ = Q - Q_prev, and
//                 T -= M Q is carried as T -= sum of M dQ, see k_sub_cols)
//   k_update_Z    Z = Q + M^T V,  R2 = Z - J,  Y2 += mu R2,  max|R2|
//   k_estep       q = E + V (= X - M Z + Y1/mu), column l2 shrinkage by
//                 lam/mu, R1 = q - Y1/mu - E,  Y1 += mu R1,  max|R1|
//   k_check       per-block stop test, freeze, advance mu
// Reductions run in a fixed order (deterministic); the max-norms use integer
// atomics on the bit patterns of non-negative doubles, which is order-free.
#include "common.hpp"
#include "kernels.hpp"

namespace lrr {

namespace {

// deterministic sum over a 256-thread workgroup; result valid in all threads
__device__ double block_sum256(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}

__device__ double block_max256(double v, double* red) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    const double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_gather_cols(const double* __restrict__ M, long ldm,
                                                      double* __restrict__ X, long ldx, int m,
                                                      const int* __restrict__ perm) {
    const int j = blockIdx.x;
    const long src = perm[j];
    for (int i = threadIdx.x; i < m; i += 256) X[i + j * ldx] = M[i + src * ldm];
}

__global__ __launch_bounds__(256) void k_scatter_cols(const double* __restrict__ X, long ldx,
                                                       double* __restrict__ S, long lds, int m,
                                                       const int* __restrict__ perm) {
    const int j = blockIdx.x;
    const long dst = perm[j];
    for (int i = threadIdx.x; i < m; i += 256) S[i + dst * lds] = X[i + j * ldx];
}

__global__ __launch_bounds__(256) void k_copy_cols(const double* __restrict__ X, long ldx,
                                                    double* __restrict__ Y, long ldy, int m) {
    const int j = blockIdx.x;
    for (int i = threadIdx.x; i < m; i += 256) Y[i + j * ldy] = X[i + j * ldx];
}

// element-type conversion of a column-major matrix (one workgroup per column):
// FP32 -> FP64 is exact, FP64 -> FP32 rounds to nearest
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_convert_cols(const TI* __restrict__ src, long lds, TO* __restrict__ dst,
                                                      long ldd, int rows) {
    const long j = blockIdx.x;
    for (int i = threadIdx.x; i < rows; i += 256) dst[i + j * ldd] = static_cast<TO>(src[i + j * lds]);
}

__global__ __launch_bounds__(256) void k_nonfinite(const double* __restrict__ M, long ldm, int m,
                                                    int* flag) {
    const int j = blockIdx.x;
    int bad = 0;
    for (int i = threadIdx.x; i < m; i += 256) bad |= !isfinite(M[i + j * ldm]);
    if (bad) atomicOr(flag, 1);
}

// Two consecutive rows of a column (16-byte access when VEC); rows at or past
// m read as zeros and are not written.
template <bool VEC>
__device__ __forceinline__ void ld2(const double* __restrict__ p, int i, int m, double& a, double& b) {
    if (VEC && i + 1 < m) {
        const double2 x = *reinterpret_cast<const double2*>(p + i);
        a = x.x;
        b = x.y;
    } else {
        a = i < m ? p[i] : 0.0;
        b = i + 1 < m ? p[i + 1] : 0.0;
    }
}
template <bool VEC>
__device__ __forceinline__ void st2(double* __restrict__ p, int i, int m, double a, double b) {
    if (VEC && i + 1 < m) {
        *reinterpret_cast<double2*>(p + i) = double2{a, b};
    } else {
        if (i < m) p[i] = a;
        if (i + 1 < m) p[i + 1] = b;
    }
}

// One workgroup per column: measured faster here than one wave per column
// with 16-byte accesses (52.5 against 55.5 us per launch on workload 4) and
// than issuing the column's loads before the block's flag is read (54.1).
__global__ __launch_bounds__(256) void k_form_Y(const double* __restrict__ Z, const double* __restrict__ Y2,
                                                 double* __restrict__ Y, double* __restrict__ colsq,
                                                 int n, long ld, const int* __restrict__ colblk,
                                                 const int* __restrict__ active, const DevIter* it) {
    __shared__ double red[4];
    const int j = blockIdx.x;
    if (!active[colblk[j]]) return;
    const double mu = it->mu;
    const long o = j * ld;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double y = Z[o + i] + Y2[o + i] / mu;
        Y[o + i] = y;
        s += y * y;
    }
    s = block_sum256(s, red);
    if (threadIdx.x == 0) colsq[j] = s;
}

__global__ __launch_bounds__(256) void k_block_fro(const double* __restrict__ colsq,
                                                    const int* __restrict__ boff, BlockState bs,
                                                    const DevIter* it) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    if (!bs.active[b]) {
        if (threadIdx.x == 0) bs.svt_run[b] = 0;
        return;
    }
    double s = 0.0;
    for (int c = boff[b] + threadIdx.x; c < boff[b + 1]; c += 256) s += colsq[c];
    s = block_sum256(s, red);
    if (threadIdx.x == 0) {
        // sigma_max <= ||Y||_F, so ||Y||_F <= tau gives J = 0 without a decomposition
        bs.svt_run[b] = (sqrt(s) > it->tau) ? 1 : 0;
        bs.rank[b] = 0;
    }
}

// Blocks that need an eigen-decomposition this iteration: those that threshold,
// and, in an iteration where some block thresholds for the first time (a cold
// eigensolve, many Jacobi sweeps), every other block not yet decomposed whose
// ||Y||_F exceeds prewarm * tau: it is close to its own first thresholding
// step, and decomposing it in the same launches costs little more than the
// rounds already paid, while its later first step then starts warm.
__global__ __launch_bounds__(256) void k_eig_select(const double* __restrict__ colsq, const int* __restrict__ boff,
                                                     int t, const int* __restrict__ active,
                                                     const int* __restrict__ svt_run, const int* __restrict__ warm,
                                                     int* __restrict__ eig_run, const DevIter* it, double prewarm) {
    __shared__ double red[4];
    __shared__ int any_cold;
    if (threadIdx.x == 0) any_cold = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < t; b += 256)
        if (svt_run[b] && !warm[b]) any_cold = 1;   // every writer stores 1
    __syncthreads();
    const double tau = it->tau;
    for (int b = 0; b < t; ++b) {
        int e = svt_run[b];
        if (!e && any_cold && prewarm > 0.0 && active[b] && !warm[b]) {
            double s = 0.0;
            for (int c = boff[b] + threadIdx.x; c < boff[b + 1]; c += 256) s += colsq[c];
            s = block_sum256(s, red);
            e = sqrt(s) > prewarm * tau ? 1 : 0;
        }
        if (threadIdx.x == 0) eig_run[b] = e;
    }
}

__global__ __launch_bounds__(256) void k_zero_J(double* __restrict__ J, int n, long ld,
                                                 const int* __restrict__ colblk, BlockState bs) {
    const int j = blockIdx.x;
    const int b = colblk[j];
    if (!bs.active[b] || bs.svt_run[b]) return;
    for (int i = threadIdx.x; i < n; i += 256) J[i + j * ld] = 0.0;
}

// SVT weights from the converged Gram eigenvalues: sigma = sqrt(lambda),
// g = (1 - tau/sigma)_+ scales the eigenvector columns, h = 1/sigma on the
// kept columns (the combine basis), rank = #{sigma > tau}.
// One wave per eigenpair i (four per workgroup): the weight g_i scales
// column i of W; the kept pairs of the workgroup are added to the block's rank
// with one atomic.
__global__ __launch_bounds__(256) void k_svt_weights(const SvtDesc* __restrict__ descs,
                                                      const DevIter* it, BlockState bs) {
    __shared__ int kept[4];
    const SvtDesc d = descs[blockIdx.y];
    if (!d.run[0]) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + w;
    int keep_i = 0;
    if (i < d.L) {
        const double tau = it->tau;
        const double lam = (i < d.l) ? d.B[i + (long)i * d.L] : 0.0;
        const double sig = sqrt(fmax(lam, 0.0));
        const bool keep = sig > tau;
        const double g = keep ? 1.0 - tau / sig : 0.0;
        if (lane == 0) {
            d.lam[i] = lam;
            d.h[i] = keep ? 1.0 / sig : 0.0;
        }
        keep_i = keep ? 1 : 0;
        const long o = (long)i * d.L;
        for (int r = lane; r < d.L; r += 64) d.Wg[o + r] = d.W[o + r] * g;
    }
    if (lane == 0) kept[w] = keep_i;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int k = kept[0] + kept[1] + kept[2] + kept[3];
        if (k) atomicAdd(&bs.rank[d.block], k);
    }
}

// With dQ set (difference form), dQ = Q_new - Q_old is written as well.
__global__ __launch_bounds__(256) void k_form_QT(const double* __restrict__ J, const double* __restrict__ Y2,
                                                  double* __restrict__ Q, double* __restrict__ dQ, int n,
                                                  long ldn, const double* __restrict__ X,
                                                  const double* __restrict__ E, const double* __restrict__ Y1,
                                                  double* __restrict__ T, int m, long ldm,
                                                  const int* __restrict__ colblk, const int* __restrict__ active,
                                                  const DevIter* it) {
    const int j = blockIdx.x;
    if (!active[colblk[j]]) return;
    const double mu = it->mu;
    const long on = j * ldn, om = j * ldm;
    if (dQ) {
        for (int i = threadIdx.x; i < n; i += 256) {
            const double q = J[on + i] - Y2[on + i] / mu;
            dQ[on + i] = q - Q[on + i];
            Q[on + i] = q;
        }
    } else {
        for (int i = threadIdx.x; i < n; i += 256) Q[on + i] = J[on + i] - Y2[on + i] / mu;
    }
    for (int i = threadIdx.x; i < m; i += 256) T[om + i] = X[om + i] - E[om + i] + Y1[om + i] / mu;
}

// T -= A on the columns of active blocks
__global__ __launch_bounds__(256) void k_sub_cols(double* __restrict__ T, const double* __restrict__ A, int m,
                                                   long ld, const int* __restrict__ colblk,
                                                   const int* __restrict__ active) {
    const int j = blockIdx.x;
    if (!active[colblk[j]]) return;
    const long o = j * ld;
    for (int i = threadIdx.x; i < m; i += 256) T[o + i] -= A[o + i];
}

// Reduced coordinates, coupling residual R2 = Qm R2r: with Qm having orthonormal
// columns, ||R2 e_j||_inf <= ||R2r e_j||_2 and ||R2 e_j||_inf >= ||R2r e_j||_2 / sqrt(n).
// A block whose largest column 2-norm is below tol, or at least sqrt(n) tol, is
// decided by the bound (which is recorded as its residual); the others get their
// residual columns expanded (expand = 1) and the exact max-norm taken.
__global__ void k_r2_decide(BlockState bs, unsigned long long* __restrict__ r2nrm, int* __restrict__ expand,
                            int t, double tol, double sqrt_n) {
    for (int b = threadIdx.x; b < t; b += blockDim.x) {
        const double x = __longlong_as_double((long long)r2nrm[b]);
        r2nrm[b] = 0ull;
        int e = 0;
        if (bs.active[b]) {
            if (x < tol) bs.r2max[b] = (unsigned long long)__double_as_longlong(x);
            else if (x >= sqrt_n * tol) bs.r2max[b] = (unsigned long long)__double_as_longlong(x / sqrt_n);
            else e = 1;
        }
        expand[b] = e;
    }
}

// max |A[:, j]| over the columns of blocks flagged in expand, into r2max
__global__ __launch_bounds__(256) void k_colmax(const double* __restrict__ A, int n, long ld,
                                                 const int* __restrict__ colblk, const int* __restrict__ expand,
                                                 unsigned long long* __restrict__ out) {
    __shared__ double red[4];
    const int j = blockIdx.x;
    const int b = colblk[j];
    if (!expand[b]) return;
    double mx = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) mx = fmax(mx, fabs(A[i + (long)j * ld]));
    mx = block_max256(mx, red);
    if (threadIdx.x == 0) atomic_max_nonneg(&out[b], mx);
}

// Wk[:, j] = W[:, idx[j]] / sqrt(lam[idx[j]]) (m rows)
__global__ __launch_bounds__(256) void k_gather_scaled(const double* __restrict__ W, long ldw,
                                                        const double* __restrict__ lam,
                                                        const int* __restrict__ idx, double* __restrict__ Wk,
                                                        long ldk, int m) {
    const int j = blockIdx.x;
    const int src = idx[j];
    const double sc = lam[src] > 0.0 ? 1.0 / sqrt(lam[src]) : 0.0;
    for (int i = threadIdx.x; i < m; i += 256) Wk[i + j * ldk] = W[i + (long)src * ldw] * sc;
}

// T = (3 I - G) / 2 (r x r), the Newton-Schulz orthogonalisation factor
__global__ __launch_bounds__(256) void k_ns_factor(const double* __restrict__ G, double* __restrict__ T, int r) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long)r * r) return;
    const int i = (int)(idx % r), j = (int)(idx / r);
    T[idx] = (i == j ? 1.5 : 0.0) - 0.5 * G[idx];
}

__global__ __launch_bounds__(256) void k_estep(double* __restrict__ E, const double* __restrict__ V,
                                                double* __restrict__ Y1, int m, long ld, double lam,
                                                const int* __restrict__ colblk, BlockState bs,
                                                const DevIter* it) {
    __shared__ double red[4];
    const int j = blockIdx.x;
    const int b = colblk[j];
    if (!bs.active[b]) return;
    const double mu = it->mu;
    const long o = j * ld;
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        const double q = E[o + i] + V[o + i];   // = X - M Z + Y1/mu
        E[o + i] = q;
        s += q * q;
    }
    s = block_sum256(s, red);
    const double nrm = sqrt(s);
    const double thr = lam / mu;
    const double scale = (nrm > thr) ? 1.0 - thr / nrm : 0.0;
    double mx = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        const double q = E[o + i];
        const double e = q * scale;
        const double y1 = Y1[o + i];
        const double r1 = q - y1 / mu - e;
        Y1[o + i] = y1 + mu * r1;
        E[o + i] = e;
        mx = fmax(mx, fabs(r1));
    }
    mx = block_max256(mx, red);
    if (threadIdx.x == 0) bs.colr1[j] = mx;
}

// The same E-step with one wavefront per column and the column held in
// registers (a single pass over HBM: E, V and Y1 read once, E and Y1 written
// once, every load issued before the norm is reduced).  Lane l holds rows 2l
// and 2l + 1 of every 128-row chunk (16-byte accesses when VEC, i.e. even
// leading dimension); NCH chunks cover m <= 128 NCH.  The column norm is a
// fixed-order sum (per lane, then the wave butterfly).

template <int NCH, bool VEC>
__global__ __launch_bounds__(256) void k_estep_w(double* __restrict__ E, const double* __restrict__ V,
                                                  double* __restrict__ Y1, int m, long ld, int ncols, double lam,
                                                  const int* __restrict__ colblk, BlockState bs,
                                                  const DevIter* it) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= ncols) return;
    const int b = colblk[j];
    if (!bs.active[b]) return;
    const int lane = threadIdx.x & 63;
    const double mu = it->mu;
    const long o = (long)j * ld;
    double q[NCH][2], y[NCH][2];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int i = c * 128 + 2 * lane;
        double e0, e1, v0, v1;
        ld2<VEC>(E + o, i, m, e0, e1);
        ld2<VEC>(V + o, i, m, v0, v1);
        ld2<VEC>(Y1 + o, i, m, y[c][0], y[c][1]);
        q[c][0] = e0 + v0;   // = X - M Z + Y1/mu
        q[c][1] = e1 + v1;
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) s += q[c][0] * q[c][0] + q[c][1] * q[c][1];
    s = wave_sum(s);
    const double nrm = sqrt(s);
    const double thr = lam / mu;
    const double scale = (nrm > thr) ? 1.0 - thr / nrm : 0.0;
    double mx = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int i = c * 128 + 2 * lane;
        double e[2], yn[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            e[h] = q[c][h] * scale;
            const double r1 = q[c][h] - y[c][h] / mu - e[h];
            yn[h] = y[c][h] + mu * r1;
            if (i + h < m) mx = fmax(mx, fabs(r1));
        }
        st2<VEC>(E + o, i, m, e[0], e[1]);
        st2<VEC>(Y1 + o, i, m, yn[0], yn[1]);
    }
    mx = wave_max(mx);
    if (lane == 0) bs.colr1[j] = mx;
}

// k_update_Z with one wavefront per column (no workgroup barriers, 16-byte
// accesses when VEC, the loads of four 128-row chunks issued before their
// stores): Z = Q + M^T V, R2 = Z - J, Y2 += mu R2, and max|R2| or, in reduced
// coordinates, the coefficient residual and its column 2-norm.
template <bool VEC>
__global__ __launch_bounds__(256) void k_update_Z_w(const double* __restrict__ Q, const double* __restrict__ MtV,
                                                     const double* __restrict__ J, double* __restrict__ Z,
                                                     double* __restrict__ Y2, double* __restrict__ R2r,
                                                     unsigned long long* __restrict__ r2nrm, int n, long ld,
                                                     int ncols, const int* __restrict__ colblk, BlockState bs,
                                                     const DevIter* it) {
    constexpr int G = 4;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= ncols) return;
    const int b = colblk[j];
    if (!bs.active[b]) return;
    const int lane = threadIdx.x & 63;
    const double mu = it->mu;
    const long o = (long)j * ld;
    double mx = 0.0, ss = 0.0;
    for (int base = 0; base < n; base += 128 * G) {
        double q[G][2], w[G][2], jj[G][2], y[G][2];
#pragma unroll
        for (int c = 0; c < G; ++c) {
            const int i = base + c * 128 + 2 * lane;
            ld2<VEC>(Q + o, i, n, q[c][0], q[c][1]);
            ld2<VEC>(MtV + o, i, n, w[c][0], w[c][1]);
            ld2<VEC>(J + o, i, n, jj[c][0], jj[c][1]);
            ld2<VEC>(Y2 + o, i, n, y[c][0], y[c][1]);
        }
#pragma unroll
        for (int c = 0; c < G; ++c) {
            const int i = base + c * 128 + 2 * lane;
            double z[2], r2[2], yn[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                z[h] = q[c][h] + w[c][h];
                r2[h] = z[h] - jj[c][h];
                yn[h] = y[c][h] + mu * r2[h];
                mx = fmax(mx, fabs(r2[h]));   // rows past n hold zeros
                ss += r2[h] * r2[h];
            }
            st2<VEC>(Z + o, i, n, z[0], z[1]);
            st2<VEC>(Y2 + o, i, n, yn[0], yn[1]);
            if (R2r) st2<VEC>(R2r + o, i, n, r2[0], r2[1]);
        }
    }
    // per-column results (one store per wave; the per-block maxima follow in
    // k_block_colmax, without atomics on t addresses from every column)
    if (R2r) {
        ss = wave_sum(ss);
        if (lane == 0) bs.colr2[j] = sqrt(ss);
    } else {
        mx = wave_max(mx);
        if (lane == 0) bs.colr2[j] = mx;
    }
}

// per block: the largest per-column value of its columns, as the bit pattern of
// a non-negative double (one workgroup per block)
__global__ __launch_bounds__(256) void k_block_colmax(const double* __restrict__ col,
                                                       const double* __restrict__ col2,
                                                       const int* __restrict__ boff, BlockState bs,
                                                       unsigned long long* __restrict__ out,
                                                       unsigned long long* __restrict__ out2) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    if (!bs.active[b]) return;
    double mx = 0.0, mx2 = 0.0;
    for (int c = boff[b] + threadIdx.x; c < boff[b + 1]; c += 256) {
        mx = fmax(mx, col[c]);
        if (col2) mx2 = fmax(mx2, col2[c]);
    }
    mx = block_max256(mx, red);
    if (col2) mx2 = block_max256(mx2, red);
    if (threadIdx.x == 0) {
        out[b] = dbl_bits(mx);
        if (col2) out2[b] = dbl_bits(mx2);
    }
}

__global__ __launch_bounds__(256) void k_check(BlockState bs, int t, DevIter* it,
                                                const double* __restrict__ mu_sched, double tol,
                                                int fixed, int* n_active) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int k = it->k;
    for (int b = threadIdx.x; b < t; b += 256) {
        if (bs.active[b]) {
            const double r1 = __longlong_as_double((long long)bs.r1max[b]);
            const double r2 = __longlong_as_double((long long)bs.r2max[b]);
            bs.res1[b] = r1;
            bs.res2[b] = r2;
            bs.iters[b] = k + 1;
            if (!fixed && r1 < tol && r2 < tol) bs.active[b] = 0;
            else atomicAdd(&cnt, 1);
        }
        bs.r1max[b] = 0ull;
        bs.r2max[b] = 0ull;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        it->k = k + 1;
        it->mu = mu_sched[k + 1];
        it->tau = 1.0 / it->mu;
        *n_active = cnt;
    }
}

__global__ void k_init_iter(DevIter* it, const double* __restrict__ mu_sched, int k, int full) {
    it->k = k;
    it->full = full;
    it->mu = mu_sched[k];
    it->tau = 1.0 / mu_sched[k];
}

__global__ __launch_bounds__(256) void k_scale_cols(double* __restrict__ U, long ld, int rows,
                                                     const double* __restrict__ h) {
    const int j = blockIdx.x;
    const double s = h[j];
    for (int i = threadIdx.x; i < rows; i += 256) U[i + j * ld] *= s;
}

// block-diagonal scatter of per-block estimates (local mode): column j of the
// concatenated blocks, block bb, rows a < l_bb go to out[perm[boff_bb + a], perm[j]]
__global__ __launch_bounds__(256) void k_scatter_block_diag(const double* __restrict__ J, long ldj,
                                                             const int* __restrict__ colblk,
                                                             const int* __restrict__ boff,
                                                             const int* __restrict__ perm, double* __restrict__ out,
                                                             long ldo) {
    const int j = blockIdx.x;
    const int bb = colblk[j];
    const int o = boff[bb], l = boff[bb + 1] - o;
    double* col = out + (long)perm[j] * ldo;
    for (int a = threadIdx.x; a < l; a += 256) col[perm[o + a]] = J[a + j * ldj];
}

__global__ void k_set_identity(double* __restrict__ W, int L) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < (long)L * L) W[idx] = ((idx % L) == (idx / L)) ? 1.0 : 0.0;
}

}  // namespace

void launch_gather_cols(const double* M, long ldm, double* X, long ldx, int m, int ncols,
                        const int* d_perm, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_cols, dim3(ncols), dim3(256), 0, s, M, ldm, X, ldx, m, d_perm);
}
void launch_scatter_cols(const double* X, long ldx, double* S, long lds, int m, int ncols,
                         const int* d_perm, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_cols, dim3(ncols), dim3(256), 0, s, X, ldx, S, lds, m, d_perm);
}
void launch_copy_cols(const double* X, long ldx, double* Y, long ldy, int m, int ncols, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_cols, dim3(ncols), dim3(256), 0, s, X, ldx, Y, ldy, m);
}
void launch_widen_cols(const float* src, long lds, double* dst, long ldd, int rows, int cols, hipStream_t s) {
    if (rows > 0 && cols > 0)
        hipLaunchKernelGGL((k_convert_cols<float, double>), dim3(cols), dim3(256), 0, s, src, lds, dst, ldd, rows);
}
void launch_narrow_cols(const double* src, long lds, float* dst, long ldd, int rows, int cols, hipStream_t s) {
    if (rows > 0 && cols > 0)
        hipLaunchKernelGGL((k_convert_cols<double, float>), dim3(cols), dim3(256), 0, s, src, lds, dst, ldd, rows);
}
void launch_nonfinite(const double* M, long ldm, int m, int n, int* d_flag, hipStream_t s) {
    hipLaunchKernelGGL(k_nonfinite, dim3(n), dim3(256), 0, s, M, ldm, m, d_flag);
}
void launch_form_Y(const double* Z, const double* Y2, double* Y, double* colsq, int n, long ld, int ncols,
                   const int* colblk, const int* active, const DevIter* it, hipStream_t s) {
    hipLaunchKernelGGL(k_form_Y, dim3(ncols), dim3(256), 0, s, Z, Y2, Y, colsq, n, ld, colblk, active, it);
}
void launch_block_fro(const double* colsq, const int* boff, int t, BlockState bs, const DevIter* it,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_block_fro, dim3(t), dim3(256), 0, s, colsq, boff, bs, it);
}
void launch_eig_select(const double* colsq, const int* boff, int t, const int* active, const int* svt_run,
                       const int* warm, int* eig_run, const DevIter* it, double prewarm, hipStream_t s) {
    hipLaunchKernelGGL(k_eig_select, dim3(1), dim3(256), 0, s, colsq, boff, t, active, svt_run, warm, eig_run, it,
                       prewarm);
}
void launch_zero_J(double* J, int n, long ld, int ncols, const int* colblk, BlockState bs, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_J, dim3(ncols), dim3(256), 0, s, J, n, ld, colblk, bs);
}
void launch_svt_weights(const SvtDesc* d, int count, int maxL, const DevIter* it, BlockState bs,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_svt_weights, dim3((maxL + 3) / 4, count), dim3(256), 0, s, d, it, bs);
}
void launch_form_QT(const double* J, const double* Y2, double* Q, double* dQ, int n, long ldn,
                    const double* X, const double* E, const double* Y1, double* T, int m, long ldm, int ncols,
                    const int* colblk, const int* active, const DevIter* it, hipStream_t s) {
    hipLaunchKernelGGL(k_form_QT, dim3(ncols), dim3(256), 0, s, J, Y2, Q, dQ, n, ldn, X, E, Y1, T, m, ldm,
                       colblk, active, it);
}
void launch_sub_cols(double* T, const double* A, int m, long ld, int ncols, const int* colblk,
                     const int* active, hipStream_t s) {
    hipLaunchKernelGGL(k_sub_cols, dim3(ncols), dim3(256), 0, s, T, A, m, ld, colblk, active);
}
void launch_update_Z(const double* Q, const double* MtV, const double* J, double* Z, double* Y2, double* R2r,
                     unsigned long long* r2nrm, int n, long ld, int ncols, const int* colblk, BlockState bs,
                     const DevIter* it, hipStream_t s) {
    const dim3 grid((ncols + 3) / 4);
    if ((ld & 1) == 0)
        hipLaunchKernelGGL((k_update_Z_w<true>), grid, dim3(256), 0, s, Q, MtV, J, Z, Y2, R2r, r2nrm, n, ld, ncols,
                           colblk, bs, it);
    else
        hipLaunchKernelGGL((k_update_Z_w<false>), grid, dim3(256), 0, s, Q, MtV, J, Z, Y2, R2r, r2nrm, n, ld, ncols,
                           colblk, bs, it);
}
void launch_block_colmax(const double* col, const int* boff, int t, BlockState bs, unsigned long long* out,
                         hipStream_t s, const double* col2, unsigned long long* out2) {
    hipLaunchKernelGGL(k_block_colmax, dim3(t), dim3(256), 0, s, col, col2, boff, bs, out, out2);
}
void launch_r2_decide(BlockState bs, unsigned long long* r2nrm, int* expand, int t, double tol, double sqrt_n,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_r2_decide, dim3(1), dim3(256), 0, s, bs, r2nrm, expand, t, tol, sqrt_n);
}
void launch_colmax(const double* A, int n, long ld, int ncols, const int* colblk, const int* expand,
                   unsigned long long* out, hipStream_t s) {
    hipLaunchKernelGGL(k_colmax, dim3(ncols), dim3(256), 0, s, A, n, ld, colblk, expand, out);
}
void launch_gather_scaled(const double* W, long ldw, const double* lam, const int* idx, double* Wk, long ldk,
                          int m, int r, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_scaled, dim3(r), dim3(256), 0, s, W, ldw, lam, idx, Wk, ldk, m);
}
void launch_ns_factor(const double* G, double* T, int r, hipStream_t s) {
    const long nn = (long)r * r;
    hipLaunchKernelGGL(k_ns_factor, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, G, T, r);
}
template <int NCH>
void launch_estep_w(double* E, const double* V, double* Y1, int m, long ld, int ncols, double lam,
                    const int* colblk, BlockState bs, const DevIter* it, hipStream_t s) {
    const dim3 grid((ncols + 3) / 4);
    if ((ld & 1) == 0)
        hipLaunchKernelGGL((k_estep_w<NCH, true>), grid, dim3(256), 0, s, E, V, Y1, m, ld, ncols, lam, colblk, bs,
                           it);
    else
        hipLaunchKernelGGL((k_estep_w<NCH, false>), grid, dim3(256), 0, s, E, V, Y1, m, ld, ncols, lam, colblk, bs,
                           it);
}

void launch_estep(double* E, const double* V, double* Y1, int m, long ld, int ncols, double lam,
                  const int* colblk, BlockState bs, const DevIter* it, hipStream_t s) {
    // the column in registers up to m = 2048; beyond, the two-pass workgroup kernel
    if (m <= 128) launch_estep_w<1>(E, V, Y1, m, ld, ncols, lam, colblk, bs, it, s);
    else if (m <= 256) launch_estep_w<2>(E, V, Y1, m, ld, ncols, lam, colblk, bs, it, s);
    else if (m <= 512) launch_estep_w<4>(E, V, Y1, m, ld, ncols, lam, colblk, bs, it, s);
    else if (m <= 1024) launch_estep_w<8>(E, V, Y1, m, ld, ncols, lam, colblk, bs, it, s);
    else if (m <= 2048) launch_estep_w<16>(E, V, Y1, m, ld, ncols, lam, colblk, bs, it, s);
    else hipLaunchKernelGGL(k_estep, dim3(ncols), dim3(256), 0, s, E, V, Y1, m, ld, lam, colblk, bs, it);
}
void launch_check(BlockState bs, int t, DevIter* it, const double* mu_sched, double tol, int fixed,
                  int* n_active, hipStream_t s) {
    hipLaunchKernelGGL(k_check, dim3(1), dim3(256), 0, s, bs, t, it, mu_sched, tol, fixed, n_active);
}
void launch_init_iter(DevIter* it, const double* mu_sched, int k, hipStream_t s, int full) {
    hipLaunchKernelGGL(k_init_iter, dim3(1), dim3(1), 0, s, it, mu_sched, k, full);
}
void launch_scale_cols(double* U, long ld, int rows, int ncols, const double* h, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_cols, dim3(ncols), dim3(256), 0, s, U, ld, rows, h);
}
void launch_scatter_block_diag(const double* J, long ldj, int ncols, const int* colblk, const int* boff,
                               const int* perm, double* out, long ldo, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_block_diag, dim3(ncols), dim3(256), 0, s, J, ldj, colblk, boff, perm, out, ldo);
}
void launch_set_identity(double* W, int L, hipStream_t s) {
    const long n = (long)L * L;
    hipLaunchKernelGGL(k_set_identity, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, L);
}

}  // namespace lrr
