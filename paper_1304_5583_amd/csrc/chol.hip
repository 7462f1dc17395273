// FP64 blocked Cholesky factorisation and explicit SPD inverse.
//
// The Z-step of the ALM solves with K = I + A^T A, or with the m x m matrix
// I + A A^T through (I + A^T A)^{-1} = I - A^T (I + A A^T)^{-1} A.  K is
// factored once per solve (it depends only on the dictionary M, which is shared
// by all blocks), K = L L^T, and K^{-1} = L^{-T} L^{-1} is formed explicitly so
// that every iteration applies it as one GEMM.  K has eigenvalues >= 1, so its
// condition number is 1 + ||A||^2 and the explicit inverse is benign.
//
// Right-looking blocked Cholesky with panels of kNB columns:
//   diag block  one workgroup factors it in LDS and inverts the factor,
//   panel       L21 = A21 L11^{-T}        (GEMM with the inverted block),
//   trailing    A22 -= L21 L21^T          (GEMM).
// The inverse factor is built block row by block row,
//   Linv[I, :I] = -Linv[I, I] (L[I, :I] Linv[:I, :I]),
// and K^{-1} = Linv^T Linv is a final GEMM.
#include "common.hpp"
#include "kernels.hpp"

#include <vector>

namespace lrr {

namespace {

constexpr int kNB = 32;

__global__ void k_add_identity(double* A, int lda, int m, double s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) A[i + (long)i * lda] += s;
}

// factor the nb x nb diagonal block at (k0, k0) of Aw into Lo, invert it into Dinv
__global__ __launch_bounds__(256) void k_potrf_diag(const double* __restrict__ Aw, int lda,
                                                     double* __restrict__ Lo, int ldl,
                                                     double* __restrict__ Dinv, int ldd,
                                                     int k0, int nb, int* info) {
    __shared__ double S[kNB][kNB + 1];
    __shared__ double X[kNB][kNB + 1];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < kNB * kNB; idx += 256) {
        const int i = idx % kNB, j = idx / kNB;
        S[i][j] = (i < nb && j < nb) ? Aw[(k0 + i) + (long)(k0 + j) * lda] : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (tid == 0) {
            const double piv = S[j][j];
            if (!(piv > 0.0)) atomicExch(info, k0 + j + 1);
            S[j][j] = sqrt(fmax(piv, 1e-300));
        }
        __syncthreads();
        const double djj = S[j][j];
        for (int i = j + 1 + tid; i < nb; i += 256) S[i][j] /= djj;
        __syncthreads();
        for (int idx = tid; idx < nb * nb; idx += 256) {
            const int i = idx % nb, k = idx / nb;
            if (k > j && i >= k) S[i][k] -= S[i][j] * S[k][j];
        }
        __syncthreads();
    }
    // inverse of the lower-triangular factor, one column per thread
    if (tid < nb) {
        const int c = tid;
        for (int i = 0; i < nb; ++i) {
            if (i < c) { X[i][c] = 0.0; continue; }
            double acc = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) acc -= S[i][k] * X[k][c];
            X[i][c] = acc / S[i][i];
        }
    }
    __syncthreads();
    for (int idx = tid; idx < nb * nb; idx += 256) {
        const int i = idx % nb, j = idx / nb;
        Lo[(k0 + i) + (long)(k0 + j) * ldl] = (i >= j) ? S[i][j] : 0.0;
        Dinv[(k0 + i) + (long)j * ldd] = X[i][j];
    }
}

// copy a diagonal inverse block into Linv
__global__ void k_copy_block(const double* __restrict__ src, int lds, double* __restrict__ dst, int ldd,
                             int rows, int cols) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i < rows && j < cols) dst[i + (long)j * ldd] = src[i + (long)j * lds];
}

}  // namespace

int spd_inverse_desc_count(int m) {
    const int nblk = (m + kNB - 1) / kNB;
    return 4 * nblk + 1;
}

// K (m x m, SPD, ld = m) is overwritten by K^{-1}.  Work buffers: Lbuf, Linv,
// Tbuf (m x m), Dinv (m x kNB), all ld = m.  d_desc holds at least
// spd_inverse_desc_count(m) descriptors; d_info receives 1 + the index of a
// non-positive pivot (0 if none).
void spd_inverse(double* K, int m, double* Lbuf, double* Linv, double* Dinv, double* Tbuf,
                 GemmDesc* d_desc, int* d_info, hipStream_t s) {
    struct Op { int kind; int a; int b; bool ta, tb; };   // 0 potrf, 1 copy, 2 gemm
    std::vector<Op> ops;
    std::vector<GemmDesc> descs;
    auto gemm = [&](const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                    int M, int N, int Kd, double alpha, double beta, bool ta, bool tb) {
        if (M <= 0 || N <= 0 || Kd <= 0) return;
        descs.push_back(GemmDesc{A, B, C, M, N, Kd, lda, ldb, ldc, alpha, beta, nullptr, nullptr});
        ops.push_back(Op{2, (int)descs.size() - 1, 0, ta, tb});
    };
    for (int k0 = 0; k0 < m; k0 += kNB) {
        const int nb = (m - k0 < kNB) ? (m - k0) : kNB;
        ops.push_back(Op{0, k0, nb, false, false});
        const int k1 = k0 + nb;
        if (k1 < m) {
            // L21 = A21 * Dinv^T
            gemm(K + k1 + (long)k0 * m, m, Dinv + k0, m, Lbuf + k1 + (long)k0 * m, m, m - k1, nb, nb,
                 1.0, 0.0, false, true);
            // A22 -= L21 L21^T
            gemm(Lbuf + k1 + (long)k0 * m, m, Lbuf + k1 + (long)k0 * m, m, K + k1 + (long)k1 * m, m,
                 m - k1, m - k1, nb, -1.0, 1.0, false, true);
        }
    }
    for (int r0 = 0; r0 < m; r0 += kNB) {
        const int nb = (m - r0 < kNB) ? (m - r0) : kNB;
        ops.push_back(Op{1, r0, nb, false, false});
        if (r0 > 0) {
            // Tm = L[I, :r0] * Linv[:r0, :r0]   (nb x r0)
            gemm(Lbuf + r0, m, Linv, m, Tbuf, m, nb, r0, r0, 1.0, 0.0, false, false);
            // Linv[I, :r0] = -Dinv_I * Tm
            gemm(Dinv + r0, m, Tbuf, m, Linv + r0, m, nb, r0, nb, -1.0, 0.0, false, false);
        }
    }
    // K^{-1} = Linv^T Linv (written over K, which the factorisation consumed)
    gemm(Linv, m, Linv, m, K, m, m, m, m, 1.0, 0.0, true, false);

    LRR_HIP(hipMemsetAsync(Lbuf, 0, sizeof(double) * (size_t)m * m, s));
    LRR_HIP(hipMemsetAsync(Linv, 0, sizeof(double) * (size_t)m * m, s));
    LRR_HIP(hipMemsetAsync(d_info, 0, sizeof(int), s));
    LRR_HIP(hipMemcpyAsync(d_desc, descs.data(), sizeof(GemmDesc) * descs.size(),
                           hipMemcpyHostToDevice, s));
    for (const Op& op : ops) {
        if (op.kind == 0) {
            hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, K, m, Lbuf, m, Dinv, m,
                               op.a, op.b, d_info);
        } else if (op.kind == 1) {
            hipLaunchKernelGGL(k_copy_block, dim3((op.b + 63) / 64, op.b), dim3(64), 0, s,
                               Dinv + op.a, m, Linv + op.a + (long)op.a * m, m, op.b, op.b);
        } else {
            const GemmDesc& h = descs[op.a];
            launch_dgemm(d_desc + op.a, 1, h.M, h.N, op.ta, op.tb, s);
        }
    }
    // the host copy of the descriptors must outlive the asynchronous upload
    LRR_HIP(hipStreamSynchronize(s));
}

void launch_add_identity(double* A, int lda, int m, double s, hipStream_t st) {
    hipLaunchKernelGGL(k_add_identity, dim3((m + 255) / 256), dim3(256), 0, st, A, lda, m, s);
}

}  // namespace lrr
