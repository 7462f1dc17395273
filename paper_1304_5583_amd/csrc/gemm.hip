// Batched FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64).
//
// Every dense contraction of the solver goes through here: the Gram matrices
// A A^T and Y^T Y, the dictionary products M Q and M^T V, the solve with the
// inverse factor, the reconstruction of the thresholded block and the combine.
//
// Tiling: a 256-thread workgroup owns a 64 x 64 tile of C; each of its four
// 64-wide wavefronts owns a 32 x 32 quarter as 2 x 2 MFMA tiles of 16 x 16.
// K advances in steps of 16 (four MFMA k-chunks of 4), operands staged
// through LDS with zero fill at the matrix edges, so any M, N, K is legal.
#include "common.hpp"
#include "kernels.hpp"

namespace lrr {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, PAD = 2;

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_dgemm(const GemmDesc* __restrict__ descs) {
    const GemmDesc d = descs[blockIdx.z];
    if (d.active && d.active[0] == 0) return;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    if (m0 >= d.M || n0 >= d.N) return;

    __shared__ double As[BK][BM + PAD];   // As[k][i] = op(A)(m0 + i, k0 + k)
    __shared__ double Bs[BK][BN + PAD];   // Bs[k][j] = op(B)(k0 + k, n0 + j)

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;

    dbl4 acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};

    const double* __restrict__ A = d.A;
    const double* __restrict__ B = d.B;
    const int M = d.M, N = d.N, K = d.K;
    const long lda = d.lda, ldb = d.ldb;

    for (int k0 = 0; k0 < K; k0 += BK) {
        if (!TA) {   // op(A)(i,k) = A[i + k*lda]: contiguous in i
            const int k = tid >> 4, i = (tid & 15) * 4;
            const int gk = k0 + k;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = m0 + i + v;
                As[k][i + v] = (gi < M && gk < K) ? A[gi + gk * lda] : 0.0;
            }
        } else {     // op(A)(i,k) = A[k + i*lda]: contiguous in k
            const int i = tid >> 2, k = (tid & 3) * 4;
            const int gi = m0 + i;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gk = k0 + k + v;
                As[k + v][i] = (gi < M && gk < K) ? A[gk + gi * lda] : 0.0;
            }
        }
        if (!TB) {   // op(B)(k,j) = B[k + j*ldb]: contiguous in k
            const int j = tid >> 2, k = (tid & 3) * 4;
            const int gj = n0 + j;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gk = k0 + k + v;
                Bs[k + v][j] = (gj < N && gk < K) ? B[gk + gj * ldb] : 0.0;
            }
        } else {     // op(B)(k,j) = B[j + k*ldb]: contiguous in j
            const int k = tid >> 4, j = (tid & 15) * 4;
            const int gk = k0 + k;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gj = n0 + j + v;
                Bs[k][j + v] = (gj < N && gk < K) ? B[gj + gk * ldb] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + lk;
            const double a0 = As[kr][wm + lr], a1 = As[kr][wm + 16 + lr];
            const double b0 = Bs[kr][wn + lr], b1 = Bs[kr][wn + 16 + lr];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }

    // accumulator layout of v_mfma_f64_16x16x4f64: register v of a lane holds
    // row lane/16 + 4v, column lane%16 of the 16 x 16 tile
    const double alpha = d.alpha, beta = d.beta;
    const long ldc = d.ldc;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int gj = n0 + wn + y * 16 + lr;
            if (gj >= N) continue;
            const int cj = d.colmap ? d.colmap[gj] : gj;
            double* __restrict__ Cc = d.C + (long)cj * ldc;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = m0 + wm + x * 16 + lk + 4 * v;
                if (gi < M) {
                    double r = alpha * acc[x][y][v];
                    if (beta != 0.0) r += beta * Cc[gi];
                    Cc[gi] = r;
                }
            }
        }
    }
}

}  // namespace

void launch_dgemm(const GemmDesc* d_descs, int count, int maxM, int maxN, bool ta, bool tb,
                  hipStream_t stream) {
    if (count <= 0 || maxM <= 0 || maxN <= 0) return;
    dim3 grid((maxM + BM - 1) / BM, (maxN + BN - 1) / BN, count);
    dim3 block(256);
    if (!ta && !tb) hipLaunchKernelGGL((k_dgemm<false, false>), grid, block, 0, stream, d_descs);
    else if (ta && !tb) hipLaunchKernelGGL((k_dgemm<true, false>), grid, block, 0, stream, d_descs);
    else if (!ta && tb) hipLaunchKernelGGL((k_dgemm<false, true>), grid, block, 0, stream, d_descs);
    else hipLaunchKernelGGL((k_dgemm<true, true>), grid, block, 0, stream, d_descs);
}

}  // namespace lrr
