// Batched FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64).
//
// Every dense contraction of the solver goes through here: the Gram matrices
// A A^T and Y^T Y, the dictionary products M Q and M^T V, the solve with the
// inverse factor, the reconstruction of the thresholded block and the combine.
//
// Tiling: a 256-thread workgroup owns a 64 x 64 tile of C; each of its four
// 64-wide wavefronts owns a 32 x 32 quarter as 2 x 2 MFMA tiles of 16 x 16.
// K advances in steps of 16 (four MFMA k-chunks of 4).  Operand tiles are
// double-buffered in LDS and the next tile is fetched into registers while the
// current one is multiplied, so a workgroup hides its own load latency.  With
// 16-deep tiles a workgroup holds 34 KB of LDS, so four fit on a CU (32-deep
// tiles allowed two and ran the batched 512-order products at 38-40 instead of
// 44-47 TFLOP/s).  Loads zero-fill at the matrix edges, so any M, N, K is legal.
#include "common.hpp"
#include "kernels.hpp"

namespace lrr {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, PAD = 2;
constexpr int NLD = (BM * BK) / 256;   // elements of each operand tile per thread

// One K-tile of op(A) (BM x BK) and op(B) (BK x BN) in registers.
struct Frag {
    double a[NLD];
    double b[NLD];
};

template <bool TA, bool TB>
__device__ __forceinline__ void load_tile(Frag& f, const double* __restrict__ A, long lda,
                                          const double* __restrict__ B, long ldb, int M, int N, int K,
                                          int m0, int n0, int k0, int tid) {
    if (!TA) {   // op(A)(i,k) = A[i + k*lda]: 16 threads cover 64 rows of one k
        const int i = (tid & 15) * 4, kk = tid >> 4;
#pragma unroll
        for (int h = 0; h < NLD / 4; ++h) {
            const int gk = k0 + kk + 16 * h;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = m0 + i + v;
                f.a[4 * h + v] = (gi < M && gk < K) ? A[gi + gk * lda] : 0.0;
            }
        }
    } else {     // op(A)(i,k) = A[k + i*lda]: 8 threads cover 32 k of one row
        const int i = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
        for (int h = 0; h < NLD / 4; ++h) {
            const int gi = m0 + i;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gk = k0 + kk + 16 * h + v;
                f.a[4 * h + v] = (gi < M && gk < K) ? A[gk + gi * lda] : 0.0;
            }
        }
    }
    if (!TB) {   // op(B)(k,j) = B[k + j*ldb]: contiguous in k
        const int j = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
        for (int h = 0; h < NLD / 4; ++h) {
            const int gj = n0 + j;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gk = k0 + kk + 16 * h + v;
                f.b[4 * h + v] = (gj < N && gk < K) ? B[gk + gj * ldb] : 0.0;
            }
        }
    } else {     // op(B)(k,j) = B[j + k*ldb]: contiguous in j
        const int j = (tid & 15) * 4, kk = tid >> 4;
#pragma unroll
        for (int h = 0; h < NLD / 4; ++h) {
            const int gk = k0 + kk + 16 * h;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gj = n0 + j + v;
                f.b[4 * h + v] = (gj < N && gk < K) ? B[gj + gk * ldb] : 0.0;
            }
        }
    }
}

template <bool TA, bool TB>
__device__ __forceinline__ void store_tile(const Frag& f, double (*As)[BM + PAD], double (*Bs)[BN + PAD],
                                           int tid) {
    if (!TA) {
        const int i = (tid & 15) * 4, kk = tid >> 4;
#pragma unroll
        for (int h = 0; h < NLD / 4; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v) As[kk + 16 * h][i + v] = f.a[4 * h + v];
    } else {
        const int i = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
        for (int h = 0; h < NLD / 4; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v) As[kk + 16 * h + v][i] = f.a[4 * h + v];
    }
    if (!TB) {
        const int j = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
        for (int h = 0; h < NLD / 4; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v) Bs[kk + 16 * h + v][j] = f.b[4 * h + v];
    } else {
        const int j = (tid & 15) * 4, kk = tid >> 4;
#pragma unroll
        for (int h = 0; h < NLD / 4; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v) Bs[kk + 16 * h][j + v] = f.b[4 * h + v];
    }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_dgemm(const GemmDesc* __restrict__ descs) {
    const GemmDesc d = descs[blockIdx.z];
    if (d.active && d.active[0] == 0) return;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    if (m0 >= d.M || n0 >= d.N) return;

    // double-buffered operand tiles: As[buf][k][i] = op(A)(m0+i, k0+k)
    __shared__ double As[2][BK][BM + PAD];
    __shared__ double Bs[2][BK][BN + PAD];

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

    Frag f;
    load_tile<TA, TB>(f, A, lda, B, ldb, M, N, K, m0, n0, 0, tid);
    store_tile<TA, TB>(f, As[0], Bs[0], tid);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < K; k0 += BK) {
        const bool more = k0 + BK < K;
        // the next tile's global loads are in flight while this one is multiplied
        if (more) load_tile<TA, TB>(f, A, lda, B, ldb, M, N, K, m0, n0, k0 + BK, tid);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + lk;
            const double a0 = As[cur][kr][wm + lr], a1 = As[cur][kr][wm + 16 + lr];
            const double b0 = Bs[cur][kr][wn + lr], b1 = Bs[cur][kr][wn + 16 + lr];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (more) store_tile<TA, TB>(f, As[cur ^ 1], Bs[cur ^ 1], tid);
        __syncthreads();
        cur ^= 1;
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
