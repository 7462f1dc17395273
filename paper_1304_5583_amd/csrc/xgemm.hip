// Reduced-precision products on the matrix cores, FP64 in and out.
//
// Same contract as the FP64 GEMM (GemmDesc: C = alpha op(A) op(B) + beta C,
// column-major FP64 storage), but the product runs on a faster matrix-core
// instruction with FP32 accumulation:
//   kFP32   operands rounded to FP32, v_mfma_f32_16x16x4f32;
//   kBF16X3 each operand split into two BF16 numbers x = hi + lo (hi = bf16(x),
//           lo = bf16(x - hi)) and the product formed as hi*hi + hi*lo + lo*hi
//           with v_mfma_f32_16x16x16_bf16 (the split-product method of Henry,
//           Tang and Heinecke, ARITH 2019).  The dropped lo*lo term and the
//           16-bit split leave a relative error of a few 2^-16 per product.
// The conversion happens while a tile is staged to LDS, so the kernel reads
// the FP64 state directly.  Tiling as in the FP64 kernel: 64 x 64 per
// 256-thread workgroup, 32 x 32 per wave as 2 x 2 MFMA tiles, K steps of 32,
// double-buffered LDS with the next tile prefetched into registers.
#include "common.hpp"
#include "kernels.hpp"

namespace lrr {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int NLD = (BM * BK) / 256;

// round-to-nearest-even FP32 -> BF16 (bit pattern), finite inputs
__device__ __forceinline__ unsigned short to_bf16(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

struct Frag {
    double a[NLD];
    double b[NLD];
};

template <bool TA, bool TB>
__device__ __forceinline__ void load_tile(Frag& f, const double* __restrict__ A, long lda,
                                          const double* __restrict__ B, long ldb, int M, int N, int K,
                                          int m0, int n0, int k0, int tid) {
    if (!TA) {
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
    } else {
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
    if (!TB) {
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
    } else {
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

// element (i, k) of the A tile / (k, j) of the B tile held by register r of a thread
template <bool TA>
__device__ __forceinline__ void a_coord(int tid, int r, int& i, int& k) {
    const int h = r >> 2, v = r & 3;
    if (!TA) { i = (tid & 15) * 4 + v; k = (tid >> 4) + 16 * h; }
    else { i = tid >> 2; k = (tid & 3) * 4 + 16 * h + v; }
}
template <bool TB>
__device__ __forceinline__ void b_coord(int tid, int r, int& k, int& j) {
    const int h = r >> 2, v = r & 3;
    if (!TB) { j = tid >> 2; k = (tid & 3) * 4 + 16 * h + v; }
    else { j = (tid & 15) * 4 + v; k = (tid >> 4) + 16 * h; }
}

// ---------------------------------------------------------------- FP32 variant
typedef float SA[2][BK][BM + 4];   // [k][i]
typedef float SB[2][BK][BN + 4];   // [k][j]

// acc += op(A) op(B) over the whole K range (tiles m0, n0 of this workgroup)
template <bool TA, bool TB>
__device__ __forceinline__ void s_kloop(f4 (&acc)[2][2], SA& As, SB& Bs, const double* __restrict__ A, long lda,
                                        const double* __restrict__ B, long ldb, int M, int N, int K, int m0,
                                        int n0) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    Frag f;
    auto stage = [&](int buf) {
#pragma unroll
        for (int r = 0; r < NLD; ++r) {
            int i, k, j, kb;
            a_coord<TA>(tid, r, i, k);
            b_coord<TB>(tid, r, kb, j);
            As[buf][k][i] = (float)f.a[r];
            Bs[buf][kb][j] = (float)f.b[r];
        }
    };
    load_tile<TA, TB>(f, A, lda, B, ldb, M, N, K, m0, n0, 0, tid);
    stage(0);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < K; k0 += BK) {
        const bool more = k0 + BK < K;
        if (more) load_tile<TA, TB>(f, A, lda, B, ldb, M, N, K, m0, n0, k0 + BK, tid);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + lk;
            const float a0 = As[cur][kr][wm + lr], a1 = As[cur][kr][wm + 16 + lr];
            const float b0 = Bs[cur][kr][wn + lr], b1 = Bs[cur][kr][wn + 16 + lr];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (more) stage(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_sgemm(const GemmDesc* __restrict__ descs) {
    const GemmDesc d = descs[blockIdx.z];
    if (d.active && d.active[0] == 0) return;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    if (m0 >= d.M || n0 >= d.N) return;
    __shared__ __attribute__((aligned(16))) SA As;
    __shared__ __attribute__((aligned(16))) SB Bs;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    f4 acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = f4{0.f, 0.f, 0.f, 0.f};
    s_kloop<TA, TB>(acc, As, Bs, d.A, d.lda, d.B, d.ldb, d.M, d.N, d.K, m0, n0);
    // f32 16x16x4 accumulator layout: register v holds row 4*(lane/16) + v, column lane%16
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int gj = n0 + wn + y * 16 + lr;
            if (gj >= d.N) continue;
            const int cj = d.colmap ? d.colmap[gj] : gj;
            double* __restrict__ Cc = d.C + (long)cj * d.ldc;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = m0 + wm + x * 16 + 4 * lk + v;
                if (gi < d.M) {
                    double r = d.alpha * (double)acc[x][y][v];
                    if (d.beta != 0.0) r += d.beta * Cc[gi];
                    Cc[gi] = r;
                }
            }
        }
}

// ---------------------------------------------------------------- BF16x3 variant
// [row][k] with k contiguous: a lane reads its 4 consecutive k as one 8-byte load
typedef unsigned short HA[2][BM][BK + 4];
typedef unsigned short HB[2][BN][BK + 4];

template <bool TA, bool TB>
__device__ __forceinline__ void b_kloop(f4 (&acc)[2][2], f4 (&acs)[2][2], HA& Ahi, HA& Alo, HB& Bhi, HB& Blo,
                                        const double* __restrict__ A, long lda, const double* __restrict__ B,
                                        long ldb, int M, int N, int K, int m0, int n0) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    Frag f;
    auto stage = [&](int buf) {
#pragma unroll
        for (int r = 0; r < NLD; ++r) {
            int i, k, j, kb;
            a_coord<TA>(tid, r, i, k);
            b_coord<TB>(tid, r, kb, j);
            const unsigned short ah = to_bf16((float)f.a[r]);
            Ahi[buf][i][k] = ah;
            Alo[buf][i][k] = to_bf16((float)(f.a[r] - (double)from_bf16(ah)));
            const unsigned short bh = to_bf16((float)f.b[r]);
            Bhi[buf][j][kb] = bh;
            Blo[buf][j][kb] = to_bf16((float)(f.b[r] - (double)from_bf16(bh)));
        }
    };
    load_tile<TA, TB>(f, A, lda, B, ldb, M, N, K, m0, n0, 0, tid);
    stage(0);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < K; k0 += BK) {
        const bool more = k0 + BK < K;
        if (more) load_tile<TA, TB>(f, A, lda, B, ldb, M, N, K, m0, n0, k0 + BK, tid);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            const int kq = kk + 4 * lk;   // this lane's 4 k values
            s4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                ah[x] = *reinterpret_cast<const s4*>(&Ahi[cur][wm + 16 * x + lr][kq]);
                al[x] = *reinterpret_cast<const s4*>(&Alo[cur][wm + 16 * x + lr][kq]);
                bh[x] = *reinterpret_cast<const s4*>(&Bhi[cur][wn + 16 * x + lr][kq]);
                bl[x] = *reinterpret_cast<const s4*>(&Blo[cur][wn + 16 * x + lr][kq]);
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    acs[x][y] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[x], bl[y], acs[x][y], 0, 0, 0);
                    acs[x][y] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[x], bh[y], acs[x][y], 0, 0, 0);
                    acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[x], bh[y], acc[x][y], 0, 0, 0);
                }
        }
        if (more) stage(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_bgemm3(const GemmDesc* __restrict__ descs) {
    const GemmDesc d = descs[blockIdx.z];
    if (d.active && d.active[0] == 0) return;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    if (m0 >= d.M || n0 >= d.N) return;
    __shared__ __attribute__((aligned(16))) HA Ahi, Alo;
    __shared__ __attribute__((aligned(16))) HB Bhi, Blo;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    // hi*hi and the two cross terms are accumulated separately
    f4 acc[2][2], acs[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) { acc[x][y] = f4{0.f, 0.f, 0.f, 0.f}; acs[x][y] = acc[x][y]; }
    b_kloop<TA, TB>(acc, acs, Ahi, Alo, Bhi, Blo, d.A, d.lda, d.B, d.ldb, d.M, d.N, d.K, m0, n0);
    // bf16 16x16x16 accumulator layout: register v holds row 4*(lane/16) + v, column lane%16
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int gj = n0 + wn + y * 16 + lr;
            if (gj >= d.N) continue;
            const int cj = d.colmap ? d.colmap[gj] : gj;
            double* __restrict__ Cc = d.C + (long)cj * d.ldc;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = m0 + wm + x * 16 + 4 * lk + v;
                if (gi < d.M) {
                    double r = d.alpha * ((double)acc[x][y][v] + (double)acs[x][y][v]);
                    if (d.beta != 0.0) r += d.beta * Cc[gi];
                    Cc[gi] = r;
                }
            }
        }
}

}  // namespace

void launch_xgemm(const GemmDesc* d_descs, int count, int maxM, int maxN, bool ta, bool tb, int mode,
                  hipStream_t stream) {
    if (mode == kGemmFP64) {
        launch_dgemm(d_descs, count, maxM, maxN, ta, tb, stream);
        return;
    }
    if (count <= 0 || maxM <= 0 || maxN <= 0) return;
    dim3 grid((maxM + BM - 1) / BM, (maxN + BN - 1) / BN, count);
    dim3 block(256);
    if (mode == kGemmFP32) {
        if (!ta && !tb) hipLaunchKernelGGL((k_sgemm<false, false>), grid, block, 0, stream, d_descs);
        else if (ta && !tb) hipLaunchKernelGGL((k_sgemm<true, false>), grid, block, 0, stream, d_descs);
        else if (!ta && tb) hipLaunchKernelGGL((k_sgemm<false, true>), grid, block, 0, stream, d_descs);
        else hipLaunchKernelGGL((k_sgemm<true, true>), grid, block, 0, stream, d_descs);
    } else {
        if (!ta && !tb) hipLaunchKernelGGL((k_bgemm3<false, false>), grid, block, 0, stream, d_descs);
        else if (ta && !tb) hipLaunchKernelGGL((k_bgemm3<true, false>), grid, block, 0, stream, d_descs);
        else if (!ta && tb) hipLaunchKernelGGL((k_bgemm3<false, true>), grid, block, 0, stream, d_descs);
        else hipLaunchKernelGGL((k_bgemm3<true, true>), grid, block, 0, stream, d_descs);
    }
}

const char* xgemm_name(int mode, bool ta, bool tb) {
    static const char* names[3][4] = {
        {"k_dgemm<false, false>", "k_dgemm<false, true>", "k_dgemm<true, false>", "k_dgemm<true, true>"},
        {"k_sgemm<false, false>", "k_sgemm<false, true>", "k_sgemm<true, false>", "k_sgemm<true, true>"},
        {"k_bgemm3<false, false>", "k_bgemm3<false, true>", "k_bgemm3<true, false>", "k_bgemm3<true, true>"}};
    const int m = (mode >= 0 && mode <= 2) ? mode : 0;
    return names[m][(ta ? 2 : 0) + (tb ? 1 : 0)];
}

}  // namespace lrr
