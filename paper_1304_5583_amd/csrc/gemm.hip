// Batched FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64).
//
// Every dense contraction of the solver goes through here: the Gram matrices
// A A^T and Y^T Y, the dictionary products M Q and M^T V, the solve with the
// inverse factor, the reconstruction of the thresholded block and the combine.
//
// Tiling: a 256-thread workgroup owns a BM x 64 tile of C; each of its four
// 64-wide wavefronts owns a (BM/2) x 32 part as MFMA tiles of 16 x 16.  BM is 64
// unless the batch has fewer than 512 such tiles; then BM = 32 doubles the
// number of workgroups, so that every CU holds two and one hides the other's
// load latency (the four Gram matrices of order 500 of a 4-block problem ran at
// 21-30 TFLOP/s with one 64-row workgroup per CU, the 40-block problem's at
// 47-55).  Both heights sum every element over K in the same order, so the
// choice does not change the result.  K advances in steps of 16 (four MFMA
// k-chunks of 4).  Operand tiles are double-buffered in LDS and the next tile is
// fetched into registers while the current one is multiplied.  With 16-deep
// tiles a 64-row workgroup holds 34 KB of LDS, so four fit on a CU (32-deep
// tiles allowed two and ran the batched 512-order products at 38-40 instead of
// 44-47 TFLOP/s).  Whole K-tiles of interior workgroups are read with 16-byte
// vector loads (7-10 % faster than element loads); loads at the matrix edges
// are bounds-tested and zero-fill, so any M, N, K is legal.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace lrr {

namespace {

constexpr int BN = 64, PAD = 2;

// K depth of a tile: 16 for both heights (LDS for four 64-row workgroups per
// CU; 32-deep tiles with 32-row tiles, whose grids hold two workgroups per CU,
// measured no faster: 507 vs 502 ms per workload-2 solve)
template <int BM>
constexpr int kDepth = 16;

// One K-tile of op(A) (BM x BK) and op(B) (BK x BN) in registers.
template <int BM>
struct Frag {
    static constexpr int BK = kDepth<BM>;
    static constexpr int NLA = (BM * BK) / 256;   // elements of the op(A) tile per thread
    static constexpr int NLB = (BN * BK) / 256;   // elements of the op(B) tile per thread
    double a[NLA];
    double b[NLB];
};

// Thread -> element map of the operand tiles.  Every thread holds a run of NLA
// (op(A)) or NLB (op(B)) elements that are contiguous in memory:
//   op(A) = A   : run along the BM rows of one k   (row (tid % (BM/NLA)) * NLA, k = tid / (BM/NLA))
//   op(A) = A^T : run along k of one row           (row tid / (BK/NLA), k = (tid % (BK/NLA)) * NLA)
//   op(B) = B   : run along k of one column        (column tid / (BK/NLB), k = (tid % (BK/NLB)) * NLB)
//   op(B) = B^T : run along the BN columns of one k (column (tid % (BN/NLB)) * NLB, k = tid / (BN/NLB))
template <int BM, bool TA>
__device__ __forceinline__ void a_slot(int tid, int& i, int& kk) {
    constexpr int NLA = Frag<BM>::NLA, BK = Frag<BM>::BK;
    if (!TA) { i = (tid % (BM / NLA)) * NLA; kk = tid / (BM / NLA); }
    else     { i = tid / (BK / NLA); kk = (tid % (BK / NLA)) * NLA; }
}
template <int BM, bool TB>
__device__ __forceinline__ void b_slot(int tid, int& j, int& kk) {
    constexpr int NLB = Frag<BM>::NLB, BK = Frag<BM>::BK;
    if (!TB) { j = tid / (BK / NLB); kk = (tid % (BK / NLB)) * NLB; }
    else     { j = (tid % (BN / NLB)) * NLB; kk = tid / (BN / NLB); }
}

// bounds-tested loads (zero outside the matrices)
template <int BM, bool TA, bool TB>
__device__ __forceinline__ void load_tile(Frag<BM>& f, const double* __restrict__ A, long lda,
                                          const double* __restrict__ B, long ldb, int M, int N, int K,
                                          int m0, int n0, int k0, int tid) {
    constexpr int NLA = Frag<BM>::NLA, NLB = Frag<BM>::NLB;
    int i, ka, j, kb;
    a_slot<BM, TA>(tid, i, ka);
    b_slot<BM, TB>(tid, j, kb);
#pragma unroll
    for (int v = 0; v < NLA; ++v) {
        const int gi = m0 + i + (TA ? 0 : v), gk = k0 + ka + (TA ? v : 0);
        f.a[v] = (gi < M && gk < K) ? (TA ? A[gk + gi * lda] : A[gi + gk * lda]) : 0.0;
    }
#pragma unroll
    for (int v = 0; v < NLB; ++v) {
        const int gj = n0 + j + (TB ? v : 0), gk = k0 + kb + (TB ? 0 : v);
        f.b[v] = (gj < N && gk < K) ? (TB ? B[gj + gk * ldb] : B[gk + gj * ldb]) : 0.0;
    }
}

// interior tile with 16-byte aligned runs: unchecked 16-byte vector loads
template <int BM, bool TA, bool TB>
__device__ __forceinline__ void load_tile_vec(Frag<BM>& f, const double* __restrict__ A, long lda,
                                              const double* __restrict__ B, long ldb, int m0, int n0, int k0,
                                              int tid) {
    constexpr int NLA = Frag<BM>::NLA, NLB = Frag<BM>::NLB;
    int i, ka, j, kb;
    a_slot<BM, TA>(tid, i, ka);
    b_slot<BM, TB>(tid, j, kb);
    const double* pa = TA ? A + (k0 + ka) + (long)(m0 + i) * lda : A + (m0 + i) + (long)(k0 + ka) * lda;
    const double* pb = TB ? B + (n0 + j) + (long)(k0 + kb) * ldb : B + (k0 + kb) + (long)(n0 + j) * ldb;
#pragma unroll
    for (int v = 0; v < NLA; v += 2) {
        const double2 x = *reinterpret_cast<const double2*>(pa + v);
        f.a[v] = x.x;
        f.a[v + 1] = x.y;
    }
#pragma unroll
    for (int v = 0; v < NLB; v += 2) {
        const double2 x = *reinterpret_cast<const double2*>(pb + v);
        f.b[v] = x.x;
        f.b[v + 1] = x.y;
    }
}

template <int BM, bool TA, bool TB>
__device__ __forceinline__ void store_tile(const Frag<BM>& f, double (*As)[BM + PAD], double (*Bs)[BN + PAD],
                                           int tid) {
    constexpr int NLA = Frag<BM>::NLA, NLB = Frag<BM>::NLB;
    int i, ka, j, kb;
    a_slot<BM, TA>(tid, i, ka);
    b_slot<BM, TB>(tid, j, kb);
#pragma unroll
    for (int v = 0; v < NLA; ++v) {
        if (!TA) As[ka][i + v] = f.a[v];
        else As[ka + v][i] = f.a[v];
    }
#pragma unroll
    for (int v = 0; v < NLB; ++v) {
        if (!TB) Bs[kb + v][j] = f.b[v];
        else Bs[kb][j + v] = f.b[v];
    }
}

// BM = 64: each wave owns a 32 x 32 quarter (2 x 2 MFMA tiles); BM = 32 (grids too
// small to give every CU two workgroups): each wave owns 16 x 32 (1 x 2 tiles).
// SYM (with TA, !TB, BM = BN, C square): C = A^T A.  Tile (P, Q) and tile (Q, P)
// multiply the same pairs of numbers in the same order (the MFMA products of a
// chunk commute), so the computed product is exactly symmetric; only the tiles
// with P <= Q run, and an off-diagonal tile also writes its transpose.
template <int BM, bool TA, bool TB, bool SYM = false>
__global__ __launch_bounds__(256) void k_dgemm(const GemmDesc* __restrict__ descs, int tiles_m, int tiles_n,
                                               int total) {
    constexpr int WM = BM / 2, TX = WM / 16, BK = Frag<BM>::BK;
    static_assert(!SYM || (TA && !TB && BM == BN), "symmetric tiles need C = A^T A with square tiles");
    const int per = SYM ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
    // double-buffered operand tiles: As[buf][k][i] = op(A)(m0+i, k0+k)
    __shared__ double As[2][BK][BM + PAD];
    __shared__ double Bs[2][BK][BN + PAD];
    // The grid is at most a few workgroups per CU; each takes the tiles
    // blockIdx.x, blockIdx.x + gridDim.x, ...  in launch order: row tiles
    // fastest, then column tiles, then products (placing each product's tiles
    // on one XCD's L2 measured 3-5% slower).  A tile of a product whose block
    // is not active is skipped after one descriptor read, so a launch with no
    // active block costs little more than its dispatch.
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int z = tile / per, tin = tile - z * per;
        const GemmDesc d = descs[z];
        if (d.active && d.active[0] == 0) continue;
        int tm_i, tn_i;
        if (SYM) {
            // upper-triangle index tin -> (P, Q), P <= Q, column by column
            int q = (int)((sqrt(8.0 * tin + 1.0) - 1.0) * 0.5);
            while (q * (q + 1) / 2 > tin) --q;
            while ((q + 1) * (q + 2) / 2 <= tin) ++q;
            tn_i = q;
            tm_i = tin - q * (q + 1) / 2;
        } else {
            tm_i = tin % tiles_m;
            tn_i = tin / tiles_m;
        }
        const int m0 = tm_i * BM, n0 = tn_i * BN;
        if (m0 >= d.M || n0 >= d.N) continue;

        const int tid = threadIdx.x;
        const int lane = tid & 63;
        const int wave = tid >> 6;
        const int wm = (wave >> 1) * WM, wn = (wave & 1) * 32;
        const int lr = lane & 15, lk = lane >> 4;

        dbl4 acc[TX][2];
    #pragma unroll
        for (int x = 0; x < TX; ++x)
            for (int y = 0; y < 2; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};

        const double* __restrict__ A = d.A;
        const double* __restrict__ B = d.B;
        const int M = d.M, N = d.N, K = d.K;
        const long lda = d.lda, ldb = d.ldb;

        // whole K-tiles of an interior workgroup with 16-byte aligned operands are
        // read with unchecked vector loads; the rest (edges, a partial last K-tile,
        // odd strides or offsets) with bounds-tested element loads
        const bool vec = m0 + BM <= M && n0 + BN <= N && (lda & 1) == 0 && (ldb & 1) == 0 &&
                         (reinterpret_cast<unsigned long>(A) & 15) == 0 &&
                         (reinterpret_cast<unsigned long>(B) & 15) == 0;
        const int kvec = vec ? (K / BK) * BK : 0;

        Frag<BM> f;
        if (BK <= kvec) load_tile_vec<BM, TA, TB>(f, A, lda, B, ldb, m0, n0, 0, tid);
        else load_tile<BM, TA, TB>(f, A, lda, B, ldb, M, N, K, m0, n0, 0, tid);
        store_tile<BM, TA, TB>(f, As[0], Bs[0], tid);
        __syncthreads();
        int cur = 0;
        for (int k0 = 0; k0 < K; k0 += BK) {
            const int kn = k0 + BK;
            // the next tile's global loads are in flight while this one is multiplied
            if (kn < K) {
                if (kn + BK <= kvec) load_tile_vec<BM, TA, TB>(f, A, lda, B, ldb, m0, n0, kn, tid);
                else load_tile<BM, TA, TB>(f, A, lda, B, ldb, M, N, K, m0, n0, kn, tid);
            }
    #pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                const int kr = kk + lk;
                double a[TX];
    #pragma unroll
                for (int x = 0; x < TX; ++x) a[x] = As[cur][kr][wm + 16 * x + lr];
                const double b0 = Bs[cur][kr][wn + lr], b1 = Bs[cur][kr][wn + 16 + lr];
    #pragma unroll
                for (int x = 0; x < TX; ++x) {
                    acc[x][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b0, acc[x][0], 0, 0, 0);
                    acc[x][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b1, acc[x][1], 0, 0, 0);
                }
            }
            if (kn < K) store_tile<BM, TA, TB>(f, As[cur ^ 1], Bs[cur ^ 1], tid);
            __syncthreads();
            cur ^= 1;
        }

        // accumulator layout of v_mfma_f64_16x16x4f64: register v of a lane holds
        // row lane/16 + 4v, column lane%16 of the 16 x 16 tile
        const double alpha = d.alpha, beta = d.beta;
        const long ldc = d.ldc;
    #pragma unroll
        for (int x = 0; x < TX; ++x) {
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
                        if (SYM && tm_i != tn_i) {
                            // the mirrored element (gj, gi); beta applies to it as well
                            double* __restrict__ Cm = d.C + (long)gi * ldc;
                            double rm = alpha * acc[x][y][v];
                            if (beta != 0.0) rm += beta * Cm[gj];
                            Cm[gj] = rm;
                        }
                    }
                }
            }
        }
        // the next tile's first LDS stores wait for every wave of this one
        __syncthreads();
    }
}

// workgroups of a GEMM launch: four per CU (the LDS of a 64-row tile allows four)
int gemm_grid_cap() {
    static int cap = 0;
    if (cap == 0) {
        int dev = 0, cus = 0;
        LRR_HIP(hipGetDevice(&dev));
        LRR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        cap = 4 * std::max(cus, 1);
    }
    return cap;
}

template <int BM>
void launch_bm(const GemmDesc* d_descs, int count, int maxM, int maxN, bool ta, bool tb, hipStream_t stream) {
    const int tm = (maxM + BM - 1) / BM, tn = (maxN + BN - 1) / BN;
    const long total = (long)tm * tn * count;
    if (total > 0x7fffffffL) throw HipError("GEMM grid too large");
    dim3 grid((unsigned)std::min<long>(total, gemm_grid_cap()));
    dim3 block(256);
    const int tt = (int)total;
    if (!ta && !tb) hipLaunchKernelGGL((k_dgemm<BM, false, false>), grid, block, 0, stream, d_descs, tm, tn, tt);
    else if (ta && !tb) hipLaunchKernelGGL((k_dgemm<BM, true, false>), grid, block, 0, stream, d_descs, tm, tn, tt);
    else if (!ta && tb) hipLaunchKernelGGL((k_dgemm<BM, false, true>), grid, block, 0, stream, d_descs, tm, tn, tt);
    else hipLaunchKernelGGL((k_dgemm<BM, true, true>), grid, block, 0, stream, d_descs, tm, tn, tt);
}

}  // namespace

bool dgemm_sym_tiles(int count, int maxN) {
    const long tm = (maxN + BN - 1) / BN;
    return tm * tm * count >= 512;
}

int gemm_grid(void) { return gemm_grid_cap(); }

void launch_dgemm_sym(const GemmDesc* d_descs, int count, int maxN, hipStream_t stream, bool always) {
    if (count <= 0 || maxN <= 0) return;
    const int tm = (maxN + BN - 1) / BN;
    // small batches keep every tile (32-row tiles give every CU two workgroups);
    // the result is the same either way
    if (!always && !dgemm_sym_tiles(count, maxN)) {
        launch_dgemm(d_descs, count, maxN, maxN, true, false, stream);
        return;
    }
    const long total = (long)tm * (tm + 1) / 2 * count;
    if (total > 0x7fffffffL) throw HipError("GEMM grid too large");
    hipLaunchKernelGGL((k_dgemm<BN, true, false, true>), dim3((unsigned)std::min<long>(total, gemm_grid_cap())),
                       dim3(256), 0, stream, d_descs, tm, tm, (int)total);
}

void launch_dgemm(const GemmDesc* d_descs, int count, int maxM, int maxN, bool ta, bool tb,
                  hipStream_t stream) {
    if (count <= 0 || maxM <= 0 || maxN <= 0) return;
    // 64-row tiles unless that leaves fewer than two workgroups per CU (256 CUs);
    // both tile heights sum every element in the same order, so the choice does
    // not change a bit of the result
    const long tiles64 = (long)((maxM + 63) / 64) * ((maxN + BN - 1) / BN) * count;
    if (tiles64 < 512) launch_bm<32>(d_descs, count, maxM, maxN, ta, tb, stream);
    else launch_bm<64>(d_descs, count, maxM, maxN, ta, tb, stream);
}

}  // namespace lrr
