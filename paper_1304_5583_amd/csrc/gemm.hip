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
// load latency.  Both heights sum every element over K in the same order (K in
// steps of 16, four MFMA k-chunks of 4 each), so the choice does not change the
// result, and neither does anything else below: only the data movement is tuned.
//
// Data movement, per K-tile of 16:
//   * global -> registers with raw buffer loads, two K-tiles ahead of the one
//     being multiplied (two register sets, the loop unrolled by two), so a load
//     has two tiles' worth of MFMA time to arrive.  An element outside the
//     matrix (M, N or K edge) gets an offset with bit 31 set, beyond the
//     buffer's range, and the hardware returns 0 for it: the loads are
//     straight-line code for every tile, edges included, and the compiler
//     waits only for the older set (vmcnt(n) instead of vmcnt(0)).  With
//     64-row tiles the offsets and the M/N edge bits are formed once per
//     output tile and only a K-tile that reaches past K tests the K edge
//     (2-3 % faster than testing every element of every K-tile: the products
//     run at the chip's power limit, where fewer vector instructions per MFMA
//     buy clock);
//   * every load instruction of a wavefront covers whole contiguous runs: the
//     threads walk the operand's contiguous dimension first (rows of A, k of
//     A^T, k of B, columns of B^T);
//   * registers -> double-buffered LDS tiles, row stride BM + 1 doubles: the
//     16 lanes that store one column of a k-contiguous operand land in 16
//     different bank pairs (an odd stride), and the 16 lanes of an MFMA read
//     take 16 consecutive doubles of one row, so neither side conflicts (the
//     bank-conflict counter reads 0; a stride of BM + 2 made those stores
//     2-way conflicted, one of 16 mod 32 8-way and 40 % slower);
//   * the kernel is held to 128 VGPRs (four waves per SIMD, the LDS of four
//     workgroups per CU): at three waves per SIMD the batched 512-order
//     products ran 17 % slower.
// Measured on 40 products of order 512 (m = 512, n = 500, K = 512), random operands: 47-48 TFLOP/s,
// against 41 for element/vector loads one tile ahead in branches.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace lrr {

namespace {

constexpr int BN = 64, PAD = 1;

constexpr int BK = 16;                         // K depth of a tile
constexpr int kList = 256;                     // products listed on chip (one per thread)
constexpr unsigned kRsrcWord3 = 0x00020000u;   // raw buffer resource, gfx9-family data format
constexpr unsigned kRange = 0x7ffffff0u;       // num_records: offsets with bit 31 set are outside

// raw buffer resource over one K-tile's panel of an operand (offsets from `base`)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t panel_rsrc(const double* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, (int)kRange, (int)kRsrcWord3);
}
__device__ __forceinline__ double buffer_ld(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// SYM (with TA, !TB, BM = BN, C square): C = A^T B for a product that is
// symmetric in exact arithmetic (A^T A, or X^T (B X) with B symmetric); only the
// tiles with P <= Q run, and an off-diagonal tile also writes its transpose, so
// the result is exactly symmetric.  For A^T A it is bitwise the full product:
// tile (P, Q) and tile (Q, P) multiply the same pairs of numbers in the same
// order (the MFMA products of a chunk commute).
// Byte offsets inside one K-tile's panel are below 2^31 while lda * BM and
// ldb * 64 stay below 2^28 doubles (leading dimensions below four million).
template <int BM, bool TA, bool TB, bool SYM = false>
__global__ __launch_bounds__(256, 4) void k_dgemm(const GemmDesc* __restrict__ descs, int tiles_m, int tiles_n,
                                                  int total) {
    constexpr int WM = BM / 2, TX = WM / 16;
    constexpr int NA = BM * BK / 256, NB = BN * BK / 256;   // operand elements per thread and K-tile
    static_assert(!SYM || (TA && !TB && BM == BN), "symmetric tiles need C = A^T B with square tiles");
    const int per = SYM ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
    // double-buffered operand tiles: As[buf][k][i] = op(A)(m0+i, k0+k)
    __shared__ double As[2][BK][BM + PAD];
    __shared__ double Bs[2][BK][BN + PAD];
    // Only the products whose block is active take part: with at most kList
    // products every workgroup first lists the active ones, in order (one flag
    // read per product), and the tiles below run over that list; with more, a
    // tile of an inactive product is skipped after one descriptor read.
    __shared__ int s_z[kList];
    __shared__ int s_n[4];
    const int count = total / per;
    const bool listed = count <= kList;
    int work = total;
    if (listed) {
        const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
        int act = 0;
        if (tid < count) {
            const int* __restrict__ a = descs[tid].active;
            act = (a == nullptr || a[0] != 0) ? 1 : 0;
        }
        const unsigned long long bal = __ballot(act);
        if (lane == 0) s_n[w] = __popcll(bal);
        __syncthreads();
        int off = __popcll(bal & ((1ull << lane) - 1ull));
        for (int i = 0; i < w; ++i) off += s_n[i];
        if (act) s_z[off] = tid;
        work = (s_n[0] + s_n[1] + s_n[2] + s_n[3]) * per;
        __syncthreads();
    }
    // The grid is at most four workgroups per CU; each takes the tiles
    // blockIdx.x, blockIdx.x + gridDim.x, ...  Workgroup w runs on XCD w % 8, so
    // the first 8 * floor(work / 8) tiles are dealt out in eight contiguous
    // ranges, one per XCD: the tiles of one product share an L2 (3 % faster than
    // dealing consecutive tiles to consecutive XCDs), and when few blocks are
    // active their tiles still spread over all eight XCDs.  Within a product,
    // row tiles run fastest.
    const int per_x = work >> 3;
    for (int t0 = blockIdx.x; t0 < work; t0 += gridDim.x) {
        const int tile = t0 < 8 * per_x ? (t0 & 7) * per_x + (t0 >> 3) : t0;
        const int zi = tile / per, tin = tile - zi * per;
        const int z = listed ? s_z[zi] : zi;
        const GemmDesc d = descs[z];
        if (!listed && d.active && d.active[0] == 0) continue;
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
        const int nt = (K + BK - 1) / BK;
        // element v of this thread in a K-tile = its first element plus v steps:
        //   op(A) = A  : row ai = tid % BM, k = tid / BM + (256 / BM) v
        //   op(A) = A^T: k = tid % 16, row ai = tid / 16 + 16 v
        //   op(B) = B  : k = tid % 16, column bj = tid / 16 + 16 v
        //   op(B) = B^T: column bj = tid % 64, k = tid / 64 + 4 v
        const int ai = TA ? tid / 16 : tid % BM, ak = TA ? tid % 16 : tid / BM;
        const int bj = TB ? tid % 64 : tid / 16, bk = TB ? tid / 64 : tid % 16;
        constexpr int dai = TA ? 16 : 0, dak = TA ? 0 : 256 / BM;
        constexpr int dbj = TB ? 0 : 16, dbk = TB ? 4 : 0;
        const unsigned aoff = (unsigned)(8 * (TA ? ak + (long)ai * lda : ai + (long)ak * lda));
        const unsigned boff = (unsigned)(8 * (TB ? bj + (long)bk * ldb : bk + (long)bj * ldb));
        const unsigned astep = (unsigned)(8 * (TA ? (long)dai * lda : (long)dak * lda));
        const unsigned bstep = (unsigned)(8 * (TB ? (long)dbk * ldb : (long)dbj * ldb));

        // offsets inside a K-tile's panel, the same for every K-tile; an element
        // outside the M (N) edge carries bit 31 for the whole K loop
        unsigned oa[NA], ob[NB];
#pragma unroll
        for (int v = 0; v < NA; ++v) oa[v] = (aoff + v * astep) | ((unsigned)(m0 + ai + dai * v >= M) << 31);
#pragma unroll
        for (int v = 0; v < NB; ++v) ob[v] = (boff + v * bstep) | ((unsigned)(n0 + bj + dbj * v >= N) << 31);

        double fa0[NA], fb0[NB], fa1[NA], fb1[NB];
        // K-tile kt of both operands into registers (zeros outside the matrices);
        // only a tile that reaches past K tests the K edge per element
        auto gload = [&](double (&fa)[NA], double (&fb)[NB], int kt) {
            const int k0 = kt * BK;
            const __amdgpu_buffer_rsrc_t ra = panel_rsrc(TA ? A + k0 + (long)m0 * lda : A + m0 + (long)k0 * lda);
            const __amdgpu_buffer_rsrc_t rb = panel_rsrc(TB ? B + n0 + (long)k0 * ldb : B + k0 + (long)n0 * ldb);
            if (BM == 32) {
                // short batches: per-element edge tests measured faster here
#pragma unroll
                for (int v = 0; v < NA; ++v) {
                    const unsigned in = (unsigned)(m0 + ai + dai * v < M) & (unsigned)(k0 + ak + dak * v < K);
                    fa[v] = buffer_ld(ra, (aoff + v * astep) | ((in ^ 1u) << 31));
                }
#pragma unroll
                for (int v = 0; v < NB; ++v) {
                    const unsigned in = (unsigned)(n0 + bj + dbj * v < N) & (unsigned)(k0 + bk + dbk * v < K);
                    fb[v] = buffer_ld(rb, (boff + v * bstep) | ((in ^ 1u) << 31));
                }
            } else if (k0 + BK <= K) {
#pragma unroll
                for (int v = 0; v < NA; ++v) fa[v] = buffer_ld(ra, oa[v]);
#pragma unroll
                for (int v = 0; v < NB; ++v) fb[v] = buffer_ld(rb, ob[v]);
            } else {
                const int kr = K - k0;
#pragma unroll
                for (int v = 0; v < NA; ++v) fa[v] = buffer_ld(ra, oa[v] | ((unsigned)(ak + dak * v >= kr) << 31));
#pragma unroll
                for (int v = 0; v < NB; ++v) fb[v] = buffer_ld(rb, ob[v] | ((unsigned)(bk + dbk * v >= kr) << 31));
            }
        };
        auto lstore = [&](const double (&fa)[NA], const double (&fb)[NB], int buf) {
#pragma unroll
            for (int v = 0; v < NA; ++v) As[buf][ak + dak * v][ai + dai * v] = fa[v];
#pragma unroll
            for (int v = 0; v < NB; ++v) Bs[buf][bk + dbk * v][bj + dbj * v] = fb[v];
        };
        // the four k-chunks of the tile in LDS buffer `buf`, in order
        auto mma = [&](int buf) {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                const int kr = kk + lk;
                double a[TX];
#pragma unroll
                for (int x = 0; x < TX; ++x) a[x] = As[buf][kr][wm + 16 * x + lr];
                const double b0 = Bs[buf][kr][wn + lr], b1 = Bs[buf][kr][wn + 16 + lr];
#pragma unroll
                for (int x = 0; x < TX; ++x) {
                    acc[x][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b0, acc[x][0], 0, 0, 0);
                    acc[x][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b1, acc[x][1], 0, 0, 0);
                }
            }
        };
        // tile 0 in LDS buffer 0, tile 1 in flight in set 0; each half of the loop
        // multiplies one tile while the tile after next loads into the other set
        gload(fa0, fb0, 0);
        lstore(fa0, fb0, 0);
        gload(fa0, fb0, 1);
        __syncthreads();
        for (int pr = 0; pr < nt / 2; ++pr) {
            const int kt = 2 * pr;
            gload(fa1, fb1, kt + 2);
            mma(0);
            lstore(fa0, fb0, 1);
            __syncthreads();
            gload(fa0, fb0, kt + 3);
            mma(1);
            lstore(fa1, fb1, 0);
            __syncthreads();
        }
        if (nt & 1) mma(0);

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
