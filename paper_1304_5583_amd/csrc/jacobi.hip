// Batched two-sided block-Jacobi eigensolver for symmetric FP64 matrices.
//
// This is the "small dense SVD in FP64" of the singular-value thresholding
// step: the SVT of a block Y (n x l) needs the eigen-decomposition of its Gram
// matrix Y^T Y (l x l).  Several matrices (one per DFC block, of different
// orders) are processed by the same launches.
//
// A matrix of padded order L is cut into nb = L / BS blocks of BS indices.  One
// sweep has nb - 1 rounds; in a round the blocks are paired by the circle
// method and every pair (p, q) is handled in two launches:
//   phase A  one workgroup per pair applies one cyclic parallel-Jacobi sweep
//            to the 2BS x 2BS sub-matrix B[p u q, p u q] in LDS and writes the
//            accumulated rotation R_pq (2BS x 2BS);
//   phase B  every tile pair (P, Q), P <= Q, of the round is replaced by
//            R_P^T B[P, Q] R_Q (and its transpose), and the eigenvector
//            accumulator gets W[:, P] <- W[:, P] R_P; the 2BS-square products
//            run on the FP64 matrix cores out of LDS.
// Rounds come from the circle method (a full sweep) or, when the check found
// couplings in only a few index-block pairs, from a host-built schedule of
// perfect matchings that covers just those pairs (EigDesc::sched).
// Pairs of indices whose Gershgorin discs both lie below tau^2 are never
// rotated: the thresholding step discards every eigenvalue of that cluster, so
// only the subspace it spans matters, not a basis of it.
// Convergence: an off-diagonal entry needs a rotation when
// |b_pq| > max(1e-15 sqrt(|b_pp b_qq|), 1e-14 max|diag B|).  The absolute floor
// sits at the rounding level of the matrix: a Gram matrix of a rank-deficient
// block has exactly-zero eigenvalues whose coupling entries are pure rounding
// noise, and rotating them only regenerates noise.  Before each sweep one
// launch checks every off-diagonal entry; pairs whose sub-matrix is already
// diagonal skip their work, and so do the tiles they touch.
#include "common.hpp"
#include "kernels.hpp"

namespace lrr {

namespace {

constexpr double kRelTol = 1e-15;
constexpr double kAbsFloor = 1e-14;
constexpr int kPairThreads = 512;  // the pair kernel's rounds are bound by the 2x2 and R updates:
                                   // 512 threads measured 6% faster than 256, 1024 no faster
constexpr int kInnerSweeps = 1;   // one cyclic sweep per pair and round (block-Jacobi
                                  // converges with 1-2 more outer sweeps, each far cheaper)

// symmetric 2x2 Schur rotation: [c s; -s c]^T [app apq; apq aqq] [c s; -s c] is diagonal
// (t = s / c is returned too; c comes from one reciprocal square root)
__device__ __forceinline__ void sym_schur2(double app, double aqq, double apq, double& c, double& s, double& t) {
    const double theta = (aqq - app) / (2.0 * apq);
    t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
    c = rsqrt(1.0 + t * t);
    s = t * c;
}

// blocks (p, q) of slot P in a round: the circle method, or the explicit schedule
__device__ __forceinline__ void round_pair(const EigDesc& d, int nb, int round, int P, int sched, int& p, int& q) {
    if (sched) {
        const int v = d.sched[round * (nb / 2) + P];
        p = v & 0xffff;
        q = v >> 16;
    } else {
        rr_pair(nb, round, P, p, q);
    }
}

template <int BS, int NT>
__global__ __launch_bounds__(NT) void k_jacobi_pairs(const EigDesc* __restrict__ descs, int round, int sched) {
    constexpr int PB = 2 * BS;
    constexpr int NP = PB / 2;   // rotations per inner round
    const EigDesc d = descs[blockIdx.y];
    if (d.run[0] == 0 || d.st[0] != 0) return;
    const int nb = d.L / BS;
    const int P = blockIdx.x;
    if (P >= nb / 2 || round >= nb - 1) return;
    int p, q;
    round_pair(d, nb, round, P, sched, p, q);

    __shared__ double S[PB][PB + 1];
    __shared__ double R[PB][PB + 1];
    __shared__ double csc[NP], css[NP], cst[NP], csd[NP], cse[NP];
    __shared__ int any;
    __shared__ int LO[PB];

    const int tid = threadIdx.x;
    const long L = d.L;
    for (int idx = tid; idx < PB * PB; idx += NT) {
        const int i = idx % PB, j = idx / PB;
        const long gi = (i < BS) ? (long)p * BS + i : (long)q * BS + (i - BS);
        const long gj = (j < BS) ? (long)p * BS + j : (long)q * BS + (j - BS);
        S[i][j] = d.B[gi + gj * L];
        R[i][j] = (i == j) ? 1.0 : 0.0;
        if (j == 0) LO[i] = d.lo[gi];
    }
    const double floor_abs = kAbsFloor * d.scale[0];
    int rotated = 0;
    __syncthreads();

    for (int sweep = 0; sweep < kInnerSweeps; ++sweep) {
        // parallel convergence test of the whole sub-matrix
        if (tid == 0) any = 0;
        __syncthreads();
        for (int idx = tid; idx < PB * PB; idx += NT) {
            const int i = idx % PB, j = idx / PB;
            if (i < j && !(LO[i] && LO[j]) &&
                fabs(S[i][j]) > fmax(kRelTol * sqrt(fabs(S[i][i] * S[j][j])), floor_abs))
                any = 1;
        }
        __syncthreads();
        if (!any) break;
        rotated = 1;
        for (int r = 0; r < PB - 1; ++r) {
            if (tid < NP) {
                int a, b;
                rr_pair(PB, r, tid, a, b);
                const double app = S[a][a], aqq = S[b][b], apq = S[a][b];
                double c = 1.0, s = 0.0, t = 0.0;
                if (!(LO[a] && LO[b]) && fabs(apq) > fmax(kRelTol * sqrt(fabs(app * aqq)), floor_abs)) {
                    sym_schur2(app, aqq, apq, c, s, t);
                }
                csc[tid] = c;
                css[tid] = s;
                cst[tid] = t;
                csd[tid] = app - t * apq;   // rotated diagonal, closed form
                cse[tid] = aqq + t * apq;
            }
            __syncthreads();
            // the sub-matrix: (P2, Q2) blocks of the round's 2 x 2 index pairs
            auto s_item = [&](int idx) {
                const int P2 = idx / NP, Q2 = idx % NP;
                int aP, bP, aQ, bQ;
                rr_pair(PB, r, P2, aP, bP);
                if (P2 == Q2) {
                    // the rotated pair itself: exact zero off the diagonal
                    if (cst[P2] != 0.0) {
                        S[aP][aP] = csd[P2];
                        S[bP][bP] = cse[P2];
                        S[aP][bP] = 0.0;
                        S[bP][aP] = 0.0;
                    }
                    return;
                }
                rr_pair(PB, r, Q2, aQ, bQ);
                const double cP = csc[P2], sP = css[P2], cQ = csc[Q2], sQ = css[Q2];
                const double s_aa = S[aP][aQ], s_ab = S[aP][bQ];
                const double s_ba = S[bP][aQ], s_bb = S[bP][bQ];
                // columns: T = S G_Q
                const double t_aa = cQ * s_aa - sQ * s_ab, t_ab = sQ * s_aa + cQ * s_ab;
                const double t_ba = cQ * s_ba - sQ * s_bb, t_bb = sQ * s_ba + cQ * s_bb;
                // rows: S' = G_P^T T
                S[aP][aQ] = cP * t_aa - sP * t_ba;
                S[aP][bQ] = cP * t_ab - sP * t_bb;
                S[bP][aQ] = sP * t_aa + cP * t_ba;
                S[bP][bQ] = sP * t_ab + cP * t_bb;
            };
            // the accumulated rotation: row i, columns of pair Q2
            auto r_item = [&](int idx) {
                const int i = idx / NP, Q2 = idx % NP;
                int aQ, bQ;
                rr_pair(PB, r, Q2, aQ, bQ);
                const double cQ = csc[Q2], sQ = css[Q2];
                const double ra = R[i][aQ], rb = R[i][bQ];
                R[i][aQ] = cQ * ra - sQ * rb;
                R[i][bQ] = sQ * ra + cQ * rb;
            };
            if constexpr (NT >= 2 * NP * NP) {
                // the two updates touch disjoint arrays: the first NP^2 threads (whole
                // waves) update S while the others rotate R, instead of every wave
                // doing both in turn
                if (tid < NP * NP) s_item(tid);
                else
                    for (int idx = tid - NP * NP; idx < PB * NP; idx += NT - NP * NP) r_item(idx);
            } else {
                for (int idx = tid; idx < NP * NP; idx += NT) s_item(idx);
                for (int idx = tid; idx < PB * NP; idx += NT) r_item(idx);
            }
            __syncthreads();
        }
    }
    if (!rotated) {
        if (tid == 0) d.prot[P] = 0;
        return;
    }
    if (tid == 0 && d.work) {
        // per round: NP angles (~30 operations), (NP^2 - NP) 2x2 updates (24), PB*NP rotations of R (6)
        const unsigned long long per_round = 30ull * NP + 24ull * (NP * NP - NP) + 6ull * PB * NP;
        atomicAdd(&d.work[work_slot(0, blockIdx.x + blockIdx.y * gridDim.x)], per_round * (PB - 1));
    }
    double* Rg = d.R + (long)P * PB * PB;
    for (int idx = tid; idx < PB * PB; idx += NT) {
        const int i = idx % PB, j = idx / PB;
        Rg[i + (long)j * PB] = R[i][j];
    }
    if (tid == 0) d.prot[P] = rotated;
}

// C (PB x PB, into LDS) = op(A) B for PB x PB operands in LDS (row stride PB + 1),
// on the FP64 matrix cores: the (PB/16)^2 output tiles of 16 x 16 are spread over
// the four waves, each a chain of PB/4 v_mfma_f64_16x16x4f64 (register v of a
// lane holds row lane/16 + 4v, column lane%16 of its tile).  TA: op(A) = A^T.
template <int PB, bool TA>
__device__ __forceinline__ void mm_lds(const double (*A)[PB + 1], const double (*B)[PB + 1], double (*C)[PB + 1],
                                       int tid) {
    constexpr int NTILE = PB / 16;
    const int wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    for (int t = wave; t < NTILE * NTILE; t += 4) {
        const int ti = (t % NTILE) * 16, tj = (t / NTILE) * 16;
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < PB; kk += 4) {
            const int k = kk + lk;
            const double a = TA ? A[k][ti + lr] : A[ti + lr][k];
            const double b = B[k][tj + lr];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) C[ti + lk + 4 * v][tj + lr] = acc[v];
    }
}

// phase B: tiles of B and row chunks of W
template <int BS>
__global__ __launch_bounds__(256) void k_jacobi_apply(const EigDesc* __restrict__ descs, int round, int sched) {
    constexpr int PB = 2 * BS;
    constexpr int RC = 64;   // rows of W per workgroup
    const EigDesc d = descs[blockIdx.y];
    if (d.run[0] == 0 || d.st[0] != 0) return;
    const int nb = d.L / BS;
    const int npair = nb / 2;
    const int ntri = npair * (npair + 1) / 2;
    const int nchunks = (d.L + RC - 1) / RC;
    const int item = blockIdx.x;
    if (item >= ntri + nchunks * npair || round >= nb - 1) return;

    __shared__ double X[PB][PB + 1];
    __shared__ double RP[PB][PB + 1];
    __shared__ double RQ[PB][PB + 1];
    __shared__ double T[PB][PB + 1];
    const int tid = threadIdx.x;
    const long L = d.L;

    if (item < ntri) {
        // decode upper-triangular index (P <= Q)
        int P = 0, rem = item;
        while (rem >= npair - P) { rem -= npair - P; ++P; }
        const int Q = P + rem;
        if (!d.prot[P] && !d.prot[Q]) return;
        if (tid == 0 && d.work)   // two PB^3 products
            atomicAdd(&d.work[work_slot(1, blockIdx.x + blockIdx.y * gridDim.x)], 4ull * PB * PB * PB);
        int p1, q1, p2, q2;
        round_pair(d, nb, round, P, sched, p1, q1);
        round_pair(d, nb, round, Q, sched, p2, q2);
        const double* RgP = d.R + (long)P * PB * PB;
        const double* RgQ = d.R + (long)Q * PB * PB;
        for (int idx = tid; idx < PB * PB; idx += 256) {
            const int i = idx % PB, j = idx / PB;
            const long gi = (i < BS) ? (long)p1 * BS + i : (long)q1 * BS + (i - BS);
            const long gj = (j < BS) ? (long)p2 * BS + j : (long)q2 * BS + (j - BS);
            X[i][j] = d.B[gi + gj * L];
            // a pair that did not rotate has R = I (its R block was not written)
            RP[i][j] = d.prot[P] ? RgP[i + (long)j * PB] : (i == j ? 1.0 : 0.0);
            RQ[i][j] = d.prot[Q] ? RgQ[i + (long)j * PB] : (i == j ? 1.0 : 0.0);
        }
        __syncthreads();
        mm_lds<PB, false>(X, RQ, T, tid);       // T = X R_Q
        __syncthreads();
        mm_lds<PB, true>(RP, T, X, tid);        // X = R_P^T T (X is free after the first product)
        __syncthreads();
        for (int idx = tid; idx < PB * PB; idx += 256) {
            const int i = idx % PB, j = idx / PB;
            const long gi = (i < BS) ? (long)p1 * BS + i : (long)q1 * BS + (i - BS);
            const long gj = (j < BS) ? (long)p2 * BS + j : (long)q2 * BS + (j - BS);
            d.B[gi + gj * L] = X[i][j];
        }
        if (P != Q) {
            // the mirrored tile, with consecutive threads on consecutive rows of it
            for (int idx = tid; idx < PB * PB; idx += 256) {
                const int j = idx % PB, i = idx / PB;
                const long gi = (i < BS) ? (long)p1 * BS + i : (long)q1 * BS + (i - BS);
                const long gj = (j < BS) ? (long)p2 * BS + j : (long)q2 * BS + (j - BS);
                d.B[gj + gi * L] = X[i][j];
            }
        }
    } else {
        const int w = item - ntri;
        const int P = w % npair, chunk = w / npair;
        if (!d.prot[P]) return;
        if (tid == 0 && d.work)   // RC x PB times PB x PB
            atomicAdd(&d.work[work_slot(1, blockIdx.x + blockIdx.y * gridDim.x)], 2ull * RC * PB * PB);
        int p1, q1;
        round_pair(d, nb, round, P, sched, p1, q1);
        const double* RgP = d.R + (long)P * PB * PB;
        const int r0 = chunk * RC;
        // reuse X as a RC x PB panel when RC <= PB, else loop in pieces of PB rows
        for (int rr = 0; rr < RC; rr += PB) {
            for (int idx = tid; idx < PB * PB; idx += 256) {
                const int i = idx % PB, j = idx / PB;
                const long gi = r0 + rr + i;
                const long gj = (j < BS) ? (long)p1 * BS + j : (long)q1 * BS + (j - BS);
                X[i][j] = (gi < L) ? d.W[gi + gj * L] : 0.0;
                if (rr == 0) RP[i][j] = RgP[i + (long)j * PB];
            }
            __syncthreads();
            mm_lds<PB, false>(X, RP, T, tid);   // T = W panel R_P
            __syncthreads();
            for (int idx = tid; idx < PB * PB; idx += 256) {
                const int i = idx % PB, j = idx / PB;
                const long gi = r0 + rr + i;
                const long gj = (j < BS) ? (long)p1 * BS + j : (long)q1 * BS + (j - BS);
                if (gi < L) d.W[gi + gj * L] = T[i][j];
            }
            __syncthreads();
        }
    }
}

// start of an eigensolve: reset flags, scale = max |diag|
__global__ __launch_bounds__(256) void k_jacobi_init(const EigDesc* __restrict__ descs) {
    const EigDesc d = descs[blockIdx.x];
    if (d.run[0] == 0) return;
    double mx = 0.0;
    for (int i = threadIdx.x; i < d.l; i += 256) mx = fmax(mx, fabs(d.B[i + (long)i * d.L]));
    mx = wave_max(mx);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        d.scale[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        d.st[0] = 0;
        d.st[1] = 0;
    }
}

// one launch per sweep: does any off-diagonal entry still need a rotation?  With
// bs > 0 and need set, the index-block pairs holding such entries are marked.
__global__ __launch_bounds__(256) void k_jacobi_offcheck(const EigDesc* __restrict__ descs, int* n_open, int bs) {
    const EigDesc d = descs[blockIdx.y];
    if (d.run[0] == 0 || d.st[0] != 0) return;
    const long L = d.L;
    const long total = (long)d.l * d.l;
    const double floor_abs = kAbsFloor * d.scale[0];
    int* const mark = (bs > 0) ? d.need : nullptr;
    const int nb = (bs > 0) ? d.L / bs : 0;
    int need = 0;
    for (long idx = (long)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (long)gridDim.x * 256) {
        const int i = (int)(idx % d.l), j = (int)(idx / d.l);
        if (i < j && !(d.lo[i] && d.lo[j])) {
            const double a = d.B[i + j * L];
            if (fabs(a) > fmax(kRelTol * sqrt(fabs(d.B[i + i * L] * d.B[j + j * L])), floor_abs)) {
                need = 1;
                if (mark) mark[(i / bs) * nb + j / bs] = 1;   // every writer stores 1
            }
        }
    }
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    if (need) any = 1;
    __syncthreads();
    if (threadIdx.x == 0 && any) atomicOr(&d.st[1], 1);
}

// after the check: a matrix with nothing left to rotate is converged
__global__ void k_jacobi_close(const EigDesc* __restrict__ descs, int count, int* n_open) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    const EigDesc d = descs[b];
    if (d.run[0] == 0 || d.st[0] != 0) return;
    if (d.st[1] == 0) d.st[0] = 1;
    else atomicAdd(n_open, 1);
    d.st[1] = 0;
}

// end of a sweep: a sweep without rotations means converged
__global__ void k_jacobi_sweep_end(const EigDesc* __restrict__ descs, int count, int* any_active) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    const EigDesc d = descs[b];
    if (d.run[0] == 0 || d.st[0] != 0) return;
    if (d.st[1] == 0) d.st[0] = 1;
    else atomicAdd(any_active, 1);
    d.st[1] = 0;
}

// eigenvalues = diagonal (padding -> 0)
__global__ void k_jacobi_eigvals(const EigDesc* __restrict__ descs) {
    const EigDesc d = descs[blockIdx.x];
    if (d.run[0] == 0) return;
    for (int i = threadIdx.x; i < d.L; i += blockDim.x)
        d.lam[i] = (i < d.l) ? d.B[i + (long)i * d.L] : 0.0;
}

}  // namespace

void launch_jacobi_init(const EigDesc* d_descs, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_init, dim3(count), dim3(256), 0, s, d_descs);
}

void launch_jacobi_pairs(const EigDesc* d_descs, int count, int maxL, int bs, int round, hipStream_t s,
                         bool sched) {
    const int npair = maxL / bs / 2;
    if (bs == 16)
        hipLaunchKernelGGL((k_jacobi_pairs<16, kPairThreads>), dim3(npair, count), dim3(kPairThreads), 0, s, d_descs,
                           round, (int)sched);
    else
        hipLaunchKernelGGL((k_jacobi_pairs<32, kPairThreads>), dim3(npair, count), dim3(kPairThreads), 0, s, d_descs,
                           round, (int)sched);
}

void launch_jacobi_apply(const EigDesc* d_descs, int count, int maxL, int bs, int round, hipStream_t s,
                         bool sched) {
    const int npair = maxL / bs / 2;
    const int ntri = npair * (npair + 1) / 2;
    const int nchunks = (maxL + 63) / 64;
    if (bs == 16)
        hipLaunchKernelGGL((k_jacobi_apply<16>), dim3(ntri + nchunks * npair, count), dim3(256), 0, s,
                           d_descs, round, (int)sched);
    else
        hipLaunchKernelGGL((k_jacobi_apply<32>), dim3(ntri + nchunks * npair, count), dim3(256), 0, s,
                           d_descs, round, (int)sched);
}

void launch_jacobi_round(const EigDesc* d_descs, int count, int maxL, int bs, int round, hipStream_t s) {
    launch_jacobi_pairs(d_descs, count, maxL, bs, round, s);
    launch_jacobi_apply(d_descs, count, maxL, bs, round, s);
}

void launch_jacobi_check(const EigDesc* d_descs, int count, int maxL, int* d_open, hipStream_t s, int bs) {
    const int blocks = (maxL * maxL + 255) / 256 < 64 ? (maxL * maxL + 255) / 256 : 64;
    hipLaunchKernelGGL(k_jacobi_offcheck, dim3(blocks, count), dim3(256), 0, s, d_descs, d_open, bs);
    hipLaunchKernelGGL(k_jacobi_close, dim3((count + 63) / 64), dim3(64), 0, s, d_descs, count, d_open);
}

void launch_jacobi_sweep_end(const EigDesc* d_descs, int count, int* d_any, hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_sweep_end, dim3((count + 63) / 64), dim3(64), 0, s, d_descs, count, d_any);
}

void launch_jacobi_eigvals(const EigDesc* d_descs, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_eigvals, dim3(count), dim3(256), 0, s, d_descs);
}

}  // namespace lrr
