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

// LDS of one pair solve
template <int BS>
struct PairLds {
    static constexpr int PB = 2 * BS, NP = BS;
    double S[PB][PB + 1];
    double R[PB][PB + 1];
    double csc[NP], css[NP], cst[NP], csd[NP], cse[NP];
    int any;
    int LO[PB];
};

// Phase A for slot P of a round, by the NT threads of a workgroup: one cyclic
// sweep of the 2BS x 2BS sub-matrix in LDS, the rotation written to R_P.
// wslot spreads the operation counter over its slots.  Every thread returns
// through the same path (the branches depend on LDS values only).
template <int BS, int NT>
__device__ void pair_solve(const EigDesc& d, int round, int P, int sched, int wslot, PairLds<BS>& sm) {
    constexpr int PB = 2 * BS;
    constexpr int NP = PB / 2;   // rotations per inner round
    const int nb = d.L / BS;
    int p, q;
    round_pair(d, nb, round, P, sched, p, q);

    auto& S = sm.S;
    auto& R = sm.R;
    auto& csc = sm.csc;
    auto& css = sm.css;
    auto& cst = sm.cst;
    auto& csd = sm.csd;
    auto& cse = sm.cse;
    auto& any = sm.any;
    auto& LO = sm.LO;

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
        atomicAdd(&d.work[work_slot(0, wslot)], per_round * (PB - 1));
    }
    double* Rg = d.R + (long)P * PB * PB;
    for (int idx = tid; idx < PB * PB; idx += NT) {
        const int i = idx % PB, j = idx / PB;
        Rg[i + (long)j * PB] = R[i][j];
    }
    if (tid == 0) d.prot[P] = rotated;
}

template <int BS, int NT>
__global__ __launch_bounds__(NT) void k_jacobi_pairs(const EigDesc* __restrict__ descs, int round, int sched) {
    const EigDesc d = descs[blockIdx.y];
    if (d.run[0] == 0 || d.st[0] != 0) return;
    const int nb = d.L / BS;
    const int P = blockIdx.x;
    if (P >= nb / 2 || round >= nb - 1) return;
    __shared__ PairLds<BS> sm;
    pair_solve<BS, NT>(d, round, P, sched, blockIdx.x + blockIdx.y * gridDim.x, sm);
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

// LDS of one phase-B item
template <int BS>
struct ApplyLds {
    static constexpr int PB = 2 * BS;
    double X[PB][PB + 1];
    double RP[PB][PB + 1];
    double RQ[PB][PB + 1];
    double T[PB][PB + 1];
};

constexpr int kApplyRows = 64;   // rows of W per phase-B item

template <int BS>
__device__ __forceinline__ int apply_items(int L) {
    const int npair = L / BS / 2;
    return npair * (npair + 1) / 2 + ((L + kApplyRows - 1) / kApplyRows) * npair;
}

// phase B, item `item` of a round (256 threads): a tile pair of B or a row
// chunk of W
template <int BS>
__device__ void apply_item(const EigDesc& d, int round, int item, int sched, int wslot, ApplyLds<BS>& sm) {
    constexpr int PB = 2 * BS;
    constexpr int RC = kApplyRows;
    const int nb = d.L / BS;
    const int npair = nb / 2;
    const int ntri = npair * (npair + 1) / 2;
    auto& X = sm.X;
    auto& RP = sm.RP;
    auto& RQ = sm.RQ;
    auto& T = sm.T;
    const int tid = threadIdx.x;
    const long L = d.L;

    if (item < ntri) {
        // decode upper-triangular index (P <= Q)
        int P = 0, rem = item;
        while (rem >= npair - P) { rem -= npair - P; ++P; }
        const int Q = P + rem;
        if (!d.prot[P] && !d.prot[Q]) return;
        if (tid == 0 && d.work)   // two PB^3 products
            atomicAdd(&d.work[work_slot(1, wslot)], 4ull * PB * PB * PB);
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
            atomicAdd(&d.work[work_slot(1, wslot)], 2ull * RC * PB * PB);
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

template <int BS>
__global__ __launch_bounds__(256) void k_jacobi_apply(const EigDesc* __restrict__ descs, int round, int sched) {
    const EigDesc d = descs[blockIdx.y];
    if (d.run[0] == 0 || d.st[0] != 0) return;
    const int nb = d.L / BS;
    const int item = blockIdx.x;
    if (item >= apply_items<BS>(d.L) || round >= nb - 1) return;
    __shared__ ApplyLds<BS> sm;
    apply_item<BS>(d, round, item, sched, blockIdx.x + blockIdx.y * gridDim.x, sm);
}

// start of an eigensolve: reset flags, scale = max |diag|
__global__ __launch_bounds__(256) void k_jacobi_init(const EigDesc* __restrict__ descs) {
    const EigDesc d = descs[blockIdx.x];
    if (d.run[0] == 0) return;
    const bool done = d.done && d.done[0];
    if (done) {
        for (int i = threadIdx.x; i < d.l; i += 256) d.B[i + (long)i * d.L] = d.lam[i];
        __syncthreads();
    }
    double mx = 0.0;
    for (int i = threadIdx.x; i < d.l; i += 256) mx = fmax(mx, fabs(d.B[i + (long)i * d.L]));
    mx = wave_max(mx);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        d.scale[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        d.st[0] = done ? 1 : 0;
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

// ---------------------------------------------------------------------------
// Persistent eigensolve: the whole pass loop of the batched block-Jacobi method
// in one launch.  Each pass: Gershgorin flags of every open matrix, the check of
// every off-diagonal entry (marking the index-block pairs that still need a
// rotation), closing converged matrices, and either a targeted pass (rounds of
// perfect matchings covering the marked pairs, planned per matrix on the
// device) or a full circle sweep; then the rounds, each a pair phase and an
// apply phase.  Phases are separated by grid-wide barriers; every workgroup
// takes the same decisions from the same global values, so the control flow
// is uniform across the grid.  The results are those of the launch-per-phase
// kernels above (same device functions, same order of operations).
//
// The grid must fit on the chip at once (the host sizes it from the occupancy
// of this kernel).  Each barrier wait is bounded: a wait that runs out sets
// JacCtl::err and every workgroup leaves at its next barrier, so the kernel
// always ends; the host reports the flag as an error.
// ---------------------------------------------------------------------------
constexpr int kSolveThreads = 256;
constexpr long kSpinLimit = 1L << 23;   // s_sleep(1) waits of one barrier (~0.4 s)
constexpr int kChecksPerMatrix = 64;    // check items per matrix (as the check launch's grid)
constexpr int kPlanMaxNb = 64;          // index blocks the device planner handles (bit masks)

// all workgroups of the grid reach this point; false once any wait ran out
__device__ bool grid_sync(JacCtl* ctl, unsigned nwg, unsigned& gen) {
    __syncthreads();
    __shared__ int bad;
    if (threadIdx.x == 0) {
        const unsigned g = gen;
        const unsigned a = __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (a == nwg - 1) {
            __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->bar_gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long spins = 0;
            while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kSpinLimit) {
                    __hip_atomic_store(&ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                // another workgroup's wait ran out: leave at once
                if ((spins & 1023) == 0 && __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    break;
            }
        }
        gen = g + 1;
        bad = __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return bad == 0;
}

// block b of item `item` given the prefix counts off[0..t]
__device__ __forceinline__ int item_block(const int* __restrict__ off, int t, int item) {
    int b = 0;
    while (b + 1 < t && off[b + 1] <= item) ++b;
    return b;
}

struct PlanLds {
    unsigned short pp[kPlanMaxNb * (kPlanMaxNb - 1) / 2];
    unsigned short qq[kPlanMaxNb * (kPlanMaxNb - 1) / 2];
    unsigned char cov[kPlanMaxNb * (kPlanMaxNb - 1) / 2];
    int cnt[kSolveThreads + 1];
    unsigned long long inner;
};

// Targeted rounds of one matrix (the device form of the host planner
// plan_rounds): the marked pairs p < q in p-major order are covered greedily,
// round by round, each round completed to a perfect matching of the nb index
// blocks (a block marked inside goes with a free partner, preferring another
// such block; the rest pair up in order).  Returns the number of rounds, or -1
// when more than cap would be needed (or nb exceeds the bit masks).
__device__ int plan_device(const int* __restrict__ need, int nb, int cap, int* __restrict__ sched, PlanLds& pl) {
    const int tid = threadIdx.x;
    if (nb > kPlanMaxNb) return -1;
    const int total = nb * nb;
    const int per = (total + kSolveThreads - 1) / kSolveThreads;
    const int i0 = tid * per, i1 = min(total, i0 + per);
    if (tid == 0) pl.inner = 0ull;
    __syncthreads();
    int c = 0;
    unsigned long long inner = 0ull;
    for (int idx = i0; idx < i1; ++idx) {
        const int p = idx / nb, q = idx % nb;
        if (q < p || !need[idx]) continue;
        if (p == q) inner |= 1ull << p;
        else ++c;
    }
    pl.cnt[tid + 1] = c;
    if (inner) atomicOr(&pl.inner, inner);
    __syncthreads();
    if (tid == 0) {
        pl.cnt[0] = 0;
        for (int k = 1; k <= kSolveThreads; ++k) pl.cnt[k] += pl.cnt[k - 1];
    }
    __syncthreads();
    int w = pl.cnt[tid];
    for (int idx = i0; idx < i1; ++idx) {
        const int p = idx / nb, q = idx % nb;
        if (q <= p || !need[idx]) continue;
        pl.pp[w] = (unsigned short)p;
        pl.qq[w] = (unsigned short)q;
        pl.cov[w] = 0;
        ++w;
    }
    __syncthreads();
    const int npend = pl.cnt[kSolveThreads];
    int rounds = 0;
    if (tid == 0) {
        unsigned long long in = pl.inner;
        const unsigned long long all = (nb == 64) ? ~0ull : ((1ull << nb) - 1ull);
        int left = npend;
        if (npend > cap * (nb / 2)) {
            rounds = -1;   // each round covers at most nb / 2 pairs
        } else {
            for (;;) {
                if (left == 0 && in == 0ull) break;
                if (rounds == cap) { rounds = -1; break; }
                int* slot = sched + (long)rounds * (nb / 2);
                int ns = 0;
                unsigned long long used = 0ull;
                for (int e = 0; e < npend; ++e) {
                    if (pl.cov[e]) continue;
                    const int p = pl.pp[e], q = pl.qq[e];
                    const unsigned long long bits = (1ull << p) | (1ull << q);
                    if (used & bits) continue;
                    slot[ns++] = p | (q << 16);
                    used |= bits;
                    in &= ~bits;   // a pair solve also sweeps inside both blocks
                    pl.cov[e] = 1;
                    --left;
                }
                for (int p = 0; p < nb; ++p) {
                    if (!((in >> p) & 1ull) || ((used >> p) & 1ull)) continue;
                    const unsigned long long fr = all & ~used & ~(1ull << p);
                    const unsigned long long fri = fr & in;
                    const int q = fri ? __ffsll((long long)fri) - 1 : __ffsll((long long)fr) - 1;
                    if (q < 0) break;   // cannot happen (nb is even, so a free partner exists)
                    const int a = min(p, q), b = max(p, q);
                    slot[ns++] = a | (b << 16);
                    const unsigned long long bits = (1ull << p) | (1ull << q);
                    used |= bits;
                    in &= ~bits;
                }
                int u = -1;
                for (int x = 0; x < nb; ++x) {
                    if ((used >> x) & 1ull) continue;
                    if (u < 0) u = x;
                    else { slot[ns++] = u | (x << 16); u = -1; }
                }
                ++rounds;
            }
        }
        pl.cnt[0] = rounds;
    }
    __syncthreads();
    rounds = pl.cnt[0];
    __syncthreads();
    return rounds;
}

template <int BS>
__global__ __launch_bounds__(kSolveThreads) void k_jacobi_solve(const EigDesc* __restrict__ descs, int t,
                                                                 const int* __restrict__ offs, int* brounds,
                                                                 JacCtl* ctl, const DevIter* it, int max_sweeps,
                                                                 int max_targeted, int nb_max, int* need_all,
                                                                 long need_total) {
    __shared__ union {
        PairLds<BS> p;
        ApplyLds<BS> a;
        PlanLds pl;
    } sm;
    __shared__ double red[4];
    const unsigned G = gridDim.x;
    const int wg = blockIdx.x, tid = threadIdx.x;
    const int* off_rows = offs;
    const int* off_pairs = offs + (t + 1);
    const int* off_apply = offs + 2 * (t + 1);
    unsigned gen = 0;

    // start of the eigensolve: scale = max |diag|, flags cleared
    for (int b = wg; b < t; b += G) {
        const EigDesc d = descs[b];
        if (d.run[0] == 0) continue;
        const bool done = d.done && d.done[0];
        if (done) {
            for (int i = tid; i < d.l; i += kSolveThreads) d.B[i + (long)i * d.L] = d.lam[i];
            __syncthreads();
        }
        double mx = 0.0;
        for (int i = tid; i < d.l; i += kSolveThreads) mx = fmax(mx, fabs(d.B[i + (long)i * d.L]));
        mx = wave_max(mx);
        if ((tid & 63) == 0) red[tid >> 6] = mx;
        __syncthreads();
        if (tid == 0) {
            d.scale[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
            d.st[0] = done ? 1 : 0;
            d.st[1] = 0;
        }
        __syncthreads();
    }
    if (!grid_sync(ctl, G, gen)) return;

    const double tau = it->tau;
    const int full_all = it->full;
    int full = 0, targeted = 0, pass = 0;
    bool counted = true;
    for (;;) {
        // Gershgorin flags of the open matrices; the marks are cleared
        for (long k = (long)wg * kSolveThreads + tid; k < need_total; k += (long)G * kSolveThreads) need_all[k] = 0;
        for (int item = wg; item < off_rows[t]; item += G) {
            const int b = item_block(off_rows, t, item);
            const EigDesc d = descs[b];
            if (d.run[0] == 0 || d.st[0] != 0) continue;
            const int i = item - off_rows[b];
            const long L = d.L;
            double rs = 0.0;   // column i of the symmetric matrix, contiguous
            for (int j = tid; j < d.l; j += kSolveThreads)
                if (j != i) rs += fabs(d.B[j + i * L]);
            rs = wave_sum(rs);
            if ((tid & 63) == 0) red[tid >> 6] = rs;
            __syncthreads();
            if (tid == 0) {
                const double r = (red[0] + red[1]) + (red[2] + red[3]);
                d.lo[i] = (i >= d.l) ? 1 : (full_all ? 0 : lo_flag(d.B[i + i * L] + r, tau, d.cut[0], d.scale[0]));
                if (i == 0 && counted) d.passes[0] += 1;
            }
            __syncthreads();
        }
        if (!grid_sync(ctl, G, gen)) return;
        // check: does any off-diagonal entry still need a rotation; mark its blocks
        for (int item = wg; item < t * kChecksPerMatrix; item += G) {
            const int b = item / kChecksPerMatrix, part = item % kChecksPerMatrix;
            const EigDesc d = descs[b];
            if (d.run[0] == 0 || d.st[0] != 0) continue;
            const long L = d.L;
            const long total = (long)d.l * d.l;
            const double floor_abs = kAbsFloor * d.scale[0];
            const int nb = d.L / BS;
            int need = 0;
            for (long idx = (long)part * kSolveThreads + tid; idx < total; idx += (long)kChecksPerMatrix * kSolveThreads) {
                const int i = (int)(idx % d.l), j = (int)(idx / d.l);
                if (i < j && !(d.lo[i] && d.lo[j])) {
                    const double a = d.B[i + j * L];
                    if (fabs(a) > fmax(kRelTol * sqrt(fabs(d.B[i + i * L] * d.B[j + j * L])), floor_abs)) {
                        need = 1;
                        d.need[(i / BS) * nb + j / BS] = 1;   // every writer stores 1
                    }
                }
            }
            if (__syncthreads_or(need) && tid == 0) atomicOr(&d.st[1], 1);
        }
        if (!grid_sync(ctl, G, gen)) return;
        // close converged matrices, count the open ones, plan targeted rounds
        for (int b = wg; b < t; b += G) {
            const EigDesc d = descs[b];
            const int nbb = d.L / BS;
            int open = 0;
            if (d.run[0] != 0 && d.st[0] == 0) {
                open = d.st[1] != 0;
                __syncthreads();
                if (tid == 0) {
                    if (!open) d.st[0] = 1;
                    else atomicAdd(&ctl->n_open[pass & 1], 1);
                    d.st[1] = 0;
                }
            }
            int rb = 0;
            if (open && targeted < max_targeted)
                rb = plan_device(d.need, nbb, min((nb_max - 1) / 2, nbb - 1), const_cast<int*>(d.sched), sm.pl);
            if (tid == 0) brounds[b] = rb;
            __syncthreads();
        }
        if (!grid_sync(ctl, G, gen)) return;
        // the same decision in every workgroup
        const int nopen = __hip_atomic_load(&ctl->n_open[pass & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (wg == 0 && tid == 0) ctl->n_open[(pass + 1) & 1] = 0;
        if (nopen == 0 || full == max_sweeps) break;
        int rounds = targeted < max_targeted ? 0 : -1;
        for (int b = 0; b < t && rounds >= 0; ++b) {
            const int rb = brounds[b];
            rounds = rb < 0 ? -1 : max(rounds, rb);
        }
        int sched;
        if (rounds > 0) {
            // matrices that need fewer rounds get circle rounds (any perfect matching is valid)
            for (int b = wg; b < t; b += G) {
                const EigDesc d = descs[b];
                const int nbb = d.L / BS, np = nbb / 2;
                const int r0 = brounds[b], r1 = min(rounds, nbb - 1);
                int* sc = const_cast<int*>(d.sched);
                for (int k = tid; k < (r1 - r0) * np; k += kSolveThreads) {
                    const int r = r0 + k / np, P = k % np;
                    int a0, b0;
                    rr_pair(nbb, r, P, a0, b0);
                    sc[r * np + P] = a0 | (b0 << 16);
                }
            }
            if (!grid_sync(ctl, G, gen)) return;
            ++targeted;
            counted = false;
            sched = 1;
        } else {
            rounds = nb_max - 1;
            ++full;
            counted = true;
            sched = 0;
        }
        for (int r = 0; r < rounds; ++r) {
            for (int item = wg; item < off_pairs[t]; item += G) {
                const int b = item_block(off_pairs, t, item);
                const EigDesc d = descs[b];
                if (d.run[0] == 0 || d.st[0] != 0 || r >= d.L / BS - 1) continue;
                pair_solve<BS, kSolveThreads>(d, r, item - off_pairs[b], sched, wg, sm.p);
                __syncthreads();
            }
            if (!grid_sync(ctl, G, gen)) return;
            for (int item = wg; item < off_apply[t]; item += G) {
                const int b = item_block(off_apply, t, item);
                const EigDesc d = descs[b];
                if (d.run[0] == 0 || d.st[0] != 0 || r >= d.L / BS - 1) continue;
                apply_item<BS>(d, r, item - off_apply[b], sched, wg, sm.a);
                __syncthreads();
            }
            if (!grid_sync(ctl, G, gen)) return;
        }
        ++pass;
    }
}

// before each launch; the error flag stays set once raised (the host clears it
// at the start of a solve and reads it with the convergence flags)
__global__ void k_jacobi_ctl_reset(JacCtl* ctl) {
    ctl->bar_count = 0u;
    ctl->bar_gen = 0u;
    ctl->n_open[0] = 0;
    ctl->n_open[1] = 0;
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

int jacobi_solve_grid(int bs) {
    static int grid[2] = {0, 0};
    int& g = grid[bs == 32 ? 1 : 0];
    if (g == 0) {
        int dev = 0, cus = 0, per = 0;
        LRR_HIP(hipGetDevice(&dev));
        LRR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        if (bs == 32)
            LRR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_jacobi_solve<32>, kSolveThreads, 0));
        else
            LRR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_jacobi_solve<16>, kSolveThreads, 0));
        if (per < 1) throw HipError("the persistent eigensolve does not fit on a CU");
        // one workgroup per CU: a grid barrier costs each workgroup an L2
        // write-back and invalidation at agent scope (measured 15-24 us with 256
        // workgroups, 67-93 us with 1024)
        g = std::max(cus, 1);
    }
    return g;
}

void launch_jacobi_solve(const EigDesc* d_descs, int count, const int* d_offs, int* d_brounds, JacCtl* ctl,
                         const DevIter* it, int max_sweeps, int max_targeted, int nb_max, int bs, int* need_all,
                         long need_total, hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_ctl_reset, dim3(1), dim3(1), 0, s, ctl);
    const dim3 grid(jacobi_solve_grid(bs));
    if (bs == 32)
        hipLaunchKernelGGL((k_jacobi_solve<32>), grid, dim3(kSolveThreads), 0, s, d_descs, count, d_offs, d_brounds,
                           ctl, it, max_sweeps, max_targeted, nb_max, need_all, need_total);
    else
        hipLaunchKernelGGL((k_jacobi_solve<16>), grid, dim3(kSolveThreads), 0, s, d_descs, count, d_offs, d_brounds,
                           ctl, it, max_sweeps, max_targeted, nb_max, need_all, need_total);
}

void launch_jacobi_eigvals(const EigDesc* d_descs, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_eigvals, dim3(count), dim3(256), 0, s, d_descs);
}

}  // namespace lrr
