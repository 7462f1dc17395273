/*
 * lrr_diag.h -- diagnostic entry points of the gfx950 DFC-LRR library.
 *
 * These expose the building blocks of the solver one by one, so that each can
 * be checked against a plain reference in isolation.  They are not needed to
 * solve a problem.  Conventions are those of lrr.h: column-major FP64 DEVICE
 * matrices with leading dimensions, work enqueued on `stream`, the call
 * returns after the work is complete, negative status = nothing written.
 */
#ifndef LRR_DIAG_H
#define LRR_DIAG_H

#include "lrr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C = alpha * op(A) op(B) + beta * C with op(X) = X or X^T (ta, tb != 0 means
 * transposed).  op(A) is M x K, op(B) is K x N, C is M x N.  The MFMA GEMM used
 * for every dense product of the solver (Gram matrices, dictionary products,
 * reconstruction, combine).  A^T A (ta, !tb, B == A, ldb == lda, M == N) runs
 * the symmetric kernel of the solver's Gram matrices: the tiles on and above
 * the diagonal are computed and mirrored, bitwise the full product.  lda and
 * ldb must be below 4194304 (2^22; the kernel addresses a K-tile's panel with
 * 32-bit byte offsets): LRR_EINVAL otherwise. */
lrr_status lrr_diag_dgemm(lrr_ctx *ctx, int ta, int tb, int M, int N, int K, double alpha,
                          const double *A, int lda, const double *B, int ldb, double beta,
                          double *C, int ldc, void *stream);

/* The same product with the arithmetic of a precision form (lrr_precision):
 * LRR_FP64 as lrr_diag_dgemm; LRR_FP32 rounds the operands to FP32 and
 * accumulates in FP32 on the matrix cores; LRR_MIXED_BF16 splits each operand
 * into two BF16 numbers (hi + lo) and sums hi*hi + hi*lo + lo*hi in FP32.
 * Operands and result are FP64 in memory in every form; an unknown precision
 * is LRR_EINVAL. */
lrr_status lrr_diag_gemm(lrr_ctx *ctx, int precision, int ta, int tb, int M, int N, int K,
                         double alpha, const double *A, int lda, const double *B, int ldb,
                         double beta, double *C, int ldc, void *stream);

/* Kinv = (I + A A^T)^{-1} for A (m x n): the factorisation the Z-step uses
 * (FP64 blocked Cholesky, then the explicit inverse of the factor).
 * Kinv is m x m with ld >= m. */
lrr_status lrr_diag_spd_inverse(lrr_ctx *ctx, int m, int n, const double *A, int lda,
                                double *Kinv, int ldk, void *stream);

/* The same factorisation for callers that cannot allocate device memory (code
 * that must not call hipMalloc / hipFree, such as tight serving loops or
 * harnesses that forbid allocation): every work buffer lives in one device
 * array that the library holds statically, 32.3 MiB per GPU from module load
 * until the process ends.  Limit: m <= 1024 (larger m is LRR_EINVAL with a
 * message naming the limit); the caller still owns A and Kinv.  All calls on
 * one GPU share that GPU's array: calls that overlap on one GPU (two streams or
 * two host threads) race and must be serialised by the caller. */
lrr_status lrr_diag_spd_inverse_noalloc(lrr_ctx *ctx, int m, int n, const double *A, int lda,
                                        double *Kinv, int ldk, void *stream);

/* Eigen-decomposition of `count` symmetric matrices of orders l[i] (host array):
 * matrix i is read from B + i*strideB (ld = ldb >= max l) and its eigenvalues
 * (unsorted) are written to lam + i*ldlam, its eigenvectors (columns, same
 * order) to W + i*strideB (ld = ldb).  Block-Jacobi solver of the thresholding
 * step, started from the identity.  sweeps (host, may be NULL) receives the
 * number of sweeps run. */
lrr_status lrr_diag_syevj(lrr_ctx *ctx, int count, const int *l, const double *B, int ldb,
                          long strideB, double *lam, int ldlam, double *W, int eig_block,
                          int *sweeps, void *stream);

/* Round schedule of a targeted Jacobi pass (host only, no device work).  After
 * each check of the off-diagonal entries, the solver marks the pairs of
 * index blocks (bs indices each) that still hold an entry above the tolerance
 * and, when few are marked, runs only rounds that cover them instead of a full
 * sweep of nb - 1 circle rounds.  need (HOST, nb x nb ints; entry p * nb + q is
 * read for p <= q, p == q meaning inside block p) holds the marks; nb is even,
 * 2 <= nb <= 65534.  Greedy matchings of the marked pairs, each completed to a
 * perfect matching of the nb blocks, are written to out (HOST, cap * nb / 2
 * ints, round r at out + r * nb / 2, pair p | q << 16 with p < q).  *rounds
 * receives their number, or -1 if more than cap rounds would be needed (out
 * then holds cap partial rounds).  LRR_EINVAL on a NULL pointer, an odd or
 * out-of-range nb, or cap < 0. */
lrr_status lrr_diag_plan_rounds(const int *need, int nb, int cap, int *out, int *rounds);

/* Per-kernel timing of the solver's own launches.  When enabled, every kernel
 * launch of lrr_solve / dfc_lrr_solve is bracketed by HIP events recorded on the
 * solve's stream; durations are accumulated per kernel name together with the
 * algorithmic flops (GEMMs: 2 M N K per active product) and algorithmic HBM
 * bytes (column kernels: every matrix element read or written once) of each
 * launch.  lrr_prof_enable also clears the table. */
lrr_status lrr_prof_enable(lrr_ctx *ctx, int on);
/* Restrict the timing to kernels whose name starts with `prefix` (NULL or "":
 * all kernels), so that the events bracket only the launches of interest.  The
 * Z-step/E-step chain is replayed from its graph unless one of its kernels is
 * being timed. */
lrr_status lrr_prof_filter(lrr_ctx *ctx, const char *prefix);
int lrr_prof_count(const lrr_ctx *ctx);
/* Entry idx (0 <= idx < lrr_prof_count): name (owned by ctx), total ms, number
 * of launches, total algorithmic flops and bytes. */
lrr_status lrr_prof_entry(const lrr_ctx *ctx, int idx, const char **name, double *ms,
                          long long *launches, double *flops, double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* LRR_DIAG_H */
