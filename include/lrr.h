/*
 * lrr.h -- C ABI of the MI355X (gfx950) DFC-LRR library.
 *
 * The library solves the low-rank representation program
 *
 *     min ||Z||_* + lambda ||E||_{2,1}   s.t.  X = A Z + E          (Eq. 1 / Eq. 2)
 *
 * where ||.||_{2,1} is the sum of the column l2 norms (Section 1), with the
 * inexact augmented-Lagrange-multiplier iteration that the paper uses as its base
 * LRR solver (Section 4 preamble), and the divide-factor-combine wrapper of
 * Algorithm 1 (Section 2.2): the columns of M are split into t blocks C_i, each
 * block solves Eq. (2) with the whole M as dictionary, and the block estimates
 * are combined by projecting onto the column space of the first one.
 *
 * Memory conventions (all entry points)
 * -------------------------------------
 *  - Matrices are column-major with an explicit leading dimension (rows <= ld
 *    < 4194304 = 2^22: the FP64 matrix-core GEMM addresses a K-tile of an
 *    operand with 32-bit byte offsets; a larger ld is LRR_EINVAL).
 *    A column is one data point, so a row-major (n, m) tensor holds M^T.
 *  - Matrix arguments are DEVICE pointers on the ctx's device, element type
 *    double by default in every precision form (the form selects the
 *    arithmetic of the large products, not the storage).  With opts.io_type =
 *    LRR_IO_FP32 the forward entry points (lrr_solve, dfc_lrr_solve,
 *    dfc_lrr_solve_local) take and return float buffers instead: the inputs
 *    are widened to FP64 copies in the ctx, the iteration state stays FP64, and
 *    the outputs are rounded to FP32 once at the end (extra ctx memory: one FP64
 *    copy of every matrix argument).
 *    Index arrays (perm, offsets) and the info arrays are HOST pointers.
 *  - The caller owns every argument buffer.  The library owns its workspace,
 *    which lives in the ctx and is reused (and grown) across calls.
 *  - All device work is enqueued on `stream`; every entry point returns after the
 *    result is complete on that stream (it reads back convergence flags).
 *  - A ctx is not thread safe: use one ctx per host thread.
 *
 * Errors
 * ------
 *  Arguments are validated before any device work.  A negative status means no
 *  output was written; LRR_NOT_CONVERGED (> 0) means outputs are valid but some
 *  block hit max_iter.  lrr_last_error() returns a message for the last failure.
 */
#ifndef LRR_H
#define LRR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lrr_ctx lrr_ctx;

typedef enum {
    LRR_OK = 0,
    LRR_NOT_CONVERGED = 1,   /* outputs valid, max_iter reached in some block      */
    LRR_EINVAL = -1,         /* bad argument (dims, ld, lambda, partition, nulls)  */
    LRR_ENOMEM = -2,         /* device workspace could not be allocated           */
    LRR_EDEVICE = -3,        /* a HIP runtime call failed                          */
    LRR_ENUMERIC = -4,       /* non-finite value in the input                      */
    LRR_ENOTAPE = -5         /* backward called without a recorded forward         */
} lrr_status;

/* Precision forms.  FP64 state in every form.  The reduced forms run the two
 * dictionary products of the Z-step (M Q and M^T V) and the last two products
 * of the combine on the FP32 or BF16 matrix cores with FP32 accumulation; the
 * Gram matrix, the reconstruction J = Y P, the Cholesky factorisation and its
 * application, the eigen-decomposition and every residual norm stay FP64.  M Q
 * is carried as a running sum of products of the changes of Q, re-formed in
 * FP64 every 16 iterations, so that its rounding error shrinks as the
 * iteration converges and the FP64 stopping tolerance stays reachable. */
typedef enum {
    LRR_FP64 = 0,            /* every product in FP64                              */
    LRR_FP32 = 1,            /* operands rounded to FP32, FP32 MFMA                */
    LRR_MIXED_BF16 = 2       /* operands split x = hi + lo in BF16, three BF16     */
                             /* MFMA products (hi hi + hi lo + lo hi), FP32 accum. */
} lrr_precision;

/* Element type of the matrix arguments of the forward entry points. */
typedef enum {
    LRR_IO_FP64 = 0,         /* double buffers (default)                            */
    LRR_IO_FP32 = 1          /* float buffers; FP64 state inside (see above)        */
} lrr_io_type;

/* The Z-step solves (I + A^T A) Z = A^T (X - E + Y1/mu) + J - Y2/mu (Eq. 2's
 * augmented Lagrangian).  Literal: the n x n matrix is factored (FP64 Cholesky)
 * and inverted once per solve, and each iteration applies it with three FP64
 * products (n x m, n x n and m x n per block).  Push-through: the same iterate
 * through (I + A^T A)^{-1} = I - A^T (I + A A^T)^{-1} A, factoring the m x m
 * matrix.  The literal form needs FP64 precision, full coordinates and no
 * recorded forward (LRR_EINVAL otherwise); the footnote variant ignores the
 * field.  AUTO takes the literal form when n <= m, the precision is FP64, the
 * coordinates are full and no forward is recorded, and push-through otherwise. */
typedef enum {
    LRR_SOLVE_AUTO = 0,
    LRR_SOLVE_LITERAL = 1,   /* Cholesky of I + A^T A (n x n)                        */
    LRR_SOLVE_PUSHTHROUGH = 2/* Cholesky of I + A A^T (m x m), same iterates        */
} lrr_solve_form;

/* Coordinates of the n-row iterates Z, J, Y2.  Started at zero, they stay in
 * range(A^T) (every update is a product with A^T or a column operation), so with
 * an orthonormal basis Qm of that range (n x r, r = numerical rank of A <= m)
 * Z = Qm Zr exactly and the iteration can run on r-row coefficients: the Gram
 * matrix of the thresholding step and the dictionary products shrink from n to
 * r rows, and the n x n states are never formed.  The results agree with the
 * full coordinates to rounding; the coupling residual max|Z - J| is bounded by
 * the coefficient columns' 2-norms (times 1 and 1/sqrt(n)) and formed in full
 * only when the bounds do not decide the stop test.  Basis directions with
 * sigma^2 <= 1e-14 sigma_max^2 are dropped. */
typedef enum {
    LRR_COORDS_AUTO = 0,     /* reduced when n >= 2m (the basis costs an m x m      */
                             /* eigensolve), never for a recorded forward or an     */
                             /* explicitly literal solve form                       */
    LRR_COORDS_FULL = 1,
    LRR_COORDS_REDUCED = 2
} lrr_coords;

/* Inexact-ALM controls.  The paper does not print the solver's constants; these
 * are explicit so that any caller (and the CPU reference) can use the same ones. */
typedef struct {
    int precision;           /* lrr_precision                                       */
    int solve_form;          /* lrr_solve_form                                      */
    double mu0;              /* initial penalty (default 1e-6)                      */
    double rho;              /* penalty growth factor (default 1.1)                 */
    double mu_max;           /* penalty cap (default 1e10)                          */
    double tol;              /* stop when both residual max-norms < tol (1e-8)      */
    int max_iter;            /* iteration cap (default 1000)                        */
    int fixed_iters;         /* > 0: run exactly this many iterations, no stop test */
    int check_every;         /* read device convergence flags every c iterations   */
    int max_sweeps;          /* Jacobi sweep cap of the eigensolver (default 30)    */
    int save_for_backward;   /* record what dfc_lrr_backward needs                  */
    int checkpoint_every;    /* adjoint checkpoint spacing k (default 20)           */
    int eig_block;           /* Jacobi block width: 0 auto, 16 or 32                */
    int use_graph;           /* how an iteration is issued:                         */
                             /*  0: the J-step's decisions (blocks to threshold,    */
                             /*     refinement steps, Jacobi passes and rounds) on  */
                             /*     the host, every launch one by one;              */
                             /*  1 (default): as 0, the Z-/E-step launches replayed */
                             /*     from a captured HIP graph;                      */
                             /*  2: every decision on the device (the refinement    */
                             /*     steps gated by per-block flags, the Jacobi pass */
                             /*     loop in one persistent launch), one graph per   */
                             /*     iteration, flags read back every check_every    */
                             /*     iterations; 3: the launches of 2 one by one.    */
                             /* All four give the same iterates.  Profiling always  */
                             /* launches one by one.                                */
    int coords;              /* lrr_coords: coordinates of the n-row iterates       */
    int tune;                /* 1: take eig_block, use_graph, check_every, coords   */
                             /* from the ctx's schedule table entry for this shape  */
                             /* (lrr_tune_load), if there is one; 0 (default): not  */
    int io_type;             /* lrr_io_type of the matrix arguments (forward entry  */
                             /* points; not with save_for_backward)                 */
    int reserved[3];         /* must be zero                                        */
} lrr_opts;

/* Per-block results; every pointer may be NULL, each non-NULL array has t entries. */
typedef struct {
    int *iters;              /* iterations run by each block                        */
    int *rank;               /* rank of each block estimate J_i                     */
    double *res_primal;      /* ||X_i - A Z_i - E_i||_max at the last iteration     */
    double *res_coupling;    /* ||Z_i - J_i||_max at the last iteration             */
    int batch_iters;         /* (out) iterations of the batched loop                */
    int combine_rank;        /* (out) rank r_1 of the combine basis                 */
} lrr_info;

/* Library version string. */
const char *lrr_version(void);

/* Fill *opts with the defaults listed above. */
void lrr_opts_default(lrr_opts *opts);

/* Create a context bound to HIP device `device`.  *out is NULL on failure. */
lrr_status lrr_ctx_create(int device, lrr_ctx **out);

/* Release the context and its workspace.  NULL is accepted. */
void lrr_ctx_destroy(lrr_ctx *ctx);

/* Message of the last failure on ctx (or of the last failure without a ctx). */
const char *lrr_last_error(const lrr_ctx *ctx);

/* Schedule table written by the autotuner (paper_1304_5583_amd/autotune.py): one
 * entry per line, "m n t maxl precision eig_block use_graph check_every coords"
 * (integers; '#' starts a comment; maxl = the largest block width).  A solve with
 * opts.tune = 1 whose (m, n, t, maxl, precision) equal an entry's runs with that
 * entry's Jacobi block width, graph use, convergence-check spacing and
 * coordinates -- schedule choices the tuner accepted only where they reproduce
 * the default schedule's iterates (same iteration counts, Z within 1e-8).  path
 * NULL clears the table; a malformed file leaves the previous table and returns
 * LRR_EINVAL naming the line.  At context creation the file named by the
 * environment variable LRR_TUNE_TABLE, if set and well formed, is loaded. */
lrr_status lrr_tune_load(lrr_ctx *ctx, const char *path);

/* Host-only check of a D-step partition (Algorithm 1, SampleCols): perm must be a
 * permutation of 0..n-1 and offsets[0] = 0 < offsets[1] < ... < offsets[t] = n.
 * perm and offsets are host int32 arrays of length n and t+1. */
lrr_status lrr_check_partition(int n, int t, const int *perm, const int *offsets);

/* Device bytes of workspace dfc_lrr_solve would hold for this problem. */
lrr_status lrr_workspace_bytes(int m, int n, int t, const int *offsets,
                               const lrr_opts *opts, size_t *bytes);

/*
 * Eq. (2) with one block: observations X (m x l, device), dictionary A (m x n,
 * device).  Writes Z (n x l, ldz >= n) and, if E is not NULL, E (m x l, lde >= m).
 * Z is the ALM iterate Z; at convergence it differs from the exactly low-rank J
 * by less than tol in max-norm.
 */
lrr_status lrr_solve(lrr_ctx *ctx, int m, int n, int l,
                     const void *A, int lda, const void *X, int ldx,
                     double lambda, const lrr_opts *opts,
                     void *Z, int ldz, void *E, int lde,
                     lrr_info *info, void *stream);

/*
 * Algorithm 1 (DFC-LRR) on M (m x n, device).  Block i holds the original
 * columns perm[offsets[i] .. offsets[i+1]-1] (host arrays, see
 * lrr_check_partition).  Every block solves Eq. (2) with C_i = M[:, block] and
 * the whole M as dictionary (same lambda for all blocks); the estimate of a block
 * is its J at termination (exactly low rank, factored).  The C step projects
 * [J_1 ... J_t] onto the column space of J_1 and puts the columns back in their
 * original order: Z (n x n, ldz >= n).  If S is not NULL it receives the outlier
 * estimates [E_1 ... E_t] in the original column order (m x n, lds >= m).
 * With t = 1 the result is J of lrr_solve(X = M, A = M).
 */
lrr_status dfc_lrr_solve(lrr_ctx *ctx, int m, int n, const void *M, int ldm,
                         double lambda, int t, const int *perm, const int *offsets,
                         const lrr_opts *opts, void *Z, int ldz, void *S, int lds,
                         lrr_info *info, void *stream);

/*
 * The alternative formulation of the Section 2.2 footnote: block i solves Eq. (1)
 * with C_i = M[:, block] as both dictionary and observations, so its estimate
 * J_i (at termination, exactly low rank) is l_i x l_i and relates the block's
 * own points; all blocks run batched as in dfc_lrr_solve, each with its own
 * (I + C_i C_i^T)^{-1}.  C step: the best rank-k approximation in the Frobenius
 * norm of diag(J_1, ..., J_t) -- the k largest singular triplets pooled over the
 * blocks -- with k = combine_rank if > 0, max_i rank(J_i) if 0, every triplet if
 * < 0.  Z (n x n, ldz >= n) receives block i at rows and columns
 * perm[offsets[i] .. offsets[i+1]-1] and zeros elsewhere; S (optional) the
 * outlier estimates in the original column order (m x n, lds >= m);
 * info->combine_rank the k used.  opts.coords and opts.solve_form are ignored
 * (full coordinates, push-through solve); save_for_backward is rejected
 * (LRR_EINVAL).
 */
lrr_status dfc_lrr_solve_local(lrr_ctx *ctx, int m, int n, const void *M, int ldm,
                               double lambda, int t, const int *perm, const int *offsets,
                               int combine_rank, const lrr_opts *opts, void *Z, int ldz,
                               void *S, int lds, lrr_info *info, void *stream);

/*
 * Reverse-mode derivative of the last dfc_lrr_solve on ctx, which must have run
 * with save_for_backward = 1 and fixed_iters > 0 (the unrolled map).  Given
 * dZ = dL/dZ (n x n, device, original column order) it writes dL/dlambda to
 * *dlambda (host) and, if dM is not NULL, dL/dM (m x n, device, lddm >= m).
 */
lrr_status dfc_lrr_backward(lrr_ctx *ctx, const void *dZ, int lddz,
                            double *dlambda, void *dM, int lddm, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LRR_H */
