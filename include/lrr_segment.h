/*
 * lrr_segment.h -- subspace segmentation from a low-rank coefficient matrix.
 *
 * Section 4.1.2 turns the coefficient matrix Z (n x n) of LRR or DFC-LRR into
 * cluster labels: the affinity U U^T, with U the top left singular vectors of
 * Z, is embedded spectrally into k dimensions and the embedded points are
 * clustered by k-means.  The paper leaves the details open; this entry point
 * fixes them as follows (the same choices as the test oracle's segmentation):
 *
 *   1. r = #{ i : sigma_i(Z) > rank_tol * sigma_1(Z) } (at least 1), U = the r
 *      leading left singular vectors of Z;
 *   2. over the points not excluded (n_keep of them, in index order),
 *      W = |U_keep U_keep^T| (entry-wise absolute value), d = row sums of W
 *      (a zero sum is replaced by 1), L = D^-1/2 W D^-1/2;
 *   3. the k eigenvectors of L with the largest eigenvalues, each row scaled to
 *      unit length (a zero row stays zero);
 *   4. Lloyd's k-means on those rows: the first centre is the point farthest
 *      from the mean of the points, each further centre the point farthest from
 *      the centres chosen so far (ties: lowest index); a point joins the nearest
 *      centre (ties: lowest centre index); a centre moves to the mean of its
 *      points (an empty cluster keeps its centre); stop when no label changes,
 *      or after 300 assignments;
 *   5. clusters are renumbered 0..k-1 in order of first appearance among the
 *      kept points; excluded points get -1.
 *
 * The labels are determined by Z up to ties in steps 1, 3 and 4: the affinity
 * depends only on the span of U, and k-means on the unit rows is invariant
 * under a rotation of the k-dimensional embedding, so any basis of the
 * leading eigenspace gives the same labels.
 *
 * Arguments
 *   ctx        a context from lrr_ctx_create (its device runs the work)
 *   n          number of points (Z is n x n), n >= 1
 *   Z, ldz     DEVICE pointer, double, column-major, ldz >= n
 *   k          number of clusters, 1 <= k <= min(n_keep, 1024)
 *   exclude    DEVICE pointer to n bytes (nonzero: the point is left out, for
 *              example a column flagged as an outlier), or NULL (keep all)
 *   rank_tol   relative singular-value cut of step 1, 0 < rank_tol < 1
 *   rank_bound 0: step 1 works on Z itself (an n x n symmetric eigenproblem,
 *              n <= 8192).  > 0: an upper bound on the rank of Z (for the
 *              DFC-LRR output, the rank of the combine basis, at most the
 *              first block's width); step 1 then works on the range sketch
 *              Z * Omega with rank_bound + 16 columns.  A bound that is too
 *              small is detected (the sketch has full rank) and reported as
 *              LRR_EINVAL.
 *   labels     DEVICE pointer to n int64 values (output)
 *   info       HOST pointer (may be NULL), filled on success
 *   stream     hipStream_t (NULL: the null stream)
 *
 * The work runs on `stream` in a workspace owned by the ctx (separate from the
 * solver's, so a recorded forward for dfc_lrr_backward stays valid); the call
 * returns when the labels are complete.  LRR_NOT_CONVERGED means the labels
 * are written but the spectral embedding did not reach its residual tolerance
 * within the iteration limit (the k-th and (k+1)-th eigenvalues of L are too
 * close for the embedding to be well defined).
 */
#ifndef LRR_SEGMENT_H
#define LRR_SEGMENT_H

#include "lrr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lrr_seg_info {
    int rank;            /* r of step 1                                          */
    int range_rank;      /* columns of the orthonormal range basis of Z           */
    int sketch;          /* columns of the range sketch (n when Z is used itself)  */
    int embed_iters;     /* subspace iterations of step 3                          */
    double embed_resid;  /* largest residual |L x - theta x| of the k vectors      */
    double theta_k;      /* k-th eigenvalue of L                                   */
    double theta_k1;     /* (k+1)-th Ritz value of L (0 when n_keep == k)          */
    int kmeans_iters;    /* label assignments of step 4                            */
    int n_keep;          /* points that were not excluded                          */
} lrr_seg_info;

lrr_status lrr_segment(lrr_ctx* ctx, int n, const void* Z, int ldz, int k, const unsigned char* exclude,
                       double rank_tol, int rank_bound, long long* labels, lrr_seg_info* info, void* stream);

/*
 * Outlier columns as the method itself identifies them (Section 4.1.1: the
 * outliers are the column support of the column-sparse estimate S of Eq. (1) /
 * Eq. (2)).  Column j of the data is flagged when its outlier estimate carries
 * more than the fraction delta of its norm,
 *
 *     ||S[:, j]||_2 > delta * ||M[:, j]||_2 .
 *
 * The paper names no threshold; delta is the caller's choice (delta = 0 flags
 * every column with a nonzero estimate).  The result can serve as the exclude
 * mask of lrr_segment.
 *
 * Arguments
 *   m, n        rows and columns of M and S (m, n >= 1)
 *   M, ldm      DEVICE pointer, double, column-major data (ldm >= m)
 *   S, lds      DEVICE pointer, double, the outlier estimate in the same column
 *               order, e.g. the S output of dfc_lrr_solve (lds >= m)
 *   delta       threshold fraction, >= 0 and finite
 *   flags       DEVICE pointer to n bytes (output: 1 flagged, 0 not)
 *   n_flagged   HOST pointer (may be NULL): number of flagged columns
 *   stream      hipStream_t (NULL: the null stream)
 * Norms are FP64 sums in a fixed order.  Returns when the flags are complete;
 * LRR_EINVAL for bad arguments (nothing written).
 */
lrr_status lrr_outlier_flags(lrr_ctx* ctx, int m, int n, const void* M, int ldm, const void* S, int lds,
                             double delta, unsigned char* flags, int* n_flagged, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LRR_SEGMENT_H */
