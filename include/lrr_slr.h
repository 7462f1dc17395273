/*
 * lrr_slr.h -- SLR-graph construction from a low-rank coefficient matrix.
 *
 * Section 4.2.2 builds a sparse graph over the n samples (columns of M) in two
 * steps: the LRR or DFC-LRR coefficient matrix Z serves as an affinity, and for
 * each sample x_i the n_k samples with the largest affinity to it form the
 * basis D_i of the non-negative Lasso of the SPG construction,
 *
 *     min_w ||x_i - D_i w||_2^2 + alpha ||w||_1   s.t.  w >= 0,
 *
 * whose (typically sparse) solution gives the weights of the edges of sample i.
 * Choices where the paper is silent (the same as the test oracle's): the
 * affinity of samples i and j is |Z_ij| + |Z_ji|; a sample is not its own
 * neighbour; equal affinities go to the lower index; neighbours are listed by
 * decreasing affinity.  The Lasso is solved to its optimality conditions
 * (|g_j| where w_j > 0, -g_j <= 0 where w_j = 0, g = 2 D^T (D w - x) + alpha)
 * within 1e-12 of the sample's scale max(1, |2 D^T x - alpha|_max,
 * 2 max_j |d_j|^2).  When D_i has dependent columns (neighbours from one
 * subspace) the optimal value is unique but the weights need not be.
 *
 * Arguments
 *   ctx        a context from lrr_ctx_create
 *   m, n       M is m x n (DEVICE, double, column-major, ldm >= m), n >= 2
 *   Z, ldz     DEVICE, double, n x n, column-major, ldz >= n, finite entries
 *   nk         neighbours per sample, 1 <= nk <= min(n - 1, 1024)
 *   alpha      l1 weight, alpha > 0 (Section 4.2.2 uses 0.05)
 *   nbr        DEVICE int32, n x nk, sample-major: nbr[i * nk + a] (output)
 *   w          DEVICE double, n x nk, same layout: the weight of edge (i, nbr) (output)
 *   obj        DEVICE double, n (may be NULL): the optimal objective per sample
 *   info       HOST (may be NULL)
 *   stream     hipStream_t (NULL: the null stream)
 *
 * The Lasso is solved by a finite active-set method (Lawson and Hanson's, with
 * the free columns kept independent, so a support never exceeds min(m, n_k));
 * a sample that exceeds 10 n_k + 20 steps stops there.  Supports up to 32 are
 * solved with their factorisations in on-chip memory; a sample whose support
 * grows beyond that is solved again by a second pass that keeps the Cholesky
 * factor of its free set in device memory and updates it as indices enter and
 * leave.  The work runs on `stream` in the ctx's segmentation workspace (not
 * the solver's), which holds one n x n FP64 matrix (first the affinities, then
 * M^T M: 3.2 GB at n = 20000); the second pass, when needed, allocates
 * (2 min(m, n_k)^2 + n_k^2) doubles per concurrently resident sample (at most
 * the samples it has, and what the device can keep resident: about 6 GB at
 * n_k = 500) and frees it before returning.  The call returns when the
 * outputs are complete.  LRR_ENOMEM: a workspace could not be allocated.
 * LRR_NOT_CONVERGED: outputs written, but some sample stopped early
 * (info->not_converged).
 */
#ifndef LRR_SLR_H
#define LRR_SLR_H

#include "lrr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lrr_slr_info {
    int max_steps;       /* most active-set steps any sample needed             */
    int not_converged;   /* samples that stopped without meeting the conditions  */
    double max_kkt;      /* largest final optimality violation / sample scale   */
    int large_support;   /* samples solved by the large-support pass            */
    int max_support;     /* largest number of positive weights of any sample     */
} lrr_slr_info;

lrr_status lrr_slr_graph(lrr_ctx* ctx, int m, int n, const void* M, int ldm, const void* Z, int ldz, int nk,
                         double alpha, int* nbr, double* w, double* obj, lrr_slr_info* info, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LRR_SLR_H */
