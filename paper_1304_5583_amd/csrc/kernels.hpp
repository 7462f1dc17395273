// Host-side launchers of the library's kernels.
#pragma once

#include "common.hpp"

namespace lrr {

// gemm.hip
void launch_dgemm(const GemmDesc* d_descs, int count, int maxM, int maxN, bool ta, bool tb,
                  hipStream_t stream);
// C = A^T B for square C (descriptors with M = N) known to be symmetric (A^T A,
// X^T (B X)): only the tiles on and above the diagonal are computed, the others
// mirrored (for A^T A bitwise the full product); batches of fewer than 512 full
// tiles take the full kernel unless `always`
void launch_dgemm_sym(const GemmDesc* d_descs, int count, int maxN, hipStream_t stream, bool always = false);
// whether launch_dgemm_sym runs the triangle of tiles for this batch
bool dgemm_sym_tiles(int count, int maxN);
// workgroups of a GEMM launch (looked up once; call before a stream capture)
int gemm_grid(void);
// leading dimensions of the FP64 GEMM's operands stay below this (32-bit panel offsets)
constexpr int kGemmMaxLd = 1 << 22;

// xgemm.hip: the same contract with the arithmetic chosen by `mode` (GemmMode)
void launch_xgemm(const GemmDesc* d_descs, int count, int maxM, int maxN, bool ta, bool tb, int mode,
                  hipStream_t stream);
const char* xgemm_name(int mode, bool ta, bool tb);

// chol.hip
int spd_inverse_desc_count(int m);
void spd_inverse(double* K, int m, double* Lbuf, double* Linv, double* Dinv, double* Tbuf,
                 GemmDesc* d_desc, int* d_info, hipStream_t s);
void launch_add_identity(double* A, int lda, int m, double s, hipStream_t st);

// jacobi.hip
void launch_jacobi_init(const EigDesc* d_descs, int count, hipStream_t s);
void launch_jacobi_round(const EigDesc* d_descs, int count, int maxL, int bs, int round, hipStream_t s);
// sched: take the round's pairs from EigDesc::sched instead of the circle method
void launch_jacobi_pairs(const EigDesc* d_descs, int count, int maxL, int bs, int round, hipStream_t s,
                         bool sched = false);
void launch_jacobi_apply(const EigDesc* d_descs, int count, int maxL, int bs, int round, hipStream_t s,
                         bool sched = false);
// bs > 0: also mark the index-block pairs that need rotations (EigDesc::need)
void launch_jacobi_check(const EigDesc* d_descs, int count, int maxL, int* d_open, hipStream_t s, int bs = 0);
void launch_jacobi_sweep_end(const EigDesc* d_descs, int count, int* d_any, hipStream_t s);
void launch_jacobi_eigvals(const EigDesc* d_descs, int count, hipStream_t s);
// The whole block-Jacobi pass loop of `count` matrices (bs = 16 or 32) in
// one persistent launch (after a reset of ctl): d_offs holds the prefix counts
// of the matrices' rows, pair slots and apply items (3 x (count + 1)); d_brounds
// count ints of scratch; need_all the marks of all matrices (need_total ints,
// EigDesc::need points into it).  ctl->err != 0 afterwards: a barrier wait ran
// out (the grid did not fit on the chip); the decompositions are then invalid.
void launch_jacobi_solve(const EigDesc* d_descs, int count, const int* d_offs, int* d_brounds, JacCtl* ctl,
                         const DevIter* it, int max_sweeps, int max_targeted, int nb_max, int bs, int* need_all,
                         long need_total, hipStream_t s);
int jacobi_solve_grid(int bs);

// refsyev.hip
void launch_ref_begin(const RefDesc* d, int count, int maxL, const int* svt_run, const int* warm, hipStream_t s);
// gid: X^T X taken as the identity (G not read; the first step of a warm refinement)
void launch_ref_rows(const RefDesc* d, int count, int maxL, const DevIter* it, hipStream_t s, bool gid = false);
void launch_ref_E(const RefDesc* d, int count, int maxL, hipStream_t s, bool gid = false);
void launch_ref_add(const RefDesc* d, int count, int maxL, hipStream_t s);
// stop: a step whose largest correction falls below it is the last one
void launch_ref_update(const RefDesc* d, int count, int step, int max_steps, double stop, hipStream_t s);
void launch_ref_next(const RefDesc* d, int count, hipStream_t s);
void launch_orth_guard(const RefDesc* d, int count, int maxL, const int* warm, hipStream_t s);
// count_pass: count this pass of the sweep loop toward the block's switch rule
void launch_lo_rows(const EigDesc* d, int count, int maxL, const DevIter* it, hipStream_t s,
                    bool count_pass = true);
void launch_orth_E(const RefDesc* d, int count, int maxL, hipStream_t s);
void launch_ref_set_run(const RefDesc* d, int count, const int* svt_run, hipStream_t s);
// the orthogonalisation steps run for the blocks that need a decomposition and did not measure
// |I - X^T X| <= 1e-8 in their last refinement step
void launch_ref_set_run_ns(const RefDesc* d, int count, const int* svt_run, hipStream_t s);
// the Jacobi matrix is formed only for the blocks that need a decomposition and are not clean
void launch_ref_set_run_jac(const RefDesc* d, int count, const int* svt_run, hipStream_t s);
// after the first orthogonalisation step: the second runs where |I - X^T X| exceeded 1e-8
void launch_orth_decide(const RefDesc* d, int count, hipStream_t s);
void launch_lo_mode(const int* svt_run, const int* warm, int* passes, double* cut, int t, hipStream_t s);
void launch_mark_warm(const int* svt_run, int* warm, int t, hipStream_t s);

// alm.hip
void launch_gather_cols(const double* M, long ldm, double* X, long ldx, int m, int ncols,
                        const int* d_perm, hipStream_t s);
void launch_scatter_cols(const double* X, long ldx, double* S, long lds, int m, int ncols,
                         const int* d_perm, hipStream_t s);
void launch_copy_cols(const double* X, long ldx, double* Y, long ldy, int m, int ncols, hipStream_t s);
// FP32 <-> FP64 copies of a column-major matrix
void launch_widen_cols(const float* src, long lds, double* dst, long ldd, int rows, int cols, hipStream_t s);
void launch_narrow_cols(const double* src, long lds, float* dst, long ldd, int rows, int cols, hipStream_t s);
void launch_nonfinite(const double* M, long ldm, int m, int n, int* d_flag, hipStream_t s);
void launch_form_Y(const double* Z, const double* Y2, double* Y, double* colsq, int n, long ld, int ncols,
                   const int* colblk, const int* active, const DevIter* it, hipStream_t s);
void launch_block_fro(const double* colsq, const int* boff, int t, BlockState bs, const DevIter* it,
                      hipStream_t s);
// eig_run: the blocks that threshold, plus (prewarm > 0, in an iteration where some block
// thresholds for the first time) the blocks not yet decomposed with ||Y||_F > prewarm * tau
void launch_eig_select(const double* colsq, const int* boff, int t, const int* active, const int* svt_run,
                       const int* warm, int* eig_run, const DevIter* it, double prewarm, hipStream_t s);
void launch_zero_J(double* J, int n, long ld, int ncols, const int* colblk, BlockState bs, hipStream_t s);
void launch_svt_weights(const SvtDesc* d, int count, int maxL, const DevIter* it, BlockState bs,
                        hipStream_t s);
void launch_form_QT(const double* J, const double* Y2, double* Q, double* dQ, int n, long ldn,
                    const double* X, const double* E, const double* Y1, double* T, int m, long ldm, int ncols,
                    const int* colblk, const int* active, const DevIter* it, hipStream_t s);
void launch_sub_cols(double* T, const double* A, int m, long ld, int ncols, const int* colblk,
                     const int* active, hipStream_t s);
void launch_update_Z(const double* Q, const double* MtV, const double* J, double* Z, double* Y2, double* R2r,
                     unsigned long long* r2nrm, int n, long ld, int ncols, const int* colblk, BlockState bs,
                     const DevIter* it, hipStream_t s);
// out[b] = max over block b's columns of col (active blocks only); with col2,
// out2[b] likewise in the same launch
void launch_block_colmax(const double* col, const int* boff, int t, BlockState bs, unsigned long long* out,
                         hipStream_t s, const double* col2 = nullptr, unsigned long long* out2 = nullptr);
void launch_r2_decide(BlockState bs, unsigned long long* r2nrm, int* expand, int t, double tol, double sqrt_n,
                      hipStream_t s);
void launch_colmax(const double* A, int n, long ld, int ncols, const int* colblk, const int* expand,
                   unsigned long long* out, hipStream_t s);
void launch_gather_scaled(const double* W, long ldw, const double* lam, const int* idx, double* Wk, long ldk,
                          int m, int r, hipStream_t s);
void launch_ns_factor(const double* G, double* T, int r, hipStream_t s);
void launch_estep(double* E, const double* V, double* Y1, int m, long ld, int ncols, double lam,
                  const int* colblk, BlockState bs, const DevIter* it, hipStream_t s);
void launch_check(BlockState bs, int t, DevIter* it, const double* mu_sched, double tol, int fixed,
                  int* n_active, hipStream_t s);
void launch_init_iter(DevIter* it, const double* mu_sched, int k, hipStream_t s, int full = 0);
void launch_scale_cols(double* U, long ld, int rows, int ncols, const double* h, hipStream_t s);
void launch_set_identity(double* W, int L, hipStream_t s);
void launch_scatter_block_diag(const double* J, long ldj, int ncols, const int* colblk, const int* boff,
                               const int* perm, double* out, long ldo, hipStream_t s);

// adjoint.hip
void launch_bw_estep(const double* E0, const double* V, double* cE, const double* cY1, double* Vb,
                     double* lamcol, int m, long ld, int ncols, const int* colblk, const int* active,
                     const DevIter* it, double lam, hipStream_t s);
void launch_bw_zt(const double* cZ, const double* cY2, const double* cJ, double* Zt, double* Jt, int n, long ld,
                  int ncols, const int* colblk, const int* active, const DevIter* it, hipStream_t s);
void launch_bw_mid(const double* Qb, double* Jt, double* cY2, const double* Wb, double* Xbar, double* cE,
                   double* cY1, int n, long ldn, int m, long ldm, int ncols, const int* colblk,
                   const int* active, const DevIter* it, hipStream_t s);
void launch_bw_final(const double* Yb, double* cY2, int n, long ld, int ncols, const int* colblk,
                     const int* active, const DevIter* it, hipStream_t s);
void launch_zero_norun(double* A, int n, long ld, int ncols, const int* colblk, const int* run, const int* active,
                       hipStream_t s);
void launch_bw_wg(const BwDesc* d, int count, int maxL, const DevIter* it, hipStream_t s);
void launch_bw_sym(const BwDesc* d, int count, int maxL, hipStream_t s);
void launch_bw_phi(const BwDesc* d, int count, int maxL, const DevIter* it, hipStream_t s);
void launch_bw_rdiag(const double* W, const double* lam, double* Wr, int L, int l, const DevIter* it,
                     hipStream_t s);
void launch_scatter_add(const double* Xb, long ldx, double* Mb, long ldm, int m, int ncols, const int* perm,
                        hipStream_t s);
void launch_add_cols(double* A, long lda, const double* B, long ldb, int rows, int ncols, hipStream_t s);

}  // namespace lrr
