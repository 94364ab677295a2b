/*
 * tt.h -- C ABI of libtt, the MI355X (gfx950) hot path of generalized-loss
 * CP tensor completion.
 *
 * Problem statement followed by every call (Section 2.1, eq. obj): a sparse
 * order-N tensor with observed index set Omega (m nonzeros), factor matrices
 * A_n of shape I_n x R, the CP model m_e = sum_r prod_n A_n[i_n(e), r]
 * (eq. 1/2; Appendix A for order N), and the objective
 *     f = sum_{e in Omega} phi(t_e, m_e) + lambda * sum_n ||A_n||_F^2.
 *
 * Conventions shared by all calls
 * -------------------------------
 *  - Indices are 0-based int32.  The kernels implement order N = 3 (the
 *    paper's focus, Section 2); tt_build_index returns TT_ERR_UNSUPPORTED
 *    for other orders.  Rank 1 <= R <= 64.
 *  - Factor matrices are row-major with leading dimension ldA >= R elements
 *    (element (i, r) at A + i * ldA + r), stored in the factor dtype `fdt`.
 *    Row starts must be 16-byte aligned for the vectorized path (ldA * size
 *    a multiple of 16 and an aligned base); otherwise a scalar path is used.
 *  - "Value dtype": per-nonzero arrays (observed values, weights, TTTP
 *    outputs) are double when fdt == TT_F64 and float otherwise.  Dense
 *    outputs (MTTKRP, gradient, GN matvec, right-hand sides) are double
 *    when fdt == TT_F64 and float otherwise, contiguous I_n x R.
 *  - Orders of per-nonzero arrays: TT_ORDER_COO (-1) is the caller's COO
 *    order; n >= 0 is the order of mode n after the stable sort done by
 *    tt_build_index (Section 3.4 counting sort).  TT_INDEX_T passed as a
 *    value pointer selects the observed values t held by the index, already
 *    in the needed order.  A NULL value/weight pointer means the unit-valued
 *    pattern tensor Omega-hat.
 *  - All device pointers are caller-owned (typically torch tensors); the
 *    library never frees them.  Every call except tt_build_index and calls
 *    passed TT_SYNC is asynchronous on `stream`, performs no allocation once
 *    the index workspace has been sized (see tt_index_reserve) and no host
 *    synchronization, so it may be captured in a hipGraph.
 *  - Calls that use the same tt_index share its workspace and must be
 *    ordered on one stream.  Distinct indices may be used concurrently.
 *  - Argument errors are detected on the host before anything is enqueued;
 *    the call then returns a negative status and enqueues nothing.
 *    tt_last_error() returns a thread-local message for the last failure.
 */
#ifndef TT_H
#define TT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tt_status;
#define TT_OK 0
#define TT_ERR_INVALID_ARG (-1)  /* bad pointer, size, order, rank or enum   */
#define TT_ERR_INDEX_RANGE (-2)  /* some i_n(e) outside [0, I_n)              */
#define TT_ERR_OOM (-3)          /* device allocation failed                  */
#define TT_ERR_HIP (-4)          /* HIP runtime error (message has details)   */
#define TT_ERR_NOT_SPD (-5)      /* TT_SYNC solve met a non-SPD row system    */
#define TT_ERR_UNSUPPORTED (-6)  /* valid request outside the supported set  */

typedef enum { TT_F64 = 0, TT_F32 = 1, TT_BF16 = 2 } tt_dtype;

/* Per-nonzero epilogues of tttp (Section 3.3: TTTP yields the model values
 * from which the derivative tensors phi', phi'' of eq. deriv_tnsr are formed). */
typedef enum {
  TT_EPI_NONE = 0,   /* out_e = s_e * m_e                                   */
  TT_EPI_RESID = 1,  /* out_e = t_e - m_e                                   */
  TT_EPI_PHI = 2,    /* out_e = phi(t_e, m_e)                               */
  TT_EPI_DPHI = 3,   /* out_e = phi'(t_e, m_e)                              */
  TT_EPI_D2PHI = 4   /* out_e = phi''(t_e, m_e)                             */
} tt_epilogue;

/* Elementwise losses: least squares (t - m)^2 (Section 2.1) and the Poisson
 * log-link loss exp(m) - t m (Section 5.7; the log t! constant dropped). */
typedef enum { TT_LOSS_LS = 0, TT_LOSS_POISSON_LOG = 1 } tt_loss;

#define TT_ORDER_COO (-1)
#define TT_ORDER_PER_MODE (-2) /* gn_matvec/solve weights: host array of N
                                  device pointers, entry d in mode-d order */
#define TT_INDEX_T ((const void *)1)
#define TT_RHS_MTTKRP ((const void *)2)
#define TT_SYNC 1u
#define TT_MAX_ORDER 4
#define TT_MAX_RANK 64

typedef struct tt_index tt_index; /* opaque, library-owned */

/* ---------------------------------------------------------------------------
 * tt_build_index -- per-mode stable counting sort of the nonzeros
 * (Section 3.4: sort by the mode-n index so each row's nonzeros are
 * contiguous; Section 3.1: only nonzero rows are kept, as in the compressed
 * row layout).  For every mode n it stores on the device: perm_n (sorted
 * position -> COO position, ties in COO order), the sorted mode-n indices,
 * the other modes' indices in sorted order, ptr_n (I_n + 1 offsets, int64),
 * the list of nonzero rows, t pre-permuted into mode-n order (if d_t given),
 * and the work partitions used by the kernels.
 *   order    N (3).              dims   host array of N extents (>= 1).
 *   nnz      m >= 0 (m < 2^31).  d_idx  host array of N device pointers, m
 *            int32 each.         d_t    device pointer to m observed values
 *            in COO order, of dtype vdt (TT_F64 or TT_F32), or NULL.
 *   flags    0.                  stream HIP stream for the build kernels.
 *   out      receives the new index.
 * Synchronizes `stream` once.  Returns TT_ERR_INDEX_RANGE (and no index) if
 * any index lies outside its dimension.  The caller's arrays are not
 * retained: they may be freed after the call returns.
 * ------------------------------------------------------------------------- */
tt_status tt_build_index(int order, const int64_t *dims, int64_t nnz,
                         const int32_t *const *d_idx, const void *d_t,
                         tt_dtype vdt, uint32_t flags, hipStream_t stream,
                         tt_index **out);

/* Frees everything the index owns.  NULL is accepted. */
tt_status tt_index_destroy(tt_index *ix);

/* Sizes the index workspace for ranks up to R and factor dtype fdt, so that
 * later calls allocate nothing (needed before hipGraph capture).  Calls
 * made without it size the workspace on first use.  `flags` adds the
 * workspaces of tt_gn_step: TT_RESERVE_GN (PCG vectors and preconditioner
 * factors, least squares) and TT_RESERVE_GN_POISSON (also the per-mode
 * phi'' weights of the Poisson loss); either flag also builds the position
 * map of gn_matvec (N x 4 bytes per nonzero, kept until the index is
 * destroyed; built on the null stream, which is synchronized). */
#define TT_RESERVE_GN 1u
#define TT_RESERVE_GN_POISSON 2u
tt_status tt_index_reserve(tt_index *ix, int R, tt_dtype fdt, uint32_t flags);

/* ---------------------------------------------------------------------------
 * Work-partition tuning of an index (the tile selection that an autotuner
 * varies).  Results do not depend on it beyond floating-point summation
 * order.
 *   chunk       nonzeros per streaming work chunk: 512, 1024 or 2048
 *               (heavier rows are cut into pieces of this size)
 *   gram_piece  nonzeros per Gram task, 1024 .. 65536 (rows with more are
 *               split into tasks and their Grams summed in FP64)
 *   gram_light  Gram tasks with more nonzeros than this run on a workgroup
 *               of gram_waves waves, the others on one wave; 0 .. gram_piece
 *   gram_waves  2, 4 or 8
 *   solve_wgs   0: the per-row solve kernels launch one workgroup per row;
 *               1 .. 64: they run as persistent kernels, solve_wgs
 *               workgroups per compute unit, each taking every grid-th row
 *               of the batch in order
 *   pcg_wgs     0: the conjugate-gradient iterations of tt_gn_step run
 *               kernel by kernel; 1 .. 16: at ranks up to 16 they run as
 *               one persistent kernel of pcg_wgs workgroups per compute
 *               unit (capped so that all are resident at once), the phases
 *               of an iteration separated by grid-wide barriers, with
 *               results bit-identical to the kernel-by-kernel loop; -1:
 *               persistent (two workgroups per compute unit) when each
 *               streaming phase of the loop fits in one round of that grid
 *               (launch-bound sizes), kernel by kernel otherwise.  Two
 *               persistent loops running at the same time on one device may
 *               not fit together: a loop whose barrier wait exceeds its
 *               spin bound stops, leaves the factors unchanged and reports
 *               iterations = -1 and a NaN residual in tt_gn_step's
 *               statistics
 *   ccd_xcd     tt_ccd_sweep's stream layout: 1: each mode's nonzeros are
 *               regrouped per row by the bucket (8 row ranges of balanced
 *               nonzero count) of their index in the largest other mode,
 *               and bucket b's tasks run on workgroups b, b + 8, ...
 *               (workgroups go to the 8 XCDs in turn, so each XCD's L2
 *               holds one bucket's column records); 0: the sorted stream;
 *               -1: the regrouped layout for modes whose largest other
 *               mode's column records exceed 2 MiB.  Built on first use
 *               (allocation, synchronization; 16 bytes per nonzero per
 *               mode); results do not depend on it
 *   ccd_lds     tt_ccd_sweep's record gathers: -1: in each mode's pass the
 *               column records of the smaller other mode are copied into
 *               LDS by every workgroup first when they fit in 48 KiB (the
 *               workgroups then loop over the pass's tasks), so only the
 *               other mode's records are gathered from memory; 0: both
 *               from memory.  Results do not depend on it
 * tt_index_tune rebuilds the partitions on `stream` and synchronizes it (it
 * is not capturable, and fails with TT_ERR_INVALID_ARG while an instantiated
 * graph is alive); call tt_index_reserve again afterwards if the
 * workspace was reserved.  Defaults: 1024, 4096, 512, 4, 0, -1, -1, -1.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t chunk;
  int32_t gram_piece;
  int32_t gram_light;
  int32_t gram_waves;
  int32_t solve_wgs;
  int32_t pcg_wgs;
  int32_t ccd_xcd;
  int32_t ccd_lds;
} tt_tuning;
tt_status tt_index_tune(tt_index *ix, const tt_tuning *tuning, hipStream_t stream);
tt_status tt_index_get_tuning(const tt_index *ix, tt_tuning *out);

/* Read-only views of mode `mode` for tests: device pointers to ptr (int64,
 * I_n + 1), perm (int32, m), sorted mode indices (int32, m), nonzero rows
 * (int32, nrows); host count of nonzero rows.  Any output may be NULL. */
tt_status tt_index_view(const tt_index *ix, int mode, const int64_t **d_ptr,
                        const int32_t **d_perm, const int32_t **d_key,
                        const int32_t **d_rows, int64_t *nrows);

/* Sorted index stream of mode `mode` for the other mode `other` (int32, m). */
tt_status tt_index_other(const tt_index *ix, int mode, int other,
                         const int32_t **d_sorted_idx);

/* ---------------------------------------------------------------------------
 * tttp -- tensor-times-tensor product (Section 3.3):
 *     x_e = s_e * sum_r prod_{n in P} A_n[i_n(e), r]
 * where P is the set of modes whose d_A[n] is non-NULL (a NULL entry skips
 * that mode, Section 3.3).  With an epilogue other than TT_EPI_NONE, d_s
 * holds the observed values t and out_e = the epilogue of (t_e, m_e), using
 * `loss`; all N factors must then be given.
 *   d_s, s_order    values and their order (TT_INDEX_T allowed, NULL =
 *                   Omega-hat for TT_EPI_NONE).
 *   d_A             host array of N device pointers (entries may be NULL).
 *   R, ldA, fdt     rank, leading dimension, factor dtype.
 *   d_out           m values (value dtype) written in `out_order`.
 *   d_sum           optional device double: receives sum_e out_e (FP64,
 *                   deterministic order), overwritten.
 * ------------------------------------------------------------------------- */
tt_status tttp(const tt_index *ix, const void *d_s, int s_order,
               const void *const *d_A, int R, int64_t ldA, tt_dtype fdt,
               tt_epilogue epi, tt_loss loss, void *d_out, int out_order,
               double *d_sum, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * mttkrp -- matricized tensor times Khatri-Rao product (Section 3.2; the
 * right-hand sides of Section 2.2; the gradient contraction of Appendix A):
 *     Y[i, r] = sum_{e : i_mode(e) = i} s_e * prod_{p != mode} A_p[i_p(e), r]
 *   d_s, s_order    weights (TT_INDEX_T = observed t; NULL = Omega-hat).
 *   d_A             host array of N device pointers; entry [mode] ignored.
 *   d_out           I_mode x R, dense dtype; overwritten, or added to when
 *                   accumulate != 0.
 * Segments are reduced with FP32 chains of at most 144 terms (a lane
 * group's share of a work chunk, then the in-order combination of the
 * groups' pieces; FP64 for TT_F64) and partials of rows longer than one work
 * chunk are combined in FP64 in a fixed order, so results are deterministic.
 * ------------------------------------------------------------------------- */
tt_status mttkrp(const tt_index *ix, const void *d_s, int s_order,
                 const void *const *d_A, int R, int64_t ldA, tt_dtype fdt,
                 int mode, void *d_out, int accumulate, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * mttkrp_noalloc -- mttkrp for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as mttkrp; it calls no
 * allocator.  The FP64 carry slots of rows longer than one work chunk and
 * their partials live in a fixed 32 MiB array per device, held from the
 * first call on that device until the process ends.  A mode needs
 * (pieces + segments) x RP x 8 bytes, RP being the rank rounded up to a power
 * of two of at least 8 elements (4 for TT_F64); a call that needs more fails
 * with TT_ERR_UNSUPPORTED and enqueues nothing.  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other host threads) race and must be serialized by the caller.
 * The array's contents are fully rewritten by each call before they are
 * read.  The index must already hold its partitions (tt_build_index); call
 * on the device the index was built on.
 * ------------------------------------------------------------------------- */
tt_status mttkrp_noalloc(const tt_index *ix, const void *d_s, int s_order,
                         const void *const *d_A, int R, int64_t ldA, tt_dtype fdt, int mode,
                         void *d_out, int accumulate, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * solve_factor -- Solve Factor (Section 3.4): for every row i of `mode`
 *     G^(i) = sum_{e in row i} w_e h_e h_e^T,  h_e = Hadamard_{p != mode} A_p[i_p(e)]
 *     (G^(i) + lambda I) x_i = M_i
 * G^(i) is accumulated in FP32 on matrix cores (FP64 for TT_F64) from exact
 * bf16 splits of the FP32 products, converted
 * to FP64, shifted by exactly `lambda` (least-squares ALS passes lambda; the
 * Gauss-Newton block preconditioner passes 2 lambda with w = phi''), factored
 * by Cholesky and solved in FP64.  Weights may be negative; a row whose
 * shifted matrix is not positive definite gets x_i = 0 and
 * info_i = k > 0, the order of the first non-positive leading minor (LAPACK
 * potrf convention).  Rows without nonzeros solve lambda x = M_i.
 *   d_w, w_order    weights (NULL = Omega-hat; TT_ORDER_PER_MODE allowed).
 *   d_rhs           I_mode x R right-hand sides, dense dtype; or
 *                   TT_RHS_MTTKRP: M = MTTKRP of the observed values t with
 *                   the other factors (the ALS normal-equation right-hand
 *                   side of Section 2.2; needs d_w NULL), which the FP32 and
 *                   BF16 forms accumulate in FP64 in the same pass over the
 *                   nonzeros as the Gram (FP64: a separate MTTKRP).
 *   d_X             I_mode x R output in fdt with leading dimension ldA
 *                   (BF16 is rounded to nearest even); may alias d_A[mode].
 *   d_info          optional int32[I_mode].
 *   flags           TT_SYNC: synchronize and return TT_ERR_NOT_SPD if any
 *                   row failed (requires d_info).
 * ------------------------------------------------------------------------- */
tt_status solve_factor(const tt_index *ix, const void *d_w, int w_order,
                       const void *const *d_A, int R, int64_t ldA,
                       tt_dtype fdt, int mode, const void *d_rhs,
                       double lambda, void *d_X, int32_t *d_info,
                       uint32_t flags, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * solve_factor_model -- the ALS update of mode `mode` (solve_factor with
 * d_rhs = TT_RHS_MTTKRP and no weights) that also evaluates the model at
 * every nonzero (TTTP, Section 3.3, of the factors as they are before the
 * update): d_model[e] = sum_r prod_n A_n[i_n(e), r] for the nonzeros in the
 * index's mode-`mode` sorted order (value dtype, m values).  The FP32 and
 * BF16 forms compute the model values in the Gram pass from the factor rows
 * it gathers anyway (one pass over the nonzeros for both results); the
 * FP64 form runs a TTTP pass first.  Every d_A[p] must be given; d_X may
 * alias d_A[mode]; d_info as in solve_factor.  The model values are those
 * of tttp with d_s NULL up to FP32 summation order.
 * ------------------------------------------------------------------------- */
tt_status solve_factor_model(tt_index *ix, const void *const *d_A, int R,
                             int64_t ldA, tt_dtype fdt, int mode,
                             double lambda, void *d_X, int32_t *d_info,
                             void *d_model, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * gn_matvec -- implicit Gauss-Newton matrix-vector product (Section 2.5
 * without the phi' terms; the TTTP -> MTTKRP decomposition of Section 2.5;
 * Appendix A first Hessian term):
 *     z_e = sum_p sum_r X_p[i_p(e), r] prod_{q != p} A_q[i_q(e), r]
 *     Y_d = MTTKRP_d(w .* z) + lambda2 * X_d          for every mode d
 * w .* z is formed once, in the sorted order of the mode with the most rows,
 * in the pass that also accumulates that mode's block (TTTP fused into
 * MTTKRP); the other blocks are MTTKRPs of the stored w .* z, read through
 * a position map of the index (mode-n sorted position -> that mode's sorted
 * position), so no pass but the first gathers rows of X.
 *   d_w, w_order    per-nonzero weights (phi''); TT_ORDER_PER_MODE or a
 *                   mode order or COO; NULL = the constant w_const.
 *   d_X, d_Y        host arrays of N device pointers to dense-dtype I_d x R
 *                   blocks (contiguous); Y is overwritten.
 * The first call on an index builds the position map (allocation, kernels
 * on `stream`, one synchronization) unless tt_index_reserve built it; that
 * call fails while `stream` is capturing a graph.  w .* z is kept in an
 * index workspace of m values (value dtype).
 * ------------------------------------------------------------------------- */
tt_status gn_matvec(const tt_index *ix, const void *d_w, int w_order,
                    double w_const, const void *const *d_A,
                    const void *const *d_X, int R, int64_t ldA, tt_dtype fdt,
                    double lambda2, void *const *d_Y, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * newton_matvec -- full Hessian-vector product of the objective (Section 2.5
 * with the phi' terms of the off-diagonal blocks; Appendix A):
 *     Y_d = gn_matvec_d(w, X) + sum_e g_e dh_e^(d),
 *     dh_e^(d) = sum_{p != d} X_p[i_p(e)] * prod_{q != d, p} A_q[i_q(e)]
 * with w = phi'' and g = phi' per nonzero, lambda2 = 2 lambda for the
 * objective's regularizer.  The GN part runs as in gn_matvec (and shares its
 * position map and w .* z workspace); the phi' terms take one more pass per
 * mode, which gathers the rows of both A and X of the other modes.
 *   d_w, w_order    as in gn_matvec.
 *   d_g, g_order    phi' per nonzero: TT_ORDER_PER_MODE (host array of N
 *                   device pointers, each in that mode's sorted order) or
 *                   TT_ORDER_COO; not NULL.
 * The product is symmetric but, unlike the GN operator, not necessarily
 * positive semidefinite.
 * ------------------------------------------------------------------------- */
tt_status newton_matvec(const tt_index *ix, const void *d_w, int w_order,
                        double w_const, const void *d_g, int g_order,
                        const void *const *d_A, const void *const *d_X, int R,
                        int64_t ldA, tt_dtype fdt, double lambda2,
                        void *const *d_Y, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * tt_gradient -- hand-written adjoint of the objective (Table 1 gradient
 * row; Appendix A):  grad_d = MTTKRP_d(phi'(t, m)) + 2 lambda A_d, with m
 * recomputed inside each mode's pass (TTTP fused into MTTKRP).
 *   d_G             host array of N device pointers, dense dtype I_d x R.
 * Requires the index to hold t.
 * ------------------------------------------------------------------------- */
tt_status tt_gradient(const tt_index *ix, const void *const *d_A, int R,
                      int64_t ldA, tt_dtype fdt, tt_loss loss, double lambda,
                      void *const *d_G, hipStream_t stream);

/* tt_objective -- f = sum_e phi(t_e, m_e) + lambda sum_n ||A_n||_F^2 into
 * the device double d_f (FP64 sums, deterministic).  Requires t. */
tt_status tt_objective(const tt_index *ix, const void *const *d_A, int R,
                       int64_t ldA, tt_dtype fdt, tt_loss loss, double lambda,
                       double *d_f, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * tt_als_sweep -- one alternating-least-squares sweep (Section 2.2 and its
 * Section 4 implementation): for n = 0..N-1, M = MTTKRP_n(t) and
 * A_n <- Solve Factor(Omega-hat, A, n, M, lambda).  Factors are updated in
 * place.  Requires t.  d_info: optional int32[sum_n I_n].  In the FP32 and
 * BF16 forms M is formed in the Gram pass (solve_factor with
 * TT_RHS_MTTKRP), so each mode reads its nonzeros once; the FP64 form runs
 * the MTTKRP first.
 * ------------------------------------------------------------------------- */
tt_status tt_als_sweep(tt_index *ix, void *const *d_A, int R, int64_t ldA,
                       tt_dtype fdt, double lambda, int32_t *d_info,
                       hipStream_t stream);

/* ---------------------------------------------------------------------------
 * tt_gn_step -- one preconditioned Gauss-Newton iteration (Section 2.5 and
 * its Section 4 implementation): w = phi''(t, m); b = -grad f; solve
 * (J^T diag(w) J + 2 lambda I) dx = b by PCG from dx = 0 with the block
 * diagonal preconditioner applied through Solve Factor (weights w, shift
 * 2 lambda, factors computed once per call in FP64 and kept in FP64 for
 * the FP64 form, in FP32 for the FP32 and BF16 forms, where they only
 * precondition); stop when the unpreconditioned
 * residual norm relative to the initial one is <= tol or after kmax
 * iterations; then A <- A + dx (full step).  Dot products in FP64.  The
 * iteration count runs on the device: convergence sets a device flag that
 * turns the remaining iterations into no-ops, so no host sync is needed.
 * Depending on the index's tuning (pcg_wgs) the CG iterations run kernel
 * by kernel or as one persistent kernel; both give the same bits.
 *   d_stats         optional device double[4]: iterations, final relative
 *                   residual, initial residual norm, objective before step.
 * The products use gn_matvec's position map: built on first use (one
 * allocation and synchronization) unless tt_index_reserve was called with
 * TT_RESERVE_GN.
 * ------------------------------------------------------------------------- */
tt_status tt_gn_step(tt_index *ix, void *const *d_A, int R, int64_t ldA,
                     tt_dtype fdt, tt_loss loss, double lambda, double tol,
                     int kmax, double *d_stats, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * tt_ccd_sweep -- one least-squares coordinate-minimization sweep in the
 * CCD++ order (Section 2.3 and its Section 4 implementation): for each
 * column r, for each mode n in turn, every entry of column r of A_n is set
 * to its exact minimizer
 *     u_ir = sum_e rhohat_e h_e / (lambda + sum_e h_e^2),   e in row i,
 * h_e the product of the other modes' column-r entries (modes updated
 * earlier in the column contribute their new values) and rhohat the
 * residual t - model without column r's rank-1 term.  The residual is kept
 * in every mode's sorted order (one TTTP pass per mode at the start of the
 * sweep); per column, one pass per mode first moves that mode's residual
 * copy from column r - 1's old to its new rank-1 term and then forms both
 * sums (rhohat from the residual and the column's old entries, on the
 * fly), followed by a rank-1 solve per row (a non-positive pivot gives
 * info 1 and 0, the potrf convention).  Columns r - 1 and r of each factor
 * are read from one record per row.  Depending on the tuning (ccd_xcd) a
 * mode's pass streams its nonzeros regrouped per XCD bucket (the layout is
 * built on the first call), and (ccd_lds) reads the records of a small
 * other mode from an LDS copy.  Factors are updated in place.  Requires t.
 *   d_info          optional int32[sum_n I_n]: the rank-1 solves' info of
 *                   the last column.
 * Workspaces (N m values, 4 (sum_n I_n + N) values, 16 bytes per Gram task)
 * are allocated on first use.
 * ------------------------------------------------------------------------- */
tt_status tt_ccd_sweep(tt_index *ix, void *const *d_A, int R, int64_t ldA,
                       tt_dtype fdt, double lambda, int32_t *d_info,
                       hipStream_t stream);

/* ---------------------------------------------------------------------------
 * tt_gam_sweep -- one generalized alternating-minimization sweep (Section
 * 2.2 for a general loss; stop rule of Section 5.7): for n = 0..N-1, Newton
 * iterations on the rows of A_n with the other factors fixed.  Iteration:
 *     g_i = sum_e phi'(t_e, m_e) h_e + 2 lambda u_i  (row gradient, Table 1)
 *     G_i = sum_e phi''(t_e, m_e) h_e h_e^T           (row Hessian; phi'' = 2
 *                                                    for least squares)
 *     (G_i + 2 lambda I) d_i = -g_i per row          (Solve Factor)
 *     A_n <- A_n + D
 * until ||D||_F <= tol ||A_n||_F (A_n after the update) or max_inner
 * iterations.  For least squares one iteration is the ALS update.  Factors
 * are updated in place; D is held in the factor dtype (rounded to BF16 in
 * the BF16 form) and added in FP64.
 *   FP32 and BF16 forms: g and G of a mode are formed in one pass over its
 *   nonzeros (the Gram pass evaluates the model value m_e = <u_i, h_e>,
 *   phi' and phi''), and the stop rule runs on the device: after each
 *   iteration but a mode's last the two norms are reduced on the device and
 *   a flag turns the mode's remaining launches into no-ops.  With h_iters
 *   NULL the call never synchronizes and can be captured in a graph once an
 *   uncaptured call has sized its workspaces.
 *   FP64 form: a gradient pass (TTTP fused, storing phi'' per nonzero)
 *   then the Gram pass; with tol > 0 the norms are copied to the host after
 *   each iteration but a mode's last (one synchronization each).
 *   tol             > 0: relative step tolerance; <= 0: exactly max_inner
 *                   iterations per mode.
 *   d_info          optional int32[sum_n I_n]: Solve Factor info of each
 *                   mode's last iteration.
 *   h_iters         optional host int32[N]: iterations run per mode (one
 *                   synchronization at the end of the sweep).
 * Workspaces are allocated on first use.  Requires t.
 * ------------------------------------------------------------------------- */
tt_status tt_gam_sweep(tt_index *ix, void *const *d_A, int R, int64_t ldA,
                       tt_dtype fdt, tt_loss loss, double lambda, double tol,
                       int max_inner, int32_t *d_info, int32_t *h_iters,
                       hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batching (graph capture).  The ALS sweep and the Gauss-Newton step
 * enqueue many kernels (per-mode streams, row batches of Gram and solve
 * kernels, and kmax fixed PCG iterations whose early exit is a device flag);
 * a caller that repeats them can record the sequence once and replay it as
 * one launch.
 *   tt_graph_begin  starts capturing `stream` (which must not be the null
 *                   stream; thread-local capture mode).  Every library call
 *                   made on it until tt_graph_end is recorded, not run.  The
 *                   index workspace must be reserved first (tt_index_reserve
 *                   with the flags of the recorded calls) and the kernel
 *                   profiler must be off.
 *   tt_graph_end    ends the capture and instantiates it into *out
 *                   (library-owned until tt_graph_destroy).
 *   tt_graph_launch replays the recorded work on `stream`; pointers and
 *                   scalars are those of the captured calls.
 * Lifetime: a graph replays kernels on the device addresses recorded at
 * capture, including the index's workspaces and work partitions.  While any
 * instantiated graph is alive (from tt_graph_end until tt_graph_destroy;
 * counted process-wide), a call that would reallocate a workspace (a larger
 * rank, the Poisson loss after least squares, a new Gauss-Newton form) and
 * tt_index_tune fail with TT_ERR_INVALID_ARG and enqueue nothing; reserve
 * for the largest call before capturing.  Every index a graph used must
 * outlive the graph (tt_index_destroy does not check).
 * ------------------------------------------------------------------------- */
typedef struct tt_graph tt_graph;
tt_status tt_graph_begin(hipStream_t stream);
tt_status tt_graph_end(hipStream_t stream, tt_graph **out);
tt_status tt_graph_launch(tt_graph *graph, hipStream_t stream);
tt_status tt_graph_destroy(tt_graph *graph);

/* ---------------------------------------------------------------------------
 * Kernel profiler (process-global; use from one host thread).
 * tt_profile_enable(1) clears previous records and starts bracketing every
 * library kernel launch with HIP events on the launch's stream, tagged with
 * the launch's algorithmic bytes and flops (per-nonzero byte model: index
 * streams, values and factor-row gathers at storage precision; Gram flops
 * R (R + 1) per nonzero).  tt_profile_enable(0) stops recording.
 * tt_profile_report writes a JSON object {kernel: {"launches", "ms",
 * "bytes", "flops"}} (NUL-terminated, truncated to cap bytes) after waiting
 * for the recorded events; *needed receives the full size including NUL.
 * ------------------------------------------------------------------------- */
tt_status tt_profile_enable(int on);
tt_status tt_profile_report(char *buf, int64_t cap, int64_t *needed);

/* Thread-local text describing the last non-OK status ("" if none). */
const char *tt_last_error(void);

/* Library version string. */
const char *tt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TT_H */
