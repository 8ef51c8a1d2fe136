/*
 * qtt.h -- C ABI of libqtt: QTT matrix by full-vector products and a
 * refined solve on AMD Instinct MI355X (gfx950).
 *
 * The operation is the QTT matrix-vector product of section 4.2 of
 * Corona, Rahimian, Zorin, "A Tensor-Train accelerated solver for integral
 * equations in complex geometries" (arXiv:1511.06029), Algorithm 2
 * (matrix by uncompressed vector), applied to a block of right-hand sides.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * A QTT matrix with d cores has ranks r_0..r_d (r_0 = r_d = 1), row mode
 * sizes m_1..m_d and column mode sizes n_1..n_d (section 3: the matrix
 * tensorized over the product of a target and a source tree).  Its entries
 * are (TT definition, section 2.2)
 *     A(i, j) = G_1(:, i_1, j_1, :) G_2(:, i_2, j_2, :) ... G_d(:, i_d, j_d, :)
 * with the flat indices built first digit fastest (section 2.1, Matlab
 * order; core 1 is the finest tree level):
 *     i = i_1 + m_1 (i_2 + m_2 (i_3 + ...)),  j = j_1 + n_1 (j_2 + ...).
 * A has M = prod m_k rows and N = prod n_k columns.
 *
 * Vectors are FP64 and live in device memory.  A block of K vectors is
 * column-major: column c starts at ptr + c * ld, ld >= length.
 *
 * Streams are hipStream_t values passed as void* (NULL: the null stream).
 * Enqueueing entry points return after enqueueing; device faults surface at
 * the caller's next synchronisation.  Argument and shape errors are detected
 * before anything is enqueued and leave outputs untouched.
 *
 * Handles are immutable after qtt_matrix_load and may be used concurrently
 * from several host threads and streams, provided the workspaces differ.
 *
 * Every function returns QTT_OK or an error code; qtt_last_error() gives a
 * message for the calling thread's last failure.
 */
#ifndef QTT_H
#define QTT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qtt_matrix_s* qtt_matrix_t;

/* Arithmetic of a sweep.  FP64: FP64 cores, intermediates and accumulation.
 * FP32: FP32 cores and intermediates, FP32 accumulation.  BF16: BF16 cores
 * and intermediates, FP32 accumulation.  Inputs are read as FP64 and
 * converted when the first core loads them; the last core writes FP64.
 * Values are bit flags so that qtt_matrix_load can take several. */
typedef enum {
  QTT_FP64 = 1,
  QTT_FP32 = 2,
  QTT_BF16 = 4
} qtt_dtype_t;

typedef enum {
  QTT_OK = 0,
  QTT_ERR_INVALID_ARG = 1,   /* null or overlapping pointers, bad flags, bad counts */
  QTT_ERR_SHAPE = 2,         /* ranks or modes inconsistent, solve with non-square modes */
  QTT_ERR_OUT_OF_MEMORY = 3, /* device allocation failed in qtt_matrix_load */
  QTT_ERR_DEVICE = 4,        /* a HIP call failed */
  QTT_ERR_NOT_CONVERGED = 5, /* qtt_solve reached max_iter above rtol */
  QTT_ERR_NONFINITE = 6,     /* qtt_solve met a NaN or Inf residual */
  QTT_ERR_WORKSPACE = 7,     /* workspace smaller than the one-vector minimum */
  QTT_ERR_DTYPE = 8,         /* the handle holds no device copy in this dtype */
  QTT_ERR_RANK = 9           /* a TT rounding needed ranks above max_rank (result kept at max_rank) */
} qtt_status_t;

/* Load a QTT matrix onto the current HIP device.
 *   d       number of cores, 1 <= d <= 64.
 *   ranks   d+1 values, ranks[0] = ranks[d] = 1, all >= 1.
 *   m, n    d row and d column mode sizes, all >= 1.
 *   cores   d host pointers; cores[k] is a dense FP64 array of shape
 *           [r_k][m_{k+1}][n_{k+1}][r_{k+1}] (0-based k, C row-major, last
 *           index fastest), i.e. G_{k+1}(a, i, j, b) at ((a*m + i)*n + j)*r + b.
 *   dtypes  OR of qtt_dtype_t: device copies to build.  Each core is stored
 *           as the matrix M_k(a_k + r_k i_k, a_{k-1} + r_{k-1} j_k) of
 *           Algorithm 2 (size r_k m_k x r_{k-1} n_k), rounded to nearest-even
 *           for FP32 and BF16, in the fragment order the kernels read.
 *   out     receives the handle.  The library owns it; free with
 *           qtt_matrix_free.  The host arrays are not retained. */
qtt_status_t qtt_matrix_load(int32_t d, const int64_t* ranks, const int64_t* m,
                             const int64_t* n, const double* const* cores,
                             uint32_t dtypes, qtt_matrix_t* out);

qtt_status_t qtt_matrix_free(qtt_matrix_t A);

/* Make A the non-translation-invariant operator of section 3 (the matrix
 * form of the Nystrom discretisation):
 *     A = a I + B K W C,   B = diag(b), W C = diag(wc),
 * with K the QTT matrix the handle was loaded with.  From then on every
 * apply through A (qtt_apply, qtt_apply_batched, and A or Ainv inside
 * qtt_solve and qtt_solve_fgmres) computes y = a x + b . K (wc . x): the
 * diagonals are elementwise passes before and after K's sweep, so the ranks
 * stay those of K (assembling the diagonals into the cores would multiply
 * them).
 *   b   host FP64, rows values, or NULL for ones; wc: host FP64, cols values
 *       (the products w_j c(y_j)), or NULL for ones.  Both are copied.
 *   a   needs rows == cols unless 0 (else QTT_ERR_SHAPE).
 * a = 0 with b = wc = NULL restores the plain K.  The workspace an apply
 * needs grows by (rows + cols) FP64 values per vector
 * (qtt_workspace_bytes reports it).  Not to be called while the handle is in
 * use on a stream.  QTT_ERR_INVALID_ARG for non-finite values,
 * QTT_ERR_OUT_OF_MEMORY if the copies cannot be allocated. */
qtt_status_t qtt_matrix_set_diagonals(qtt_matrix_t A, double a, const double* b, const double* wc);

/* Shape of a loaded matrix; any output pointer may be NULL. */
qtt_status_t qtt_matrix_info(qtt_matrix_t A, int32_t* d, int64_t* rows, int64_t* cols,
                             int64_t* max_rank, uint32_t* dtypes);

/* Ranks (d + 1 values) and row and column mode sizes (d values each) of a
 * loaded matrix; any output pointer may be NULL. */
qtt_status_t qtt_matrix_shape(qtt_matrix_t A, int64_t* ranks, int64_t* m, int64_t* n);

/* Device bytes of workspace that let qtt_apply / qtt_apply_batched run nrhs
 * vectors in one sweep: two ping-pong buffers of the largest intermediate
 * (r_k x prod_{l<=k} m_l x prod_{l>k} n_l values per vector, Algorithm 2's
 * y_k) in the compute dtype, plus alignment; for an operator with
 * diagonals (qtt_matrix_set_diagonals) also rows + cols FP64 values per
 * vector.  A smaller workspace (at least the value for nrhs = 1) makes the
 * library process the vectors in waves. */
qtt_status_t qtt_workspace_bytes(qtt_matrix_t A, qtt_dtype_t compute, int64_t nrhs,
                                 size_t* bytes);

/* Y = A X (Algorithm 2 on every column).
 *   X    device FP64, N x nrhs, column stride ldx >= N.
 *   Y    device FP64, M x nrhs, column stride ldy >= M; must not overlap X.
 *   ws   device workspace of ws_bytes (see qtt_workspace_bytes); the caller
 *        owns it and must not use it concurrently for another call.
 * nrhs = 0 is a no-op. */
qtt_status_t qtt_apply(qtt_matrix_t A, qtt_dtype_t compute, int64_t nrhs,
                       const double* X, int64_t ldx, double* Y, int64_t ldy,
                       void* ws, size_t ws_bytes, void* stream);

/* Uneven blocks: block b has widths[b] vectors at X[b] (stride ldx[b]) and
 * writes A X[b] to Y[b] (stride ldy[b]).  All blocks go through the same
 * sweep: each core is one persistent launch over the tiles of every vector
 * that fits the workspace.  Blocks of width 0 are skipped.  No Y[b] may
 * overlap any X[b']. */
qtt_status_t qtt_apply_batched(qtt_matrix_t A, qtt_dtype_t compute, int32_t nblocks,
                               const int64_t* widths, const double* const* X,
                               const int64_t* ldx, double* const* Y, const int64_t* ldy,
                               void* ws, size_t ws_bytes, void* stream);

/* qtt_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as qtt_apply, with the workspace taken from a
 * static 512 MiB device array that every GPU holds for the life of the
 * process.  The vectors run in waves that fit it.  Allocates nothing and
 * captures no graph; the caller passes only inputs and outputs.
 *   X, Y, ldx, ldy, nrhs as in qtt_apply; the handle's device must be current.
 * QTT_ERR_WORKSPACE when one vector needs more than 512 MiB of workspace
 * (qtt_workspace_bytes for nrhs = 1; e.g. an FP64 or FP32 sweep with a
 * 2^21-long intermediate of rank 32).  Nothing in the array needs to start
 * at zero.  All calls on one GPU share the array: calls that overlap on that
 * GPU (concurrent streams or host threads) race and give wrong results. */
qtt_status_t qtt_apply_noalloc(qtt_matrix_t A, qtt_dtype_t compute, int64_t nrhs,
                               const double* X, int64_t ldx, double* Y, int64_t ldy, void* stream);

/* Tune tile shapes for this matrix, dtype and vector count: every candidate
 * kernel configuration is timed on each core (outputs written to scratch in
 * ws), and the fastest is kept in the handle and in a process-wide table
 * keyed by (dtype, core shape).  For FP64 the whole sweep is then timed
 * core by core and with fused core pairs, and the
 * fastest of the three is kept.  X/Y are used as in qtt_apply and hold A X
 * on return.  Synchronises the stream. */
qtt_status_t qtt_autotune(qtt_matrix_t A, qtt_dtype_t compute, int64_t nrhs,
                          const double* X, int64_t ldx, double* Y, int64_t ldy,
                          void* ws, size_t ws_bytes, void* stream);

/* Pin the kernel configuration of one core for one compute dtype: shape is a
 * configuration id (as chosen by qtt_autotune), -1 restores the default
 * choice.  A configuration that cannot serve the core (wrong dtype, shape
 * restrictions, misaligned operands) falls back to the default at launch.
 * core = -2 (FP64, FP32) switches fused core pairs off (shape 0) or on
 * (shape 1): with pairs on, which is the default, two
 * consecutive cores k, k + 1 with r_k in 17..32 and m_k = n_{k+1} = 8, core
 * k + 1 not the last, run as one kernel that keeps the tile's intermediate
 * y_k on chip (Algorithm 2 applied two cores at a time).  Pinning a
 * configuration on a core (shape != -1) switches that dtype's pairs off, so that the
 * pinned configuration is the one that runs.  Returns QTT_ERR_INVALID_ARG
 * for an unknown id or core index.  Used by the tests to run every kernel
 * variant, and to replay a tuning result.
 *
 * Configuration 38 (QTT_FP32 only, interior cores; never chosen by default,
 * by qtt_autotune or listed by qtt_list_shapes) forms each FP32 product on
 * the BF16 matrix instruction from split operands: every FP32 core value and
 * input value v is written bf16(v) + bf16(v - bf16(v)) and the product
 * M b as M_hi b_hi + M_hi b_lo + M_lo b_hi with FP32 accumulation.  Cores,
 * intermediates and accumulation stay FP32; the error of each product term
 * is at most about 3 * 2^-16 of its size instead of 2^-24, for about a fifth of the
 * FP32 matrix-instruction time.  It serves cores with K_in <= 256,
 * K_in % 8 == 0, r_k m_k a multiple of 64 up to 256, r_k % 4 == 0 and
 * C_k % 32 == 0 (the handle builds the split copy at load for every FP32
 * core with K_in <= 256, K_in % 8 == 0); other cores keep the default. */
qtt_status_t qtt_set_shape(qtt_matrix_t A, qtt_dtype_t compute, int32_t core, int32_t shape);

/* Ids of the configurations available for a dtype (up to cap written to
 * ids); *count receives the total. */
qtt_status_t qtt_list_shapes(qtt_dtype_t compute, int32_t* ids, int32_t cap, int32_t* count);

typedef struct {
  int32_t iters;         /* passes of x += Ainv r done for this column */
  double rel_residual;   /* ||F_c - A x_c||_2 / ||F_c||_2 after the last pass */
} qtt_solve_col_t;

/* Device bytes of workspace for qtt_solve: the apply workspace for nrhs
 * vectors plus the N x nrhs FP64 residual and the norm buffers. */
qtt_status_t qtt_solve_workspace_bytes(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                       int64_t nrhs, size_t* bytes);

/* Solve A sigma = F with the compressed inverse and iterative refinement:
 * sigma = 0, r = F; repeat { sigma += Ainv r ; r = F - A sigma } until
 * ||r_c|| <= rtol ||F_c|| for every column, or max_iter passes.  The first
 * pass is the direct solve sigma = Ainv F of section 5.  A is applied in
 * FP64 (the residual, fused into its last core, stays FP64); Ainv is applied
 * in inv_compute (FP64, FP32 or BF16), and the update is accumulated in FP64.
 *   A, Ainv   square modes, identical mode sizes.
 *   F         device FP64, N x nrhs, stride ldf.  Sigma: device FP64, stride lds.
 *   info      host array of nrhs entries (may be NULL).
 * Synchronises the stream once per pass to read the nrhs residual norms.
 * Columns never mix, so a column whose F or residual norm is not finite
 * (NaN or Inf) is set aside (its info holds that norm; a column with a
 * non-finite F is not written) while the others are solved; the call then
 * returns QTT_ERR_NONFINITE.  Otherwise QTT_ERR_NOT_CONVERGED when a column is
 * above rtol after max_iter passes (Sigma holds the last iterate). */
qtt_status_t qtt_solve(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute, int64_t nrhs,
                       const double* F, int64_t ldf, double* Sigma, int64_t lds,
                       double rtol, int32_t max_iter, void* ws, size_t ws_bytes,
                       void* stream, qtt_solve_col_t* info);

/* The schedule of a refined solve (qtt_solve_schedule).  Refinement as
 * section 5 uses it fixes no precision per pass; each pass multiplies the
 * error by the contraction of its own inverse apply, so a cheaper apply
 * costs only its own factor, in the pass where it runs.
 *   inv_first, first_compute, first_passes
 *       passes 1 .. first_passes apply inv_first in first_compute, the later
 *       ones Ainv in inv_compute (first_passes = 0: inv_first is ignored and
 *       may be NULL).
 *   A_lo, lo_compute, lo_below
 *       a column that starts a pass with ||r_c|| <= lo_below ||F_c|| keeps
 *       its correction dx = Ainv r apart and updates its residual as
 *       r -= A_lo dx (A_lo applied in lo_compute, the update fused into
 *       A_lo's last core and accumulated in FP64) instead of recomputing
 *       r = F - A sigma with A in FP64.  The choice is made per column, so a
 *       column's arithmetic does not depend on the other columns of the
 *       call (in a pass, the columns of each route form their own sweeps of
 *       A or A_lo; the inverse sweep is shared).  The computed residual
 *       then differs from the true one by the error of A_lo's apply on dx,
 *       about u_lo ||A|| ||dx||, and ||dx|| is about ||Ainv|| lo_below ||F_c||:
 *       choose lo_below <= 0.01 rtol / u_lo (u_lo the relative error of one
 *       A_lo apply).  A_lo = NULL: every residual is recomputed in FP64.
 *       A_lo holds the same operator as A (same modes); the library does not
 *       check its values. */
typedef struct {
  qtt_matrix_t inv_first;
  qtt_dtype_t first_compute;
  int32_t first_passes;
  qtt_matrix_t A_lo;
  qtt_dtype_t lo_compute;
  double lo_below;
} qtt_schedule_t;

/* Device bytes of workspace for qtt_solve_schedule: qtt_solve's, with the
 * apply workspace of every handle the schedule names, plus an N x nrhs FP64
 * correction block when A_lo is given.  sched may be NULL (qtt_solve's). */
qtt_status_t qtt_solve_schedule_workspace_bytes(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                                const qtt_schedule_t* sched, int64_t nrhs, size_t* bytes);

/* qtt_solve with a schedule (qtt_schedule_t); sched = NULL, or one with
 * first_passes = 0 and A_lo = NULL, is qtt_solve with Ainv.  The stopping
 * rule, the column handling and the return values are those of qtt_solve;
 * info's rel_residual is the computed residual (updated with A_lo in the
 * passes that do so).  QTT_ERR_INVALID_ARG for first_passes < 0, a NULL
 * inv_first with first_passes > 0, or lo_below < 0 or not finite. */
qtt_status_t qtt_solve_schedule(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                const qtt_schedule_t* sched, int64_t nrhs, const double* F, int64_t ldf,
                                double* Sigma, int64_t lds, double rtol, int32_t max_iter, void* ws,
                                size_t ws_bytes, void* stream, qtt_solve_col_t* info);

/* Device bytes of workspace for qtt_solve_fgmres: max_iter + 1 Krylov blocks
 * V and, with a preconditioner, max_iter preconditioned blocks Z (each
 * N x nrhs FP64), small coefficient buffers, and the apply workspace.
 * Ainv may be NULL (no preconditioner; inv_compute is then ignored). */
qtt_status_t qtt_fgmres_workspace_bytes(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                        int64_t nrhs, int32_t max_iter, size_t* bytes);

/* Solve A sigma = F by unrestarted flexible GMRES with the compressed
 * inverse as right preconditioner, as section 5.3 uses GMRES (relative
 * residual tolerance, no restart) around the QTT approximate inverse.  Each
 * column c runs its own Krylov space; all active columns share every apply:
 *   z_j = Ainv v_j (inv_compute), w = A z_j (FP64), two passes of classical
 *   Gram-Schmidt against v_1..v_j, v_{j+1} = w / ||w||, Givens rotations on
 *   the host, and sigma_c = Z y once ||F_c - A sigma_c|| <= rtol ||F_c||.
 * The flexible form keeps the z_j, so a BF16 or FP32 inverse, linear only up
 * to rounding, is still exact in the minimised residual.  Ainv = NULL runs
 * plain GMRES (z_j = v_j).  A step costs one Ainv and one A apply, as a pass
 * of qtt_solve does; scaling Ainv changes no step.
 *   A, Ainv   square modes, identical mode sizes.
 *   F, Sigma  device FP64, N x nrhs, strides ldf and lds (no overlap).
 *   info      host, nrhs entries or NULL: steps taken and the residual
 *             estimate |g_{k+1}| / ||F_c|| of the rotated Hessenberg system,
 *             which equals the true relative residual up to FP64 rounding of
 *             the Arnoldi relation (A applied in FP64).
 * A zero column of F gives a zero column of Sigma in no steps; a column of F
 * that is not finite is skipped (not written, its info holds the norm) while
 * the others are solved, and the call returns QTT_ERR_NONFINITE.
 * Synchronises the stream once per step.  Returns QTT_ERR_NOT_CONVERGED
 * after max_iter steps (Sigma holds each column's minimal-residual iterate),
 * QTT_ERR_NONFINITE for a non-finite norm or a singular Hessenberg matrix,
 * QTT_ERR_WORKSPACE below qtt_fgmres_workspace_bytes' fixed part plus the
 * one-vector apply workspace. */
qtt_status_t qtt_solve_fgmres(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute, int64_t nrhs,
                              const double* F, int64_t ldf, double* Sigma, int64_t lds,
                              double rtol, int32_t max_iter, void* ws, size_t ws_bytes,
                              void* stream, qtt_solve_col_t* info);

/* qtt_solve_fgmres with a schedule (qtt_schedule_t).  Steps 1 ..
 * first_passes are preconditioned with inv_first in first_compute (the
 * flexible method allows a different preconditioner per step; needs Ainv),
 * and a column whose residual estimate before a step is at or below
 * lo_below forms that step's w = A_lo z_j (lo_compute) instead of A z_j in
 * FP64, decided per column.  Step j's basis vector enters the solution with
 * a weight about the residual before the step, so the true residual moves
 * by about u_lo ||A|| times that residual: choose lo_below <= 0.01 rtol /
 * u_lo.  info holds the residual estimates of the rotations.  sched = NULL
 * is qtt_solve_fgmres. */
qtt_status_t qtt_fgmres_schedule_workspace_bytes(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                                 const qtt_schedule_t* sched, int64_t nrhs, int32_t max_iter,
                                                 size_t* bytes);
qtt_status_t qtt_solve_fgmres_schedule(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                       const qtt_schedule_t* sched, int64_t nrhs, const double* F, int64_t ldf,
                                       double* Sigma, int64_t lds, double rtol, int32_t max_iter, void* ws,
                                       size_t ws_bytes, void* stream, qtt_solve_col_t* info);

/* Compressed matrix-vector product (section 4.2): for vectors b given in
 * TT form, the cores of c = A b,
 *   c_k(alpha + rA_{k-1} beta, i, alpha' + rA_k beta')
 *       = sum_j G_k(alpha, i, j, alpha') b_k(beta, j, beta'),
 * for nvec vectors that share the TT ranks rb.  The ranks of c are
 * rA_k rb_k; nothing is rounded.
 *   rb   host, d + 1 ranks, rb[0] = rb[d] = 1.
 *   B    d device pointers; B[k] holds nvec FP64 cores of rb[k] x n_k x
 *        rb[k+1] values each, vector v's at B[k] + v rb[k] n_k rb[k+1], C
 *        row-major [beta][j][beta'].
 *   C    d device pointers; C[k] receives nvec cores of (rA_k rb[k]) x m_k x
 *        (rA_{k+1} rb[k+1]) values, row-major [beta][alpha][i][beta'][alpha']
 *        (the merged index alpha + rA beta, matrix rank fastest).
 * Needs A's FP64 copy (QTT_ERR_DTYPE otherwise) and no diagonals
 * (QTT_ERR_INVALID_ARG).  Output cores must not overlap each other or the
 * input cores.  Asynchronous on the stream; allocates nothing. */
qtt_status_t qtt_matvec_compressed(qtt_matrix_t A, int64_t nvec, const int64_t* rb,
                                   const double* const* B, double* const* C, void* stream);

/* qtt_solve_fgmres with section 4.1's product-form preconditioner: the compressed
 * inverse is the product of two QTT matrices, Ainv = M Y (the inversion
 * solves A M Y = I for Y with an easily inverted M), applied as two chained
 * sweeps, z_j = M (Y v_j), both in inv_compute.  Y v_j is staged in the slot
 * of v_{j+1}, so no memory is added: the workspace is the larger of
 * qtt_fgmres_workspace_bytes for M and for Y.  M and Y must both be given
 * (QTT_ERR_INVALID_ARG otherwise); everything else as qtt_solve_fgmres. */
qtt_status_t qtt_solve_fgmres_product(qtt_matrix_t A, qtt_matrix_t M, qtt_matrix_t Y, qtt_dtype_t inv_compute,
                                      int64_t nrhs, const double* F, int64_t ldf, double* Sigma, int64_t lds,
                                      double rtol, int32_t max_iter, void* ws, size_t ws_bytes,
                                      void* stream, qtt_solve_col_t* info);

/* ------------------------------------------------------------------------
 * Tensors in TT form.  A TT tensor (eq. TTdeccores, section 2.2) with d cores
 * has ranks r_0..r_d (r_0 = r_d = 1) and modes n_1..n_d; core k is a device
 * FP64 array [r_{k-1}][n_k][r_k], C row-major, and the entries, first index
 * fastest (section 2.1), are
 *     c(i_1, ..., i_d) = G_1(:, i_1, :) G_2(:, i_2, :) ... G_d(:, i_d, :).
 * A QTT matrix core [r][m][n][r'] is the TT core of mode m n (j fastest).
 * These calls allocate device scratch of their own and synchronise the
 * stream before returning (ranks are decided on the host).
 * ------------------------------------------------------------------------ */

/* TT rounding: the TT decomposition that Algorithm 1 (section 2.3: truncated
 * SVDs of the unfoldings, each to accuracy eps ||c||_F / sqrt(d - 1), so the
 * result c' has ||c - c'||_F <= eps ||c||_F up to the sketch's error) gives
 * for the tensor c that the input cores represent, computed from the cores:
 * a randomized range finder with Gaussian sketch cores (Philox4x32-10
 * normals from seed), then a right-to-left truncation with the rank rule of
 * Algorithm 1.  The sketch rank grows from 32 up to max_rank (1..128) while a
 * kept rank comes within an eighth of it.
 *   ranks, n     the input's ranks (d + 1) and modes (d), host arrays.
 *   cores        d device pointers to the input cores (not modified).
 *   out          d device pointers; out[k] must hold
 *                min(max_rank, ranks[k]) n_k min(max_rank, ranks[k+1]) values.
 *   out_ranks    host, d + 1 values: the ranks of the result.
 * The result's cores 2..d have orthonormal rows (as r_{k-1} x n_k r_k
 * matrices); core 1 carries the norm.  QTT_ERR_RANK when max_rank was
 * reached while the tolerance asked for more (the result is then the best
 * found at max_rank). */
qtt_status_t qtt_tt_round(int32_t d, const int64_t* n, const int64_t* ranks, const double* const* cores,
                          double eps, int32_t max_rank, uint64_t seed, double* const* out, int64_t* out_ranks,
                          void* stream);

/* Compression of a full vector x (device FP64, prod n_k values, first digit
 * fastest) into TT form to relative accuracy eps: Algorithm 1 with a
 * randomized low-rank routine (Gaussian sketch of each unfolding's columns,
 * thin QR), then the same truncation as qtt_tt_round.  The "compress" step of
 * section 5.2's "QTT solve".  out / out_ranks as in qtt_tt_round. */
qtt_status_t qtt_tt_compress(int32_t d, const int64_t* n, const double* x, double eps, int32_t max_rank,
                             uint64_t seed, double* const* out, int64_t* out_ranks, void* stream);

/* Read back the FP64 cores of a handle (as loaded): host_cores[k] receives
 * r_{k-1} m_k n_k r_k values, [r_{k-1}][m_k][n_k][r_k].  QTT_ERR_DTYPE when
 * the handle has no FP64 copy.  Synchronous. */
qtt_status_t qtt_matrix_cores(qtt_matrix_t A, double* const* host_cores);

/* QTT inversion by the Newton-Hotelling-Schulz iteration (named in section 1.3
 * among the QTT inversion methods): from X_0 (the handle X0), repeat
 *     R_t = round(I - round(A X_t)),   X_{t+1} = round(X_t round(I + R_t)),
 * every product in QTT form (ranks multiply) and every round a qtt_tt_round
 * to relative accuracy eps with ranks up to max_rank, except R_t's, whose
 * accuracy is eps ||I||_F (the scale of X's error, not R_t's own norm).
 * I - A X_{t+1} =
 * (I - A X_t)^2 before rounding, so the residual squares each step once
 * ||I - A X_0|| < 1.  theta > 0 rounds I + R_t and X_{t+1} to accuracy
 * max(eps, theta h_t^2), h_t = ||R_t||_F / ||I||_F (X_{t+1} is within about
 * h_t^2 of the inverse; early iterates then keep the ranks the inverse
 * needs, not the higher ones a tight eps would give them); theta = 0 rounds
 * everything at eps.  Stops when h_t <= tol or after max_iter steps.  A and X0 need FP64 copies and square, identical modes.
 *   Xinv     receives a new handle with device copies in dtypes (free it
 *            with qtt_matrix_free).
 *   history  host, max_iter + 1 values or NULL: ||R_t||_F / ||I||_F.
 *   steps    host or NULL: the number of updates done.
 * QTT_ERR_RANK if some rounding hit max_rank (Xinv is still returned). */
qtt_status_t qtt_invert_newton_schulz(qtt_matrix_t A, qtt_matrix_t X0, double eps, int32_t max_rank,
                                      int32_t max_iter, double tol, double theta, uint64_t seed, uint32_t dtypes,
                                      qtt_matrix_t* Xinv, double* history, int32_t* steps, void* stream);

const char* qtt_status_string(qtt_status_t s);
const char* qtt_last_error(void);

/* Per-launch device timing of the core-step kernels, for roofline figures.
 * When enabled, every core-step launch on the calling thread is bracketed by
 * HIP events recorded on the stream it is launched on.  qtt_timing_read
 * synchronises on the recorded events and reports, for one compute dtype
 * and one core position (0 = interior cores, 1 = first core, 2 = last core,
 * 3 = single-core matrices), the number of launches, their summed device
 * time, and their summed algorithmic flops (2 x rows x cols x columns of
 * each core's product) and bytes (input read once, output written once).
 * qtt_timing_reset drops what was recorded. */
qtt_status_t qtt_timing_enable(int32_t on);
qtt_status_t qtt_timing_reset(void);
qtt_status_t qtt_timing_read(qtt_dtype_t compute, int32_t position, int64_t* launches,
                             double* milliseconds, double* flops, double* bytes);
/* The same sums over the launches of one kernel configuration id (any core
 * position); ids as in qtt_list_shapes, plus 90..97 (FP64) and 100..107
 * (FP32) for the kernels that apply two consecutive cores k, k + 1 in one
 * launch: base + 4 (k is the first core) + 2 (r_k other than 24: the
 * 256-row kernel, exact at r_k = 32, padded for the other ranks in 17..32)
 * + (R_out of core k + 1 above 192).
 * Such a launch is recorded at the position of core k, with the flops of
 * both cores.  Launches of a configuration id that was never timed give
 * zeros. */
qtt_status_t qtt_timing_read_shape(qtt_dtype_t compute, int32_t shape, int64_t* launches,
                                   double* milliseconds, double* flops, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* QTT_H */
