/*
 * libdopinf: the data-parallel hot path of distributed Operator Inference
 * (dOpInf, arXiv:2504.14338) on one AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers without an `_h` suffix are DEVICE pointers; `_h` marks host
 *    arrays.  All matrices are row-major with an explicit leading dimension.
 *  - The caller owns every buffer and the stream (`stream` is a hipStream_t
 *    passed as void*; NULL means the default stream).  The library never
 *    allocates or frees device memory: scratch comes from a caller-provided
 *    workspace `ws` of at least the size returned by the matching
 *    `*_workspace` query, aligned to 256 bytes (a misaligned workspace
 *    returns DOPINF_E_WORKSPACE with nothing enqueued).
 *  - Calls only enqueue work on `stream` and return; they do not synchronize
 *    unless documented (dopinf_reduce with r_req == 0).  Separate streams may
 *    be used concurrently with separate workspaces.
 *  - Every call returns a status.  Argument errors return immediately with
 *    nothing enqueued; the message is available from dopinf_last_error()
 *    (thread-local).  Data-dependent conditions (non-finite data, a
 *    non-positive Cholesky pivot, ...) are reported through device-side
 *    status words that the caller reads after its own synchronization.
 *
 * Notation (paper): Q is n x k (rows: degrees of freedom, columns: the k
 * snapshots), each state variable a contiguous block of rows; r reduced
 * dimension; s = r(r+1)/2 quadratic terms; d = r + s + 1 operator columns.
 */
#ifndef DOPINF_H
#define DOPINF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------- */
#define DOPINF_OK 0
#define DOPINF_E_ARG 1         /* invalid argument; nothing enqueued          */
#define DOPINF_E_HIP 2         /* a HIP runtime call or launch failed         */
#define DOPINF_E_WORKSPACE 3   /* workspace missing, too small or not 256-byte aligned */
#define DOPINF_E_RANK 4        /* lambda_r <= 0 or r > k                       */
#define DOPINF_E_NOTSPD 5      /* non-positive Cholesky pivot                  */
#define DOPINF_E_NONFINITE 6   /* NaN/Inf in data or results                   */
#define DOPINF_E_NOSTABLE 7    /* no candidate passes the growth bound         */
#define DOPINF_E_TIMEOUT 8     /* a device-wide barrier exceeded its spin cap  */

/* ---- element types and options -------------------------------------------- */
#define DOPINF_F64 0
#define DOPINF_F32 1

#define DOPINF_CENTER 1u  /* subtract each row's temporal mean                */
#define DOPINF_SCALE 2u   /* divide each variable by its max |centered value|  */
#define DOPINF_APPLY 4u   /* also overwrite Q with the transformed data        */

#define DOPINF_GRAM_NATIVE 0  /* MFMA in the storage type (F64 or F32)       */
#define DOPINF_GRAM_BF16X3 1  /* F32 data, split hi+lo bfloat16, 3 products  */
#define DOPINF_GRAM_BF16X6 2  /* F32 data, split hi+mid+lo bfloat16, 6 products */
#define DOPINF_GRAM_I8X6 3    /* F32 data, three int8 fixed-point slices, 6 products */

#define DOPINF_MAX_VARS 64

/* Per-candidate outcome written by dopinf_rollout. */
#define DOPINF_ITEM_PASS 0        /* finite and growth < max_growth            */
#define DOPINF_ITEM_NONFINITE 1   /* the rollout produced NaN/Inf              */
#define DOPINF_ITEM_GROWTH 2      /* growth >= max_growth                      */
#define DOPINF_ITEM_SOLVE 3       /* the regularized solve failed (not SPD)    */
#define DOPINF_ITEM_TIMEOUT 4     /* a multi-workgroup rollout gave up waiting */

#define DOPINF_ROLLOUT_FULL 1u    /* no early exit: run every state            */
#define DOPINF_ROLLOUT_ONE_WG 2u  /* one workgroup per item even for few items */

const char* dopinf_last_error(void);
const char* dopinf_version(void);

/* ---- Step II: centering and scaling (Sec. 3.3) -----------------------------
 * mean[i]  = (1/k) sum_t Q[i,t]                       (per row, if CENTER)
 * scale[v] = max over rows i of variable v and all t of |Q[i,t] - mean[i]|
 *            (if SCALE; 1 otherwise, and 1 with zero_range[v] = 1 when the
 *            variable is constant).
 * With APPLY, Q[i,t] <- (Q[i,t] - mean[i]) / scale[v] in place.
 * Q: n x k, leading dimension ldq >= k, element type `dtype`; statistics are
 * accumulated in double.  var_rows_h[0..nvars]: host array, var_rows_h[0] = 0,
 * strictly increasing, var_rows_h[nvars] = n; nvars <= DOPINF_MAX_VARS.
 * mean: n doubles; scale: nvars doubles; zero_range: nvars ints or NULL.
 * info (device int, may be NULL): DOPINF_OK, or DOPINF_E_NONFINITE when Q
 * holds a NaN or an infinity; then the means of the rows concerned are not
 * finite, the scale of each variable concerned is NaN (with SCALE; 1
 * without), and its zero_range entry is 0. */
size_t dopinf_preprocess_workspace(int64_t n, int64_t k, int nvars);
int dopinf_preprocess(void* stream, int dtype, void* Q, int64_t n, int64_t k,
                      int64_t ldq, int nvars, const int64_t* var_rows_h,
                      unsigned flags, double* mean, double* scale,
                      int* zero_range, int* info, void* ws, size_t ws_bytes);

/* ---- Step II: lifting transformations (Sec. 3.3) ---------------------------
 * New variables that expose polynomial structure, formed point by point
 * before centering.  Q holds nvars_in input variables as consecutive blocks
 * of n_cells rows (row = one cell, k snapshots, ldq >= k).  spec_h (host,
 * 3 n_out ints) lists the output variables in order as (op, a, b):
 *   DOPINF_LIFT_COPY        L_j = Q_a
 *   DOPINF_LIFT_PRODUCT     L_j = Q_a * Q_b   (elementwise)
 *   DOPINF_LIFT_RECIPROCAL  L_j = 1 / Q_a     (IEEE: 1/0 = Inf)
 * L: n_out blocks of n_cells rows (ldl >= k), written; must not overlap Q.
 * n_out <= DOPINF_MAX_VARS; a, b in [0, nvars_in) (b read for PRODUCT only). */
#define DOPINF_LIFT_COPY 0
#define DOPINF_LIFT_PRODUCT 1
#define DOPINF_LIFT_RECIPROCAL 2
int dopinf_lift(void* stream, const double* Q, int64_t n_cells, int64_t k,
                int64_t ldq, int nvars_in, int n_out, const int* spec_h,
                double* L, int64_t ldl);

/* ---- Step III: Gram matrix D = Qs^T Qs (Eq. (5)) ---------------------------
 * Qs[i,t] = (Q[i,t] - mean[i]) * (1 / scale[v(i)]) formed on load when mean
 * and scale are given (either may be NULL: no centering / no scaling).
 * D: k x k doubles, leading dimension ldd >= k, written in full (symmetric).
 * algo: DOPINF_GRAM_NATIVE (F64: FP64 MFMA; F32: FP32 MFMA),
 * DOPINF_GRAM_BF16X3, DOPINF_GRAM_BF16X6 or DOPINF_GRAM_I8X6 (F32 data
 * only).  The bfloat16 forms first pack the transformed data (rounded to
 * float32, split into bfloat16 parts) into the workspace, then accumulate in
 * float over row slabs of at most 512 rows and sum slabs in double.
 * DOPINF_GRAM_I8X6 scales column j of the transformed data (in double) by
 * 127 / a_j with a_j its max-abs, splits it into three int8 slices of radix
 * 254 and sums six slice products exactly in int32 on the int8 matrix cores;
 * the error per entry is |dD_jl| <= 2.5e-7 a_j a_l per row of Q, and a
 * non-finite input value makes its column's entries of D NaN.
 * Deterministic: no floating-point atomics; repeated calls give identical
 * bits. */
size_t dopinf_gram_workspace(int dtype, int algo, int64_t n, int64_t k);
int dopinf_gram(void* stream, int dtype, int algo, const void* Q, int64_t n,
                int64_t k, int64_t ldq, const double* mean, const double* scale,
                int nvars, const int64_t* var_rows_h, double* D, int64_t ldd,
                void* ws, size_t ws_bytes);

/* Cross Gram C = X^T Y (the same kernel, no triangle symmetry): X is n x mx,
 * Y is n x my (float64, leading dimensions ldx, ldy), C is mx x my (ldc).
 * With mean / scale (each may be NULL; var_rows_h as above when scale is
 * given) both operands are transformed on load with the SAME per-row mean and
 * per-variable scale, e.g. held-out snapshots centered and scaled with the
 * training statistics, so that T_r^T (Qs^T Qs_test) projects them onto the
 * reduced coordinates through Eq. (8) without forming the basis. */
size_t dopinf_cross_gram_workspace(int64_t n, int64_t mx, int64_t my);
int dopinf_cross_gram(void* stream, const double* X, int64_t ldx,
                      const double* Y, int64_t ldy, int64_t n, int64_t mx,
                      int64_t my, const double* mean, const double* scale,
                      int nvars, const int64_t* var_rows_h, double* C,
                      int64_t ldc, void* ws, size_t ws_bytes);

/* ---- Out-of-core statistics and Gram (Sec. 3.2 loading; Eq. (5)) ---------
 * For snapshot matrices larger than device memory: Q_h is a HOST array
 * (n x k, ldq), read in chunks of chunk_rows rows through two device
 * staging buffers; the copy of the next chunk (on a stream of the library's,
 * created and released per call) overlaps the kernels of the current one
 * (on `stream`).  Pinned host memory (hipHostMalloc) is needed for that
 * overlap; pageable memory works, with synchronous copies.  Results are
 * those of dopinf_preprocess / dopinf_gram on the whole matrix: per-row
 * means are computed row by row, per-variable maxima combine by max, and
 * the Gram matrix is the sum of the chunks' Gram matrices (Eq. (5)), added
 * in chunk order (deterministic; summation order differs from the one-shot
 * dopinf_gram by the chunking).  Workspace: dopinf_stream_workspace(
 * chunk_rows, k, nvars) bytes (two chunks, a k x k partial and the chunk
 * kernels' scratch).  Q_h must stay valid and unchanged until the work on
 * `stream` has finished.
 * dopinf_preprocess_stream: flags CENTER and SCALE (no APPLY); mean, scale,
 *   zero_range, info as for dopinf_preprocess.
 * dopinf_gram_stream: float64 data; mean / scale as for dopinf_gram. */
size_t dopinf_stream_workspace(int64_t chunk_rows, int64_t k, int nvars);
int dopinf_preprocess_stream(void* stream, const double* Q_h, int64_t n,
                             int64_t k, int64_t ldq, int nvars,
                             const int64_t* var_rows_h, unsigned flags,
                             double* mean, double* scale, int* zero_range,
                             int* info, int64_t chunk_rows, void* ws,
                             size_t ws_bytes);
int dopinf_gram_stream(void* stream, const double* Q_h, int64_t n, int64_t k,
                       int64_t ldq, const double* mean, const double* scale,
                       int nvars, const int64_t* var_rows_h, double* D,
                       int64_t ldd, int64_t chunk_rows, void* ws,
                       size_t ws_bytes);

/* ---- Step III: eigenpairs and basis-free reduced data (Eqs. (6)-(9)) ------
 * D (k x k, symmetric, ldd) is read, not modified.
 * lambda[0..k): all eigenvalues of D in descending order.
 * Qhat: r x k (ldqh >= k) = Lambda_r^{1/2} U_r^T, i.e. T_r^T D (Eq. (8));
 * Tr (NULL or k x r, ldtr >= r) = U_r Lambda_r^{-1/2}.
 * Each eigenvector u_j is signed so that its largest-magnitude entry is
 * positive (lowest index on a tie); when the two largest magnitudes agree
 * to 1e-8 relative with opposite signs, the sign of sum_t (t+1) u_t decides.
 * r_req > 0: r = r_req (no host synchronization).  r_req == 0: r is the
 * smallest value whose retained energy (Eq. (9)) exceeds tau; the call then
 * synchronizes `stream`.  r must be <= r_max (capacity of Qhat / Tr).
 * r_out_h (host, may be NULL) receives r.  info (device int) receives
 * DOPINF_OK, DOPINF_E_RANK (lambda_r <= k * 2^-52 * lambda_1, i.e. numerically
 * zero), DOPINF_E_NONFINITE or
 * DOPINF_E_TIMEOUT. */
size_t dopinf_reduce_workspace(int64_t k, int r_max);
int dopinf_reduce(void* stream, const double* D, int64_t k, int64_t ldd,
                  int r_req, double tau, int r_max, int* r_out_h,
                  double* lambda, double* Tr, int64_t ldtr, double* Qhat,
                  int64_t ldqh, int* info, void* ws, size_t ws_bytes);

/* Partial eigendecomposition for a prescribed r (Sec. 3.4: only the r
 * leading eigenpairs enter Eqs. (7)-(8)).  Same outputs as dopinf_reduce with
 * r_req = r (same sign rule, Qhat = Lambda_r^{1/2} U_r^T, T_r), except that
 * lambda receives only the r leading eigenvalues.  Method: block subspace
 * iteration on a block of p = min(128, max(r + 16, 2 r) rounded up to 16)
 * vectors with shifted Cholesky QR, and Rayleigh-Ritz steps solved by the
 * dense eigensolver; the iteration count comes from the Ritz values of a
 * first Rayleigh-Ritz step (theta_p / theta_r)^m <= 1e-17, so the call
 * synchronizes `stream` once.  When r does not fit the block (r > 120, or
 * k < 64) or the spectrum decays too slowly (more than 80 iterations), the
 * full eigensolver of dopinf_reduce runs instead.
 * iters_h (host, may be NULL): subspace iterations used, 0 when the full
 * eigensolver ran.  info: as for dopinf_reduce. */
size_t dopinf_reduce_topr_workspace(int64_t k, int r);
int dopinf_reduce_topr(void* stream, const double* D, int64_t k, int64_t ldd,
                       int r, double* lambda, double* Tr, int64_t ldtr,
                       double* Qhat, int64_t ldqh, int* info, int* iters_h,
                       void* ws, size_t ws_bytes);

/* ---- Step IV: regularized operator inference (Eqs. (11)-(13)) ------------
 * For every reduced size r_g in r_list_h[0..n_r) (group g uses the first r_g
 * rows of Qhat, r x k, ldqh) and every pair p in [0, n_pairs):
 *   Dhat = [Qhat_1^T | quad(Qhat_1^T) | 1],  Qhat_1 = Qhat[:, 0:k-1],
 *   Qhat_2 = Qhat[:, 1:k], quad() the non-redundant products in the order
 *   (0,0),(0,1),...,(0,r-1),(1,1),...,
 *   (Dhat^T Dhat + diag(beta1_h[p] x r, beta2_h[p] x s, beta1_h[p])) O^T
 *     = Dhat^T Qhat_2^T,
 * solved by Cholesky.  O = [A | H | c] (r_g x d_g, row-major) is stored at
 * O + dopinf_operator_offset(n_r, r_list_h, n_pairs, g*n_pairs + p):
 * groups in r_list order, pairs inside a group in the given order.
 * status[item] (device ints, n_r * n_pairs) = DOPINF_OK or DOPINF_E_NOTSPD.
 * r_g >= 1, k >= 2, n_pairs >= 1.
 * With several reduced sizes the groups run concurrently on internal streams
 * of the calling host thread (at most GPU_MAX_HW_QUEUES - 1 of them, 4 - 1
 * when unset; the largest groups get one each), forked from `stream` after
 * the shared data Gram and joined back before the call's work ends on
 * `stream`; the results do not depend on the fork.  Under stream capture
 * the fork becomes parallel graph branches. */
size_t dopinf_operator_offset(int n_r, const int* r_list_h, int n_pairs,
                              int item);
size_t dopinf_infer_workspace(int64_t k, int n_r, const int* r_list_h,
                              int n_pairs);
int dopinf_infer(void* stream, const double* Qhat, int64_t ldqh, int64_t k,
                 int n_r, const int* r_list_h, int n_pairs,
                 const double* beta1_h, const double* beta2_h, double* O,
                 int* status, void* ws, size_t ws_bytes);

/* ---- Step IV: ROM rollouts, scoring and selection (Sec. 3.5) -------------
 * For every item of dopinf_infer's layout: qt_0 = Qhat[0:r_g, 0] (or, when
 * q0 is not NULL, the item's r_g entries of q0: device float64, the items'
 * initial states packed in item order, item i at dopinf_traj_offset(n_r,
 * r_list_h, n_pairs, 1, i)),
 * qt_{t+1} = A qt_t + H quad(qt_t) + c for n_states states (qt_0 included).
 * train_err[item] = max_{t < min(k_train, n_states)} ||qt_t - qhat_t|| / ||qhat_t||;
 * growth[item]    = max_{t,i} |qt_t[i] - m_i| / max_{t<k_train,i} |qhat_t[i] - m_i|
 *                   with m the temporal mean of Qhat[0:r_g, 0:k_train];
 * outcome[item]   = DOPINF_ITEM_*: pass iff every state is finite and
 *                   growth < max_growth.  Without DOPINF_ROLLOUT_FULL a
 *                   rollout stops as soon as its outcome is decided to be a
 *                   failure (selection is unchanged; train_err/growth then
 *                   hold the values reached so far).
 * solve_status (NULL or dopinf_infer's status): items with a failed solve
 * are not rolled out (outcome DOPINF_ITEM_SOLVE).
 * Few items (n_r * n_pairs small) are rolled out by teams of workgroups that
 * keep the operator rows on chip and exchange the state every step; a team
 * whose exchange does not complete within seconds gives up with outcome
 * DOPINF_ITEM_TIMEOUT (and train_err = growth = NaN).  Many items are
 * rolled out one workgroup per item (a persistent grid of resident
 * workgroups taking items from a device counter when there are more items
 * than resident workgroups), the operator streamed from memory every step.
 * DOPINF_ROLLOUT_ONE_WG forces the one-workgroup form.
 * best[g] (device ints, n_r): item index (within the whole layout) of the
 * smallest train_err among passing items of group g, the first in layout
 * order on ties, -1 if none passes.
 * traj (NULL or n_states x r_g per item at
 * dopinf_traj_offset(n_r, r_list_h, n_pairs, n_states, item)): the states,
 * time-major; states after an early exit are NaN. */
size_t dopinf_traj_offset(int n_r, const int* r_list_h, int n_pairs,
                          int n_states, int item);
size_t dopinf_rollout_workspace(int n_r, const int* r_list_h, int n_pairs,
                                int64_t k_train);
int dopinf_rollout(void* stream, int n_r, const int* r_list_h, int n_pairs,
                   const double* O, const double* Qhat, int64_t ldqh,
                   const double* q0, int64_t k_train, int n_states, double max_growth,
                   unsigned flags, const int* solve_status, double* traj,
                   double* train_err, double* growth, int* outcome, int* best,
                   void* ws, size_t ws_bytes);

/* ---- Step V: postprocessing of the reduced solution (Sec. 3.6) ------------
 * The reduced solution Qtilde (r x n_out, ldqt) mapped back to the original
 * coordinates at m selected rows, with the basis formed only at those rows
 * (Eq. (7) with the method of snapshots, V_r = Qs T_r):
 *   V[i, :]    = Qs[rows[i], :] T_r,  Qs = (Q - mean 1^T) / scale_v (Step II;
 *                mean / scale may be NULL: no centering / no scaling)
 *   pred[i, t] = scale_v(rows[i]) (V[i, :] Qtilde[:, t]) + mean[rows[i]]
 * Q: n x k (ldq), element type dtype (F64 or F32; arithmetic in double).
 * rows: device array of m row indices, or NULL for rows 0 .. m-1 (m <= n).
 * Tr: k x r (ldtr), as written by dopinf_reduce.  V: m x r (ldv), written.
 * pred: NULL (basis rows only) or m x n_out (ldp).  var_rows_h as for
 * dopinf_preprocess (read only when scale is given).
 * info (device int, may be NULL): DOPINF_OK, or DOPINF_E_ARG when a row
 * index lies outside [0, n) (those rows of V and pred are NaN).
 * No workspace; nothing is allocated. */
int dopinf_postprocess(void* stream, int dtype, const void* Q, int64_t n,
                       int64_t k, int64_t ldq, const double* mean,
                       const double* scale, int nvars,
                       const int64_t* var_rows_h, const int64_t* rows,
                       int64_t m, const double* Tr, int64_t ldtr, int r,
                       const double* Qtilde, int64_t ldqt, int64_t n_out,
                       double* V, int64_t ldv, double* pred, int64_t ldp,
                       int* info);

/* ---- Allocation-free rollout ---------------------------------------------
 * For callers that cannot allocate device memory or bring a workspace: code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc.  dopinf_rollout_noalloc takes the arguments and gives the
 * results of dopinf_rollout (the same kernels), but its scratch is a fixed
 * array in the library's device memory, one copy per GPU, held until the
 * process ends: dopinf_rollout_noalloc_max_bytes() bytes (4 MiB).  A call
 * whose dopinf_rollout_workspace size exceeds that returns
 * DOPINF_E_WORKSPACE with nothing enqueued.  The call allocates nothing and
 * calls no allocating routine; the first call with a device current looks up
 * that device's copy of the array.  Every call on one GPU uses the same
 * array, whatever its stream: calls that overlap on one GPU (concurrent
 * streams, or host threads) race and give undefined results; order them on
 * one stream or with events. */
size_t dopinf_rollout_noalloc_max_bytes(void);
int dopinf_rollout_noalloc(void* stream, int n_r, const int* r_list_h,
                           int n_pairs, const double* O, const double* Qhat,
                           int64_t ldqh, int64_t k_train, int n_states,
                           double max_growth, unsigned flags,
                           const int* solve_status, double* traj,
                           double* train_err, double* growth, int* outcome,
                           int* best);

/* ---- Continuous-time variant (Sec. 3.5, Eq. (10)) -------------------------
 * dq/dt = A q + H quad(q) + c inferred from the same reduced data: the data
 * matrix uses all k snapshots, Dhat = [Qhat^T | quad(Qhat^T) | 1] (k x d),
 * and the right-hand side is the time derivative of Qhat by second-order
 * finite differences at snapshot spacing dt (central inside, one-sided
 * three-point at both ends; k >= 3).  Regularizer, solver, layout of O and
 * status as for dopinf_infer.
 * dopinf_rollout_continuous: as dopinf_rollout, with state t+1 one classical
 * fourth-order Runge-Kutta step of size dt from state t (state t is scored
 * against snapshot t); teams of workgroups (one exchange per stage, four per
 * step) while a group's teams fit one workgroup per CU, else one workgroup
 * per candidate; flags, time-out and workspace query as for
 * dopinf_rollout. */
size_t dopinf_infer_continuous_workspace(int64_t k, int n_r,
                                         const int* r_list_h, int n_pairs);
int dopinf_infer_continuous(void* stream, const double* Qhat, int64_t ldqh,
                            int64_t k, double dt, int n_r,
                            const int* r_list_h, int n_pairs,
                            const double* beta1_h, const double* beta2_h,
                            double* O, int* status, void* ws,
                            size_t ws_bytes);
int dopinf_rollout_continuous(void* stream, int n_r, const int* r_list_h,
                              int n_pairs, const double* O,
                              const double* Qhat, int64_t ldqh,
                              int64_t k_train, int n_states, double dt,
                              double max_growth, unsigned flags,
                              const int* solve_status, double* traj,
                              double* train_err, double* growth,
                              int* outcome, int* best, void* ws,
                              size_t ws_bytes);

/* ---- Tuned launch parameters and the autotuner (batched form) ------------
 * The regularization sweep of Sec. 3.5 (every (r, beta1, beta2) of a grid)
 * factors G_qq + beta2 I (s x s, s = r(r+1)/2) once per distinct beta2 with
 * a blocked Cholesky, and solves triangular systems with that factor; both
 * are blocked in block columns whose width is a launch parameter: wider
 * blocks read the trailing matrix or the right-hand sides fewer times,
 * narrower ones start the trailing work sooner.  An optional inner width
 * (a divisor of the outer one) blocks each block column once more: its
 * 64-wide panels then update only their inner block, and the block column
 * takes updates of the inner depth.  A process-wide table holds the widths
 * per s (untuned sizes use 256 and no inner width):
 *   DOPINF_TUNE_CHOL_KB   the Cholesky's block-column width,
 *   DOPINF_TUNE_TRSM_KB   the triangular solves' block-column depth,
 *   DOPINF_TUNE_CHOL_KB2  the Cholesky's inner width (0: none),
 *   DOPINF_TUNE_TRSM_KB2  the triangular solves' inner depth (0: none).
 * An inner width that is not smaller than the outer one or does not divide
 * it is ignored.
 * dopinf_tune_set: value = width (multiple of 64 in [64, 4096]) or 0 to
 *   clear; returns DOPINF_E_ARG for an unknown parameter or a bad value.
 * dopinf_tune_get: the stored width, 0 when untuned.
 * dopinf_autotune_candidates: the (outer, inner) width pairs the autotuner
 *   tries, the same list for the Cholesky and the solves: the outer widths
 *   for DOPINF_TUNE_CHOL_KB / _TRSM_KB, the inner ones (0: none), in the
 *   same order, for DOPINF_TUNE_CHOL_KB2 / _TRSM_KB2; writes up to
 *   max_values of them to values_h (may be NULL) and returns their number.
 * dopinf_autotune_infer: dopinf_infer with the same arguments and results,
 *   preceded by the autotuner: for every group, on its first beta2 chunk,
 *   every Cholesky width pair is timed, then every solve pair; the fastest
 *   are stored for that s.  The stream is synchronized while timing.
 *   times_h (NULL or n_r x 2 x candidates floats, ms): per group the
 *   Cholesky timings, then the solve timings (0 where a group had nothing
 *   to time).
 * Persistence: when the environment variable DOPINF_TUNE_CACHE names a
 *   file, the table is read from it at first use (lines "param key value")
 *   and rewritten after every change, and dopinf_autotune_infer does not
 *   time again a group whose outer widths the table already holds. */
#define DOPINF_TUNE_CHOL_KB 1
#define DOPINF_TUNE_TRSM_KB 2
#define DOPINF_TUNE_CHOL_KB2 3
#define DOPINF_TUNE_TRSM_KB2 4
int dopinf_tune_set(int param, int64_t key, int value);
int dopinf_tune_get(int param, int64_t key);
int dopinf_autotune_candidates(int param, int* values_h, int max_values);
int dopinf_autotune_infer(void* stream, const double* Qhat, int64_t ldqh,
                          int64_t k, int n_r, const int* r_list_h,
                          int n_pairs, const double* beta1_h,
                          const double* beta2_h, double* O, int* status,
                          void* ws, size_t ws_bytes, float* times_h);

/* ---- The sweep as one captured graph (batched form, Sec. 3.5) ------------
 * dopinf_sweep_create validates the arguments as dopinf_infer and
 * dopinf_rollout do, uploads the beta tables into the workspace, optionally
 * runs the autotuner (flags & DOPINF_SWEEP_AUTOTUNE), then captures the
 * kernels of dopinf_infer followed by those of dopinf_rollout (one workgroup
 * per item, no trajectories) on `stream` into a graph and instantiates it.
 * Nothing of the sweep runs during capture.  `stream` must not be the null
 * stream.  dopinf_sweep_launch replays the whole sweep on any stream: it
 * reads Qhat at replay time and overwrites O, status, train_err, growth,
 * outcome and best, exactly as the eager calls would.  The caller keeps
 * every buffer named at creation (and ws, of dopinf_sweep_workspace bytes)
 * alive and unchanged in size until dopinf_sweep_destroy; replays of one
 * sweep must not overlap.  The stream is synchronized before create returns.
 */
#define DOPINF_SWEEP_AUTOTUNE 1u
typedef struct dopinf_sweep_s* dopinf_sweep_t;
size_t dopinf_sweep_workspace(int64_t k, int n_r, const int* r_list_h,
                              int n_pairs);
int dopinf_sweep_create(void* stream, const double* Qhat, int64_t ldqh,
                        int64_t k, int n_r, const int* r_list_h, int n_pairs,
                        const double* beta1_h, const double* beta2_h,
                        int n_states, double max_growth, unsigned flags,
                        double* O, int* status, double* train_err,
                        double* growth, int* outcome, int* best, void* ws,
                        size_t ws_bytes, dopinf_sweep_t* sweep_out);
int dopinf_sweep_launch(dopinf_sweep_t sweep, void* stream);
int dopinf_sweep_destroy(dopinf_sweep_t sweep);


/* ---- Learned closure of the discrete ROM (an addition to the paper) --------
 * g: R^r -> R^r, an MLP r -> 128 -> 128 -> r with GELU (error-function form),
 * corrects the one-step ROM map of Eq. (11): q_{t+1} = f_ROM(q_t) + g(q_t).
 * Parameters are float32, packed as [W1 (128 x r) | b1 (128) | W2 (128 x 128)
 * | b2 (128) | W3 (r x 128) | b3 (r)], row-major; dopinf_closure_param_count
 * gives their number (0 when r is outside [1, 64]).  Standardization `norm`
 * (4r doubles) = [mean_x | std_x | mean_y | std_y] per mode (population std,
 * 0 -> 1).  Standardized inputs, weights and hidden activations are rounded
 * to bfloat16 (nearest even) before each product; sums are float32.
 * Initial weights are an input (the caller draws them). */
int64_t dopinf_closure_param_count(int r);

/* R[t, :] = Qhat[:, t+1] - f_ROM(Qhat[:, t]), t = 0 .. k-2; O is r x d
 * (dopinf_infer's layout), Qhat r x k (ldqh), R (k-1) x r row-major. */
int dopinf_rom_residuals(void* stream, const double* O, int r,
                         const double* Qhat, int64_t ldqh, int64_t k,
                         double* R);

/* Per-mode statistics of inputs X and targets Y (N x r row-major). */
int dopinf_closure_norms(void* stream, int r, const double* X,
                         const double* Y, int64_t N, double* norm);

/* Minibatch Adam (Kingma & Ba 2015) on the mean squared error of the
 * standardized targets.  Epoch e visits row (a*i + c) mod N at position i,
 * a = max(1, (e*2654435761 + 1) mod N) advanced to the next value coprime with
 * N, c = (e*40503 + 17) mod N; minibatches are consecutive runs of `batch`
 * (<= 256) positions.  params: in = initial, out = trained; norm: out;
 * adam_m, adam_v: P floats each (zeroed by the call); loss_log (NULL or
 * `epochs` floats): mean loss per epoch.  One cooperative launch of
 * ceil(batch / 32) workgroups runs the whole training on `stream` (the
 * workgroups meet at two device-wide barriers per minibatch); the workspace
 * (dopinf_closure_fit_workspace, about 0.9 MB at r = 64) holds their
 * gradient shares, a float image of the weights and the barrier words.  A
 * barrier that times out (bounded spin) ends the training early and the
 * loss log reads NaN from that epoch on.  DOPINF_E_HIP if the device has no
 * cooperative launches. */
size_t dopinf_closure_fit_workspace(int r, int64_t N);
int dopinf_closure_fit(void* stream, int r, const double* X, const double* Y,
                       int64_t N, int epochs, int batch, double lr,
                       double beta1, double beta2, double eps, float* params,
                       double* norm, float* adam_m, float* adam_v,
                       float* loss_log, void* ws, size_t ws_bytes);

/* Gradient (packed like params) and mean loss of one batch of N <= 256 rows;
 * uses dopinf_closure_fit_workspace(r, N). */
int dopinf_closure_grad(void* stream, int r, const float* params,
                        const double* norm, const double* X, const double* Y,
                        int64_t N, float* grad, float* loss, void* ws,
                        size_t ws_bytes);

/* G (NULL or N x r) = g(X) in physical units; gmax (NULL or one double) =
 * max over rows of ||g(x_row)||_2. */
size_t dopinf_closure_eval_workspace(int64_t N);
int dopinf_closure_eval(void* stream, int r, const float* params,
                        const double* norm, const double* X, int64_t N,
                        double* G, double* gmax, void* ws, size_t ws_bytes);

/* M rollouts of n_states states from q0 (M x r): q_{t+1} = f_ROM(q_t) + g(q_t).
 * Once ||g(q_t)|| > threshold (or is not finite) rollout m latches to the plain
 * ROM for the rest of the horizon; fallback_at[m] = that t, or -1.
 * threshold <= 0 runs the plain ROM (params / norm may be NULL).
 * Qref (r x k_ref, ldref) is the reference: err[m] = max_{t<k_ref}
 * ||q_t - Qref[:, t]|| / ||Qref[:, t]||; growth[m] = max_{t,i} |q_t[i] - m_i| /
 * max_{t,i} |Qref[i, t] - m_i| (m: temporal mean of Qref); outcome[m] as in
 * dopinf_rollout.  traj: NULL or M x n_states x r. */
size_t dopinf_closure_rollout_workspace(int r);
int dopinf_closure_rollout(void* stream, int r, const double* O,
                           const float* params, const double* norm,
                           double threshold, const double* q0, int64_t M,
                           int n_states, const double* Qref, int64_t ldref,
                           int64_t k_ref, double max_growth, double* traj,
                           double* err, double* growth, int* outcome,
                           int* fallback_at, void* ws, size_t ws_bytes);

#ifdef __cplusplus
}
#endif

#endif /* DOPINF_H */
