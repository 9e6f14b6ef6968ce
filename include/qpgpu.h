/*
 * qpgpu -- C ABI of the MI355X (gfx950) implementation of the preconditioned
 * inexact interior point method of Karim & Solomonik, "Efficient
 * Preconditioners for Interior Point Methods via a new Schur Complement-Based
 * Strategy" (arXiv 2104.12916).
 *
 * Problem (eq. qp, Sec. 1):
 *     minimize 1/2 x^T H x + c^T x   subject to  A x = b,  C x >= d,
 * with H (n x n) symmetric positive definite, A (m1 x n) of full row rank,
 * 0 < m1 <= n, C (m2 x n), m2 >= 1.  Multipliers follow the Lagrangian of
 * eq. lagrangian: lambda (free) for A x = b, nu >= 0 for C x >= d, and
 * H x + c - A^T lambda - C^T nu = 0 at the optimum.
 *
 * Method.  Each IPM iteration solves the inequality-constraint reduced system
 * K_F dnu = r_nu (eq. ineq-const-reduced) by preconditioned CG in implicit form,
 * using one factorization of the fixed KKT block done once per QP (Sec. 4.1).
 * This library factorizes K0 = [H A^T; A 0] (the paper's F = [-H A^T; A 0] up to
 * the sign change K0 = -J F J, J = diag(-I_n, I_m1)), so that
 *     K_F = D + [C 0] K0^{-1} [C^T; 0],  D = V^{-1} S (eq. diag-d).
 *
 * Conventions shared by every entry point
 *   Layout     dense, row-major, float64; the leading dimension equals the
 *              number of columns (H: n, A: n, C: n).  Vectors are contiguous.
 *   Memory     `where` says whether caller pointers are host (QP_MEM_HOST) or
 *              device (QP_MEM_DEVICE, on the context's device) memory.  Inputs
 *              are copied into device memory owned by the context and are only
 *              read during the call; outputs are written to caller buffers.
 *   Streams    all device work runs on the stream given to qp_setup (a
 *              hipStream_t, or NULL for a stream owned by the context); calls
 *              return after their results are complete.  Device inputs are
 *              read on that stream, and a context-owned stream does not wait
 *              for any other: the caller orders the work that wrote them
 *              before the call (by passing its stream, or by synchronizing it).
 *   Errors     status codes only; no C++ exception crosses the ABI.  The text
 *              of the last error of a context is available from qp_last_error.
 *   Threads    a context is not thread-safe; distinct contexts are independent.
 */
#ifndef QPGPU_H
#define QPGPU_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QPGPU_ABI_VERSION 5

typedef struct qp_ctx qp_ctx;

typedef enum {
  QP_OK = 0,
  QP_E_INVALID = 1, /* bad sizes, NaN/Inf input, non-symmetric H, bad option    */
  QP_E_NOT_SPD = 2, /* Cholesky of H failed: H is not positive definite (Sec. 1) */
  QP_E_RANK = 3,    /* Cholesky of A H^{-1} A^T failed: A is rank deficient      */
  QP_E_NOCONV = 4,  /* iteration limit reached (PCG or IPM); outputs are filled  */
  QP_E_NOMEM = 5,   /* device allocation failed                                  */
  QP_E_DEVICE = 6,  /* HIP runtime error                                         */
  QP_E_STATE = 7    /* call order violated (e.g. solve before qp_factor_K0)      */
} qp_status;

typedef enum {
  QP_PREC_NONE = 0,    /* unpreconditioned CG (the paper's U-KF variant)           */
  QP_PREC_LOW_DOF = 1, /* P_L = D, eq. preconditioner-1                            */
  QP_PREC_FEW_EQ = 2,  /* P_H = D + C H^{-1} C^T, eq. preconditioner-2 (exact H)   */
  QP_PREC_AUTO = 3     /* P_L if min(m2, n-m1) <= min(m2, m1), else P_H: the
                          smaller of the bounds of Theorems thm1 and thm2          */
} qp_precond;

typedef enum {
  QP_FP64 = 0, /* every kernel in float64                                        */
  QP_MIXED = 1 /* CG operator and preconditioner applies in float32 with float32
                  accumulation; factorization, IPM residuals and an iterative
                  refinement of each reduced solve stay float64                  */
} qp_precision;

typedef enum { QP_MEM_HOST = 0, QP_MEM_DEVICE = 1 } qp_mem;

typedef enum {
  QP_PH_EXACT = 0, /* P_H = D + C H^{-1} C^T (eq. preconditioner-2; the default)     */
  QP_PH_DIAG = 1   /* P_H = D + C diag(H)^{-1} C^T: the form of the PH-KF variant of
                      the cost models and experiments (Sec. 5.2, Sec. 6); equal to
                      the exact form when H is diagonal                            */
} qp_ph_form;

typedef enum {
  QP_KF_IMPLICIT = 0, /* each CG step applies C^T, the K0 inverse factor twice and C
                         (Sec. 4.1, implicit form; the default)                     */
  QP_KF_EXPLICIT = 1  /* K_F - D = C K0^{-1}_{11} C^T (eq. ineq-const-reduced) formed
                         once per QP after the K0 factorization (m2 x m2, float64,
                         MFMA GEMMs); each CG step is one m2 x m2 row sweep          */
} qp_kf_form;

typedef struct {
  double rtol_kkt;  /* IPM stops when the relative KKT score <= rtol_kkt (1e-9)   */
  double cg_theta;  /* IPM's CG stop: max_i |nu_i r_i| <= cg_theta * mu (0.1)     */
  double cg_rtol;   /* CG relative residual floor inside the IPM (1e-12)          */
  double tau;       /* fraction of the step to the boundary (0.995)              */
  int max_ipm;      /* IPM iteration limit (200)                                 */
  int max_pcg;      /* CG iterations per reduced solve in the IPM; 0: 20 * m2     */
  int poll_every;   /* CG steps launched between host polls of the stop flag;
                       0 (default): single-QP solves size each chunk, up to
                       the previous solve's step count on the context, then an
                       eighth of the steps taken (8..512 steps), and batches,
                       shared-matrix solves and captured graphs use 32         */
  qp_precond prec;  /* preconditioner used by qp_ipm_solve (QP_PREC_AUTO)        */
  qp_precision precision; /* QP_FP64                                              */
  int verbose;      /* 1: one line per IPM iteration on stderr                    */
  int profile;      /* 1: time the operator kernels of the first CG step of every
                       poll chunk with HIP events (read with qp_profile_get)     */
  qp_kf_form kf_form; /* how the CG step applies K_F (QP_KF_IMPLICIT)            */
  qp_ph_form ph_form; /* which H the few-equalities preconditioner uses (EXACT)   */
  int cg_graph;     /* 1: a single-QP solve captures its chunk of poll_every CG
                       steps (32 when poll_every is 0) once as a hipGraph and
                       replays it for every chunk
                       (same kernels and arguments; no profile samples); 0: the
                       steps are launched one by one (0)                        */
} qp_options;

typedef struct {
  int iters;           /* CG steps taken (all refinement sweeps together)         */
  int status;          /* qp_status of the solve                                  */
  double rel_res;      /* ||r_nu - K_F dnu||_2 / ||r_nu||_2, recomputed in float64 */
  int refinements;     /* float64 refinement sweeps (QP_MIXED), else 0            */
  int fp64_fallback;   /* 1 if a mixed solve fell back to float64 CG             */
} qp_pcg_info;

typedef struct {
  int ipm_iters;
  long long pcg_iters_total;
  double rel_kkt;          /* max of the parts below (computed on the device)     */
  double rel_kkt_parts[5]; /* dual, equality, inequality violation, gap, nu < 0   */
  double obj;              /* 1/2 x^T H x + c^T x                                  */
  double mu;               /* s^T nu / m2 at the returned point                    */
  int status;
  int refinements_total;   /* float64 refinement sweeps over all reduced solves   */
  int fp64_fallbacks;      /* mixed reduced solves finished by float64 CG          */
  double t_solve_ms;       /* wall time of qp_ipm_solve (host clock)              */
  long long pcg_iters_fp64; /* CG steps run in float64: all of pcg_iters_total with
                              QP_FP64, the float64 fallback's share with QP_MIXED */
} qp_ipm_info;

/* Defaults listed in the field comments above. */
void qp_default_options(qp_options* opt);

/* Create a context for one QP and copy its data to the device.
 *   out        receives the context (NULL on failure)
 *   n, m1, m2  sizes; require 0 < m1 <= n and m2 >= 1 (Sec. 1)
 *   H (n x n, symmetric within 1e-14 ||H||_F), c (n), A (m1 x n), b (m1),
 *   C (m2 x n), d (m2): the data of eq. qp
 *   opt        options (NULL: defaults)
 *   hip_stream hipStream_t to run on, or NULL for a stream owned by the context
 * Allocates every device buffer the solves need; later calls allocate nothing
 * except qp_factor_K0's setup scratch, which it frees before returning. */
qp_status qp_setup(qp_ctx** out, int n, int m1, int m2, const double* H, const double* c, const double* A,
                   const double* b, const double* C, const double* d, qp_mem where, const qp_options* opt,
                   void* hip_stream);

/* Factorize K0 = L Sigma L^T once (Sec. 4.1, single factorization), Sigma =
 * diag(I_n, -I_m1), L = [L_H 0; W^T L_S] with L_H L_H^T = H, W = L_H^{-1} A^T,
 * L_S L_S^T = A H^{-1} A^T, and store the inverse factor L^{-1} for the solves.
 * Also forms C H^{-1} C^T when the options' preconditioner resolves to P_H, and
 * with QP_KF_EXPLICIT the reduced operator E = Y_1^T Y_1 - Y_2^T Y_2 from
 * Y = L^{-1}[:, :n] C^T (top n rows Y_1, bottom m1 rows Y_2), so K_F = D + E.
 * QP_E_NOT_SPD / QP_E_RANK when a Cholesky pivot is not positive. */
qp_status qp_factor_K0(qp_ctx* ctx);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): qp_factor_K0 with the same kernels and the
 * same results, bitwise, but its set-up scratch (the working copy of H, W^T,
 * A H^{-1} A^T, the recursion temporaries, C L_H^{-T} for P_H, Y for the
 * explicit operator) taken from a fixed device array of
 * QPGPU_STATIC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  Calls no hipMalloc/hipFree.  QP_E_INVALID (nothing
 * run, the context unchanged) when the QP's scratch exceeds that size (about
 * n <= 1500 at m1 = n/4, m2 = n/2, P_H); QP_E_STATE for contexts of a batch or
 * a shared set.  The array is shared by every call on one GPU: the library
 * serializes its own calls per device, and the call returns after its stream
 * is idle, so the next call finds it free; what a call leaves there is
 * overwritten before it is read.  Calls that overlapped on one GPU without
 * that lock (e.g. from two copies of the library in one process) would race.
 * Synchronizes the context's stream, so it cannot be captured in a graph. */
#define QPGPU_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
qp_status qp_factor_K0_static(qp_ctx* ctx);

/* out = K0^{-1} rhs (both n + m1 long) with the stored factor.  Requires
 * qp_factor_K0.  Used by the IPM for r_nu and the recovery of eq. schur-delta-x. */
qp_status qp_k0_solve(qp_ctx* ctx, const double* rhs, double* out, qp_mem where);

/* q = K_F p = D p + [C 0] K0^{-1} [C^T p; 0] (m2 vectors, dvec = diag(D) > 0),
 * the implicit product of one CG step, in float64. */
qp_status qp_kf_apply(qp_ctx* ctx, const double* dvec, const double* p, double* q, qp_mem where);

/* Solve K_F dnu = rhs (eq. ineq-const-reduced) by PCG from a zero initial guess
 * (Sec. 6 protocol) until ||r||_2 <= rtol ||rhs||_2 or maxit steps (maxit <= 0:
 * 10 * m2).  dvec (m2, all > 0) is diag(D); prec selects P_L, P_H or none (AUTO
 * resolves as documented above).  In QP_MIXED precision the CG runs in float32
 * inside float64 iterative refinement.  info may be NULL.  Returns QP_E_NOCONV
 * (with dnu and info filled) when the tolerance is not met. */
qp_status qp_pcg_solve(qp_ctx* ctx, const double* dvec, const double* rhs, double* dnu, qp_mem where,
                       qp_precond prec, double rtol, int maxit, qp_pcg_info* info);

/* Run the interior point method (Mehrotra predictor-corrector, both directions
 * from the reduced system with the preconditioner of the options) and write the
 * final iterate: x (n), lambda (m1), nu (m2), s (m2).  info may be NULL.
 * Returns QP_E_NOCONV (outputs filled) if rtol_kkt is not met in max_ipm. */
qp_status qp_ipm_solve(qp_ctx* ctx, double* x, double* lambda, double* nu, double* s, qp_mem where,
                       qp_ipm_info* info);

/* Diagnostic: average device time (ms) of one launch of a CG-step operator
 * kernel, measured with HIP events around `reps` back-to-back launches on the
 * context's stream, in the launch configuration qp_pcg_solve uses:
 *   op 0  u = C^T p            (row sweep over the stored C^T, or column sweep over C)
 *   op 1  v = Sigma M u        (row sweep over M = L^{-1}[:, :n]); with the
 *                              one-pass K0 product (qp_k0_one_pass): the
 *                              single sweep of M that forms M^T Sigma M u as
 *                              per-workgroup partials
 *   op 2  w = M^T v            (row sweep over the stored M^T, or column sweep
 *                              over M); one-pass: the sum of the partials
 *   op 3  q = C w              (row sweep over C)
 *   op 4  one whole P_L CG step (ops 0-2 and the fused q/update kernel)
 * precision QP_MIXED times the float32 copies (context created QP_MIXED).
 * Overwrites the context's CG work vectors.  Requires qp_factor_K0. */
qp_status qp_op_time(qp_ctx* ctx, int op, qp_precision precision, int reps, double* avg_ms);

/* Diagnostic: the HBM read rate of a plain streaming kernel on the current
 * device, the practical ceiling of the CG-step sweeps (all of which stream a
 * matrix, Sec. 4.1).  Allocates a device buffer of `bytes` (a multiple of 16;
 * pick several times the 256 MB last-level cache), reads it with 16-byte
 * non-temporal loads from cu_count * wg_per_cu workgroups (1..32), and writes
 * the average time (ms) of `reps` back-to-back passes to *avg_ms; frees the
 * buffer before returning.  QP_E_INVALID for bad arguments (no device work),
 * QP_E_NOMEM if the buffer does not fit, QP_E_DEVICE on a HIP error. */
qp_status qp_hbm_read_time(size_t bytes, int wg_per_cu, int reps, double* avg_ms);

/* Diagnostic: average device time (ms) of `reps` back-to-back runs of a dense
 * float64 kernel of the factorization (Sec. 4.1, the single factorization of the
 * fixed block and of P_H) on the current device, with operands of size n
 * (1..16384) that it allocates, fills deterministically and frees:
 *   op 0  C = A B^T, n x n x n (the GEMM of the factorization)
 *   op 1  the same with B^T upper triangular (k range trimmed per tile)
 *   op 2  X = chol(P)^{-1} of an n x n SPD P (the recursive Cholesky-inverse,
 *         leaves, fused nodes and GEMMs; P restored by a copy before each run,
 *         whose time is included)
 * QP_E_INVALID for bad arguments, QP_E_NOMEM if the operands do not fit,
 * QP_E_NOT_SPD if op 2 rejects a pivot, QP_E_DEVICE on a HIP error. */
qp_status qp_dense_time(int op, int n, int reps, double* avg_ms);

/* Launch-shape table (workgroups per CU, loads in flight, one-pass sweep shape,
 * update width, cache policy of the matrix loads) of the streaming kernels, per
 * size bucket: calls on one QP use the bucket of its n, batches the base entry.
 * qp_tune_set replaces the table with `spec`, in the text format of the cache
 * that paper_2104_12916_amd/autotune.py writes: lines "default k=v,...",
 * "n<=N k=v,..." (kernel shapes only), "arch NAME", "# ...".  The layout keys
 * (ld_pad, op_t, k0_sym) must keep their values: QP_E_INVALID otherwise, or for
 * an unknown key or value.  Not to be called while other threads launch.
 * qp_tune_get writes the current table (needed = bytes including the NUL;
 * buf NULL: only needed). */
qp_status qp_tune_set(const char* spec);
qp_status qp_tune_get(char* buf, size_t len, size_t* needed);

/* Average device time (ms) per launch and sample counts of the CG-step kernels
 * sampled while options.profile is set, in the order of qp_op_time's ops 0-3
 * (C^T p, Sigma M u or the one-pass sweep of M, M^T v or the sum of its
 * partials, q = C w + D p), then for P_H the apply z = X_P^T X_P r: its one pass
 * over X_P and the sum of its partials when m2 <= 4096 and the one-pass K0
 * product is on, else the X_P r row sweep and the X_P^T t column sweep.
 * reset != 0 clears them. */
qp_status qp_profile_get(qp_ctx* ctx, double avg_ms[6], long long samples[6], int reset);

/* 1 if the context's implicit CG step forms K0^{-1}_{11} u = M^T Sigma M u
 * (K0^{-1} = L^{-T} Sigma L^{-1}, M = L^{-1}[:, :n]; Sec. 4.1)
 * in one pass over M instead of the two triangular sweeps: same product, M read
 * once.  Chosen at qp_create from n (n <= 4096) and the K_F form; 0 otherwise
 * or for NULL. */
int qp_k0_one_pass(const qp_ctx* ctx);

/* 1 if qp_factor_K0 found C = I (m2 = n; simple bounds x >= d, Sec. 4.2): the CG
 * step then takes u = p and q = K0^{-1}_{11} p + D p, with no product by C, and
 * P_H = D + H^{-1}.  0 before qp_factor_K0, otherwise, or for NULL. */
int qp_c_identity(const qp_ctx* ctx);

/* CG steps of the predictor and of the corrector reduced solve of every IPM
 * iteration of the last qp_ipm_solve on this context (the counts of the paper's
 * CG-iteration experiment, Sec. 6.2; bounded by Theorems thm1 and thm2 in exact
 * arithmetic).  Writes the first min(iterations, cap) counts into each array
 * that is not NULL and the number of iterations into *count.  QP_E_INVALID for
 * NULL ctx or count, or cap < 0. */
qp_status qp_ipm_cg_steps(const qp_ctx* ctx, int* predictor, int* corrector, int cap, int* count);

/* Device bytes held by the context (all buffers, factor included). */
size_t qp_ctx_bytes(const qp_ctx* ctx);

/* Free every resource of the context.  NULL is accepted. */
void qp_destroy(qp_ctx* ctx);

/* Static description of a status code. */
const char* qp_status_str(qp_status st);

/* Message of the last failure on this context ("" if none; never NULL). */
const char* qp_last_error(const qp_ctx* ctx);

/* ---- Batches of independent QPs ------------------------------------------
 * A batch keeps many QPs of different sizes in flight on one stream and runs
 * the interior point method of qp_ipm_solve for all of them, each QP at its
 * own pace.  Work proceeds in ticks: one chunk of poll_every CG steps for
 * every QP inside a reduced solve (eq. ineq-const-reduced), one launch per
 * operator sweep for all of them, then every QP moves on through the steps
 * that need no CG (KKT check, right-hand sides, recovery, step, refinement),
 * batched over the QPs at the same point.  A QP's arithmetic and launch shapes
 * depend only on that QP, so its result does not depend on the other QPs of
 * the batch.  Preconditioner and precision come from the batch options
 * (QP_PREC_AUTO resolves per QP).
 *
 * Memory: the batch takes one device allocation of hbm_budget_bytes at
 * creation (0: 80% of the free device memory) and gives every admitted QP its
 * buffers from it; a QP's memory returns as soon as it finishes.  Admission is
 * refused with QP_E_NOMEM while the QP does not fit (qp_batch_footprint tells
 * its size), or when 4096 QPs are in flight.
 *
 * Device inputs of qp_batch_admit are read on the batch's stream, which waits
 * for no other stream: the caller finishes the work that wrote them first.
 *
 * Flow: qp_batch_admit (any time between steps) -> qp_batch_step (ticks) ->
 * qp_batch_finished lists finished tickets -> qp_batch_collect copies a result
 * out and forgets the ticket.  Calls on one batch must not overlap. */
typedef struct qp_batch qp_batch;

/* Create a batch.  opt: NULL for defaults; hip_stream: hipStream_t or NULL for
 * a stream owned by the batch. */
qp_status qp_batch_create(qp_batch** out, const qp_options* opt, size_t hbm_budget_bytes, void* hip_stream);

/* Admit one QP (arguments as for qp_setup) and receive its ticket (> 0).  The
 * data is copied to the device before the call returns.  QP_E_NOMEM: no room
 * now, retry after qp_batch_step has retired QPs; QP_E_INVALID: bad problem. */
qp_status qp_batch_admit(qp_batch* b, int n, int m1, int m2, const double* H, const double* c, const double* A,
                         const double* b_eq, const double* C, const double* d, qp_mem where, long long* ticket);

/* Run up to max_rounds ticks (fewer when nothing is in flight); QPs admitted
 * since the last call are factored in the first.  n_done (may be NULL)
 * receives the number of finished, uncollected QPs.  A QP that fails
 * (H not SPD, A rank deficient, no convergence) finishes with that status and
 * does not affect the others; a device error fails the call. */
qp_status qp_batch_step(qp_batch* b, int max_rounds, int* n_done);

/* Tickets of finished, uncollected QPs in increasing order (at most cap). */
qp_status qp_batch_finished(qp_batch* b, long long* tickets, int cap, int* count);

/* Copy the final iterate of a finished QP: x (n), lambda (m1), nu (m2), s (m2),
 * host or device memory per `where`; info (may be NULL) as for qp_ipm_solve,
 * with t_solve_ms measured from admission to completion.  Returns the QP's own
 * status (QP_OK, QP_E_NOCONV, QP_E_NOT_SPD, ...); QP_E_STATE if the ticket has
 * not finished, QP_E_INVALID if it is unknown.  The ticket is then forgotten
 * (outputs are left untouched when the QP failed before its first iterate). */
qp_status qp_batch_collect(qp_batch* b, long long ticket, double* x, double* lambda, double* nu, double* s,
                           qp_mem where, qp_ipm_info* info);

/* Counters: QPs admitted and not finished, finished and not collected, arena
 * bytes in use and in total, ticks run.  Any pointer may be NULL. */
qp_status qp_batch_query(const qp_batch* b, int* in_flight, int* finished, size_t* bytes_used,
                         size_t* bytes_capacity, long long* rounds);

/* Arena bytes a QP of these sizes takes under these options (0 if invalid). */
size_t qp_batch_footprint(const qp_options* opt, int n, int m1, int m2);

/* Message of the last batch-level failure ("" if none; never NULL). */
const char* qp_batch_last_error(const qp_batch* b);

/* Sampled batched CG-step sweeps (options.profile set at creation): the first
 * step of every poll chunk is timed with HIP events.  Per sweep, in the order
 * of qp_profile_get: average device time per launch (ms), average algorithmic
 * matrix bytes per launch over the QPs the launch covered, and the number of
 * samples.  reset != 0 clears them. */
qp_status qp_batch_profile_get(qp_batch* b, double avg_ms[6], double avg_bytes[6], long long samples[6], int reset);

/* Free the batch, its arena and every result not collected.  NULL accepted. */
void qp_batch_destroy(qp_batch* b);

/* ---- QPs sharing H, A and C ---------------------------------------------
 * Many QPs that differ only in c, b and d share K0 and its factorization
 * (Sec. 4.1) and the operator C K0^{-1}_{11} C^T of eq. ineq-const-reduced;
 * only D differs.  A qp_shared factorizes K0 once; its solves run the reduced
 * systems of k such QPs as a block PCG: every CG step applies the shared
 * operator to the k direction vectors at once, streaming C^T, M, M^T and C once
 * for all k, while the scalars, the stop test and the preconditioner stay per
 * QP (P_L or none: P_H would need one factorization of D + C H^{-1} C^T per QP).
 * The k interior point iterations advance in lockstep.  FP64, implicit K_F.
 * Arrays of the k QPs are stacked row by row (QP j at offset j * length).
 */
typedef struct qp_shared qp_shared;

/* Upload H (n x n), A (m1 x n), C (m2 x n) and factorize K0.  opt: precision
 * QP_FP64, kf_form QP_KF_IMPLICIT and prec P_L, none or AUTO (= P_L), else
 * QP_E_INVALID.  Failures of the factorization as qp_factor_K0. */
qp_status qp_shared_setup(qp_shared** out, int n, int m1, int m2, const double* H, const double* A, const double* C,
                          qp_mem where, const qp_options* opt, void* hip_stream);

/* k reduced solves K_F(d_j) dnu_j = rhs_j (dvec, rhs, dnu: k x m2) by block PCG
 * from zero, each to ||r_j||_2 <= rtol ||rhs_j||_2 or maxit steps; info (k
 * entries, may be NULL) as qp_pcg_solve.  prec: P_L, none or AUTO (= P_L). */
qp_status qp_shared_pcg_solve(qp_shared* sh, int k, const double* dvec, const double* rhs, double* dnu, qp_mem where,
                              qp_precond prec, double rtol, int maxit, qp_pcg_info* info);

/* Solve k QPs min 1/2 x^T H x + c_j^T x, A x = b_j, C x >= d_j (c: k x n, b:
 * k x m1, d: k x m2; outputs x, lambda, nu, s stacked the same way; info: k
 * entries or NULL).  Returns the first failure of any QP (all are still solved). */
qp_status qp_shared_ipm_solve(qp_shared* sh, int k, const double* c, const double* b, const double* d, double* x,
                              double* lambda, double* nu, double* s, qp_mem where, qp_ipm_info* info);

/* Message of the last failure ("" if none; never NULL). */
const char* qp_shared_last_error(const qp_shared* sh);

/* Free everything of the shared set.  NULL accepted. */
void qp_shared_destroy(qp_shared* sh);

#ifdef __cplusplus
}
#endif
#endif /* QPGPU_H */
