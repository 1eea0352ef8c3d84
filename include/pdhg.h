/*
 * pdhg.h -- C ABI of the MI355X PDHG solver for LP relaxations of unit
 * commitment (restarted, adaptive-step primal-dual hybrid gradient).
 *
 * Problem (the LP pair of the paper's "PDHG Background" section, read with
 * the signs of its Lagrangian and update equations and widened to equality
 * rows and bounds):
 *
 *     min  c'x   s.t.  a_i'x  = b_i   (row_kind[i] == PDHG_ROW_EQ)
 *                      a_i'x >= b_i   (row_kind[i] == PDHG_ROW_GE)
 *                      l <= x <= u
 *
 * Iteration (the Chambolle-Pock update of that section with the box
 * projection on x and the sign-cone projection on the duals of >= rows),
 * on the diagonally rescaled problem, tau = eta/omega, sigma = eta*omega:
 *
 *     x' = proj_[l,u]( x - tau (c - A'y) )
 *     y' = proj_Y  ( y + sigma (b - A(2x' - x)) )
 *
 * with the adaptive step size and restart scheme of the PDLP method that the
 * section cites.  Every call returns PDHG_OK (0) or a negative error code;
 * pdhg_last_error() gives a thread-local message for the last failure.
 * No C++ exception crosses this interface.
 *
 * Memory: the library never allocates device memory.  The caller passes a
 * device workspace (size from pdhg_workspace_bytes) that must stay alive
 * until pdhg_destroy.  pdhg_setup creates one pinned host record of the
 * control state per handle (hipHostMalloc).
 *
 * Streams: each handle runs its device work on a stream of its own
 * (non-blocking, default priority) created by pdhg_setup.  Every call orders
 * that work after what the caller queued on the stream given to pdhg_setup
 * (0 = the null stream) by recording an event there and waiting on it, and
 * before anything the caller queues there afterwards by the reverse.  Calls
 * that return results in host memory synchronize before they return.
 */
#ifndef PDHG_H
#define PDHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
enum {
  PDHG_OK = 0,
  PDHG_ERR_ARG = -1,       /* bad argument: null pointer, m or n <= 0, bad row kind, bad option */
  PDHG_ERR_CSR = -2,       /* not canonical CSR: row_ptr[0] != 0, row_ptr not monotone,
                              row_ptr[m] != nnz, column out of range, columns of a row not
                              strictly ascending */
  PDHG_ERR_BOUNDS = -3,    /* l > u, l = +inf, u = -inf or a NaN bound */
  PDHG_ERR_NONFINITE = -4, /* non-finite entry of A, b or c */
  PDHG_ERR_OOM = -5,       /* workspace smaller than pdhg_workspace_bytes */
  PDHG_ERR_HIP = -6,       /* a HIP runtime call failed; the handle is unusable afterwards */
  PDHG_ERR_STATE = -7      /* call out of order (e.g. backward without an unrolled forward) */
};

/* solve status (pdhg_info.status) */
enum {
  PDHG_OPTIMAL = 1,        /* relative KKT error <= tol */
  PDHG_ITER_LIMIT = 2,
  PDHG_TIME_LIMIT = 3,
  PDHG_NUMERICAL = 4,      /* NaN or Inf reached the iterates */
  PDHG_PRIMAL_INFEASIBLE = 5, /* y is a certificate: with lambda = -A'y and y >= 0 on >= rows,
                              b'y + sum_j min(lambda_j lo_j, lambda_j hi_j) > 0 over the
                              implied bounds, beyond its rounding allowance (Farkas) */
  PDHG_DUAL_INFEASIBLE = 6 /* x is a ray d (caller's order): c'd < 0, and the largest
                              violation of (A d)_i = 0 on = rows, (A d)_i >= 0 on >= rows
                              and of d_j in the recession cone of [lo_j, hi_j] (implied
                              bounds) is at most dinf_tol (-c'd): a tolerance test, not a
                              proof.  The LP is unbounded if it is feasible. */
};

enum { PDHG_ROW_EQ = 0, PDHG_ROW_GE = 1 };
enum { PDHG_FP64 = 0, PDHG_MIXED = 1 };

/* The LP, borrowed for the duration of pdhg_setup (which copies it).
 * CSR: row_ptr[m+1] int32 with row_ptr[0] = 0 and row_ptr[m] = nnz,
 * col_idx[nnz] int32 strictly ascending inside each row, val[nnz] finite.
 * row_kind[m] uint8; b[m], c[n] finite; l[n] may hold -INFINITY, u[n] +INFINITY.
 * obj_offset: a finite constant of the objective, c'x + obj_offset.  It is added
 * to the reported primal_obj, dual_obj and dual_bound only: the relative gap and
 * every termination test use the objectives of min c'x without it, so a solve
 * takes the same steps whatever the offset (nonfinite: PDHG_ERR_NONFINITE).
 * on_device = 0: host pointers; 1: device pointers (validated on the GPU). */
typedef struct {
  int64_t m, n, nnz;
  const int32_t *row_ptr;
  const int32_t *col_idx;
  const double *val;
  const uint8_t *row_kind;
  const double *b, *c, *l, *u;
  double obj_offset;
  int on_device;
} pdhg_lp;

typedef struct {
  double tol;             /* relative KKT target (default 1e-4) */
  int64_t max_iter;       /* attempts (default 1e7) */
  double time_limit_s;    /* wall-clock limit of pdhg_solve (default 1e30) */
  int precision;          /* PDHG_FP64 or PDHG_MIXED */
  int eval_period;        /* attempts between evaluations (default 64) */
  int step_mode;          /* 0 adaptive (default), 1 constant eta */
  double fixed_eta;       /* step_mode 1 / unrolled mode: eta; <= 0: 0.9/||A^||_2 */
  double fixed_omega;     /* > 0: initial primal weight; <= 0: ||c^||/||b^|| */
  int scaling_iters;      /* Ruiz passes (default 10) */
  int pock_chambolle;     /* 1 (default): one Pock-Chambolle pass after Ruiz */
  int restart;            /* 1 (default): restart scheme on */
  int use_average;        /* 1 (default): weighted average is a candidate */
  int64_t unroll_iters;   /* > 0: unrolled fixed-step mode with this many steps */
  int64_t checkpoint_every; /* unrolled mode: checkpoint period (default 50) */
  int use_graph;          /* 1 (default): replay iteration blocks as HIP graphs */
  int verbose;            /* 1: one log line per evaluation on stderr (a batch: one line
                             per 64 evaluations with the instances still running) */
  double polish_tol;      /* mixed precision: FP32 phase stops at this KKT (default tol) */
  int pw_update;          /* 1 (default): primal weight updated at restarts; 0: kept */
  double pw_theta;        /* smoothing of the primal-weight update in log space (default 0.5) */
  int tiles_per_block;    /* SpMV partition: 256-row tiles per workgroup; 0 = automatic */
  int autotune;           /* 1: pdhg_setup times candidate SpMV partitions (tiles per
                             workgroup, LDS-staged or per-row loops, long-row threshold)
                             and keeps the fastest; cached per matrix in the process */
  int spmv_direct;        /* partition without autotune: 1 = per-row loops, 0 = LDS tiles */
  int long_seg;           /* rows/columns longer than this get a workgroup; 0 = 64 */
  int reorder;            /* 1 (default): the solver works on P A Q' with P, Q a reverse
                             Cuthill-McKee order of A's row/column graph (better locality
                             of the SpMV gathers); every argument and result stays in the
                             caller's order.  0: the caller's order */
  int compact_index;      /* 1 (default): the attempt kernels read the matrix structure in a
                             16-bit form relative to each 256-row tile (row ends counted from
                             the tile's first nonzero, indices from the tile's smallest one)
                             when every tile of A and A' has at most 65535 nonzeros and an
                             index span of at most 65535; otherwise, and with 0, the 32-bit
                             CSR.  The results do not depend on it */
  int infeas_every;       /* every this many evaluations (default 4; 0: never) the current y
                             is tested as a certificate of primal infeasibility; a proof
                             ends the solve with PDHG_PRIMAL_INFEASIBLE and returns it.
                             The ray test of dinf_tol runs at the same evaluations */
  int polish_pw_update;   /* mixed precision: 1 (default) updates the primal weight at the
                             FP64 phase's restarts as in the FP32 phase; 0 keeps the weight
                             the FP32 phase ended with (faster on some LPs, stalls on others) */
  int fp32_stall_evals;   /* mixed precision: the FP32 phase hands over to FP64 when the
                             relative KKT error has not fallen below 0.9 of its best value
                             for this many evaluations (default 300); 0: only at polish_tol.
                             NaN or Inf in the FP32 phase also hands over */
  double dinf_tol;        /* at the infeasibility tests (infeas_every), the primal iterate's
                             displacement since the last restart is tested as a ray with this
                             tolerance (default 1e-8; 0: never): PDHG_DUAL_INFEASIBLE.
                             Skipped where c'x is bounded below on the implied box (every
                             column bounded on both sides, or its cost of the sign that the
                             one finite bound limits, or zero): no ray can improve there */
  int batch_pack;         /* 1: batched instances that share a matrix (same base, one tile
                             per workgroup, LDS-staged tiles) run the attempt kernels a
                             pack of 4 instances per workgroup, the tile's structure
                             loaded once for the pack; 0 (default): one instance per
                             workgroup.  The results do not depend on it */
  int stream_nt;          /* load policy of the attempt kernels' streams (matrix, read-once
                             vectors): 1 non-temporal, 0 ordinary loads, -1 (default)
                             per precision: non-temporal when the larger attempt kernel
                             moves at least 192 MiB (three quarters of the 256 MiB
                             Infinity Cache), ordinary below.  The results do not depend
                             on it */
  int polish_fp32_matrix; /* PDHG_MIXED with tol >= 1e-6: 1 (default) the FP64 phase's
                             attempt kernels multiply the FP32 copies of the matrix values
                             (widened exactly; its evaluations, restarts and termination
                             keep the FP64 matrix); their rounding moves the fixed point
                             by about 1e-7 relative, so tighter tolerances, and 0, use
                             the FP64 values */
} pdhg_opts;

typedef struct {
  int status;
  int which;              /* returned point: 0 current iterate, 1 average */
  int64_t attempts;       /* one attempt = one A'y and one Ax product */
  int64_t accepted, restarts;
  int64_t attempts_fp32;  /* mixed precision: attempts spent in the FP32 phase */
  double primal_obj, dual_obj;
  double rel_primal, rel_dual, rel_gap, rel_kkt;
  double eta, omega;      /* final step size and primal weight (scaled space) */
  double setup_s, solve_s;
  /* A lower bound on the LP optimum that holds whatever the accuracy of the
   * returned y (weak duality; the LP relaxation bounds of the paper's
   * "PDHG Execution & Crossover Refinement" discussion), computed once after
   * the solve: b'y~ + sum_j min over x_j in [lo_j, hi_j] of lambda_j x_j with
   * lambda = c - A'y~, lowered by an allowance that exceeds the rounding of
   * the sums.  y~ is y projected on >= rows and clamped so that the reduced
   * costs of single-entry columns with an infinite bound (penalty slacks)
   * keep their sign; [lo, hi] are l, u with infinite ends replaced by
   * implied bounds (pdhg_implied_bounds) where the LP's rows give them.  A
   * lambda_j whose sign is within its rounding error counts with both bounds.
   * -INFINITY when a bound that is needed is infinite; -INFINITY in the
   * unrolled mode. */
  double dual_bound;
} pdhg_info;

typedef struct pdhg_handle pdhg_handle;

void pdhg_default_opts(pdhg_opts *opts);

/* Bytes of device workspace needed for this LP and options. */
int pdhg_workspace_bytes(const pdhg_lp *lp, const pdhg_opts *opts, size_t *bytes);

/* Validate the LP, copy it into the workspace, build the bound kinds, the
 * transpose A' (canonical CSR, rows ascending inside each column) and the
 * power-of-two diagonal scaling (Ruiz, then Pock-Chambolle).  stream is a
 * hipStream_t passed as void*.  Synchronizes the stream once. */
int pdhg_setup(const pdhg_lp *lp, const pdhg_opts *opts, void *workspace,
               size_t workspace_bytes, void *stream, pdhg_handle **handle);

/* Solve from x0, y0 (nullable; original space, device pointers if the LP
 * was given on the device, else host) and write x[n], y[m] (same memory
 * kind).  info is host memory.  x, y are the returned point (info.which);
 * with PDHG_PRIMAL_INFEASIBLE y is the certificate, with
 * PDHG_DUAL_INFEASIBLE x is the ray (y then the current iterate).  The same
 * holds per instance for pdhg_solve_batch. */
int pdhg_solve(pdhg_handle *h, const double *x0, const double *y0, double *x,
               double *y, pdhg_info *info);

/* One instance of a batched solve (for example a branch-and-bound node or a
 * load scenario).  Instances whose base handle is the same share that
 * handle's preprocessed matrix; b, c, l, u override the base's vectors when
 * non-null (original space, same memory kind as the base LP), and the n_fix
 * (index, value) pairs fix variables (l = u = value) on top of the bounds.
 * x0[n], y0[m] (nullable, same memory kind) warm-start the instance, e.g.
 * a child node from its parent's solution; omega0, eta0 > 0 replace the
 * initial primal weight and step size (scaled-space values, as pdhg_info
 * reports them: a child can continue with its parent's), 0 keeps the
 * defaults; the primal weight keeps its initial value (no update at
 * restarts) during the first hold_omega attempts, which suits a start close
 * to the optimum, and is updated as usual after them (0: from the start).
 * The dual bound of an instance uses the base's implied bounds
 * only when b, l and u are not overridden (fixings only tighten the bounds
 * the implied ones were derived from), and its repair intervals only when
 * b, c, l and u are not overridden. */
typedef struct {
  int32_t base;
  const double *b, *c, *l, *u;
  const int32_t *fix_idx;
  const double *fix_val;
  int64_t n_fix;
  const double *x0, *y0;
  double omega0, eta0;
  int64_t hold_omega;
} pdhg_instance;

/* Device workspace bytes for pdhg_solve_batch with these instances. */
int pdhg_batch_workspace_bytes(pdhg_handle *const *handles, int n_handles,
                               const pdhg_instance *inst, int batch, size_t *bytes);

/* Solve `batch` instances together: every kernel launch serves all instances
 * still running (per-instance step size, primal weight, restarts and
 * termination), blocks of attempts are replayed as HIP graphs, and finished
 * instances leave the launch tables.  The options (tolerance, precision,
 * limits) are those of handles[0]; all handles must share the precision.
 * x[k], y[k] receive instance k's solution (memory kind of its base LP) and
 * infos[k] its report (solve_s is the wall time of the whole batch).  Runs on
 * handles[0]'s stream after synchronizing the other handles. */
int pdhg_solve_batch(pdhg_handle *const *handles, int n_handles,
                     const pdhg_instance *inst, int batch, void *workspace,
                     size_t workspace_bytes, double *const *x, double *const *y,
                     pdhg_info *infos);

/* Feasibility polishing of a point (x, y), e.g. a solve's result, toward a
 * vertex-ready start for crossover (the PDHG-then-crossover pipeline of the
 * paper's "PDHG Execution & Crossover Refinement" section): two further PDHG
 * solves on the handle's matrix, in FP64 whatever opts.precision, adaptive,
 * restarted, with no infeasibility tests.
 *   1. Primal feasibility: the LP with c = 0, from (x, 0), until the relative
 *      primal residual is at most tol; its x is kept.
 *   2. Dual feasibility: the LP with b = 0 and every finite bound set to 0
 *      (the same cone of admissible reduced costs), from (0, y), until the
 *      relative dual residual is at most tol; its y is kept.
 * x_out, y_out receive the combined point (caller's order, original space,
 * memory kind of the LP; they may not alias x, y).  info reports the combined
 * point on the original problem (relative residuals, gap, objectives, dual
 * bound; status PDHG_OPTIMAL when its relative KKT error is at most
 * opts.tol, else PDHG_ITER_LIMIT), attempts and restarts of both steps
 * together.  max_iter: attempts per step (<= 0: opts.max_iter); omega > 0:
 * initial primal weight of both steps (scaled space, as pdhg_info reports
 * it; 0: 1).  PDHG_ERR_STATE in the unrolled mode. */
int pdhg_polish(pdhg_handle *h, const double *x, const double *y, double tol, int64_t max_iter,
                double omega, double *x_out, double *y_out, pdhg_info *info);

/* pdhg_solve_batch for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * batched solve and results, with no workspace argument.  Its workspace is a
 * file-scope device array of the library of PDHG_STATIC_SCRATCH_BYTES
 * (64 MiB), one per GPU, held until the process ends; the call allocates no
 * device or pinned host memory and captures no graph (blocks of attempts
 * are launched directly).  Returns PDHG_ERR_OOM when the batch's workspace
 * (pdhg_batch_workspace_bytes) exceeds 64 MiB or batch exceeds
 * PDHG_STATIC_MAX_BATCH (64), and PDHG_ERR_HIP when the array's device
 * address cannot be found.  The handles must belong to the current device.
 * Every call on a GPU shares its array, which keeps the last call's contents;
 * calls from one process are serialized, and work that overlaps such a call
 * on the same GPU through the array would race. */
#define PDHG_STATIC_SCRATCH_BYTES (64u << 20)
#define PDHG_STATIC_MAX_BATCH 64
int pdhg_solve_batch_static(pdhg_handle *const *handles, int n_handles,
                            const pdhg_instance *inst, int batch, double *const *x,
                            double *const *y, pdhg_info *infos);

/* Unrolled mode (opts.unroll_iters = K > 0, FP64): pdhg_solve runs exactly K
 * fixed-step iterations from x = proj(x0 or 0), y = proj(y0 or 0), with
 * eta = opts.fixed_eta (or 0.9/||A^||_2 by 50 power iterations), the primal
 * weight of the usual rule (or opts.fixed_omega), no restarts and no
 * average, and keeps (x, y, Ax) every opts.checkpoint_every steps.  It returns
 * x_K, y_K with status PDHG_ITER_LIMIT; info.primal_obj is V = c'x_K.
 *
 * pdhg_backward then gives the gradient of V with respect to b and c
 * (original space), times grad_value, by the exact transpose of the unrolled
 * map: segments are recomputed from their checkpoints with bit-packed
 * projection masks, then swept backwards with one A' and one A product per
 * step.  At a point where a pre-projection value sits exactly on a bound the
 * mask counts it as projected (the one-sided derivative of the clamp from
 * inside the active side).  grad_b[m], grad_c[n]: same memory kind as the LP.
 * Returns PDHG_ERR_STATE without a preceding unrolled solve. */
int pdhg_backward(pdhg_handle *h, double grad_value, double *grad_b, double *grad_c);

/* Replace b and/or c (original space, nullable, same memory kind as the
 * LP) of a set-up problem: rescales them with the stored diagonals and resets
 * the step size and primal weight rules.  Invalidates a previous unrolled
 * solve for pdhg_backward. */
int pdhg_update(pdhg_handle *h, const double *b, const double *c);

void pdhg_destroy(pdhg_handle *h);

const char *pdhg_last_error(void);

/* ---- inspection entry points (diagnostics and parity tests) ---- */

/* Copy the preprocessed problem to host memory (any pointer may be null):
 * bound kinds var_kind[n] (0 free, 1 lower, 2 upper, 3 boxed, 4 fixed),
 * the transpose (colptr[n+1], rowidx[nnz], valT[nnz]), the scaled A values
 * val_s[nnz], and the scaling diagonals Dr[m], Dc[n]
 * (A_scaled = diag(Dr) A diag(Dc)). */
int pdhg_export_setup(pdhg_handle *h, uint8_t *var_kind, int32_t *colptr,
                      int32_t *rowidx, double *valT, double *val_s, double *Dr,
                      double *Dc);

/* Copy the FP32 data the mixed-precision attempt kernels read (host memory,
 * caller's order; any pointer may be null): the scaled values of A in CSR
 * order val_s[nnz], of the transpose valT[nnz] (rows ascending inside each
 * column), and the scaled b[m], c[n], l[n], u[n], each the round-to-nearest
 * FP32 cast of the FP64 scaled value.  PDHG_ERR_STATE for an FP64 handle. */
int pdhg_export_fp32(pdhg_handle *h, float *val_s, float *valT, float *b, float *c, float *l,
                     float *u);

/* out = A_scaled x (transpose = 0, x[n], out[m]) or A_scaled' x
 * (transpose = 1, x[m], out[n]) with the solver's FP64 SpMV kernels; host
 * memory. */
int pdhg_spmv(pdhg_handle *h, int transpose, const double *x, double *out);

/* The implied bounds pdhg_setup derived for the dual bound (host memory,
 * caller's order, original units): lo[n], hi[n] are l, u with infinite ends
 * replaced where propagation over the rows bounds them, each widened by
 * more than its rounding: r -+ (2 (len + 2) 2^-53 (|b_i| + sum_k |a_ik bound_k|)
 * / |a_ij| + 4 2^-53 |r|) for a bound r derived from row i of len entries,
 * and no bound where that is not finite.  After pdhg_update with a new b they no longer apply
 * and this returns l, u. */
int pdhg_implied_bounds(pdhg_handle *h, double *lo, double *hi);

/* The locality ordering pdhg_setup applies when opts.reorder = 1, for a
 * canonical CSR structure in host memory (host code only, no GPU needed):
 * row_order[m] receives the original row of each internal row, col_order[n]
 * the original column of each internal column.  Returns PDHG_ERR_CSR for a
 * structure that is not canonical CSR. */
int pdhg_locality_order(int64_t m, int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                        int32_t *row_order, int32_t *col_order);

/* The SpMV partition in use, out[7]: out[0] tiles per workgroup, out[1] 1 for
 * per-row loops (0: LDS-staged tiles), out[2] long-segment threshold, out[3]
 * number of long rows plus long columns, out[4] 1 when the attempt kernels
 * read the 16-bit structure (opts.compact_index), out[5] and out[6] 1 when
 * the FP64 and the FP32 attempt kernels use non-temporal stream loads
 * (opts.stream_nt). */
int pdhg_get_partition(pdhg_handle *h, int *out);

/* Run `attempts` more attempts from the handle's current iterate (the state
 * the last pdhg_solve left) on the library's stream, each kernel launched
 * with start/stop events that take its dispatch's own timestamps, and report
 * average milliseconds per launch: ms_out[0] primal step (A'y row-dot +
 * projection, long columns included), ms_out[1] dual step (Ax row-dot +
 * projection, long rows included), ms_out[2] step control, ms_out[3] whole
 * attempt (first kernel's start to last kernel's end, launch gaps
 * included).  Precision as set up.  On a handle that has not solved yet the
 * attempts start from the zero point after 16 untimed ones. */
int pdhg_time_kernels(pdhg_handle *h, int attempts, double *ms_out);

/* pdhg_time_kernels with cold caches: before each attempt the library reads
 * flush_bytes of the caller's device buffer `flush` (contents ignored; make it
 * larger than twice the 256 MB Infinity Cache), which evicts the previous
 * attempt's lines from L2 and the Infinity Cache, so the kernels fetch the
 * matrix and vectors from HBM.  Same outputs as pdhg_time_kernels. */
int pdhg_time_kernels_cold(pdhg_handle *h, int attempts, const void *flush, size_t flush_bytes,
                           double *ms_out);

/* Merge-path CSR SpMV, y = A x, the load-balanced partition of the sparse
 * products that the PDHG iteration applies twice per step (the A x and A'y
 * of the "PDHG Background" section): the m row ends and nnz nonzeros form one
 * merged sequence, and every workgroup and every lane take an equal share of
 * it whatever the row lengths.  A row's products are rounded on their own and
 * summed in a fixed order (within a lane in CSR order, then the lanes' and
 * workgroups' partial sums in order), so repeated calls give the same bits;
 * the order differs from the attempt kernels' sum in CSR order.
 *
 * All pointers are device memory; stream may be null (the null stream).
 * row_ptr[m+1] int32, col_idx[nnz] int32 in [0, n), val[nnz], x[n], y[m]
 * (written, not read).  The workspace (256-byte aligned, caller-owned) holds
 * the plan and the workgroups' carries; its size comes from
 * pdhg_spmv_merge_workspace_bytes.  m + nnz must stay below 2^31
 * (PDHG_ERR_ARG); m = 0 is a no-op. */
int pdhg_spmv_merge_workspace_bytes(int64_t m, int64_t nnz, size_t *bytes);

/* The plan: the start of every workgroup's share, found by a binary search on
 * the merge path, written into the workspace, once per sparsity structure.
 * It first checks the structure on the device (row_ptr[0] = 0, nondecreasing,
 * row_ptr[m] = nnz, 0 <= col_idx < n: else PDHG_ERR_CSR) and synchronizes
 * the stream to read the result.  Later SpMV calls on the workspace must pass
 * the same row_ptr and col_idx. */
int pdhg_spmv_merge_plan(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                         const int32_t *col_idx, void *workspace, size_t ws_bytes, void *stream);

/* y = A x in FP64 / FP32 on a planned workspace; asynchronous on stream.
 * PDHG_ERR_OOM for a workspace below the needed size. */
int pdhg_spmv_merge_f64(int64_t m, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                        const double *val, const double *x, double *y, void *workspace,
                        size_t ws_bytes, void *stream);
int pdhg_spmv_merge_f32(int64_t m, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                        const float *val, const float *x, float *y, void *workspace,
                        size_t ws_bytes, void *stream);

/* Average ms of the merge-path SpMV on the handle's own scaled matrices in
 * its iteration precision (FP32 for PDHG_MIXED): ms_out[0] for A'y (n rows of
 * the stored transpose), ms_out[1] for A x (m rows), each the SpMV and its
 * carry fix-up, timed with HIP events on the handle's stream over `attempts`
 * repetitions after planning both.  The workspace holds both plans:
 * pdhg_spmv_merge_workspace_bytes(n, nnz) + (m, nnz) bytes.  It overwrites
 * the handle's iterate buffers (the next solve starts afresh). */
int pdhg_time_spmv_merge(pdhg_handle *h, int attempts, void *workspace, size_t ws_bytes,
                         double *ms_out);

#ifdef __cplusplus
}
#endif
#endif /* PDHG_H */
