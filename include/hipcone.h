/*
 * hipcone — C-ABI of an MI355X (gfx950) primal-dual interior-point solver for
 *
 *     minimize 1/2 x'Px + q'x   subject to   Ax + s = b,  s in K          (P)
 *
 * with K a product of zero, nonnegative, second-order, exponential, 3-d power
 * and PSD cones (arXiv 2412.19027, Sec. 1 problem (P) and Sec. 2.1
 * "Supported cones"; PSD cones may have different sides, which the paper
 * leaves to future work, Sec. 5).  Every per-iteration step of the method
 * (Algorithm 1, Sec. 3.2) runs in this library's HIP kernels: residuals and
 * termination, the cone scalings and their writes into the KKT system, the
 * quasi-definite LDL' factorisation and triangular solves with iterative
 * refinement, direction recovery, step lengths and the iterate update.
 *
 * Conventions
 *   - Every function returns an int32 status: 0 = OK, < 0 = error (HC_ERR_*).
 *     No C++ exception or abort crosses this boundary.  The text of the last
 *     error of a handle is available from hc_last_error(handle) (or of the
 *     last failed handle-less call from hc_last_error(NULL)).
 *   - Host pointers unless a parameter says "device".  All input arrays are
 *     copied; the caller may free them when the call returns.
 *   - A solver handle is not thread-safe; distinct handles are independent.
 *   - Solver outcomes (solved, infeasible, iteration limit, ...) are not
 *     errors: they are reported in hc_info.status.
 */
#ifndef HIPCONE_H
#define HIPCONE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define HC_OK              0
#define HC_ERR_INVALID_ARG (-1)  /* NULL pointer or a size out of range            */
#define HC_ERR_DIM         (-2)  /* cone rows do not add up to m, or n/m <= 0       */
#define HC_ERR_CSR         (-3)  /* unsorted/duplicate/out-of-range CSR, or P has
                                    an entry below its diagonal                    */
#define HC_ERR_CONE        (-4)  /* unknown cone type, SOC dim < 2, EXP/POW dim !=
                                    3, alpha outside (0,1), PSD side outside
                                    [1, 32]                                        */
#define HC_ERR_NONFINITE   (-5)  /* NaN or Inf in P, q, A or b                      */
#define HC_ERR_OOM         (-6)  /* device memory (arena too small or allocation
                                    failed); hc_last_error names the bytes needed */
#define HC_ERR_DEVICE      (-7)  /* a HIP runtime call failed                       */
#define HC_ERR_STATE       (-8)  /* call out of order (e.g. solve before bind)      */
#define HC_ERR_UNSUPPORTED (-9)  /* problem shape this build does not handle        */
#define HC_ERR_TOO_LARGE   (-10) /* server: one problem's workspace exceeds the
                                    whole HBM budget                               */
#define HC_PENDING         1     /* server: the ticket's solve has not finished    */

/* ---- cone list (Sec. 2.1) ------------------------------------------------ */
#define HC_CONE_ZERO   0   /* {0}^dim                                          */
#define HC_CONE_NONNEG 1   /* R_+^dim                                          */
#define HC_CONE_SOC    2   /* {(t, x) : |x|_2 <= t}, dim = 1 + len(x) >= 2     */
#define HC_CONE_EXP    3   /* exponential cone, dim = 3                        */
#define HC_CONE_POW    4   /* power cone with exponent alpha in (0,1), dim = 3 */
#define HC_CONE_PSD    5   /* k x k PSD cone; dim = k, rows = k (k+1) / 2 in the
                              svec encoding: upper triangle column by column,
                              off-diagonal entries scaled by sqrt(2)            */

typedef struct {
  int32_t type;   /* HC_CONE_*                                  */
  int32_t dim;    /* rows (PSD: the matrix side k)              */
  double alpha;   /* POW exponent; ignored by the other types   */
} hc_cone;

/* ---- problem data (Sec. 1 (P)); CSR is 0-based, columns sorted, unique ------ */
typedef struct {
  int64_t n, m;
  const int64_t* P_rowptr;  /* n+1; upper triangle of P (col >= row); may be NULL
                               together with P_col/P_val when P = 0              */
  const int32_t* P_col;
  const double* P_val;
  const double* q;          /* n */
  const int64_t* A_rowptr;  /* m+1 */
  const int32_t* A_col;
  const double* A_val;
  const double* b;          /* m */
  const hc_cone* cones;     /* in row order; rows must add up to m */
  int32_t ncones;
} hc_problem;

/* ---- settings (defaults from hc_settings_default) ------------------------ */
#define HC_PRECISION_FP64  0   /* factor and solve in FP64 (the paper's default)  */
#define HC_PRECISION_MIXED 1   /* factor and triangular solves in FP32, residuals,
                                  refinement updates and everything else in FP64
                                  (Sec. 3.7 mixed precision)                     */
typedef struct {
  double eps_feas;        /* 1e-8: optimality tests (eq. termination-check)        */
  double eps_inf;         /* 1e-8: infeasibility tests (eq. infeasibility-check)   */
  int32_t max_iter;       /* 200                                                   */
  int32_t precision;      /* HC_PRECISION_FP64                                     */
  double static_reg;      /* delta_s: 1e-8 (FP64) / sqrt(eps_32) (mixed); <= 0 picks
                             the value for the precision                          */
  double dyn_reg;         /* delta_d: eps^2 of the factor precision; < 0 picks it   */
  double ir_abstol;       /* 1e-12 (refinement stop, Sec. 3.7)                      */
  double ir_reltol;       /* 1e-12                                                  */
  int32_t ir_max;         /* 10 corrections after the first solve                  */
  double beta;            /* 1e-6: neighbourhood N(beta) (Sec. 2.2)                 */
  double backtrack;       /* 0.8: exp/pow backtracking ratio                        */
  double step_fraction;   /* 0.99 (Algorithm 1 update)                              */
  int32_t equilibrate;    /* 1: modified Ruiz scaling of P, A, q, b at setup        */
  int32_t equil_iters;    /* 10                                                     */
  int32_t force_dual_scaling; /* 0: exp/pow use the primal-dual (BFGS) scaling      */
  int32_t verbose;        /* 0                                                      */
  int32_t profile;        /* 1: time the factorisation's MFMA update kernels and the
                             cone-layer launches with HIP events (hc_info.gemm_*,
                             cone_*); 2: the same with the look-ahead's trailing
                             updates on the handle's stream, so that no timed
                             kernel overlaps another; 0 = off                     */
  int32_t leaf_blocks;    /* 1: columns of the Schur complement that fall into small
                             connected components once the high-degree columns are
                             set aside are factored as leaf blocks ahead of the
                             dense tail (two-level LDL'); 0: one dense block      */
  int32_t warm_start;     /* 1: a solve after hc_update_data starts from the blend
                             (1 - warm_blend) v_prev + warm_blend v_0 of the last
                             solved iterate v_prev = (x, s, z)/tau, carried over
                             to the new equilibration, and the usual initial point
                             v_0 (tau = kappa = 1); 0: always from v_0 (0)        */
  double warm_blend;      /* 0.02                                                   */
  double ir_mu_frac;      /* the refinement also stops once its residual is at most
                             ir_mu_frac min(mu, 1) (1 + |rhs|_inf), mu the
                             iteration's complementarity; < 0 picks 1e-3 for the
                             mixed mode and 0 (off: the fixed tolerances alone) for
                             FP64                                                 */
} hc_settings;

/* ---- device hand-off ------------------------------------------------------ */
typedef struct {
  void* arena;          /* device memory the library sub-allocates from, or NULL
                           to let the library allocate (and free) its own        */
  size_t arena_bytes;
  void* stream;         /* hipStream_t to run on; NULL = the null stream          */
  int32_t device;       /* HIP device ordinal                                     */
  void* host_stage;     /* pinned host memory (hipHostMalloc) for the per-iteration
                           read-backs of reduction partials, owned by the caller
                           and used only while the handle runs; NULL, or fewer
                           than hc_host_stage_bytes bytes: the library allocates
                           (and frees) its own                                     */
  size_t host_stage_bytes;
} hc_device;

/* ---- results -------------------------------------------------------------- */
#define HC_STATUS_UNSOLVED              0
#define HC_STATUS_SOLVED                1
#define HC_STATUS_PRIMAL_INFEASIBLE     2
#define HC_STATUS_DUAL_INFEASIBLE       3
#define HC_STATUS_MAX_ITER              4
#define HC_STATUS_INSUFFICIENT_PROGRESS 5
#define HC_STATUS_NUMERICAL_ERROR       6
#define HC_STATUS_CANCELLED             7   /* server destroyed before the solve ended */

typedef struct {
  int32_t status;          /* HC_STATUS_*                                          */
  int32_t iterations;
  double obj_primal;       /* g_p (eq. residuals-objectives), unscaled             */
  double obj_dual;         /* g_d                                                  */
  double res_primal;       /* |r_p|_inf                                            */
  double res_dual;         /* |r_d|_inf                                            */
  double gap;              /* |g_p - g_d|                                          */
  double mu;
  double setup_ms;         /* host analysis + upload + initial point               */
  double solve_ms;         /* the iterations                                       */
  double factor_ms;        /* summed over iterations (device events)               */
  double solve_kkt_ms;
  double cone_ms;
  int64_t ir_solves;       /* triangular-solve passes including refinement         */
  int64_t pivot_guard_hits;
  int64_t dual_switches;   /* iterations redone with the dual exp/pow scaling      */
  int64_t n_ordered;       /* size of the dense tail of the Schur complement       */
  double factor_flops;     /* per factorisation                                    */
  int64_t factorizations;
  double gemm_ms;          /* with settings.profile: summed duration of the MFMA     */
  double gemm_flops;       /* update kernels and their algorithmic flops (2K per    */
  int64_t gemm_launches;   /* lower-triangle entry updated)                          */
  int64_t fp64_fallbacks;  /* mixed mode: iterations refactored in FP64 because the
                              FP32-factor refinement left a residual above
                              1e-6 (1 + |rhs|_inf) or not finite; in a served
                              result of the batched engine, plus one when the
                              whole solve broke down in mixed precision and ran
                              again in FP64 (iterations then count both runs) */
  int64_t n_leaves;        /* leaf blocks factored ahead of the tail               */
  int64_t leaf_columns;    /* columns inside leaf blocks (n = leaf_columns + n_ordered) */
  int64_t psd_gathered_rows; /* rows of PSD cones whose Schur blocks enter through
                              T = M_c A_c and a column gather (0: row pairs only)  */
  double cone_kernel_ms;   /* with settings.profile: summed device time (events on
                              the handle's stream) of the cone-layer launches:
                              scaling, M blocks, H applications, d_s, direction
                              recovery and step lengths                           */
  double cone_bytes;       /* their algorithmic HBM bytes (each launch's minimum
                              reads and writes of iterate, direction and scaling
                              state)                                              */
  int64_t cone_launches;
  int64_t sym_split_columns; /* columns outside the tail's dense rows and hubs
                              whose graph the setup ordered (approximate
                              minimum degree) and split along its elimination
                              tree: subtrees of at most 32 columns coupled to
                              at most 64 others became leaf blocks, the rest
                              joined the tail (0: no such columns)              */
  int64_t sym_supernodes;  /* fundamental supernodes of that graph's factor      */
  int64_t sym_levels;      /* levels of its supernodal tree                     */
  int64_t sym_nnz_l;       /* nonzeros of its Cholesky factor (column counts)    */
} hc_info;

typedef struct hc_solver hc_solver;

/* Fill `out` with the defaults listed above.  HC_ERR_INVALID_ARG on NULL. */
int32_t hc_settings_default(hc_settings* out);

/* Validate and copy the problem, reorder rows by cone family, equilibrate and
 * build the KKT structure on the host (setup phase of Algorithm 1).  No device
 * memory is touched.  `settings` may be NULL (defaults).
 * Errors: HC_ERR_INVALID_ARG, HC_ERR_DIM, HC_ERR_CSR, HC_ERR_CONE,
 * HC_ERR_NONFINITE, HC_ERR_UNSUPPORTED.  On error *out is NULL. */
int32_t hc_setup(hc_solver** out, const hc_problem* prob, const hc_settings* settings);

/* Device bytes hc_bind needs for this handle (arena size). */
int32_t hc_workspace_bytes(const hc_solver* s, size_t* bytes);
/* Pinned host bytes of the read-back staging (hc_device.host_stage) this
 * handle needs.  HC_ERR_INVALID_ARG on NULL. */
int32_t hc_host_stage_bytes(const hc_solver* s, size_t* bytes);

/* Place the solver on a device: sub-allocate the arena (or allocate) and upload
 * the data.  The arena and stream must outlive the
 * handle.  Errors: HC_ERR_STATE (already bound), HC_ERR_OOM, HC_ERR_DEVICE. */
int32_t hc_bind(hc_solver* s, const hc_device* dev);

/* Compute the initial point and run the iterations of Algorithm 1 to
 * termination on the handle's stream; blocks until the status is known.  Each
 * call is a complete solve from the initial point (repeat calls give the same
 * result).  Errors: HC_ERR_STATE, HC_ERR_DEVICE. */
int32_t hc_solve(hc_solver* s);

int32_t hc_get_info(const hc_solver* s, hc_info* out);

/* For callers that cannot allocate (tight serving loops, harnesses that
 * forbid device allocation): hc_bind + hc_solve
 * + hc_get_solution of a set-up, unbound handle without allocating.  The
 * workspace is the library's static device array of HC_NOALLOC_BYTES bytes
 * (each device the library runs on holds its own copy until the process
 * ends; its address is taken once per device, on the first call there), the
 * read-back staging a static 4 MiB host block, and the dense factorisation
 * issues its look-ahead schedule's launches on `stream` alone (no stream or
 * event is created).  No hipMalloc, hipHostMalloc or hipFree is called.
 * Calls are serialised by a process-wide lock, so calls on one GPU never
 * overlap (the array is shared by all of them and keeps the last call's
 * contents; each call initialises what it reads) and each returns after its
 * work on the GPU has finished.  stream: a HIP stream of `device` (NULL: the
 * null stream).  x (n), sv (m), z (m): host buffers for the solution as
 * hc_get_solution returns it, any may be NULL; info: as hc_get_info, may be
 * NULL.  The handle is left unbound (timing settings are ignored).  Errors:
 * HC_ERR_INVALID_ARG (NULL handle, device outside 0-63), HC_ERR_STATE (the
 * handle is bound), HC_ERR_TOO_LARGE (workspace above HC_NOALLOC_BYTES or
 * staging above 4 MiB; both sizes are in hc_last_error), HC_ERR_DEVICE. */
#define HC_NOALLOC_BYTES ((size_t)64 << 20)
int32_t hc_solve_noalloc(hc_solver* s, void* stream, int32_t device, double* x, double* sv, double* z,
                         hc_info* info);


/* Solution in the user's row order, unscaled and divided by tau (Sec. 2.2:
 * x/tau, s/tau, z/tau): x (n), s (m), z (m), caller-owned buffers (any may be
 * NULL).  on_device = 0: host buffers; nonzero: device buffers of the handle's
 * device, written by a kernel on the handle's stream (complete on return).
 * For an infeasible status the unnormalised certificate (eq.
 * infeasibility-check) is returned instead.  HC_ERR_STATE before hc_bind. */
int32_t hc_get_solution(const hc_solver* s, double* x, double* sv, double* z, int32_t on_device);

/* Raw internal iterate (scaled, rows in the library's family order):
 * x (n), s (m), z (m), tau, kappa; and the internal->user row map (m int64). */
int32_t hc_get_iterate(const hc_solver* s, double* x, double* sv, double* z, double* tau,
                       double* kappa, int64_t* row_of_internal);

/* Replace the internal iterate (same order and scaling as hc_get_iterate;
 * host arrays x (n), s (m), z (m); tau, kappa > 0).  The next hc_solve starts
 * from its own initial point again; this exists for the KKT test below and
 * for callers that restart a solve step by step. */
int32_t hc_set_iterate(hc_solver* s, const double* x, const double* sv, const double* z,
                       double tau, double kappa);

/* Test entry: one KKT solve of an interior-point iteration at the current
 * iterate (Sec. 3.3 and 3.7, Algorithm 1): the cone scalings at (s, z) with the
 * given mu (force_dual != 0 forces the dual scaling of the exp/pow cones),
 * the regularised factorisation, and
 *   [P  A'; A  -H] [x; z] = [r1; r2]
 * solved with iterative refinement against the unregularised matrix, exactly
 * as inside hc_solve.  r1 (n), r2 (m), xo (n), zo (m): host arrays in the
 * internal row order.  stats (NULL or 4 doubles): solves used, delta, number
 * of exp/pow cones on the primal-dual (rank-4) scaling, FP64
 * refactorisations of the mixed mode. */
int32_t hc_test_kkt_solve(hc_solver* s, double mu, int32_t force_dual, const double* r1,
                          const double* r2, double* xo, double* zo, double* stats);

/* Test entry: the two operators of the refinement at the current iterate,
 * after the same scaling and factorisation: one regularised solve
 *   [P + delta I,  A'; A,  -(H + delta I)] [xr; zr] = [r1; r2]
 * (z eliminated through M = (H + delta I)^-1, then S xr = r1 + A' M r2), and
 * the unregularised product [kx; kz] = [P xr + A' zr; A xr - H zr].  Host
 * arrays in the internal row order: r1, xr, kx (n); r2, zr, kz (m). */
int32_t hc_test_kkt_ops(hc_solver* s, double mu, int32_t force_dual, const double* r1,
                        const double* r2, double* xr, double* zr, double* kx, double* kz);

/* hc_test_ordered_sums: host-only check of a set-up handle's ordered Schur
 * sums (the A' M A products of Sec. 3.7's Schur complement grouped by the
 * entry of S they land on, and the leaf blocks' updates of the tail grouped
 * by tail entry; no device).  With synthetic weights in place of M it adds
 * every product where it lands, one by one, and again from the ordered
 * lists: out[0] = max |difference| / max |entry|, out[1] = leaf update slots
 * not listed exactly once or listed under the wrong tail entry, out[2] = the
 * number of destinations.  *ordered = 0 when the lists were not built
 * (beyond their size limit: the FP64-atomic kernels run), and then out is
 * zero.  HC_ERR_INVALID_ARG on NULL. */
int32_t hc_test_ordered_sums(hc_solver* s, int32_t* ordered, double* out);

/* Test entry: the Schur complement S = P + delta I + A' M A (Sec. 3.7, cone
 * rows eliminated) assembled at the scaling of the current iterate, and its
 * Cholesky factor.  Only for solvers whose columns all sit in the dense block
 * (settings.leaf_blocks = 0, else HC_ERR_STATE).  S_out, L_out (NULL allowed):
 * host n x n, column-major; the lower triangle (i >= j) is written, the rest
 * is unspecified.  L_out is the factor the iteration would use (FP32 values in
 * the mixed mode).  stats (NULL or 3 doubles): delta, exp/pow cones on the
 * primal-dual scaling, factor precision in bits. */
int32_t hc_test_schur(hc_solver* s, double mu, int32_t force_dual, double* S_out, double* L_out,
                      double* stats);

/* Parametric re-solve (Sec. 4.6, re-solving with new data of one structure):
 * replace the values of P (upper triangle, in the set-up's CSR order; nnz
 * of P), q (n), A (set-up's CSR order; nnz of A) and b (m); NULL keeps an
 * array as it is.  The sparsity pattern and cones stay those of hc_setup:
 * the row order, the assembly plan, the leaf blocks and the tail ordering
 * are reused, only equilibration and the scaled data are recomputed and
 * copied into the bound device buffers.  The next hc_solve starts from the
 * method's initial point (no warm start).  Host arrays, copied.  Errors:
 * HC_ERR_NONFINITE (nothing changed), HC_ERR_CSR if P's pattern changed. */
int32_t hc_update_data(hc_solver* s, const double* P_val, const double* q, const double* A_val,
                       const double* b);

void hc_destroy(hc_solver* s);                /* NULL is a no-op */
const char* hc_last_error(const hc_solver* s);
const char* hc_status_str(int32_t status);

/* ---- kernel test entry points (device pointers, one cone family) ----------
 * They run exactly the kernels hc_solve runs, on `count` cones of one family
 * given cone by cone (AoS: cone i occupies rows [i*rows, (i+1)*rows)), and
 * exist so a test can compare single steps with a reference.  `alpha` is the
 * POW exponent per cone (NULL otherwise); `dim` is rows per cone (PSD: side).
 * All buffers are device memory of count*rows doubles unless stated.
 *
 * hc_test_cone_scale: scaling at (s, z) with global mu (Appendix A): writes
 *   H_out (count*rows*rows, row-major H of each cone), lam_out (count*rows:
 *   nonneg/SOC/PSD lambda (PSD: k eigenvalues, rest 0), exp/pow: the shadow
 *   point z~ = -grad f*(s)), branch_out (count int32: exp/pow 1 = dual
 *   scaling taken, else 0).
 * hc_test_cone_ds: combined-step d_s (eq. ds-correction-step) from the scaling
 *   at (s, z) and the affine directions (dsa, dza), sigma*mu = sm.
 * hc_test_cone_step: per cone the largest alpha <= amax with s + alpha ds and
 *   z + alpha dz in the closed cones (nonneg/SOC/PSD: exact boundary step;
 *   exp/pow: interior membership tested at alpha = amax * 0.8^j, j = 0..63,
 *   reported as the first passing trial, or 0).
 * hc_test_cone_step_min: the minimum over all `count` cones of that exact
 *   boundary step (no cap; INFINITY when no direction leaves its cone), by the
 *   launch hc_solve uses for the step length (Sec. 2.2, "Update iterates"),
 *   written to the host double *alpha_min.  Nonneg, SOC and PSD only
 *   (HC_ERR_INVALID_ARG otherwise).
 * force_dual (scale, mblock, ds): nonzero selects the dual scaling
 *   H = mu grad^2 f(z) for exp/pow cones (Appendix A), as hc_solve does after a
 *   short primal-dual step; ignored by the symmetric families.
 */
int32_t hc_test_cone_scale(int32_t type, int64_t count, int32_t dim, const double* alpha,
                           const double* s, const double* z, double mu, int32_t force_dual,
                           double* H_out, double* lam_out, int32_t* branch_out, void* stream);
/* hc_test_cone_mblock: the explicit blocks M_c = (H_c + delta I)^-1 that the
 *   Schur complement is assembled from (eq. linsys_2x2 with the cone rows
 *   eliminated first), at the scaling of (s, z); M_out (device, count x rows
 *   x rows, dense symmetric).  delta > 0. */
int32_t hc_test_cone_mblock(int32_t type, int64_t count, int32_t dim, const double* alpha,
                            const double* s, const double* z, double mu, int32_t force_dual,
                            double delta, double* M_out, void* stream);
int32_t hc_test_cone_ds(int32_t type, int64_t count, int32_t dim, const double* alpha,
                        const double* s, const double* z, const double* dsa, const double* dza,
                        double mu, int32_t force_dual, double sm, double* ds_out, void* stream);
int32_t hc_test_cone_step(int32_t type, int64_t count, int32_t dim, const double* alpha,
                          const double* s, const double* z, const double* ds, const double* dz,
                          double amax, double* alpha_out, void* stream);
int32_t hc_test_cone_step_min(int32_t type, int64_t count, int32_t dim, const double* alpha,
                              const double* s, const double* z, const double* ds, const double* dz,
                              double* alpha_min, void* stream);

/* Dense Cholesky of an SPD matrix (device, column-major, n x n, leading dim
 * ld >= n, lower triangle referenced) followed by the solve of `nrhs`
 * right-hand sides (device, n x nrhs column-major) in place, in the factor
 * precision (HC_PRECISION_*): the kernels of the KKT solve's Schur
 * complement.  The matrix is overwritten by the factor.  guard_hits may be
 * NULL. */
int32_t hc_test_dense_chol_solve(int32_t precision, int64_t n, int64_t ld, double* A, int32_t nrhs,
                                 double* B, int64_t* guard_hits, void* stream);
/* The same with the envelope that the solver derives for its dense tail:
 * `last` (host, n entries, NULL = dense) with last[j] - 1 the largest row
 * holding a nonzero of columns 0..j (j < last[j] <= n, non-decreasing; else
 * HC_ERR_INVALID_ARG).  The factorisation touches only rows inside it, which
 * is exact when A is zero below it (Cholesky fill stays in the envelope). */
int32_t hc_test_dense_chol_solve_env(int32_t precision, int64_t n, int64_t ld, double* A,
                                     const int64_t* last, int32_t nrhs, double* B, int64_t* guard_hits,
                                     void* stream);

/* ---- served form --------------------------------------------------------
 * Continuous batching of many independent problems on one GPU (the paper's
 * parametric re-solve setting, Sec. 4.6, served as a request stream).
 * Requests are analysed on the submitting thread (as hc_setup: the problem is
 * copied, the caller may free it on return), queued first in first out, and
 * admitted into active slots while their device workspace fits the HBM
 * budget; the server carves every workspace from one device pool of
 * hbm_budget_bytes: the caller's (hc_server_config.pool, as hc_device.arena
 * for one handle) or one it allocates at creation (the batched engine's
 * descriptor table, a few bytes per slot, is allocated apart).  `workers` host threads each
 * own a stream and a share of the slots; a tick advances each of a worker's
 * problems by one interior-point iteration, so problems of uneven size
 * interleave and a finished problem's slot and memory go to the next request.
 * A server handle is internally locked: submit, poll, wait and stats may be
 * called from any thread. */
typedef struct {
  size_t hbm_budget_bytes;  /* device pool for all active workspaces (64 GiB)      */
  int32_t max_slots;        /* problems in flight at most (64)                     */
  int32_t workers;          /* host threads / streams, 1..16 (4)                   */
  hc_settings settings;     /* applied to every problem (hc_settings_default)     */
  int32_t device;           /* HIP device ordinal (0)                              */
  int32_t batched;          /* 1: problems the batched engine takes (hc_batch_check)
                               run there, one wavefront each, all of them advanced
                               by one graph-launched kernel per tick; the others on
                               the per-slot workers.  0: every problem per slot (1) */
  int32_t batch_slots;      /* problems in flight on the batched engine (1024)      */
  void* pool;               /* caller's device memory of hbm_budget_bytes on
                               `device` (256-byte aligned) to carve the workspaces
                               from, owned by the caller and kept until
                               hc_server_destroy returns; NULL: the server
                               allocates the pool itself (NULL)                     */
} hc_server_config;

typedef struct {
  /* filled by hc_server_poll / hc_server_wait */
  uint64_t tag;             /* as given to hc_server_submit                       */
  int32_t status;           /* HC_STATUS_*                                         */
  int32_t error;            /* HC_OK, or the error code that ended the solve     */
  int32_t iterations;
  double obj_primal, obj_dual, res_primal, res_dual;
  double queue_ms;          /* submit -> admitted                                 */
  double solve_ms;          /* admitted -> finished                               */
  double latency_ms;        /* submit -> finished                                 */
  int64_t n, m;
  /* set by the caller before poll/wait: host buffers of n, m, m doubles that
     receive x, s, z (user row order, unscaled, divided by tau), or NULL */
  double* x;
  double* s;
  double* z;
} hc_result;

/* Batched engine (the served form's tick, also callable directly): small
 * problems with zero, nonnegative and second-order cones of at most 16 rows
 * whose Schur complement S = P + delta I + A'MA has, after a reverse
 * Cuthill-McKee ordering of its columns, a band half-width of at most 56.
 * Each problem runs on one 64-lane wavefront and every problem in the batch
 * advances by one iteration of Algorithm 1 per kernel launch (Sec. 3.2; the
 * KKT system of eq. linsys_2x2 eliminated to S and factored as a band).
 *
 * hc_batch_check: HC_OK and the band half-width in *band when `s` (from
 *   hc_setup) is eligible; HC_ERR_UNSUPPORTED with the reason in
 *   hc_last_error(NULL) otherwise.
 * hc_solve_batch: solves `count` set-up handles (they stay unbound) on
 *   `stream` of `device`, allocating one device block for all of them and
 *   freeing it on return; results[i] receives the outcome of handles[i] and,
 *   where the caller set results[i].x/s/z, the solution (user coordinates,
 *   divided by tau; the certificate for an infeasible status).  solve_ms is
 *   the batch's device time.  Errors: HC_ERR_INVALID_ARG, HC_ERR_UNSUPPORTED
 *   (a handle is not eligible: nothing is solved), HC_ERR_OOM, HC_ERR_DEVICE. */
int32_t hc_batch_check(const hc_solver* s, int32_t* band);
int32_t hc_solve_batch(hc_solver* const* handles, int32_t count, void* stream, int32_t device,
                       hc_result* results);

typedef struct {
  int64_t submitted, completed, rejected, cancelled, active, pending, iterations;
  double p50_latency_ms, p99_latency_ms, mean_latency_ms;
  double solves_per_s;      /* completed / (last completion - first submission)   */
  double busy_ms;           /* summed tick time of the workers                    */
  size_t hbm_in_use, hbm_peak;
} hc_server_report;

typedef struct hc_server hc_server;

/* Defaults listed above.  HC_ERR_INVALID_ARG on NULL. */
int32_t hc_server_config_default(hc_server_config* out);
/* Creates the pool (unless the caller gives one) and the workers.
 * HC_ERR_INVALID_ARG (bad config, or a pool not 256-byte aligned),
 * HC_ERR_DEVICE, HC_ERR_OOM (pool allocation failed). */
int32_t hc_server_create(hc_server** out, const hc_server_config* cfg);
/* Validates and analyses `p` (errors as hc_setup; HC_ERR_TOO_LARGE when its
 * workspace exceeds the budget) and queues it; *ticket identifies it. */
int32_t hc_server_submit(hc_server* s, const hc_problem* p, uint64_t tag, uint64_t* ticket);
/* HC_PENDING while the solve runs; HC_OK once `out` is filled (the ticket is
 * then retired); HC_ERR_INVALID_ARG for an unknown or retired ticket. */
int32_t hc_server_poll(hc_server* s, uint64_t ticket, hc_result* out);
/* Blocks until the ticket's solve has finished, then as hc_server_poll. */
int32_t hc_server_wait(hc_server* s, uint64_t ticket, hc_result* out);
int32_t hc_server_stats(hc_server* s, hc_server_report* out);
/* Stops the workers (problems still queued or active end as
 * HC_STATUS_CANCELLED), frees the pool.  NULL is a no-op. */
void hc_server_destroy(hc_server* s);

/* Plain device-to-device copy of `bytes` bytes (src, dst: device, 16-byte
 * aligned, bytes a multiple of 16; HC_ERR_INVALID_ARG otherwise), run to
 * completion on `stream`.  It is the reference kernel of known traffic
 * (bytes read, bytes written) against which hardware byte counters of the
 * other kernels are scaled. */
int32_t hc_test_copy(const void* src, void* dst, int64_t bytes, void* stream);

/* hc_test_symbolic: the setup's symbolic analysis (host only, no device) of a
 * caller's symmetric graph: n vertices, CSR adjacency ptr (n + 1) / adj
 * (both directions of every edge, self loops ignored).  Writes the
 * approximate minimum degree order with its elimination tree postordered
 * (order[k] = vertex eliminated k-th), the tree (parent[k]: position of the
 * parent, -1 for a root), the Cholesky column counts (diagonal included),
 * the fundamental supernodes (sn_first: nsuper + 1 column starts, sn_parent,
 * sn_level; every array sized n, or n + 1 for sn_first) and the number of
 * levels.  HC_ERR_INVALID_ARG on NULL, HC_ERR_CSR on a malformed graph. */
int32_t hc_test_symbolic(int32_t n, const int64_t* ptr, const int32_t* adj, int32_t* order, int32_t* parent,
                         int64_t* count, int32_t* sn_first, int32_t* sn_parent, int32_t* sn_level,
                         int32_t* nsuper, int32_t* nlevels);

#ifdef __cplusplus
}
#endif
#endif /* HIPCONE_H */
