/*
 * bmg.h — C ABI of the MI355X (gfx950) hot path of BM-Global for
 * nuclear-norm-regularised matrix completion.
 *
 * Problem (MC) of Sec. 1 of the paper:
 *     min_X  1/2 || P_Omega(X - A) ||_F^2 + lambda ||X||_*
 * solved in the factored form X = W H^T (problem (MF) / (BM-nuclear)) by
 * Algorithm 1: BM-phase steps on (W, H) alternating with inexact
 * proximal-gradient steps whose partial SVD comes from block subspace
 * iteration (Algorithm 2 with p = 0) followed by singular-value
 * soft-thresholding (eqs. exactSVD, approxSVD, truncate of Suppl. A.1.1).
 *
 * Conventions for every call:
 *   - Pointers marked (device) point to GPU memory, (host) to CPU memory.
 *     The caller owns every buffer it passes.  The library never allocates
 *     device memory itself: all of its internal arrays live in the workspace
 *     the caller passes to bmg_problem_create (size from bmg_workspace_size,
 *     which also reserves what the solver variants of the given options need),
 *     the server's in the arena the caller passes to bmg_server_create.
 *     Host side, each problem pins one staging buffer of 24 * qb^2 bytes
 *     (hipHostMalloc; qb the subspace block width, about 2 * k_cap) for the
 *     small q x q transfers of the solver, released by bmg_problem_destroy;
 *     when pinning fails the transfers use pageable memory instead.
 *   - Dense factors are row-major FP64: W is m x ld, H is n x ld, with the
 *     first k columns in use (ld >= k, ld a multiple of 8, rows 16-byte aligned).
 *   - Omega is CSR: row_ptr[m+1] int64, col[nnz] int32 sorted and duplicate-free
 *     within each row, val[nnz] FP64 observed values A_ij.
 *   - Work is issued on the problem's HIP stream; calls that return host
 *     scalars synchronise that stream before returning.
 *   - Errors: a negative bmg_status; bmg_last_error() gives a message
 *     (thread-local).  No C++ exception crosses the ABI.
 */
#ifndef BMG_H
#define BMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BMG_OK = 0,
  BMG_NOT_CONVERGED = 1, /* max_iter reached; outputs hold the last iterate        */
  BMG_EINVAL = -1,       /* bad argument (shape, CSR not sorted/duplicate-free, ...) */
  BMG_ENOMEM = -2,       /* workspace too small, or rank would exceed k_cap         */
  BMG_EDEVICE = -3,      /* a HIP call failed                                        */
  BMG_ENONFINITE = -4,   /* NaN/Inf in the observed values or in a reduction         */
  BMG_ECANCELLED = -5
} bmg_status;

/* Arithmetic of the sparse passes.  FP64: everything in FP64.  FP32: factors,
 * residual and sparse values stored and multiplied in FP32, every Gram,
 * Cholesky, eigen-decomposition and scalar reduction in FP64.  BF16: factors
 * kept in BF16 for the sparse passes (FP32 accumulation), with the residual and
 * objective recomputed in FP64 every refresh_every outer iterations. */
typedef enum { BMG_FP64 = 0, BMG_FP32 = 1, BMG_BF16 = 2 } bmg_precision;

typedef struct {
  int64_t m, n, nnz;
  const int64_t *row_ptr; /* (device) [m+1] */
  const int32_t *col;     /* (device) [nnz] */
  const double *val;      /* (device) [nnz] */
} bmg_csr;

typedef struct bmg_problem bmg_problem;

/* Step-size rule of the PG step (Algorithm 1, convex-lifting phase). */
typedef enum {
  BMG_STEP_FIXED = 0,  /* alpha at every step (Sec. 6.1: alpha = 1.99 for L = 1)      */
  BMG_STEP_SPARSA = 1  /* Suppl., the SpaRSA variant: from the second PG step on, the  *
                        * BB step of eq. proxBB (read as ||dX||^2 / <dX, d grad f>)   *
                        * clipped to [alpha_min, alpha_max], times sparsa_beta^i for   *
                        * the smallest i whose prox output satisfies eq. back with     *
                        * sparsa_delta, floored at alpha_min; every trial is a full    *
                        * subspace iteration + prox from the same warm start.  The     *
                        * stop residual ||X~ - X+|| is taken at the accepted step      */
} bmg_step_rule;

/* Solver of the BM phase (Algorithm 1; any solver meeting eq. nonincrease). */
typedef enum {
  BMG_BM_PSD = 0,    /* preconditioned steepest descent, exact line search, W step then H step */
  BMG_BM_POLYMF = 1  /* polyMF-SS (Sec. 6.1.1): block coordinate descent over the column pairs  *
                      * (w_j, h_j), direction = block gradient scaled by the diagonal of each   *
                      * half's block Hessian, step = exact minimiser of the block quartic      */
} bmg_bm_solver;

typedef struct {
  double lambda;        /* regularisation weight of (MC)                         */
  double alpha;         /* fixed PG step (Sec. 6.1: L = 1, alpha = 1.99)         */
  double tol;           /* stop when the relative optimality residual <= tol     */
  double ssi_tol_floor; /* floor of the subspace-iteration stopping tolerance    */
  double psi0;          /* initial safeguard noise level (Suppl. A.1.3: 0.1)     */
  int bm_epochs;        /* y: BM epochs per PG step (Sec. 6.1.1: 3)              */
  int max_iter;         /* outer iterations                                      */
  int ssi_max_iter;     /* subspace iterations per PG step                       */
  int k_init;           /* k_{-1}: width of the initial range finder             */
  int refresh_every;    /* BF16 mode: FP64 refresh period (outer iterations)     */
  int verbose;          /* print one line per outer iteration to stderr          */
  int timing;           /* time every sparse-pass kernel with HIP events         */
  int lmsvd_p;          /* p_t of Algorithm 2: history blocks of the subspace     *
                         * (0: block subspace iteration; at most 4, see below)   */
  uint64_t seed;        /* counter-based RNG seed (sketch and safeguard draws)   */
  int step_rule;        /* bmg_step_rule                                         */
  int bm_solver;        /* bmg_bm_solver                                         */
  double alpha_min;     /* SpaRSA: step bounds (alpha_min < 2 delta / L, L = 1)  */
  double alpha_max;
  double sparsa_beta;   /* SpaRSA: backtracking factor in (0, 1)                 */
  double sparsa_delta;  /* SpaRSA: delta of eq. back in (0, 1)                   */
  double dense_rows;    /* rows of Omega (on the shorter side) with at least     *
                         * dense_rows * (longer side) entries go to a dense      *
                         * panel (0: none; see bmg_problem_create)               */
} bmg_options;

typedef struct {
  int k;              /* final rank                                              */
  int iters;          /* outer iterations done                                   */
  int ssi_iters;      /* subspace iterations summed over all PG steps            */
  int status;         /* bmg_status of the solve                                 */
  double F;           /* objective of (MC) at the returned X = W H^T             */
  double F_bm;        /* BM objective after the last BM phase                    */
  double residual;    /* last relative optimality residual                       */
  double eps;         /* last ||Z~ - Z||_F (inexactness of the last PG step)     */
  double seconds;     /* wall time of the solve                                  */
  double sparse_bytes;/* algorithmic bytes moved by the sparse passes            */
  int sparse_passes;  /* number of sparse passes launched                        */
  /* with opt->timing: per kernel class (0 fused residual+product of the BM
   * gradient, 1 sampled residual / curvature, 2 sparse x dense of the subspace
   * iteration) the summed kernel time from HIP events on the problem's stream,
   * the algorithmic bytes of those launches, and their count */
  double kernel_ms[3];
  double kernel_bytes[3];
  int kernel_launches[3];
  /* host time of the solve in the q x q FP64 linear algebra, and waiting for
   * the device (the synchronisations that bring small results to the host),
   * and the number of those synchronisations */
  double host_la_seconds;
  double host_wait_seconds;
  int host_syncs;
  int pg_trials;      /* prox computations summed over all PG steps (backtracking) */
  double alpha_last;  /* step of the last PG step                                */
  int bf16_passes;    /* BMG_BF16: sparse passes that gathered BF16 operands      */
} bmg_result;

/* Fills the defaults: alpha 1.99, tol 1e-6, ssi_tol_floor 1e-12, psi0 0.1,
 * bm_epochs 3, max_iter 500, ssi_max_iter 50, k_init 8, refresh_every 5,
 * lmsvd_p 0, bm_solver BMG_BM_POLYMF, step_rule BMG_STEP_FIXED, alpha_min 1.99, alpha_max 1e3,
 * sparsa_beta 0.5, sparsa_delta 0.999.
 * BMG_STEP_SPARSA keeps the previous PG point (W, H and its residual) and the
 * warm start in the workspace: min(m,n) x qb, (m + n) x ld_k and 2 nnz elements
 * of the working precision (FP64 in BMG_FP64, FP32 otherwise), qb = 2 k_cap + 2
 * and ld_k = k_cap, each rounded up to a multiple of 16.
 * lmsvd_p = p >= 1 (Algorithm 2 with history, Suppl. A.1.2: the Ritz step runs
 * over ran(U^{t,i}, ..., U^{t,i-p}) with the basis of eqs. PUi and orth-W) keeps
 * (2p-1) blocks of min(m,n) x qb and 3p blocks of max(m,n) x qb elements in the
 * workspace.  Both regions are reserved when the workspace is sized with those
 * options (bmg_workspace_size / bmg_problem_create); a solve or prox step that
 * asks for more than was reserved fails with BMG_ENOMEM.  BMG_EINVAL for p
 * outside [0, 4]. */
void bmg_options_default(bmg_options *opt);

/* Bytes of device workspace a problem of this shape needs when the rank may
 * reach k_cap (subspace blocks hold up to 2*k_cap+1 columns).  k_cap is at most
 * 256 in BMG_FP64 and 512 in BMG_FP32 / BMG_BF16 (BMG_EINVAL beyond).
 * opt: (host) the options the problem will be solved with, or NULL for the
 * defaults; its lmsvd_p (history blocks, 0..4) and step_rule (SpaRSA state)
 * add the regions described at bmg_options_default.  (host) out. */
bmg_status bmg_workspace_size(int64_t m, int64_t n, int64_t nnz, int k_cap, bmg_precision prec,
                              const bmg_options *opt, size_t *bytes);

/* Validates the CSR (sorted, in range, duplicate-free, finite values), builds the
 * column-major copy of Omega used by the transposed products (a stable sort of
 * the column indices on the device), and the load-balancing plans of both
 * orientations.  opt: (host) as for bmg_workspace_size (NULL: defaults); it
 * fixes the variants the workspace holds.  ws: (device) workspace of at least
 * bmg_workspace_size(..., opt) bytes (BMG_ENOMEM otherwise); stream: a
 * hipStream_t (or NULL for the default stream).  The CSR arrays must stay alive
 * and unchanged while the problem exists.  m > n is allowed; the library then
 * works on the transpose internally (the paper assumes m <= n, Sec. 1) and the
 * W/H arguments of every call keep their user meaning. */
bmg_status bmg_problem_create(const bmg_csr *csr, int k_cap, bmg_precision prec,
                              const bmg_options *opt, void *ws, size_t ws_bytes, void *stream,
                              bmg_problem **out);
void bmg_problem_destroy(bmg_problem *p);

/* Sampled residual (the sparse gradient of the MC loss, Sec. 5.1):
 *   R[p] = w_i . h_j - A_ij for every stored entry p = (i, j) in CSR order.
 * R: (device) [nnz] FP64 or NULL (then only the sums are produced).
 * half_sq: (host) 1/2 sum R^2.  W (m x ld), H (n x ld): (device). */
bmg_status bmg_sddmm(bmg_problem *p, const double *W, const double *H, int k, int ld, double *R,
                     double *half_sq);

/* Sparse products with the Omega-supported matrix S whose values are given in
 * CSR order (S: (device) [nnz]):
 *   transpose = 0:  C (m x q) = S   B,  B (n x q)
 *   transpose = 1:  C (n x q) = S^T B,  B (m x q)
 * These are the products the subspace iteration needs from Z^T U and Z B
 * (Suppl. A.1.2).  B, C: (device), leading dimensions ldb, ldc (multiples of 8). */
bmg_status bmg_spmm(bmg_problem *p, const double *S, const double *B, int q, int ldb, double *C,
                    int ldc, int transpose);

/* BM phase of Algorithm 1: `epochs` epochs, each a W step then an H step of
 * preconditioned steepest descent on (MF) with exact line search (the only
 * requirement, eq. nonincrease, holds by construction).  W, H: (device), updated
 * in place.  F_bm: (host) BM objective after the last step. */
bmg_status bmg_bm_epochs(bmg_problem *p, double *W, double *H, int k, int ld, double lambda,
                         int epochs, double *F_bm);

/* The BM phase with the polyMF-SS solver instead: `epochs` sweeps over the
 * column pairs j = 0..k-1 (Sec. 6.1.1), each block moved to the exact minimiser
 * of the BM objective along its direction (a quartic in the step).  Same
 * arguments and outputs as bmg_bm_epochs; BMG_EINVAL for lambda <= 0. */
bmg_status bmg_polymf_epochs(bmg_problem *p, double *W, double *H, int k, int ld, double lambda,
                             int epochs, double *F_bm);

/* ------------------------------------------------------------------ kernel-estimation QSDP
 * BM-Global on  min f(X) + lambda tr(X)  over {X psd, <E, X> = 0} (QSDP section,
 * unit weights), f(X) = 1/2 sum over pairs (X_ii + X_jj - 2 X_ij - d_ij^2)^2, in the
 * BM form X = W W^T, W^T e = 0 (eq. bm2).  The problem must be BMG_FP64 and
 * square with Omega and its values symmetric: both (i, j) and (j, i) stored with
 * the value d_ij^2 (BMG_EINVAL otherwise). */

/* r (device, nnz, CSR order, or NULL) = ||w_i - w_j||^2 - d_ij^2 for every stored
 * entry; deg (device, n, or NULL) = the row sums of r; sumsq (host) = sum r^2
 * over stored entries (twice the sum over pairs).  W (device, n x ld). */
bmg_status bmg_rke_residual(bmg_problem *p, const double *W, int k, int ld, double *r, double *deg,
                            double *sumsq);

/* Algorithm 1 on that problem: the first PG step from X = 0 (subspace iteration
 * from J times an n x k_init Gaussian block), then per outer iteration bm_epochs
 * nonlinear conjugate-gradient steps on W with the exact (quartic) line search,
 * and one PG step with alpha = opt->alpha / (2 + 2 max degree) (a bound on
 * ||A^* A||), whose prox P_S+(J Z J) (Lemma PiX) comes from Algorithm 2 with
 * history opt->lmsvd_p (0 or 1; BMG_EINVAL otherwise) on the shifted operator,
 * started from [orth(J W), the rank safeguard column of eq. rt]; the positive
 * Ritz pairs give the new W and rank (so the rank grows by at most one per
 * step).  With lmsvd_p = 1 the newest Ritz value of the subspace iteration's
 * stop test is held to a tenth of the previous PG step.  Stops when
 * ||X~ - X+||_F / (alpha (1 + ||X~||_F + ||grad f~||_F)) <= opt->tol.
 * Uses opt->lambda, alpha, tol, bm_epochs, max_iter, ssi_max_iter, ssi_tol_floor,
 * k_init, seed, psi0, lmsvd_p, verbose; lmsvd_p = 1 needs a problem created with
 * lmsvd_p >= 1 reserved (BMG_ENOMEM otherwise).  W (device, n x ld) output,
 * *k_out its rank; res (host) fills k, iters, ssi_iters, status, F, residual,
 * seconds, sparse bytes/passes. */
bmg_status bmg_rke_solve(bmg_problem *p, double *W, int ld, const bmg_options *opt, int *k_out,
                         bmg_result *res);

/* Objective of (MC) at X = W H^T:  F = 1/2 ||P_Omega(X - A)||^2 + lambda ||X||_*,
 * the nuclear norm from the k x k core of thin QR factors of W and H. (host) F.
 * residual: (host) optional; the relative optimality residual at X,
 *   ||X - prox_{alpha lambda ||.||_*}(X - alpha grad f(X))||_F / (1 + ||X||_F + ||grad f(X)||_F)
 * (the norm of the prox-gradient mapping times alpha, the paper leaving the
 * residual of (MC) undefined in Sec. 6.1), from one inexact PG step at the
 * bmg_options_default step and subspace settings, warm-started from W as in
 * bmg_prox_step; W and H are not modified.  It needs lambda > 0. */
bmg_status bmg_objective(bmg_problem *p, const double *W, const double *H, int k, int ld,
                         double lambda, double *F, double *residual);

/* One inexact PG step (Algorithm 1, convex-lifting phase) from X~ = W H^T with
 * step alpha, warm-started from the columns of W only (eq. rt0 with no previous
 * prox output) plus one safeguard column drawn with the given seed/stream:
 * block subspace iteration to tolerance, exact SVD of the projected matrix and
 * soft-thresholding at alpha*lambda.  On return W, H hold the balanced factors
 * U sqrt(Sigma), V sqrt(Sigma) of the new iterate and *k_inout its rank.
 * sigma: (host) optional, receives the kept singular values (capacity k_cap).
 * residual: (host) optional, relative optimality residual at X~. */
bmg_status bmg_prox_step(bmg_problem *p, double *W, double *H, int *k_inout, int ld,
                         const bmg_options *opt, double *sigma, double *residual);

/* Algorithm 1 end to end: HMT + Nystrom initialisation (Suppl. A.1.4), then
 * outer iterations of y BM epochs + one inexact PG step with warm start
 * (eqs. rt0, rt0-1) and rank safeguard (eq. rt), until the relative optimality
 * residual <= opt->tol or opt->max_iter.  W (m x ld), H (n x ld): (device)
 * outputs; *k_out the rank.  res: (host) statistics. */
bmg_status bmg_solve(bmg_problem *p, double *W, double *H, int ld, const bmg_options *opt,
                     int *k_out, bmg_result *res);

/* ------------------------------------------------------------------ serving
 * A request loop over many completion problems of different shapes on one
 * GPU.  The caller gives the server one device arena; every admitted problem
 * lives in a first-fit allocation inside it (its CSR copy, W, H and its
 * workspace, sized for the request's own options), so admission is by HBM
 * footprint.  Requests are admitted in arrival order, a later request may be
 * admitted ahead of an earlier one that does not fit yet (backfill).  Each of
 * max_slots slots has its own HIP stream; a slot and its memory are reused as
 * soon as a problem finishes.  Every problem's computation is independent of
 * the others (own stream, own memory, deterministic kernels): a result is the
 * same alone and in the mix.  The paper has no serving loop; this one is an
 * addition for running many problems on one GPU. */
typedef struct bmg_server bmg_server;

typedef struct {
  int state;          /* 0 queued, 1 running, 2 done, 3 failed                  */
  int status;         /* bmg_status of the solve (when done or failed)          */
  int k;              /* rank of the result                                     */
  double queued_s;    /* submit -> admission                                    */
  double run_s;       /* admission -> result copied back                        */
  double total_s;     /* submit -> result copied back                           */
  size_t footprint;   /* arena bytes the request occupied                       */
  bmg_result result;
} bmg_request_info;

/* Arena bytes one request needs (CSR copy + factors at ld = k_cap rounded to 8
 * + workspace for the options opt, NULL: defaults).  (host) out. */
bmg_status bmg_server_footprint(int64_t m, int64_t n, int64_t nnz, int k_cap, bmg_precision prec,
                                const bmg_options *opt, size_t *bytes);
/* arena: (device) memory owned by the caller, kept alive until destroy.
 * threads = 1: each of the max_slots (1..64) slots is a host worker thread that
 * runs its solves to the end, and the sparse passes of the running problems
 * that are pending together share launches.  threads = 0: no threads; the
 * caller drives the server with bmg_server_tick. */
bmg_status bmg_server_create(void *arena, size_t arena_bytes, int max_slots, int threads,
                             bmg_server **out);
/* A server created with threads = 0: on the calling thread, admits queued
 * requests into free slots (arrival order, backfill by footprint; admission
 * copies the CSR and runs the initialisation) and advances every running solve
 * by one outer iteration of Algorithm 1 (BM epochs + one PG step), retiring
 * those that finish.  With worker threads it only reports.  running / queued:
 * (host, optional) requests running and waiting after the call. */
bmg_status bmg_server_tick(bmg_server *s, int *running, int *queued);
/* Copies the (host) CSR and queues the request; *ticket identifies it.
 * BMG_ENOMEM if the request could never fit in the arena. */
bmg_status bmg_server_submit(bmg_server *s, const bmg_csr *host_csr, int k_cap, bmg_precision prec,
                             const bmg_options *opt, uint64_t *ticket);
/* Non-blocking.  info: (host).  When the request is done and W_host/H_host are
 * non-null, the factors are copied out (m x ld and n x ld row-major, FP64,
 * columns beyond k zero). */
bmg_status bmg_server_poll(bmg_server *s, uint64_t ticket, bmg_request_info *info, double *W_host,
                           double *H_host, int ld);
/* Blocks until every submitted request is done or failed (with threads = 0 it
 * calls bmg_server_tick until then). */
bmg_status bmg_server_drain(bmg_server *s);
/* Peak number of concurrently running problems and peak arena bytes in use. */
bmg_status bmg_server_stats(bmg_server *s, int *peak_running, size_t *peak_bytes);
/* Shared launches of sparse passes so far, and the passes they ran (the
 * running problems' passes that are pending together of the same precision,
 * kind and width class share one launch).  (host) out, either may be NULL. */
bmg_status bmg_server_batch_stats(bmg_server *s, int64_t *launches, int64_t *passes);
/* Waits for running requests, drops queued ones, frees host state. */
void bmg_server_destroy(bmg_server *s);

/* ------------------------------------------------------------------ no allocation
 * For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.
 *
 * bmg_sddmm_static computes what bmg_sddmm computes (R[p] = w_i . h_j - A_ij for
 * every stored entry p = (i, j) in CSR order, half_sq = 1/2 sum R^2) straight
 * from a device CSR, with no problem object and no workspace.  Its scratch (the
 * per-wave partial sums, the reduction's stages and the CSR check's flag word)
 * is one static device array of BMG_STATIC_SCRATCH_BYTES per GPU, held until the
 * process ends; the call allocates nothing.  Every call on a GPU shares that
 * GPU's array and needs nothing in it to start at zero (each call clears its
 * flag word and writes every slot it later reads); calls that overlap on one
 * GPU (from several host threads or streams) race on it.
 *   csr: (host) struct of device arrays, as for bmg_problem_create, in the
 *        caller's orientation (m > n is fine); validated on the device first
 *        (BMG_EINVAL / BMG_ENONFINITE as bmg_problem_create reports them).
 *   W (m x ld), H (n x ld): (device) FP64 row-major, 16-byte aligned rows,
 *        0 <= k <= 256, ld >= k, ld a multiple of 8.
 *   R: (device) [nnz] FP64 or NULL (then only the sum).  half_sq: (host) or NULL.
 *   stream: a hipStream_t or NULL; the call synchronises it twice (after the
 *        CSR check and before returning half_sq).
 * Rows are processed in their own order, one lane team per row (long rows are
 * not split as in a problem's plan): the entries of R are bit for bit those of
 * bmg_sddmm; half_sq adds the same terms in another order.
 * BMG_ENOMEM (before any device work) when m > BMG_STATIC_MAX_ROWS. */
#define BMG_STATIC_SCRATCH_BYTES (2u << 20)
#define BMG_STATIC_MAX_ROWS 523120
bmg_status bmg_sddmm_static(const bmg_csr *csr, const double *W, const double *H, int k, int ld,
                            double *R, double *half_sq, void *stream);

/* Thread-local message of the last failing call on this thread. */
const char *bmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BMG_H */
