/*
 * sknr.h -- C ABI of libsknr: entropic optimal transport on one AMD MI355X
 * (gfx950) by log-domain Sinkhorn-Knopp (SK) and SK-NR(l), the spectral
 * warm start of Chhaibi, Gratton and Vaiter (arXiv 2506.14780).
 *
 * Problem (paper, Sec. 2).  Two discrete measures alpha = a (length n) and
 * beta = b (length m), probability vectors; a cost C (n x m), either stored
 * or built from point clouds x (n x d), y (m x d) as
 * C_ij = cost_scale * ||x_i - y_j||^2; a regularisation eps > 0 or an eps
 * schedule; a tolerance omega on the L1 marginal error
 * ||pi 1_m - a||_1 + ||pi^T 1_n - b||_1 (the convergence test of
 * Algorithm 4.1).
 *
 * Potentials follow the paper's convention (eq. Optimal_P_epsilon): they
 * are relative to a (x) b, so pi_ij = a_i b_j exp((f_i + g_j - C_ij)/eps).
 * Returned potentials are gauge-normalised to <f,a> = <g,b> (the dual is
 * invariant under (f,g) -> (f,g) + c(1,-1), Sec. 2).
 *
 * Conventions for every entry point:
 *   - Every function returns an int status (SKNR_OK = 0, SKNR_NOT_CONVERGED
 *     = 1 as a warning, negative values are errors) and never throws.
 *     On error, sknr_last_error() gives a message (thread-local).
 *   - Array pointers marked [device] are HIP device pointers of the
 *     context's device; pointers marked [host] are host memory.
 *   - Arrays are dense and row-major unless stated; the caller owns every
 *     input and output buffer.  The library never frees caller memory and
 *     does not keep pointers to it after the call returns, except where
 *     sknr_submit documents a copy.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are synchronous with respect to the host: when a call returns,
 *     its outputs are written and the stream is idle.
 *   - A context is not thread-safe; use one per host thread.
 *
 * Precision: the O(nm) sweeps run in FP32 with compensated (double-float)
 * potentials; FP64 is used for the small projected Newton / eigen systems,
 * for the scalar objective values that decide the Newton acceptance test,
 * and for the final marginal-error check and reported values.
 */
#ifndef SKNR_H_
#define SKNR_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define SKNR_OK 0
#define SKNR_NOT_CONVERGED 1   /* warning: outputs valid, tolerance not reached */
#define SKNR_EINVAL (-1)       /* invalid argument (message in sknr_last_error) */
#define SKNR_ENOMEM (-2)       /* device allocation failed / over budget */
#define SKNR_EDEVICE (-3)      /* HIP runtime error */
#define SKNR_EBUSY (-4)        /* serving queue full */
#define SKNR_ECANCELED (-5)    /* request cancelled */
#define SKNR_EINTERNAL (-6)    /* internal failure */

#define SKNR_MAX_STAGES 32     /* maximum length of an eps schedule */
#define SKNR_MAX_ELL 32        /* maximum number of low-frequency modes l */

/* --------------------------------------------------------------- problem */
enum sknr_cost_kind {
  SKNR_COST_STORED = 0,   /* C given as an n x m FP32 matrix */
  SKNR_COST_SQEUCLID = 1  /* C_ij = cost_scale * ||x_i - y_j||^2 built per tile */
};

/* How the cross term of the squared distance is formed when the cost is
 * built from points.  FP32 evaluates sum_k (x_ik - y_jk)^2 in FP32 in the
 * order k = 0..d-1; BF16 / BF16X3 form ||x||^2 + ||y||^2 - 2 x.y with the
 * x.y products on bf16 matrix cores with FP32 accumulation, from one bf16
 * term per coordinate (BF16) or a hi/lo bf16 split keeping hi*hi + hi*lo +
 * lo*hi (BF16X3).  AUTO picks FP32 for d < 16 and BF16X6 for d >= 16. */
enum sknr_xterm {
  SKNR_XTERM_AUTO = 0,
  SKNR_XTERM_FP32 = 1,
  SKNR_XTERM_BF16 = 2,
  SKNR_XTERM_BF16X3 = 3,
  SKNR_XTERM_BF16X6 = 4  /* hi + mid + lo bf16 split: hi*hi + hi*mid + mid*hi + hi*lo + lo*hi + mid*mid */
};
/* Matrix-core cost in detail (BF16, BF16X3, BF16X6): the points are
 * centred on mu, the FP64 mean of all n + m points rounded to bf16;
 * v = fl32(x - mu) is rounded to bf16 hi = bf16(v) (x~ = hi for BF16);
 * BF16X3 adds lo = bf16(v - hi) (x~ = hi + lo); BF16X6 adds mid =
 * bf16(v - hi) and lo = bf16(v - hi - mid) (x~ = hi + mid + lo); per point
 * n_i = fl32(cost_scale * ||x~_i||^2) with the norm summed in FP64; and
 *   C~_ij = fma(-2 fl32(cost_scale), x~_i . y~_j, n_i + n_j)
 * in FP32 with the dot product on matrix cores (FP32 accumulation, any
 * order; |error| <= (N - 1) u sum |products| over the N kept products,
 * dpad = d rounded up to 32, u = 2^-24), keeping hi*hi + hi*lo + lo*hi
 * (BF16X3) or hi*hi + hi*mid + mid*hi + hi*lo + lo*hi + mid*mid (BF16X6).
 * C~ is symmetric in the roles of x and y, so both c-transforms use the
 * same matrix. */

typedef struct sknr_problem {
  int64_t n;            /* number of source points / size of a (n >= 1) */
  int64_t m;            /* number of target points / size of b (m >= 1) */
  int32_t d;            /* point dimension (SQEUCLID only, 1 <= d <= 1024) */
  int32_t kind;         /* enum sknr_cost_kind */
  int32_t xterm;        /* enum sknr_xterm (SQEUCLID only) */
  int32_t on_host;      /* 0: C, x, y, a, b below are device pointers.  1: they
                           are host pointers; the call first copies them into a
                           staging block of device memory that the context
                           holds (and regrows) until sknr_ctx_destroy, so the
                           transfer over the host link is part of the call.
                           Not accepted by sknr_solve_noalloc. */
  const float* C;       /* [device] STORED: n x m FP32, row stride ldc */
  int64_t ldc;          /* STORED: row stride in elements (>= m) */
  const float* x;       /* [device] SQEUCLID: n x d FP32 */
  const float* y;       /* [device] SQEUCLID: m x d FP32 */
  double cost_scale;    /* SQEUCLID: positive multiplier (0 means 1) */
  const double* a;      /* [device] n FP64 weights, positive, sum 1 */
  const double* b;      /* [device] m FP64 weights, positive, sum 1 */
} sknr_problem;

/* ------------------------------------------------------------ solve opts */
enum sknr_warm_mode {
  SKNR_WARM_SEQUENTIAL = 0, /* V_l of stage s from the optimum of stage s-1 */
  SKNR_WARM_STATIC = 1,     /* V_l from a plain SK solve at eps_prime */
  SKNR_WARM_USER = 2        /* V_l given in opts.V0 for every stage */
};

typedef struct sknr_opts {
  const double* eps;      /* [host] eps schedule, n_eps values, each > 0 */
  int32_t n_eps;          /* 1 .. SKNR_MAX_STAGES */
  int32_t max_iter;       /* SK iterations allowed per stage (>= 1) */
  double tol;             /* omega: L1 marginal error target per stage (> 0) */
  int32_t ell;            /* l: number of low-frequency modes (0 = plain SK) */
  int32_t warm_mode;      /* enum sknr_warm_mode */
  double eps_prime;       /* STATIC: eps' of the warm-start solve */
  int32_t eig_oversample; /* extra subspace columns (0 -> 8) */
  int32_t eig_max_iter;   /* subspace iterations cap (0 -> 100) */
  double eig_tol;         /* subspace iteration stops when every leading Ritz
                             value rho_i^2 moves by less than
                             eig_tol * (1 - rho_i^2) (0 -> 0.1) */
  int32_t check_every;    /* iterations per host convergence poll (0 -> auto) */
  int32_t first_stage_nr; /* 1: SK-NR also on stage 0 (WARM_USER or WARM_STATIC) */
  const double* f0;       /* [device] optional n FP64 initial f at eps[0] (NULL -> 0;
                             see g0 for how the two combine) */
  const double* V0;       /* [device] WARM_USER: FP64 basis of l columns on the
                             semi-dual side (the smaller of n and m, Sec. 2):
                             n x ell when n <= m, m x ell (a basis for g)
                             otherwise; sknr_get_subspace returns one */
  uint64_t seed;          /* seed of the subspace-iteration start block */
  void* stream;           /* hipStream_t */
  int32_t nr_switch_iters;/* WARM_SEQUENTIAL only.  0: every stage after the
                             first runs SK-NR (the protocol of Sec. 5).  T > 0:
                             stages run plain SK until one needs more than T
                             iterations; the stages after it run SK-NR, each
                             with V_l from the optimum of the stage before.
                             SK counts grow as eps falls (Lemma 3.2, rate
                             rho_1^2), so the switch happens once.  The optimum
                             is the same; only the iterates differ. */
  int32_t newton_solver;  /* enum sknr_newton_solver: how the l x l Newton
                             system is solved (0 = Gauss-Jordan with the
                             Cholesky pivot test) */
  int32_t newton_max_iter;/* iterative solvers: step cap (0 -> 2 l for CG,
                             64 for Newton-Schulz) */
  double newton_rtol;     /* iterative solvers: CG stops at ||grad - G z|| <=
                             rtol ||grad||, Newton-Schulz at ||I - G^ X||_F <=
                             rtol (0 -> 1e-12) */
  double nr_min_gain;     /* WARM_SEQUENTIAL only.  0: off.  g > 0: a stage runs
                             its Newton steps only when the warm start's Ritz
                             values promise a rate gain (1 - rho_{l+1}^2) /
                             (1 - rho_1^2) >= g, the ratio of the SK-NR rate of
                             Theorem 4.2 to the SK rate of Lemma 3.2 (iteration
                             counts scale with 1 / (1 - rate)); otherwise the
                             stage runs plain SK.  rho_{l+1} is the first Ritz
                             value past the basis (rho_l when l = 32).  On a
                             spectrum that is flat past l (many near-degenerate
                             modes) the Newton steps cost more than they save. */
  const double* g0;       /* [device] optional m FP64 initial g at eps[0].  The
                             iteration runs on the potential of the semi-dual
                             side (f when n <= m, g otherwise).  If that side's
                             initial potential is given it is used and the other
                             one is ignored; if only the other side's is given,
                             the solve starts from its c-transform (eq. foc_f,
                             or foc_g for n > m), half an SK step; with neither,
                             from 0. */
} sknr_opts;

/* Solvers of the projected Newton system G c = eps grad (Algorithm 4.1, NR
 * update).  DIRECT eliminates (Gauss-Jordan without pivoting; its pivots
 * are those of G = L D L^T, so the positive-definiteness test is
 * Cholesky's).  CG and NEWTON_SCHULZ are the GPU friendly alternatives the
 * paper names for the NR step (Sec. 4, disadvantages of the algorithm):
 * Jacobi-preconditioned conjugate gradients, and Newton-Schulz iterative
 * inversion X <- X (2 I - G^ X) of the Jacobi-scaled G^ = D^-1/2 G D^-1/2;
 * both use only products of G with vectors or matrices and need no
 * pivoting.  A direction with p^T G p <= 0 (CG), a residual above 1e-6
 * after the step cap (Newton-Schulz) or a non-positive diagonal fails the
 * positive-definiteness test, and the step is not tried. */
enum sknr_newton_solver {
  SKNR_NEWTON_DIRECT = 0,
  SKNR_NEWTON_CG = 1,
  SKNR_NEWTON_SCHULZ = 2
};

typedef struct sknr_stage_stats {
  double eps;
  int32_t iters;          /* SK iterations of Algorithm 4.1 in this stage */
  int32_t newton_tried;   /* projected Newton steps attempted */
  int32_t newton_accepted;/* ... and accepted by the Q^semi test */
  int32_t eig_iters;      /* subspace iterations of the warm start feeding this stage */
  double marginal_err;    /* L1 marginal error at the end of the stage: the FP64
                             check for the last stage, the sweeps' FP32
                             estimate for the others */
  double seconds;         /* wall time of the stage (incl. its warm start) */
  double rate_gain;       /* (1 - rho_{l+1}^2) / (1 - rho_1^2) from the Ritz values
                             of this stage's sequential warm start (0: none) */
  int32_t nr_skipped;     /* 1: the nr_min_gain test ran this stage as plain SK */
  int32_t reserved0;
} sknr_stage_stats;

typedef struct sknr_result {
  int32_t status;
  int32_t n_stages;
  int32_t total_iters;
  int32_t transposed;       /* 1 when solved on the transpose (n > m) */
  sknr_stage_stats stage[SKNR_MAX_STAGES];
  double marginal_err;      /* FP64 L1 marginal error vs the solver's cost */
  double row_err;           /* ||pi 1 - a||_1 (FP64) */
  double col_err;           /* ||pi^T 1 - b||_1 (FP64) */
  double transport_cost;    /* <C, pi> (FP64) */
  double dual_value;        /* Q_eps(f, g), eq. def_Q (FP64) */
  double primal_value;      /* <C,pi> + eps KL(pi || a(x)b) (FP64) */
  double mass;              /* sum_ij pi_ij */
  double marginal_err_exact;   /* FP64 L1 marginal error vs the exact cost (SQEUCLID:
                                  FP64 squared distances of the FP32 points; STORED:
                                  equal to marginal_err) */
  double transport_cost_exact; /* <C, pi> on that exact cost */
  double seconds;           /* wall time of the solve itself */
  double queue_seconds;     /* serving: submit -> start of the solve (0 for sknr_solve) */
  double latency_seconds;   /* serving: submit -> completion (0 for sknr_solve) */
} sknr_result;

/* --------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * device memory the context may hold for workspaces and queued serving
 * requests (0 = 90% of the free memory at creation).  *out receives the
 * context.  Errors: EINVAL (bad device), EDEVICE. */
int sknr_ctx_create(int device, uint64_t hbm_budget_bytes, void** out);

/* Destroy a context, waiting for outstanding work and freeing its memory. */
int sknr_ctx_destroy(void* ctx);

/* ----------------------------------------------------------- full solves */

/* Solve the EOT problem along the eps schedule of `opts` (Sec. 5 "sequential
 * warm start"): stage s starts from the potentials of stage s-1; with
 * ell > 0 stages run Algorithm 4.1 with V_l from the spectral warm start
 * (Sec. 4) chosen by warm_mode, otherwise plain SK (eq. SK_iterations).
 * The first stage is plain SK unless first_stage_nr is set with WARM_USER.
 * With nr_switch_iters = T > 0 (WARM_SEQUENTIAL) easy stages stay plain SK:
 * the warm start and the Newton steps begin at the stage after the first
 * one that needs more than T SK iterations.
 * f_out [device] n FP64 and g_out [device] m FP64 receive the potentials of
 * the last stage, res [host] the statistics.  When n > m the solve runs on
 * the transposed problem (semi-dual on the smaller side, Sec. 2); outputs
 * are always in the caller's orientation.
 * Returns OK, NOT_CONVERGED (some stage hit max_iter), or an error. */
int sknr_solve(void* ctx, const sknr_problem* prob, const sknr_opts* opts,
               double* f_out, double* g_out, sknr_result* res);

/* The same solve without device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Arguments, results and errors
 * as sknr_solve; the caller still provides the inputs and f_out / g_out.
 * The workspace lives in a static device array of the library (64 MiB per
 * device, held from the first context on that device until the process
 * ends) instead of the context's workspace allocation, and no iteration
 * graphs are captured (instantiation may allocate).  A problem whose
 * workspace exceeds the array is rejected with SKNR_EINVAL and a message
 * naming its size (about (n + m) (100 + 64 l) bytes plus the split
 * partials: a 4096 x 4096 problem with l = 16 needs about 12 MiB).
 * Every call on one device shares that device's array: calls that overlap
 * on one device (from several contexts or threads) race, so issue them one
 * at a time per device. */
int sknr_solve_noalloc(void* ctx, const sknr_problem* prob, const sknr_opts* opts,
                       double* f_out, double* g_out, sknr_result* res);

/* ------------------------------------------- single steps of the path */

/* Row c-transform f = g^{C,eps} (eq. foc_f), one FP32 sweep with
 * compensated accumulation:  f_i = -eps log sum_j b_j exp((g_j - C_ij)/eps).
 * g [device] m FP64 in, f_out [device] n FP64 out. */
int sknr_c_transform_row(void* ctx, const sknr_problem* prob, double eps,
                         const double* g, double* f_out, void* stream);

/* Column c-transform g = f^{C,eps} (eq. foc_g), fused with the marginal
 * error of the pair (f, g_prev):  err = sum_j b_j |exp((g_prev_j - g_j)/eps)
 * - 1| = ||pi(f,g_prev)^T 1 - b||_1 when f = g_prev^{C,eps} (the test of
 * Algorithm 4.1), and with <g, b>.  f [device] n FP64, g_prev [device] m
 * FP64 or NULL (err then 0), g_out [device] m FP64; err_out and gdot_out
 * [host] scalars or NULL. */
int sknr_c_transform_col(void* ctx, const sknr_problem* prob, double eps,
                         const double* f, const double* g_prev, double* g_out,
                         double* err_out, double* gdot_out, void* stream);

/* Semi-dual value and its gradient / Hessian restricted to span(V)
 * (eq. def_Q_semi, dQ_semi, d2Q_semi; Algorithm 4.1, computing the value
 * and the derivatives on V_l):
 *   qsemi = <f,a> + <f^{C,eps}, b>,
 *   grad  = V^T (a - P~ 1_m),               P~ = pi(f, f^{C,eps}),
 *   G     = -eps V^T (grad^2 Q^semi) V = V^T diag(P~ 1) V - W^T diag(b)^-1 W,
 *           W = P~^T V.
 * f [device] n FP64, V [device] n x ell FP64 (1 <= ell <= 32);
 * G_out [host] ell x ell, grad_out [host] ell, qsemi_out [host] scalar. */
int sknr_projected_system(void* ctx, const sknr_problem* prob, double eps,
                          const double* f, const double* V, int32_t ell,
                          double* G_out, double* grad_out, double* qsemi_out,
                          void* stream);

/* One projected Newton-Raphson step with the acceptance test of Algorithm
 * 4.1: Delta f = eps V G^-1 grad (Cholesky, FP64), f' = f + Delta f, kept
 * iff Q^semi(f') > Q^semi(f).  f_inout [device] n FP64 is replaced by f'
 * when accepted.  accepted/q0/q1 [host] may be NULL. */
int sknr_newton_step(void* ctx, const sknr_problem* prob, double eps,
                     double* f_inout, const double* V, int32_t ell,
                     int32_t* accepted, double* q0, double* q1, void* stream);

/* The coefficients c of the projected Newton step Delta f = V c (Algorithm
 * 4.1, NR update; G and grad as in sknr_projected_system), c = eps G^-1
 * grad, computed by `solver` (enum sknr_newton_solver; max_iter and rtol
 * as in sknr_opts, 0 for the defaults).  f [device] n FP64, V [device]
 * n x ell FP64; coef_out [host] ell; ok_out [host] 1 when G passed the
 * solver's positive-definiteness test (0: coef_out is not a step);
 * iters_out [host] iterations of an iterative solver (0 for DIRECT), may
 * be NULL. */
int sknr_newton_coef(void* ctx, const sknr_problem* prob, double eps,
                     const double* f, const double* V, int32_t ell, int32_t solver,
                     int32_t max_iter, double rtol, double* coef_out, int32_t* ok_out,
                     int32_t* iters_out, void* stream);

/* Spectral warm-start basis (Sec. 4): at the pair (f, f^{C,eps}) the top
 * ell non-constant eigenvectors of M = diag(a)^-1 P diag(b)^-1 P^T (the
 * semi-dual Hessian at the optimum is -(1/eps) diag(a) (Id - M), eq.
 * semidual_Hessian) by block subspace iteration with ell + oversample
 * columns and FP64 Rayleigh-Ritz, stopped when every leading Ritz value
 * rho_i^2 moves by less than tol * (1 - rho_i^2) or after max_iter.  Modes
 * below what the FP32 products resolve (rho_i^2 below ~1e-4 rho_1^2) come
 * back as zero columns.  V_out [device] n x ell FP64 (nonzero columns
 * orthonormal in L2(a), orthogonal to constants, descending rho);
 * rho_out [host] ell+1 values sqrt(eigenvalue), rho_out[0] = 1 for the
 * constant mode; iters_out [host] subspace iterations used (may be NULL). */
int sknr_spectral_basis(void* ctx, const sknr_problem* prob, double eps,
                        const double* f, int32_t ell, int32_t oversample,
                        int32_t max_iter, double tol, uint64_t seed,
                        double* V_out, double* rho_out, int32_t* iters_out,
                        void* stream);

/* The basis V_l that the last sknr_solve on this context held at its end:
 * that of its last stage that ran SK-NR steps or a warm start (sequential
 * or static warm start: Ritz vectors of M, orthonormal in L2(alpha) and
 * orthogonal to the constants, Sec. 4; WARM_USER: opts.V0 rounded to FP32).
 * It lives on the semi-dual side: rows = min(n, m) of that solve (the x
 * side when n <= m, else the y side), columns = its ell.  V_out [device]
 * rows x ell FP64, row-major; side_out [host] (nullable) gets 0 for the x
 * side, 1 for the y side.  The basis can be passed back as opts.V0 with
 * WARM_USER (Algorithm 4.1 takes V_l as an input; Sec. 4 reuses one basis
 * across eps).  EINVAL when that solve ran no SK-NR stage, when rows / ell
 * do not match, or when another call has used the context since (the
 * basis lives in the context's workspace, which the next call reuses). */
int sknr_get_subspace(void* ctx, double* V_out, int64_t rows, int32_t ell, int32_t* side_out, void* stream);

typedef struct sknr_eval {
  double row_err, col_err, marginal_err;   /* L1 marginal errors */
  double transport_cost, dual_value, primal_value, mass;
  /* the same marginal errors and <C,pi> on the exact cost (SQEUCLID: FP64
   * squared distances of the FP32 points; STORED: copies of the above) */
  double row_err_exact, col_err_exact, marginal_err_exact, transport_cost_exact;
} sknr_eval;

/* FP64 evaluation of a pair (f, g) on the solver's cost C~ (the FP32 or
 * matrix-core cost the sweeps use, per xterm): marginal errors, <C,pi>,
 * Q_eps (eq. def_Q) and the primal value <C,pi> + eps KL(pi||a(x)b)
 * (eq. primal_EOT); plus marginal errors and <C,pi> on the exact cost.
 * f, g [device] FP64; out [host]. */
int sknr_evaluate(void* ctx, const sknr_problem* prob, double eps,
                  const double* f, const double* g, sknr_eval* out, void* stream);

/* The coupling pi (eq. Optimal_P_epsilon) as FP32: P_out [device] n x m
 * row-major.  Diagnostic; O(nm) memory. */
int sknr_coupling(void* ctx, const sknr_problem* prob, double eps,
                  const double* f, const double* g, float* P_out, void* stream);

/* Gradients of W_eps (eq. primal_EOT / dual_EOT) with respect to the
 * problem data: the partial derivatives of Q_eps (eq. def_Q) at the given
 * potentials, which at the optimum are the derivatives of W_eps (the
 * potentials are stationary, so no implicit differentiation of the solver
 * is needed; the paper notes SK-NR cannot be differentiated through its
 * loop).  On the solver's cost C~:
 *   grad_x[i,k] = 2 s (r_i x_ik - sum_j pi_ij y_jk)     (n x d, SQEUCLID only)
 *   grad_y[j,k] = 2 s (c_j y_jk - sum_i pi_ij x_ik)     (m x d, SQEUCLID only)
 *   grad_a[i]   = f_i - eps r_i / a_i,  grad_b[j] = g_j - eps c_j / b_j
 * with s = cost_scale and r, c the row and column sums of pi; dW/dC is the
 * coupling (sknr_coupling).  f, g [device] FP64 in the caller's
 * orientation; each output [device] FP64 row-major, or NULL to skip it.
 * The weighted sums run in the sweep kernels, 32 coordinates per pass.
 * Errors: SKNR_EINVAL for a missing f or g, or point gradients of a stored
 * cost. */
int sknr_gradient(void* ctx, const sknr_problem* prob, double eps,
                  const double* f, const double* g, double* grad_x, double* grad_y,
                  double* grad_a, double* grad_b, void* stream);

/* -------------------------------------------------------------- serving */
/* Continuous batching of independent solves (mixed n, m, d, cost kind and
 * eps schedule) on one device.  The context runs `max_active` worker lanes,
 * each with its own HIP stream; device memory for requests comes from one
 * pool allocated at the first submit.  A queued request is admitted, in
 * arrival order with bounded backfilling, as soon as a lane is idle and its
 * footprint (inputs, workspace and outputs) fits in the pool; admitted
 * requests run concurrently, their kernels overlapping on the device, and
 * each runs exactly the schedule sknr_solve would (Sec. 5 sequential or
 * static warm start, Algorithm 4.1 per stage), so its result does not
 * depend on the other requests.  The serving calls below are thread-safe
 * with respect to each other. */

/* Configure serving before the first submit on ctx: max_active lanes (1 ..
 * 64, 0 -> env SKNR_SERVE_LANES or 8) and the pool size in bytes (0 ->
 * min(budget, 8 GiB)).  Errors: EBUSY once serving has started, EINVAL. */
int sknr_serve_config(void* ctx, int32_t max_active, uint64_t pool_bytes);

/* Batched execution (1) or per-lane launches (0, the default), before the
 * first submit on ctx.  Batched: the lanes still drive their requests'
 * schedules, but their iteration chunks (SK and SK-NR iterations of
 * Algorithm 4.1) are handed to one batcher thread, which runs the same
 * phase of all requests with the same kernel sequence as one launch per
 * kernel over a tile table (Sec. 4: several EOT problems solved
 * simultaneously); every request is gated by its own device state and
 * computes exactly what its own launches would.  Requests whose chunks
 * use a kernel without a batched form (the row sweep of a stored cost)
 * launch on their lane.  Measured on the 2048-request mixed trace (closed
 * loop, SK-NR): 190-215 solves/s batched (3.6-9 requests per batch with
 * 8-32 lanes) against 370 with per-lane launches: a batch still runs each
 * iteration as a chain of about 16 dependent launches on one stream, where
 * per-lane launches overlap 8 such chains on the hardware queues, and the
 * warm starts stay per lane.  Errors: EBUSY once serving has started,
 * EINVAL. */
int sknr_serve_batching(void* ctx, int32_t batched);

/* Queue one solve.  prob and opts as for sknr_solve (opts.f0, opts.V0 and
 * WARM_USER are not accepted; opts.stream orders the copy of the inputs).
 * The inputs are validated and deep-copied before the call returns, so
 * the caller may free them at once.  *ticket identifies the request.
 * Errors: EINVAL, ENOMEM (footprint larger than the pool), EDEVICE. */
int sknr_submit(void* ctx, const sknr_problem* prob, const sknr_opts* opts, uint64_t* ticket);

/* *done = 1 when the request has finished (converged, not converged,
 * failed or cancelled), else 0.  Errors: EINVAL (unknown ticket). */
int sknr_poll(void* ctx, uint64_t ticket, int32_t* done);

/* Block until the request finishes, copy its potentials into f_out [device]
 * n FP64 and g_out [device] m FP64 (either may be NULL) and its statistics
 * into res [host] (may be NULL), release the request and return its status
 * (OK, NOT_CONVERGED, ECANCELED or the error it failed with).  The ticket
 * is invalid afterwards. */
int sknr_wait(void* ctx, uint64_t ticket, double* f_out, double* g_out, sknr_result* res);

/* Cancel a request: a queued request is dropped, a running one stops at
 * its next convergence poll.  sknr_wait still has to collect it (status
 * ECANCELED unless it had already finished). */
int sknr_cancel(void* ctx, uint64_t ticket);

typedef struct sknr_serve_info {
  int32_t lanes;        /* worker lanes */
  int32_t queued;       /* requests waiting for admission */
  int32_t running;      /* requests on the device */
  int32_t reserved0;
  int64_t completed;    /* requests finished since serving started */
  uint64_t pool_bytes;  /* size of the device pool */
  uint64_t pool_used;   /* bytes reserved now */
  uint64_t pool_peak;   /* largest reservation so far */
  int64_t batches;          /* batched execution: batches launched */
  int64_t batched_jobs;     /* ... iteration chunks (one per request) they carried */
  int64_t batched_launches; /* ... kernel launches they took */
} sknr_serve_info;

/* Snapshot of the serving runtime (all zero before the first submit). */
int sknr_serve_stats(void* ctx, sknr_serve_info* out);

/* ------------------------------------------------------------ profiling */
typedef struct sknr_kprof {
  char name[64];        /* kernel kind, e.g. "sweep_stream_points_l0" */
  int64_t launches;     /* launches timed */
  double total_ms;      /* summed duration (HIP events on the launch stream) */
  double units;         /* algorithmic cost elements processed (n_out * n_red per sweep) */
} sknr_kprof;

/* Enable (1) or disable (0) per-kernel timing: every c-transform sweep
 * launched by this context is bracketed by HIP events recorded on its
 * stream, and durations are accumulated per kernel kind.  Resets the
 * accumulated table.  Adds two event records per sweep. */
int sknr_profile(void* ctx, int32_t enable);

/* Copy up to max_entries accumulated entries into out [host]; *count
 * [host] receives the number of kinds recorded. */
int sknr_profile_read(void* ctx, sknr_kprof* out, int32_t max_entries, int32_t* count);

/* ---------------------------------------------------------------- errors */
const char* sknr_status_str(int status);
const char* sknr_last_error(void);

/* Library version string. */
const char* sknr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SKNR_H_ */
