/*
 * jlanczos.h -- C ABI of the MI355X (gfx950) thick-restart Lanczos solver for
 * Hermitian J-symmetric eigenproblems (TRLAN-JSYM, Ishikawa & Sogabe,
 * arXiv:2001.07428).
 *
 * Problem (Sec. 1): A in C^{n x n} Hermitian with J A J^-1 = A^T, J real,
 * J^T = -J = J^-1 (eq. symmetry).  With the canonical J = [[0, -I], [I, 0]]
 * (n even, J acts as [a; b] -> [-b; a]) A has the block form
 * A = [[A11, A12], [A12^H, A11^T]], A11^H = A11, A12^T = -A12 (eq. blockform).
 * Every eigenvalue is doubly degenerate; the partner of an eigenvector x is
 * y = J x^* (eq. pairev).  The solver runs the Lanczos iteration inside one of
 * the two J-split Krylov subspaces (Algorithms 1 and 2) and returns the nev
 * lowest (or largest) distinct pair eigenvalues with one eigenvector each.
 *
 * Conventions for every entry point
 *  - Return value: JL_OK (0) on success, a negative jl_status on error, a
 *    positive jl_status for a result that is valid but qualified.  On error
 *    the message is available from jl_last_error(ctx).
 *  - Complex numbers are interleaved (re, im).  JL_C64 = two floats,
 *    JL_C128 = two doubles.  The operator dtype also selects the solver
 *    precision: JL_C64 stores and applies the operator and the Lanczos basis
 *    in FP32 complex, while the reorthogonalisation inner products, norms,
 *    residual checks and the Ritz eigenproblem are FP64; JL_C128 is FP64
 *    throughout.
 *  - Vectors are [top; bottom] with halves of length n/2 (Sec. 1, the block
 *    form); for the stencil each half is site-major (x0 slowest, x3
 *    fastest) with the internal index fastest.  Blocks of vectors are
 *    column-major with a leading dimension in elements.
 *  - "device" pointers are HIP device memory on the context's device;
 *    "host" pointers are ordinary host memory.  The library never takes
 *    ownership of caller buffers; dense operator data are borrowed for the
 *    lifetime of the operator, other buffers for the duration of the call.
 *  - All GPU work is ordered after the context's stream.  Calls that return
 *    host results (jl_solve) wait for their own work before returning.
 *  - The solver's scratch space is the caller's workspace (size from
 *    jl_workspace_bytes).  Device memory the library itself holds:
 *      . the stencil operator's tiled copy of its links, 64 V complex
 *        elements (twice that with per-site B), jl_op_create_stencil until
 *        jl_op_destroy;
 *      . the Case B operator's padded links, product matrices, projection
 *        tables and product jobs, about 56 Np^2 complex elements
 *        (Np = N rounded up to 64), jl_op_create_tek until jl_op_destroy;
 *      . a static 17.5 MB scratch array per GPU for the allocation-free
 *        entry point (jlanczos_kernels.h), part of the loaded library;
 *      . HIP events, streams and the batch's captured graph.
 *    Pinned host memory: a few scalars per jl_solve call, and a batch's
 *    results (jl_batch_create until jl_batch_destroy).
 */
#ifndef JLANCZOS_H
#define JLANCZOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t jl_status;
enum {
  JL_OK = 0,
  JL_EINVAL = -1,          /* invalid argument (message says which)        */
  JL_EHIP = -2,            /* a HIP runtime call failed                    */
  JL_ENOMEM = -3,          /* workspace smaller than jl_workspace_bytes    */
  JL_EUNSUPPORTED = -4,    /* valid request the library does not implement */
  JL_NOT_CONVERGED = 1,    /* max_cycles reached; first stats.icnv valid   */
  JL_BREAKDOWN = 2         /* invariant subspace reached before nev pairs  */
};

typedef enum { JL_C64 = 1, JL_C128 = 2 } jl_dtype;
typedef enum { JL_LOWEST = 0, JL_LARGEST = 1 } jl_which;

typedef struct jl_ctx_s* jl_ctx;
typedef struct jl_op_s* jl_op;

/* Context on HIP device `device`, ordering all work on `hip_stream`
 * (a hipStream_t, borrowed; NULL = the device's null stream).  jl_solve
 * issues its launches on a non-blocking stream the context owns (created on
 * first use, default priority), started after the work already queued on
 * hip_stream, and synchronises it before returning. */
jl_status jl_ctx_create(jl_ctx* out, int32_t device, void* hip_stream);
jl_status jl_ctx_destroy(jl_ctx ctx);
/* Last error message of `ctx` (or of the calling thread when ctx is NULL). */
const char* jl_last_error(jl_ctx ctx);
const char* jl_status_string(jl_status s);

/* Dense operator from the blocks of eq. (blockform).  A11 and A12 are device
 * pointers to h x h row-major complex matrices (h = n/2) with row stride
 * `ld` elements; A11 must be Hermitian and A12 antisymmetric (not checked).
 * Errors: JL_EINVAL for odd or non-positive n, ld < h, NULL pointers. */
jl_status jl_op_create_dense(jl_ctx ctx, int64_t n, const void* A11, const void* A12,
                             int64_t ld, jl_dtype dtype, jl_op* out);

/* Matrix-free 4D periodic J-stencil on an L[0] x L[1] x L[2] x L[3] lattice
 * with internal dimension d (n = 2 * V * d, V = prod L):
 *   A11 = diag I - sum_mu (U_mu T_mu + (U_mu T_mu)^H),
 *   A12 = a12_scale sum_mu (B_mu T_mu - (B_mu T_mu)^T),
 * (T_mu a)(x) = a(x + mu_hat) periodic.  U: device [4][V][d][d] row-major
 * complex links (unitarity not required); B: device [4][d][d] (b_per_site =
 * 0) or [4][V][d][d] (b_per_site = 1).  The result is Hermitian J-symmetric
 * by construction.  The operator keeps its own device copy of U and B in
 * tiles of 64 sites (within a tile the site is the fastest index; 64 V
 * complex elements of the dtype, V rounded up to 64, twice that with
 * per-site B; freed by jl_op_destroy), made on the ctx
 * stream before the call returns: U and B are not referenced afterwards.
 * Vectors passed to this operator must be 16-byte aligned.  Errors:
 * JL_EINVAL for L[i] < 2, 2^31 sites or more, or NULL pointers;
 * JL_EUNSUPPORTED for d != 4;
 * JL_ENOMEM when the link copy cannot be allocated. */
jl_status jl_op_create_stencil(jl_ctx ctx, const int32_t L[4], int32_t d, double diag,
                               double a12_scale, const void* U, const void* B,
                               int32_t b_per_site, jl_dtype dtype, jl_op* out);
/* The Case B operator of Sec. 4.2: A = D D^H (eq. TEKmatrix) with the
 * twisted Eguchi-Kawai Wilson-Dirac matrix of eq. (TEKWDmatrix),
 *   D = I - kappa sum_mu [(I - gamma_mu) (x) V_mu + (I + gamma_mu) (x) V_mu^T],
 * gamma_mu as in the appendix and V_mu the adjoint representation of U_mu:
 * V_mu(a, b) = 2 tr(T_a U_mu T_b U_mu^H) over the generalised Gell-Mann
 * basis T_a of su(N) (tr(T_a T_b) = delta_ab / 2; per spin N^2 - 1
 * coefficients: the symmetric (E_jk + E_kj)/2 for j < k in row-major order
 * of the strict upper triangle, the antisymmetric (-i E_jk + i E_kj)/2 in the
 * same order, the diagonal diag(1, ..., 1, -l, 0, ...)/sqrt(2 l (l+1)) for
 * l = 1..N-1).  n = 4 (N^2 - 1).  J = C gamma_5 pairs the spins (0, 1) and
 * (2, 3), so vectors are laid out as [psi_0; psi_2; psi_1; psi_3] (spin
 * blocks of N^2 - 1 coefficients), in which J is the canonical
 * [[0, -I], [I, 0]] of every other call here.
 *  U: device [4][N][N] row-major complex of the dtype (U_mu in SU(N); not
 *     checked), copied at creation (not referenced afterwards).
 * The operator owns 56 Np^2 complex elements of device scratch (Np = N
 * rounded up to 64), so two applies of one operator must not run at the
 * same time.  D is applied through (V_mu psi)_a T_a = U_mu X U_mu^H with
 * X = psi_b T_b, on the rank-2 spin projections of I -/+ gamma_mu: 64 N x N
 * complex products per apply of A, on the matrix cores in the storage
 * precision.  Errors: JL_EINVAL for N outside 2..1024
 * or NULL pointers, JL_ENOMEM when the scratch cannot be allocated. */
jl_status jl_op_create_tek(jl_ctx ctx, int32_t N, double kappa, const void* U, jl_dtype dtype,
                           jl_op* out);
jl_status jl_op_destroy(jl_op op);
/* Dimension n of the operator. */
jl_status jl_op_dim(jl_op op, int64_t* n);

/* y(:, r) = A x(:, r) for r < nrhs; x, y device, column-major with leading
 * dimension n (element type = operator dtype, accumulation in that
 * precision).  x and y must not overlap. */
jl_status jl_op_apply(jl_op op, const void* x, void* y, int32_t nrhs);

typedef struct {
  int32_t nev;          /* number of desired pairs (1 <= nev <= mwin)          */
  int32_t m;            /* maximum Krylov dimension (mwin < m <= n/2; with
                           standard, m <= n)                                   */
  int32_t mwin;         /* restart window: k = min(icnv + mwin, m - 1)         */
  int32_t which;        /* jl_which                                            */
  double tol;           /* residual tolerance: ||A x - lambda x|| < tol          */
  int32_t tol_relative; /* nonzero: the tolerance is tol * max |theta| over
                           every Ritz value of this and the earlier cycles (a
                           non-decreasing estimate of ||A||_2, so a pair
                           decoupled as converged stays converged)            */
  int32_t max_cycles;   /* outer-iteration cap (<= 0: 10000)                   */
  int32_t max_passes;   /* reorthogonalisation passes per step cap (<= 0: 16)  */
  int32_t min_passes;   /* passes before the sqrt(2) test applies (<= 0: 1)    */
  int32_t timing;       /* 1: time each kernel class with HIP events; s > 1:
                           the operator applies and reorthogonalisation
                           kernels only at every s-th Lanczos step (the other
                           classes at every launch), and then t_matvec,
                           t_dots, t_update, n_*_launch and bytes_* of those
                           three classes cover the timed launches only      */
  int32_t trace_cap;    /* record alpha_j, beta_j of the first trace_cap steps */
  double* trace_ab;     /* host [2 * trace_cap]: alpha then beta (may be NULL) */
  int32_t verbose;      /* nonzero: one progress line per cycle on stderr      */
  int32_t standard;     /* nonzero: the standard thick-restart Lanczos the
                           paper compares against (Sec. 3): no projection on
                           J V^*, so each pair is found twice; zero (the
                           default): the J-restricted method of Alg. 1/2     */
  int32_t invert;       /* nonzero: invert mode (Alg. 1 and 2, invert
                           branches; Sec. 4.2): every Lanczos step takes
                           u = A^-1 v_j by conjugate gradients, so A must be
                           Hermitian positive definite; the Ritz values theta
                           are those of A^-1, the pairs returned have
                           ev = 1/theta, the residual estimate is
                           ||A v_{m+1}|| |t_{m+1,i} ev_i| and the true residual
                           ||A x - ev x||.  which names the end of A's
                           spectrum (JL_LOWEST: the smallest eigenvalues).
                           With tol_relative the scale is the running max of
                           ||A v_{m+1}|| and the wanted |ev|.                */
  int32_t cg_maxit;     /* CG iterations per solve cap (<= 0: 10000)            */
  double cg_tol;        /* CG stops once ||v_j - A u|| <= cg_tol ||v_j|| on the
                           recursively updated residual (<= 0: tol)           */
  int32_t b0_rule;      /* the norm b0 the first sqrt(2) test of Alg. 2 compares
                           against: 0 (default) after the local three-term step
                           u - t_jj v_j - beta_{j-1} v_{j-1}; 1 after
                           u - t_jj v_j alone, as Alg. 2 prints it (the first
                           pass then also removes the beta_{j-1} v_{j-1} part,
                           so about every other step takes a second pass)      */
  int32_t basis_cycle;  /* > 0: export the Lanczos decomposition of this outer
                           iteration (1-based), taken after its last Lanczos
                           step and before its Rayleigh-Ritz step:            */
  void* basis_out;      /*   device n x (m + 1), leading dimension n, op dtype:
                           columns 0 .. m_eff of V (m_eff = m unless the
                           iteration broke down); may be NULL               */
  double* T_out;        /*   host (m + 1) x m column-major FP64: the projected
                           matrix Tbar (lower triangle: t_jj, t_{j+1,j} and the
                           restart row t_{k+1,i}; the rest zero); may be NULL */
  int32_t cycle_times_cap;  /* entries of cycle_times                        */
  double* cycle_times;  /* host [cycle_times_cap] or NULL: wall time [s] from the
                           start of jl_solve to the end of outer iteration c
                           (its convergence check done, the device idle), at
                           cycle_times[c - 1]                                */
} jl_params;

typedef struct {
  int32_t cycles;       /* outer iterations N_conv                              */
  int32_t n_mv;         /* Lanczos matvecs N_MV (residual checks excluded)      */
  int32_t n_resid;      /* operator applies spent on true-residual checks       */
  int32_t gs_passes;    /* reorthogonalisation passes over all steps            */
  int32_t icnv;         /* converged pairs at return                            */
  int32_t status;       /* same as the return value of jl_solve                 */
  int64_t sum_ncol;     /* sum over Lanczos steps of the basis width j + 1      */
  /* Per kernel class (only with params.timing): accumulated GPU time [s],
   * launch count and algorithmic bytes (or flops for the GEMM); with
   * params.timing = s > 1 the matvec, dots and update figures are those of
   * the timed launches. */
  double t_total;       /* wall time of jl_solve [s] (always set)               */
  double t_matvec, t_dots, t_update, t_gemm, t_ritz, t_resid;
  int64_t n_matvec_launch, n_dots_launch, n_update_launch, n_gemm_launch;
  double bytes_matvec, bytes_dots, bytes_update, flops_gemm;
  /* Invert mode: CG iterations over all solves (each one operator apply),
   * the most in one solve, solves stopped by cg_maxit, (with timing) the GPU
   * time of the CG solves [s], and their algorithmic bytes (per iteration
   * one operator apply, plus r read and p written by the direction step
   * fused into it, plus x, r, p, q read and x, r written by the update:
   * eight vector passes). */
  int64_t cg_iters;
  int32_t cg_max_iters;
  int32_t cg_unconverged;
  double t_cg;
  double bytes_cg;
} jl_stats;

/* Workspace bytes jl_solve needs for `op` and `p`. */
jl_status jl_workspace_bytes(jl_op op, const jl_params* p, size_t* bytes);

/* Thick-restart J-Lanczos (Algorithm 1 with Algorithm 2 as its inner step).
 * Each step subtracts the three-term recurrence t_jj v_j + beta_{j-1} v_{j-1}
 * (t_jj alone on the first step after a restart) before the iterated
 * Gram-Schmidt against [V_j, J V_j^*] of Alg. 2; the loop stops when
 * sqrt(2) * (norm after a pass) > (norm before it), the norm before the first
 * pass being the one after the local step (params.b0_rule = 0) or the one
 * after subtracting t_jj v_j alone (b0_rule = 1).  The basis update of the
 * restart computes only the Ritz vectors the next iteration keeps: first the
 * nev candidates (rounded up to the GEMM tile), then, once the convergence
 * check has fixed k = min(icnv + mwin, m - 1), the rest up to k.
 *  v1      device start vector (n, op dtype) or NULL for the all-ones vector
 *          the paper uses; it is normalised internally.
 *  ws      device workspace of ws_bytes >= jl_workspace_bytes.
 *  evals   host [nev]: pair eigenvalues in the desired order.
 *  X       device n x nev (leading dimension ldx >= n), op dtype: one unit
 *          eigenvector per pair; the partners are J X^* (jl_pair_vectors).
 *  res     host [nev]: true residual norms ||A x_i - lambda_i x_i|| (FP64).
 *  stats   host, may be NULL.
 * Returns JL_OK when all nev pairs converged, JL_NOT_CONVERGED after
 * max_cycles (the first stats.icnv entries are converged), JL_BREAKDOWN when
 * the Krylov space became invariant before nev pairs converged (converged
 * entries first).  Errors: JL_EINVAL for parameters outside the ranges
 * above or, in invert mode, when CG meets p^H A p <= 0 (A not positive
 * definite), JL_ENOMEM for a short workspace, JL_EHIP for runtime failures.
 * In invert mode "matvec" in n_mv means one solve A^-1 v_j (as Sec. 3 counts
 * it); the applications of A for ||A v_{m+1}|| count in n_resid. */
jl_status jl_solve(jl_op op, const jl_params* p, const void* v1, void* ws, size_t ws_bytes,
                   double* evals, void* X, int64_t ldx, double* res, jl_stats* stats);

/* Partner vectors Y = J X^* = [-conj(X_bottom); conj(X_top)] (eq. pairev) for
 * k columns; X, Y device, leading dimensions ldx, ldy >= n; may alias only if
 * X == Y and ldx == ldy. */
jl_status jl_pair_vectors(jl_ctx ctx, int64_t n, int32_t k, jl_dtype dtype, const void* X,
                          int64_t ldx, void* Y, int64_t ldy);

/* ------------------------------------------------------------------------
 * Batched solve: many independent dense problems of (possibly different)
 * even sizes, each A = [[A11, A12], [A12^H, A11^T]] with h_i x h_i row-major
 * contiguous blocks (device), solved with the same jl_params in one
 * persistent launch.  Every workgroup runs the whole of Algorithms 1 and 2
 * for the problems it takes from a shared queue, largest first.  The launch,
 * the queue reset and the result copies are captured once in a hipGraph at
 * jl_batch_create and replayed by every jl_batch_run.
 *
 * Limits: m + (m mod 2) <= 60, 2 <= n_i, m <= n_i / 2, nev <= mwin < m;
 * normal mode, J-restricted only (p->standard and p->invert must be 0, else
 * JL_EUNSUPPORTED).
 * The launch shape (jl_batch_shape, NULL for the defaults) holds the tuning
 * knobs the autotuner picks per batch.
 * X[i] (device, n_i x nev column-major, leading dimension n_i) receives the
 * eigenvectors of problem i; the operator and X pointers are borrowed until
 * jl_batch_destroy.  Errors: JL_EINVAL, JL_ENOMEM, JL_EHIP.
 * ------------------------------------------------------------------------ */
typedef struct jl_batch_s* jl_batch;

typedef struct {
  int32_t threads;          /* workgroup size: 128, 256 or 512 (0: 256)                */
  int32_t blocks;           /* persistent workgroups (0: min(count, 2 x compute units)) */
  int32_t rows_per_wave;    /* rows of [A11 A12] a wavefront applies at once: 1 or 2
                               (0: 1)                                                  */
  int32_t unroll;           /* column steps whose loads each lane issues together:
                               4 or 8 (0: 4)                                          */
  int32_t lds_matrix_bytes; /* LDS bytes per workgroup for a problem's whole
                               [A11 A12] (2 h^2 complex elements): a problem that fits
                               is read from LDS for its whole solve (0: none; a
                               multiple of 16, within the device's per-workgroup LDS
                               with the solver's own use)                         */
} jl_batch_shape;

typedef struct {
  int32_t cycles;       /* outer iterations                                     */
  int32_t n_mv;         /* Lanczos matvecs                                      */
  int32_t gs_passes;    /* reorthogonalisation passes                           */
  int32_t icnv;         /* converged pairs                                      */
  int32_t n_resid;      /* operator applies spent on true-residual checks       */
  /* Seconds the problem's workgroup spent in each phase, from the device's
   * constant-rate wall clock read where the workgroup is in step: the operator
   * apply of the Lanczos steps; the J-restricted Gram-Schmidt passes with the
   * normalisation (and the start and restart bookkeeping); the Rayleigh-Ritz
   * step (in-LDS Jacobi, sort); the restart product V_m Z; the true-residual
   * checks.  Their sum is the problem's time in the solver. */
  double t_apply, t_gs, t_ritz, t_restart, t_resid;
} jl_batch_stats;

jl_status jl_batch_workspace_bytes(int32_t count, const int64_t* n, jl_dtype dtype,
                                   const jl_params* p, const jl_batch_shape* shape, size_t* bytes);
jl_status jl_batch_create(jl_ctx ctx, int32_t count, const int64_t* n, const void* const* A11,
                          const void* const* A12, jl_dtype dtype, const jl_params* p,
                          void* const* X, void* ws, size_t ws_bytes, const jl_batch_shape* shape,
                          jl_batch* out);
/* The launch shape the batch uses, with the defaults resolved. */
jl_status jl_batch_shape_used(jl_batch b, jl_batch_shape* shape);
/* Runs the captured graph and waits for it.  evals, res: host [count * nev]
 * (problem-major, converged pairs first); status: host [count] (JL_OK,
 * JL_NOT_CONVERGED or JL_BREAKDOWN per problem); stats: host [count] or NULL.
 * Returns JL_OK if every problem converged, else JL_NOT_CONVERGED. */
jl_status jl_batch_run(jl_batch b, double* evals, double* res, int32_t* status,
                       jl_batch_stats* stats);
jl_status jl_batch_destroy(jl_batch b);

#ifdef __cplusplus
}
#endif

#endif /* JLANCZOS_H */
