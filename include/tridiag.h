/*
 * tridiag -- block-tridiagonal solver for AMD MI355X (gfx950), C ABI.
 *
 * Solves P X = F for one fixed block-tridiagonal matrix P and many right-hand
 * sides, with the matrix factored once and the factor reused for every F.
 * P is the matrix of eq. (main-eq) in Sec. 1 of A. V. Terekhov, "A fast
 * parallel algorithm for solving block-tridiagonal systems of linear
 * equations including the domain decomposition method": N block rows of
 * M x M blocks, block row j reading
 *
 *     -A_j X_{j-1} + C_j X_j - B_j X_{j+1} = F_j ,   j = 1..N,
 *
 * (note the minus signs on A and B; A_1 and B_N are not part of P and are
 * ignored).  The solver is the paper's Algorithm 2 (Sec. 2.2): the rows are
 * cut into p subdomains whose first rows are the interface rows; per
 * subdomain the sub-problems of eqs. (sub1)-(sub3) give U, V and W; the
 * interface unknowns solve the reduced system of eq. (red1) by the dichotomy
 * of Algorithm 1 (Sec. 2.1) with stored rows of the inverse; eq.
 * (superposition) then gives every other row.  Everything runs in HIP
 * kernels on one GPU; all pointers to matrix and vector data are DEVICE
 * pointers unless stated otherwise.
 *
 * Layouts (all float64):
 *   DENSE block field   : [N][M][M], block j column-major (entry (r,c) at j*M*M + r + c*M)
 *   DIAG block field    : [N][M], the diagonal of each block
 *   TRIDIAG block field : [N][3][M], (sub, diag, super): C_j(i,i-1) = [j][0][i],
 *                         C_j(i,i) = [j][1][i], C_j(i,i+1) = [j][2][i]; [j][0][0] and
 *                         [j][2][M-1] are ignored
 *   right-hand sides and solutions: column-major (N*M) x K with leading dimension
 *                         ld >= N*M; column k holds X_1..X_N of right-hand side k
 *
 * Threading: a plan may be used from one host thread at a time.  Calls are
 * stream-ordered on the HIP stream passed in (NULL = the default stream).
 */
#ifndef TRIDIAG_H
#define TRIDIAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TD_OK = 0,
  TD_EINVAL = 1,     /* an argument is out of range; nothing was launched */
  TD_ENOMEM = 2,     /* the plan or its workspace does not fit in free device memory */
  TD_ESINGULAR = 3,  /* a pivot block (or a block of the reduced system) is singular */
  TD_ENOCONV = 4,    /* iterative refinement did not reach the requested residual */
  TD_ENOADJ = 5,     /* an adjoint solve on a plan factored without the transpose */
  TD_EHIP = 6,       /* a HIP runtime call failed; tridiag_last_error() has its text */
  TD_ENOTSUP = 7     /* a valid but unsupported combination (for example M > 512) */
} td_status;

typedef enum { TD_FMT_DENSE = 0, TD_FMT_DIAG = 1, TD_FMT_TRIDIAG = 2 } td_format;

typedef enum { TD_PREC_F64 = 0, TD_PREC_F32 = 1, TD_PREC_BF16 = 2 } td_precision;

/*
 * Device memory callbacks (not in the paper).  When td_desc.dev_alloc and td_desc.dev_free are both
 * set, every device buffer of the plan (factor, compact input copies, solve and refinement workspaces,
 * the temporaries of the factor) is obtained from dev_alloc and returned through dev_free, so that a
 * caller's caching allocator (for example PyTorch's) holds and accounts for it; both NULL: hipMalloc /
 * hipFree.  dev_alloc(ctx, bytes, stream) returns a device pointer aligned to at least 256 bytes, or NULL
 * when the memory is not available (the library then frees what it holds and returns TD_ENOMEM).
 * `stream` is the hipStream_t (as void*) of the call that allocates; the library only frees a buffer
 * after the work that uses it on the plan's last stream has completed.  The callbacks are called from
 * tridiag_factor, tridiag_solve(_adjoint) (when the workspace grows) and tridiag_destroy, on the calling
 * host thread.
 */
typedef void* (*td_alloc_fn)(void* ctx, size_t bytes, void* stream);
typedef void (*td_free_fn)(void* ctx, void* ptr, void* stream);

/* Description of the matrix and of the plan to build. */
typedef struct {
  int64_t N;            /* block rows, >= 1 */
  int64_t M;            /* block size, 1 <= M <= 512 */
  int64_t subdomains;   /* p in [1, N]: number of subdomains of Algorithm 2; 0 = the library's default rule
                           for k_hint right-hand sides (tridiag_default_subdomains) */
  int32_t fmt_A;        /* TD_FMT_DENSE or TD_FMT_DIAG (DENSE A or B: sweep_prec must be F64,
                           else TD_ENOTSUP; every coupling then becomes a block product) */
  int32_t fmt_B;        /* TD_FMT_DENSE or TD_FMT_DIAG */
  int32_t fmt_C;        /* TD_FMT_DENSE or TD_FMT_TRIDIAG */
  int32_t sweep_prec;   /* TD_PREC_F64: plain float64 solve; TD_PREC_F32 / TD_PREC_BF16: the
                           subdomain sweeps and the superposition run on rounded copies of the
                           factor (float32 accumulation), see tridiag_solve */
  int32_t adjoint;      /* nonzero: also factor P^T so that tridiag_solve_adjoint can be used */
  int32_t reserved;     /* must be 0 */
  int64_t k_hint;       /* right-hand sides per solve the default subdomain count is chosen for (<= 0: 512) */
  td_alloc_fn dev_alloc; /* device memory callbacks (see above); both NULL = hipMalloc / hipFree */
  td_free_fn dev_free;
  void* alloc_ctx;      /* passed to dev_alloc / dev_free */
} td_desc;

/* Iterative refinement (used by tridiag_solve and tridiag_solve_adjoint). */
typedef struct {
  int32_t enable;       /* nonzero: refine in float64 until the residual test passes */
  int32_t max_iter;     /* at most this many correction solves (<= 0: 10) */
  double tol;           /* stop when max_k ||F_k - P X_k||_2 / ||F_k||_2 <= tol (<= 0: 1e-10) */
} td_refine;

/* Result report of one solve (host memory). */
typedef struct {
  int32_t iterations;          /* correction solves done after the first solve */
  int32_t nonfinite;           /* nonzero if F or the result held Inf/NaN */
  double max_col_rel_residual; /* max_k ||F_k - P X_k||_2 / ||F_k||_2 (float64), or -1 if not computed */
} td_info;

typedef struct td_plan_s* td_plan;

/*
 * Default number of subdomains for N block rows and K right-hand sides per solve (not in the paper,
 * which leaves p to the machine): p = N / L with L the longest of 32, 16 and 8 rows for which the
 * subdomain sweeps still get about 512 work-groups ((N / L) * ceil(K / 32) >= 512; else L = 8), clamped
 * to [1, N].  K <= 0 means 512.  This is the rule tridiag_factor applies for subdomains == 0.
 */
td_status tridiag_default_subdomains(int64_t N, int64_t K, int64_t* p);

/*
 * Device bytes a tridiag_factor with this description needs at its peak (the footprint it checks
 * against free device memory before allocating anything).  TD_EINVAL / TD_ENOTSUP as tridiag_factor.
 */
td_status tridiag_plan_bytes(const td_desc* desc, int64_t* bytes);

/*
 * Factor P once (Algorithm 2, preliminary step 1 of Sec. 2.2).
 *   desc    : host pointer to the description.
 *   A, B, C : device pointers to the blocks in the formats named by desc.  They are read
 *             during the call only; the plan keeps its own compact copies.
 *   stream  : hipStream_t (as void*), or NULL.
 *   out     : receives the plan (NULL on failure).
 * The call is synchronous: it returns after the factor is complete and its pivots have been
 * checked.  Before allocating, the footprint (tridiag_plan_bytes) is compared with the free device
 * memory (hipMemGetInfo): above 95% of it the call returns TD_ENOMEM and allocates nothing.
 * Returns TD_ESINGULAR if a diagonal block of the elimination (or of the reduced system) has a
 * pivot below 1e-14 times its infinity norm; tridiag_last_error() names the block row.  The plan owns all its device memory until tridiag_destroy.
 */
td_status tridiag_factor(const td_desc* desc, const double* A, const double* B, const double* C,
                         void* stream, td_plan* out);

/*
 * Solve P X = F for K right-hand sides (Algorithm 2, solution step 2 of Sec. 2.2).
 *   F, ldf : device, column-major (N*M) x K, ldf >= N*M.  Read only.
 *   X, ldx : device, column-major (N*M) x K, ldx >= N*M.  Written.  Must not overlap F.
 *   refine : host, may be NULL (= disabled).  For a plan with sweep_prec F32/BF16 and refine
 *            disabled, the result carries the rounding error of that precision.
 *   info   : host, may be NULL.  If non-NULL, or if refinement is on, the call computes the
 *            float64 residual and synchronises the stream before returning.
 * Without refinement and with info == NULL the call only enqueues work on the stream.
 * K == 0 is a no-op.  Returns TD_ENOCONV if refinement stops at max_iter above tol (X then
 * holds the last iterate).
 */
td_status tridiag_solve(td_plan plan, const double* F, int64_t ldf, double* X, int64_t ldx, int64_t K,
                        const td_refine* refine, td_info* info, void* stream);

/*
 * tridiag_solve without any device memory allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels as a plain
 * tridiag_solve (no refinement, no report), with the solve workspace placed in a fixed device array of
 * 64 MiB that the library holds on each GPU it runs on until the process ends, instead of the plan's
 * workspace.  F, X, ldf, ldx, K as in tridiag_solve; the result equals tridiag_solve's.  The workspace
 * a solve needs is ((p + 2) + p + chunks + slab slots) * Mp * K float64 words plus the sweep workspace
 * (N * Mp * K float64 words, or float32 words in panels of 64 columns for low-precision plans); above
 * 64 MiB the call returns TD_EINVAL and launches nothing.  Every call on one GPU shares that array
 * (it keeps the last call's contents; each call clears what must start at zero), so calls on one GPU
 * must not overlap: order them on one stream or synchronise between them.  Asynchronous on `stream`;
 * calls no hipMalloc / hipFree and no allocation callback.
 */
td_status tridiag_solve_noalloc(td_plan plan, const double* F, int64_t ldf, double* X, int64_t ldx, int64_t K,
                                void* stream);

/*
 * Solve P^T Lam = G (same conventions as tridiag_solve).  The transposed matrix is again
 * block tridiagonal with blocks C'_j = C_j^T, A'_j = B_{j-1}^T, B'_j = A_{j+1}^T.
 * Returns TD_ENOADJ if the plan was factored with desc.adjoint == 0.
 */
td_status tridiag_solve_adjoint(td_plan plan, const double* G, int64_t ldg, double* Lam, int64_t ldl,
                                int64_t K, const td_refine* refine, td_info* info, void* stream);

/*
 * Gradient with respect to a shift sigma added to the diagonal of the blocks C_j:
 *   out[r] = - sum_{k < K} Lam[r + k*ldl] * X[r + k*ldx],   r < n   (n = N*M)
 * with Lam = P^{-T} dL/dX and X = P^{-1} F.  All device pointers; out has n entries.
 * The sum over k runs in a fixed order (bitwise reproducible).
 */
td_status tridiag_diag_grad(const double* Lam, int64_t ldl, const double* X, int64_t ldx, int64_t n, int64_t K,
                            double* out, void* stream);

/* Free every device buffer of the plan (synchronises the plan's last stream). */
td_status tridiag_destroy(td_plan plan);

/* Plan facts (host memory). */
typedef struct {
  int64_t N, M, subdomains;
  int64_t Mp;                 /* block size padded for the kernels (multiple of 16, 32 or 64) */
  int64_t tree_depth;         /* levels of the dichotomy tree over the p interface rows */
  int64_t device_bytes;       /* device memory owned by the plan */
  double factor_ms;           /* wall time of tridiag_factor */
  int32_t sweep_prec, adjoint;
} td_plan_info;
td_status tridiag_plan_info(td_plan plan, td_plan_info* out);

/*
 * Per-stage timing of the solves (HIP events recorded on each solve's own stream, no extra
 * synchronisation).  While enabled, every solve (up to 4096 between read-outs) records events
 * around its stages.  tridiag_stage_times waits for the last recorded solve and writes the
 * average milliseconds per solve over the solves recorded since the previous read-out of:
 * [0] subdomain sweeps, [1] interface right-hand side, [2] dichotomy partial sums,
 * [3] dichotomy levels, [4] superposition, [5] residual tests and refinement, [6] whole
 * solve, and, if n >= 8, [7] the number of solves averaged; then it starts a new count.
 * With refinement the stage times [0]-[4] are those of the last correction pass.
 */
td_status tridiag_set_profiling(td_plan plan, int enable);
td_status tridiag_stage_times(td_plan plan, double* ms, int n);

/*
 * Autotuner: times the solve of a probe system (probe_N block rows of M x M blocks,
 * C = tridiag(-1, 4.5, -1), A = B = I, K hashed right-hand sides) for each candidate subdomain
 * length L (p = probe_N / L) in the given precision and returns the fastest L in *best_L and
 * the per-candidate milliseconds per solve in ms_per_solve (ncand entries, may be NULL).
 * Allocates and frees its own device memory; synchronises the stream.
 */
td_status tridiag_autotune(int64_t M, int64_t K, int32_t sweep_prec, int64_t probe_N, const int64_t* candidates,
                           int ncand, void* stream, int64_t* best_L, double* ms_per_solve);

/*
 * Launch shapes of a plan's solve kernels (not in the paper): right-hand-side columns per
 * work-group (sweep_cols, sup_cols: 8, 16 or 32 for float64 plans; 16, 32 or 64 for float32 and
 * bfloat16 plans) and waves per work-group (sweep_waves, sup_waves: a divisor of Mp / 16 that
 * gives 16, 32 or 64 rows per wave, at most 8) of the subdomain sweeps and of the superposition.
 * 0, or a value that the block size, the precision or the LDS does not allow, keeps the library's
 * rule for that field.  They change the solution at most at the rounding level (every shape runs
 * the same products; the half-panel superposition above block size 256 adds the two interface
 * halves in an order that alternates by row, the other forms in one order).  tridiag_set_tiles
 * (tiles NULL = all rules) applies to the plan and to its transposed plan; it drops the plan's
 * captured solve graph.  Not for calls that overlap a solve of the plan.
 */
typedef struct td_tiles {
  int32_t sweep_cols, sweep_waves, sup_cols, sup_waves;
} td_tiles;
td_status tridiag_set_tiles(td_plan plan, const td_tiles* tiles);
td_status tridiag_get_tiles(td_plan plan, td_tiles* tiles);

/*
 * Autotuner over the subdomain length and the launch shapes together (not in the paper): for
 * each candidate subdomain length L the probe system of tridiag_autotune is factored once and its
 * solve of K right-hand sides timed with the library's rules and with each alternative column
 * count and wave count of the sweeps and of the superposition (one field changed at a time, then
 * the best of each field together).  Returns the fastest length in *best_L, its launch shapes in
 * *best_tiles (0 where the rule was fastest) and its milliseconds per solve in *best_ms (may be
 * NULL).  Allocates and frees its own device memory; synchronises the stream.
 */
td_status tridiag_autotune_tiles(int64_t M, int64_t K, int32_t sweep_prec, int64_t probe_N,
                                 const int64_t* candidates, int ncand, void* stream, int64_t* best_L,
                                 td_tiles* best_tiles, double* best_ms);

/*
 * Batched solve of many independent systems (not in the paper): a work list of all systems'
 * stages (sweep tiles, interface right-hand sides, dichotomy partial sums and levels,
 * superposition tiles, residual chunks), captured once in a HIP graph and replayed by
 * tridiag_batch_solve.  By default the graph holds one launch per stage, each running the
 * independent items of all systems for that stage; with the environment variable
 * TD_BATCH_MODE=persistent at creation it holds one persistent launch in which every item
 * waits (bounded) on counters of the items it depends on.  Both give bitwise the same result.
 * Each pass solves every system (pass 0 with F, later passes with the
 * float64 residual, adding the correction to X); a system that has reached `tol` skips the
 * remaining passes.  The plans must have sweep_prec TD_PREC_F64 or TD_PREC_F32, diagonal A and B,
 * tridiagonal C and padded block sizes 64, 128 or 256; they must outlive the batch, and the
 * F / X buffers given here are the ones every replay reads and writes (device pointers, one
 * per system, column-major N_q*M_q x K_q).  Calls that share a plan's workspace must not
 * overlap.  tridiag_batch_info synchronises and reports, per system, the passes used after the
 * first (iterations) and the final max column relative residual; it returns TD_ENOCONV if
 * a system did not reach `tol`, TD_EHIP if a dependency wait inside the persistent launch timed
 * out.
 * Plans may mix TD_PREC_F64 (float64 sweeps) and TD_PREC_F32.  tol == 0 means 1e-10; tol < 0
 * runs a single pass without residual test (infos then report -1).
 */
typedef struct td_batch_s* td_batch;

/*
 * One-call form of the batched solve: solves P_q X_q = F_q for the n plans (F_q, X_q device, column-major
 * N_q M_q x K_q with leading dimension N_q M_q).  The first call with a given set of (plan, F, X, K) and
 * refinement settings builds and captures the batch (tridiag_batch_create); later calls with the same
 * arguments replay it; other arguments replace it.  refine NULL or disabled: one pass, no residual test;
 * enabled: up to 1 + max_iter passes (max_iter <= 0: 2) with per-system early exit at tol (<= 0: 1e-10).
 * infos (host, n entries) may be NULL; if given, the call synchronises and fills them (TD_ENOCONV if a
 * system missed tol).  Plans, F and X must stay alive while the captured batch may be replayed; the
 * cached batch is released by tridiag_solve_batched(0, ...) or when the arguments change.  One host
 * thread at a time.
 */
td_status tridiag_solve_batched(int n, const td_plan* plans, const double* const* F, double* const* X,
                                const int64_t* K, const td_refine* refine, td_info* infos, void* stream);
td_status tridiag_batch_create(int n, const td_plan* plans, const double* const* F, const int64_t* ldf,
                               double* const* X, const int64_t* ldx, const int64_t* K, int passes, double tol,
                               void* stream, td_batch* out);
td_status tridiag_batch_solve(td_batch batch, void* stream);
td_status tridiag_batch_info(td_batch batch, td_info* infos);
td_status tridiag_batch_destroy(td_batch batch);

/*
 * Band matrices (Sec. 3: the PML subdomain matrix and the probing preconditioner are band
 * matrices, and a band matrix is block-tridiagonal with upper-triangular A_j and lower-
 * triangular B_j).  Writes the blocks of the n x n band matrix with kl sub- and ku
 * super-diagonals, given in general band storage (device, column-major, entry (i, j) at
 * ab[ku + i - j + j * ldab], ldab >= kl + ku + 1), as DENSE blocks of size M >= max(kl, ku, 1):
 * N = ceil(n / M) block rows, A, B, C each [N][M][M] (device, caller-allocated, column-major
 * blocks), in the sign convention of tridiag_factor (the band entries left of the diagonal
 * block are -A_I, right of it -B_I).  Rows at or beyond n get a unit diagonal and no couplings,
 * so right-hand sides padded with zeros to N*M rows give solutions whose padded rows are zero.
 * Asynchronous on `stream`; TD_EINVAL for inconsistent sizes or null pointers.
 */
td_status tridiag_band_to_blocks(int64_t n, int32_t kl, int32_t ku, const double* ab, int64_t ldab, int64_t M,
                                 double* A, double* B, double* C, void* stream);

/*
 * Schur-complement solver on interface block rows (Sec. 3: eq. (linear_decomp) orders the
 * unknowns as interiors of the subdomains, then interfaces; eq. (schur_decomp) defines the
 * Schur complement S = A_GG - A_GI A_II^{-1} A_IG and the interface system
 * S x_G = f_G - A_GI A_II^{-1} f_I, solved by conjugate gradients with a probing preconditioner;
 * eq. (domains_equation) gives x_I = A_II^{-1}(f_I - A_IG x_G)).  Here the whole problem is one
 * block-tridiagonal P (N block rows of size M, diagonal A and B, tridiagonal C; device, the
 * layouts of tridiag_factor) whose block rows icol[0..nif) (host array) are the interfaces: they
 * must increase, lie in [1, N-2] and leave at least one interior block row between two of them,
 * so the interior rows fall into nif + 1 strips.  CG needs P symmetric (A_{j+1} = B_j and every
 * C_j symmetric; checked, else TD_EINVAL) and positive definite (else CG fails: TD_ENOCONV).
 * The interior rows of all strips are factored as one block-tridiagonal plan; every product
 * with A_II^{-1} is one solve of it.  band >= 0 builds the probing preconditioner: S applied to
 * 2 (2 band + 1) probe vectors gives a symmetric band matrix of half-width `band` per interface
 * (couplings between interfaces dropped), factored through tridiag_band_to_blocks; band = -1
 * runs plain CG.  tridiag_schur_create synchronises `stream` and keeps copies of A, B, C.
 *
 * tridiag_schur_apply: Y = S V for K interface vectors (device, column-major nif*M x K,
 * ldv, ldy >= nif*M; the rows of interface k are block row icol[k]).  Asynchronous.
 * tridiag_schur_solve: X = P^{-1} F through the interface system (F, X device, column-major
 * (N*M) x K, ld >= N*M, no overlap), one CG per column, stopping when every column has
 * ||r_k|| <= tol ||g_k|| (tol <= 0: 1e-10) or after max_iter iterations (<= 0: 500,
 * TD_ENOCONV).  Synchronises `stream` once per iteration.  info (host, may be NULL):
 * iterations done, columns still above tol, largest ||r_k|| / ||g_k||.
 */
typedef struct td_schur_s* td_schur;
typedef struct {
  int32_t iterations;
  int32_t active;
  double max_rel_residual;
} td_schur_info;
td_status tridiag_schur_create(int64_t N, int64_t M, const double* A, const double* B, const double* C, int64_t nif,
                               const int64_t* icol, int32_t band, void* stream, td_schur* out);
td_status tridiag_schur_apply(td_schur s, const double* V, int64_t ldv, double* Y, int64_t ldy, int64_t K,
                              void* stream);
td_status tridiag_schur_solve(td_schur s, const double* F, int64_t ldf, double* X, int64_t ldx, int64_t K, double tol,
                              int32_t max_iter, td_schur_info* info, void* stream);
td_status tridiag_schur_destroy(td_schur s);

const char* tridiag_status_string(td_status s);
/* Text of the last error on the calling host thread ("" if none). */
const char* tridiag_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TRIDIAG_H */
