/*
 * luqr.h -- C ABI of the MI355X hybrid LU-QR dense solver.
 *
 * Method: Faverge, Herrmann, Langou, Lowery, Robert, Dongarra, "Designing
 * LU-QR hybrid solvers for performance and stability" (arXiv 1401.5522).
 * At each panel step k of a tiled factorization (Alg. 1) the diagonal tile is
 * factored with partial pivoting on a copy, a robustness criterion on tile
 * norms (Sec. 3: Max, Sum, MUMPS) decides, on the device, between an LU step
 * (Alg. 2, variant A1: GETRF / TRSM / SWPTRSM / GEMM) and a QR step (Alg. 3
 * and 4a with a flat tree of TS kernels: GEQRT / TSQRT / UNMQR / TSMQR); the
 * solve replays the stored transformations on the right-hand sides and
 * back-substitutes (Sec. 2.4).
 *
 * Conventions shared by every entry point
 *  - Matrices are column-major.  "Device pointer" means memory the HIP
 *    runtime can access from the GPU the calling thread has current
 *    (hipMalloc or torch CUDA tensors); "host pointer" means ordinary memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call only enqueues work on it and returns without waiting, except
 *    the luqr_get_* calls, which wait for the stream, luqr_solve_gmres_ir
 *    (its Arnoldi least-squares runs on the host) and luqr_solve_noalloc with
 *    a status to fill.
 *  - The library never allocates device memory: the caller provides one
 *    workspace whose size luqr_workspace_bytes reports and keeps it alive
 *    until luqr_destroy.  The library owns only the small host handle and,
 *    for the lookahead of luqr_factor, two streams and three events of its own.
 *  - Return codes: 0 = success; -i = argument i (1-based) is invalid;
 *    LUQR_ERR_UNSUPPORTED for a valid but unimplemented combination;
 *    LUQR_ERR_HIP - e for a HIP runtime error e.  Numerical conditions
 *    (zero pivot, non-finite criterion input, refinement not converged) are
 *    found on the device and reported by luqr_get_status; results are still
 *    written, as LAPACK's getrf does.
 */
#ifndef LUQR_H
#define LUQR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LUQR_ERR_UNSUPPORTED (-900)
#define LUQR_ERR_HIP (-1000)

/* Robustness criterion of a panel step (Sec. 3). */
typedef enum {
    LUQR_CRIT_MAX = 0,    /* LU iff alpha/||A_kk^-1||_1 >= max_{i>k} ||A_ik||_1   (Sec. 3.1) */
    LUQR_CRIT_SUM = 1,    /* LU iff alpha/||A_kk^-1||_1 >= sum_{i>k} ||A_ik||_1   (Sec. 3.2) */
    LUQR_CRIT_MUMPS = 2,  /* LU iff alpha pivot(j) >= estimate_max(j) for all j   (Sec. 3.3) */
    LUQR_CRIT_RANDOM = 3, /* LU with probability alpha/100 (the random choice of Sec. 5.2);
                             draw k = SplitMix64 output k of `seed`, top 53 bits / 2^53 */
    LUQR_CRIT_FORCED = 4  /* decisions given in opts.forced (1 = LU, 0 = QR) */
} luqr_criterion;

/* Arithmetic of the trailing contractions (GEMM update of LU steps, TSMQR
 * update of QR steps) and of the stored factors.  The diagonal-tile GETRF,
 * the inverse norm and all criterion norms are FP64 in every mode. */
typedef enum {
    LUQR_FP64 = 0, /* everything in FP64 */
    LUQR_FP32 = 1, /* FP32 factor storage, FP32 MFMA contractions */
    LUQR_BF16 = 2  /* FP32 factor storage, BF16 MFMA contraction operands with a
                      power-of-two scale per tile, FP32 accumulation */
} luqr_precision;

typedef struct {
    int32_t nb;          /* tile size n_b: 32, 64, 128, 256 or 512 (512 not with FP64) */
    int32_t criterion;   /* luqr_criterion */
    double alpha;        /* threshold alpha >= 0; +inf = always LU, 0 = always QR */
    int32_t precision;   /* luqr_precision */
    int32_t nrhs_max;    /* largest nrhs later passed to luqr_solve / luqr_solve_refined (>= 1) */
    uint64_t seed;       /* LUQR_CRIT_RANDOM stream */
    const int8_t *forced;/* host pointer, n = ceil(N/nb) decisions, read by luqr_factor (FORCED only) */
    int32_t nsteps;      /* run only the first nsteps panel steps (< 0: all); a partial
                            factorization cannot be solved with */
    int32_t timing;      /* nonzero: record HIP events between the kernels of each step
                            (read back with luqr_get_step_times) */
    int32_t no_lookahead;/* 0 (default): lookahead (the Sec. 4 task graph's overlap of
                            consecutive steps): step k+1's panel factor and criterion run
                            while step k's bulk trailing work runs on two streams of the
                            library's own: the LU update of columns k+2.., joined before
                            step k+1's branch, and a QR step's R^-1 and full T factors,
                            joined at the end; nonzero: every kernel in order on the
                            caller's stream */
    int32_t domain_stride; /* 0 (default): the LU attempt pivots within the diagonal tile.
                            p > 0: within the diagonal domain (Sec. 2.1, last paragraph):
                            the panel tiles k, k+p, k+2p, ... (the tiles a node holds when
                            tile rows are dealt cyclically over p rows of nodes), stacked;
                            the criterion then sees A_kk and the tiles below after the
                            domain's interchanges (Sec. 3.1), MUMPS takes local_max over the
                            domain and away_max off it (Sec. 3.3), and an LU step applies
                            the interchanges to the trailing columns of the domain's rows.
                            The pivots of such a step (luqr_export_factors) are stacked row
                            indices.  Supported while the first step's domain has at most
                            512 rows ((1 + (n-1)/p) nb <= 512), else LUQR_ERR_UNSUPPORTED;
                            not by the batched entry points. */
    int32_t invnorm_estimate; /* 0 (default): the Max and Sum criteria take ||A_kk^-1||_1
                            exactly (the product U^-1 L^-1 of the explicit FP64 inverses).
                            1: from the O(n_b^2)-per-iteration estimate of Sec. 3.4 (Hager's
                            iteration with Higham's refinements, as in LAPACK's condition
                            estimator; at most five products with A_kk^-1 and four with
                            its transpose, each through the explicit inverses).  The
                            estimate is a lower bound, so s_k = 1/est can only be larger
                            than the exact one: an LU step of the exact criterion stays
                            LU.  Not by the batched entry points. */
    int32_t lu_variant;  /* LU step variant.  0 or 1 (default): A1 (Alg. 2): the panel
                            factors an FP64 backup copy of A_kk by GEPP and a QR step
                            starts afresh from the untouched tile.  2: A2 (Sec. 2.3):
                            every step first QR-factors A_kk in place (GEQRT, storage
                            precision, V and R kept in the tile, no backup); the
                            criterion takes ||A_kk^-1||_1 = ||R^-1 Q^T||_1 (FP64, from
                            those factors); an LU step eliminates with R (A_ik R^-1),
                            applies Q^T to the tiles A_kj and updates as in A1; a QR
                            step continues from the same GEQRT.  Pivots of an A2 LU step
                            are the identity.  With Max, Sum, Random and Forced only,
                            without a domain or the estimate (else LUQR_ERR_UNSUPPORTED);
                            not by the batched entry points. */
    int32_t qr_tree;     /* QR steps' elimination tree (Sec. 2.2, Alg. 3 and 4).  0 (default):
                            the flat tree, A_kk eliminates every A_ik with TS kernels (Alg. 4a).
                            S > 0: the panel tiles k..n-1 form groups of S consecutive tiles
                            (a last group of one tile joins the group before it); each
                            group's first tile eliminates the others with TS kernels, and the
                            groups' first tiles are then reduced by a binary tree of TT
                            kernels (Alg. 4b): at distance d = 1, 2, 4, .. group g eliminates
                            group g+d for g = 0, 2d, ..  S = 1 is the binary TT tree; S >= n
                            is the flat tree.  The tree changes the factors and so the later
                            decisions; the workspace grows by one T factor per panel tile.
                            Not by the batched entry points. */
} luqr_opts;

/* Device-side numerical status, read back by luqr_get_status. */
typedef struct {
    int64_t info;        /* first exactly-zero pivot of an LU step, 1-based global row; 0 if none */
    int32_t nonfinite;   /* a criterion input (s_k or m_k) was NaN or Inf at some step */
    int32_t n_lu;        /* number of LU steps taken */
    int32_t ir_iters;    /* refinement iterations done by the last luqr_solve_refined */
    int32_t ir_converged;/* 1 if the last refinement met its backward-error target */
    double ir_eta;       /* backward error ||b-Ax||_inf/(||A||_inf ||x||_inf) of the returned x
                            (largest over right-hand sides) */
    int32_t watchdog;    /* a device-side wait exceeded its spin bound (result invalid) */
    int32_t reserved;
} luqr_status;

typedef struct luqr_factors_s *luqr_factors;

/* Bytes of device workspace luqr_factor needs for an N x N matrix with the
 * given options.  Returns < 0 (an argument code as above) on invalid input. */
int64_t luqr_workspace_bytes(int64_t N, const luqr_opts *opts);

/* Factor the N x N matrix dA (device, column-major, leading dimension lda,
 * FP64, not modified) with the hybrid LU-QR algorithm (Alg. 1).  Factors,
 * decisions and all scratch live in dWork (device, >= luqr_workspace_bytes,
 * 256-byte aligned).  On success *out receives a new handle.  Asynchronous:
 * returns once the work is enqueued on `stream` (with lookahead, part of it on
 * the handle's own streams, which are joined back to `stream` at the end, so work
 * enqueued on `stream` afterwards sees the whole factorization).  The decision
 * of step k is written on the device and read there by the LU and QR branch
 * kernels: the host never waits for it. */
int luqr_factor(int64_t N, const double *dA, int64_t lda, const luqr_opts *opts,
                void *dWork, int64_t work_bytes, void *stream, luqr_factors *out);

/* Overwrite dB (device, N x nrhs, leading dimension ldb, FP64) with A^{-1} B
 * using the stored factors: forward replay of the step transformations
 * (Sec. 2.4, second pass) then block back-substitution.  The arithmetic is
 * FP64 over factors in their storage precision; B and the result are FP64.
 * nrhs <= opts.nrhs_max.  Only enqueues: the kernels read each step's
 * decision on the device (the kernels of the branch a step did not take
 * return at once), so the host never waits for the factorization. */
int luqr_solve(luqr_factors f, int64_t nrhs, double *dB, int64_t ldb, void *stream);

/* Mixed-precision solve with FP64 iterative refinement: x0 = solve(b), then
 * up to max_iter times r = b - A x (FP64, from dA), d = solve(r) with the
 * stored factors, x += d (FP64), stopping once every column has
 * ||r||_inf <= N * 1e-16 * ||A||_inf ||x||_inf.  dA is the FP64 matrix that
 * was factored; dB is read, dX (N x nrhs, ldx) written.  Only enqueues: all
 * max_iter passes are enqueued, the convergence test runs on the device, and
 * once it has passed the kernels of the remaining passes return at once
 * (each reads the device flag), so a pass after convergence costs only its
 * launches.  Iteration count and final backward error are reported by
 * luqr_get_status. */
int luqr_solve_refined(luqr_factors f, const double *dA, int64_t lda, int64_t nrhs,
                       const double *dB, int64_t ldb, double *dX, int64_t ldx,
                       int32_t max_iter, void *stream);

/* GMRES-based iterative refinement for one right-hand side (for factors too
 * inaccurate for luqr_solve_refined to converge: ill-conditioned A, BF16
 * contractions).  x0 = solve(b); then up to max_outer times r = b - A x in
 * FP64 with the same convergence test as luqr_solve_refined, and x += d
 * where d solves A d = r by GMRES in FP64 left-preconditioned by the stored
 * factors (each inner step: one product with dA and one solve), restarted
 * after max_inner (1..30) vectors or once the preconditioned residual has
 * dropped by 1e-6.  db and dx are device vectors of N doubles.  The host
 * waits on `stream` once per inner step for two short vectors.  The outer
 * iteration count and backward error are reported by luqr_get_status; the
 * number of inner steps is written to *inner_total (host, may be NULL). */
int luqr_solve_gmres_ir(luqr_factors f, const double *dA, int64_t lda, const double *db,
                        double *dx, int32_t max_outer, int32_t max_inner,
                        int32_t *inner_total, void *stream);

/* alpha from a growth budget, for the Max and Sum criteria (the choice of alpha
 * is left open in Sec. 5.2 and Sec. 7; this takes it from the bounds of Sec. 3):
 * the largest alpha whose worst-case growth of the tile norms,
 * max_{i,j,k} ||A_ij^(k)||_1 / max_{i,j} ||A_ij||_1, stays within `growth`
 * for an N x N matrix in n = ceil(N/nb) tiles.
 *   Max (Sec. 3.1): growth <= (1 + alpha)^(n-1), so alpha = growth^(1/(n-1)) - 1.
 *   Sum (Sec. 3.2): the column sums of tile norms grow by at most max(1, alpha)
 *     per step, so growth <= n max(1, alpha)^(n-1): alpha = (growth/n)^(1/(n-1))
 *     for growth >= n, and 0 (every step QR) below n, which no alpha > 0 meets.
 *   One tile (n = 1): +inf (the step is the tile's own GEPP).
 * Host arithmetic only.  Returns alpha >= 0, or -1 (N < 1 or nb < 1), -3 (a
 * criterion other than Max or Sum), -4 (growth < 1 or NaN). */
double luqr_alpha_for_growth(int64_t N, int32_t nb, int32_t criterion, double growth);

/* Copy the decision sequence (1 = LU, 0 = QR), s_k = 1/||A_kk^-1||_1, m_k (the
 * max or sum of sub-diagonal tile norms) and the relative margin
 * (alpha s_k - m_k)/max(alpha s_k, m_k) of the first n steps to host arrays
 * (each may be NULL).  Waits for the handle's stream. */
int luqr_get_decisions(luqr_factors f, int8_t *dec, double *s, double *m, double *margin, int64_t n);

/* Read the device status (waits for the handle's stream). */
int luqr_get_status(luqr_factors f, luqr_status *st);

/* Per-step kernel durations in milliseconds, from HIP events recorded on the
 * factorization stream when opts.timing was set.  t (host, 5 n floats) receives
 * for each step k < n, at t[5 k + p]:
 *   p = 0  panel: GETRF on the diagonal-tile copy, tile norms, triangular
 *          inverses, inverse norm and decision
 *   p = 1  LU Eliminate and Apply (A_ik U^-1, L^-1 P A_kj)
 *   p = 2  LU trailing update (A_ij -= A_ik A_kj)
 *   p = 3  QR step: GEQRT, TSQRT, UNMQR and TSMQR in their single launch
 *   p = 4  R_kk^-1 for the back-substitution of a QR step and the completion
 *          of its block reflectors' T factors for the solve
 * A phase that the decision skipped still appears, with the few microseconds
 * its early-exit launch takes.  Waits for the stream.  Returns
 * LUQR_ERR_UNSUPPORTED if the handle was created without timing. */
#define LUQR_NPHASE 5
int luqr_get_step_times(luqr_factors f, float *t, int64_t n);

/* Copy the factored matrix to dF (device, FP64, N x N, column-major, ldf) in
 * the layout the paper describes in-place (L\U or V\R on the diagonal tiles,
 * L or Y below, U_kj to the right), the LU pivots of every step to the host
 * array ipiv (N entries, local 0-based row exchanged at each column; identity
 * for QR steps; may be NULL).  For inspection and tests. */
int luqr_export_factors(luqr_factors f, double *dF, int64_t ldf, int32_t *ipiv, void *stream);

/* Release the host handle (the workspace belongs to the caller). */
void luqr_destroy(luqr_factors f);

/* ---- for callers that cannot allocate --------------------------------------
 * For callers that cannot call hipMalloc or hand over a workspace: code that
 * runs while a HIP graph is being captured, tight serving loops, harnesses
 * that forbid allocation.  luqr_factor followed by luqr_solve_refined in one
 * call, with the workspace taken from a buffer the library itself holds in
 * device memory: LUQR_NOALLOC_SCRATCH_BYTES (64 MiB) on every GPU it runs
 * on, kept until the process ends.  Neither the call nor anything it
 * launches allocates device memory (no hipMalloc, hipFree or allocating
 * library routine) and no handle is created.
 *   Arguments as for luqr_factor and luqr_solve_refined: dA (device, N x N,
 *   lda, FP64, not modified), opts (opts.timing must be 0; lookahead is not
 *   used, every kernel runs on `stream`), dB (device, N x nrhs, ldb, read),
 *   dX (device, N x nrhs, ldx, written), max_iter >= 0 refinement passes
 *   (0: the solve with the factors plus one backward-error check), status
 *   (host, may be NULL) receives what luqr_get_status would report.
 *   Returns LUQR_ERR_TOO_LARGE when the workspace this N, tile size,
 *   precision and opts.nrhs_max need (luqr_workspace_bytes) exceeds
 *   LUQR_NOALLOC_SCRATCH_BYTES; for example N = 2048 fits in FP64 at
 *   n_b = 128 and in FP32 at n_b = 256.
 *   Only enqueues when status is NULL (then it can be captured in a HIP
 *   graph); with a status it waits for `stream` before filling it.
 *   Every call on one GPU uses that GPU's one buffer, which keeps the last
 *   call's contents: calls that overlap on one GPU (from several host threads
 *   or streams) race and must be serialized by the caller. */
#define LUQR_NOALLOC_SCRATCH_BYTES (64ll << 20)
#define LUQR_ERR_TOO_LARGE (-901)
int luqr_solve_noalloc(int64_t N, const double *dA, int64_t lda, const luqr_opts *opts, int64_t nrhs,
                       const double *dB, int64_t ldb, double *dX, int64_t ldx, int32_t max_iter,
                       luqr_status *status, void *stream);

/* ---- many independent systems ------------------------------------------ */

/* Solve batch independent systems A_s x_s = b_s (N_s <= 1024, one right-hand
 * side each) with the hybrid LU-QR algorithm in one persistent launch: each
 * workgroup takes systems from a queue ordered largest first and runs Alg. 1
 * (Max or Sum criterion), the solve of Sec. 2.4 and FP64 iterative
 * refinement on one system.  FP32 tile storage and MFMA contractions
 * (opts.precision must be LUQR_FP32); tile size 32 or 64 per system.
 *
 * Use: luqr_batched_workspace_bytes -> luqr_batched_plan (once per size
 * set; copies small descriptors into the workspace and waits) ->
 * luqr_batched_run (only enqueues a counter reset and the persistent kernel,
 * so it can be captured into a hipGraph and replayed) -> luqr_batched_destroy.
 * The caller owns the workspace and keeps it alive while the plan is used.
 */
typedef struct luqr_batch_s *luqr_batch;

/* Workspace bytes for the systems of sizes N[s] (host) with tile sizes nb[s]
 * (host, 32 or 64; NULL = opts.nb for all).  < 0 on invalid input. */
int64_t luqr_batched_workspace_bytes(int64_t batch, const int64_t *N, const int32_t *nb, const luqr_opts *opts);

/* Plan: N, nb (may be NULL), lda, ldb, ldx are host arrays of batch entries;
 * dWork (device, 256-byte aligned, >= luqr_batched_workspace_bytes).  Uses
 * opts.criterion (MAX or SUM), opts.alpha, opts.precision (FP32); max_iter
 * bounds the refinement per system.  Waits for the descriptor copy.  Returns
 * LUQR_ERR_UNSUPPORTED for other precisions or criteria. */
int luqr_batched_plan(int64_t batch, const int64_t *N, const int32_t *nb, const int64_t *lda, const int64_t *ldb,
                      const int64_t *ldx, const luqr_opts *opts, int32_t max_iter, void *dWork, int64_t work_bytes,
                      luqr_batch *out);

/* Run: dA, dB, dX are device arrays of batch device pointers (FP64,
 * column-major with the plan's leading dimensions; x_s written to dX[s]).
 * dDec (device, may be NULL): decisions of system s at dDec + s *
 * luqr_batched_decision_stride(plan).  dEta, dIters (device, may be NULL):
 * backward error ||b-Ax||_inf / (||A||_inf ||x||_inf) and refinement count per
 * system.  Only enqueues on `stream`. */
int luqr_batched_run(luqr_batch plan, const double *const *dA, const double *const *dB, double *const *dX,
                     int8_t *dDec, double *dEta, int32_t *dIters, void *stream);

/* Largest tile count over the plan's systems (stride of dDec). */
int luqr_batched_decision_stride(luqr_batch plan);

void luqr_batched_destroy(luqr_batch plan);

/* Autotuner: for each size class [64*2^c, 64*2^(c+1)) (c = 0..5, the last
 * open-ended) time up to `sample` of its systems with tile size 32 and with
 * 64 (one warm-up and one timed persistent launch each, HIP events) and write
 * the faster tile size of the class for each system to nb_out (host, batch
 * entries).  ms_out (host, 12 floats, may be NULL) receives the timings as
 * [2c] (nb 32) and [2c+1] (nb 64).  Arguments as for plan/run; the systems'
 * own data are used and dX is overwritten.  Waits for the device.  The
 * workspace is used as scratch: plan afterwards. */
int luqr_batched_autotune(int64_t batch, const int64_t *N, const int64_t *lda, const int64_t *ldb,
                          const int64_t *ldx, const luqr_opts *opts, int32_t max_iter,
                          const double *const *dA, const double *const *dB, double *const *dX, int32_t sample,
                          void *dWork, int64_t work_bytes, void *stream, int32_t *nb_out, float *ms_out);

#ifdef __cplusplus
}
#endif
#endif /* LUQR_H */
