/*
 * emin.h -- C ABI of the MI355X energy-minimization prolongation library.
 *
 * The library computes the energy-minimal prolongation P of arXiv 2208.02995:
 * P minimizes tr(P^T A P) (Sec. 3, eq. trace) over a fixed sparsity pattern
 * while keeping the near-kernel constraint P * B_c = B (Sec. 3, eqs. inKern,
 * TSP), by the preconditioned restricted conjugate gradient of Alg. 3
 * (Sec. 3.4.1) started from the tentative prolongation corrected by Alg. 2
 * (Sec. 3.2).  The pattern is S^k P0 with S = struct(A) (Sec. 3, eq. enlPatt).
 * Every row of P is free (aggregation form); the classical C/F form with fixed
 * identity rows is not covered.
 *
 * Conventions shared by every entry point
 *   - Matrices are CSR with int32 row pointers and column indices, columns
 *     sorted strictly ascending inside each row (no duplicates).  Dense
 *     blocks are row-major.
 *   - Pointers to matrix/vector data are DEVICE pointers (HIP global memory
 *     of the context's device) unless an argument is marked "host".
 *   - The caller owns every array it passes.  Arrays given to
 *     emin_problem_create (A, P0, B, B_c) are referenced, not copied: they
 *     must stay allocated until emin_problem_destroy.  Their structure (row
 *     pointers, column indices, shapes) must not change; their VALUES may
 *     change between calls -- every emin_solve re-reads them (the numeric
 *     phase recomputes all value-dependent data).
 *   - The library owns handles and their device workspace.
 *   - Work is enqueued on the context's stream.  Calls that return a host
 *     value (sizes, energies, statistics) synchronize that stream.
 *   - Every call returns an emin_status; nothing throws across the ABI.
 *     emin_last_error() gives a thread-local message for the last failure.
 *   - Numbers: FP64 inputs.  EMIN_MIXED runs the bulk sparse products and
 *     vector updates in FP32 (FP32 accumulation) while the per-row constraint
 *     factors, all dot-product accumulations, the CG scalars and the final
 *     re-projection stay FP64.
 */
#ifndef EMIN_H
#define EMIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EMIN_OK = 0,
  EMIN_ERR_ARG = -1,         /* null pointer, negative size, bad option value           */
  EMIN_ERR_SHAPE = -2,       /* inconsistent dimensions between arguments               */
  EMIN_ERR_CSR = -3,         /* rowptr not monotone / column out of range / unsorted    */
  EMIN_ERR_PATTERN = -4,     /* the pattern does not contain P0's pattern               */
  EMIN_ERR_DIAG = -5,        /* A(i,i) <= 0 or missing, or a singular diagonal block    */
  EMIN_ERR_BREAKDOWN = -6,   /* <y, Pi K y> <= 0 or gamma < 0 (A not SPD on pattern)     */
  EMIN_ERR_HIP = -7,         /* a HIP runtime call failed                               */
  EMIN_ERR_OOM = -8,         /* device allocation failed                                */
  EMIN_ERR_UNSUPPORTED = -9, /* m > EMIN_MAX_M, or a row longer than supported          */
  EMIN_WARN_RANK = 1         /* solve done; >= 1 row had rank(G_i) < m (see stats)      */
} emin_status;

#define EMIN_MAX_M 8          /* largest near-kernel dimension m                         */

enum { EMIN_FP64 = 0, EMIN_MIXED = 1 };
/* preconditioners of Alg. 3: Jacobi M_1, nodal block Jacobi, projected
 * symmetric Gauss-Seidel M_2 (Sec. 3.4.1, eq. SGS_prec without its second
 * term: z = Pi (L+D)^{-T} D (L+D)^{-1} r on K, rows swept by colour, then
 * index, the colours of Jones-Plassmann rounds on A's graph with priority
 * (h(i), i), h the MurmurHash3 32-bit finalizer; A structurally symmetric) */
enum { EMIN_JACOBI = 0, EMIN_BJACOBI = 1, EMIN_SGS = 2 };
enum { EMIN_STOP_MAXIT = 0, EMIN_STOP_CONVERGED = 1, EMIN_STOP_TAU = 2, EMIN_STOP_BREAKDOWN = 3 };

typedef struct emin_ctx emin_ctx;
typedef struct emin_problem emin_problem;
typedef struct emin_batch emin_batch;
typedef struct emin_tape emin_tape;

/* A sparse matrix in CSR form.  rowptr: n_rows+1 entries, rowptr[0] = 0,
 * rowptr[n_rows] = nnz.  vals may be NULL where only the structure is read
 * (a caller-supplied pattern). */
typedef struct {
  int64_t n_rows;
  int64_t n_cols;
  int64_t nnz;
  const int32_t *rowptr;
  const int32_t *colind;
  const double *vals;
} emin_csr;

typedef struct {
  int precision;      /* EMIN_FP64 (default) or EMIN_MIXED                               */
  int precond;        /* EMIN_JACOBI (default, Sec. 3.4.1 M_1), EMIN_BJACOBI or EMIN_SGS  */
  int block;          /* node block size for EMIN_BJACOBI (1..4); rows b*a..b*a+b-1       */
  int maxit;          /* RCG iterations (Alg. 3 maxit), >= 0                             */
  double tau;         /* energy-monitor stop dE_k < tau dE_1 (Sec. 3.3, eq. relRed); 0 off */
  int pattern_power;  /* k in S^k P0 (eq. enlPatt) when no pattern is passed, >= 1        */
  int profile;        /* 1: time the masked-product launches with HIP events              */
  int k1_group;       /* masked-product shape hint: lanes per row (power of 2), 0 = auto,
                         -2 = one lane per row with 16-byte row loads (rows <= 8 long),
                         -4 = node kernel with a three-deep single-block pipeline,
                         -5 = node kernel through the slot-level map even where the
                              group-level (slot-pair) one applies,
                         -6, -7, -8 = slot-pair node kernel with 2, 3, 4 neighbour
                              blocks of Y in flight                                  */
  int k1_slots;       /* masked-product shape hint: slots per row (>= row length), 0 = auto,
                         -1 = use the precomputed intersection map                        */
} emin_opts;

typedef struct {
  int32_t iterations;          /* RCG updates applied                                    */
  int32_t stop;                /* EMIN_STOP_*                                             */
  int32_t rank_deficient_rows; /* rows whose local block G_i had rank < m                 */
  int32_t m;
  int64_t nnz_pattern;         /* nnz of the pattern of P                                  */
  double gamma1;               /* first preconditioned residual norm <r, z>               */
  double dE_first;             /* energy decrease of iteration 1 (gamma alpha)            */
  double dE_last;              /* energy decrease of the last applied iteration           */
  double k1_ms;                /* profile: summed masked-product kernel time              */
  int64_t k1_launches;         /* profile: number of masked-product launches timed        */
  double solve_ms;             /* profile: event time of the whole solve                  */
} emin_stats;

/* Fill *o with the defaults: FP64, Jacobi, block 1, maxit 10, tau 0,
 * pattern_power 1, profile 0, automatic kernel shapes. */
void emin_opts_default(emin_opts *o);

/* Create a context on HIP device `device` enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  The context owns a
 * device-memory pool reused by the problems created on it, and a pinned
 * host staging buffer for the tables problem creation builds on the host;
 * a context is used by one host thread at a time.
 * Errors: EMIN_ERR_ARG (out NULL), EMIN_ERR_HIP (bad device). */
emin_status emin_ctx_create(int device, void *hip_stream, emin_ctx **out);
/* Destroy every problem and batch made on ctx first. */
void emin_ctx_destroy(emin_ctx *ctx);

/* Symbolic phase (Sec. 3, eq. enlPatt; Sec. 4 "pattern communicated once").
 * Validates A (n x n, FP64 SPD; its stored structure, explicit zeros included,
 * defines S), P0 (n x nc), B (n x m, row-major, device) and B_c (nc x m,
 * row-major, device), then builds the pattern of P (value arrays of empty
 * matrices, and B for n = 0, may be NULL):
 *   pattern == NULL: struct(A^k P0) with k = opts->pattern_power, 0/1 product;
 *   pattern != NULL: the caller's pattern (structure only, vals ignored).
 * The pattern must contain P0's pattern.  Allocates the problem's workspace
 * and picks kernel shapes.  m must be 1..EMIN_MAX_M.
 * Errors: EMIN_ERR_ARG, EMIN_ERR_SHAPE, EMIN_ERR_CSR, EMIN_ERR_PATTERN,
 * EMIN_ERR_DIAG (A(i,i) <= 0 or missing; singular/indefinite node block for
 * EMIN_BJACOBI), EMIN_ERR_UNSUPPORTED, EMIN_ERR_OOM, EMIN_ERR_HIP.
 * On error *out is NULL and nothing is leaked. */
emin_status emin_problem_create(emin_ctx *ctx, const emin_csr *A, const emin_csr *P0,
                                const emin_csr *pattern, int m, const double *B,
                                const double *Bc, const emin_opts *opts, emin_problem **out);
void emin_problem_destroy(emin_problem *prob);

/* The classical C/F form P = [W; I] (Sec. 2, eqs. CFspl and prol), the
 * paper's native setting: cf (device, n ints) holds the coarse index
 * (0 .. nc-1, each held by one node) of every COARSE node and -1 for every
 * FINE node; P0's COARSE rows must be their identity rows (one entry 1 at
 * column cf[i], as Alg. 1 and emin_ptent_setup give).  COARSE rows are not
 * unknowns: the pattern is struct(A^k P0) (eq. enlPatt) on FINE rows and the
 * identity column on COARSE rows (a given pattern must hold exactly that
 * column on COARSE rows); with that single column, Alg. 2 leaves the row
 * at its identity entry and Pi_i = 0, so the RCG moves FINE rows only and
 * the A_FC coupling enters the residual through mask(A P).  Otherwise as
 * emin_problem_create (the library keeps its own copy of cf); opts.block
 * must be 1 and opts.precond EMIN_JACOBI or EMIN_SGS.  COARSE rows are not
 * counted in stats.rank_deficient_rows, and emin_solve writes them as
 * exactly their identity entry.  Errors as emin_problem_create;
 * EMIN_ERR_ARG also for an invalid cf or non-identity COARSE rows of P0,
 * EMIN_ERR_PATTERN for a given pattern whose COARSE rows differ. */
emin_status emin_problem_create_cf(emin_ctx *ctx, const emin_csr *A, const emin_csr *P0,
                                   const emin_csr *pattern, const int32_t *cf, int m,
                                   const double *B, const double *Bc, const emin_opts *opts,
                                   emin_problem **out);

/* Alg. 1 (Sec. 3.2): the tentative prolongation of a C/F splitting.  For
 * every FINE node i and l = 1 .. lmax: the COARSE nodes within distance l
 * of i in the graph of S (hops over S's stored off-diagonal structure),
 * ordered by coarse index; max vol on their rows of V (Gaussian elimination
 * with partial pivoting, pivots below 1e-12 of the largest entry skipped,
 * then swaps while a coefficient exceeds 1.05 in modulus, ties to the first
 * row); the fit B w = v_i for B = V(J, :)^T of the selected nodes J (the
 * square system by Gaussian elimination with partial pivoting, a smaller
 * one by its normal equations), kept at the first l where the relative
 * residual is at most 1e-10.  A row never fitted stays empty.  COARSE rows
 * are the identity.
 *   S: n x n CSR (structure; vals may be NULL).  cf: device, n ints, as in
 *   emin_problem_create_cf, with nc COARSE nodes.  V: device, n x m
 *   row-major (m 1..8).  lmax: 1..16.
 *   Out: rowptr (device, n + 1), colind / vals (device, capacity n * m:
 *   every row holds at most m entries), *nnz (host), level (device, n ints,
 *   optional: the fitted distance, 0 COARSE, -1 never fitted).
 * Errors: EMIN_ERR_ARG, EMIN_ERR_CSR (S), EMIN_ERR_UNSUPPORTED (a
 * neighbourhood within lmax holds more than 1024 nodes or 128 COARSE
 * nodes), EMIN_ERR_OOM, EMIN_ERR_HIP.  Synchronizes the stream. */
emin_status emin_ptent_setup(emin_ctx *ctx, const emin_csr *S, const int32_t *cf, int32_t nc,
                             const double *V, int m, int lmax, int64_t *nnz, int32_t *rowptr,
                             int32_t *colind, double *vals, int32_t *level);

/* Copy the pattern out.  Two-phase: with rowptr == NULL and colind == NULL
 * only *nnz (host) is written; otherwise rowptr (n+1) and colind (nnz) are
 * device arrays the caller allocated.  Synchronizes the stream. */
emin_status emin_pattern_get(emin_problem *prob, int64_t *nnz, int32_t *rowptr, int32_t *colind);

/* The sweep colouring of an EMIN_SGS problem (see EMIN_SGS): *ncolours
 * (host) is always written; with colour != NULL, colour (device, n ints) gets
 * every row's colour.  EMIN_ERR_ARG when the problem is not EMIN_SGS.
 * Synchronizes the stream. */
emin_status emin_sgs_colours_get(emin_problem *prob, int32_t *ncolours, int32_t *colour);

/* Numeric phase: Alg. 2 on every row (local constraint factor, min-norm
 * correction of P0, rank check), then Alg. 3 for opts.maxit iterations (or
 * until the tau stop, or until gamma_k <= 1e-26 gamma_1), then P = P0' + dP;
 * with EMIN_MIXED or EMIN_BJACOBI, P is re-projected onto the constraint in
 * FP64 (the correction step of Alg. 2).  P_vals (device, nnz(pattern), row-wise on the
 * pattern) receives P.  dE_hist (host, may be NULL) receives gamma_k alpha_k
 * for k = 1..opts.maxit (0 after the last applied iteration).  stats (host,
 * may be NULL).  Synchronizes the stream.
 * Returns EMIN_WARN_RANK when rows were rank deficient (P still written),
 * EMIN_ERR_BREAKDOWN when the iteration broke down (P holds the last
 * iterate before the breakdown). */
emin_status emin_solve(emin_problem *prob, double *P_vals, double *dE_hist, emin_stats *stats);

/* tr(P^T A P) = <P, mask(A P)> (Sec. 3, eq. trace) for P_vals on the
 * pattern (device, FP64).  *E is host.  Synchronizes. */
emin_status emin_energy(emin_problem *prob, const double *P_vals, double *E);

/* emin_energy without any device allocation, for callers that cannot
 * allocate (tight serving or evaluation loops, harnesses that forbid
 * hipMalloc).  Same result as emin_energy, bit for bit (same kernels, same
 * reduction order).  Everything the call needs beyond P_vals and the problem's
 * own arrays -- the result slot, the per-block partial sums and a copy of P
 * with slack for the row-chunk kernels -- lives in one fixed 16 MiB device
 * array per GPU, held until the process ends; the call allocates nothing,
 * also not on its first use.  Every call on one GPU shares that array, so
 * calls that overlap on one GPU (other host threads, other contexts) race;
 * the caller serializes them.  Nothing in the array has to start at zero.
 * Errors: EMIN_ERR_ARG, EMIN_ERR_UNSUPPORTED when the pattern needs more than
 * the array holds (about 2 million pattern entries; the message gives the
 * sizes), EMIN_ERR_HIP.  Synchronizes. */
emin_status emin_energy_noalloc(emin_problem *prob, const double *P_vals, double *E);

/* ||P B_c - B||_F / ||B||_F for P_vals on the pattern (the absolute
 * ||P B_c - B||_F when B = 0; 0 for n = 0).  *rel is host.  Synchronizes. */
emin_status emin_constraint_error(emin_problem *prob, const double *P_vals, double *rel);

/* Y_hat = Pi mask(A Y) (the K y product of Sec. 4 followed by the block
 * projector) for FP64 Y on the pattern; Y_hat (device, nnz(pattern)) is
 * written.  Requires a prior emin_solve (it uses the constraint factors).
 * Exposed for testing and timing the dominant kernel.  Asynchronous. */
emin_status emin_masked_product(emin_problem *prob, const double *Y, double *Y_hat);

/* Batched form (not in the paper): many independent problems solved as one
 * block-diagonal problem, with per-problem CG scalars (each member runs its
 * own Alg. 3, so every member's result matches its single-problem solve up
 * to rounding order).  The members (created with emin_problem_create on the
 * same context) must share m, precision, maxit and tau, use EMIN_JACOBI, and
 * have pattern rows of at most 32 entries.  The batch references the
 * members' arrays (values re-read at every solve; members must outlive the
 * batch).  Creation concatenates the structures -- each member's rows in a
 * breadth-first (Cuthill-McKee) order of A's graph, for locality; values are
 * gathered into, and P scattered out of, that order at every solve, so the
 * caller sees its own order -- buckets the rows by pattern length, picks the
 * masked-product bucket plan with an autotuner (timing the
 * candidates on this batch; with tune_cache a text file path, results are
 * read from / appended to it keyed by the batch's sizes; NULL: always time),
 * and captures the whole solve into one HIP graph.
 * Errors: EMIN_ERR_ARG (mismatched members), EMIN_ERR_UNSUPPORTED, EMIN_ERR_OOM,
 * EMIN_ERR_HIP.  On error *out is NULL. */
emin_status emin_batch_create(emin_ctx *ctx, int count, emin_problem *const *probs,
                              const char *tune_cache, emin_batch **out);

/* Replay the captured solve.  P_vals (host array of `count` device pointers)
 * receives each member's P on its own pattern; stats (host, `count` entries,
 * may be NULL).  Synchronizes the context stream.  Returns the worst status
 * over the members (EMIN_ERR_DIAG, EMIN_ERR_BREAKDOWN, EMIN_WARN_RANK). */
emin_status emin_batch_solve(emin_batch *batch, double *const *P_vals, emin_stats *stats);

/* JSON description of the autotuner's candidates and choice, copied into buf
 * (host, cap bytes, NUL-terminated, truncated if short).  Returns the length
 * needed including the NUL, or -1 for a NULL batch. */
int emin_batch_plan(const emin_batch *batch, char *buf, int cap);
void emin_batch_destroy(emin_batch *batch);

/* ---- Reverse mode (not in the paper) --------------------------------------
 * Derivatives of the map (values of A, values of P0) -> P of emin_solve, with
 * the pattern, B and B_c held fixed.  With B_c fixed the constraint factors
 * of Alg. 2 are constants, so Alg. 2 is affine in P0 and each step of Alg. 3
 * (Sec. 3.4.1) is a product, sum or quotient of its inputs; the reverse sweep
 * runs those steps backwards.  Requires EMIN_FP64, EMIN_JACOBI, symmetric A
 * (the transpose of the masked product is taken equal to it), and pattern
 * rows of at most 64 entries. */

/* emin_solve that also records, per applied iteration k, the direction Y_k
 * and the residual R_k (2 nnz(pattern) doubles each), the CG scalars, and
 * copies of P0', A's values and 1/A(i,i): memory (2 maxit + 1) nnz(pattern)
 * + nnz(A) + n doubles, held by the tape.  P_vals as in emin_solve.  *tape
 * (host) receives the tape (NULL on error); later solves on the same problem
 * do not alter it.  Synchronizes.  Returns what emin_solve returns, or
 * EMIN_ERR_UNSUPPORTED for the forms listed above. */
emin_status emin_solve_taped(emin_problem *prob, double *P_vals, emin_tape **tape);

/* Reverse sweep: given dL_dP (device, nnz(pattern)), ADDS dL/dA to dL_dA
 * (device, nnz(A), A's stored entries in CSR order) and WRITES dL/dP0 to
 * dL_dP0 (device, nnz(P0), P0's stored entries).  May be called several
 * times on one tape.  B and B_c must not have changed since the taped solve.
 * Synchronizes. */
emin_status emin_backward(emin_tape *tape, const double *dL_dP, double *dL_dA, double *dL_dP0);

/* Release a tape.  Tapes must be destroyed before their problem. */
void emin_tape_destroy(emin_tape *tape);

/* Differentiation loss of P (device, on the pattern), with A's current values:
 *     L = w_energy tr(P^T A P) + w_twogrid ||e - P c||_A^2,
 *     c = (P^T A P)^{-1} P^T A e
 * (the energy of Sec. 3, eq. trace, and the A-norm error left by a two-grid
 * coarse correction of the vector e, Sec. 2).  e: device, n entries, or NULL
 * for the energy alone.  *L: host.  dL_dP (device, nnz(pattern), may be NULL)
 * is WRITTEN with dL/dP at fixed A; dL_dA (device, nnz(A), may be NULL) has
 * dL/dA at fixed P ADDED to it (A symmetric).  The coarse system is solved by
 * Jacobi-preconditioned CG to a relative residual of 1e-14.  Synchronizes. */
emin_status emin_loss(emin_problem *prob, const double *P_vals, const double *e,
                      double w_energy, double w_twogrid, double *L, double *dL_dP,
                      double *dL_dA);

/* The loss as a forward / backward pair: emin_loss_forward is emin_loss
 * with no gradient (dL_dP = dL_dA = NULL); emin_loss_backward is emin_loss
 * with *L not returned, dL_dP written and dL_dA accumulated into (either may
 * be NULL).  Same arguments, errors and synchronization as emin_loss. */
emin_status emin_loss_forward(emin_problem *prob, const double *P_vals, const double *e,
                              double w_energy, double w_twogrid, double *L);
emin_status emin_loss_backward(emin_problem *prob, const double *P_vals, const double *e,
                               double w_energy, double w_twogrid, double *dL_dP, double *dL_dA);

/* Thread-local description of the last error on this thread ("" if none). */
const char *emin_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EMIN_H */
