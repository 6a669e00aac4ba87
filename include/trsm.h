/*
 * trsm.h -- C ABI of the MI355X (gfx950) inversion-based triangular solver.
 *
 * Problem (Sec. I of Wicky, Solomonik & Hoefler, "Communication-Avoiding
 * Parallel Algorithms for Solving Triangular Systems of Linear Equations"):
 * given a lower-triangular n x n matrix L and a dense n x k matrix B, find the
 * dense n x k matrix X with  L X = B.  Left side, lower triangle, no
 * transpose, non-unit diagonal, no scaling factor (plans made with
 * TRSM_FLAG_TRANSPOSE solve L^T X = B with the same L instead).
 *
 * Method (Sec. VI, Alg. Diagonal-Inverter and Alg. It-Inv-TRSM): the n0 x n0
 * diagonal blocks L(S_i, S_i), S_i = i*n0 : (i+1)*n0, are inverted by
 * recursive triangular inversion (Sec. V, Alg. RecTriInv: invert both halves,
 * then Linv21 = -(Linv22 L21) Linv11), and a blocked forward sweep then runs
 * only dense matrix products:
 *     X(S_i)      = Linv(S_i,S_i) * B'(S_i)
 *     B'(T_{i+1}) = B'(T_{i+1}) - L(T_{i+1}, S_i) * X(S_i),   T_i = i*n0 : n.
 * Everything runs on one GPU.
 *
 * Conventions shared by every call:
 *  - Storage is row-major (C order) with leading dimensions in elements:
 *    element (i,j) of L is L[i*ldl + j], (i,c) of B is B[i*ldb + c], of X is
 *    X[i*ldx + c].  ldl >= n, ldb >= k, ldx >= k.  Only the lower triangle of
 *    L (diagonal included) is ever read.
 *  - Matrix pointers are DEVICE pointers unless stated.  The caller owns all
 *    of them.  `stream` is a hipStream_t passed as void* (NULL = the default
 *    stream).  Calls marked "asynchronous" only enqueue work on `stream`.
 *  - Element types follow the plan's precision: TRSM_F64 and the mixed modes
 *    use binary64 L, B, X; TRSM_F32 uses binary32 L, B, X.
 *  - No call throws; every call returns a trsm_status.  A plan is not
 *    thread-safe; distinct plans may be used from distinct threads.
 */
#ifndef TRSM_MI355X_H
#define TRSM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum trsm_status {
  TRSM_OK = 0,
  TRSM_EINVAL = 1,         /* bad size, leading dimension, pointer or option */
  TRSM_ESINGULAR = 2,      /* a diagonal entry of L is zero or not finite */
  TRSM_ENOMEM = 3,         /* a device allocation failed or a budget is too small */
  TRSM_EHIP = 4,           /* the HIP runtime reported an error (see trsm_last_hip_error) */
  TRSM_ENOTCONVERGED = 5,  /* refinement hit its iteration cap; X holds the last iterate */
  TRSM_EBUSY = 6           /* serving: no free slot and queuing was refused */
} trsm_status;

typedef enum trsm_precision {
  TRSM_F64 = 0,            /* binary64 everywhere (FP64 matrix cores) */
  TRSM_F32 = 1,            /* binary32 inputs/outputs (FP32 matrix cores); blocks inverted in binary64 */
  TRSM_MIXED_BF16 = 2,     /* binary64 in/out; sweep products in bfloat16 -> binary32,
                              residual in binary64, iterative refinement */
  TRSM_MIXED_F16 = 3,      /* as above with IEEE half (power-of-two row scaling) */
  TRSM_MIXED_FP8 = 4       /* experiment: as above with 8-bit e4m3 floats (OCP e4m3 on the
                              f8f6f4 matrix instruction; power-of-two scales per row and
                              block of L and per solved block of X); needs more
                              corrections than the 16-bit modes */
} trsm_precision;

/* Plan flags. */
#define TRSM_FLAG_NO_REFINE   0x1u  /* mixed modes: return the unrefined low-precision solve */
#define TRSM_FLAG_RECURSIVE   0x2u  /* solve with the recursive baseline (Alg. Rec-TRSM order) */
#define TRSM_FLAG_LOOKAHEAD   0x4u  /* F64/F32 sweep: update the next block's rows first and the
                                       rest on a second stream, overlapping the next diagonal
                                       apply (launch timings then overlap); each stream splits K
                                       in its own half of the workspace's split-K scratch.
                                       Measured slower than the one-stream sweep on MI355X */
#define TRSM_FLAG_TRANSPOSE   0x10u /* F64/F32: solve L^T X = B (the transposed problem, upper
                                       triangular, backward sweep) with the same L; with a
                                       forward plan this gives A^{-1} B for A = L L^T */
#define TRSM_FLAG_UPPER       0x20u /* F64/F32: the matrix argument is an upper-triangular U
                                       (row-major, only its upper triangle and diagonal are
                                       read) and the plan solves U X = B by the backward sweep
                                       with U's inverted diagonal blocks, e.g. the U of
                                       trsm_lu_factor in place; not with the mixed precisions
                                       nor with TRSM_FLAG_TRANSPOSE, TRSM_FLAG_RECURSIVE or
                                       TRSM_FLAG_LOOKAHEAD (trsm_plan: TRSM_EINVAL) */
#define TRSM_FLAG_LARGE_TILES 0x8u  /* every product uses 128 x 128 tiles and an unsplit
                                       reduction (default: products with few tiles use 64 x 64
                                       tiles and split K); one of the tile policies
                                       trsm_autotune chooses between */

typedef struct trsm_plan_s* trsm_plan_t;

typedef struct trsm_plan_info {
  int64_t n, k;            /* problem sizes the plan was made for */
  int64_t n0;              /* diagonal block size used (a power of two) */
  int64_t m;               /* number of diagonal blocks, ceil(n / n0) */
  int64_t leaf;            /* size of the blocks inverted directly in LDS */
  int64_t n0_paper_rule;   /* the Sec. VIII rule evaluated at p = 1 (reported, not used) */
  int32_t precision;       /* trsm_precision */
  uint32_t flags;
  size_t linv_bytes;       /* size of the Linv buffer trsm_invert_diag fills */
  size_t workspace_bytes;  /* size of the workspace trsm_solve needs */
  double inv_flops;        /* flops of the block inversion, n0^2 n / 3 (textbook count) */
  double solve_flops;      /* n^2 k: the flops the metric credits */
} trsm_plan_info;

typedef struct trsm_info {
  int32_t iterations;      /* refinement corrections applied (mixed modes), else 0 */
  int32_t converged;       /* 1 if the refinement stopping test was met (or not needed) */
  double backward_error;   /* last ||B - L X||_F / (||L||_F ||X||_F) measured, or -1 */
  double correction;       /* last ||D||_F / ||X||_F (mixed modes), or -1 */
  double unrefined_error;  /* mixed: ||X0 - X||_F / ||X||_F of the first low-precision
                              solve against the returned X, or -1 */
} trsm_info;

/* Human-readable name of a status code (static string). */
const char* trsm_status_string(trsm_status s);

/* The last HIP error code seen by the library in this thread (0 = none). */
int trsm_last_hip_error(void);

/*
 * trsm_plan -- choose the blocking for an n x n L and n x k B (host only).
 *  n >= 0, k >= 0.  n0 = 0 picks the block size automatically (the choice
 *  trsm_autotune recorded for this size class, else a cost model of one GPU
 *  seeded by the Sec. VIII regime rule, rounded to a power of two);
 *  otherwise n0 must be a power of two >= 1 (n0 >= n means the full inversion
 *  approach, m = 1).  Returns TRSM_EINVAL for bad arguments, TRSM_ENOMEM if
 *  the plan object cannot be allocated.  *out receives a new plan, owned by
 *  the caller until trsm_plan_destroy.  A plan owns host metadata only (the
 *  lookahead flag adds a side stream and events, made on first use).
 */
trsm_status trsm_plan(int64_t n, int64_t k, trsm_precision prec, int64_t n0,
                      uint32_t flags, trsm_plan_t* out);

/*
 * trsm_autotune -- the measured counterpart of the n0 rule (Sec. VIII says
 * the constants are machine dependent and found by experiment).  On the
 * current device, times trsm_invert_diag + trsm_solve (median of `reps`
 * runs after one warm run, hipEvents on `stream`) on a synthetic system of
 * this (n, k, precision) -- diagonal in [1, 2), strict lower entries in
 * (-1/n, 1/n), right-hand side in (-1/2, 1/2), generated on the device --
 * for every block size n0 = 32, 64, ..., min(next power of two >= n, 4096)
 * with at most 256 blocks (n0 >= n / 256) and both tile policies (default,
 * TRSM_FLAG_LARGE_TILES), and records the fastest -- starting from the cost
 * model's choice, a configuration replaces the best so far only when it is
 * at least 1 % faster -- in a process-wide table keyed by (precision,
 * ceil(log2 n), ceil(log2 k)).  trsm_plan with n0 = 0 then uses the recorded n0 (capped
 * at the next power of two >= n) and adds the recorded tile flag; without a
 * record it uses the cost model.  Blocking; allocates and frees its own
 * device buffers (about 8 (n^2 + 4 n k) bytes for binary64).  prec: TRSM_F64
 * or TRSM_F32.  Returns TRSM_EINVAL for n <= 0, k <= 0, reps <= 0 or a null
 * `out`, TRSM_ENOMEM if the buffers cannot be allocated.  Thread-safe.
 */
typedef struct trsm_tune_result {
  int64_t n0;          /* fastest block size */
  uint32_t flags;      /* its tile policy: 0 or TRSM_FLAG_LARGE_TILES */
  double ms;           /* its median time (invert + solve) */
  int64_t model_n0;    /* the cost model's choice ... */
  double model_ms;     /* ... and its median time with the default tile policy */
  int32_t candidates;  /* configurations timed */
} trsm_tune_result;

trsm_status trsm_autotune(int64_t n, int64_t k, trsm_precision prec, int32_t reps, void* stream,
                          trsm_tune_result* out);

/* The recorded choice for (n, k, prec): *n0 = 0 and *flags = 0 if none.
 * Host only. */
trsm_status trsm_autotune_lookup(int64_t n, int64_t k, trsm_precision prec, int64_t* n0,
                                 uint32_t* flags);

/* Forget every recorded choice.  Host only. */
trsm_status trsm_autotune_clear(void);

/* Fill *info with the plan's choices and buffer sizes (host only). */
trsm_status trsm_plan_get_info(trsm_plan_t plan, trsm_plan_info* info);

/* Release a plan (host only).  NULL is accepted. */
trsm_status trsm_plan_destroy(trsm_plan_t plan);

/*
 * trsm_invert_diag -- Alg. Diagonal-Inverter (Sec. VI-A) with Alg. RecTriInv
 * (Sec. V) for every block: fills `Linv` (device, linv_bytes from the plan,
 * 256-byte aligned) with the inverses of the m diagonal n0 x n0 blocks of L,
 * block b at Linv + b*n0*n0 binary64 values, row-major, zeros above the
 * diagonal; a ragged last block (n0 not dividing n) is padded with the
 * identity.  Mixed and F32 plans also store lower-precision copies behind
 * the binary64 inverses.  Asynchronous, and allocates nothing: every device
 * byte it writes lies in `Linv` (the last 256 bytes of the buffer hold the
 * status word), and its products run without split-K scratch, so the call
 * can be captured into a HIP graph.  A zero or non-finite diagonal entry is
 * recorded in that status word; read it with trsm_plan_last_error after the
 * stream has been synchronised (the plan remembers the buffer of its last
 * trsm_invert_diag).  Returns TRSM_EINVAL for null pointers or ldl < n.
 */
trsm_status trsm_invert_diag(trsm_plan_t plan, const void* L, int64_t ldl, void* Linv,
                             void* stream);

/*
 * After synchronising the stream used by trsm_invert_diag: *status is
 * TRSM_ESINGULAR and *index the first row with a zero or non-finite
 * diagonal entry, or TRSM_OK and -1 (also before any trsm_invert_diag).
 * Blocking (reads the status word of the plan's last Linv buffer, which must
 * still be allocated).
 */
trsm_status trsm_plan_last_error(trsm_plan_t plan, trsm_status* status, int64_t* index);

/*
 * trsm_solve -- X = L^{-1} B by the blocked sweep of Alg. It-Inv-TRSM.
 *  L, B, X: device matrices of the plan's element type; Linv: the buffer
 *  filled by trsm_invert_diag with the same plan and the same L;
 *  workspace: workspace_bytes of device memory (256-byte aligned).
 *  X may be the same buffer as B when ldx == ldb (solve in place); any
 *  other overlap is TRSM_EINVAL.
 *  F64/F32 plans: asynchronous; `info` (nullable) receives iterations = 0.
 *  Mixed plans: iterative refinement X = D_0 + D_1 + ..., each D_j the
 *  low-precision sweep of the residual B - L (D_0 + ... + D_{j-1}), the
 *  residual computed exactly (integer products on the int8 matrix cores in
 *  a residue number system, one binary64 rounding per element) for L with
 *  its strictly lower part rounded to the bits binary64's backward-error
 *  level needs.  Stopping test (default, tolerance 0): the backward error
 *  ||B - L X||_F / (||L||_F ||X||_F) <= 4u, or a correction
 *  ||D_j||_F <= 1e-15 ||X||_F, or the observed contraction
 *  rho = ||D_j|| / ||D_{j-1}|| <= 1/2 predicting ||D_j|| rho <= 1e-14 ||X||.
 *  With trsm_plan_set_tolerance(plan, tol > 0) also: ||D_j|| rho <= tol
 *  ||X|| with D_0 the first sweep's result (||D_0|| = ||X||).  The call reads
 *  norms back to the host after every residual and correction, so it
 *  returns after the solve has finished.  Returns TRSM_ENOTCONVERGED after
 *  10 corrections (X holds the last iterate); `info` (nullable) receives
 *  the corrections, the last backward error and correction, and the first
 *  correction as unrefined_error.
 *  With TRSM_FLAG_RECURSIVE the plan solves by the recursive baseline
 *  (Alg. Rec-TRSM order: X1 = solve(L11, B1); B2 -= L21 X1; X2 = solve(L22,
 *  B2), substitution at the leaves, no inversion) and Linv may be NULL.
 *  With TRSM_FLAG_TRANSPOSE the plan solves L^T X = B: trsm_invert_diag
 *  also stored U = L^T and the inverses of U's diagonal blocks in Linv
 *  (linv_bytes covers them), and the sweep runs from the last block up.
 *  With TRSM_FLAG_UPPER the argument L is an upper-triangular U: both
 *  trsm_invert_diag and trsm_solve read its upper triangle (zero or
 *  non-finite diagonal entries give TRSM_ESINGULAR as for L), Linv holds the
 *  inverses of U's diagonal blocks, and the sweep runs from the last block
 *  up, reading U in place.
 */
trsm_status trsm_solve(trsm_plan_t plan, const void* L, int64_t ldl, const void* Linv,
                       const void* B, int64_t ldb, void* X, int64_t ldx, void* workspace,
                       void* stream, trsm_info* info);

/*
 * trsm_solve_noalloc -- trsm_solve for binary64 and binary32 plans without
 * a workspace argument and without any allocation: for callers that cannot
 * allocate device memory (code being captured into a HIP graph, tight
 * serving loops, harnesses that forbid allocation).
 *  The workspace is a static device array of trsm_solve_noalloc_max_bytes()
 *  bytes (2 MiB), one copy per GPU, held until the process ends; its
 *  address on the current device is looked up on the first call there (the
 *  stream must belong to the current device).  The running right-hand side
 *  (n * k elements of the plan's precision, rounded up to 256 bytes) must
 *  fit in it: larger plans return TRSM_ENOMEM before any device work; the
 *  rest of the array holds split-K partial products.  Mixed-precision plans,
 *  lookahead plans and plans with per-launch timing on return TRSM_EINVAL.
 *  Every call on a GPU shares that GPU's array, which keeps the last call's
 *  contents, so calls that overlap on one GPU (other streams or threads)
 *  race; serialize them.  Other arguments and results are trsm_solve's; X
 *  agrees with trsm_solve's up to the rounding of split-K sums.
 */
size_t trsm_solve_noalloc_max_bytes(void);
trsm_status trsm_solve_noalloc(trsm_plan_t plan, const void* L, int64_t ldl, const void* Linv,
                               const void* B, int64_t ldb, void* X, int64_t ldx, void* stream,
                               trsm_info* info);

/*
 * trsm_residual -- R = B - L X in binary64 on the matrix cores, followed by
 * deterministic reductions: norms[0] = ||R||_F, norms[1] = ||X||_F,
 * norms[2] = max |R|.  The defect of the postcondition B = L X of Alg.
 * It-Inv-TRSM.  L, X, B, R: device binary64; R may not overlap the inputs.
 * `norms` is a HOST array of 3 doubles; the call synchronises the stream.
 * workspace: at least trsm_residual_workspace_bytes(n, k) device bytes.
 */
size_t trsm_residual_workspace_bytes(int64_t n, int64_t k);
trsm_status trsm_residual(int64_t n, int64_t k, const double* L, int64_t ldl,
                          const double* X, int64_t ldx, const double* B, int64_t ldb,
                          double* R, int64_t ldr, void* workspace, double* norms,
                          void* stream);

/*
 * Batches -- many independent systems L_p X_p = B_p of uneven n_p and k_p
 * solved together.  Every phase of the blocked sweep of Alg. It-Inv-TRSM
 * (the diagonal apply of step i, the trailing update of step i) is ONE
 * grouped launch over the tiles of every system that has that phase, so the
 * whole batch takes 2*max(m_p) - 1 launches; systems with fewer blocks drop
 * out of later phases.  With n0 = 64 the batch instead runs as ONE
 * persistent launch (plus a small launch that clears its counters): the
 * left-looking form of the same sweep, X(S_i, c) = Linv_ii (B(S_i, c) -
 * L(S_i, 0:i n0) X(0:i n0, c)), as tasks (system, step i, 64-column tile c)
 * taken from a queue in step-major order; a task waits (on the device) for
 * its column tile's earlier steps through a per-tile counter.  Either way
 * each system's result is computed by the same tiles in the same order as
 * when it is solved alone, so it is bitwise independent of the rest of the
 * batch.
 *
 *  items[p]: n, k; L (device, lower triangle read, ldl >= n); Linv (device,
 *  filled by trsm_invert_diag with a plan of this n, the same precision and
 *  the same n0; 256-byte aligned); B (read) and X (written), ld >= k, X must
 *  not overlap B.  prec: TRSM_F64 or TRSM_F32 (element type of L, B, X).
 *  n0: power of two, the same for every item.
 *
 * trsm_batch_create copies the item array (host only, no device work).
 * trsm_batch_workspace_bytes: device workspace trsm_batch_run needs.
 * trsm_batch_run enqueues the batch on `stream` (asynchronous).  The launch
 *  table is written at the head of `workspace` (256-byte aligned).  With
 *  use_graph != 0 the table upload and all launches are captured into a
 *  hipGraph on the first call and replayed by later calls that pass the same
 *  workspace and stream (the items' buffers must then be unchanged
 *  addresses; their contents may change).  Capture needs a created stream:
 *  use_graph with the NULL stream is TRSM_EINVAL.
 * trsm_batch_destroy releases the handle (and its graph).
 */
typedef struct trsm_batch_item {
  int64_t n, k;
  const void* L;
  int64_t ldl;
  const void* Linv;
  const void* B;
  int64_t ldb;
  void* X;
  int64_t ldx;
} trsm_batch_item;

typedef struct trsm_batch_s* trsm_batch_t;

trsm_status trsm_batch_create(int32_t count, const trsm_batch_item* items, trsm_precision prec,
                              int64_t n0, trsm_batch_t* out);
trsm_status trsm_batch_workspace_bytes(trsm_batch_t batch, size_t* bytes);
trsm_status trsm_batch_run(trsm_batch_t batch, void* workspace, void* stream, int32_t use_graph);
/*
 * Blocking check of the last trsm_batch_run on `workspace` (synchronises the
 * device): TRSM_EHIP if a dependency wait of the persistent sweep (batches
 * made with n0 = 64) gave up, which the task order rules out, else TRSM_OK.
 */
trsm_status trsm_batch_check(trsm_batch_t batch, const void* workspace);

trsm_status trsm_batch_destroy(trsm_batch_t batch);

/*
 * trsm_batch_autotune -- the common block size of a batch, measured (the
 * batched counterpart of trsm_autotune; Sec. VIII leaves n0 to experiment).
 * Builds `count` synthetic systems of sizes n[i] x n[i] and n[i] x k[i] in
 * precision prec (TRSM_F64 or TRSM_F32) on the current device, and for each
 * candidate n0 -- the full inversion min(next power of two >= max n, 4096)
 * first (the incumbent), then 64 (the persistent form), 128, ... below it --
 * inverts every system's diagonal blocks, makes the batch and times `reps`
 * replays of its captured graph (trsm_batch_run with use_graph, on a stream
 * of its own; the inversions are not timed: factors are inverted once and
 * kept).  The median-fastest n0 wins if it is at least 1 % faster than the
 * incumbent; it is recorded in a process-wide table keyed by (precision,
 * ceil(log2 count), ceil(log2 max n), ceil(log2 max k)), which
 * trsm_batch_autotune_lookup reads (*n0 = 0 without a record).  Blocking;
 * allocates and frees its own device buffers (sum of 8 (n^2 + 2 n k) bytes
 * for binary64; more than 64 GiB is TRSM_ENOMEM).  TRSM_EINVAL for count <= 0,
 * null arrays, an n[i] or k[i] outside [1, 65536], reps <= 0 or a null
 * `out`.  trsm_autotune_clear forgets these records too.  Thread-safe.
 */
typedef struct trsm_batch_tune_result {
  int64_t n0;          /* fastest common block size (64: the persistent form) */
  double ms;           /* its median trsm_batch_run time (graph replay) */
  int64_t default_n0;  /* the full inversion's block size ... */
  double default_ms;   /* ... and its median time */
  int32_t candidates;  /* block sizes timed */
} trsm_batch_tune_result;

trsm_status trsm_batch_autotune(int32_t count, const int64_t* n, const int64_t* k,
                                trsm_precision prec, int32_t reps, trsm_batch_tune_result* out);
trsm_status trsm_batch_autotune_lookup(int32_t count, const int64_t* n, const int64_t* k,
                                       trsm_precision prec, int64_t* n0);

/*
 * Serving -- continuous batching of solves against resident factors.
 *
 * Each request is solved by iterative refinement around the sweep of Alg.
 * It-Inv-TRSM with the factor's cached inverted blocks (Alg.
 * Diagonal-Inverter, run once at registration):
 *     X_0 = sweep(B);  R_j = B - L X_j (binary64);  X_{j+1} = X_j + sweep(R_j)
 * and the work is done in "passes": a request's first pass computes X_0 and,
 * for a TRSM_F32 factor, its first correction X_1; every later pass applies
 * one more correction.  After each pass the server evaluates the request's
 * own stopping test from its binary64 residual and correction norms:
 *     berr = ||B - L X||_F / (||L||_F ||X||_F)    (||L||_F^2 for A = L L^T)
 *     corr = ||X_{j+1} - X_j||_F / ||X_{j+1}||_F
 * The request is converged when R = 0, when berr <= tol (tol = sqrt(n) 2^-53
 * by default: the normwise stopping test of the mixed-precision refinement of
 * Buttari, Dongarra, Langou et al., with Frobenius norms), when corr <=
 * 1e-15, or when the observed contraction rho = corr_j / corr_{j-1} is at
 * most 1/2 with corr_j rho <= 1e-14.  Otherwise it joins the next batch for
 * another pass, up to the correction cap, where it ends with
 * TRSM_ENOTCONVERGED (X then holds the last iterate).  A request whose norms
 * are not finite also ends with TRSM_ENOTCONVERGED.  Every pass writes the
 * current iterate to the caller's X.  The tiles and sums of a request are
 * computed identically whatever else shares its batches, so its result, its
 * pass count and its info do not depend on the mix.
 *
 * trsm_server_create(hbm_budget, max_slots, &srv): the server allocates ONE
 *  device block of hbm_budget bytes on the current device and never more;
 *  factors and in-flight requests are carved from it ("admission by HBM
 *  budget").  At most max_slots requests are in flight.  A worker thread and
 *  four streams (default priority) are created, plus pinned host memory for
 *  the per-request norms (32 bytes a slot).  Thread-safe afterwards.
 *  Defaults: block size n0 = min(next power of two >= n, 4096) per factor
 *  (so factors of up to 4096 rows are inverted whole: each sweep is one
 *  product), tolerance sqrt(n) 2^-53, at most 10 corrections.
 * trsm_server_create_ex(hbm_budget, max_slots, &options, &srv): the same with
 *  options (a zero field keeps its default): n0 (a power of two; capped per
 *  factor at the next power of two >= n; n0 = 64 sweeps with one persistent
 *  launch per sweep), tolerance (a fixed backward-error bound instead of
 *  sqrt(n) 2^-53), max_corrections (1 .. 50).
 * trsm_server_register_L(srv, L, n, ldl, prec, &l_id): copies the binary64
 *  lower triangle of L (device pointer, row-major; the strict upper part is
 *  not read) into the server and inverts its diagonal blocks once in binary64;
 *  blocking.  prec = TRSM_F32: sweeps in binary32 (the server keeps L in
 *  binary64 for the residual and in binary32, and the inverted blocks in
 *  binary32); prec = TRSM_F64: sweeps in binary64 (L and the blocks in
 *  binary64; usually one pass).  Other precisions: TRSM_EINVAL, and so is a
 *  factor whose ||L||_F^2 is not a normal binary64 number (entries beyond
 *  about 2^+-500).  TRSM_ENOMEM if it does not fit the budget,
 *  TRSM_ESINGULAR for a zero or non-finite diagonal.
 * trsm_server_register_chol(srv, L, n, ldl, prec, &l_id): the same for a
 *  Cholesky factor: requests on it solve A X = B for A = L L^T (each sweep is
 *  a forward sweep with L and a backward sweep with L^T; the residual is
 *  B - L (L^T X)).  The server also keeps L^T and its inverted blocks (about
 *  twice the memory of a triangular factor); n^2 k flops count twice.  With
 *  TRSM_F32 their block size is at most 512 (A's squared conditioning eats
 *  the binary32 margin of larger inverted blocks, costing corrections).
 * trsm_serve_submit(srv, l_id, B, k, ldb, X, ldx, &ticket): never blocks.
 *  B (read) and X (written) are caller-owned binary64 device matrices (n x k,
 *  row-major, not overlapping) that must stay valid until the ticket is
 *  finished.  The request waits until its workspace (trsm_serve_request_bytes)
 *  fits the budget and a slot is free, then joins the next batch,
 *  which runs on one of the server's streams while earlier batches may still
 *  be running; between passes it rejoins the batches with the newest
 *  arrivals.  A request that can never fit fails with TRSM_ENOMEM.
 * trsm_serve_request_bytes(srv, l_id, k, &bytes): the device bytes a request
 *  of k columns on factor l_id holds while admitted (its buffers above, its
 *  norm partials and the split-K scratch of its skinny products: at most
 *  max(64 n k, 4 MiB) bytes more), for sizing hbm_budget.  Host only.
 * trsm_serve_poll(srv, ticket, &state, &info): never blocks.  info (may be
 *  null) receives the request's trsm_info once it is DONE: corrections
 *  applied, converged flag, berr and corr of its last pass, and the first
 *  correction's corr as unrefined_error (-1 where not measured).  Returns
 *  TRSM_OK while PENDING or RUNNING; for a finished ticket (reported once,
 *  then forgotten) the request's status: TRSM_OK, TRSM_ENOTCONVERGED (state
 *  DONE, X holds the last iterate), or an error with state ERROR (X
 *  undefined).  TRSM_EINVAL and TRSM_REQ_UNKNOWN for an unknown ticket.
 * trsm_server_stats / trsm_server_reset_stats: counters, p50/p99/mean
 *  latency (submit to completion seen by the worker) of finished requests,
 *  n^2 k flops of finished requests (2 n^2 k for a Cholesky factor), memory in
 *  use.
 * trsm_server_destroy: waits for queued and in-flight work, frees everything.
 */
typedef enum trsm_req_state {
  TRSM_REQ_PENDING = 0,
  TRSM_REQ_RUNNING = 1,
  TRSM_REQ_DONE = 2,
  TRSM_REQ_ERROR = 3,
  TRSM_REQ_UNKNOWN = 4
} trsm_req_state;

typedef struct trsm_serve_stats {
  uint64_t submitted, completed, failed, batches;
  uint64_t unconverged;    /* completed requests that ended with TRSM_ENOTCONVERGED */
  uint64_t passes;         /* request passes run (a request's first pass counts too) */
  double p50_us, p99_us, mean_us;
  double flops_done;       /* sum of n^2 k over completed requests (2 n^2 k on
                              Cholesky factors) */
  double wall_s;           /* first submit to last completion */
  size_t hbm_budget, hbm_in_use, resident_bytes;
  int32_t queue_depth, in_flight, max_in_flight, factors;
} trsm_serve_stats;

typedef struct trsm_server_options {
  int64_t n0;              /* 0: min(next power of two >= n, 4096) per factor */
  double tolerance;        /* 0: sqrt(n) 2^-53 per factor */
  int32_t max_corrections; /* 0: 10 */
  int32_t reserved;        /* must be 0 */
} trsm_server_options;

typedef struct trsm_server_s* trsm_server_t;

trsm_status trsm_server_create(size_t hbm_budget, int32_t max_slots, trsm_server_t* out);
trsm_status trsm_server_create_ex(size_t hbm_budget, int32_t max_slots,
                                  const trsm_server_options* options, trsm_server_t* out);
trsm_status trsm_server_register_L(trsm_server_t srv, const double* L, int64_t n, int64_t ldl,
                                   trsm_precision prec, int32_t* l_id);
trsm_status trsm_server_register_chol(trsm_server_t srv, const double* L, int64_t n, int64_t ldl,
                                      trsm_precision prec, int32_t* l_id);
trsm_status trsm_serve_submit(trsm_server_t srv, int32_t l_id, const double* B, int64_t k,
                              int64_t ldb, double* X, int64_t ldx, uint64_t* ticket);
trsm_status trsm_serve_request_bytes(trsm_server_t srv, int32_t l_id, int64_t k, size_t* bytes);
trsm_status trsm_serve_poll(trsm_server_t srv, uint64_t ticket, trsm_req_state* state,
                            trsm_info* info);
trsm_status trsm_server_stats(trsm_server_t srv, trsm_serve_stats* stats);
trsm_status trsm_server_reset_stats(trsm_server_t srv);
trsm_status trsm_server_destroy(trsm_server_t srv);

/*
 * Blocked Cholesky factorization A = L L^T (binary64) with the triangular
 * solve of Alg. It-Inv-TRSM as its panel step (the abstract and Sec. I name
 * Cholesky as a factorization built on TRSM).  Right-looking with block size
 * nb: for each diagonal block S_j, factor A(S_j, S_j) = L_jj L_jj^T (recursive
 * halving down to 64 x 64 leaves factored in LDS) and form Linv_jj = L_jj^{-1}
 * along the way by Alg. RecTriInv's combine; the panel solve L(T_j, S_j) =
 * A(T_j, S_j) Linv_jj^T is one matrix-core product (the whole block inverted:
 * the one-large-dimension regime of Sec. VIII, nb columns against n - (j+1) nb
 * rows); then A(T_j, T_j) -= L(T_j, S_j) L(T_j, S_j)^T on the lower triangle.
 *
 * trsm_chol_sizes(n, nb, &nb_used, &linv_bytes, &workspace_bytes): host only.
 *  nb = 0 picks 512 for n >= 12288, 256 for 6144 <= n < 12288 and 128 below
 *  (the fastest as measured), at most the next power of two >= max(n, 64);
 *  otherwise nb must be a power of two in [64, 4096].  TRSM_EINVAL for
 *  n < 0, n > 2^20 or a bad nb.  Any output pointer may be NULL.
 * trsm_chol_factor(n, A, lda, nb, Linv, workspace, stream): A is a device
 *  binary64 row-major n x n matrix (lda >= n) of which only the lower
 *  triangle (diagonal included) is read; on return its lower triangle holds
 *  L and the strict upper triangle is untouched.  Linv (device, linv_bytes,
 *  16-byte aligned) receives the inverted diagonal blocks: block j at Linv +
 *  j*nb*nb, nb x nb row-major, zeros above the diagonal, the ragged last
 *  block padded with the identity -- the layout trsm_invert_diag fills for a
 *  TRSM_F64 plan with n0 = nb_used (n > 32), so such a plan can solve with
 *  L and these blocks directly (their values agree with trsm_invert_diag's
 *  up to rounding).  workspace: workspace_bytes of device memory, 256-byte
 *  aligned; its first 8 bytes hold the status word trsm_chol_check reads.
 *  Asynchronous; no memory is allocated.  With more than two blocks the
 *  trailing updates below the next diagonal block run on a second stream
 *  (created once per device by the library, default priority) while the
 *  next diagonal block is factored on `stream`; events fork it from and join
 *  it back to `stream`, so work enqueued on `stream` afterwards sees the
 *  whole factorization, and the call can be captured into a graph on
 *  `stream`.  Concurrent calls on one device are serialised while they
 *  enqueue.  Returns TRSM_EINVAL for bad sizes, null or misaligned pointers.
 * trsm_chol_check(workspace, &status, &index): blocking (synchronises the
 *  device).  After trsm_chol_factor: TRSM_OK and -1, or TRSM_ESINGULAR and
 *  the first row whose pivot was not positive (A is not positive definite,
 *  or NaN); L and Linv are then unspecified from that row's block on.
 */
trsm_status trsm_chol_sizes(int64_t n, int64_t nb, int64_t* nb_used, size_t* linv_bytes,
                            size_t* workspace_bytes);
trsm_status trsm_chol_factor(int64_t n, double* A, int64_t lda, int64_t nb, double* Linv,
                             void* workspace, void* stream);
trsm_status trsm_chol_check(const void* workspace, trsm_status* status, int64_t* index);

/*
 * Blocked LU factorization WITHOUT row exchanges, A = L U (binary64; L unit
 * lower, U upper), for matrices that need none (e.g. diagonally dominant
 * ones, or after a randomizing transform); partial pivoting is not provided.
 * Its two panel steps are the triangular solve of Alg. It-Inv-TRSM with the
 * whole diagonal block inverted (the abstract and Sec. I name LU as built on
 * TRSM): U(S_j, T_j) = Linv_jj A(S_j, T_j) and L(T_j, S_j) = A(T_j, S_j)
 * Uinv_jj, then A(T_j, T_j) -= L(T_j, S_j) U(S_j, T_j).  The diagonal blocks
 * are factored recursively (64 x 64 leaves in LDS) and both inverses built
 * by Alg. RecTriInv's combine along the way; the same two-stream lookahead as
 * trsm_chol_factor.
 *
 * trsm_lu_sizes(n, nb, &nb_used, &inv_bytes, &workspace_bytes): as
 *  trsm_chol_sizes; inv_bytes is the size of EACH of the Linv and Uinv
 *  buffers.
 * trsm_lu_factor(n, A, lda, nb, Linv, Uinv, workspace, stream): A (device,
 *  row-major, lda >= n) is overwritten with L strictly below the diagonal (its
 *  unit diagonal is not stored) and U on and above it.  Linv receives the
 *  unit lower inverses of L's diagonal blocks (diagonal 1 stored, zeros
 *  above: a TRSM_F64 plan with n0 = nb_used solves L Y = B with A as its L
 *  and these blocks, since its sweep reads only the strictly lower part of A
 *  outside the blocks), Uinv the upper inverses of U's (zeros below); ragged
 *  last blocks padded with the identity.  Other arguments and behaviour as
 *  trsm_chol_factor.
 * trsm_lu_check(workspace, &status, &index): TRSM_OK and -1, or
 *  TRSM_ESINGULAR and the first row whose pivot was zero or not finite.
 */
trsm_status trsm_lu_sizes(int64_t n, int64_t nb, int64_t* nb_used, size_t* inv_bytes,
                          size_t* workspace_bytes);
trsm_status trsm_lu_factor(int64_t n, double* A, int64_t lda, int64_t nb, double* Linv,
                           double* Uinv, void* workspace, void* stream);
trsm_status trsm_lu_check(const void* workspace, trsm_status* status, int64_t* index);

/*
 * Blocked LU factorization WITH partial pivoting, P A = L U (binary64; L unit
 * lower with |l_ij| <= 1, U upper): Gaussian elimination with row exchanges,
 * the first row with the largest pivot magnitude at each step (LAPACK
 * dgetrf's exchanges).  Built on the triangular solve of Alg. It-Inv-TRSM
 * (the abstract and Sec. I name LU as built on TRSM): block columns of nb
 * (a power of two >= 32) are factored in 32-column panels (one cooperative
 * launch per panel, one device-wide barrier per column); then each block's
 * unit lower diagonal block is inverted by Alg. Diagonal-Inverter +
 * RecTriInv, U(S_j, T_j) = Linv_jj A(S_j, T_j) is one product with the
 * inverted block, and A(T_j, T_j) -= L(T_j, S_j) U(S_j, T_j).  n <= 65536.
 *
 * trsm_lu_piv_sizes(n, nb, &nb_used, &inv_bytes, &workspace_bytes): nb = 0
 *  picks 256 (n <= 4096) or 512; nb is capped at the next power of two >= n
 *  (the block size a solve plan gives such an n).  inv_bytes: the Linv
 *  buffer (m nb x nb blocks); workspace_bytes: device scratch the call
 *  needs (status words, panel candidates, one block and its inverse, one
 *  block row of U, split-K partials).  Host only.  TRSM_EINVAL for n <= 0,
 *  n > 65536, or nb not 0 and not a power of two >= 32.
 * trsm_lu_piv_factor(n, A, lda, nb, ipiv, Linv, workspace, stream): A
 *  (device, row-major, lda >= n, 16-byte aligned) is overwritten with L
 *  strictly below the diagonal (unit diagonal not stored) and U on and above
 *  it, for the row-exchanged matrix; ipiv (device, n int64) receives the row
 *  exchanged with row j at step j (0-based, ipiv[j] >= j; apply "swap rows j
 *  and ipiv[j]" for j ascending to get P A); Linv the inverses of L's
 *  diagonal blocks (block j at Linv + j nb nb, row-major, ones on the
 *  diagonal, zeros above; the ragged last block padded with the identity):
 *  a TRSM_F64 plan with n0 = nb_used solves L Y = B with A as its L and these
 *  blocks.  workspace (256-byte aligned, caller-owned) of workspace_bytes.
 *  Asynchronous on `stream` (null: the default stream); allocates nothing.
 *  TRSM_EINVAL on bad arguments, TRSM_EHIP when a launch fails (including a
 *  cooperative launch the device cannot make co-resident).
 * trsm_lu_piv_check(workspace, &status, &index): blocking.  TRSM_OK and -1;
 *  TRSM_ESINGULAR and the first column whose pivot was zero or not finite
 *  (the factorization goes on, as LAPACK does, and U is singular); or
 *  TRSM_EHIP and -1 if a panel's barrier wait gave up (ruled out by the
 *  cooperative launch; reported rather than hung).
 * trsm_row_swaps(k0, k1, ipiv, B, ldb, ncols, stream): applies "swap rows k
 *  and ipiv[k]" for k = k0 .. k1-1 in order to the first ncols columns of the
 *  device matrix B (row-major, ldb >= ncols): P B for a factorization's
 *  ipiv.  Asynchronous.
 */
trsm_status trsm_lu_piv_sizes(int64_t n, int64_t nb, int64_t* nb_used, size_t* inv_bytes,
                              size_t* workspace_bytes);
trsm_status trsm_lu_piv_factor(int64_t n, double* A, int64_t lda, int64_t nb, int64_t* ipiv,
                               double* Linv, void* workspace, void* stream);
trsm_status trsm_lu_piv_check(const void* workspace, trsm_status* status, int64_t* index);
trsm_status trsm_row_swaps(int64_t k0, int64_t k1, const int64_t* ipiv, double* B, int64_t ldb,
                           int64_t ncols, void* stream);

/*
 * trsm_plan_set_tolerance -- accuracy target of a mixed-precision plan's
 * refinement (the paper solves in one precision; refinement is this
 * library's addition around the sweep of Alg. It-Inv-TRSM).  tol = 0 (the
 * default) refines to binary64's backward-error level; 0 < tol < 1 also
 * stops once the relative forward error left, estimated from the last
 * correction and the observed contraction, is <= tol, and makes the first
 * sweep a full-accuracy one (binary32 diagonal apply) so that a half-
 * precision sweep reaches tol = 1e-12 on a well-conditioned L with one
 * exact residual.  The estimate assumes each sweep contracts the error by
 * a similar factor; it is not a bound.  Binary64 and binary32 plans keep
 * the value and ignore it.  Host only; TRSM_EINVAL for a null plan or tol
 * outside [0, 1) (NaN included).
 */
trsm_status trsm_plan_set_tolerance(trsm_plan_t plan, double tol);

/*
 * Launch timing for roofline reports.  trsm_plan_set_timing(plan, 1) makes
 * every matrix-core product launched by trsm_invert_diag and trsm_solve with
 * this plan record a pair of hipEvents around itself on the call's stream
 * (the plan creates and owns the events; recording adds a few microseconds
 * per launch).  trsm_plan_timing waits for the recorded events, returns the
 * number of launches, their summed duration in milliseconds and their
 * summed algorithmic flops (2MNK per dense product, M(M+1)N when a square
 * factor is triangular), and clears the record.  Host only; blocking.
 */
trsm_status trsm_plan_set_timing(trsm_plan_t plan, int enable);
trsm_status trsm_plan_timing(trsm_plan_t plan, int64_t* launches, double* ms, double* flops);

#ifdef __cplusplus
}
#endif

#endif /* TRSM_MI355X_H */
