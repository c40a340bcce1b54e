/*
 * gencd.h — C ABI of the GenCD Propose/Update library for MI355X (gfx950).
 *
 * The library solves the l1-regularised loss minimisation problem of Eq. (1)
 * of Scherrer, Halappanavar, Tewari & Haglin, "Scaling Up Coordinate Descent
 * Algorithms for Large l1 Regularization Problems":
 *
 *     min_w  (1/n) sum_i loss(y_i, (Xw)_i) + lambda ||w||_1
 *
 * with the squared loss 1/2 (y-t)^2 or the logistic loss log(1+exp(-yt))
 * (section 1), by the generic coordinate-descent loop of Algorithm 1
 * (Select, Propose, Accept, Update) under the rules of Table 2.
 *
 * Conventions for every call
 *   - Pointers documented "device" point to memory on the current HIP
 *     device; "host" pointers to ordinary host memory.  The caller allocates
 *     and owns every buffer, including the workspace; the library never
 *     allocates or frees device memory and keeps no pointer after a call
 *     returns (the server keeps its arena until gencd_server_destroy).
 *   - All device work is enqueued on the given stream.  Calls that return
 *     results to the host (statistics, lambda_max) synchronise that stream.
 *   - Every call returns a gencd_status.  Arguments are validated on the host
 *     before any device work; on an error no output has been modified unless
 *     stated.  Nothing crosses the ABI as a C++ exception.
 *   - Calls on different streams with disjoint workspaces are independent.
 *     The library has no global mutable state, apart from the static scratch
 *     of gencd_solve_noalloc and the table of its per-device addresses.
 *
 * Matrix X (n x k) is CSC: col_ptr int64[k+1] (col_ptr[0] = 0,
 * non-decreasing, col_ptr[k] = nnz), row_idx int32[nnz] (sorted and unique
 * within a column, each in [0, n)), val float32[nnz].  All three are device
 * pointers.  Labels y are float32[n] (device); the logistic loss needs
 * y_i in {-1, +1}.
 */
#ifndef GENCD_H
#define GENCD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GENCD_OK = 0,
  GENCD_NOT_CONVERGED = 1,        /* warning: outputs valid, stats filled */
  GENCD_ERR_INVALID_ARG = -1,     /* null pointer, bad size or scalar */
  GENCD_ERR_BAD_MATRIX = -2,      /* CSC structure invalid (device check) */
  GENCD_ERR_BAD_LABELS = -3,      /* logistic labels not in {-1, +1} */
  GENCD_ERR_WORKSPACE = -4,       /* workspace null or too small */
  GENCD_ERR_UNSUPPORTED = -5,     /* option combination not implemented */
  GENCD_ERR_DIVERGED = -6,        /* non-finite objective at a check */
  GENCD_ERR_HIP = -7,             /* a HIP runtime call failed */
  GENCD_ERR_BUDGET = -8,          /* server: request larger than the arena */
  GENCD_ERR_TOO_LARGE = -9        /* the problem needs more device scratch than the
                                     fixed static scratch of an allocation-free call */
} gencd_status;

typedef enum { GENCD_SQUARED = 0, GENCD_LOGISTIC = 1 } gencd_loss;

/* Selection / acceptance rules of Table 2 (plus the sequential special cases
 * of section 2.1). */
typedef enum {
  GENCD_CYCLIC = 0,        /* J = {one column}, columns in index order */
  GENCD_STOCHASTIC = 1,    /* J = {one random column} (Shotgun with |J| = 1) */
  GENCD_SHOTGUN = 2,       /* random |J| columns, accept all */
  GENCD_THREAD_GREEDY = 3, /* random |J| columns, best proposal per block of B */
  GENCD_GREEDY = 4,        /* all columns, single best proposal */
  GENCD_COLORING = 5,      /* one colour class per iteration, accept all */
  GENCD_TOP_GREEDY = 6,    /* random |J| columns, the `block` proposals with the smallest
                              phi over the whole window (ties: lowest position);
                              Thread-Greedy with global acceptance, section 4.1 */
  GENCD_BLOCK_SHOTGUN = 7  /* `block` preset random blocks of the live columns, each with
                              its own P_b* = floor(k_b / (2 rho_b)) (section 7); an
                              epoch visits the blocks in a permuted order and each
                              block's members, permuted, in windows of P_b*; accept all */
} gencd_rule;

/* flags */
#define GENCD_WARM_START 0x1u      /* w holds the starting point on entry */
#define GENCD_VALIDATE_DEVICE 0x2u /* check CSC structure and labels on the device */
#define GENCD_USE_GRAPH 0x4u       /* replay each epoch as a captured HIP graph */
#define GENCD_PROFILE 0x8u         /* time every Propose and Update launch with HIP events
                                      (plain launch path only; each epoch starts behind a
                                      short wait on the device clock, about 15 us per
                                      iteration and at most 4 ms, so that the host has
                                      queued the epoch and no event pair spans a wait for
                                      the host: the solve's wall time grows by that much) */
#define GENCD_EXACT_ACCUM 0x10u    /* TwoSum-compensate every atomic update of z */
#define GENCD_FUSED 0x20u          /* accept-all rules except Coloring: fused asynchronous
                                      Propose+Update (section 4.1); each column reads z as
                                      others of its window update it and split columns
                                      are applied one launch later, so the trajectory is
                                      not the Jacobi one (the optimum is the same).  Not
                                      with EXACT_ACCUM or improve_steps (UNSUPPORTED).
                                      gencd_solve_path: one launch per shared window,
                                      improve_steps allowed, EXACT_ACCUM UNSUPPORTED */
#define GENCD_FUSED_EPOCH 0x40u    /* gencd_solve_path with GENCD_FUSED: the whole epoch in one
                                      launch of |J| workgroups, workgroup b taking positions
                                      b, b + |J|, b + 2|J|, ... of the epoch order one column
                                      at a time; at most |J| columns are in flight and none
                                      waits for another (asynchronous Shotgun with |J|
                                      concurrent updates, section 4.1).  UNSUPPORTED without
                                      GENCD_FUSED and in server requests; ignored by the
                                      other calls */

/* Device CSC matrix (see the conventions above). */
typedef struct {
  int64_t n, k, nnz;
  const int64_t *col_ptr;
  const int32_t *row_idx;
  const float *val;
} gencd_csc;

typedef struct {
  int32_t loss;          /* gencd_loss */
  int32_t rule;          /* gencd_rule */
  double lambda;         /* lambda >= 0 of Eq. (1) */
  int64_t select_size;   /* |J| (Shotgun, Thread-Greedy); 0: P* = floor(k_live / (2 rho))
                            clamped to [1, k_live], rho estimated by 20 power
                            iterations (gencd_estimate_rho; section 4.1) */
  int64_t block;         /* B, proposals per accepting block (Thread-Greedy);
                            |J'|, proposals accepted per iteration (Top-Greedy);
                            number of preset blocks, 1..4096 (Block Shotgun) */
  uint64_t seed;         /* seed of the per-epoch selection permutation */
  double kkt_tol;        /* stop when max_j KKT violation <= kkt_tol ... */
  double gap_tol;        /* ... and duality gap <= gap_tol * |objective| (0: off) */
  int64_t max_epochs;    /* epoch = one pass of Select over the live columns */
  int64_t check_every;   /* epochs between FP64 convergence checks; 0: adaptive, a
                            tenth of the epochs run so far (between 1 and 64), so a
                            solve stops at most about 10% of its epochs after its
                            first converged epoch (gencd_solve_path: the epochs of
                            its youngest slot); -m (m >= 1): adaptive with an m-th
                            of the epochs run instead of a tenth (fewer checks,
                            up to about 1/m of the epochs after convergence) */
  uint32_t flags;        /* GENCD_* flags */
  const int32_t *color;  /* COLORING: device int32[k] colours (gencd_color) */
  int32_t num_colors;    /* COLORING: number of colours */
  int32_t piece;         /* nonzeros per piece of a long column (multiple of 64,
                            64..2^22); 0 = library default */
  int32_t group;         /* lanes per short column (4, 8, 16 or 32); columns of
                            at most 4 * group nonzeros are short; 0 = default */
  int32_t improve_steps; /* "Improve delta_j" (Algorithm 3, section 4.1): up to this
                            many further quadratic-approximation steps on each
                            accepted proposal's 1-D objective, from the state at
                            the start of the iteration; stops early once a step
                            no longer changes the increment.  0 = off (default);
                            the paper used 500.  gencd_solve, gencd_step and
                            gencd_solve_path (0..1000000; on the path every slot
                            of a column takes its own steps, with GENCD_FUSED
                            from the z its workgroup read, so concurrent
                            columns may have moved z meanwhile; for a column of
                            at most 32 nonzeros the steps use the hardware
                            exponential and reciprocal, about 1 ulp each) */
  int32_t residual;      /* how Propose forms l'(y_i, z_i) (Algorithm 2): 1 = per
                            entry from the gathered z_hi, z_lo, y of its row;
                            2 = from a residual vector refreshed (one pass over
                            the rows) before the window's Propose, so entries
                            gather 4 bytes; 0 = automatic: 2 when the window's
                            expected nonzeros (|window| nnz / live columns)
                            reach 4 n, else 1.  The same FP32 arithmetic either
                            way.  gencd_solve / gencd_step only */
  int32_t stagger;       /* gencd_solve_path: a lambda takes a free slot only once its
                            predecessor has run this many epochs (or finished), so it
                            starts from a partly converged iterate; 0 = as soon as a
                            slot is free */
} gencd_params;

/* Host-side statistics filled by the solve calls. */
typedef struct {
  int64_t iters;          /* GenCD iterations (Algorithm 1 loop trips) */
  int64_t epochs;
  int64_t coord_updates;  /* accepted proposals */
  int64_t nnz_visits;     /* sum over proposals of nnz_j (Propose work) */
  int64_t nnz_updates;    /* sum over accepted proposals of nnz_j */
  double objective;       /* Eq. (1) at the last check, FP64 from z = Xw */
  double kkt_max;         /* max_j KKT violation at the last check */
  double gap;             /* duality gap P(w) - D(u) at the last check (FP64) */
  double lambda_max;      /* ||X^T l'(y, 0)||_inf / n */
  double seconds;         /* wall time of the call */
  int64_t nnz_w;          /* nonzeros of w at the last check */
  int32_t converged;
  int32_t num_colors;
  /* GENCD_PROFILE: Propose launches, their summed duration (HIP events on
   * the solve's stream) and the algorithmic bytes they moved: 12 B per
   * proposed nonzero (row index, value, and the row's residual) and 28 B per
   * proposed column (column bounds, w, c, delta and phi).  The per-entry
   * form gathers z_hi, z_lo and y (12 B) instead of the residual, so it
   * moves more than this count. */
  int64_t prof_launches;
  double prof_kernel_ms;
  double prof_bytes;
  double rho;             /* spectral-radius estimate when |J| came from it, else 0 */
  int64_t select_size;    /* |J| used by the solve (after any halving by the
                             divergence guard) */
  /* GENCD_PROFILE: Update launches (Algorithm 3), their summed duration (HIP
   * events) and algorithmic bytes: 24 B per nonzero of every accepted column
   * (its row index and value, and a read-modify-write of the 8-byte fitted
   * value pair z_hi, z_lo) plus 8 B per accepted column (w_j, delta_j).
   * Columns whose increment is zero cost nothing in the kernel; their
   * nonzeros still count here, see nnz_scattered. */
  int64_t prof_update_launches;
  double prof_update_ms;
  double prof_update_bytes;
  int64_t nnz_scattered;  /* GENCD_PROFILE: nonzeros the Update launches actually
                             scattered (columns with delta_j != 0); 0 otherwise */
  double z_drift;         /* largest max_i |z_i - (Xw)_i| / rms(Xw) over the FP64
                             checks after the first: z_i is the FP32 pair
                             z_hi + z_lo that the iterations accumulated since the
                             previous re-sync, Xw the FP64 product of the check */
} gencd_stats;

const char *gencd_status_string(int status);

/* Workspace bytes needed by gencd_solve / gencd_step / gencd_check /
 * gencd_lambda_max for this matrix shape and these parameters.  Host only. */
int gencd_workspace_bytes(const gencd_csc *X, const gencd_params *p, size_t *out_bytes);

/* lambda_max = max_j |X_j^T l'(y, 0)| / n in FP64: the smallest lambda at
 * which w = 0 satisfies the optimality conditions of Eq. (1).  *out is host. */
int gencd_lambda_max(const gencd_csc *X, const float *y, int32_t loss, double *out, void *ws,
                     size_t ws_bytes, hipStream_t stream);

/* Solve Eq. (1) by Algorithm 1 with the rule of p->rule.
 *   w: device float32[k]; read as the starting point when GENCD_WARM_START
 *      is set (else zero-initialised), holds the solution on return.
 *   z: device float32[n] or NULL; receives Xw (FP32 rounding of the FP64
 *      product) on return.
 *   stats: host, may be NULL.
 * Returns GENCD_OK when the FP64 KKT check met kkt_tol, GENCD_NOT_CONVERGED
 * after max_epochs, GENCD_ERR_DIVERGED on a non-finite objective. */
int gencd_solve(const gencd_csc *X, const float *y, const gencd_params *p, float *w, float *z,
                void *ws, size_t ws_bytes, hipStream_t stream, gencd_stats *stats);

/* Allocation-free variant of gencd_solve, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The workspace is a static device array of
 * 64 MiB that the library holds on every device it runs on until the
 * process ends; the call itself allocates nothing (no hipMalloc, hipFree or
 * allocating library routine).  Every call on a device shares that device's
 * array and the solve initialises every part of it that it reads, so the
 * contents left by an earlier call do not matter; calls that overlap on one
 * device (several host threads, or streams running concurrently) race on it
 * and must not be made.  Arguments as gencd_solve.  Errors: those of
 * gencd_solve; GENCD_ERR_TOO_LARGE (before any device work) when
 * gencd_workspace_bytes of the problem exceeds 64 MiB; GENCD_ERR_UNSUPPORTED
 * with GENCD_USE_GRAPH or GENCD_PROFILE (they create HIP objects). */
int gencd_solve_noalloc(const gencd_csc *X, const float *y, const gencd_params *p, float *w,
                        float *z, hipStream_t stream, gencd_stats *stats);

/* One iteration of Algorithm 1 on a given selected set, for step-by-step
 * comparison.  J: device int32[nJ] distinct column indices.  The state is
 * (w, z_hi + z_lo), all device float32; z_lo may not be NULL.  The
 * iteration proposes for every j in J from the state at entry (Algorithm 2 /
 * Algorithm 4), accepts all (block == 0 rules) or the best of each block of
 * p->block positions (Thread-Greedy), and updates w, z_hi, z_lo
 * (Algorithm 3).  Optional device outputs of length nJ: g (gradient),
 * delta, phi, accepted (0/1).  The accept rule follows p->rule. */
int gencd_step(const gencd_csc *X, const float *y, const gencd_params *p, const int32_t *J,
               int64_t nJ, float *w, float *z_hi, float *z_lo, float *g, float *delta,
               float *phi, int32_t *accepted, void *ws, size_t ws_bytes, hipStream_t stream);

/* FP64 check of a point w (device float32[k]): z64 = Xw, the gradient
 * g64 = X^T l'(y, z64) / n, the KKT violations, the objective of Eq. (1),
 * nnz(w) and the duality gap, all in double precision.  The gap is P(w)
 * minus the Fenchel dual of Eq. (1) at the scaled residual
 * u = s l'(y, z64) / n, s = min(1, lambda / |g64|_inf), so that
 * P(w) - P* <= gap.  z64 (device double[n]) and g64 (device double[k]) are
 * optional outputs.  Fills stats->objective, kkt_max, gap, nnz_w. */
int gencd_check(const gencd_csc *X, const float *y, int32_t loss, double lambda, const float *w,
                double *z64, double *g64, gencd_stats *stats, void *ws, size_t ws_bytes,
                hipStream_t stream);

/* Position p -> image of the per-epoch selection permutation of m items
 * (keyed Feistel bijection, section 2.1's random subsets).  out: device
 * int32[m]. */
int gencd_select_perm(int64_t m, uint64_t seed, int64_t epoch, int32_t *out, hipStream_t stream);

/* Greedy partial distance-2 colouring of the columns (section 4.1): columns
 * are visited by decreasing nnz (ties by index) and each takes the smallest
 * colour not used by an earlier column sharing a row.  color: device
 * int32[k]; *num_colors: host.  Workspace from gencd_color_workspace_bytes. */
int gencd_color_workspace_bytes(const gencd_csc *X, size_t *out_bytes);
int gencd_color(const gencd_csc *X, int32_t *color, int32_t *num_colors, void *ws,
                size_t ws_bytes, hipStream_t stream);

/* Balanced colouring ("more colours, even class sizes"): every class of the
 * colouring `color` (device int32[k], values in [0, num_colors)) with more
 * than `cap` live columns is split into ceil(size / cap) near-equal parts,
 * its members in column order (rank r of a class of size s split into p
 * parts goes to part floor(r p / s)); cap <= 0 takes the mean class size
 * ceil(k_live / num_colors).  A part of an independent set is independent,
 * so the result is a valid colouring for GENCD_COLORING with classes of at
 * most cap columns.  New colours are numbered class by class, parts in
 * order; an empty column gets its class's first part.
 *   balanced      device int32[k] output (may not alias color)
 *   num_balanced  host: number of colours of the result
 *   ws            device workspace of gencd_balance_workspace_bytes bytes
 * Synchronises the stream.  Errors: INVALID_ARG (also a colour outside
 * [0, num_colors)), WORKSPACE, UNSUPPORTED, HIP. */
int gencd_balance_workspace_bytes(const gencd_csc *X, int32_t num_colors, size_t *out_bytes);
int gencd_balance_colors(const gencd_csc *X, const int32_t *color, int32_t num_colors,
                         int64_t cap, int32_t *balanced, int32_t *num_balanced, void *ws,
                         size_t ws_bytes, hipStream_t stream);

/* Regularisation path: solve Eq. (1) for L values of lambda (any order;
 * decreasing order makes the warm starts effective) on one matrix, B of them
 * at a time in one batched launch sequence (B in {16, 32, 64}).  All slots
 * share the selected sets of the Shotgun rule (p->rule must be
 * GENCD_SHOTGUN, |J| = p->select_size); each slot has its own lambda, its
 * own FP64 KKT test and stops independently.  When a slot finishes, the next
 * lambda takes it, starting from the latest iterate of the previous lambda
 * (section 4.1 mentions starting from a large lambda and decreasing it).
 *   lambdas: host double[L];  W: device float32[L][k] (row t = solution for
 *   lambdas[t]);  Z: device float32[L][n] or NULL (row t = X W[t], the FP32
 *   rounding of the FP64 product of the slot's final check);
 *   stats: host gencd_stats[L].
 * Flags: GENCD_FUSED (one launch per window, see above), GENCD_FUSED_EPOCH
 * (with GENCD_FUSED: one launch per epoch, see above), GENCD_USE_GRAPH
 * (every epoch replays one captured HIP graph; which lambdas the slots hold
 * lives in device arrays, so the graph is captured once per call),
 * GENCD_PROFILE (without GENCD_USE_GRAPH: HIP events around every fused
 * launch, or every Propose and every Update launch; stats[0].prof_launches,
 * prof_kernel_ms and prof_bytes then hold the call's totals for the fused
 * or Propose launches, prof_update_* those of the Update launches.  Bytes
 * per nonzero of a launch's columns: fused 12 + 16 B, Propose 12 + 8 B,
 * Update 8 + 8 B; per column: fused and Propose 20 + 8 B, Update
 * 16 + 4 B; the improve steps re-read nothing for a column of at most 32
 * nonzeros and are not counted).
 * p->improve_steps > 0: "improve delta_j" on every slot's increment
 * (Algorithm 3, section 4.1), before it is applied.
 * Errors: those of gencd_solve (INVALID_ARG also for B, L or a lambda out
 * of range), and UNSUPPORTED for a rule other than SHOTGUN, GENCD_FUSED with
 * GENCD_EXACT_ACCUM, or GENCD_FUSED_EPOCH without GENCD_FUSED.
 * Workspace bytes from gencd_path_workspace_bytes. */
int gencd_path_workspace_bytes(const gencd_csc *X, const gencd_params *p, int32_t B,
                               size_t *out_bytes);
int gencd_solve_path(const gencd_csc *X, const float *y, const gencd_params *p,
                     const double *lambdas, int32_t L, int32_t B, float *W, float *Z, void *ws,
                     size_t ws_bytes, hipStream_t stream, gencd_stats *stats);

/* Schedule autotuner.  Times every candidate schedule (lanes per short
 * column in {4, 8, 16} x nonzeros per long piece in {128, 256, 512} x
 * captured-epoch graph on/off x residual per entry / refreshed vector) on
 * `epochs` epochs of the real solve from w = 0 and returns the fastest in
 * *out; copy out->group, out->piece, out->flags and out->residual into
 * gencd_params to use it.  Results are cached (JSON lines) in cache_path, or
 * in $GENCD_TUNE_CACHE when cache_path is NULL, under a key made of the
 * device, the problem shape and rule, and the histogram of column lengths;
 * a cached key is answered without timing.  w_scratch: device float32[k];
 * the workspace must be at least gencd_workspace_bytes for piece = 128 and
 * group = 4 (the candidate needing the most); candidates that do not fit
 * are skipped. */
typedef struct {
  int32_t group, piece;
  uint32_t flags;            /* GENCD_USE_GRAPH or 0 */
  double seconds_per_epoch;  /* measured on the tuning run */
  int32_t from_cache;
  int32_t residual;          /* gencd_params.residual of the schedule (1 or 2) */
} gencd_schedule;

int gencd_autotune(const gencd_csc *X, const float *y, const gencd_params *p, int32_t epochs,
                   const char *cache_path, float *w_scratch, void *ws, size_t ws_bytes,
                   hipStream_t stream, gencd_schedule *out);

/* Path autotuner: times gencd_solve_path on the caller's lambdas for every
 * slot count B in {16, 32, 64}, each without GENCD_FUSED, with it, and with
 * GENCD_FUSED | GENCD_FUSED_EPOCH, and returns the fastest (B and the flags
 * to add).  Cached like gencd_autotune,
 * under a key that also holds L and the lambda range.
 *   W_scratch  device float32[L][k] (overwritten)
 *   ws         at least gencd_path_workspace_bytes(X, p, 64) bytes
 * Errors: those of gencd_solve_path; NOT_CONVERGED of a candidate run is
 * accepted (its time still counts). */
typedef struct {
  int32_t B;
  uint32_t flags;            /* 0, GENCD_FUSED or GENCD_FUSED | GENCD_FUSED_EPOCH */
  double seconds;            /* whole path, measured on the tuning run */
  int32_t from_cache;
} gencd_path_schedule;

int gencd_autotune_path(const gencd_csc *X, const float *y, const gencd_params *p,
                        const double *lambdas, int32_t L, const char *cache_path,
                        float *W_scratch, void *ws, size_t ws_bytes, hipStream_t stream,
                        gencd_path_schedule *out);

/* ------------------------------------------------------------------------
 * Spectral radius of the column-normalised Gram matrix (section 4.1: Shotgun
 * is guaranteed to converge with at most P* = k / (2 rho) coordinates per
 * iteration, rho the largest eigenvalue of X^T X for unit-norm columns).
 *
 * rho is estimated by power iteration on G = D^{-1/2} X^T X D^{-1/2},
 * D = diag(X^T X), restricted to the non-empty columns, starting from the
 * unit vector with equal entries on those columns: u = G v, rho_t = ||u||,
 * v = u / rho_t.  FP64 on the device.  Each rho_t is a lower bound of rho and
 * the sequence does not decrease.
 *
 *   p            schedule (piece, group) and flags (GENCD_VALIDATE_DEVICE)
 *                are read; loss, lambda and rule are ignored.  May be NULL.
 *   iters        1..1024
 *   rho_hist     host double[iters]: rho_t after iteration t (0 from the
 *                first iteration with G v = 0 on)
 *   k_live       host, may be NULL: number of non-empty columns
 *   select_size  host, may be NULL: floor(k_live / (2 rho_iters)) clamped to
 *                [1, k_live], the |J| gencd_solve takes for select_size 0
 *   ws           device workspace of gencd_rho_workspace_bytes bytes
 * Synchronises the stream.  Errors: INVALID_ARG, BAD_MATRIX (with
 * VALIDATE_DEVICE), WORKSPACE, UNSUPPORTED, HIP.
 * ------------------------------------------------------------------------ */
int gencd_rho_workspace_bytes(const gencd_csc *X, const gencd_params *p, size_t *out_bytes);

/* Per-block estimate behind Block Shotgun (section 7).  The live columns, in
 * the order of a seeded permutation (p->seed), are cut into num_blocks
 * contiguous preset blocks [b k_live / nb, (b+1) k_live / nb); for every
 * block the same power iteration runs on its own normalised Gram matrix.
 *   num_blocks   1..min(k_live, 4096)
 *   iters        1..64 (gencd_solve uses 20)
 *   rho_out      host double[num_blocks]: rho_b after `iters` iterations
 *   pstar_out    host int64[num_blocks]: floor(k_b / (2 rho_b)) clamped to [1, k_b]
 *   ws           device workspace of gencd_block_rho_workspace_bytes bytes
 * Synchronises the stream.  Errors: INVALID_ARG (also num_blocks > k_live),
 * BAD_MATRIX (with VALIDATE_DEVICE), WORKSPACE, UNSUPPORTED, HIP. */
int gencd_block_rho_workspace_bytes(const gencd_csc *X, const gencd_params *p, int64_t num_blocks,
                                    size_t *out_bytes);
int gencd_estimate_block_rho(const gencd_csc *X, const gencd_params *p, int64_t num_blocks,
                             int32_t iters, double *rho_out, int64_t *pstar_out, void *ws,
                             size_t ws_bytes, hipStream_t stream);
int gencd_estimate_rho(const gencd_csc *X, const gencd_params *p, int32_t iters, double *rho_hist,
                       int64_t *k_live, int64_t *select_size, void *ws, size_t ws_bytes,
                       hipStream_t stream);

/* ------------------------------------------------------------------------
 * Continuous-batching server.  Requests are Shotgun solves of Eq. (1)
 * (rule GENCD_SHOTGUN; |J| = select_size, or 0 for P* = floor(k_live /
 * (2 rho)) as in gencd_solve).  They are admitted in arrival order while a
 * slot is free and their state fits in the caller's device arena; a request
 * larger than the whole arena is rejected with GENCD_ERR_BUDGET.  Admitted
 * requests advance together: each round is one Propose launch and one
 * Update launch (Algorithms 2-4, then Algorithm 3) over a device work table
 * holding a window of every admitted request, on the stream given at
 * creation.  Each request keeps its state (w, the fitted values, the epoch
 * order, the FP64 check arrays) in the arena until it finishes; its FP64
 * check runs at each of its epoch ends with an asynchronous read-back, and a
 * request that meets its tolerance leaves the table while the others go on.
 * Results are the checked iterates: the same computation as gencd_solve with
 * the same parameters (default flags), up to the order of the FP32 atomic
 * additions.  Supported flags: GENCD_WARM_START, GENCD_VALIDATE_DEVICE,
 * GENCD_FUSED (the request's Propose launch scatters each column's step as
 * soon as it is formed, section 4.1's fused loops; its columns read the
 * fitted values while others of the window update them, and a round whose
 * requests are all fused is one launch); GENCD_USE_GRAPH is ignored.
 * GENCD_FUSED_EPOCH, GENCD_EXACT_ACCUM, GENCD_PROFILE, other rules and
 * improve_steps give GENCD_ERR_UNSUPPORTED at submission.
 * ------------------------------------------------------------------------ */
typedef struct gencd_server gencd_server;

typedef struct {
  gencd_csc X;          /* device matrix, caller owned, valid until polled */
  const float *y;       /* device labels, idem */
  gencd_params params;  /* loss, lambda, select_size, seed, kkt_tol, ... */
  float *w;             /* device float32[k] solution (read first with WARM_START);
                           it holds iterates while the request runs */
  float *z;             /* device float32[n] fitted values Xw or NULL */
  int64_t user_tag;     /* returned unchanged in the result */
} gencd_request;

typedef struct {
  int64_t ticket, user_tag;
  int32_t status;       /* GENCD_OK, GENCD_NOT_CONVERGED or an error */
  gencd_stats stats;
  double submit_s, start_s, finish_s;  /* seconds since gencd_server_create */
} gencd_result;

typedef struct {
  int32_t running, waiting, finished_unpolled;
  size_t arena_used, arena_bytes;
  int64_t rounds;        /* rounds so far (a Propose and an Update launch, or one
                            launch when every request of the round is fused) */
  int64_t slot_rounds;   /* sum over rounds of the requests each advanced */
  int64_t shared_rounds; /* rounds that advanced two or more requests */
} gencd_server_status;

/* arena: device memory owned by the caller for the server's lifetime (the
 * server keeps 4 MiB plus 104 B per slot of it for its work tables);
 * max_slots: concurrent requests (1..256); stream: the rounds run on it and
 * it must stay valid until gencd_server_destroy.  The device current at
 * creation is used by the server's threads.  The server creates one stream
 * of its own (admission work), events and pinned host buffers, released by
 * gencd_server_destroy. */
int gencd_server_create(void *arena, size_t arena_bytes, int32_t max_slots, hipStream_t stream,
                        gencd_server **out);
/* Arena bytes one request holds while it is admitted (its solve workspace
 * and the best checked iterate), and the fixed part of the arena the server
 * keeps for its work tables; an arena of gencd_server_overhead_bytes(s) plus
 * the sum of any s requests' bytes admits those s requests together. */
int gencd_server_request_bytes(const gencd_csc *X, const gencd_params *p, size_t *out_bytes);
size_t gencd_server_overhead_bytes(int32_t max_slots);
/* Non-blocking; *ticket identifies the request in its result. */
int gencd_server_submit(gencd_server *sv, const gencd_request *req, int64_t *ticket);
/* Moves up to max finished results to out (host).  wait_for > 0 first
 * blocks until that many results are available (or all in flight ended). */
int gencd_server_poll(gencd_server *sv, gencd_result *out, int32_t max, int32_t wait_for,
                      int32_t *n_out);
int gencd_server_info(gencd_server *sv, gencd_server_status *out);
/* Waits for every submitted request, then releases the server. */
int gencd_server_destroy(gencd_server *sv);
/* ------------------------------------------------------------------------
 * Synthetic serving requests on the device (inputs of the serving
 * benchmark; not part of a solve).  Every entry of the n x k matrix is
 * nonzero independently with probability `density` (0 < density < 1), the
 * nonzero values are N(0, 1), and the labels come from a ground truth w*
 * with `support` N(0, 1) weights on non-empty columns: y = Xw* + N(0, 0.01)
 * for GENCD_SQUARED, y = +1 with probability sigma((Xw*)_i) else -1 for
 * GENCD_LOGISTIC.  The result depends only on (n, k, density, seed, loss,
 * support).  Two calls, so that the caller can size row_idx and val:
 *   gencd_gen_count writes col_ptr (device int64[k+1]) and *nnz (host),
 *     synchronising the stream;
 *   gencd_gen_fill writes row_idx (device int32[nnz]), val (device
 *     float32[nnz]) and y (device float32[n]) from that col_ptr.
 * ws: device workspace of gencd_gen_workspace_bytes(n, k) bytes, the same
 * for both calls.  Errors: INVALID_ARG, WORKSPACE, UNSUPPORTED (nnz >= 2^31),
 * HIP. */
int gencd_gen_workspace_bytes(int64_t n, int64_t k, size_t *out_bytes);
int gencd_gen_count(int64_t n, int64_t k, double density, uint64_t seed, int64_t *col_ptr,
                    int64_t *nnz, void *ws, size_t ws_bytes, hipStream_t stream);
int gencd_gen_fill(int64_t n, int64_t k, double density, uint64_t seed, int32_t loss,
                   int32_t support, const int64_t *col_ptr, int32_t *row_idx, float *val, float *y,
                   void *ws, size_t ws_bytes, hipStream_t stream);

/* Host-only replay of the admission policy (capacity planning, tests):
 * request i arrives at arrival[i] (non-decreasing), needs bytes[i] of arena
 * and holds its slot for service[i] seconds; start[i] receives its start time
 * or -1 if it can never fit. */
int gencd_server_plan(size_t arena_bytes, int32_t max_slots, int32_t n, const size_t *bytes,
                      const double *arrival, const double *service, double *start);

#ifdef __cplusplus
}
#endif

#endif /* GENCD_H */
