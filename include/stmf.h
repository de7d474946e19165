/* stmf.h -- C ABI of the MI355X (gfx950) FastSTMF library.
 *
 * Sparse tropical matrix factorization R ~ U (x) V over the max-plus semiring,
 * (U (x) V)_ij = max_l (U_il + V_lj)  (paper, Section 2), scored by the b-norm
 * sum |R_ij - (U (x) V)_ij| over the observed cells only (Section 3.6), with
 * the factors updated by FastSTMF (Algorithm 3: ByRow strategy, random row
 * permutation, TD_A candidate selection, wide orientation) through the F-ULF
 * and F-URF steps (Algorithms 1 and 2).
 *
 * Conventions for every entry point:
 *   - Matrices are dense, row-major, contiguous.  Values are IEEE binary32
 *     (float); error sums are binary64 (double).
 *   - Pointers documented "device" point to GPU memory owned by the caller;
 *     "host" pointers to host memory owned by the caller.  The library never
 *     allocates GPU memory: calls that need scratch take a workspace
 *     (ws, ws_bytes) whose required size is returned by the matching
 *     *_workspace() function; ws must be 256-byte aligned.
 *   - M is a uint8 mask: 0 = missing, nonzero = observed.  Values of R at
 *     missing cells are never used in arithmetic (they may be NaN).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     stream-ordered; argument errors are detected and returned before any
 *     work is queued.  Calls documented "synchronous" wait for the stream.
 *   - Indices are 0-based.  Ties in an argmax go to the lowest index
 *     (Section 3.2.1, TD selection).
 *   - Return value: an stmf_status.  After STMF_EHIP the stream's state is
 *     unspecified.
 *   - Thread safety: calls on different streams with disjoint buffers and
 *     workspaces may run concurrently; the library keeps no global mutable
 *     state besides a per-device property cache.
 */
#ifndef STMF_H
#define STMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STMF_OK = 0,
  STMF_EINVAL = 1,      /* bad argument (size, rank, index, null pointer, option)   */
  STMF_EEMPTY_LINE = 2, /* a row or column of M has no observed cell                 */
  STMF_ERANGE = 3,      /* integer-exact mode: a value with |x| >= 2^24, or a value
                           outside the finite range the library accepts (|x| < 1e30) */
  STMF_ENOMEM = 4,      /* workspace too small or misaligned                         */
  STMF_EHIP = 5,        /* a HIP runtime call failed                                 */
  STMF_EBUSY = 6,       /* serving engine: no slot or not enough memory free         */
  STMF_ETIMEOUT = 7     /* a fit stopped: a group barrier waited longer than its
                           bound (barrier_wait_us; 4 s by default)             */
} stmf_status;

/* Short English description of a status code (static string). */
const char* stmf_status_str(int status);

/* Library version as "major.minor.patch" (static string). */
const char* stmf_version(void);

/* ---------------------------------------------------------------- primitives */

/* Max-plus product P = U (x) V (Section 2):
 *   P[i*n + j] = max_l U[i*r + l] + V[l*n + j],  U m x r, V r x n (device).
 * argmax (device, nullable, m x n int32) gets the lowest l reaching the max
 * (the index f(i,j) of Section 3.2.1).  1 <= r <= 64; m, n >= 1. */
int stmf_maxplus_product(const float* U, const float* V, int m, int r, int n,
                         float* P, int32_t* argmax, void* stream);

/* Workspace bytes of stmf_masked_error for an m x n matrix. */
size_t stmf_masked_error_workspace(int m, int n, int r);

/* Masked b-norm (Section 3.6, restricted to observed cells):
 *   err[0] = sum over observed (i,j) of |R_ij - (U (x) V)_ij|
 * Each difference is one FP32 subtraction, widened to FP64 and summed in a
 * fixed order.  td_col (device, nullable, n doubles) gets the per-column sums
 * td_col(j) of Section 3.2.1.  R m x n, M m x n, U m x r, V r x n (device);
 * err is a device pointer to one double. */
int stmf_masked_error(const float* R, const uint8_t* M, const float* U,
                      const float* V, int m, int n, int r, double* err,
                      double* td_col, void* ws, size_t ws_bytes, void* stream);

/* stmf_masked_error without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation).  Same arguments (minus ws, ws_bytes), kernels and
 * result bits as stmf_masked_error.  Its scratch is a static device array
 * of 8 MiB per device, held from the library's load until the process ends:
 * shapes whose partials need more (ceil(m/64) * ceil(n/64) * 64 doubles
 * above 2^20, e.g. m = n = 8192 fits, m = 8192, n = 8256 does not) return
 * STMF_ENOMEM before any work is queued.  No call allocates: the first call
 * on a device only looks up the array's device address.  Every call on a
 * device shares that device's array, so calls that overlap on one device
 * (on different streams, or from several threads) race and must be
 * serialised by the caller. */
int stmf_masked_error_noalloc(const float* R, const uint8_t* M, const float* U,
                              const float* V, int m, int n, int r, double* err,
                              double* td_col, void* stream);

/* Workspace bytes of stmf_update_U / stmf_update_V. */
size_t stmf_update_workspace(int m, int n, int r);

/* F-ULF (Algorithm 1) at (i, j, k), in place on U (m x r) and V (r x n):
 *   U_col_prev <- U[:,k], V_row_prev <- V[k,:]   (the backups Algorithm 1 returns)
 *   U_ik <- R_ij - V_kj
 *   V_kc <- min over observed t of R_tc - U_tk   for every column c
 *   U_tk <- min over observed c of R_tc - V_kc   for every row t
 *   err[0] <- masked b-norm of the new state
 * The call never accepts or restores: the caller compares err with the
 * previous error and copies the backups back to reject.  Requires M[i,j]
 * observed (checked, synchronously: STMF_EINVAL otherwise) and 0 <= k < r.
 * Every row and column of M must hold an observed cell (a residual over an
 * empty line is undefined): otherwise STMF_EEMPTY_LINE, returned before any
 * launch (M is copied back and checked on the host, synchronously on the
 * stream), so U and V are untouched.
 * U_col_prev (m floats), V_row_prev (n floats), err (1 double): device. */
int stmf_update_U(const float* R, const uint8_t* M, float* U, float* V, int m,
                  int n, int r, int i, int j, int k, float* U_col_prev,
                  float* V_row_prev, double* err, void* ws, size_t ws_bytes,
                  void* stream);

/* F-URF (Algorithm 2): as stmf_update_U with V_kj <- R_ij - U_ik as the
 * written value and the two residual steps in the order row residual of
 * V_k. into U_.k first, then column residual of U_.k into V_k.. */
int stmf_update_V(const float* R, const uint8_t* M, float* U, float* V, int m,
                  int n, int r, int i, int j, int k, float* U_col_prev,
                  float* V_row_prev, double* err, void* ws, size_t ws_bytes,
                  void* stream);

/* ---------------------------------------------------------------- fitting */

typedef struct {
  int init_mode;        /* 0 random integers in [init_lo, init_hi] (default),
                           1 Random Acol (Section 3.3): U_tl = mean of the observed
                             values of row t over acol_p randomly drawn columns,
                             falling back to the row's observed mean,
                           2 given: U0 (host, m' x rank, working orientation)     */
  float init_lo, init_hi;
  int acol_p;           /* columns averaged per U column in Random Acol (default 5) */
  const float* U0;      /* host, init_mode 2                                        */
  const int32_t* perm;  /* host, nullable: working-row permutation (m' entries)     */
  double eps;           /* stop when a pass lowers the error by less (0 = off)      */
  int count_scope;      /* TD_A counts over: 0 observed cells (default), 1 all cells */
  int noop_rule;        /* 1 (default): a trial whose written value equals the
                           stored one on a component last set by an accepted
                           update is rejected without evaluation                     */
  int integer_exact;    /* 1: STMF_ERANGE unless every observed |R| and |U0| < 2^24  */
  void* decision_log;   /* device, nullable: one stmf_log_rec per row visit          */
  int log_cap;          /* capacity of decision_log in records                       */
  int batch_first;      /* speculative trials in the first batch of a row's first
                           visit; 0 (default): 512 / tiles per workgroup, a power
                           of two, at least 4.  Later visits of a row start with
                           the power of two at or above the trials its previous
                           visit needed (at least 16)                           */
  int batch_max;        /* largest batch, <= 1024; 0 (default): 2048 / tiles per
                           workgroup, a power of two in [64, 1024].  The trial
                           buffers of the workspace are sized by it              */
  int group_size;       /* workgroups cooperating on one fit (0 = automatic)          */
  int max_row_visits;   /* stop after this many row visits (0 = no limit)            */
  int selection;        /* ByRow choice of (j, k) within a row visit (Sec. 3.2.1):
                           0 TD_A (default, Algorithm 3): columns by td_col
                             descending, k counted most often in the two argmax
                             multisets of row i and column j;
                           1 TD: the row's observed columns by the entry error
                             |R_ij - (U (x) V)_ij| descending, k = f(i, j);
                           2 TD_B: columns as TD_A, j0 the first of them, i0 the
                             first working row (td_col does not depend on the
                             row), k = f(i, j0) if (U (x) V)_{i j0} >=
                             (U (x) V)_{i0 j}, else f(i0, j);
                           3 SEQ: every (j, k, operation) of the row, j and k
                             ascending, F-ULF first; the smallest error below
                             the current one is applied (the first on ties).
                           Ties in every order: the lower index first.         */
  int perm_mode;        /* working-row order when perm is null (Sec. 3.3):
                           0 random permutation drawn from the seed (default),
                           1 PermR: rows by increasing minimum observed value,
                             ties by the lower working index,
                           2 none (identity),
                           3 PermC: rows as given (perm, else identity) and the
                             working columns by increasing minimum observed
                             value, ties by the lower index (V's columns are
                             put back at the output).
                           With 1-3 the seed's stream starts with the initial U. */
  int strategy;         /* 0 ByRow (default; Sec. 3.2.1, with `selection`),
                           1 ByElement (Sec. 3.2.2 and its supplementary
                             pseudocode): every observed entry of each working
                             row in working column order, k = f(i, j), entries
                             with R_ij = (U (x) V)_ij skipped, F-ULF then F-URF;
                             an accepted update does not end the row visit.
                             `selection` is ignored.  decision_log: one record
                             per accepted update (trials and no-op skips since
                             the previous record of the visit) and one closing
                             each row visit (j = -1).  The paper's
                             STMF_ByElement_PermC_TD_W is strategy 1 with
                             perm_mode 3.
                           2 ByMatrix (Sec. 3.2.3 and its supplementary
                             pseudocode): `iters` counts iterations, each with
                             at most one accepted update: every observed cell
                             is keyed by td_row(i) + td_col(j) - td(i, j) (FP64)
                             and tried by that key descending (ties row-major)
                             with k = f(i, j) and one operation drawn per cell
                             tried (F-URF when the top bit of output c of
                             SplitMix64 seeded with seed ^ 0xA0761D6478BD642F
                             is set, c counting the fit's cells tried, no-op
                             skips included) until the first strict decrease;
                             an iteration without one ends the fit.
                             decision_log: one record per iteration (row = the
                             accepted row, else -1).  The paper's
                             STMF_ByMatrix_NoPerm_TD_W is strategy 2 with
                             perm_mode 2.  stmf_fit only (the batched and
                             serving calls return STMF_EINVAL); the workspace
                             grows by about 20 bytes per cell.                  */
  int barrier_wait_us;  /* bound of each wait at the fit's group barrier, in
                           microseconds: 0 the default (4 s); a fit whose wait
                           runs out stops with STMF_ETIMEOUT.  A negative value
                           ends a wait at its first poll that finds the
                           barrier still closed, so a fit on many workgroups
                           stops at one of its first barriers (for tests of
                           the abort path).                                   */
} stmf_options;

/* Per-row-visit decision record (decision_log). */
typedef struct {
  int32_t iter, row, trials, noops, j, k, op, pad; /* op 0 F-ULF, 1 F-URF; j = -1: none */
  double e;                                        /* error after the visit             */
} stmf_log_rec;

/* Counters of a finished fit. */
typedef struct {
  long long trials;       /* trials the method evaluates (up to each accepted one) */
  long long spec_trials;  /* trials evaluated, speculative ones included            */
  long long noops;        /* trials skipped by the no-op rule                       */
  long long accepted;     /* accepted updates                                       */
  long long row_visits;
  long long cells;        /* sum over evaluated trials of the observed-cell count   */
  int iters_done;         /* passes run (fewer than iters at a fixed point)         */
  int transposed;         /* 1 if the working orientation is R^T                    */
  int m_work, n_work;     /* working shape (m' <= n')                               */
  int group_size;         /* workgroups used                                        */
  int nlog;               /* row visits logged (may exceed log_cap)                 */
  long long batches;      /* speculative batches evaluated                          */
  double phase_ms[8];     /* time of the fit kernel's phases on the group leader,
                             by index: 0 row start, 1 batch lists, 2 residual pass,
                             3 error reduction and decision, 4 apply and refresh,
                             5 bookkeeping, 6 error pass, 7 unused                  */
  double kernel_ms;       /* fit kernel time, HIP events on the fit's stream        */
} stmf_fit_info;

/* Defaults for every option. */
void stmf_options_default(stmf_options* opt);

/* Workspace bytes of stmf_fit for an m x n matrix at this rank and options. */
size_t stmf_fit_workspace(int m, int n, int rank, int iters, const stmf_options* opt);

/* FastSTMF (Algorithm 3).  Synchronous.
 *   R, M: m x n (device).  U_out: m x rank, V_out: rank x n (device), in the
 *   caller's orientation and row order.  err_traj (host, nullable): iters + 1
 *   doubles, err_traj[p] = error after pass p (after initialisation for p = 0);
 *   after a fixed point (a pass with no accepted update) or the eps stop the
 *   rest is padded with the last value.  info (host, nullable).
 *   seed drives SplitMix64: the working-row permutation is drawn first
 *   (Durstenfeld shuffle; not with perm_mode 1 or 2), then the initial U.
 * Errors: STMF_EINVAL, STMF_EEMPTY_LINE, STMF_ERANGE, STMF_ENOMEM, STMF_EHIP,
 * STMF_ETIMEOUT. */
int stmf_fit(const float* R, const uint8_t* M, int m, int n, int rank, int iters,
             uint64_t seed, float* U_out, float* V_out, double* err_traj,
             const stmf_options* opt, stmf_fit_info* info, void* ws,
             size_t ws_bytes, void* stream);

/* Setup draws of stmf_fit without fitting (host outputs): the working-row
 * permutation (m' = min(m, n) entries) and the initial U (m' x rank, working
 * orientation, before Random Acol averaging when init_mode = 1, which instead
 * writes the drawn column indices, rank x acol_p, as floats).  perm_mode 2
 * gives the identity; perm_mode 1 (PermR depends on R, not on the seed) is
 * STMF_EINVAL unless perm is given. */
int stmf_draw_init(int m, int n, int rank, uint64_t seed, const stmf_options* opt,
                   int32_t* perm_out, float* U0_out);

/* ---------------------------------------------------------------- batched */

/* One problem of a batched fit.  R, M, U_out, V_out, err_traj: device.
 * U_out holds `restarts` consecutive m x rank blocks, V_out `restarts`
 * rank x n blocks and err_traj `restarts` blocks of iters + 1 doubles.
 * status (written by the call) is per problem. */
typedef struct {
  const float* R;
  const uint8_t* M;
  int m, n, rank, iters;
  uint64_t seed;
  float* U_out;
  float* V_out;
  double* err_traj;
  int status;
  int pad;
} stmf_problem;

/* Workspace bytes of stmf_fit_batched with these problems and options on the
 * current device (the group size, and with it each fit's layout, depends on
 * group_size, on the problems and on how many fit-kernel workgroups the
 * device holds at once); 0 for invalid arguments or when the device cannot
 * be queried. */
size_t stmf_fit_batched_workspace(const stmf_problem* probs, int nprob, int restarts,
                                  const stmf_options* opt);

/* Many independent fits (Algorithm 3 for each, as stmf_fit) in one
 * persistent launch: the grid is cut into groups of G workgroups that take
 * fits from a device queue, largest estimated work first, until it is empty.
 * G = opt->group_size (at most the co-resident workgroup count), or with 0
 * the library's choice from the fits' work (a power of two up to 64).  The
 * device side (queue reset, the launch, every fit's output and trajectory)
 * is one captured HIP graph launched on `stream`.  A fit's result equals
 * stmf_fit's with the same seed and options on any group size.  With one
 * restart a problem's fit uses its seed; with several, restart q uses output
 * q of SplitMix64 seeded with the problem's seed.  max_row_visits > 0 stops
 * every fit after that many row visits (a prefix, for timing: the outputs
 * are then those of the state reached).  Synchronous.  info (host,
 * nullable) gets the summed counters and group_size the G used.  Options
 * decision_log, perm, init_mode 2 and strategy 2 are rejected; a problem
 * whose input fails the checks gets its status and no fit, the others run. */
int stmf_fit_batched(stmf_problem* probs, int nprob, int restarts,
                     const stmf_options* opt, stmf_fit_info* info, void* ws,
                     size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- serving */

typedef struct stmf_engine stmf_engine;

/* A continuous-batching engine over a caller-owned device arena (ws, bytes).
 * Up to max_slots fits are resident at once; each holds its working matrix,
 * factors and state in the arena from admission to retirement.
 * opt->group_size is the most workgroups one job runs on (0: no limit but
 * the co-resident workgroup count): a job gets the smaller of it and its tile
 * count (64 x 64 tiles of the working matrix), fixed at admission, and its
 * result is that of stmf_fit with that group_size and the same seed and
 * options (with group_size 0, stmf_fit's own result).  Options decision_log, perm,
 * init_mode 2, max_row_visits and strategy 2 are rejected (STMF_EINVAL). */
int stmf_engine_create(void* ws, size_t ws_bytes, int max_slots,
                       const stmf_options* opt, stmf_engine** out);
void stmf_engine_destroy(stmf_engine* eng);

/* Arena bytes one job of this shape needs (admission footprint), with the
 * default options (acol_p 5, batch_max 0) and one workgroup per job. */
size_t stmf_job_footprint(int m, int n, int rank, int iters);

/* The same for a job of this engine (its options and group size); 0 for an
 * invalid shape. */
size_t stmf_engine_job_footprint(const stmf_engine* eng, int m, int n, int rank,
                                 int iters);

/* Admit a job: copies R/M (device) into the arena and initialises the fit.
 * STMF_EBUSY if no slot or not enough contiguous arena memory is free.
 * Stream-ordered on `stream`; *slot gets the job's slot. */
int stmf_engine_admit(stmf_engine* eng, const float* R, const uint8_t* M, int m,
                      int n, int rank, int iters, uint64_t seed, int* slot,
                      void* stream);

/* Advance every active job by at most max_rows row visits.  With one
 * workgroup per job this is one launch whose workgroups take jobs from a
 * queue; with larger groups the jobs (in slot order) are laid side by side
 * over as many launches as the co-resident workgroups need.  Stream-ordered;
 * call stmf_engine_poll after synchronising the stream to see which jobs
 * finished.  STMF_ETIMEOUT from poll: a group barrier waited more than its
 * bound (another kernel held the device's compute units). */
int stmf_batch_tick(stmf_engine* eng, int max_rows, void* stream);

/* Ticks as a captured HIP graph (on = 1, the default) or as eager launches
 * (on = 0).  A graph holds the tick's launches (with one workgroup per job, a
 * fill kernel resetting the queue and the fit kernel); it is captured again
 * when the launch plan (jobs per launch and their groups) or max_rows
 * changes, and the device table of resident jobs is uploaded only when that
 * set changes.  Both give the same results. */
int stmf_engine_set_graph(stmf_engine* eng, int on);

/* Synchronous: *done = 1 when the job in `slot` has finished. */
int stmf_engine_poll(stmf_engine* eng, int slot, int* done, void* stream);

/* Copy a finished job's results out (device U_out m x rank, V_out rank x n,
 * host err_traj iters + 1 or NULL) and free its slot and arena memory.
 * Synchronous. */
int stmf_engine_retire(stmf_engine* eng, int slot, float* U_out, float* V_out,
                       double* err_traj, stmf_fit_info* info, void* stream);

/* ---------------------------------------------------------------- quality */

/* Workspace bytes of stmf_distance_correlation for N samples. */
size_t stmf_dcor_workspace(int N);

/* Distance correlation (Sec. 3.6, the DC of Szekely, Rizzo and Bakirov,
 * Ann. Statist. 35(6), 2007; V-statistic form) of the samples x[0..N) and
 * y[0..N) (device, FP32).  out (host, 4 doubles): dCor, dCov^2(x, y),
 * dVar^2(x), dVar^2(y); dCor = 0 when a variance is 0 (N = 0 gives zeros).
 * row_terms (device, nullable, N x 5 doubles): per sample k the sums over
 * all l of |x_k - x_l|, |y_k - y_l|, their product and their squares.
 * Every sum is FP64 in a fixed order (deterministic).  Synchronous.
 * Errors: STMF_EINVAL (N < 0, null pointer), STMF_ENOMEM (workspace smaller
 * than stmf_dcor_workspace(N) or not 256-byte aligned), STMF_EHIP. */
int stmf_distance_correlation(const float* x, const float* y, int N, double* out,
                              double* row_terms, void* ws, size_t ws_bytes,
                              void* stream);

/* Workspace bytes of stmf_completion_metrics (0 for invalid sizes). */
size_t stmf_completion_metrics_workspace(int m, int n, int r);

/* Completion quality of a factorization on a held-out split (Sec. 3.6 and the
 * 20% held-out protocol of Sec. 3.7), with P = U (x) V formed in FP32
 * (R, M_train, M_test m x n row-major, U m x r, V r x n; all device):
 *   out[0] RMSE-A = sqrt(mean over M_train cells of (R - P)^2)
 *   out[1] RMSE-P = sqrt(mean over M_test cells of (R - P)^2)
 *   out[2] DC of the M_test cells' (R, P) pairs (row-major order)
 *   out[3], out[4] the numbers of training and held-out cells
 * out: host, 5 doubles.  A cell in both masks counts in both; an empty set
 * gives RMSE 0.  Differences and sums FP64, fixed orders.  Synchronous.
 * Errors: STMF_EINVAL, STMF_ENOMEM, STMF_EHIP. */
int stmf_completion_metrics(const float* R, const uint8_t* M_train,
                            const uint8_t* M_test, const float* U, const float* V,
                            int m, int n, int r, double* out, void* ws,
                            size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* STMF_H */
