/*
 * tpilu.h -- C ABI of the gfx950 level-of-fill ILU(k) library.
 *
 * What it computes (Dong & Cooperman, "A Bit-Compatible Shared Memory
 * Parallelization for ILU(k) Preconditioning and a Bit-Compatible
 * Generalization to Distributed Memory"):
 *
 *   tpilu_symbolic   Phase I, Sec. 2.2, Algorithm 1 with the levels of Def. 2.3:
 *                    the pattern of the filled matrix F = L~ + U~ - I, every
 *                    entry of level <= k.
 *   tpilu_numeric    Phase II, Eq. 2 and Eqs. 6a/6b: row-wise IKJ elimination
 *                    of A restricted to that pattern.
 *   tpilu_apply      y = U~^-1 L~^-1 b, the triangular solves of Eq. 1
 *                    (forward substitution Eq. 3b, then backward substitution).
 *   tpilu_gmres      restarted GMRES(m) preconditioned on the right by
 *                    M = L~ U~ (Sec. 2: the solver works on A U~^-1 L~^-1).
 *   tpilu_apply_adjoint / tpilu_numeric_adjoint
 *                    reverse-mode derivative of b -> U~^-1 L~^-1 b and of the
 *                    elimination, giving d/d(values of A) and d/db.
 *   tpilu_batched_graph_*
 *                    many matrices sharing one pattern: all numeric
 *                    factorizations plus all solves captured in one HIP graph.
 *
 * Results are bit-identical to the plain sequential algorithm: every entry of
 * F receives its updates in ascending pivot order, every product and every
 * difference is rounded on its own (no FMA contraction), divisions and
 * square roots are correctly rounded IEEE-754 binary64, and every reduction
 * has one fixed shape that does not depend on the launch configuration.
 *
 * Conventions for every entry point
 *   - 0-based indices.  A CSR row lists its columns strictly ascending and
 *     must store its diagonal (its value may be 0).  Every stored entry is an
 *     entry of level 0, explicit zeros included.
 *   - All double/int arrays passed as arguments are DEVICE pointers (memory
 *     of the ctx's device) unless the parameter comment says "host".  The
 *     caller owns them; the library never frees or keeps them beyond the
 *     call, except where a graph handle records them (see below).
 *   - Batches: `batch` instances share one pattern; their values are stored
 *     entry-major, instance-minor: value of entry p of instance b is at
 *     val[p * batch + b].  Vectors likewise: v[i * batch + b].
 *   - Every call enqueues its work on the ctx stream and returns without
 *     waiting, except where a host output (bad_row, iters, relres, info) is
 *     requested: then it waits for the stream and reports.
 *   - Errors: every entry point returns a tpilu_status; nothing aborts and no
 *     C++ exception crosses the ABI.  tpilu_last_error(ctx) gives a message.
 *   - The bit pattern 0x7FF4A5A5A5A5A5A5 (one signalling-NaN payload) is
 *     reserved: the kernels use it to mark values not yet produced.  An input
 *     value with exactly that pattern is replaced by the default quiet NaN
 *     and the call reports TPILU_E_INVAL.
 *   - Calls that use the same pattern handle must not run concurrently (they
 *     share the handle's scratch memory and control block).
 */
#ifndef TPILU_H
#define TPILU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPILU_API __attribute__((visibility("default")))

typedef enum {
    TPILU_OK = 0,
    TPILU_E_INVAL = 1,     /* malformed CSR, bad size or argument, reserved NaN in input */
    TPILU_E_NOMEM = 2,     /* device allocation failed */
    TPILU_E_ZEROPIVOT = 3, /* a final pivot f_jj is +-0; the smallest such j is reported */
    TPILU_E_DEVICE = 4,    /* a HIP runtime call failed */
    TPILU_E_NOTCONV = 5,   /* GMRES reached maxit without meeting rtol */
    TPILU_E_TIMEOUT = 6    /* a kernel's bounded wait for a dependency ran out (watchdog) */
} tpilu_status;

typedef struct tpilu_ctx_s *tpilu_ctx;
typedef struct tpilu_pattern_s *tpilu_pattern;
typedef struct tpilu_graph_s *tpilu_graph;

/* Optional device allocator: alloc returns device memory of the ctx's device
 * (NULL on failure); free releases it.  With both NULL the library uses
 * hipMalloc/hipFree.  Only handle creation and workspace growth allocate. */
typedef void *(*tpilu_alloc_fn)(size_t bytes, void *user);
typedef void (*tpilu_free_fn)(void *ptr, void *user);

/* Library context bound to one device and one HIP stream (a hipStream_t
 * passed as void*; NULL = the device's null stream). */
TPILU_API tpilu_status tpilu_ctx_create(int device, void *hip_stream, tpilu_alloc_fn alloc,
                                        tpilu_free_fn free_fn, void *user, tpilu_ctx *out);
TPILU_API tpilu_status tpilu_ctx_set_stream(tpilu_ctx ctx, void *hip_stream);
TPILU_API void tpilu_ctx_destroy(tpilu_ctx ctx);
TPILU_API const char *tpilu_status_string(tpilu_status st);
TPILU_API const char *tpilu_last_error(tpilu_ctx ctx);

/* Watchdog for the dependency waits inside the persistent kernels: a wait
 * gives up after `timeout_us` microseconds of wall-clock time (0 = library
 * default, 10 s), every other wait of the call then gives up at once, and the
 * call reports TPILU_E_TIMEOUT.  `skip_publish_row` >= 0 makes the numeric
 * kernel never publish that row (a host-forced failure for testing the
 * watchdog); -1 turns that off. */
TPILU_API tpilu_status tpilu_ctx_set_watchdog(tpilu_ctx ctx, uint32_t timeout_us,
                                              int64_t skip_publish_row);

/* Number of wavefronts launched for the persistent kernels (numeric, solves,
 * adjoints); 0 = library default (the resident maximum).  Any value >= 1
 * gives the same bits; it only changes speed.  Used to test that claim. */
TPILU_API tpilu_status tpilu_ctx_set_grid(tpilu_ctx ctx, int32_t waves);

/* Launch shape of the single-instance triangular solves: 0 = automatic
 * (lane per row when a triangle's rows hold at most 40 entries on average
 * and a dependency level at least max(64, 16 x that average) rows, else a
 * wavefront per row), 1 = a wavefront per row (on the whole device or on
 * one XCD, see tpilu_ctx_set_placement), 2 = one workgroup on one CU (a lane
 * per row, rows handed over through an LDS ring; measured far slower than
 * mode 1 on every workload tried, kept as the alternative shape), 3 = a lane
 * per row (64 rows per wavefront) over the whole device.  The same setting picks the shape of the
 * two products of tpilu_apply_inverse: 1 a wavefront per row, 3 a thread per
 * row, 0 automatic (64 rows per wavefront staged through LDS when the
 * longest row of F is at most 1.5 x the average and the average at most 512
 * entries, else a wavefront per row).  Same bits in every mode. */
enum { TPILU_SOLVER_AUTO = 0, TPILU_SOLVER_DEVICE = 1, TPILU_SOLVER_WORKGROUP = 2, TPILU_SOLVER_LANES = 3 };
TPILU_API tpilu_status tpilu_ctx_set_solver(tpilu_ctx ctx, int mode);

/* Kernel of the single-instance numeric factorization: 0 = automatic (the
 * dataflow kernel when the pattern's rows fit its LDS staging, the strict
 * lower part holds at least 4n entries, an entry receives fewer than 12
 * updates on average and a dependency level holds fewer than 64 rows on
 * average, else the pivot-serial one),
 * 1 = dataflow (lanes own the entries of a row and take
 * their updates in ascending pivot order; a later tpilu_numeric fails with
 * TPILU_E_INVAL if the pattern's rows do not fit), 2 = pivot-serial (the
 * wavefront walks the pivots of a row in ascending order, lanes over one
 * pivot's updates).  Same bits in every mode. */
enum { TPILU_NUMERIC_AUTO = 0, TPILU_NUMERIC_FLOW = 1, TPILU_NUMERIC_PIVOT = 2 };
TPILU_API tpilu_status tpilu_ctx_set_numeric(tpilu_ctx ctx, int mode);

/* Rounding of the update of Eq. 6b (f_jt <- f_jt - l_jh u_ht) in the numeric
 * factorization (tpilu_numeric and the batched graphs created afterwards):
 * 0 (default) rounds the product and the difference on their own, 1 rounds
 * the exact f_jt - l_jh u_ht once (a fused multiply-add).  Both are fixed
 * by IEEE-754 binary64 alone, so either mode gives the same bits in every
 * kernel, launch shape and placement, and matches a sequential CPU
 * elimination computed the same way; the two modes differ from each other in
 * the last bits.  The divisions, the substitutions, the incomplete inverses
 * and the reverse mode are not affected.  TPILU_E_INVAL for other values. */
TPILU_API tpilu_status tpilu_ctx_set_fused(tpilu_ctx ctx, int on);

/* Placement of the single-instance numeric kernels, of the
 * wavefront-per-row solves and of the single-instance transposed solves of
 * tpilu_apply_adjoint: 0 = automatic (the numeric kernels on the whole
 * device; a solve on one XCD when its device-wide shape would take at most
 * 256 wavefronts, i.e. a dependency level holds fewer than 32 rows, or fewer
 * than 64 short ones, and a row half at most 128 entries on average),
 * 1 = the whole device, 2 = one XCD (then also the batched factorization
 * and solves, and the dependency-level computation of tpilu_symbolic, one XCD
 * per dependency graph, when its nodes have long dependency lists).  On one
 * XCD, grid wavefronts are
 * launched per XCD; the first workgroup to start names its XCD and the
 * workgroups of the other XCDs exit at once.  Values are then handed from
 * row to row through that XCD's L2 (ordinary stores, agent-scope loads)
 * instead of through memory, a round trip of about 0.5 us instead of 0.9 us
 * on MI355X: deep, narrow dependency graphs gain, work that needs many rows
 * in flight loses the other XCDs.  Same bits in every placement.
 * Assumption: that a workgroup-scope store by one CU is seen by an
 * agent-scope load from another CU of the same XCD rests on the hardware
 * (the CU's vector L1 writes through to the XCD's L2, which serves the
 * agent-scope load), not on a promise of the scoped memory model; it is
 * tested bit for bit in every placement (and under the race check build),
 * and placement 1 never relies on it. */
enum { TPILU_PLACE_AUTO = 0, TPILU_PLACE_DEVICE = 1, TPILU_PLACE_XCD = 2 };
TPILU_API tpilu_status tpilu_ctx_set_placement(tpilu_ctx ctx, int where);

/* Rows per ticket of the kernels that give a wavefront one row at a time
 * (numeric factorization, wavefront-per-row solves, incomplete inverses):
 * a wavefront takes `rows` consecutive positions of the dependency-level
 * order from the shared counter and works through them in order.  0 =
 * automatic, else 1 to 64.  Automatic: 1 for the numeric factorization
 * (its kernels overlap a row's work with the wait on earlier levels, which
 * a group would serialise); for the solves 1, 2 or 3 and for the inverses 1
 * or 2, growing with the average rows per dependency level.  Same bits for every value;
 * it only changes speed.  Returns TPILU_E_INVAL outside [0, 64]. */
TPILU_API tpilu_status tpilu_ctx_set_group(tpilu_ctx ctx, int32_t rows);

/* Task counters the same kernels draw their groups of rows from: groups are
 * dealt round robin to `counters` counters on separate cache lines, so that
 * wide dependency levels are not held up by the atomics on one address.
 * 0 = automatic, else 1 to 8 (never more than the launch's wavefronts).
 * Same bits for every value.  Returns TPILU_E_INVAL outside [0, 8]. */
TPILU_API tpilu_status tpilu_ctx_set_tickets(tpilu_ctx ctx, int32_t counters);

/* Kernel timing.  With timing on, the library brackets the main kernel of
 * every numeric factorization, forward solve and backward solve it launches
 * with a pair of hipEvents recorded on the ctx stream (outside graph
 * capture).  tpilu_ctx_read_timing waits for those events, returns the summed
 * duration in milliseconds and the number of launches of one kernel kind
 * (TPILU_KERNEL_*) since the last read, and resets that kind. */
enum { TPILU_KERNEL_NUMERIC = 0, TPILU_KERNEL_FORWARD = 1, TPILU_KERNEL_BACKWARD = 2 };

/* Per-row timeline for analysing the dependency critical path: with a
 * device buffer of 4n uint64 set (NULL turns it off), the single-instance
 * numeric factorization and forward solve record, for every row i, the
 * wall-clock tick (s_memrealtime, the device's wall clock rate) at which a
 * wavefront started it in buf[i] and published it in buf[n + i]; the
 * backward solve uses buf[2n + i] and buf[3n + i].  The numeric
 * factorization also records in buf[2n + i] when the row's last wait on a
 * pivot ended (left untouched if it never waited) and in buf[3n + i] when it
 * began to publish.  The buffer must hold 4n entries of every pattern used
 * while it is set. */
TPILU_API tpilu_status tpilu_ctx_set_trace(tpilu_ctx ctx, uint64_t *rows4n);
TPILU_API tpilu_status tpilu_ctx_set_timing(tpilu_ctx ctx, int on);
TPILU_API tpilu_status tpilu_ctx_read_timing(tpilu_ctx ctx, int kernel, double *total_ms /* host */,
                                             int64_t *launches /* host */);

/* ---------------------------------------------------------------------------
 * Phase I -- symbolic factorization (Sec. 2.2, Algorithm 1; Def. 2.3).
 *
 * Input: the structure of A, n x n, nnz entries: rowptr[n+1] (int64, device),
 * col[nnz] (int32, device).  k >= 0 is the level limit; any k >= n-1 gives the
 * complete LU pattern.  The library copies the structure; the arrays may be
 * freed after the call.  On success *out receives a pattern handle that
 * holds, on the device: the pattern of F (rows sorted), the level of every
 * entry, the diagonal slot of every row, the map from A's entries to F's
 * slots, and the per-row update schedule the numeric phase replays.  The
 * pattern is immutable and is reused by any number of numeric calls.
 * Errors: TPILU_E_INVAL for a malformed CSR (unsorted or duplicate column,
 * out-of-range index, missing diagonal, rowptr not monotone), n or nnz out of
 * range (n < 2^31, nnz(F) < 2^31); TPILU_E_NOMEM; TPILU_E_DEVICE.
 * Waits for the stream (the pattern size is needed on the host).
 * ------------------------------------------------------------------------- */
TPILU_API tpilu_status tpilu_symbolic(tpilu_ctx ctx, int64_t n, int64_t nnz, const int64_t *rowptr,
                                      const int32_t *col, int32_t k, tpilu_pattern *out);

typedef struct {
    int64_t n, nnz_a, nnz_f;
    int64_t nnz_l;       /* strictly lower entries of F (L~ without its unit diagonal) */
    int64_t nnz_u;       /* entries on and above the diagonal */
    int64_t n_updates;   /* number of f_jt <- f_jt - f_jh f_ht operations of Phase II */
    int32_t k;
    int32_t max_row;     /* longest row of F */
    int32_t max_lrow;    /* most pivots in one row */
    int32_t depth_l;     /* rows on the longest dependency chain of L~ (forward order) */
    int32_t depth_u;     /* rows on the longest dependency chain of U~ (backward order) */
    int32_t overflow_rows; /* rows the symbolic pass had to redo in global memory */
    int32_t flow_ready;  /* 1 if the dataflow numeric kernel can run on this pattern */
    int32_t long_rows;   /* rows the symbolic pass built with its larger LDS maps */
} tpilu_pattern_info_t;

TPILU_API tpilu_status tpilu_pattern_info(tpilu_pattern pat, tpilu_pattern_info_t *info /* host */);

/* Copy the pattern out (device pointers, each nullable): rowptr[n+1] int64,
 * col[nnz_f] int32, diag[n] int32 (slot of f_ii), level[nnz_f] uint8 (level of
 * each entry, saturated at 255), a2f[nnz_a] int32 (F slot of A's entry p). */
TPILU_API tpilu_status tpilu_pattern_export(tpilu_ctx ctx, tpilu_pattern pat, int64_t *rowptr,
                                            int32_t *col, int32_t *diag, uint8_t *level,
                                            int32_t *a2f);
TPILU_API void tpilu_pattern_destroy(tpilu_pattern pat);

/* ---------------------------------------------------------------------------
 * Phase II -- numeric factorization (Eq. 2, Eqs. 6a/6b).
 *
 * a_val[nnz_a * batch]: values of A in the pattern's A order.  f_val[nnz_f *
 * batch] receives F: strictly lower slots hold L~ (unit diagonal implicit),
 * the others hold U~.  F starts as A with fill entries +0.0; for each row j
 * ascending and each pivot h < j of row j ascending: f_jh <- f_jh / f_hh, then
 * f_jt <- f_jt - f_jh * f_ht for every t > h stored in rows h and j.
 * A zero pivot does not stop the elimination (IEEE division gives inf/NaN);
 * the call returns TPILU_E_ZEROPIVOT and *bad_row (host, nullable) receives
 * the smallest row whose final pivot is +-0, or -1 (for batches: smallest
 * over all instances).  With bad_row == NULL the call does not wait and the
 * status of the device work is read later with tpilu_pattern_check.
 * Batches (batch > 1) whose longest row of F has more than 80 entries keep
 * each in-flight row in a global-memory workspace that the pattern owns and
 * reuses (up to 1 GiB; fewer wavefronts when a row is very long), else in
 * LDS; TPILU_E_NOMEM if it cannot be allocated.  Same bits either way.
 * ------------------------------------------------------------------------- */
TPILU_API tpilu_status tpilu_numeric(tpilu_ctx ctx, tpilu_pattern pat, const double *a_val,
                                     int32_t batch, double *f_val, int64_t *bad_row);

/* Wait for the stream and report the sticky device status of the last calls
 * on this pattern (zero pivot, watchdog, reserved NaN), then clear it.
 * bad_row (host, nullable) as for tpilu_numeric. */
TPILU_API tpilu_status tpilu_pattern_check(tpilu_ctx ctx, tpilu_pattern pat, int64_t *bad_row);

/* ---------------------------------------------------------------------------
 * Apply the preconditioner (Eq. 1): y = U~^-1 (L~^-1 b).
 *   forward  (Eq. 3b): x_i = b_i - sum_{h<i} f_ih x_h, subtractions in
 *                      ascending h;
 *   backward:          y_i = (x_i - sum_{j>i} f_ij y_j) / f_ii, subtractions
 *                      from right to left (j descending), then the
 *                      division.  The paper leaves this order open; right
 *                      to left is fixed here because the value that arrives
 *                      last (that of the nearest row) is then the last term
 *                      of the chain.
 * f_val, b, y: [n * batch] / [nnz_f * batch] device arrays; x_out (nullable,
 * n * batch) receives the intermediate x.  b and y may not alias.
 * ------------------------------------------------------------------------- */
TPILU_API tpilu_status tpilu_apply(tpilu_ctx ctx, tpilu_pattern pat, const double *f_val,
                                   int32_t batch, const double *b, double *y, double *x_out);

/* tpilu_apply for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, and harnesses that forbid hipMalloc.
 * Same result, bit for bit, as tpilu_apply(ctx, pat, f_val, batch, b, y,
 * NULL); the intermediate x is kept in a fixed scratch array of the library
 * (4,194,304 doubles = 32 MiB per device, held by each device the library
 * runs on until the process ends) instead of the pattern's workspace.  The
 * call allocates nothing and creates no timing events.  Rejects n * batch >
 * 4,194,304 with TPILU_E_INVAL (nothing is launched); TPILU_E_DEVICE if the
 * scratch's device address could not be taken when the ctx was created.
 * Every call on one device shares that device's scratch, which keeps the
 * last call's contents: calls that overlap on one device (any stream, any
 * ctx, any pattern) race and must be ordered by the caller.  Status
 * (reserved NaN, watchdog) is read with tpilu_pattern_check. */
TPILU_API tpilu_status tpilu_apply_noalloc(tpilu_ctx ctx, tpilu_pattern pat, const double *f_val,
                                           int32_t batch, const double *b, double *y);

/* ---------------------------------------------------------------------------
 * Restarted GMRES(m), right preconditioned by M = L~ U~ (single instance).
 * Modified Gram-Schmidt, Givens rotations with rho = sqrt(a*a + b*b), inner
 * loop stopped when the implicit residual |g_{j+1}| <= rtol ||b||, outer
 * loop stopped on the true residual; maxit counts inner iterations over all
 * cycles.  Inner products use one fixed shape: 16384 strided partial sums
 * (lane l adds elements l, l+16384, ... in ascending order from +0.0) then
 * a pairwise tree (strides 1, 2, 4, ...).  SpMV row sums run from +0.0 in
 * ascending column order.
 * a_val: values of A (the pattern's A structure); f_val: the factor; b, x:
 * n-vectors, x holds x0 on entry and the result on return.  iters, relres
 * (host) receive the inner iteration count and ||b - A x|| / ||b||; hist
 * (host, nullable, maxit entries) receives |g_{j+1}| per inner iteration.
 * Returns TPILU_E_NOTCONV (with the last x) when maxit is reached.
 * ------------------------------------------------------------------------- */
TPILU_API tpilu_status tpilu_gmres(tpilu_ctx ctx, tpilu_pattern pat, const double *a_val,
                                   const double *f_val, const double *b, double *x,
                                   int32_t restart, int32_t maxit, double rtol, int32_t *iters,
                                   double *relres, double *hist);

/* ---------------------------------------------------------------------------
 * Level-based incomplete inverses (Sec. 3.5, the optional TPIILU(k) step):
 * the triangular solve stage becomes two matrix-vector products.
 *
 * tpilu_inverse computes, from a factor F of this pattern, G shaped like F:
 *   strict lower slots: the inverse of L~ kept on L~'s pattern, entry (i, t)
 *     = -beta_it, beta_it = f_it - sum over the pivots h of row i with t < h,
 *     in ascending h, of f_ih beta_ht (Eqs. 5, 6c, 6d); contributions to
 *     positions outside the pattern are dropped;
 *   upper slots (diagonal included): the inverse of U~ kept on U~'s pattern,
 *     rows from the last to the first, row i = (e_i - sum over the pivots
 *     j > i of row i, from right to left, of u_ij * (row j of the inverse)) /
 *     u_ii (the paper omits these details; this is its order for the U~
 *     stage).
 * Rows run in dependency-level order; the result is bit-identical to the
 * sequential recurrence.  f_val, g_val: [nnz_f] device arrays, no aliasing;
 * batch must be 1.  The first call on a pattern builds the update lists
 * (kept with the pattern).  Waits for the stream; reports a watchdog timeout
 * like the factorization.
 * ------------------------------------------------------------------------- */
TPILU_API tpilu_status tpilu_inverse(tpilu_ctx ctx, tpilu_pattern pat, const double *f_val, int32_t batch,
                                     double *g_val);

/* y = U~~^-1 (L~~^-1 b) with the incomplete inverses G (Eq. 3a):
 *   x_i = (sum over t < i of G_it b_t, from +0.0 in ascending t) + b_i,
 *   y_i = sum over t >= i of G_it x_t, from +0.0 in ascending t.
 * Fully parallel (two products).  g_val [nnz_f], b, y [n], x_out (nullable,
 * [n]) receives x; no two vectors may alias; batch must be 1. */
TPILU_API tpilu_status tpilu_apply_inverse(tpilu_ctx ctx, tpilu_pattern pat, const double *g_val,
                                           int32_t batch, const double *b, double *y, double *x_out);

/* ---------------------------------------------------------------------------
 * BiCGSTAB, the Krylov method of the paper's experiments (Sec. 4), right
 * preconditioned like tpilu_gmres: the textbook iteration with the shadow
 * residual fixed to the first residual, every scalar and vector step one
 * fixed expression (beta = (rho / rho_old) * (alpha / omega);
 * p = r + beta * (p - omega * v); s = r - alpha * v; x = (x + alpha * ph) +
 * omega * sh; r = s - omega * t), inner products of the fixed shape above.
 * m_val: the factor F (inverse = 0, M^-1 by the two substitutions) or the
 * incomplete inverses G (inverse != 0, by two products).  maxit and *iters
 * count half steps (one per preconditioner application); hist (host,
 * nullable, maxit entries) gets ||s|| or ||r|| after each half step.  Stops
 * when that norm <= rtol ||b||.  Returns TPILU_E_NOTCONV on a breakdown (a
 * zero rho, (rs, v), (t, t) or omega) or when maxit is reached, with the last
 * x, *iters and the true *relres = ||b - A x|| / ||b||.
 * ------------------------------------------------------------------------- */
TPILU_API tpilu_status tpilu_bicgstab(tpilu_ctx ctx, tpilu_pattern pat, const double *a_val,
                                      const double *m_val, int32_t inverse, const double *b, double *x,
                                      int32_t maxit, double rtol, int32_t *iters, double *relres, double *hist);

/* tpilu_gmres with M^-1 applied through the incomplete inverses g_val
 * (tpilu_apply_inverse) instead of the two substitutions; every other step,
 * argument and result as for tpilu_gmres. */
TPILU_API tpilu_status tpilu_gmres_inverse(tpilu_ctx ctx, tpilu_pattern pat, const double *a_val,
                                           const double *g_val, const double *b, double *x, int32_t restart,
                                           int32_t maxit, double rtol, int32_t *iters, double *relres,
                                           double *hist);

/* Building blocks exposed for testing and reuse (single instance). */
/* y = A x with the pattern's A structure. */
TPILU_API tpilu_status tpilu_spmv(tpilu_ctx ctx, tpilu_pattern pat, const double *a_val,
                                  const double *x, double *y);
/* *result (host) = fixed-shape inner product of x and y, both of length n. */
TPILU_API tpilu_status tpilu_dot(tpilu_ctx ctx, int64_t n, const double *x, const double *y,
                                 double *result);

/* Measurements of the dependency critical path (no numeric result).
 *
 * tpilu_numeric_critical_path runs the dataflow elimination kernel in a mode
 * that carries, instead of values, the length of the longest chain of
 * dependencies ending in each entry of F, and writes the largest length over
 * F into *length (host).  On a chain, every hand-off between rows (an update
 * of f_jt needs f_ht, and l_jh needs f_hh, from row h) weighs w_hop, and
 * every l of a row (a division whose result entries of the same row wait
 * for) weighs w_step; other work inside a row weighs nothing.  With w_hop = 1
 * and w_step = 0 the length is the number of row-to-row hand-offs that must
 * happen one after another in any parallel factorization that keeps the
 * bits of Eq. 2; with both set to measured times it models a latency floor.
 * Weights must be finite and >= 0.  TPILU_E_INVAL when the pattern's rows do
 * not fit the dataflow kernel.  Waits for the stream.
 *
 * tpilu_handoff_probe has two wavefronts pass a value back and forth
 * `rounds` times (1 .. 2^24) through device memory with the publish and poll
 * operations of the persistent kernels, on one XCD (same_xcd != 0: plain
 * stores kept in that XCD's L2) or on two different XCDs (stores written
 * through), and writes the mean round trip in nanoseconds into
 * *ns_round_trip (host); one hand-off is half of it.  Waits for the stream;
 * TPILU_E_TIMEOUT if no partner wavefront appeared within the watchdog. */
TPILU_API tpilu_status tpilu_numeric_critical_path(tpilu_ctx ctx, tpilu_pattern pat, double w_hop,
                                                   double w_step, double *length);
TPILU_API tpilu_status tpilu_handoff_probe(tpilu_ctx ctx, int32_t same_xcd, int32_t rounds,
                                           double *ns_round_trip);

/* Givens rotations of `count` pairs (a_i, b_i), with the device code of the
 * rotation step of tpilu_gmres: rho_i = sqrt(a_i * a_i + b_i * b_i) (each
 * product and the sum rounded on their own, no hypot), c_i = a_i / rho_i,
 * s_i = b_i / rho_i, every operation correctly rounded binary64.  All five
 * arrays device, [count], no aliasing of inputs with outputs.  Exposed so
 * that the square root and the divisions of the GMRES step can be checked
 * bit for bit on many operands. */
TPILU_API tpilu_status tpilu_givens(tpilu_ctx ctx, int64_t count, const double *a, const double *b,
                                    double *rho, double *c, double *s);

/* ---------------------------------------------------------------------------
 * Reverse mode of y = U~^-1 L~^-1 b (given x = L~^-1 b and y from the forward
 * pass, and ybar = dLoss/dy):
 *   z = U~^-T ybar: z_i = (ybar_i - sum_{j<i} f_ji z_j) / f_ii, ascending i,
 *                   subtractions in ascending j;
 *   w = L~^-T z:    w_i = z_i - sum_{j>i} f_ji w_j, descending i,
 *                   subtractions in descending j;
 *   bbar = w;  fbar_ij = -(z_i * y_j) on U~ (j >= i);  fbar_ih = -(w_i * x_h)
 *   on the strictly lower part.
 * All arrays device, [n * batch] or [nnz_f * batch].
 * ------------------------------------------------------------------------- */
TPILU_API tpilu_status tpilu_apply_adjoint(tpilu_ctx ctx, tpilu_pattern pat, const double *f_val,
                                           int32_t batch, const double *x, const double *y,
                                           const double *ybar, double *bbar, double *fbar);

/* Reverse sweep of the elimination (adjoint of Eqs. 6a/6b).  fbar[nnz_f *
 * batch] holds dLoss/dF on entry and is overwritten; abar[nnz_a * batch]
 * receives dLoss/d(values of A).  Rows are undone in descending order; for
 * pivot h of row j with l = f_jh:
 *   lbar = fbar_jh - sum_t fbar_jt f_ht  (t ascending, t stored in rows h, j)
 *   fbar_ht <- fbar_ht - fbar_jt * l     (contributions to row h arrive in
 *                                         descending j)
 *   fbar_jh <- lbar / f_hh;  fbar_hh <- fbar_hh - (lbar * l) / f_hh.
 * ------------------------------------------------------------------------- */
TPILU_API tpilu_status tpilu_numeric_adjoint(tpilu_ctx ctx, tpilu_pattern pat, const double *f_val,
                                             int32_t batch, double *fbar, double *abar);

/* ---------------------------------------------------------------------------
 * Batched factor + solve under one captured HIP graph.  Records, on the ctx
 * stream, tpilu_numeric(a_val -> f_val) followed by tpilu_apply(f_val, b ->
 * y) for all `batch` instances, and instantiates the graph.  The device
 * arrays passed here are baked into the graph: each launch recomputes f_val
 * and y from the CURRENT contents of a_val and b.  The graph owns its
 * intermediate vector (n * batch doubles), its control block and, for rows
 * of more than 80 entries, its working rows (see tpilu_numeric), allocated
 * here and freed by tpilu_batched_graph_destroy, so later calls on the same
 * pattern never touch them; it reads the pattern's arrays, so the pattern
 * must outlive the graph.  Launch with tpilu_batched_graph_launch on any
 * stream of the ctx's device; two launches of one graph must not overlap
 * (they share its vector and control block).  b and y may not alias.
 *
 * tpilu_batched_graph_check waits for `hip_stream` (a hipStream_t as void*,
 * NULL = the null stream) and reports the status of the graph's last launch
 * on it: TPILU_E_ZEROPIVOT with *bad_row (host, nullable) = the smallest row
 * with a +-0 final pivot over all instances (else -1), TPILU_E_TIMEOUT after a
 * watchdog timeout, TPILU_E_INVAL for the reserved NaN in an input.
 * ------------------------------------------------------------------------- */
TPILU_API tpilu_status tpilu_batched_graph_create(tpilu_ctx ctx, tpilu_pattern pat,
                                                  const double *a_val, int32_t batch,
                                                  double *f_val, const double *b, double *y,
                                                  tpilu_graph *out);
TPILU_API tpilu_status tpilu_batched_graph_launch(tpilu_graph g, void *hip_stream);
TPILU_API tpilu_status tpilu_batched_graph_check(tpilu_graph g, void *hip_stream, int64_t *bad_row);
TPILU_API void tpilu_batched_graph_destroy(tpilu_graph g);

#ifdef __cplusplus
}
#endif

#endif /* TPILU_H */
